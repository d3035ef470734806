"""Structured-box geometry and numbering for the oracle.

The mesh is a box of n0 x n1 x n2 hexahedra with per-axis vertex coordinates X
(graded or uniform) mapped by a global affine map x = A X + x0 (Sec. 4.4: the
elements are affine, so J^{-1} and det J are constant per element).

Numbering (the paper is silent; the reading used on both sides of the parity
check):

* element e = ex + n0*(ey + n1*ez);
* global node (gx,gy,gz) on the (n0 p+1) x (n1 p+1) x (n2 p+1) grid has index
  gx + (n0 p+1)*(gy + (n1 p+1)*gz);
* global dof (c, node) = c*Nn + node (component blocks, "by nodes");
* local node a = ix + D*(iy + D*iz), D = p+1 (ix fastest, Sec. 4.4 X-contraction).
"""
from __future__ import annotations

import numpy as np

from . import rules


def axis_vertices(mesh, a: int) -> np.ndarray:
    return np.asarray(mesh.axis_nodes(a), dtype=np.float64)


def element_jacobians(mesh) -> np.ndarray:
    """Constant Jacobians J_e (NE,3,3) of the maps [0,1]^3 -> element: J_e = A diag(h)."""
    hs = [np.diff(axis_vertices(mesh, a)) for a in range(3)]
    n0, n1, n2 = mesh.n
    hx = np.tile(hs[0], n1 * n2)
    hy = np.tile(np.repeat(hs[1], n0), n2)
    hz = np.repeat(hs[2], n0 * n1)
    H = np.zeros((mesh.num_elements, 3, 3))
    H[:, 0, 0], H[:, 1, 1], H[:, 2, 2] = hx, hy, hz
    return np.einsum("ij,ejk->eik", mesh.A, H)


def axis_node_coords(mesh, a: int, p: int) -> np.ndarray:
    """Reference coordinates of the n_a*p+1 nodes along axis a (GLL nodes per element)."""
    X = axis_vertices(mesh, a)
    xi = rules.gll_nodes(p)
    out = np.empty(mesh.n[a] * p + 1)
    for e in range(mesh.n[a]):
        out[e * p:(e + 1) * p + 1] = X[e] + (X[e + 1] - X[e]) * xi
    return out


def node_coords(mesh, p: int) -> np.ndarray:
    """Physical coordinates (Nn,3) of all nodes in global node order."""
    cx, cy, cz = (axis_node_coords(mesh, a, p) for a in range(3))
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    R = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return R @ mesh.A.T + np.asarray(mesh.x0)


def grid_shape(mesh, p: int):
    return tuple(mesh.n[a] * p + 1 for a in range(3))


def element_nodes(mesh, p: int) -> np.ndarray:
    """Global node index of each local node: (NE, D^3), local order ix fastest."""
    D = p + 1
    Nx, Ny, _ = grid_shape(mesh, p)
    n0, n1, n2 = mesh.n
    ez, ey, ex = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    iz, iy, ix = np.meshgrid(np.arange(D), np.arange(D), np.arange(D), indexing="ij")
    gx = (ex.ravel() * p)[:, None] + ix.ravel()[None, :]
    gy = (ey.ravel() * p)[:, None] + iy.ravel()[None, :]
    gz = (ez.ravel() * p)[:, None] + iz.ravel()[None, :]
    return gx + Nx * (gy + Ny * gz)


def element_dofs(mesh, p: int) -> np.ndarray:
    """Global dof index of each local dof: (NE, 3*D^3), local order (c, a)."""
    nodes = element_nodes(mesh, p)
    Nn = mesh.num_nodes(p)
    return np.concatenate([nodes + c * Nn for c in range(3)], axis=1)


def essential_mask(mesh, p: int) -> np.ndarray:
    """Boolean mask over the 3*Nn dofs of the clamped faces (all components)."""
    Nx, Ny, Nz = grid_shape(mesh, p)
    gz, gy, gx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    gx, gy, gz = gx.ravel(), gy.ravel(), gz.ravel()
    m = np.zeros(gx.shape, dtype=bool)
    f = mesh.clamped_faces
    if f & 1:
        m |= gx == 0
    if f & 2:
        m |= gx == Nx - 1
    if f & 4:
        m |= gy == 0
    if f & 8:
        m |= gy == Ny - 1
    if f & 16:
        m |= gz == 0
    if f & 32:
        m |= gz == Nz - 1
    return np.concatenate([m, m, m])
