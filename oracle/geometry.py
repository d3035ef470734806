"""Non-affine (trilinear) hexahedra: the elasticity operator with the Jacobian
evaluated at every quadrature point (FP64 oracle; test infrastructure only -- only
tests/, the smoke check and the benchmark's CPU baseline use oracle/).

The paper's kernels assume affine elements, for which J^{-1} and det J are constant
per element (Sec. 4.4), and name non-affine geometry as future work (Sec. 6), where
storing quadrature-point data competes with recomputing it.
This module keeps the bilinear form of Sec. 2 (eqs. 3-4), a(u, v) = sum_e int_e
sigma(u) : eps(v) dx, integrated by the q^3 Gauss-Legendre rule, and replaces the
affine map by the trilinear map of each hexahedron through its 8 vertices,

    x(xi) = sum_{a,b,c in {0,1}} N_a(xi_0) N_b(xi_1) N_c(xi_2) X_{abc},
    N_0(t) = 1 - t, N_1(t) = t on [0,1],

so that J(alpha) = dx/dxi, det J(alpha) and J^{-1}(alpha) vary over the points.  On
the distorted box (TrilinearOperator) the vertices are given as an array
[(n0+1)(n1+1)(n2+1), 3] with vertex (i, j, k) at i + (n0+1)(j + (n1+1)k); element
e = (ex, ey, ez) uses the vertices (ex+a, ey+b, ez+c), and element, node and dof
numbering are those of oracle.mesh.  On an unstructured mesh (UnstructuredOperator)
every element lists its 8 vertices and the global node of each of its local nodes
(an explicit element-to-node map), with arbitrary element order and orientation.

The apply evaluates, element by element, the reference gradients of u at every
point (dense basis-gradient matrices), maps them by J^{-1}(alpha), forms the
isotropic stress (eq. 3) scaled by w_alpha det J(alpha), and tests it against the
physical basis gradients -- the quadrature sum written out, no sum factorization.
"""
from __future__ import annotations

import numpy as np

from . import mesh as omesh
from . import rules
from .elasticity import reference_basis


def element_vertices(mesh, verts: np.ndarray) -> np.ndarray:
    """[NE, 8, 3] vertex coordinates of every element, local vertex v = a + 2(b + 2c)."""
    verts = np.asarray(verts, dtype=np.float64)
    n0, n1, n2 = mesh.n
    if verts.shape != ((n0 + 1) * (n1 + 1) * (n2 + 1), 3):
        raise ValueError(f"vertices must be [{(n0 + 1) * (n1 + 1) * (n2 + 1)}, 3], got {verts.shape}")
    ez, ey, ex = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    out = np.empty((mesh.num_elements, 8, 3))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                out[:, a + 2 * (b + 2 * c)] = verts[(ex + a) + (n0 + 1) * ((ey + b) + (n1 + 1) * (ez + c))]
    return out


def _corner_shape(xi: np.ndarray):
    """Values and derivatives of the 8 trilinear shape functions at points xi [K, 3]."""
    N = [(1.0 - xi[:, d], xi[:, d]) for d in range(3)]
    dN = (-1.0, 1.0)
    val = np.empty((xi.shape[0], 8))
    der = np.empty((xi.shape[0], 8, 3))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                v = a + 2 * (b + 2 * c)
                val[:, v] = N[0][a] * N[1][b] * N[2][c]
                der[:, v, 0] = dN[a] * N[1][b] * N[2][c]
                der[:, v, 1] = N[0][a] * dN[b] * N[2][c]
                der[:, v, 2] = N[0][a] * N[1][b] * dN[c]
    return val, der


def quadrature_points(q: int) -> np.ndarray:
    """[q^3, 3] Gauss-Legendre points on [0,1]^3, point alpha = qx + q (qy + q qz)."""
    xq, _ = rules.gauss_legendre(q)
    Z, Y, X = np.meshgrid(xq, xq, xq, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def jacobians(V8: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """J[e, k, i, m] = d x_i / d xi_m of the trilinear maps at the points xi [K, 3]."""
    _, der = _corner_shape(xi)
    return np.einsum("kvm,evi->ekim", der, V8)


def map_points(V8: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """x[e, k, :] = trilinear image of xi[k] in element e."""
    val, _ = _corner_shape(xi)
    return np.einsum("kv,evi->eki", val, V8)


def node_coords(mesh, verts: np.ndarray, p: int) -> np.ndarray:
    """Physical coordinates (Nn, 3) of all nodes: the trilinear image of the element's
    GLL points (shared nodes get the same point from every element: neighbouring maps
    agree on the shared face)."""
    D = p + 1
    g = rules.gll_nodes(p)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)     # local node a = ix + D(iy + D iz)
    x = map_points(element_vertices(mesh, verts), xi)            # [NE, D^3, 3]
    out = np.empty((mesh.num_nodes(p), 3))
    out[omesh.element_nodes(mesh, p).ravel()] = x.reshape(-1, 3)
    return out


class HexOperator:
    """y = A x over hexahedra given by their corner vertices V8 [NE, 8, 3] (local vertex
    a + 2(b + 2c)) and their global dofs edofs [NE, 3 D^3] (local order (c, a)), with
    per-element Lame parameters; ess masks the clamped dofs."""

    def __init__(self, V8, edofs, ess, N: int, p: int, q: int, lam, mu):
        if q < p + 1:
            raise ValueError("q must be >= p+1")
        self.p, self.q, self.N = int(p), int(q), int(N)
        NE = V8.shape[0]
        self.NE = NE
        self.lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (NE,)).copy()
        self.mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (NE,)).copy()
        self.edofs, self.ess = edofs, ess
        _, self.dphi, self.w = reference_basis(p, q)               # (3, D^3, Q^3), (Q^3,)
        self.J = jacobians(V8, quadrature_points(q))               # [NE, Q^3, 3, 3]
        self.detJ = np.linalg.det(self.J)
        if np.any(self.detJ <= 0):
            raise ValueError("an element has a non-positive Jacobian at a quadrature point")
        self.Jinv = np.linalg.inv(self.J)                          # Jinv[e, k, m, i] = d xi_m / d x_i

    def volume(self) -> float:
        """sum_e sum_alpha w_alpha det J(alpha) -- the mesh volume (exact for trilinear maps)."""
        return float(np.einsum("k,ek->", self.w, self.detJ))

    def apply(self, x, constrained: bool = False, chunk: int = 256) -> np.ndarray:
        x_in = np.asarray(x, dtype=np.float64)
        x = x_in
        if constrained:
            x = x_in.copy()
            x[self.ess] = 0.0
        nb = self.dphi.shape[1]
        y = np.zeros(self.N)
        for s in range(0, self.NE, chunk):
            ee = np.arange(s, min(s + chunk, self.NE))
            dofs = self.edofs[ee]
            xe = x[dofs].reshape(len(ee), 3, nb)                                # [e, c, a]
            ref = np.einsum("mak,eca->ekcm", self.dphi, xe)                     # d u_c / d xi_m
            gu = np.einsum("ekcm,ekmi->ekci", ref, self.Jinv[ee])               # d u_c / d x_i
            eps = 0.5 * (gu + np.swapaxes(gu, 2, 3))
            tr = np.trace(eps, axis1=2, axis2=3)
            sig = (2.0 * self.mu[ee, None, None, None] * eps
                   + (self.lam[ee, None] * tr)[:, :, None, None] * np.eye(3))
            sig *= (self.w[None, :] * self.detJ[ee])[:, :, None, None]
            t = np.einsum("ekci,ekmi->ekcm", sig, self.Jinv[ee])                # sigma J^{-T}
            ye = np.einsum("mak,ekcm->eca", self.dphi, t)
            y += np.bincount(dofs.ravel(), ye.reshape(len(ee), -1).ravel(), minlength=self.N)
        if constrained:
            y[self.ess] = x_in[self.ess]
        return y

    def dense(self) -> np.ndarray:
        """Assembled unconstrained matrix (small problems only), column by column."""
        A = np.zeros((self.N, self.N))
        e = np.zeros(self.N)
        for j in range(self.N):
            e[j] = 1.0
            A[:, j] = self.apply(e)
            e[j] = 0.0
        return A


class TrilinearOperator(HexOperator):
    """y = A x on the distorted box with per-element Lame parameters."""

    def __init__(self, mesh, p: int, q: int, verts, lam, mu):
        self.mesh = mesh
        super().__init__(element_vertices(mesh, verts), omesh.element_dofs(mesh, p), omesh.essential_mask(mesh, p),
                         mesh.num_dofs(p), p, q, lam, mu)


class UnstructuredOperator(HexOperator):
    """y = A x on an unstructured hexahedral mesh described by vertex positions, the 8
    vertices of each element, the global node of each local node and a clamped-node
    mask (the fields of synthetic.HexMesh)."""

    def __init__(self, hm, q: int, lam, mu):
        en = np.asarray(hm.elem_nodes, dtype=np.int64)
        nn = int(hm.num_nodes)
        V8 = np.asarray(hm.vertices, dtype=np.float64)[np.asarray(hm.elem_vertices, dtype=np.int64)]
        edofs = np.concatenate([en + c * nn for c in range(3)], axis=1)
        ess = np.tile(np.asarray(hm.clamped, dtype=bool), 3)
        super().__init__(V8, edofs, ess, 3 * nn, hm.p, q, lam, mu)
        self.hm = hm
