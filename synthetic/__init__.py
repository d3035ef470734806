"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle scripts.

This module only *describes* workloads: structured box meshes (element counts,
box lengths, an optional global affine map and optional graded node
coordinates, clamped faces), per-element material parameters and random
vectors.  It holds none of the elasticity method's arithmetic: element
Jacobians, basis functions, quadrature, operators and solvers live on each side
of the parity check separately (the HIP library and the oracle).

Conventions (all shared by both sides through this description only):

* Elements are numbered lexicographically with ``ex`` fastest.
* ``clamped_faces`` is a bitmask: bit0 x-, bit1 x+, bit2 y-, bit3 y+, bit4 z-, bit5 z+.
* Random streams use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

FACE_XMIN, FACE_XMAX, FACE_YMIN, FACE_YMAX, FACE_ZMIN, FACE_ZMAX = 0, 1, 2, 3, 4, 5


@dataclasses.dataclass
class BoxMesh:
    """A structured box of n[0] x n[1] x n[2] hexahedra.

    Reference node coordinates along axis ``a`` are ``grade[a]`` (length
    ``n[a]+1``, strictly increasing) or uniform on ``[0, L[a]]``; the physical
    point is ``A @ X + x0`` with ``det(A) > 0``, so every element is an affine
    parallelepiped.
    """

    n: tuple
    L: tuple = (1.0, 1.0, 1.0)
    A: np.ndarray = dataclasses.field(default_factory=lambda: np.eye(3))
    x0: tuple = (0.0, 0.0, 0.0)
    grade: Optional[Sequence[Optional[np.ndarray]]] = None
    clamped_faces: int = 0

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        self.L = tuple(float(v) for v in self.L)
        self.A = np.asarray(self.A, dtype=np.float64).reshape(3, 3)
        self.x0 = tuple(float(v) for v in self.x0)
        if self.grade is not None:
            g = []
            for a in range(3):
                ga = self.grade[a]
                g.append(None if ga is None else np.ascontiguousarray(ga, dtype=np.float64))
            self.grade = tuple(g)

    @property
    def num_elements(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def axis_nodes(self, a: int) -> np.ndarray:
        """Vertex coordinates along reference axis ``a`` (length n[a]+1)."""
        if self.grade is not None and self.grade[a] is not None:
            return np.asarray(self.grade[a], dtype=np.float64)
        return np.linspace(0.0, self.L[a], self.n[a] + 1)

    def num_nodes(self, p: int) -> int:
        return (self.n[0] * p + 1) * (self.n[1] * p + 1) * (self.n[2] * p + 1)

    def num_dofs(self, p: int) -> int:
        return 3 * self.num_nodes(p)


def lame_from_young_poisson(E, nu):
    """Lame parameters of an isotropic material from Young's modulus and Poisson ratio."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def uniform_vector(n: int, seed: int = 0, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


# --------------------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------------------

SHEAR_A = np.array([[1.0, 0.2, 0.2], [0.0, 1.0, 0.2], [0.0, 0.0, 1.0]])


def unit_cube_4(clamped: bool = False) -> BoxMesh:
    """Unit cube, 4x4x4 elements (clamped on x=0 when ``clamped``)."""
    return BoxMesh(n=(4, 4, 4), L=(1.0, 1.0, 1.0), clamped_faces=(1 << FACE_XMIN) if clamped else 0)


def sheared_box_mesh(p: int) -> BoxMesh:
    """Fixed-size (~4.2M dofs) sheared box of the operator sweep.

    The reference box [0,1.25]^2 x [0,1] is split into (120/p,120/p,96/p) cubes
    for p in {1,2,3,4,6,8}; p=5 and p=7 use (24,24,19) and (17,17,14), the
    nearly-cubic counts that keep ~4.2M dofs.  The global map A is a shear with
    0.2 above the diagonal (det A = 1).
    """
    table = {1: (120, 120, 96), 2: (60, 60, 48), 3: (40, 40, 32), 4: (30, 30, 24),
             5: (24, 24, 19), 6: (20, 20, 16), 7: (17, 17, 14), 8: (15, 15, 12)}
    n = table[p]
    return BoxMesh(n=n, L=(1.25, 1.25, 1.0), A=SHEAR_A.copy())


def two_material_lame(num_elements: int, seed: int = 1, E=(1.0, 100.0), nu: float = 0.3):
    """Per-element Lame parameters, material drawn uniformly from two (seeded)."""
    mat = np.random.default_rng(seed).integers(0, 2, num_elements)
    Es = np.where(mat == 0, E[0], E[1])
    return lame_from_young_poisson(Es, np.full(num_elements, nu))


def random_spd_stiffness(num: int, seed: int = 11, lam: float = 1.0, mu: float = 1.0,
                         spread: float = 0.5) -> np.ndarray:
    """[num, 6, 6] symmetric positive definite Voigt stiffnesses: an isotropic matrix
    (lam, mu) plus spread * M M^T / 6 with M ~ U[-1,1]^{6x6} (general anisotropy)."""
    rng = np.random.default_rng(seed)
    base = np.zeros((6, 6))
    base[:3, :3] = lam
    base += np.diag([2 * mu, 2 * mu, 2 * mu, mu, mu, mu])
    M = rng.uniform(-1.0, 1.0, (num, 6, 6))
    return base[None] + spread * np.einsum("nij,nkj->nik", M, M) / 6.0


def quadrature_point_lame(lam_e, mu_e, q: int, seed: int = 13, spread: float = 0.3):
    """Per-point Lame parameters [NE, q^3]: the element values times (1 + spread u),
    u ~ U[-1,1] independently per point (point alpha = qx + q (qy + q qz))."""
    rng = np.random.default_rng(seed)
    lam_e = np.asarray(lam_e, dtype=np.float64)
    mu_e = np.asarray(mu_e, dtype=np.float64)
    n = lam_e.shape[0]
    f1 = 1.0 + spread * rng.uniform(-1.0, 1.0, (n, q ** 3))
    f2 = 1.0 + spread * rng.uniform(-1.0, 1.0, (n, q ** 3))
    return lam_e[:, None] * f1, mu_e[:, None] * f2


def cantilever_mesh(nx: int = 80, ny: int = 8, nz: int = 8, length: float = 8.0) -> BoxMesh:
    """8:1:1 cantilever [0,8]x[0,1]^2 clamped at x=0 (traction goes on x=8)."""
    return BoxMesh(n=(nx, ny, nz), L=(length, 1.0, 1.0), clamped_faces=1 << FACE_XMIN)


def graded_mesh(n, seed: int, L=(1.0, 1.0, 1.0), A=None, clamped_faces: int = 0,
                spread: float = 0.35) -> BoxMesh:
    """A box with random strictly-increasing per-axis vertex coordinates."""
    rng = np.random.default_rng(seed)
    grade = []
    for a in range(3):
        h = rng.uniform(1.0 - spread, 1.0 + spread, n[a])
        x = np.concatenate([[0.0], np.cumsum(h)])
        grade.append(x * (L[a] / x[-1]))
    return BoxMesh(n=n, L=L, A=np.eye(3) if A is None else A, grade=grade, clamped_faces=clamped_faces)


def perturbed_vertices(mesh: BoxMesh, amp: float = 0.2, seed: int = 17, interior_only: bool = True) -> np.ndarray:
    """Vertex positions [(n0+1)(n1+1)(n2+1), 3] of a distorted box: the box vertices
    (A X + x0, vertex (i,j,k) at i + (n0+1)(j + (n1+1)k)) moved by amp times the
    smallest local reference spacing times U[-1,1]^3, on interior vertices only or on
    all of them.  With amp below ~0.25 every element keeps a positive Jacobian."""
    rng = np.random.default_rng(seed)
    ax = [np.asarray(mesh.axis_nodes(a), dtype=np.float64) for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    R = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    # smallest spacing of the reference cells touching each vertex, per axis
    hs = []
    for a in range(3):
        d = np.diff(ax[a])
        h = np.minimum(np.concatenate([[d[0]], d]), np.concatenate([d, [d[-1]]]))
        hs.append(h)
    Hz, Hy, Hx = np.meshgrid(hs[2], hs[1], hs[0], indexing="ij")
    H = np.minimum(np.minimum(Hx, Hy), Hz).ravel()
    dR = amp * H[:, None] * rng.uniform(-1.0, 1.0, R.shape)
    if interior_only:
        n0, n1, n2 = mesh.n
        k, j, i = np.meshgrid(np.arange(n2 + 1), np.arange(n1 + 1), np.arange(n0 + 1), indexing="ij")
        edge = (i == 0) | (i == n0) | (j == 0) | (j == n1) | (k == 0) | (k == n2)
        dR[edge.ravel()] = 0.0
    return (R + dR) @ mesh.A.T + np.asarray(mesh.x0)


def random_rotation(seed: int) -> np.ndarray:
    """A random proper rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((3, 3))
    Qm, R = np.linalg.qr(M)
    Qm = Qm @ np.diag(np.sign(np.diag(R)))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] = -Qm[:, 0]
    return Qm


@dataclasses.dataclass
class ServeRequest:
    rid: int
    arrival: float
    n: tuple
    p: int
    E: float
    nu: float
    f: tuple


def serving_stream(num: int = 512, rate: float = 1.0, seed: int = 5, n_lo: int = 4, n_hi: int = 32,
                   ps=(2, 4, 6, 8)):
    """Poisson arrivals of box solves with random sizes, orders and materials."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(num):
        t += rng.exponential(1.0 / rate)
        n = tuple(int(v) for v in rng.integers(n_lo, n_hi + 1, 3))
        p = int(rng.choice(ps))
        E = float(10.0 ** rng.uniform(0.0, 2.0))
        nu = float(rng.uniform(0.2, 0.4))
        f = tuple(float(v) for v in rng.uniform(-1.0, 1.0, 3))
        out.append(ServeRequest(i, t, n, p, E, nu, f))
    return out
