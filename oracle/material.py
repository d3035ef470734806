"""General material data of the elasticity operator: per-quadrature-point isotropic
Lame parameters and anisotropic stiffness (FP64 oracle; test infrastructure only --
only tests/, the smoke check and the benchmark's CPU baseline use oracle/).

Definition followed: the generalized Hooke law of Sec. 2.1 (eq. 2),
sigma_ij = C_ijkl eps_kl, written in Voigt form

    sigma_V = C_V eps_V,   eps_V = (e_xx, e_yy, e_zz, 2 e_yz, 2 e_xz, 2 e_xy)

(engineering shear strains) with a symmetric 6x6 stiffness C_V; the isotropic law
(eq. 3) is C_V = lambda 1 1^T + mu diag(2, 2, 2, 1, 1, 1).  The paper's partial-
assembly data holds the material at every quadrature point (Sec. 4.5), so C_V may
vary per element and per point.  The element matrix is the textbook strain-
displacement form, a different route from elasticity.element_matrix_parts:

    K^e = sum_alpha w_alpha detJ B_alpha^T C_V(alpha) B_alpha,

B_alpha the 6 x 3D^3 matrix mapping the element's nodal displacements (component
blocks, local node a = ix + D (iy + D iz)) to eps_V at point alpha, with physical
gradients J^{-T} grad_ref phi on the q^3 Gauss-Legendre points.  The apply forms
y_e = sum_alpha w detJ B^T (C_V (B x_e)) directly, without assembling K^e.
"""
from __future__ import annotations

import numpy as np

from . import mesh as omesh
from .elasticity import reference_basis

# Voigt index of the symmetric tensor entry (i, j)
VOIGT = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (2, 1): 3, (0, 2): 4, (2, 0): 4, (0, 1): 5, (1, 0): 5}


def isotropic_voigt(lam, mu) -> np.ndarray:
    """C_V of the isotropic law; lam, mu scalars or arrays (returns [..., 6, 6])."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    C = np.zeros(lam.shape + (6, 6))
    C[..., :3, :3] = lam[..., None, None]
    for k, f in enumerate((2.0, 2.0, 2.0, 1.0, 1.0, 1.0)):
        C[..., k, k] += f * mu
    return C


def strain_matrix(p: int, q: int, J: np.ndarray):
    """(B [Q^3, 6, 3 D^3], W [Q^3]) for an affine element with Jacobian J."""
    _, dphi, w = reference_basis(p, q)
    J = np.asarray(J, dtype=np.float64)
    detJ = np.linalg.det(J)
    if detJ <= 0:
        raise ValueError("element Jacobian must have positive determinant")
    g = np.einsum("mi,mat->ati", np.linalg.inv(J), dphi)   # g[a, alpha, i] = d phi_a / d x_i
    nb = g.shape[0]
    B = np.zeros((g.shape[1], 6, 3 * nb))
    for c in range(3):              # displacement component of the trial function
        for i in range(3):          # derivative direction
            k = VOIGT[(c, i)]
            B[:, k, c * nb:(c + 1) * nb] += g[:, :, i].T
    return B, w * detJ


def packed_upper(C: np.ndarray) -> np.ndarray:
    """The 21 upper-triangle entries of [..., 6, 6], row by row."""
    iu = np.triu_indices(6)
    return np.asarray(C)[..., iu[0], iu[1]]


def unpack_upper(c21: np.ndarray) -> np.ndarray:
    c21 = np.asarray(c21, dtype=np.float64)
    C = np.zeros(c21.shape[:-1] + (6, 6))
    iu = np.triu_indices(6)
    C[..., iu[0], iu[1]] = c21
    C[..., iu[1], iu[0]] = c21
    return C


class GeneralOperator:
    """y = A x with a stiffness C_V per element ([NE, 6, 6]) or per element and
    quadrature point ([NE, q^3, 6, 6]); point alpha = qx + q (qy + q qz)."""

    def __init__(self, mesh, p: int, q: int, C):
        if q < p + 1:
            raise ValueError("q must be >= p+1")
        self.mesh, self.p, self.q = mesh, int(p), int(q)
        NE = mesh.num_elements
        C = np.asarray(C, dtype=np.float64)
        if C.shape == (NE, 6, 6):
            C = np.broadcast_to(C[:, None], (NE, q ** 3, 6, 6))
        if C.shape != (NE, q ** 3, 6, 6):
            raise ValueError(f"C must be [NE,6,6] or [NE,q^3,6,6], got {C.shape}")
        self.C = C
        self.N = mesh.num_dofs(p)
        self.edofs = omesh.element_dofs(mesh, p)
        self.ess = omesh.essential_mask(mesh, p)
        J = omesh.element_jacobians(mesh)
        keys = np.round(J.reshape(NE, 9), 14)
        uniq, inv = np.unique(keys, axis=0, return_inverse=True)
        self.groups = []
        for gi in range(len(uniq)):
            els = np.nonzero(inv.ravel() == gi)[0]
            B, W = strain_matrix(p, q, J[els[0]])
            self.groups.append((els, B, W))

    def apply(self, x, constrained: bool = False, chunk: int = 4096) -> np.ndarray:
        """y = A x; constrained: clamped inputs read as 0 and clamped outputs equal the input."""
        x_in = np.asarray(x, dtype=np.float64)
        x = x_in
        if constrained:
            x = x_in.copy()
            x[self.ess] = 0.0
        y = np.zeros(self.N)
        for els, B, W in self.groups:
            for s in range(0, len(els), chunk):
                ee = els[s:s + chunk]
                dofs = self.edofs[ee]
                eps = np.einsum("akn,en->eak", B, x[dofs])                 # eps_V at every point
                sig = np.einsum("eakl,eal->eak", self.C[ee], eps) * W[None, :, None]
                ye = np.einsum("akn,eak->en", B, sig)
                y += np.bincount(dofs.ravel(), ye.ravel(), minlength=self.N)
        if constrained:
            y[self.ess] = x_in[self.ess]
        return y

    def element_matrix(self, e: int) -> np.ndarray:
        """K^e = sum_alpha w_alpha detJ B_alpha^T C_V(alpha) B_alpha ([3 D^3, 3 D^3])."""
        for els, B, W in self.groups:
            k = np.searchsorted(els, e)
            if k < len(els) and els[k] == e:
                return self._element_matrix(B, W, self.C[e])
        raise IndexError(e)

    @staticmethod
    def _element_matrix(B, W, C):
        # sum over points alpha and Voigt rows k of (W B)_akn (C B)_akm, as one matrix product
        CB = np.einsum("akl,alm->akm", C, B)
        nk = B.shape[0] * B.shape[1]
        return (B * W[:, None, None]).reshape(nk, -1).T @ CB.reshape(nk, -1)

    def dense(self, constrained: bool = False) -> np.ndarray:
        """Assembled dense matrix (small problems only); constrained: identity on the
        clamped rows and columns."""
        A = np.zeros((self.N, self.N))
        for els, B, W in self.groups:
            for e in els:
                d = self.edofs[e]
                A[np.ix_(d, d)] += self._element_matrix(B, W, self.C[e])
        if constrained:
            A[self.ess, :] = 0.0
            A[:, self.ess] = 0.0
            A[self.ess, self.ess] = 1.0
        return A

    def diagonal(self, constrained: bool = False) -> np.ndarray:
        """diag(A): per element, K^e_nn = sum_alpha w detJ sum_kl B_akn C_akl B_aln."""
        d = np.zeros(self.N)
        for els, B, W in self.groups:
            dofs = self.edofs[els]
            DE = np.stack([np.einsum("akn,akn->n", B * W[:, None, None], np.einsum("akl,aln->akn", self.C[e], B))
                           for e in els])
            d += np.bincount(dofs.ravel(), DE.ravel(), minlength=self.N)
        if constrained:
            d[self.ess] = 1.0
        return d

    def energy_of_affine(self, E: np.ndarray) -> float:
        """(1/2) sum_e sum_alpha w detJ eps_V^T C_V eps_V for u(X) = E X (constant strain)."""
        eps = 0.5 * (E + E.T)
        ev = np.array([eps[0, 0], eps[1, 1], eps[2, 2], 2 * eps[1, 2], 2 * eps[0, 2], 2 * eps[0, 1]])
        tot = 0.0
        for els, _, W in self.groups:
            tot += 0.5 * np.einsum("a,eakl,k,l->", W, self.C[els], ev, ev)
        return float(tot)
