"""Element stiffness matrices, the global operator and load vectors (FP64).

Definition followed (Sec. 2.1, eqs. 3-5): for trial function u = phi_b e_d and
test function v = phi_a e_c,

    K^e[(c,a),(d,b)] = integral over the element of  sigma(u) : eps(v),
    sigma(u) = lambda (div u) I + 2 mu eps(u),   eps(u) = (grad u + grad u^T)/2,

evaluated by a tensor Gauss-Legendre rule with q points per direction over the
full 3D basis functions of eq. 6 (no sum factorization).  Physical gradients use
grad phi = J^{-T} grad_ref phi (Sec. 4.4, forward Z contraction).  With affine
elements and q >= p+1 the rule integrates the (polynomial) integrand exactly, so
the matrix does not depend on q.

The global operator is A = sum_e G_e^T K^e G_e (Sec. 2.2, the operator chain
with P = I on one device); the constrained form zeroes the clamped entries of
the input and returns them unchanged on output (identity rows and columns on
the clamped dofs, homogeneous Dirichlet data, Sec. 5.1.4).
"""
from __future__ import annotations

import numpy as np

from . import mesh as omesh
from . import rules


def reference_basis(p: int, q: int):
    """3D basis values and reference gradients at the q^3 tensor GL points.

    Returns (phi (D^3,Q^3), dphi (3,D^3,Q^3), w (Q^3,)) with local node
    a = ix + D*(iy + D*iz) and point alpha = qx + Q*(qy + Q*qz).
    """
    D = p + 1
    xq, wq = rules.gauss_legendre(q)
    B, G = rules.lagrange(rules.gll_nodes(p), xq)  # (D, Q)

    def tp(fx, fy, fz):
        # t[iz,iy,ix,qz,qy,qx] = fx[ix,qx] fy[iy,qy] fz[iz,qz]
        t = np.einsum("xu,yv,zw->zyxwvu", fx, fy, fz)
        return t.reshape(D ** 3, q ** 3)

    phi = tp(B, B, B)
    dphi = np.stack([tp(G, B, B), tp(B, G, B), tp(B, B, G)])
    w = np.einsum("u,v,w->wvu", wq, wq, wq).reshape(-1)
    return phi, dphi, w


def element_matrix_parts(p: int, q: int, J: np.ndarray):
    """(K_lambda, K_mu) with K^e = lambda K_lambda + mu K_mu, local dof order (c, a)."""
    phi, dphi, w = reference_basis(p, q)
    J = np.asarray(J, dtype=np.float64)
    Jinv = np.linalg.inv(J)
    detJ = np.linalg.det(J)
    if detJ <= 0:
        raise ValueError("element Jacobian must have positive determinant")
    # physical gradients g[i, a, alpha] = sum_m Jinv[m, i] * dphi[m, a, alpha]
    g = np.einsum("mi,mat->iat", Jinv, dphi)
    W = w * detJ
    nb = g.shape[1]
    eye = np.eye(3)
    # grad of the vector basis function phi_b e_d: gradU[d][b, k, l, alpha] = delta_kd g[l, b, alpha]
    gradU = np.zeros((3, nb, 3, 3, g.shape[2]))
    for d in range(3):
        gradU[d, :, d, :, :] = np.transpose(g, (1, 0, 2))
    eps = 0.5 * (gradU + np.swapaxes(gradU, 2, 3))          # eps(u) for every trial function
    tr = np.einsum("dbkkt->dbt", eps)
    sig_lam = tr[:, :, None, None, :] * eye[None, None, :, :, None]  # lambda (div u) I, lambda = 1
    sig_mu = 2.0 * eps                                              # 2 mu eps(u),     mu = 1
    parts = []
    for sig in (sig_lam, sig_mu):
        K = np.zeros((3 * nb, 3 * nb))
        for c in range(3):
            epsV = eps[c] * W                                   # eps(v) for test functions phi_a e_c
            for d in range(3):
                # K[(c,a),(d,b)] = sum_{k,l,alpha} W sigma(phi_b e_d)_{kl} eps(phi_a e_c)_{kl}
                K[c * nb:(c + 1) * nb, d * nb:(d + 1) * nb] = (
                    epsV.reshape(nb, -1) @ sig[d].reshape(nb, -1).T)
        parts.append(K)
    return parts[0], parts[1]


class Operator:
    """y = A x for a box mesh with per-element Lame parameters (oracle, FP64)."""

    def __init__(self, mesh, p: int, q: int, lam, mu):
        self.mesh, self.p, self.q = mesh, int(p), int(q)
        if q < p + 1:
            raise ValueError("q must be >= p+1 for exact integration on affine elements")
        NE = mesh.num_elements
        self.lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (NE,)).copy()
        self.mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (NE,)).copy()
        self.N = mesh.num_dofs(p)
        self.edofs = omesh.element_dofs(mesh, p)
        self.ess = omesh.essential_mask(mesh, p)
        J = omesh.element_jacobians(mesh)
        # group elements by identical Jacobian (uniform grids have a single group)
        keys = np.round(J.reshape(NE, 9), 14)
        uniq, inv = np.unique(keys, axis=0, return_inverse=True)
        self.groups = []
        for gi in range(len(uniq)):
            els = np.nonzero(inv.ravel() == gi)[0]
            Kl, Km = element_matrix_parts(p, q, J[els[0]])
            self.groups.append((els, Kl, Km))

    def element_matrix(self, e: int) -> np.ndarray:
        for els, Kl, Km in self.groups:
            if e in els:
                return self.lam[e] * Kl + self.mu[e] * Km
        raise IndexError(e)

    def apply(self, x, constrained: bool = False) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        multi = x.ndim == 2
        X = x if multi else x[:, None]
        if constrained:
            X = X.copy()
            X[self.ess] = 0.0
        Y = np.zeros((self.N, X.shape[1]))
        for els, Kl, Km in self.groups:
            dofs = self.edofs[els]                       # (nE, nd)
            XE = X[dofs]                                 # (nE, nd, m)
            YE = (self.lam[els, None, None] * np.einsum("ij,ejm->eim", Kl, XE)
                  + self.mu[els, None, None] * np.einsum("ij,ejm->eim", Km, XE))
            for m in range(X.shape[1]):
                Y[:, m] += np.bincount(dofs.ravel(), YE[:, :, m].ravel(), minlength=self.N)
        if constrained:
            Y[self.ess] = (x if multi else x[:, None])[self.ess]
        return Y if multi else Y[:, 0]

    def abs_apply(self, x, constrained: bool = False) -> np.ndarray:
        """sum_e G_e^T |K^e| G_e x, with |K^e| the entrywise absolute values of each element
        matrix: for x >= 0 this is the sum of the magnitudes of the element products that an
        evaluation of A x adds up, the scale of its rounding error.  The constrained form
        has 0 on the clamped columns and x on the clamped rows (identity rows and columns)."""
        x_in = np.asarray(x, dtype=np.float64)
        x = x_in
        if constrained:
            x = x_in.copy()
            x[self.ess] = 0.0
        y = np.zeros(self.N)
        for els, Kl, Km in self.groups:
            # elements with the same (lambda, mu) in a group share |K^e|
            pairs = np.stack([self.lam[els], self.mu[els]], axis=1)
            uniq, inv = np.unique(pairs, axis=0, return_inverse=True)
            for k, (lv, mv) in enumerate(uniq):
                d = self.edofs[els[inv.ravel() == k]]
                ye = np.einsum("ij,ej->ei", np.abs(lv * Kl + mv * Km), x[d])
                y += np.bincount(d.ravel(), ye.ravel(), minlength=self.N)
        if constrained:
            y[self.ess] = x_in[self.ess]
        return y

    def dense(self, constrained: bool = False) -> np.ndarray:
        """Assembled dense matrix (small problems only)."""
        A = np.zeros((self.N, self.N))
        for els, Kl, Km in self.groups:
            for e in els:
                d = self.edofs[e]
                A[np.ix_(d, d)] += self.lam[e] * Kl + self.mu[e] * Km
        if constrained:
            A[self.ess, :] = 0.0
            A[:, self.ess] = 0.0
            A[self.ess, self.ess] = 1.0
        return A

    def diagonal(self, constrained: bool = False) -> np.ndarray:
        d = np.zeros(self.N)
        for els, Kl, Km in self.groups:
            dofs = self.edofs[els]
            DE = self.lam[els, None] * np.diag(Kl)[None, :] + self.mu[els, None] * np.diag(Km)[None, :]
            d += np.bincount(dofs.ravel(), DE.ravel(), minlength=self.N)
        if constrained:
            d[self.ess] = 1.0
        return d


def body_force_vector(mesh, p: int, q: int, f) -> np.ndarray:
    """F[(c,node)] = sum_e integral f_c phi_a (constant body force f)."""
    phi, _, w = reference_basis(p, q)
    J = omesh.element_jacobians(mesh)
    detJ = np.linalg.det(J)
    fe = (phi @ w)[None, :] * detJ[:, None]             # (NE, D^3)
    nodes = omesh.element_nodes(mesh, p)
    Nn = mesh.num_nodes(p)
    s = np.bincount(nodes.ravel(), fe.ravel(), minlength=Nn)
    return np.concatenate([f[c] * s for c in range(3)])


def traction_vector(mesh, p: int, q: int, face: int, t) -> np.ndarray:
    """F[(c,node)] = integral over box face `face` of t_c phi (constant traction t).

    face: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+.  The surface measure of the affine
    face spanned by columns J[:,i1], J[:,i2] is |J[:,i1] x J[:,i2]| d(xi_i1) d(xi_i2).
    """
    D = p + 1
    axis, side = face // 2, face % 2
    t1, t2 = [a for a in range(3) if a != axis]
    xq, wq = rules.gauss_legendre(q)
    B, _ = rules.lagrange(rules.gll_nodes(p), xq)
    end, _ = rules.lagrange(rules.gll_nodes(p), np.array([float(side)]))
    end = end[:, 0]
    # face integrals of the 1D factors: s1[i] = sum_q w B[i,q]
    s1 = B @ wq
    J = omesh.element_jacobians(mesh)
    nodes = omesh.element_nodes(mesh, p)
    Nn = mesh.num_nodes(p)
    n = mesh.n
    e_idx = np.arange(mesh.num_elements)
    epos = [e_idx % n[0], (e_idx // n[0]) % n[1], e_idx // (n[0] * n[1])]
    on_face = epos[axis] == (0 if side == 0 else n[axis] - 1)
    els = np.nonzero(on_face)[0]
    area = np.linalg.norm(np.cross(J[els, :, t1], J[els, :, t2]), axis=1)   # (nF,)
    fac = [None, None, None]
    fac[axis] = end
    fac[t1] = s1
    fac[t2] = s1
    loc = np.einsum("z,y,x->zyx", fac[2], fac[1], fac[0]).reshape(-1)     # (D^3,)
    vals = area[:, None] * loc[None, :]
    s = np.bincount(nodes[els].ravel(), vals.ravel(), minlength=Nn)
    return np.concatenate([t[c] * s for c in range(3)])
