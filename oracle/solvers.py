"""Reference solvers and multigrid components (dense FP64, small problems).

* Direct solves of the constrained system A U = F (eq. 5): dense, and a block
  Cholesky over the element slabs of a box along x (block tridiagonal there).
* Power iteration for lambda_max(D^{-1} A) and Chebyshev-Jacobi smoothing
  (Sec. 3.1: a Chebyshev polynomial in D^{-1} A applied to the residual,
  lambda_max from 10 power iterations).  The Chebyshev recurrence is the
  classical Chebyshev acceleration (Saad, Iterative Methods for Sparse Linear
  Systems, 2nd ed., Alg. 12.1) applied to the Jacobi-preconditioned system.
* p- and h-prolongation matrices (Sec. 3: polynomial interpolation between
  p-levels, natural injection between h-levels); restriction is the transpose.
* A V(1,1)-cycle and PCG with the MFEM-style preconditioned stopping test
  (Sec. 3.2).
* A counter-based start-vector generator (SplitMix64) so that the power
  iteration can be reproduced bit-for-bit on both sides of a parity check.
"""
from __future__ import annotations

import numpy as np

from . import mesh as omesh
from . import rules

MASK64 = (1 << 64) - 1


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """Element i is 2u-1, u = (z >> 11) * 2^-53, z the (i+1)-th SplitMix64 output for `seed`.

    SplitMix64 (Steele, Lea, Flood 2014; Vigna's reference code): state advances
    by 0x9E3779B97F4A7C15, output z = mix(state) with the two xor-shift-multiply
    rounds (30, 0xBF58476D1CE4E5B9), (27, 0x94D049BB133111EB) and a final >> 31.
    """
    out = np.empty(n)
    for i in range(n):
        z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & MASK64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        z = z ^ (z >> 31)
        out[i] = 2.0 * ((z >> 11) * (1.0 / 9007199254740992.0)) - 1.0
    return out


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.linalg.solve(A, b)


def power_iteration(A: np.ndarray, d: np.ndarray, v0: np.ndarray, iters: int = 10) -> float:
    """Estimate lambda_max(D^{-1}A) with `iters` applications of A.

    v <- v0/|v0|; each step: w = A v, lambda = (v.w)/(v.Dv), v <- D^{-1}w/|D^{-1}w|.
    Returns the last lambda (a generalized Rayleigh quotient, so <= lambda_max).
    """
    v = v0 / np.linalg.norm(v0)
    lam = 0.0
    for _ in range(iters):
        w = A @ v
        lam = float(v @ w) / float(v @ (d * v))
        z = w / d
        v = z / np.linalg.norm(z)
    return lam


def chebyshev_interval(lam_hat: float, lo_frac: float = 0.1, safety: float = 1.2):
    lmax = safety * lam_hat
    return lo_frac * lmax, lmax


def chebyshev_smooth(A, d, b, x0, k: int, lmin: float, lmax: float):
    """k steps of Chebyshev acceleration for D^{-1}A x = D^{-1}b on [lmin, lmax] (Saad Alg. 12.1)."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    dvec = (r / d) / theta
    for j in range(k):
        x = x + dvec
        if j == k - 1:
            break
        r = r - A @ dvec
        rho_new = 1.0 / (2.0 * sigma - rho)
        dvec = rho_new * rho * dvec + (2.0 * rho_new / delta) * (r / d)
        rho = rho_new
    return x


def prolongation_p(mesh, pc: int, pf: int) -> np.ndarray:
    """Dense P (Nf x Nc): fine nodal values of the coarse degree-pc field (same mesh)."""
    I1, _ = rules.lagrange(rules.gll_nodes(pc), rules.gll_nodes(pf))   # (Dc, Df): l^c_j(xi^f_i)
    Ie = np.einsum("zw,yv,xu->wvuzyx", I1, I1, I1).reshape((pf + 1) ** 3, (pc + 1) ** 3)
    nf, nc = omesh.element_nodes(mesh, pf), omesh.element_nodes(mesh, pc)
    Nnf, Nnc = mesh.num_nodes(pf), mesh.num_nodes(pc)
    Pn = np.zeros((Nnf, Nnc))
    for e in range(mesh.num_elements):
        Pn[np.ix_(nf[e], nc[e])] = Ie
    return np.kron(np.eye(3), Pn)


def _hat_matrix(xf: np.ndarray, xc: np.ndarray) -> np.ndarray:
    """1D piecewise-linear coarse basis (vertices xc) evaluated at points xf."""
    P = np.zeros((len(xf), len(xc)))
    for g, x in enumerate(xf):
        j = int(np.searchsorted(xc, x, side="right") - 1)
        j = min(max(j, 0), len(xc) - 2)
        t = (x - xc[j]) / (xc[j + 1] - xc[j])
        if abs(t) < 1e-14:
            P[g, j] = 1.0
        elif abs(t - 1.0) < 1e-14:
            P[g, j + 1] = 1.0
        else:
            P[g, j], P[g, j + 1] = 1.0 - t, t
    return P


def prolongation_h(mesh_f, mesh_c) -> np.ndarray:
    """Dense P (Nf x Nc) between nested p=1 meshes: the coarse trilinear field at fine nodes."""
    P1 = [_hat_matrix(mesh_f.axis_nodes(a), mesh_c.axis_nodes(a)) for a in range(3)]
    Pn = np.kron(P1[2], np.kron(P1[1], P1[0]))
    return np.kron(np.eye(3), Pn)


class DenseLevel:
    def __init__(self, A, d, ess, lmin=None, lmax=None):
        self.A, self.d, self.ess, self.lmin, self.lmax = A, d, ess, lmin, lmax


def vcycle(levels, P, r, k: int, l: int = 0):
    """z = B r for the V(1,1)-cycle; levels[0] finest, levels[-1] coarsest (exact solve).

    P[l] maps level l+1 (coarse) to level l (fine).  Pre- and post-smoothing use
    the same Chebyshev polynomial, so B is symmetric.
    """
    L = levels[l]
    if l == len(levels) - 1:
        return np.linalg.solve(L.A, r)
    x = chebyshev_smooth(L.A, L.d, r, np.zeros_like(r), k, L.lmin, L.lmax)
    rc = P[l].T @ (r - L.A @ x)
    rc[levels[l + 1].ess] = 0.0
    ec = vcycle(levels, P, rc, k, l + 1)
    corr = P[l] @ ec
    corr[L.ess] = 0.0
    x = x + corr
    return chebyshev_smooth(L.A, L.d, r, x, k, L.lmin, L.lmax)


def pcg(A, b, prec, rtol: float, max_iter: int = 1000, stop: str = "prec"):
    """Preconditioned CG from x=0. stop='prec': sqrt(r.z/r0.z0) <= rtol; 'true': |r|/|b| <= rtol."""
    x = np.zeros_like(b)
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    rz0, nb = rz, float(np.linalg.norm(b))
    it = 0
    for it in range(1, max_iter + 1):
        Ap = A @ p
        alpha = rz / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = prec(r)
        rz_new = float(r @ z)
        crit = np.sqrt(rz_new / rz0) if stop == "prec" else np.linalg.norm(r) / nb
        if crit <= rtol:
            break
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it


class SlabCholesky:
    """Direct solve of the constrained system A_c U = F (eq. 5) of a box operator
    (oracle.elasticity.Operator) by block Cholesky over the element slabs along x.

    The dofs are grouped by node plane gx: block s holds the planes s p + 1 .. (s+1) p,
    block 0 also plane 0.  An element of slab s couples only the planes s p .. (s+1) p,
    so the assembled matrix is block tridiagonal in these blocks, and block s meets block
    s-1 only through the interface plane s p (the last plane of block s-1).  Elimination:
    S_0 = A_00 and S_s = A_ss - A_{s,s-1} S_{s-1}^{-1} A_{s-1,s}, each factored by dense
    Cholesky (a library routine); a solve is the forward and back substitution.  The
    blocks are assembled from the oracle's element matrices; clamped dofs get identity
    rows and columns.  Memory: one dense block of 3 p (n1 p + 1)(n2 p + 1) dofs per slab.
    """

    def __init__(self, op):
        from scipy.linalg import cho_factor
        mesh, p = op.mesh, op.p
        Nx, Ny, Nz = omesh.grid_shape(mesh, p)
        Nn = Nx * Ny * Nz
        nx = mesh.n[0]
        dof = np.arange(3 * Nn)
        gx = (dof % Nn) % Nx
        blk = np.maximum(gx - 1, 0) // p                      # plane -> block (planes 0..p: block 0)
        order = np.lexsort((dof, blk))                        # dofs grouped by block, ascending
        loc = np.empty(3 * Nn, dtype=np.int64)
        sizes = np.bincount(blk, minlength=nx)
        starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        loc[order] = np.arange(3 * Nn) - np.repeat(starts, sizes)
        self.nblk, self.blk, self.loc = nx, blk, loc
        self.members = [order[starts[s]:starts[s] + sizes[s]] for s in range(nx)]
        # interface of block s with block s+1: its dofs on plane (s+1) p, in local order
        self.iface = [np.sort(loc[self.members[s][gx[self.members[s]] == (s + 1) * p]]) for s in range(nx)]
        ipos = [np.full(sizes[s], -1, dtype=np.int64) for s in range(nx)]
        for s in range(nx):
            ipos[s][self.iface[s]] = np.arange(len(self.iface[s]))
        Ad = [np.zeros((sizes[s], sizes[s])) for s in range(nx)]
        Ao = [None] + [np.zeros((sizes[s], len(self.iface[s - 1]))) for s in range(1, nx)]
        ex = np.arange(mesh.num_elements) % nx
        for e in range(mesh.num_elements):
            K = op.element_matrix(e)
            d = op.edofs[e]
            s = ex[e]
            own = blk[d] == s
            io, ip = np.nonzero(own)[0], np.nonzero(~own)[0]
            lo, lp = loc[d[io]], loc[d[ip]]
            Ad[s][np.ix_(lo, lo)] += K[np.ix_(io, io)]
            if len(ip):
                Ad[s - 1][np.ix_(lp, lp)] += K[np.ix_(ip, ip)]
                Ao[s][np.ix_(lo, ipos[s - 1][lp])] += K[np.ix_(io, ip)]
        ess = op.ess
        for s in range(nx):
            m = ess[self.members[s]]
            Ad[s][m, :] = 0.0
            Ad[s][:, m] = 0.0
            Ad[s][m, m] = 1.0
            if s > 0:
                Ao[s][m, :] = 0.0
                Ao[s][:, ess[self.members[s - 1]][self.iface[s - 1]]] = 0.0
        self.Ao = Ao
        self.F = []
        for s in range(nx):
            S = Ad[s]
            if s > 0:
                I = self.iface[s - 1]
                E = np.zeros((len(self.members[s - 1]), len(I)))
                E[I, np.arange(len(I))] = 1.0
                Z = self._solve_block(s - 1, E)[I]             # (S_{s-1}^{-1})_{II}
                S = S - Ao[s] @ Z @ Ao[s].T
            self.F.append(cho_factor(S, lower=True))
            Ad[s] = None

    def _solve_block(self, s, B):
        from scipy.linalg import cho_solve
        return cho_solve(self.F[s], B)

    def solve(self, b) -> np.ndarray:
        b = np.asarray(b, dtype=np.float64)
        nx = self.nblk
        y = [b[self.members[s]].copy() for s in range(nx)]
        for s in range(1, nx):
            y[s] -= self.Ao[s] @ self._solve_block(s - 1, y[s - 1])[self.iface[s - 1]]
        x = [None] * nx
        x[nx - 1] = self._solve_block(nx - 1, y[nx - 1])
        for s in range(nx - 2, -1, -1):
            t = y[s].copy()
            t[self.iface[s]] -= self.Ao[s + 1].T @ x[s + 1]
            x[s] = self._solve_block(s, t)
        out = np.empty_like(b)
        for s in range(nx):
            out[self.members[s]] = x[s]
        return out
