"""The collocated form the p <= 2 box kernels use for affine elements with per-element Lame data,
restated in numpy and checked against the oracle's element matrices (no GPU).

J^{-1} and the Lame weights are constant over an affine element, so each entry of the reference
gradient, of the stress and of Q = sigma J^{-T} is a polynomial of degree at most p in each
coordinate and equals its interpolant through the p+1 Gauss-Lobatto nodes per axis.  Putting
that interpolant into the quadrature sums (paper Sec. 2.1, eqs. 3-5; the pointwise stage of
Sec. 4.4, eq. 7) regroups them exactly: the pointwise stage runs at the (p+1)^3 nodes, and the
rule enters only through the 1D matrices Mm[j][i] = sum_r w_r l_j(xi_r) l_i(xi_r) and
Nm[j][i] = sum_r w_r l_j(xi_r) l'_i(xi_r).  Pinned for p = 1..4 and q = p+1..p+3."""
import numpy as np
import pytest

from oracle import rules
from oracle.elasticity import element_matrix_parts


def collocated_apply(x, J, lam, mu, p, q):
    """y = K_e x for one affine element; x[c, ix, iy, iz]."""
    xg = rules.gll_nodes(p)
    xq, wq = rules.gauss_legendre(q)
    B, G = rules.lagrange(xg, xq)      # (p+1, q)
    _, Dn = rules.lagrange(xg, xg)     # l'_i at the Gauss-Lobatto nodes
    Mm, Nm = (B * wq) @ B.T, (B * wq) @ G.T
    Ji, det = np.linalg.inv(J), np.linalg.det(J)
    g = np.stack([np.einsum("cabz,aj->cjbz", x, Dn), np.einsum("cabz,bj->cajz", x, Dn),
                  np.einsum("cabz,zj->cabj", x, Dn)], axis=1)
    du = np.einsum("cmxyz,mi->cixyz", g, Ji)
    tr = du[0, 0] + du[1, 1] + du[2, 2]
    sig = det * (lam * tr[None, None] * np.eye(3)[:, :, None, None, None] + mu * (du + du.transpose(1, 0, 2, 3, 4)))
    Qv = np.einsum("cjxyz,kj->ckxyz", sig, Ji)
    return (np.einsum("cxyz,xa,yb,zg->cabg", Qv[:, 0], Nm, Mm, Mm)
            + np.einsum("cxyz,xa,yb,zg->cabg", Qv[:, 1], Mm, Nm, Mm)
            + np.einsum("cxyz,xa,yb,zg->cabg", Qv[:, 2], Mm, Mm, Nm))


def _reference(x, J, lam, mu, p, q):
    D = p + 1
    Kl, Km = element_matrix_parts(p, q, J)
    xv = np.transpose(x, (0, 3, 2, 1)).reshape(-1)   # oracle dof order (c, ix + D (iy + D iz))
    return ((lam * Kl + mu * Km) @ xv).reshape(3, D, D, D).transpose(0, 3, 2, 1)


def _jacobian(rng):
    while True:
        J = np.diag(rng.uniform(0.4, 2.0, 3)) + 0.3 * rng.standard_normal((3, 3))
        if np.linalg.det(J) > 0.05:
            return J


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_collocated_equals_quadrature(p):
    rng = np.random.default_rng(50 + p)
    for q in (p + 1, p + 2, p + 3):
        J = _jacobian(rng)
        lam, mu = rng.uniform(0.1, 5.0), rng.uniform(0.1, 5.0)
        x = rng.standard_normal((3, p + 1, p + 1, p + 1))
        ref = _reference(x, J, lam, mu, p, q)
        y = collocated_apply(x, J, lam, mu, p, q)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max(), (p, q)


def test_collocated_needs_the_rule_in_the_backward_tables():
    """Collocating at the nodes with plain nodal weights (the Lobatto rule, not exact for this
    integrand) gives a different operator: the rule's mass matrices are what makes it exact."""
    rng = np.random.default_rng(9)
    p, q = 2, 4
    J, lam, mu = _jacobian(rng), 1.3, 0.8
    x = rng.standard_normal((3, 3, 3, 3))
    ref = _reference(x, J, lam, mu, p, q)
    xg = rules.gll_nodes(p)
    wg = rules.gll_weights(p)
    _, Dn = rules.lagrange(xg, xg)
    Mm, Nm = np.diag(wg), np.diag(wg) @ Dn.T
    Ji, det = np.linalg.inv(J), np.linalg.det(J)
    g = np.stack([np.einsum("cabz,aj->cjbz", x, Dn), np.einsum("cabz,bj->cajz", x, Dn),
                  np.einsum("cabz,zj->cabj", x, Dn)], axis=1)
    du = np.einsum("cmxyz,mi->cixyz", g, Ji)
    tr = du[0, 0] + du[1, 1] + du[2, 2]
    sig = det * (lam * tr[None, None] * np.eye(3)[:, :, None, None, None] + mu * (du + du.transpose(1, 0, 2, 3, 4)))
    Qv = np.einsum("cjxyz,kj->ckxyz", sig, Ji)
    lumped = (np.einsum("cxyz,xa,yb,zg->cabg", Qv[:, 0], Nm, Mm, Mm)
              + np.einsum("cxyz,xa,yb,zg->cabg", Qv[:, 1], Mm, Nm, Mm)
              + np.einsum("cxyz,xa,yb,zg->cabg", Qv[:, 2], Mm, Mm, Nm))
    assert np.abs(lumped - ref).max() > 1e-3 * np.abs(ref).max()
