"""The regrouping the p = 1 kernel uses for per-element Lame data, restated in numpy and
checked against the oracle's element matrices (no GPU).

With centred coordinates s = xi - 1/2 the trilinear basis is prod_k (1/2 + sgn(i_k) s_k), so
the element's displacement, gradient, stress and test gradients are sums over monomials s^a,
a in {0,1}^3, with coefficients from the 8-point Walsh-Hadamard transform of the nodal
values.  A product of two monomials sums over the tensor Gauss rule to a product of the
rule's centred 1D moments W_m = sum w s^m; the rule is symmetric about 1/2, so its odd
moments vanish and only equal monomials pair up (weight W0^(3-|t|) W2^|t|).  This test pins
that identity for the rules the operator offers at p = 1 (q = 2, 3, 4), on sheared and
rotated Jacobians, against the oracle's direct quadrature (paper Sec. 2.1, eqs. 3-5; Sec. 4.4,
the pointwise stress and Q = sigma J^{-T} of eq. 7)."""
import numpy as np
import pytest

from oracle import rules
from oracle.elasticity import element_matrix_parts

SGN = np.array([-1.0, 1.0])


def _walsh(a):
    """prod_k sgn(i_k)^(a_k) over the nodes i = (ix, iy, iz), as an array [ix, iy, iz]."""
    return np.einsum("i,j,k->ijk", SGN ** a[0], SGN ** a[1], SGN ** a[2])


def closed_form_apply(x, J, lam, mu, q, w2=None):
    """y = K_e x for one affine element; x[c, ix, iy, iz] (component, node).  w2 replaces
    the rule's second centred moment (to show that the result depends on it)."""
    xq, wq = rules.gauss_legendre(q)
    s = xq - 0.5
    W0, W2 = wq.sum(), (wq * s * s).sum() if w2 is None else w2
    Ji = np.linalg.inv(J)
    det = np.linalg.det(J)
    H = {a: np.einsum("cijk,ijk->c", x, _walsh(a)) for a in np.ndindex(2, 2, 2)}
    Y = {a: np.zeros(3) for a in np.ndindex(2, 2, 2)}
    for t in np.ndindex(2, 2, 2):
        n = sum(t)
        if n == 3:
            continue
        beta = 4.0 ** (n - 2) * W0 ** (3 - n) * W2 ** n
        free = [k for k in range(3) if not t[k]]
        D = sum(np.outer(H[tuple(t[m] + (m == k) for m in range(3))], Ji[k]) for k in free)
        S = beta * det * (lam * np.trace(D) * np.eye(3) + mu * (D + D.T))
        for k in free:
            Y[tuple(t[m] + (m == k) for m in range(3))] += S @ Ji[k]
    return sum(Y[a][:, None, None, None] * _walsh(a)[None] for a in np.ndindex(2, 2, 2))


@pytest.mark.parametrize("q", [2, 3, 4])
def test_odd_centred_moments_vanish(q):
    xq, wq = rules.gauss_legendre(q)
    s = xq - 0.5
    for m in (1, 3):
        assert abs((wq * s ** m).sum()) < 1e-16
    assert abs(wq.sum() - 1.0) < 1e-15
    assert abs((wq * s * s).sum() - 1.0 / 12.0) < 1e-16


@pytest.mark.parametrize("q", [2, 3, 4])
def test_closed_form_equals_quadrature(q):
    rng = np.random.default_rng(100 + q)
    for trial in range(6):
        while True:
            J = np.diag(rng.uniform(0.3, 2.0, 3)) + 0.4 * rng.standard_normal((3, 3))
            if np.linalg.det(J) > 0.05:
                break
        lam, mu = rng.uniform(0.1, 5.0), rng.uniform(0.1, 5.0)
        Kl, Km = element_matrix_parts(1, q, J)
        K = lam * Kl + mu * Km
        x = rng.standard_normal((3, 2, 2, 2))
        # oracle dof order (c, a), a = ix + 2 (iy + 2 iz)
        ref = (K @ np.transpose(x, (0, 3, 2, 1)).reshape(-1)).reshape(3, 2, 2, 2).transpose(0, 3, 2, 1)
        y = closed_form_apply(x, J, lam, mu, q)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max(), (q, trial)


def test_closed_form_sees_every_term():
    """A plausible slip in the regrouping (a dropped monomial, the wrong moment weight, a
    transposed J^{-1}) changes the result: each breaks agreement with the oracle."""
    rng = np.random.default_rng(7)
    J = np.diag([1.3, 0.7, 1.1]) + 0.3 * rng.standard_normal((3, 3))
    lam, mu, q = 1.7, 0.9, 3
    Kl, Km = element_matrix_parts(1, q, J)
    x = rng.standard_normal((3, 2, 2, 2))
    ref = ((lam * Kl + mu * Km) @ np.transpose(x, (0, 3, 2, 1)).reshape(-1)).reshape(3, 2, 2, 2).transpose(0, 3, 2, 1)
    good = closed_form_apply(x, J, lam, mu, q)
    assert np.abs(good - ref).max() <= 1e-13 * np.abs(ref).max()
    bad_J = closed_form_apply(x, J.T, lam, mu, q)
    assert np.abs(bad_J - ref).max() > 1e-3 * np.abs(ref).max()
    # the second moment of the nodes instead of the rule's (1/4 instead of 1/12)
    bad_w = closed_form_apply(x, J, lam, mu, q, w2=0.25)
    assert np.abs(bad_w - ref).max() > 1e-3 * np.abs(ref).max()
