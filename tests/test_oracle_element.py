"""Pins of the oracle's element stiffness matrix.

* Exact rational element matrices from sympy for p=1,2 on the unit cube and on a
  rational sheared parallelepiped.  The symbolic route differs from the oracle's
  at every step: basis functions are composed with the inverse affine map and
  differentiated in physical coordinates by sympy (no J^{-T} formula), the
  bilinear form is written as  lambda div u div v + 2 mu eps(u):eps(v)  (the
  Hessian of the strain energy, instead of sigma(u):eps(v)), and the integrals
  are exact polynomial integrals (no quadrature).
* q-independence for q >= p+1 (exact integration on affine elements).
* Element-level rigid-body nullspace and symmetry.
"""
import functools
import itertools

import numpy as np
import pytest
import sympy as sp

from oracle import elasticity


def _sym_gram(p, Jrat):
    """Exact Gram tensor M[(a,k),(b,l)] = int_element d_k phi_a d_l phi_b dx (rationals)."""
    xi = sp.symbols("xi0:3")
    X = sp.symbols("X0:3")
    D = p + 1
    nodes = [sp.Rational(i, p) for i in range(p + 1)]  # GLL nodes are 0,1 (p=1) and 0,1/2,1 (p=2)

    def lag(i, v):
        e = sp.Integer(1)
        for j in range(D):
            if j != i:
                e *= (v - nodes[j]) / (nodes[i] - nodes[j])
        return e

    J = sp.Matrix(Jrat)
    detJ = J.det()
    ref_of_phys = J.inv() * sp.Matrix(X)
    phys_of_ref = {X[k]: (J * sp.Matrix(xi))[k] for k in range(3)}
    grads = []  # grads[a][k] as Poly in xi
    for iz, iy, ix in itertools.product(range(D), repeat=3):
        phi_phys = lag(ix, ref_of_phys[0]) * lag(iy, ref_of_phys[1]) * lag(iz, ref_of_phys[2])
        grads.append([sp.Poly(sp.expand(sp.diff(phi_phys, X[k]).subs(phys_of_ref)), *xi, domain="QQ")
                      for k in range(3)])

    def integ(poly):
        s = sp.Rational(0)
        for (a, b, c), coef in poly.terms():
            s += coef / ((a + 1) * (b + 1) * (c + 1))
        return s

    n = D ** 3
    M = np.empty((n, 3, n, 3), dtype=object)
    for a in range(n):
        for b in range(a, n):
            for k in range(3):
                for l in range(3):
                    v = integ(grads[a][k] * grads[b][l]) * detJ
                    M[a, k, b, l] = v
                    M[b, l, a, k] = v
    return M


def _sym_element_parts(p, Jrat):
    M = _sym_gram(p, Jrat)
    n = M.shape[0]
    Kl = np.zeros((3 * n, 3 * n))
    Km = np.zeros((3 * n, 3 * n))
    for c in range(3):
        for d in range(3):
            for a in range(n):
                for b in range(n):
                    # lambda div(phi_a e_c) div(phi_b e_d)
                    Kl[c * n + a, d * n + b] = float(M[a, c, b, d])
                    # 2 mu eps(phi_a e_c):eps(phi_b e_d) = mu (delta_cd grad.grad + d_d phi_a d_c phi_b)
                    v = M[a, d, b, c]
                    if c == d:
                        v = v + M[a, 0, b, 0] + M[a, 1, b, 1] + M[a, 2, b, 2]
                    Km[c * n + a, d * n + b] = float(v)
    return Kl, Km


SHEAR = [[sp.Rational(1, 2), sp.Rational(1, 15), sp.Rational(1, 20)],
         [0, sp.Rational(1, 3), sp.Rational(1, 20)],
         [0, 0, sp.Rational(1, 4)]]
CUBE = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]


@functools.lru_cache(maxsize=None)
def _sym_cached(p, which):
    return _sym_element_parts(p, CUBE if which == "cube" else SHEAR)


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("which", ["cube", "shear"])
def test_element_matrix_exact_sympy(p, which):
    Kl_s, Km_s = _sym_cached(p, which)
    J = np.array(CUBE if which == "cube" else SHEAR, dtype=float)
    Kl, Km = elasticity.element_matrix_parts(p, p + 2, J)
    scale = max(np.abs(Kl_s).max(), np.abs(Km_s).max())
    assert np.abs(Kl - Kl_s).max() <= 1e-14 * scale
    assert np.abs(Km - Km_s).max() <= 1e-14 * scale


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_q_independence(p):
    rng = np.random.default_rng(p)
    J = np.diag(rng.uniform(0.5, 2, 3)) + 0.2 * np.triu(rng.standard_normal((3, 3)), 1)
    ref = elasticity.element_matrix_parts(p, p + 1, J)
    for q in (p + 2, p + 5):
        other = elasticity.element_matrix_parts(p, q, J)
        for a, b in zip(ref, other):
            assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_element_rigid_modes_and_symmetry(p):
    rng = np.random.default_rng(10 + p)
    J = rng.standard_normal((3, 3)) * 0.3 + np.eye(3)
    if np.linalg.det(J) < 0:
        J[:, 0] *= -1
    Kl, Km = elasticity.element_matrix_parts(p, p + 2, J)
    K = 1.7 * Kl + 0.6 * Km
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    # nodal reference coordinates of the element, mapped by J
    from oracle import rules
    x1 = rules.gll_nodes(p)
    Z, Y, X = np.meshgrid(x1, x1, x1, indexing="ij")
    R = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1) @ J.T
    modes = []
    for c in range(3):
        u = np.zeros((3, R.shape[0]))
        u[c] = 1.0
        modes.append(u.ravel())
    for w in np.eye(3):
        u = np.cross(np.broadcast_to(w, R.shape), R).T
        modes.append(u.ravel())
    for u in modes:
        assert np.linalg.norm(K @ u) <= 1e-12 * np.abs(K).max() * np.linalg.norm(u)
    ev = np.linalg.eigvalsh(K)
    assert ev[0] >= -1e-12 * ev[-1]
    assert np.sum(ev > 1e-10 * ev[-1]) == K.shape[0] - 6   # exactly 6 zero modes
