"""1D point sets and the Lagrange basis on the reference interval [0,1].

Paper Sec. 5.1.4 (benchmark discretization): (p+1) Gauss-Lobatto-Legendre nodes
per direction carry the basis, (p+2) Gauss-Legendre points per direction carry
the quadrature.  Eq. 6: the 3D basis is the tensor product of these 1D
Lagrange polynomials.  The reference interval is a free choice (the operator
does not depend on it); [0,1] is used here.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre(q: int):
    """q Gauss-Legendre points and weights on [0,1] (library rule, mapped)."""
    x, w = npleg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def gll_nodes(p: int) -> np.ndarray:
    """p+1 Gauss-Lobatto-Legendre nodes on [0,1]: the end points and the roots of P_p'."""
    if p < 1:
        raise ValueError("p must be >= 1")
    if p == 1:
        inner = np.zeros(0)
    else:
        c = np.zeros(p + 1)
        c[p] = 1.0
        inner = np.sort(npleg.legroots(npleg.legder(c)).real)
    x = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (x + 1.0)


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Values and first derivatives of the Lagrange polynomials of ``nodes`` at ``x``.

    Returns (V, dV) of shape (len(nodes), len(x)) with V[i,k] = l_i(x_k),
    computed from the product formula and the product rule.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((n, len(x)))
    dV = np.zeros((n, len(x)))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
        for k in range(n):
            if k == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[k]))
            for j in range(n):
                if j != i and j != k:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            dV[i] += term
    return V, dV


def gll_weights(p: int) -> np.ndarray:
    """Integrals of the GLL Lagrange polynomials over [0,1] (by an exact GL rule)."""
    nodes = gll_nodes(p)
    xq, wq = gauss_legendre(p + 1)
    V, _ = lagrange(nodes, xq)
    return V @ wq
