"""Pins of the oracle's 1D rules and Lagrange basis (closed forms and textbook tables)."""
import json
import os

import numpy as np
import pytest

from oracle import rules

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("q", range(1, 13))
def test_gauss_legendre_exactness(q):
    x, w = rules.gauss_legendre(q)
    assert np.all((x > 0) & (x < 1))
    for k in range(2 * q):
        assert abs(w @ x ** k - 1.0 / (k + 1)) < 1e-14
    # not exact one degree higher (the defect shrinks quickly with q)
    if q <= 6:
        assert abs(w @ x ** (2 * q) - 1.0 / (2 * q + 1)) > 1e-9


@pytest.mark.parametrize("p", range(1, 10))
def test_gll_nodes_and_weights(p):
    x = rules.gll_nodes(p)
    assert len(x) == p + 1 and x[0] == 0.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    assert np.allclose(x + x[::-1], 1.0, atol=1e-15)
    w = rules.gll_weights(p)
    for k in range(2 * p):  # Lobatto rule with p+1 nodes is exact to degree 2p-1
        assert abs(w @ x ** k - 1.0 / (k + 1)) < 1e-14


def test_gll_textbook_table():
    with open(os.path.join(GOLD, "lobatto_rules.json")) as f:
        g = json.load(f)
    for p in (2, 3):
        ref = g[f"p{p}"]
        assert np.allclose(rules.gll_nodes(p), ref["nodes"], atol=1e-15)
        assert np.allclose(rules.gll_weights(p), ref["weights"], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 10))
def test_lagrange_basis(p):
    nodes = rules.gll_nodes(p)
    V, dV = rules.lagrange(nodes, nodes)
    assert np.allclose(V, np.eye(p + 1), atol=1e-14)
    pts = np.linspace(0, 1, 17)
    V, dV = rules.lagrange(nodes, pts)
    assert np.allclose(V.sum(0), 1.0, atol=1e-13)
    assert np.allclose(dV.sum(0), 0.0, atol=1e-10)
    # interpolation of x^p and its derivative is exact
    f = nodes ** p
    assert np.allclose(f @ V, pts ** p, atol=1e-13)
    assert np.allclose(f @ dV, p * pts ** (p - 1), atol=1e-10)
    # derivative of a lower-degree polynomial, e.g. (2x-1)^(p-1)
    f = (2 * nodes - 1) ** (p - 1)
    assert np.allclose(f @ dV, 2 * (p - 1) * (2 * pts - 1) ** max(p - 2, 0) * (p > 1), atol=1e-10)
