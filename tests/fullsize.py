"""The operator-sweep workload at full size and its oracle apply, shared by the GPU parity
tests (a helper module, not a test module).

The sheared box of the sweep: (120/p, 120/p, 96/p) elements (p = 5, 7: (24,24,19),
(17,17,14)), ~4.2M dofs, two materials E in {1, 100}, nu = 0.3 (seed 1), x ~ U[-1,1]
(seed 0).  The constrained form clamps the x- and z+ faces.  Each oracle apply
(oracle.elasticity, element matrices by direct quadrature) is computed once per process
and reused by every test that compares a GPU form with it.
"""
from __future__ import annotations

import functools

import numpy as np

import synthetic as syn
from oracle import elasticity, mesh as omesh

CLAMP = 0b100001          # x- and z+ clamped in the constrained form
TOL = {0: 1e-12, 1: 1e-5}


def mesh(p: int, clamped: bool = False):
    m = syn.sheared_box_mesh(p)
    if clamped:
        m.clamped_faces = CLAMP
    return m


@functools.lru_cache(maxsize=None)
def lame(p: int):
    return syn.two_material_lame(syn.sheared_box_mesh(p).num_elements, seed=1)


@functools.lru_cache(maxsize=8)
def x_vec(p: int) -> np.ndarray:
    return syn.uniform_vector(syn.sheared_box_mesh(p).num_dofs(p), seed=0)


@functools.lru_cache(maxsize=16)
def oracle_apply(p: int, clamped: bool = False) -> np.ndarray:
    """The oracle's y = A x (constrained form when clamped) on the full-size box."""
    lam, mu = lame(p)
    op = elasticity.Operator(mesh(p, clamped), p, p + 2, lam, mu)
    return op.apply(x_vec(p), constrained=clamped)


@functools.lru_cache(maxsize=8)
def single_material_dofs(p: int):
    """(soft, stiff): dof masks of the nodes all of whose elements have E = 1 (soft) or
    all have E = 100 (stiff).  A wrong value at a node of the soft material is small
    against the norm of the whole output; the error is also measured on each set."""
    m = syn.sheared_box_mesh(p)
    lam, _ = lame(p)
    stiff_e = lam > 10 * lam.min()
    en = omesh.element_nodes(m, p)
    Nn = m.num_nodes(p)
    has_stiff = np.zeros(Nn, dtype=bool)
    has_soft = np.zeros(Nn, dtype=bool)
    has_stiff[en[stiff_e].ravel()] = True
    has_soft[en[~stiff_e].ravel()] = True
    return np.tile(has_soft & ~has_stiff, 3), np.tile(has_stiff & ~has_soft, 3)


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check_whole_vector(y: np.ndarray, ref: np.ndarray, p: int, dtype: int, what: str):
    """Relative 2-norm error over the whole output and over each single-material node set."""
    soft, stiff = single_material_dofs(p)
    errs = (rel(y, ref), rel(y[soft], ref[soft]), rel(y[stiff], ref[stiff]))
    print(f"{what}: rel err whole {errs[0]:.2e} soft {errs[1]:.2e} stiff {errs[2]:.2e}", flush=True)
    assert soft.any() and stiff.any()
    assert max(errs) <= TOL[dtype], (what, errs)


# ---- the first 1/8 of the box (n // 2 elements per axis, same element size), where the
# oracles of the general forms (per-point quadrature sums) finish in seconds
def eighth(p: int):
    m = syn.sheared_box_mesh(p)
    n = tuple(max(1, k // 2) for k in m.n)
    return syn.BoxMesh(n=n, L=tuple(m.L[a] * n[a] / m.n[a] for a in range(3)), A=m.A, x0=m.x0)


def eighth_lame(p: int):
    return syn.two_material_lame(eighth(p).num_elements, seed=1)


def eighth_x(p: int) -> np.ndarray:
    return syn.uniform_vector(eighth(p).num_dofs(p), seed=0)


def eighth_vertices(p: int) -> np.ndarray:
    """The box's vertices, interior ones moved by up to 0.2 of the spacing (seed 17)."""
    return syn.perturbed_vertices(eighth(p), amp=0.2, seed=17)


@functools.lru_cache(maxsize=2)
def eighth_trilinear_oracle(p: int) -> np.ndarray:
    """The oracle's y = A x (unconstrained) on the distorted 1/8 box (trilinear hexahedra)."""
    from oracle import geometry
    lam, mu = eighth_lame(p)
    op = geometry.TrilinearOperator(eighth(p), p, p + 2, eighth_vertices(p), lam, mu)
    return op.apply(eighth_x(p))
