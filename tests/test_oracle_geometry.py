"""Pins of the non-affine (trilinear) oracle, oracle/geometry.py.

* affine vertex positions reproduce the affine oracle (element matrices by a different
  route, oracle.elasticity);
* the quadrature volume of a box whose interior vertices moved is the box volume
  (det J is a polynomial the Gauss rule integrates exactly);
* the energy of an affine displacement u = E x is (1/2) V (lambda tr(e)^2 + 2 mu e:e)
  on a distorted mesh (u = E x lies in the discrete space: the trilinear map is in Q_p);
* patch test: for u = E x the rows of every interior node vanish (the integrand
  sigma : adj(J)^T grad phi is a polynomial of degree <= p+1 per variable);
* infinitesimal rotations and translations lie in the nullspace;
* the assembled matrix is symmetric positive semi-definite with exactly six zero
  eigenvalues.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import elasticity, geometry, mesh as omesh


def _box(n=(3, 2, 2), seed=0, clamped=0):
    A = syn.random_rotation(seed) @ syn.SHEAR_A
    return syn.graded_mesh(n, seed=seed, L=(1.2, 0.9, 1.1), A=A, clamped_faces=clamped)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_affine_vertices_match_affine_oracle(p):
    mesh = _box(seed=p, clamped=0b000101)
    verts = syn.perturbed_vertices(mesh, amp=0.0)
    NE = mesh.num_elements
    rng = np.random.default_rng(p)
    lam, mu = rng.uniform(0.5, 2.0, NE), rng.uniform(0.5, 2.0, NE)
    x = syn.uniform_vector(mesh.num_dofs(p), seed=p)
    ref = elasticity.Operator(mesh, p, p + 2, lam, mu)
    op = geometry.TrilinearOperator(mesh, p, p + 2, verts, lam, mu)
    for c in (False, True):
        a, b = op.apply(x, constrained=c), ref.apply(x, constrained=c)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_node_coords_affine_case():
    mesh = _box(seed=3)
    for p in (1, 3):
        got = geometry.node_coords(mesh, syn.perturbed_vertices(mesh, amp=0.0), p)
        assert np.abs(got - omesh.node_coords(mesh, p)).max() <= 1e-14


@pytest.mark.parametrize("p", [1, 2, 3])
def test_volume_and_affine_energy(p):
    mesh = _box(n=(3, 3, 2), seed=10 + p)
    verts = syn.perturbed_vertices(mesh, amp=0.22, seed=p, interior_only=True)
    lam, mu = 1.7, 0.6
    op = geometry.TrilinearOperator(mesh, p, p + 2, verts, lam, mu)
    V = abs(np.linalg.det(mesh.A)) * np.prod([mesh.axis_nodes(a)[-1] - mesh.axis_nodes(a)[0] for a in range(3)])
    assert abs(op.volume() - V) <= 1e-13 * V
    E = np.random.default_rng(p).uniform(-1, 1, (3, 3))
    X = geometry.node_coords(mesh, verts, p)
    u = (X @ E.T).T.ravel()                     # component blocks
    eps = 0.5 * (E + E.T)
    want = 0.5 * V * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    got = 0.5 * u @ op.apply(u)
    assert abs(got - want) <= 1e-12 * abs(want)


@pytest.mark.parametrize("p,q", [(1, 2), (1, 3), (2, 4), (3, 4), (3, 5)])
def test_patch_test_interior_rows(p, q):
    mesh = syn.BoxMesh(n=(3, 3, 3), L=(1.0, 1.1, 0.9), A=syn.SHEAR_A)
    verts = syn.perturbed_vertices(mesh, amp=0.24, seed=7, interior_only=False)
    op = geometry.TrilinearOperator(mesh, p, q, verts, 1.3, 0.8)
    E = np.random.default_rng(1).uniform(-1, 1, (3, 3))
    u = (geometry.node_coords(mesh, verts, p) @ E.T).T.ravel()
    r = op.apply(u)
    Nx, Ny, Nz = omesh.grid_shape(mesh, p)
    gz, gy, gx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    inner = ((gx > 0) & (gx < Nx - 1) & (gy > 0) & (gy < Ny - 1) & (gz > 0) & (gz < Nz - 1)).ravel()
    inner3 = np.concatenate([inner, inner, inner])
    scale = np.abs(r).max()
    assert scale > 1e-3                         # boundary rows carry the traction
    assert np.abs(r[inner3]).max() <= 1e-12 * scale


@pytest.mark.parametrize("p", [1, 2, 4])
def test_rigid_motions_in_nullspace(p):
    mesh = syn.BoxMesh(n=(2, 2, 1), L=(1.0, 0.7, 0.5))
    verts = syn.perturbed_vertices(mesh, amp=0.24, seed=9, interior_only=False)
    op = geometry.TrilinearOperator(mesh, p, p + 2, verts, 2.0, 1.0)
    X = geometry.node_coords(mesh, verts, p)
    x = syn.uniform_vector(op.N, seed=1)
    nrm = np.linalg.norm(op.apply(x)) / np.linalg.norm(x)
    W = np.array([[0.0, 0.3, -0.7], [-0.3, 0.0, 0.2], [0.7, -0.2, 0.0]])
    for u in ((X @ W.T).T.ravel(), np.concatenate([np.full(len(X), 1.0), np.zeros(2 * len(X))])):
        assert np.linalg.norm(op.apply(u)) <= 1e-12 * nrm * np.linalg.norm(u)


def test_dense_symmetric_psd_six_zero_modes():
    mesh = syn.BoxMesh(n=(2, 1, 1), L=(1.0, 0.6, 0.8))
    verts = syn.perturbed_vertices(mesh, amp=0.24, seed=4, interior_only=False)
    A = geometry.TrilinearOperator(mesh, 2, 4, verts, 1.0, 1.0).dense()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev[0] >= -1e-12 * ev[-1]
    assert np.sum(ev < 1e-10 * ev[-1]) == 6


def test_inverted_element_rejected():
    mesh = syn.BoxMesh(n=(1, 1, 1))
    verts = syn.perturbed_vertices(mesh, amp=0.0)
    verts[7] = verts[0] - 0.1                   # the far corner pulled behind the origin
    with pytest.raises(ValueError):
        geometry.TrilinearOperator(mesh, 1, 3, verts, 1.0, 1.0)
