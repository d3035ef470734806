"""Pins of the oracle's general material forms (oracle/material.py): per-point and
anisotropic Voigt stiffness (Sec. 2.1 eq. 2; data per quadrature point, Sec. 4.5).

The B-matrix route is checked against the isotropic tensor route of
oracle/elasticity.py (itself pinned by exact rational element matrices), against the
closed-form energy of affine displacement fields for arbitrary stiffness (uniaxial and
simple-shear fields isolate single Voigt entries, so a wrong index order or a missing
engineering-shear factor fails), and against the rigid-body nullspace, symmetry and
positivity."""
import numpy as np
import pytest

import synthetic as syn
from oracle import elasticity, material, mesh as omesh


def _mesh(seed, n=(3, 2, 2), clamped=0):
    A = syn.random_rotation(seed) @ syn.SHEAR_A
    return syn.graded_mesh(n, seed=seed, L=(1.2, 0.9, 1.1), A=A, clamped_faces=clamped)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_isotropic_voigt_equals_tensor_route(p):
    m = _mesh(p, clamped=0b000101)
    NE = m.num_elements
    rng = np.random.default_rng(p)
    lam, mu = rng.uniform(0.3, 2.0, NE), rng.uniform(0.3, 2.0, NE)
    ref = elasticity.Operator(m, p, p + 2, lam, mu)
    gen = material.GeneralOperator(m, p, p + 2, material.isotropic_voigt(lam, mu))
    x = syn.uniform_vector(m.num_dofs(p), seed=4)
    for constrained in (False, True):
        a, b = gen.apply(x, constrained), ref.apply(x, constrained)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_constant_per_point_equals_per_element():
    m = _mesh(5)
    q = 4
    C = syn.random_spd_stiffness(m.num_elements, seed=2)
    a = material.GeneralOperator(m, 2, q, C)
    b = material.GeneralOperator(m, 2, q, np.repeat(C[:, None], q ** 3, axis=1))
    x = syn.uniform_vector(m.num_dofs(2), seed=1)
    assert np.allclose(a.apply(x), b.apply(x), rtol=0, atol=1e-13 * np.abs(b.apply(x)).max())


def _affine_nodal(m, p, E):
    X = omesh.node_coords(m, p)                 # physical node coordinates [Nn, 3]
    return (X @ E.T).T.reshape(-1)              # component blocks


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("per_point", [False, True])
def test_affine_energy_closed_form(p, per_point):
    """x^T A x / 2 of u(x) = E x equals sum_e sum_alpha w detJ eps_V^T C eps_V / 2 (constant
    strain, integrated exactly) for arbitrary stiffness per element or per point."""
    m = _mesh(7 + p)
    q = p + 2
    NE = m.num_elements
    C = syn.random_spd_stiffness(NE, seed=3)
    if per_point:
        rng = np.random.default_rng(9)
        C = C[:, None] * rng.uniform(0.5, 1.5, (NE, q ** 3, 1, 1))
    op = material.GeneralOperator(m, p, q, C)
    rng = np.random.default_rng(10)
    for _ in range(3):
        E = rng.uniform(-1.0, 1.0, (3, 3))
        x = _affine_nodal(m, p, E)
        assert abs(0.5 * x @ op.apply(x) - op.energy_of_affine(E)) <= 1e-12 * op.energy_of_affine(E)


def test_uniaxial_and_shear_fields_isolate_voigt_entries():
    """On an unsheared box of volume V: u = (a x, 0, 0) has energy a^2 C_11 V / 2 and
    u = (g y, 0, 0) (engineering shear g in the xy entry, Voigt index 6) g^2 C_66 V / 2."""
    m = syn.BoxMesh(n=(2, 2, 2), L=(1.0, 2.0, 0.5))
    V = 1.0 * 2.0 * 0.5
    C = syn.random_spd_stiffness(1, seed=21)[0]
    op = material.GeneralOperator(m, 2, 4, np.broadcast_to(C, (8, 6, 6)))
    for E, k in ((np.diag([0.7, 0.0, 0.0]), 0), (np.array([[0, 0.4, 0], [0, 0, 0], [0, 0, 0]]), 5),
                 (np.array([[0, 0, 0], [0, 0, 0.3], [0, 0, 0]]), 3), (np.array([[0, 0, 0.2], [0, 0, 0], [0, 0, 0]]), 4)):
        x = _affine_nodal(m, 2, E)
        amp = E.sum()
        assert abs(0.5 * x @ op.apply(x) - 0.5 * amp ** 2 * C[k, k] * V) <= 1e-12 * abs(C[k, k])


@pytest.mark.parametrize("p", [1, 2])
def test_nullspace_symmetry_positivity(p):
    m = _mesh(12 + p)
    q = p + 2
    C = syn.random_spd_stiffness(m.num_elements, seed=4)
    C = C[:, None] * np.random.default_rng(5).uniform(0.5, 1.5, (m.num_elements, q ** 3, 1, 1))
    op = material.GeneralOperator(m, p, q, C)
    X = omesh.node_coords(m, p)
    nrm = np.linalg.norm(op.apply(syn.uniform_vector(op.N, seed=6)))
    for R in (np.zeros((3, 3)), np.array([[0, -1, 0], [1, 0, 0], [0, 0, 0.0]])):
        for t in (np.array([1.0, -2.0, 0.5]),):
            u = (X @ R.T + t).T.reshape(-1)
            assert np.linalg.norm(op.apply(u)) <= 1e-12 * nrm * np.linalg.norm(u)
    x, y = syn.uniform_vector(op.N, seed=7), syn.uniform_vector(op.N, seed=8)
    assert abs(y @ op.apply(x) - x @ op.apply(y)) <= 1e-12 * abs(x @ op.apply(x))
    assert x @ op.apply(x) > 0


def test_packing_roundtrip():
    C = syn.random_spd_stiffness(3, seed=1)
    assert np.array_equal(material.unpack_upper(material.packed_upper(C)), C)


@pytest.mark.parametrize("p", [1, 2])
def test_dense_and_diagonal(p):
    """The assembled matrix reproduces the matrix-free apply column by column (a different
    route: K^e formed, not applied), its diagonal equals diagonal(), and for per-element
    isotropic stiffness both equal the tensor-route oracle's dense matrix and diagonal."""
    m = _mesh(20 + p, n=(2, 2, 1), clamped=0b000001)
    NE = m.num_elements
    q = p + 2
    rng = np.random.default_rng(p)
    lq = rng.uniform(0.3, 2.0, (NE, q ** 3))
    mq = rng.uniform(0.3, 2.0, (NE, q ** 3))
    gen = material.GeneralOperator(m, p, q, material.isotropic_voigt(lq, mq))
    N = m.num_dofs(p)
    for constrained in (False, True):
        A = gen.dense(constrained)
        cols = np.stack([gen.apply(np.eye(N)[j], constrained) for j in range(N)], axis=1)
        assert np.abs(A - cols).max() <= 1e-13 * np.abs(A).max()
        assert np.abs(np.diag(A) - gen.diagonal(constrained)).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(gen.element_matrix(NE - 1) - gen.element_matrix(NE - 1).T).max() <= 1e-13
    lam, mu = lq[:, 0], mq[:, 0]
    iso = material.GeneralOperator(m, p, q, material.isotropic_voigt(lam, mu))
    ref = elasticity.Operator(m, p, q, lam, mu)
    for constrained in (False, True):
        Ar = ref.dense(constrained)
        assert np.abs(iso.dense(constrained) - Ar).max() <= 1e-13 * np.abs(Ar).max()
        assert np.abs(iso.diagonal(constrained) - ref.diagonal(constrained)).max() <= 1e-13 * np.abs(Ar).max()
