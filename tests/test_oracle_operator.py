"""Pins of the oracle's global operator and load vectors.

Invariants of the linear-elasticity operator (rigid-body nullspace, symmetry,
positive semi-definiteness, patch test with constant strain, closed-form energy
of an affine field, linearity in (lambda, mu), scaling, rotation equivariance)
and closed forms of the load vectors.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import elasticity, mesh as omesh, rules


def _op(mesh, p, lam=None, mu=None, seed=3):
    NE = mesh.num_elements
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.5, 2.0, NE) if lam is None else lam
    mu = rng.uniform(0.5, 2.0, NE) if mu is None else mu
    return elasticity.Operator(mesh, p, p + 2, lam, mu)


def _fields(mesh, p):
    return omesh.node_coords(mesh, p)


def _rigid_modes(R):
    modes = []
    for c in range(3):
        u = np.zeros((3, len(R)))
        u[c] = 1.0
        modes.append(u.ravel())
    for w in np.eye(3):
        modes.append(np.cross(np.broadcast_to(w, R.shape), R).T.ravel())
    return modes


def _norm_est(op, seed=0):
    x = np.random.default_rng(seed).uniform(-1, 1, op.N)
    return np.linalg.norm(op.apply(x)) / np.linalg.norm(x)


MESHES = {
    "cube": lambda: syn.BoxMesh(n=(2, 3, 2), L=(1.0, 1.3, 0.7)),
    "sheared": lambda: syn.BoxMesh(n=(3, 2, 2), L=(1.25, 1.25, 1.0), A=syn.SHEAR_A),
    "graded_rot": lambda: syn.graded_mesh((2, 2, 3), seed=4, A=syn.random_rotation(2) @ np.diag([1.0, 0.8, 1.2])),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("p", [1, 2, 3])
def test_rigid_symmetry_psd(name, p):
    mesh = MESHES[name]()
    op = _op(mesh, p)
    nrm = _norm_est(op)
    R = _fields(mesh, p)
    for u in _rigid_modes(R):
        assert np.linalg.norm(op.apply(u)) <= 1e-13 * nrm * np.linalg.norm(u)
    rng = np.random.default_rng(1)
    x, y = rng.uniform(-1, 1, (2, op.N))
    xAy, yAx = x @ op.apply(y), y @ op.apply(x)
    assert abs(xAy - yAx) <= 1e-13 * nrm * np.linalg.norm(x) * np.linalg.norm(y)
    for _ in range(3):
        u = rng.uniform(-1, 1, op.N)
        assert u @ op.apply(u) >= -1e-13 * nrm * (u @ u)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_rigid_modes_high_order_single_element(p):
    mesh = syn.BoxMesh(n=(1, 1, 1), A=syn.SHEAR_A)
    op = _op(mesh, p)
    A = op.dense()
    ev = np.linalg.eigvalsh(A)
    assert np.sum(np.abs(ev) <= 1e-11 * ev[-1]) == 6
    assert ev[0] >= -1e-11 * ev[-1]


def test_rigid_modes_p8():
    mesh = syn.BoxMesh(n=(2, 1, 1), A=syn.SHEAR_A)
    op = _op(mesh, 8)
    nrm = _norm_est(op)
    for u in _rigid_modes(_fields(mesh, 8)):
        assert np.linalg.norm(op.apply(u)) <= 1e-12 * nrm * np.linalg.norm(u)


@pytest.mark.parametrize("p", [2, 3])
def test_patch_test_constant_strain(p):
    """u = Gx + c: interior rows vanish; face rows equal (sigma n) times face weights."""
    A = syn.SHEAR_A
    mesh = syn.BoxMesh(n=(3, 2, 2), L=(1.2, 1.0, 0.9), A=A)
    lam, mu = 1.3, 0.7
    op = _op(mesh, p, lam=np.full(mesh.num_elements, lam), mu=np.full(mesh.num_elements, mu))
    rng = np.random.default_rng(7)
    Gm = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    R = _fields(mesh, p)
    u = (R @ Gm.T + c).T.ravel()
    y = op.apply(u).reshape(3, -1)
    Nx, Ny, Nz = omesh.grid_shape(mesh, p)
    gz, gy, gx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    gx, gy, gz = gx.ravel(), gy.ravel(), gz.ravel()
    interior = (gx > 0) & (gx < Nx - 1) & (gy > 0) & (gy < Ny - 1) & (gz > 0) & (gz < Nz - 1)
    scale = np.abs(y).max()
    assert np.abs(y[:, interior]).max() <= 1e-12 * scale
    # closed form on the x+ face: sigma n |A e_y x A e_z| h_y h_z w_iy w_iz for nodes
    # whose tangential local indices are strictly inside an element face.
    eps = 0.5 * (Gm + Gm.T)
    sigma = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
    nvec = np.cross(A[:, 1], A[:, 2])
    area = np.linalg.norm(nvec)
    nvec /= area
    hy, hz = 1.0 / 2, 0.9 / 2
    w = rules.gll_weights(p)
    for (iy, iz) in [(1, 1), (p - 1, 1), (1, p - 1)]:
        node = (Nx - 1) + Nx * (iy + Ny * iz)
        expect = sigma @ nvec * area * hy * hz * w[iy] * w[iz]
        assert np.allclose(y[:, node], expect, atol=1e-12 * scale)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_energy_of_affine_field(p):
    mesh = syn.BoxMesh(n=(2, 2, 3), L=(1.1, 0.9, 1.3), A=syn.SHEAR_A @ np.diag([1.0, 1.1, 0.9]))
    lam, mu = 2.0, 0.8
    op = _op(mesh, p, lam=np.full(mesh.num_elements, lam), mu=np.full(mesh.num_elements, mu))
    Gm = np.random.default_rng(5).standard_normal((3, 3))
    R = _fields(mesh, p)
    u = (R @ Gm.T).T.ravel()
    eps = 0.5 * (Gm + Gm.T)
    vol = np.linalg.det(mesh.A) * np.prod(mesh.L)
    energy = vol * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    assert abs(u @ op.apply(u) - energy) <= 1e-12 * abs(energy)


def test_linear_in_lame_and_scaling():
    mesh = syn.graded_mesh((2, 2, 2), seed=1)
    NE = mesh.num_elements
    rng = np.random.default_rng(2)
    l1, l2, m1, m2 = rng.uniform(0.5, 2, (4, NE))
    x = rng.uniform(-1, 1, mesh.num_dofs(2))
    a = elasticity.Operator(mesh, 2, 4, l1 + l2, m1 + m2).apply(x)
    b = elasticity.Operator(mesh, 2, 4, l1, m1).apply(x) + elasticity.Operator(mesh, 2, 4, l2, m2).apply(x)
    assert np.allclose(a, b, rtol=0, atol=1e-13 * np.abs(a).max())
    s = 2.5
    big = syn.BoxMesh(n=mesh.n, grade=[s * g for g in mesh.grade])
    c = elasticity.Operator(big, 2, 4, l1, m1).apply(x)
    d = elasticity.Operator(mesh, 2, 4, l1, m1).apply(x)
    assert np.allclose(c, s * d, rtol=0, atol=1e-13 * np.abs(c).max())


@pytest.mark.parametrize("p", [1, 3])
def test_rotation_equivariance(p):
    base = syn.SHEAR_A @ np.diag([1.0, 0.9, 1.2])
    Rm = syn.random_rotation(11)
    m0 = syn.graded_mesh((2, 2, 2), seed=6, A=base)
    m1 = syn.graded_mesh((2, 2, 2), seed=6, A=Rm @ base)
    op0, op1 = _op(m0, p, seed=9), _op(m1, p, seed=9)
    x = np.random.default_rng(3).uniform(-1, 1, op0.N).reshape(3, -1)
    y0 = op0.apply(x.ravel()).reshape(3, -1)
    y1 = op1.apply((Rm @ x).ravel()).reshape(3, -1)
    assert np.allclose(y1, Rm @ y0, rtol=0, atol=1e-12 * np.abs(y0).max())


def test_constrained_operator():
    mesh = syn.BoxMesh(n=(2, 2, 2), clamped_faces=0b000101)
    op = _op(mesh, 2)
    x = np.random.default_rng(0).uniform(-1, 1, op.N)
    y = op.apply(x, constrained=True)
    xt = x.copy()
    xt[op.ess] = 0
    y2 = op.apply(xt)
    y2[op.ess] = x[op.ess]
    assert np.array_equal(y, y2)
    A = op.dense(constrained=True)
    assert np.allclose(A @ x, y, atol=1e-13 * np.abs(y).max())
    assert np.all(np.linalg.eigvalsh(A) > 0)  # SPD once clamped


# ------------------------------------------------------------------------------- loads

def test_body_force_config1_closed_form():
    mesh = syn.unit_cube_4()
    p = 2
    F = elasticity.body_force_vector(mesh, p, 4, (0.0, 0.0, -1.0)).reshape(3, -1)
    assert np.allclose(F[:2], 0.0)
    assert abs(F[2].sum() + 1.0) < 1e-14
    # nodal values are products of per-axis GLL weights times element size h = 1/4,
    # with shared element ends counted from both sides
    w = rules.gll_weights(p)
    ax = np.zeros(9)
    for e in range(4):
        ax[2 * e:2 * e + 3] += w * 0.25
    expect = -np.einsum("z,y,x->zyx", ax, ax, ax).ravel()
    assert np.allclose(F[2], expect, atol=1e-15)
    assert np.isclose(ax[0], 1.0 / 24) and np.isclose(ax[1], 1.0 / 6)


@pytest.mark.parametrize("face", range(6))
def test_traction_sum(face):
    mesh = syn.BoxMesh(n=(2, 3, 2), L=(1.2, 0.8, 1.5), A=syn.SHEAR_A)
    t = np.array([0.3, -1.0, 2.0])
    F = elasticity.traction_vector(mesh, 3, 5, face, t).reshape(3, -1)
    axis = face // 2
    t1, t2 = [a for a in range(3) if a != axis]
    area = np.linalg.norm(np.cross(mesh.A[:, t1], mesh.A[:, t2])) * mesh.L[t1] * mesh.L[t2]
    assert np.allclose(F.sum(1), t * area, rtol=1e-13)


def test_body_force_sum_graded():
    mesh = syn.graded_mesh((3, 2, 2), seed=2, L=(2.0, 1.0, 0.5), A=syn.SHEAR_A)
    F = elasticity.body_force_vector(mesh, 3, 5, (1.0, 2.0, -3.0)).reshape(3, -1)
    vol = np.linalg.det(mesh.A) * 2.0 * 1.0 * 0.5
    assert np.allclose(F.sum(1), np.array([1.0, 2.0, -3.0]) * vol, rtol=1e-13)


@pytest.mark.parametrize("face", [1, 2, 5])
def test_traction_nodal_values_closed_form(face):
    """On a graded sheared box the traction load on a face node is t times the face area
    factor |A e_1 x A e_2| times, per in-face axis, the sum over the adjacent element edges of
    h_e w_i (GLL weights: the integral of each 1D Lagrange factor), and zero off the face;
    its first moments are t times the integrals of the in-face reference coordinates."""
    mesh = syn.graded_mesh((3, 2, 4), seed=8, L=(1.1, 0.7, 1.4), A=syn.SHEAR_A)
    p = 3
    t = np.array([0.4, -1.0, 0.7])
    F = elasticity.traction_vector(mesh, p, p + 2, face, t).reshape(3, -1)
    axis, side = face // 2, face % 2
    t1, t2 = [a for a in range(3) if a != axis]
    w = rules.gll_weights(p)
    ax = []
    for a in (t1, t2):
        X = mesh.axis_nodes(a)
        s = np.zeros(mesh.n[a] * p + 1)
        for e in range(mesh.n[a]):
            s[e * p:e * p + p + 1] += w * (X[e + 1] - X[e])
        ax.append(s)
    area = np.linalg.norm(np.cross(mesh.A[:, t1], mesh.A[:, t2]))
    shape = omesh.grid_shape(mesh, p)
    idx = np.indices(shape[::-1]).reshape(3, -1)[::-1]          # (gx, gy, gz) of every node
    on = idx[axis] == (0 if side == 0 else shape[axis] - 1)
    expect = np.zeros(idx.shape[1])
    expect[on] = area * ax[0][idx[t1][on]] * ax[1][idx[t2][on]]
    for c in range(3):
        assert np.allclose(F[c], t[c] * expect, rtol=1e-13, atol=1e-15)
    # first moments: sum_a F_a X_a = t * area * int X dX over the face (reference coordinates)
    g1 = omesh.axis_node_coords(mesh, t1, p)[idx[t1]]
    L1, L2 = mesh.axis_nodes(t1)[-1], mesh.axis_nodes(t2)[-1]
    assert np.allclose((F * g1).sum(1), t * area * 0.5 * L1 ** 2 * L2, rtol=1e-12)
