"""Pins of the oracle's solver references (textbook bounds, reproduction, physics)."""
import numpy as np
import pytest

import synthetic as syn
from oracle import elasticity, mesh as omesh, solvers


def _system(mesh, p, lam=1.0, mu=1.0):
    op = elasticity.Operator(mesh, p, p + 2, np.full(mesh.num_elements, lam), np.full(mesh.num_elements, mu))
    return op, op.dense(constrained=True), op.diagonal(constrained=True)


def test_splitmix64_reference_values():
    # First outputs of SplitMix64 seeded with 0 (published reference sequence):
    # 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    v = solvers.splitmix64_uniform(0, 3)
    expect = [2.0 * ((z >> 11) / 2.0 ** 53) - 1.0 for z in ref]
    assert np.array_equal(v, expect)


def test_config1_direct_solve():
    mesh = syn.unit_cube_4(clamped=True)
    op, A, _ = _system(mesh, 2)
    b = elasticity.body_force_vector(mesh, 2, 4, (0.0, 0.0, -1.0))
    b[op.ess] = 0.0
    u = solvers.solve_dense(A, b)
    assert np.linalg.norm(A @ u - b) <= 1e-13 * np.linalg.norm(b)
    assert np.all(u[op.ess] == 0.0)
    uz = u.reshape(3, -1)[2]
    assert uz.min() < 0 and uz[~op.ess[:op.N // 3]].max() <= 1e-12  # sags everywhere


def test_cantilever_tip_deflection_beam_theory():
    """End-loaded 8:1:1 cantilever, E=1, nu=0.3: tip sag ~ PL^3/(3EI) (+ shear)."""
    mesh = syn.cantilever_mesh(8, 1, 1)
    lam, mu = syn.lame_from_young_poisson(1.0, 0.3)
    p = 4
    op, A, _ = _system(mesh, p, float(lam), float(mu))
    b = elasticity.traction_vector(mesh, p, p + 2, 1, (0.0, 0.0, -1.0))
    b[op.ess] = 0.0
    u = solvers.solve_dense(A, b).reshape(3, -1)
    R = omesh.node_coords(mesh, p)
    tip = np.isclose(R[:, 0], 8.0)
    defl = -u[2, tip].mean()
    euler = 1.0 * 8.0 ** 3 / (3 * 1.0 / 12.0)   # 2048
    assert 0.95 * euler < defl < 1.05 * euler * 1.012


def test_power_iteration_bounds():
    mesh = syn.BoxMesh(n=(3, 2, 2), clamped_faces=1)
    op, A, d = _system(mesh, 2, 1.5, 0.7)
    ev = np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))
    v0 = solvers.splitmix64_uniform(7, op.N)
    v0[op.ess] = 0
    lam10 = solvers.power_iteration(A, d, v0, 10)
    lam50 = solvers.power_iteration(A, d, v0, 200)
    assert lam10 <= ev[-1] * (1 + 1e-12)
    assert lam10 >= 0.8 * ev[-1]
    assert abs(lam50 - ev[-1]) <= 1e-3 * ev[-1]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_chebyshev_error_bound(k):
    """With [lmin,lmax] containing spec(D^{-1}A), |e_k|_A <= |e_0|_A / T_k(theta/delta)."""
    mesh = syn.BoxMesh(n=(2, 2, 2), clamped_faces=1 | 4)
    op, A, d = _system(mesh, 2)
    ev = np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))
    lmin, lmax = ev[0], ev[-1]
    rng = np.random.default_rng(k)
    xstar = rng.uniform(-1, 1, op.N)
    b = A @ xstar
    x0 = rng.uniform(-1, 1, op.N)
    xk = solvers.chebyshev_smooth(A, d, b, x0, k, lmin, lmax)
    eA = lambda e: np.sqrt(e @ A @ e)
    sig = (lmax + lmin) / (lmax - lmin)
    Tk = np.cosh(k * np.arccosh(sig))
    assert eA(xk - xstar) <= eA(x0 - xstar) / Tk * (1 + 1e-9)
    if k == 1:  # one step is damped Jacobi with weight 1/theta
        theta = 0.5 * (lmax + lmin)
        assert np.allclose(xk, x0 + (b - A @ x0) / d / theta, atol=1e-13)


@pytest.mark.parametrize("pc,pf", [(1, 2), (2, 4), (4, 8), (3, 6), (1, 3)])
def test_p_prolongation_reproduces_polynomials(pc, pf):
    mesh = syn.graded_mesh((2, 1, 2), seed=3, A=syn.SHEAR_A)
    P = solvers.prolongation_p(mesh, pc, pf)
    Rc, Rf = omesh.node_coords(mesh, pc), omesh.node_coords(mesh, pf)
    # a polynomial of degree pc in each reference variable is in both spaces
    Xc = (np.linalg.inv(mesh.A) @ Rc.T).T
    Xf = (np.linalg.inv(mesh.A) @ Rf.T).T
    f = lambda X: np.stack([X[:, 0] ** pc * X[:, 1] + 1, X[:, 2] ** pc - X[:, 1], (X[:, 0] * X[:, 1] * X[:, 2]) ** pc])
    uc, uf = f(Xc).ravel(), f(Xf).ravel()
    assert np.allclose(P @ uc, uf, atol=1e-12)


def test_h_prolongation_reproduces_trilinear():
    fine = syn.graded_mesh((4, 3, 2), seed=8, A=syn.SHEAR_A)
    coarse_ax = [fine.axis_nodes(a)[[i for i in range(0, fine.n[a] + 1, 2)] + ([fine.n[a]] if fine.n[a] % 2 else [])]
                 for a in range(3)]
    coarse = syn.BoxMesh(n=tuple(len(c) - 1 for c in coarse_ax), A=fine.A, grade=coarse_ax)
    P = solvers.prolongation_h(fine, coarse)
    Xc = np.stack(np.meshgrid(*coarse_ax[::-1], indexing="ij")[::-1], -1).reshape(-1, 3)
    Xf = np.stack(np.meshgrid(*[fine.axis_nodes(a) for a in range(3)][::-1], indexing="ij")[::-1], -1).reshape(-1, 3)
    f = lambda X: np.stack([X[:, 0] * X[:, 1] * X[:, 2], 1 + X[:, 0], X[:, 1] * X[:, 2] - X[:, 0]])
    assert np.allclose(P @ f(Xc).ravel(), f(Xf).ravel(), atol=1e-13)


def _two_level(p=4):
    mesh = syn.BoxMesh(n=(2, 2, 1), L=(2.0, 1.0, 0.5), clamped_faces=1)
    levels, P = [], []
    for pl in (p, p // 2, 1):
        op, A, d = _system(mesh, pl, 1.2, 0.9)
        ev = np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))
        lmin, lmax = solvers.chebyshev_interval(ev[-1])
        levels.append(solvers.DenseLevel(A, d, op.ess, lmin, lmax))
    P = [solvers.prolongation_p(mesh, p // 2, p), solvers.prolongation_p(mesh, 1, p // 2)]
    return levels, P


def test_vcycle_symmetric_positive():
    levels, P = _two_level()
    N = levels[0].A.shape[0]
    rng = np.random.default_rng(0)
    Bm = np.stack([solvers.vcycle(levels, P, e, 3) for e in np.eye(N)[:: max(1, N // 60)]], 1)
    idx = np.arange(N)[:: max(1, N // 60)]
    sub = Bm[idx]
    assert np.allclose(sub, sub.T, atol=1e-10 * np.abs(sub).max())
    x, y = rng.uniform(-1, 1, (2, N))
    bx, by = solvers.vcycle(levels, P, x, 3), solvers.vcycle(levels, P, y, 3)
    assert abs(x @ by - y @ bx) <= 1e-11 * abs(x @ by)
    assert x @ bx > 0


def test_pcg_matches_direct():
    levels, P = _two_level()
    A = levels[0].A
    b = np.random.default_rng(1).uniform(-1, 1, A.shape[0])
    b[levels[0].ess] = 0
    x, it = solvers.pcg(A, b, lambda r: solvers.vcycle(levels, P, r, 3), 1e-12)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert it < 40


@pytest.mark.parametrize("k", [1, 2, 3, 5])
@pytest.mark.parametrize("lo_frac", [0.1, 0.3])
def test_chebyshev_error_polynomial(k, lo_frac):
    """The smoother is exactly the Chebyshev polynomial of the interval: with D^{-1}A =
    D^{-1/2} V diag(l) V^T D^{1/2} (A v = l D v), the error after k steps is
    e_k = D^{-1/2} V diag(T_k((theta - l)/delta) / T_k(theta/delta)) V^T D^{1/2} e_0,
    theta, delta the centre and half-width of [lmin, lmax] (here an interval that does not
    contain the whole spectrum, as in the multigrid smoother, so T_k is evaluated inside
    and outside [-1, 1])."""
    mesh = syn.BoxMesh(n=(2, 2, 1), clamped_faces=1)
    op, A, d = _system(mesh, 2, 1.3, 0.6)
    sq = np.sqrt(d)
    lam, V = np.linalg.eigh(A / np.outer(sq, sq))
    lmax = 1.2 * lam[-1]
    lmin = lo_frac * lmax
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)

    def T(n, t):   # Chebyshev polynomial of the first kind by its three-term recurrence
        a, b = np.ones_like(t), t
        if n == 0:
            return a
        for _ in range(n - 1):
            a, b = b, 2 * t * b - a
        return b

    rng = np.random.default_rng(10 + k)
    xstar = rng.uniform(-1, 1, op.N)
    b = A @ xstar
    x0 = rng.uniform(-1, 1, op.N)
    xk = solvers.chebyshev_smooth(A, d, b, x0, k, lmin, lmax)
    pk = T(k, (theta - lam) / delta) / T(k, np.array(theta / delta))
    ek = (V @ (pk * (V.T @ (sq * (x0 - xstar))))) / sq
    assert np.linalg.norm((xk - xstar) - ek) <= 1e-11 * np.linalg.norm(x0 - xstar)


def test_abs_apply_is_the_sum_of_element_magnitudes():
    """abs_apply = sum_e G_e^T |K^e| G_e x assembled densely from the element matrices (two
    materials, a graded sheared mesh), and |A x| <= abs_apply(|x|) entrywise; constrained
    form: 0 on clamped columns, the input on clamped rows."""
    mesh = syn.graded_mesh((3, 2, 2), seed=5, A=syn.SHEAR_A, clamped_faces=0b000101)
    p = 2
    lam, mu = syn.two_material_lame(mesh.num_elements, seed=3)
    op = elasticity.Operator(mesh, p, p + 2, lam, mu)
    M = np.zeros((op.N, op.N))
    for e in range(mesh.num_elements):
        d = op.edofs[e]
        M[np.ix_(d, d)] += np.abs(op.element_matrix(e))
    x = syn.uniform_vector(op.N, 4)
    assert np.allclose(op.abs_apply(x), M @ x, rtol=1e-13, atol=1e-13 * np.abs(M @ x).max())
    assert np.all(np.abs(op.apply(x)) <= op.abs_apply(np.abs(x)) * (1 + 1e-12) + 1e-14)
    xc = x.copy()
    xc[op.ess] = 0.0
    ref = M @ xc
    ref[op.ess] = x[op.ess]
    assert np.allclose(op.abs_apply(x, constrained=True), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("n,p,faces", [((4, 1, 1), 2, 1), ((3, 2, 2), 3, 0b100001), ((5, 2, 1), 1, 0b010011),
                                       ((2, 1, 1), 4, 1), ((1, 1, 1), 2, 0b000010), ((3, 1, 2), 2, 0b000110)])
def test_slab_cholesky_matches_dense_solve(n, p, faces):
    """The block solve over x-slabs equals the dense solve of the assembled constrained system
    (graded, rotated, sheared mesh, two materials, clamped faces across several blocks); clamped
    entries of the solution equal those of the right-hand side (identity rows)."""
    mesh = syn.graded_mesh(n, seed=3, A=syn.random_rotation(2) @ syn.SHEAR_A, clamped_faces=faces)
    lam, mu = syn.two_material_lame(mesh.num_elements, seed=2)
    op = elasticity.Operator(mesh, p, p + 2, lam, mu)
    b = syn.uniform_vector(op.N, 1)
    x = solvers.SlabCholesky(op).solve(b)
    xr = np.linalg.solve(op.dense(constrained=True), b)
    assert np.linalg.norm(x - xr) <= 1e-12 * np.linalg.norm(xr)
    assert np.array_equal(x[op.ess], b[op.ess])
