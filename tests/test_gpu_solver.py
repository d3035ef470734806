"""GPU parity of the multigrid components and the GMG-PCG solves against the oracle.

Each multigrid component is compared with the oracle's dense reference of the
same linear map (transfers, Chebyshev polynomial, coarse solve, V-cycle) with
the Chebyshev interval passed to both sides; the power iteration is compared
with the oracle's power iteration from the same SplitMix64 start vector; solves
are compared with direct solves (small) or with the oracle's FP64 residual of
the GPU solution (full size).
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import elasticity, mesh as omesh, solvers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pa():
    import paper_2601_08374_amd as pa
    return pa


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _np(t):
    return t.double().cpu().numpy()


def _coarsen(mesh):
    """The h-coarsening rule of the hierarchy: merge element pairs on every axis with n > 1."""
    grade = []
    for a in range(3):
        X = mesh.axis_nodes(a)
        n = mesh.n[a]
        if n <= 1:
            grade.append(X)
        else:
            nc = (n + 1) // 2
            grade.append(np.array([X[2 * k] for k in range(nc)] + [X[n]]))
    return syn.BoxMesh(n=tuple(len(g) - 1 for g in grade), A=mesh.A, grade=grade, clamped_faces=mesh.clamped_faces)


def _level_meshes(mesh, p, n_h):
    out = []
    pl = p
    while True:
        out.append((mesh, pl))
        if pl == 1:
            break
        pl //= 2
    m = mesh
    for _ in range(n_h):
        m = _coarsen(m)
        out.append((m, 1))
    return out


def _coarse_lame(mesh_f, lam, mu):
    """Volume-weighted Lame parameters on the merged elements (matches the hierarchy's rule)."""
    mc = _coarsen(mesh_f)
    hs = [np.diff(mesh_f.axis_nodes(a)) for a in range(3)]
    cl, cm, cv = np.zeros(mc.num_elements), np.zeros(mc.num_elements), np.zeros(mc.num_elements)
    for ez in range(mesh_f.n[2]):
        for ey in range(mesh_f.n[1]):
            for ex in range(mesh_f.n[0]):
                e = ex + mesh_f.n[0] * (ey + mesh_f.n[1] * ez)
                cx = ex // 2 if mesh_f.n[0] > 1 else ex
                cy = ey // 2 if mesh_f.n[1] > 1 else ey
                cz = ez // 2 if mesh_f.n[2] > 1 else ez
                ce = cx + mc.n[0] * (cy + mc.n[1] * cz)
                vol = hs[0][ex] * hs[1][ey] * hs[2][ez]
                cl[ce] += vol * lam[e]
                cm[ce] += vol * mu[e]
                cv[ce] += vol
    return mc, cl / cv, cm / cv


def _oracle_levels(mesh, p, lam, mu, n_h):
    """Dense oracle operators of every level (finest first)."""
    levels = []
    m, l_, m_ = mesh, np.asarray(lam, float), np.asarray(mu, float)
    for (lm, pl) in _level_meshes(mesh, p, 0):
        op = elasticity.Operator(lm, pl, pl + 2, l_, m_)
        levels.append((lm, pl, op))
    for _ in range(n_h):
        m, l_, m_ = _coarse_lame(m, l_, m_)
        levels.append((m, 1, elasticity.Operator(m, 1, 3, l_, m_)))
    return levels


def _transfer(levels, l):
    (mf, pf, _), (mc, pc, _) = levels[l], levels[l + 1]
    if pf != pc:
        return solvers.prolongation_p(mf, pc, pf)
    return solvers.prolongation_h(mf, mc)


SMALL = dict(mesh=lambda: syn.graded_mesh((3, 2, 2), seed=21, L=(1.5, 1.0, 0.8), A=syn.SHEAR_A, clamped_faces=1),
             p=4, n_h=1)


def _small_setup(p=4, n_h=1, lam_override=True, k=3, seed=21):
    pa = _pa()
    mesh = syn.graded_mesh((3, 2, 2), seed=seed, L=(1.5, 1.0, 0.8), A=syn.SHEAR_A, clamped_faces=1)
    NE = mesh.num_elements
    rng = np.random.default_rng(seed)
    lam, mu = rng.uniform(0.5, 2.0, NE), rng.uniform(0.5, 2.0, NE)
    lv = _oracle_levels(mesh, p, lam, mu, n_h)
    lhat = []
    for (_, _, op) in lv[:-1]:
        A = op.dense(True)
        d = op.diagonal(True)
        lhat.append(float(np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))[-1]))
    op = pa.Operator(mesh, p, lam, mu)
    kw = dict(h_levels=n_h, cheb_degree=k)
    if lam_override:
        kw["lambda_max"] = lhat + [0.0]
    H = op.hierarchy(**kw)
    return pa, mesh, op, H, lv, lhat


def test_hierarchy_shape_and_level_operators():
    pa, mesh, op, H, lv, _ = _small_setup()
    assert H.num_levels == len(lv)
    for l, (m, pl, oop) in enumerate(lv):
        info = H.level_info(l)
        assert info["p"] == pl and info["n"] == m.n and info["N"] == oop.N
        x = torch.tensor(syn.uniform_vector(oop.N, l), device="cuda")
        y = H.level_apply(l, x)
        assert _rel(_np(y), oop.apply(_np(x), constrained=True)) <= 1e-12


def test_transfers_match_dense_interpolation():
    pa, mesh, op, H, lv, _ = _small_setup(p=4, n_h=2)
    for l in range(H.num_levels - 1):
        P = _transfer(lv, l)
        ess_f, ess_c = lv[l][2].ess, lv[l + 1][2].ess
        xc = syn.uniform_vector(P.shape[1], 10 + l)
        xc[ess_c] = 0
        xf = _np(H.prolong(l, torch.tensor(xc, device="cuda")))
        ref = P @ xc
        ref[ess_f] = 0
        assert _rel(xf, ref) <= 1e-13, l
        rf = syn.uniform_vector(P.shape[0], 20 + l)
        rc = _np(H.restrict(l, torch.tensor(rf, device="cuda")))
        ref = P.T @ rf
        ref[ess_c] = 0
        assert _rel(rc, ref) <= 1e-13, l


@pytest.mark.parametrize("pf", [2, 3, 6, 8])
def test_p_transfer_orders(pf):
    pa = _pa()
    mesh = syn.BoxMesh(n=(2, 1, 2), L=(1.0, 0.5, 1.0), A=syn.SHEAR_A, clamped_faces=0b10)
    op = pa.Operator(mesh, pf, np.ones(4), np.ones(4))
    H = op.hierarchy(p_levels=1, h_levels=0, lambda_max=[1.0, 0.0])
    pc = pf // 2
    P = solvers.prolongation_p(mesh, pc, pf)
    essf, essc = omesh.essential_mask(mesh, pf), omesh.essential_mask(mesh, pc)
    xc = syn.uniform_vector(P.shape[1], 3)
    xc[essc] = 0
    ref = P @ xc
    ref[essf] = 0
    assert _rel(_np(H.prolong(0, torch.tensor(xc, device="cuda"))), ref) <= 1e-13
    rf = syn.uniform_vector(P.shape[0], 4)
    ref = P.T @ rf
    ref[essc] = 0
    assert _rel(_np(H.restrict(0, torch.tensor(rf, device="cuda"))), ref) <= 1e-13


def test_power_iteration_matches_oracle():
    pa, mesh, op, H, lv, lhat = _small_setup(lam_override=False)
    for l in range(H.num_levels - 1):
        oop = lv[l][2]
        A, d = oop.dense(True), oop.diagonal(True)
        v0 = solvers.splitmix64_uniform(7 + l, oop.N)
        v0[oop.ess] = 0
        ref = solvers.power_iteration(A, d, v0, 10)
        got = H.level_info(l)["lambda_max"] / 1.2
        assert abs(got - ref) <= 1e-10 * ref, (l, got, ref)
        assert got <= lhat[l] * (1 + 1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_chebyshev_smoother_matches_oracle(k):
    pa, mesh, op, H, lv, lhat = _small_setup(k=k)
    oop = lv[0][2]
    A, d = oop.dense(True), oop.diagonal(True)
    lmin, lmax = solvers.chebyshev_interval(lhat[0])
    b = syn.uniform_vector(oop.N, 5)
    b[oop.ess] = 0
    ref0 = solvers.chebyshev_smooth(A, d, b, np.zeros(oop.N), k, lmin, lmax)
    got0 = _np(H.smooth(0, torch.tensor(b, device="cuda")))
    assert _rel(got0, ref0) <= 1e-12
    x0 = syn.uniform_vector(oop.N, 6)
    x0[oop.ess] = 0
    ref1 = solvers.chebyshev_smooth(A, d, b, x0, k, lmin, lmax)
    got1 = _np(H.smooth(0, torch.tensor(b, device="cuda"), torch.tensor(x0, device="cuda")))
    assert _rel(got1, ref1) <= 1e-12


def test_coarse_solve_matches_direct():
    pa, mesh, op, H, lv, _ = _small_setup(p=2, n_h=2)
    oop = lv[-1][2]
    A = oop.dense(True)
    b = syn.uniform_vector(oop.N, 8)
    b[oop.ess] = 0
    got = _np(H.coarse_solve(torch.tensor(b, device="cuda")))
    assert _rel(got, np.linalg.solve(A, b)) <= 1e-11


@pytest.mark.parametrize("n", [(6, 5, 4), (10, 9, 8)])
def test_coarse_inverse_several_blocks(n):
    """The coarse inverse at sizes spanning many 32-pivot blocks with a ragged last block and
    several 64 x 64 update tiles (630 and 2970 dofs): coarse solve vs a dense direct solve."""
    pa = _pa()
    mesh = syn.graded_mesh(n, seed=3, L=(1.2, 1.0, 0.9), A=syn.SHEAR_A, clamped_faces=1)
    NE = mesh.num_elements
    rng = np.random.default_rng(4)
    lam, mu = rng.uniform(0.5, 2.0, NE), rng.uniform(0.5, 2.0, NE)
    op = pa.Operator(mesh, 2, lam, mu)
    H = op.hierarchy(h_levels=0)
    lv = _oracle_levels(mesh, 2, lam, mu, 0)
    oop = lv[-1][2]
    assert H.num_levels == 2 and H.level_info(1)["N"] == oop.N
    assert oop.N % 32 != 0 and oop.N > 2 * 64
    A = oop.dense(True)
    b = syn.uniform_vector(oop.N, 8)
    b[oop.ess] = 0
    got = _np(H.coarse_solve(torch.tensor(b, device="cuda")))
    assert _rel(got, np.linalg.solve(A, b)) <= 1e-10
    H.close()
    op.close()


@pytest.mark.parametrize("p,n_h", [(4, 1), (2, 2), (3, 1)])
def test_vcycle_matches_oracle(p, n_h):
    pa, mesh, op, H, lv, lhat = _small_setup(p=p, n_h=n_h)
    levels = []
    for l, (_, _, oop) in enumerate(lv):
        A, d = oop.dense(True), oop.diagonal(True)
        lo, hi = solvers.chebyshev_interval(lhat[l]) if l < len(lhat) else (None, None)
        levels.append(solvers.DenseLevel(A, d, oop.ess, lo, hi))
    P = [_transfer(lv, l) for l in range(len(lv) - 1)]
    r = syn.uniform_vector(lv[0][2].N, 9)
    r[lv[0][2].ess] = 0
    ref = solvers.vcycle(levels, P, r, 3)
    got = _np(H.vcycle(torch.tensor(r, device="cuda")))
    assert _rel(got, ref) <= 1e-11


def test_config1_pcg_vs_direct():
    """Unit cube 4x4x4, p=2, x=0 clamped, f=(0,0,-1), rtol 1e-10 (p 2->1, h 4->2->1)."""
    pa = _pa()
    mesh = syn.unit_cube_4(clamped=True)
    op = pa.Operator(mesh, 2, np.ones(64), np.ones(64))
    b = op.rhs((0.0, 0.0, -1.0))
    ref_op = elasticity.Operator(mesh, 2, 4, 1.0, 1.0)
    bref = elasticity.body_force_vector(mesh, 2, 4, (0.0, 0.0, -1.0))
    bref[ref_op.ess] = 0
    assert _rel(_np(b), bref) <= 1e-14
    u = solvers.solve_dense(ref_op.dense(True), bref)
    x, info, rc = op.solve(b, rtol=1e-10, h_levels=2, cheb_degree=3)
    assert rc == 0 and info.num_levels == 4
    assert _rel(_np(x), u) <= 1e-8
    assert info.rel_res_true <= 1e-9
    print("config1 iterations", info.iters)


@pytest.mark.parametrize("p", [4, 8])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_small_cantilever_vs_direct(p, mode):
    pa = _pa()
    nx = 8 if p == 4 else 4
    mesh = syn.cantilever_mesh(nx, 1, 1, length=float(nx))
    lam, mu = syn.lame_from_young_poisson(1.0, 0.3)
    NE = mesh.num_elements
    op = pa.Operator(mesh, p, np.full(NE, lam), np.full(NE, mu))
    b = op.rhs((0.0, 0.0, 0.0), 1, (0.0, 0.0, -1.0))
    ref_op = elasticity.Operator(mesh, p, p + 2, lam, mu)
    u = solvers.solve_dense(ref_op.dense(True), _np(b))
    x, info, rc = op.solve(b, rtol=1e-8, mode=mode, stop=1, cheb_degree=3)
    assert rc == 0, (rc, info.iters)
    assert info.rel_res_true <= 1e-8 * (1 + 1e-6)
    # error of a solve to relative residual 1e-8 (condition number of this small beam ~1e5)
    assert _rel(_np(x), u) <= 1e-4
    print(f"cantilever {nx}x1x1 p={p} mode={mode}: iters {info.iters} outer {info.outer_iters} "
          f"err {_rel(_np(x), u):.2e}")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_solve_bitwise_reproducible(mode):
    """Every reduction of setup and solve runs in a fixed order (no atomics): two solves on
    freshly built operators and hierarchies give bitwise identical iterates."""
    pa = _pa()
    mesh = syn.graded_mesh((6, 3, 2), seed=3, L=(3.0, 1.0, 1.0), clamped_faces=1)
    NE = mesh.num_elements
    lam, mu = syn.two_material_lame(NE, seed=4)
    out = []
    for _ in range(2):
        op = pa.Operator(mesh, 4, lam, mu)
        b = op.rhs((0.1, 0.0, -1.0), 1, (0.0, 0.3, -1.0))
        d = op.diagonal()
        x, info, rc = op.solve(b, rtol=1e-9, mode=mode, stop=1, cheb_degree=3, h_levels=1)
        assert rc == 0
        out.append((_np(b), _np(d), _np(x), info.iters))
        op.close()
    for a, c in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, c)
    assert out[0][3] == out[1][3]


def test_step_api_interleaved_equals_blocking():
    pa = _pa()
    import ctypes as C
    cap = pa.capi
    meshes = [syn.cantilever_mesh(4, 1, 1, length=4.0), syn.BoxMesh(n=(3, 2, 2), clamped_faces=1)]
    ps = [4, 2]
    ops, hs, bs, xs_ref = [], [], [], []
    for m, p in zip(meshes, ps):
        NE = m.num_elements
        op = pa.Operator(m, p, np.full(NE, 1.0), np.full(NE, 0.7))
        H = op.hierarchy(cheb_degree=2)
        b = op.rhs((0.3, -0.2, -1.0))
        x, info, rc = H.pcg(b, rtol=1e-9)
        assert rc == 0
        ops.append(op), hs.append(H), bs.append(b), xs_ref.append(_np(x))
    xs = [torch.zeros_like(b) for b in bs]
    solves = []
    for H, b, x in zip(hs, bs, xs):
        s = C.c_void_p()
        cap.check(cap.gmg_pcg_begin(H.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), 1e-9,
                                    C.byref(s)))
        solves.append(s)
    done = [False, False]
    for _ in range(10000):
        for i, s in enumerate(solves):
            if done[i]:
                continue
            cap.check(cap.gmg_pcg_step(s, 2))
            d, st = C.c_int(), C.c_int()
            cap.check(cap.gmg_pcg_poll(s, C.byref(d), C.byref(st)))
            done[i] = bool(d.value)
        if all(done):
            break
    assert all(done)
    for i, s in enumerate(solves):
        info = cap.pa_solve_info_t()
        assert cap.gmg_pcg_end(s, C.byref(info)) == 0
        assert _rel(_np(xs[i]), xs_ref[i]) <= 1e-12


def _full_cantilever(p, mode):
    pa = _pa()
    mesh = syn.cantilever_mesh(80, 8, 8)
    lam, mu = syn.lame_from_young_poisson(1.0, 0.3)
    NE = mesh.num_elements
    op = pa.Operator(mesh, p, np.full(NE, lam), np.full(NE, mu))
    b = op.rhs((0.0, 0.0, 0.0), 1, (0.0, 0.0, -1.0))
    x, info, rc = op.solve(b, rtol=1e-8, mode=mode, stop=1, cheb_degree=3, h_levels=2)
    return mesh, op, b, x, info, rc, lam, mu


EPS64 = float(np.finfo(np.float64).eps)


def _residual_and_rounding(ref_op, b, x):
    """(|b - A x| / |b|, rounding scale of that evaluation / |b|), both computed by the oracle.

    The rounding scale is eps |(|b| + sum_e G_e^T |K^e| G_e |x|)| / |b|: the first-order term of
    the classical error bound of a sum of products (eps times the sum of the magnitudes of the
    terms, here the element products and b), without the bound's length factor.  A residual near
    rtol = 1e-8 is a cancellation of terms much larger than b (the cantilever's tip deflection is
    ~2000 under a unit traction), so this scale is of the order of rtol itself."""
    nb = np.linalg.norm(b)
    r = b - ref_op.apply(x, constrained=True)
    scale = EPS64 * np.linalg.norm(np.abs(b) + ref_op.abs_apply(np.abs(x), constrained=True)) / nb
    return float(np.linalg.norm(r) / nb), float(scale)


@pytest.mark.parametrize("p,mode", [(8, 0), (8, 1), (8, 2), (6, 0), (6, 1), (6, 2), (4, 0), (4, 1)])
def test_full_size_cantilever_oracle_residual(p, mode):
    """The 80x8x8 cantilever (8.1M dofs at p=8): the oracle's own FP64 apply gives the
    true residual of the GPU solution; tip deflection vs beam theory as a sanity check."""
    print(f"full cantilever p={p} mode={mode}", flush=True)
    mesh, op, b, x, info, rc, lam, mu = _full_cantilever(p, mode)
    assert rc == 0, rc
    ref_op = elasticity.Operator(mesh, p, p + 2, lam, mu)
    bref = elasticity.traction_vector(mesh, p, p + 2, 1, (0.0, 0.0, -1.0))
    bref[ref_op.ess] = 0
    bh = _np(b)
    assert _rel(bh, bref) <= 1e-13
    xh = _np(x)
    res, scale = _residual_and_rounding(ref_op, bref, xh)
    # The solver stops on its own FP64 evaluation of the true residual, which must meet rtol;
    # the oracle's evaluation (element matrices, another summation order) may differ from it
    # by the rounding of each, so it must lie within rtol plus one rounding scale, and within
    # two rounding scales of the GPU's value.
    print(f"p={p} mode={mode}: iters {info.iters} outer {info.outer_iters} res {res:.3e} "
          f"(GPU {info.rel_res_true:.3e}) rounding scale {scale:.3e}", flush=True)
    assert info.rel_res_true <= 1e-8 * (1 + 1e-12), info.rel_res_true
    assert res <= 1e-8 + scale, (res, scale)
    assert abs(res - info.rel_res_true) <= 2 * scale, (res, info.rel_res_true, scale)
    R = omesh.node_coords(mesh, p)
    tip = np.isclose(R[:, 0], 8.0)
    defl = -xh.reshape(3, -1)[2, tip].mean()
    assert 0.95 * 2048 < defl < 1.05 * 2048 * 1.012
    print(f"  t_setup {info.t_setup:.2f}s t_solve {info.t_solve:.2f}s tip {defl:.2f}")


_REDUCED = {}


def _reduced_cantilever_oracle():
    """The reduced cantilever 16x2x2 at p = 8 (111,843 dofs; same 8:1:1 beam, clamped x = 0,
    unit downward traction on x = 8, E = 1, nu = 0.3): the oracle's load vector, its direct
    solution (block Cholesky over x-slabs), and the bounds used to judge a solution."""
    if not _REDUCED:
        mesh = syn.cantilever_mesh(16, 2, 2)
        lam, mu = (float(v) for v in syn.lame_from_young_poisson(1.0, 0.3))
        ref_op = elasticity.Operator(mesh, 8, 10, lam, mu)
        b = elasticity.traction_vector(mesh, 8, 10, 1, (0.0, 0.0, -1.0))
        b[ref_op.ess] = 0
        F = solvers.SlabCholesky(ref_op)
        x = F.solve(b)
        # lambda_max <= the largest row sum of |A| (Gershgorin); lambda_min from inverse iteration
        # (a Rayleigh quotient: an upper estimate, halved for the bound below)
        lmax = float(ref_op.abs_apply(np.ones(ref_op.N), constrained=True).max())
        v = syn.uniform_vector(ref_op.N, 3)
        v[ref_op.ess] = 0
        for _ in range(4):
            v = F.solve(v / np.linalg.norm(v))
        v /= np.linalg.norm(v)
        lmin = float(v @ ref_op.apply(v, constrained=True))
        _REDUCED.update(mesh=mesh, lam=lam, mu=mu, ref_op=ref_op, b=b, x=x, lmax=lmax, lmin=lmin)
    return _REDUCED


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_reduced_cantilever_vs_direct_solve(mode):
    """GPU GMG-PCG solve (all three modes, rtol 1e-8 on the true residual) of the reduced
    cantilever vs the oracle's direct solve.  With r the residual of a solution and x* the
    exact one, |x - x*|_A / |x*|_A <= sqrt(kappa) |r| / |b| (A SPD); the difference of the GPU
    and direct solutions is bounded by the sum of both, each residual taken with its rounding
    scale, kappa from the Gershgorin bound and twice the inverse-iteration estimate."""
    pa = _pa()
    print(f"reduced cantilever 16x2x2 p=8 mode={mode}: oracle direct solve", flush=True)
    R = _reduced_cantilever_oracle()
    mesh, ref_op, b, xd = R["mesh"], R["ref_op"], R["b"], R["x"]
    NE = mesh.num_elements
    op = pa.Operator(mesh, 8, np.full(NE, R["lam"]), np.full(NE, R["mu"]))
    bt = op.rhs((0.0, 0.0, 0.0), 1, (0.0, 0.0, -1.0))
    assert _rel(_np(bt), b) <= 1e-13
    xg, info, rc = op.solve(bt, rtol=1e-8, mode=mode, stop=1, cheb_degree=3)
    assert rc == 0, rc
    xg = _np(xg)
    res_g, sc_g = _residual_and_rounding(ref_op, b, xg)
    res_d, sc_d = _residual_and_rounding(ref_op, b, xd)
    kappa = R["lmax"] / (0.5 * R["lmin"])
    e = xg - xd
    err_a = float(np.sqrt(e @ ref_op.apply(e, constrained=True) / (xd @ b)))
    bound = np.sqrt(kappa) * (res_g + sc_g + res_d + sc_d)
    print(f"  iters {info.iters} outer {info.outer_iters}: res GPU {res_g:.2e} direct {res_d:.2e} "
          f"(rounding {sc_g:.1e}), kappa <= {kappa:.2e}, |x - x_direct|_A / |x|_A = {err_a:.2e} "
          f"(bound {bound:.2e}), rel 2-norm {_rel(xg, xd):.2e}", flush=True)
    assert info.rel_res_true <= 1e-8 * (1 + 1e-12)
    assert err_a <= bound, (err_a, bound)


def test_solver_mode_validation():
    pa = _pa()
    mesh = syn.BoxMesh(n=(2, 2, 2), clamped_faces=1)
    op = pa.Operator(mesh, 2, np.full(8, 1.0), np.full(8, 1.0))
    with pytest.raises(pa.PaError) as e:
        op.hierarchy(mode=3)
    assert e.value.code == pa.capi.PA_EINVAL
    H = op.hierarchy(mode=pa.PA_SOLVE_F32_PREC)
    assert H.num_levels >= 2
    H.close()
