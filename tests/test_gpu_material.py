"""GPU parity of the apply with general material data (per-quadrature-point Lame
parameters, per-element anisotropic Voigt stiffness) against the oracle's
strain-displacement form (oracle.material.GeneralOperator).

Tolerances (relative, 2-norm over the output): FP64 1e-12, FP32 1e-5, the bars of the
apply in double and single precision.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import elasticity, material, mesh as omesh, solvers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


def _pa():
    import paper_2601_08374_amd as pa
    return pa


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _mesh(p, seed):
    # several workgroup tiles with a ragged tail; graded + sheared + rotated at low p
    rot = syn.random_rotation(seed) @ syn.SHEAR_A
    if p <= 3:
        return syn.graded_mesh((5, 3, 2), seed=seed, L=(1.3, 0.8, 1.0), A=rot, clamped_faces=0b010001)
    if p <= 5:
        return syn.graded_mesh((3, 2, 2), seed=seed, L=(1.0, 1.2, 0.9), A=rot, clamped_faces=0b000110)
    return syn.BoxMesh(n=(3, 2, 1), L=(1.5, 1.0, 0.6), A=rot, clamped_faces=0b100000)


def _material(kind, NE, q, seed):
    """(data for the C ABI, Voigt stiffness for the oracle)."""
    pa = _pa()
    rng = np.random.default_rng(seed)
    lam_e, mu_e = rng.uniform(0.3, 3.0, NE), rng.uniform(0.3, 3.0, NE)
    if kind == pa.PA_MAT_QP_ISO:
        lam, mu = syn.quadrature_point_lame(lam_e, mu_e, q, seed=seed + 1, spread=0.4)
        return np.stack([lam, mu], axis=-1), material.isotropic_voigt(lam, mu)
    C = syn.random_spd_stiffness(NE, seed=seed + 2, lam=1.3, mu=0.8, spread=1.0)
    return material.packed_upper(C), C


def _gpu(op, x, flags):
    tdt = torch.float64 if op.dtype == 0 else torch.float32
    y = op.apply(torch.tensor(x, dtype=tdt, device="cuda"), flags=flags)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("dtype", [0, 1])
def test_material_parity(p, kind, dtype):
    pa = _pa()
    q = p + 2
    print(f"material parity p={p} kind={kind} dtype={dtype}", flush=True)
    mesh = _mesh(p, seed=20 + p)
    data, C = _material(kind, mesh.num_elements, q, seed=30 + p)
    ref_op = material.GeneralOperator(mesh, p, q, C)
    op = pa.Operator.with_material(mesh, p, kind, data, dtype=dtype)
    x = syn.uniform_vector(mesh.num_dofs(p), seed=p)
    for flags, constrained in ((0, True), (pa.PA_UNCONSTRAINED, False)):
        ref = ref_op.apply(x, constrained=constrained)
        y = _gpu(op, x, flags)
        assert _rel(y, ref) <= TOL[dtype], (flags, _rel(y, ref))


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_material_add_flag(p):
    pa = _pa()
    mesh = _mesh(p, seed=40 + p)
    data, C = _material(pa.PA_MAT_ANISO, mesh.num_elements, p + 2, seed=50 + p)
    op = pa.Operator.with_material(mesh, p, pa.PA_MAT_ANISO, data)
    x = syn.uniform_vector(op.N, seed=1)
    y0 = syn.uniform_vector(op.N, seed=2)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    yt = torch.tensor(y0, dtype=torch.float64, device="cuda")
    op.apply(xt, yt, flags=pa.PA_ADD | pa.PA_UNCONSTRAINED)
    ref = y0 + material.GeneralOperator(mesh, p, p + 2, C).apply(x)
    assert _rel(yt.cpu().numpy(), ref) <= TOL[0]


@pytest.mark.parametrize("p", [1, 3, 8])
def test_isotropic_forms_agree(p):
    """Per-point data constant over each element, and the isotropic Voigt matrix, give the
    per-element operator (three kernels, one operator)."""
    pa = _pa()
    mesh = _mesh(p, seed=60 + p)
    NE, q = mesh.num_elements, p + 2
    rng = np.random.default_rng(p)
    lam, mu = rng.uniform(0.3, 3.0, NE), rng.uniform(0.3, 3.0, NE)
    x = syn.uniform_vector(mesh.num_dofs(p), seed=3)
    base = _gpu(pa.Operator(mesh, p, lam, mu), x, 0)
    qp = np.stack([np.repeat(lam[:, None], q ** 3, 1), np.repeat(mu[:, None], q ** 3, 1)], axis=-1)
    y1 = _gpu(pa.Operator.with_material(mesh, p, pa.PA_MAT_QP_ISO, qp), x, 0)
    y2 = _gpu(pa.Operator.with_material(mesh, p, pa.PA_MAT_ANISO,
                                        material.packed_upper(material.isotropic_voigt(lam, mu))), x, 0)
    assert _rel(y1, base) <= TOL[0] and _rel(y2, base) <= TOL[0]


def _sampled_reference(mesh, p, C, x, nodes):
    """A x at the given nodes from the elements around them (uniform Jacobian)."""
    q, D = p + 2, p + 1
    J = omesh.element_jacobians(syn.BoxMesh(n=(1, 1, 1), L=tuple(mesh.L[a] / mesh.n[a] for a in range(3)),
                                            A=mesh.A))[0]
    B, W = material.strain_matrix(p, q, J)
    Nx, Ny, Nz = omesh.grid_shape(mesh, p)
    Nn = Nx * Ny * Nz
    iz, iy, ix = np.meshgrid(np.arange(D), np.arange(D), np.arange(D), indexing="ij")
    out = []
    for node in nodes:
        gx, gy, gz = node % Nx, (node // Nx) % Ny, node // (Nx * Ny)
        acc = np.zeros(3)
        rng_x = {min(gx // p, mesh.n[0] - 1), (gx - 1) // p if gx % p == 0 and gx > 0 else -1}
        rng_y = {min(gy // p, mesh.n[1] - 1), (gy - 1) // p if gy % p == 0 and gy > 0 else -1}
        rng_z = {min(gz // p, mesh.n[2] - 1), (gz - 1) // p if gz % p == 0 and gz > 0 else -1}
        for ex in rng_x:
            for ey in rng_y:
                for ez in rng_z:
                    if min(ex, ey, ez) < 0:
                        continue
                    e = ex + mesh.n[0] * (ey + mesh.n[1] * ez)
                    g = (ex * p + ix.ravel()) + Nx * ((ey * p + iy.ravel()) + Ny * (ez * p + iz.ravel()))
                    xe = np.concatenate([x[c * Nn + g] for c in range(3)])
                    Ce = C[e] if C.ndim == 4 else np.broadcast_to(C[e], (q ** 3, 6, 6))
                    eps = np.einsum("akn,n->ak", B, xe)
                    ye = np.einsum("akn,ak->n", B, np.einsum("akl,al->ak", Ce, eps) * W[:, None])
                    a = (gx - ex * p) + D * ((gy - ey * p) + D * (gz - ez * p))
                    acc += ye[[a, D ** 3 + a, 2 * D ** 3 + a]]
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("p", [1, 2, 4, 8])
@pytest.mark.parametrize("kind", [1, 2])
def test_material_full_size_sampled(p, kind):
    """The material workload at the operator sweep's full size (~4.2M dofs), same launch as
    the benchmark: sampled outputs vs the oracle element by element around the nodes."""
    pa = _pa()
    print(f"material full size p={p} kind={kind}", flush=True)
    mesh = syn.sheared_box_mesh(p)
    NE, q = mesh.num_elements, p + 2
    data, C = _material_full(kind, NE, q)
    op = pa.Operator.with_material(mesh, p, kind, data)
    x = syn.uniform_vector(op.N, seed=0)
    y = _gpu(op, x, pa.PA_UNCONSTRAINED)
    Nn = op.N // 3
    nodes = np.random.default_rng(5).integers(0, Nn, 24)
    ref = _sampled_reference(mesh, p, C, x, nodes)
    got = np.stack([y[nodes], y[Nn + nodes], y[2 * Nn + nodes]], axis=1)
    assert np.abs(got - ref).max() <= 50 * TOL[0] * np.abs(y).max()


def _material_full(kind, NE, q):
    if kind == 1:
        lam_e, mu_e = syn.two_material_lame(NE, seed=1)
        lam, mu = syn.quadrature_point_lame(lam_e, mu_e, q, seed=4)
        return np.stack([lam, mu], axis=-1), _LazyIso(lam, mu)
    C = syn.random_spd_stiffness(NE, seed=5)
    return material.packed_upper(C), C


class _LazyIso:
    """Per-point isotropic Voigt matrices built on demand (the full array would not fit)."""

    ndim = 4

    def __init__(self, lam, mu):
        self.lam, self.mu = lam, mu

    def __getitem__(self, e):
        return material.isotropic_voigt(self.lam[e], self.mu[e])


def test_material_errors():
    pa = _pa()
    mesh = syn.BoxMesh(n=(2, 2, 2))
    NE = 8
    good = material.packed_upper(syn.random_spd_stiffness(NE))
    with pytest.raises(pa.PaError) as ei:
        pa.Operator.with_material(mesh, 2, pa.PA_MAT_ANISO, good, q=5)
    assert ei.value.code == pa.capi.PA_EUNSUPPORTED
    bad = good.copy()
    bad[3, 0] = -1.0                     # C_xx < 0: not positive definite
    with pytest.raises(pa.PaError) as ei:
        pa.Operator.with_material(mesh, 2, pa.PA_MAT_ANISO, bad)
    assert ei.value.code == pa.capi.PA_EINVAL
    qp = np.ones((NE, 64, 2))
    qp[5, 17, 1] = 0.0                   # mu = 0 at one point
    with pytest.raises(pa.PaError) as ei:
        pa.Operator.with_material(mesh, 2, pa.PA_MAT_QP_ISO, qp)
    assert ei.value.code == pa.capi.PA_EINVAL
    with pytest.raises(pa.PaError) as ei:
        pa.Operator.with_material(mesh, 2, 7, good)
    assert ei.value.code == pa.capi.PA_EINVAL
    op = pa.Operator.with_material(mesh, 2, pa.PA_MAT_ANISO, good)
    with pytest.raises(pa.PaError) as ei:
        op.apply_variant(op.empty().zero_(), variant=pa.capi.PA_VARIANT_UNFUSED_SF)
    assert ei.value.code == pa.capi.PA_EUNSUPPORTED
    # per-point Lame data: the hierarchy needs a coarser level than the finest
    qpop = pa.Operator.with_material(syn.BoxMesh(n=(3, 2, 2), clamped_faces=1), 1, pa.PA_MAT_QP_ISO,
                                     np.ones((12, 27, 2)))
    with pytest.raises(pa.PaError) as ei:
        qpop.hierarchy()
    assert ei.value.code == pa.capi.PA_EUNSUPPORTED
    with pytest.raises(pa.PaError) as ei:   # a mesh without elements is rejected like pa_elast_setup's
        pa.Operator.with_material(syn.BoxMesh(n=(0, 2, 2)), 2, pa.PA_MAT_ANISO, np.zeros((0, 21)))
    assert ei.value.code == pa.capi.PA_EINVAL


@pytest.mark.parametrize("p", [1, 2, 8])
@pytest.mark.parametrize("kind", [1, 2])
def test_material_single_element(p, kind):
    """One element (the smallest workgroup tail), all faces clamped but the top."""
    pa = _pa()
    mesh = syn.BoxMesh(n=(1, 1, 1), L=(0.7, 1.1, 0.9), A=syn.SHEAR_A, clamped_faces=0b011111)
    data, C = _material(kind, 1, p + 2, seed=70 + p)
    op = pa.Operator.with_material(mesh, p, kind, data)
    x = syn.uniform_vector(op.N, seed=4)
    ref = material.GeneralOperator(mesh, p, p + 2, C).apply(x, constrained=True)
    assert _rel(_gpu(op, x, 0), ref) <= TOL[0]


@pytest.mark.parametrize("p", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("dtype", [0, 1])
def test_material_diagonal_parity(p, kind, dtype):
    """Diagonal with general material data (the Jacobi smoother's diagonal) vs the oracle's
    element matrices: per-point Lame data in both layouts (point-major at p = 1), and the
    anisotropic Voigt stiffness."""
    pa = _pa()
    print(f"material diagonal p={p} kind={kind} dtype={dtype}", flush=True)
    mesh = _mesh(p, seed=60 + p) if p < 8 else syn.BoxMesh(n=(2, 1, 1), L=(1.0, 0.6, 0.7), A=syn.SHEAR_A,
                                                            clamped_faces=0b000001)
    NE, q = mesh.num_elements, p + 2
    data, C = _material(kind, NE, q, seed=p)
    op = pa.Operator.with_material(mesh, p, kind, data, dtype=dtype)
    ref = material.GeneralOperator(mesh, p, q, C)
    for flags, constrained in ((0, True), (pa.PA_UNCONSTRAINED, False)):
        d = op.diagonal(flags)
        torch.cuda.synchronize()
        want = ref.diagonal(constrained)
        assert _rel(d.double().cpu().numpy(), want) <= TOL[dtype], flags


def _qp_problem(p, seed, kind=1):
    """A clamped box whose hierarchy has a coarser level, with per-point Lame data that
    varies by +-40% inside every element around its element material (two materials,
    E = 1 and 100, below p = 4), or (kind 2) a random anisotropic stiffness per element."""
    mesh = {1: syn.BoxMesh(n=(4, 4, 4), L=(2.0, 1.0, 1.0), A=syn.SHEAR_A, clamped_faces=1),
            2: syn.graded_mesh((4, 2, 2), seed=seed, L=(2.0, 1.0, 1.0), clamped_faces=1),
            4: syn.graded_mesh((3, 2, 2), seed=seed, L=(1.5, 1.0, 1.0), clamped_faces=1)}[p]
    NE, q = mesh.num_elements, p + 2
    if p < 4:
        lam_e, mu_e = syn.two_material_lame(NE, seed=seed)
    else:   # one base material: a residual of 1e-10 stays within FP64 reach at p = 4
        lam_e, mu_e = (np.full(NE, v) for v in syn.lame_from_young_poisson(1.0, 0.3))
    b = elasticity.body_force_vector(mesh, p, q, (0.1, -0.2, -1.0))
    if kind == 2:   # a general anisotropic stiffness per element around E = 1, nu = 0.3
        lam0, mu0 = syn.lame_from_young_poisson(1.0, 0.3)
        C = syn.random_spd_stiffness(NE, seed=seed + 2, lam=float(lam0), mu=float(mu0), spread=1.0)
        ref = material.GeneralOperator(mesh, p, q, C)
        b[ref.ess] = 0.0
        return mesh, material.packed_upper(C), ref, b
    lam, mu = syn.quadrature_point_lame(lam_e, mu_e, q, seed=seed + 1, spread=0.4)
    ref = material.GeneralOperator(mesh, p, q, material.isotropic_voigt(lam, mu))
    b[ref.ess] = 0.0
    return mesh, np.stack([lam, mu], axis=-1), ref, b


@pytest.mark.parametrize("p", [1, 2, 4])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("kind", [1, 2])
def test_material_solve_vs_direct(p, mode, kind):
    """GMG-PCG with general material data on the finest level (coarser levels take the
    quadrature-weighted element means of per-point data, or the trace-matched isotropic
    stiffness of an anisotropic C): the solution of the constrained system vs a dense
    direct solve of the oracle's assembled matrix, in all three solver modes."""
    pa = _pa()
    print(f"material solve p={p} mode={mode} kind={kind}", flush=True)
    mesh, data, ref, b = _qp_problem(p, seed=30 + p, kind=kind)
    u = solvers.solve_dense(ref.dense(True), b)
    op = pa.Operator.with_material(mesh, p, kind, data)
    x, info, rc = op.solve(torch.tensor(b, device="cuda"), rtol=1e-10, mode=mode, stop=1, cheb_degree=3,
                           h_levels=1 if p == 1 else 0)
    assert rc == 0, (rc, info.iters)
    assert info.rel_res_true <= 1e-10 * (1 + 1e-6)
    got = x.cpu().numpy()
    assert _rel(got, u) <= 1e-7, _rel(got, u)
    print(f"  iters {info.iters} outer {info.outer_iters} err {_rel(got, u):.2e}")


def test_qp_material_solve_fp32_operator():
    """An FP32 operator with per-point data: the FP64 outer operator is rebuilt from the
    host copy of the data, so the FP64 solve meets the same tolerance."""
    pa = _pa()
    mesh, data, ref, b = _qp_problem(2, seed=41)
    u = solvers.solve_dense(ref.dense(True), b)
    op = pa.Operator.with_material(mesh, 2, pa.PA_MAT_QP_ISO, data, dtype=pa.PA_F32)
    for mode in (0, 1):
        x, info, rc = op.solve(torch.tensor(b, device="cuda"), rtol=1e-10, mode=mode, stop=1, cheb_degree=3)
        assert rc == 0 and info.rel_res_true <= 1e-10 * (1 + 1e-6)
        assert _rel(x.cpu().numpy(), u) <= 1e-7


def test_qp_material_full_cantilever():
    """The benchmark's per-point cantilever solve at full size (80x8x8 at p = 8, 8.1M dofs,
    lambda, mu per point x (1 + 0.4 u)): converged to a true FP64 residual of 1e-8, the
    apply at the solution matches the oracle on sampled rows (so the residual the GPU
    reports is the oracle's), and the tip deflection is the beam's."""
    pa = _pa()
    print("per-point material cantilever p=8", flush=True)
    p, q = 8, 10
    mesh = syn.cantilever_mesh(80, 8, 8)
    NE = mesh.num_elements
    lam0, mu0 = syn.lame_from_young_poisson(1.0, 0.3)
    lq, mq = syn.quadrature_point_lame(np.full(NE, lam0), np.full(NE, mu0), q, seed=11, spread=0.4)
    op = pa.Operator.with_material(mesh, p, pa.PA_MAT_QP_ISO, np.stack([lq, mq], axis=-1))
    bref = elasticity.traction_vector(mesh, p, q, 1, (0.0, 0.0, -1.0))
    bref[omesh.essential_mask(mesh, p)] = 0.0
    x, info, rc = op.solve(torch.tensor(bref, device="cuda"), rtol=1e-8, stop=1, cheb_degree=3, h_levels=2)
    assert rc == 0 and info.rel_res_true <= 1e-8 * (1 + 1e-6), (rc, info.rel_res_true)
    xh = x.cpu().numpy()
    y = _gpu(op, xh, pa.PA_UNCONSTRAINED)
    Nn = op.N // 3
    nodes = np.random.default_rng(8).integers(0, Nn, 16)
    ref = _sampled_reference(mesh, p, _LazyIso(lq, mq), xh, nodes)
    got = np.stack([y[nodes], y[Nn + nodes], y[2 * Nn + nodes]], axis=1)
    assert np.abs(got - ref).max() <= 50 * TOL[0] * np.abs(y).max()
    R = omesh.node_coords(mesh, p)
    defl = -xh.reshape(3, -1)[2, np.isclose(R[:, 0], 8.0)].mean()
    assert 0.9 * 2048 < defl < 1.1 * 2048 * 1.012, defl
    print(f"  iters {info.iters} tip {defl:.1f} t_solve {info.t_solve:.3f}s")


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_material_full_size_whole_vector(p):
    """The operator sweep's full-size sheared box (~4.2M dofs), the benchmark's launch, with
    the two per-element materials carried by the general forms: per-point data constant over
    each element's points, and each element's isotropic Voigt stiffness as an anisotropic C.
    Both are the operator the oracle applies to the sweep workload: the whole output vs the
    oracle, FP64 and FP32, over all dofs and over each single-material node set."""
    import fullsize
    pa = _pa()
    mesh = fullsize.mesh(p)
    NE, q = mesh.num_elements, p + 2
    lam, mu = fullsize.lame(p)
    x = fullsize.x_vec(p)
    print(f"material full size whole vector p={p}: oracle", flush=True)
    ref = fullsize.oracle_apply(p)
    qp = np.empty((NE, q ** 3, 2))
    qp[..., 0] = lam[:, None]
    qp[..., 1] = mu[:, None]
    forms = ((pa.PA_MAT_QP_ISO, qp), (pa.PA_MAT_ANISO, material.packed_upper(material.isotropic_voigt(lam, mu))))
    for kind, data in forms:
        for dtype in (0, 1):
            op = pa.Operator.with_material(mesh, p, kind, data, dtype=dtype)
            y = _gpu(op, x, pa.PA_UNCONSTRAINED)
            op.close()
            fullsize.check_whole_vector(y, ref, p, dtype, f"material kind={kind} p={p} dtype={dtype}")


@pytest.mark.parametrize("p", [1, 2, 4, 8])
@pytest.mark.parametrize("kind", [1, 2])
def test_material_eighth_box_whole_vector(p, kind):
    """General material data on the first 1/8 of the sweep's box (~0.5M dofs; many more
    workgroups than the GPU has compute units): random per-point (lambda, mu) (two
    materials x (1 +- 0.3 u)) or a random anisotropic C per element; the whole output vs
    the oracle's strain-displacement form, FP64 and FP32, unconstrained."""
    import fullsize
    pa = _pa()
    sub = fullsize.eighth(p)
    NE, q = sub.num_elements, p + 2
    print(f"material 1/8 box p={p} kind={kind}: oracle", flush=True)
    if kind == pa.PA_MAT_QP_ISO:
        lam_e, mu_e = fullsize.eighth_lame(p)
        lam, mu = syn.quadrature_point_lame(lam_e, mu_e, q, seed=4)
        data, C = np.stack([lam, mu], axis=-1), material.isotropic_voigt(lam, mu)
    else:
        C = syn.random_spd_stiffness(NE, seed=5)
        data = material.packed_upper(C)
    x = fullsize.eighth_x(p)
    ref = material.GeneralOperator(sub, p, q, C).apply(x)
    del C
    for dtype in (0, 1):
        op = pa.Operator.with_material(sub, p, kind, data, dtype=dtype)
        y = _gpu(op, x, pa.PA_UNCONSTRAINED)
        op.close()
        err = _rel(y, ref)
        print(f"  dtype={dtype}: rel err {err:.2e}", flush=True)
        assert err <= TOL[dtype], err
