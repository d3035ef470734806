"""GPU parity of the apply on non-affine (trilinear) hexahedra, both geometry forms
(J^{-1}, w det J stored per quadrature point; Jacobian recomputed per point from the
element's map coefficients), against the oracle's quadrature sum written out
(oracle.geometry.TrilinearOperator).

Tolerances (relative, 2-norm over the output): FP64 1e-12, FP32 1e-5, the bars of the
apply in double and single precision.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import geometry, mesh as omesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}
KINDS = [1, 2]   # PA_GEOM_QP_DATA, PA_GEOM_TRILINEAR


def _pa():
    import paper_2601_08374_amd as pa
    return pa


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _mesh(p, seed):
    # several workgroup tiles with a ragged tail; graded + sheared + rotated boxes whose
    # vertices (boundary ones included) are moved by up to 0.2 of the local spacing
    rot = syn.random_rotation(seed) @ syn.SHEAR_A
    if p <= 3:
        m = syn.graded_mesh((5, 3, 2), seed=seed, L=(1.3, 0.8, 1.0), A=rot, clamped_faces=0b010001)
    elif p <= 5:
        m = syn.graded_mesh((3, 2, 2), seed=seed, L=(1.0, 1.2, 0.9), A=rot, clamped_faces=0b000110)
    else:
        m = syn.BoxMesh(n=(3, 2, 1), L=(1.5, 1.0, 0.6), A=rot, clamped_faces=0b100000)
    return m, syn.perturbed_vertices(m, amp=0.2, seed=seed, interior_only=False)


def _gpu(op, x, flags=0):
    tdt = torch.float64 if op.dtype == 0 else torch.float32
    y = op.apply(torch.tensor(x, dtype=tdt, device="cuda"), flags=flags)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("dtype", [0, 1])
def test_geometry_parity(p, kind, dtype):
    pa = _pa()
    print(f"geometry parity p={p} kind={kind} dtype={dtype}", flush=True)
    mesh, verts = _mesh(p, seed=80 + p)
    NE = mesh.num_elements
    rng = np.random.default_rng(p)
    lam, mu = rng.uniform(0.3, 3.0, NE), rng.uniform(0.3, 3.0, NE)
    ref_op = geometry.TrilinearOperator(mesh, p, p + 2, verts, lam, mu)
    op = pa.Operator.with_geometry(mesh, p, verts, lam, mu, kind=kind, dtype=dtype)
    x = syn.uniform_vector(mesh.num_dofs(p), seed=p)
    for flags, constrained in ((0, True), (pa.PA_UNCONSTRAINED, False)):
        ref = ref_op.apply(x, constrained=constrained)
        y = _gpu(op, x, flags)
        assert _rel(y, ref) <= TOL[dtype], (flags, _rel(y, ref))


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_affine_vertices_match_box_operator(p):
    """Vertices on the box map: both non-affine forms reproduce the affine operator."""
    pa = _pa()
    mesh, _ = _mesh(p, seed=90 + p)
    verts = syn.perturbed_vertices(mesh, amp=0.0)
    NE = mesh.num_elements
    lam, mu = syn.two_material_lame(NE, seed=2)
    x = syn.uniform_vector(mesh.num_dofs(p), seed=5)
    base = _gpu(pa.Operator(mesh, p, lam, mu), x)
    for kind in KINDS:
        y = _gpu(pa.Operator.with_geometry(mesh, p, verts, lam, mu, kind=kind), x)
        assert _rel(y, base) <= TOL[0], kind


@pytest.mark.parametrize("p", [1, 3, 8])
def test_patch_test_on_gpu(p):
    """u = E x on a distorted mesh: rows of interior nodes vanish (FP64, both forms)."""
    pa = _pa()
    mesh = syn.BoxMesh(n=(3, 3, 2), L=(1.0, 1.1, 0.9), A=syn.SHEAR_A)
    verts = syn.perturbed_vertices(mesh, amp=0.22, seed=3, interior_only=False)
    E = np.random.default_rng(4).uniform(-1, 1, (3, 3))
    u = (geometry.node_coords(mesh, verts, p) @ E.T).T.ravel()
    Nx, Ny, Nz = omesh.grid_shape(mesh, p)
    gz, gy, gx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    inner = ((gx > 0) & (gx < Nx - 1) & (gy > 0) & (gy < Ny - 1) & (gz > 0) & (gz < Nz - 1)).ravel()
    inner3 = np.concatenate([inner, inner, inner])
    for kind in KINDS:
        r = _gpu(pa.Operator.with_geometry(mesh, p, verts, 1.3, 0.8, kind=kind), u, pa.PA_UNCONSTRAINED)
        assert np.abs(r[inner3]).max() <= 1e-12 * np.abs(r).max(), kind


def _patch_row(mesh, verts, p, lam, mu, x, node):
    """The row of A x at one node from the oracle on the sub-box of elements around it."""
    Nx, Ny, Nz = omesh.grid_shape(mesh, p)
    Nn = Nx * Ny * Nz
    g = (node % Nx, (node // Nx) % Ny, node // (Nx * Ny))
    lo, hi = [], []
    for a in range(3):
        e_hi = min(g[a] // p, mesh.n[a] - 1)
        e_lo = e_hi - 1 if (g[a] % p == 0 and g[a] > 0 and e_hi == g[a] // p) else e_hi
        lo.append(e_lo)
        hi.append(e_hi)
    n = tuple(hi[a] - lo[a] + 1 for a in range(3))
    sub = syn.BoxMesh(n=n)
    n0, n1 = mesh.n[0], mesh.n[1]
    K, J, I = np.meshgrid(np.arange(lo[2], hi[2] + 2), np.arange(lo[1], hi[1] + 2), np.arange(lo[0], hi[0] + 2),
                          indexing="ij")
    sv = verts[(I + (n0 + 1) * (J + (n1 + 1) * K)).ravel()]
    ee = [(lo[0] + i) + n0 * ((lo[1] + j) + n1 * (lo[2] + k))
          for k in range(n[2]) for j in range(n[1]) for i in range(n[0])]
    sx, sy, sz = (n[a] * p + 1 for a in range(3))
    K, J, I = np.meshgrid(np.arange(lo[2] * p, lo[2] * p + sz), np.arange(lo[1] * p, lo[1] * p + sy),
                          np.arange(lo[0] * p, lo[0] * p + sx), indexing="ij")
    gnodes = (I + Nx * (J + Ny * K)).ravel()
    xs = np.concatenate([x[c * Nn + gnodes] for c in range(3)])
    ys = geometry.TrilinearOperator(sub, p, p + 2, sv, lam[ee], mu[ee]).apply(xs)
    loc = (g[0] - lo[0] * p) + sx * ((g[1] - lo[1] * p) + sy * (g[2] - lo[2] * p))
    sn = sx * sy * sz
    return ys[[loc, sn + loc, 2 * sn + loc]]


@pytest.mark.parametrize("p", [1, 2, 4, 8])
@pytest.mark.parametrize("kind", KINDS)
def test_geometry_full_size_sampled(p, kind):
    """The distorted sheared box at the operator sweep's full size (~4.2M dofs), same launch
    as the benchmark: sampled rows vs the oracle on the elements around each node."""
    pa = _pa()
    print(f"geometry full size p={p} kind={kind}", flush=True)
    mesh = syn.sheared_box_mesh(p)
    verts = syn.perturbed_vertices(mesh, amp=0.2, seed=17)
    lam, mu = syn.two_material_lame(mesh.num_elements, seed=1)
    op = pa.Operator.with_geometry(mesh, p, verts, lam, mu, kind=kind)
    x = syn.uniform_vector(op.N, seed=0)
    y = _gpu(op, x, pa.PA_UNCONSTRAINED)
    Nn = op.N // 3
    scale = np.abs(y).max()
    for node in np.random.default_rng(6).integers(0, Nn, 16):
        ref = _patch_row(mesh, verts, p, lam, mu, x, int(node))
        got = y[[node, Nn + node, 2 * Nn + node]]
        assert np.abs(got - ref).max() <= 50 * TOL[0] * scale, (node, got, ref)


@pytest.mark.parametrize("p", [1, 2, 8])
def test_geometry_single_element(p):
    pa = _pa()
    mesh = syn.BoxMesh(n=(1, 1, 1), L=(0.7, 1.1, 0.9), A=syn.SHEAR_A, clamped_faces=0b011111)
    verts = syn.perturbed_vertices(mesh, amp=0.2, seed=11, interior_only=False)
    x = syn.uniform_vector(mesh.num_dofs(p), seed=4)
    ref = geometry.TrilinearOperator(mesh, p, p + 2, verts, 1.1, 0.7).apply(x, constrained=True)
    for kind in KINDS:
        assert _rel(_gpu(pa.Operator.with_geometry(mesh, p, verts, 1.1, 0.7, kind=kind), x), ref) <= TOL[0]


def test_geometry_errors():
    pa = _pa()
    mesh = syn.BoxMesh(n=(2, 2, 2))
    verts = syn.perturbed_vertices(mesh, amp=0.1, seed=1, interior_only=False)
    with pytest.raises(pa.PaError) as ei:
        pa.Operator.with_geometry(mesh, 2, verts, 1.0, 1.0, q=5)
    assert ei.value.code == pa.capi.PA_EUNSUPPORTED
    bad = verts.copy()
    bad[26] = bad[0] - 0.05                  # the far corner behind the origin: an inverted element
    for kind in KINDS:
        with pytest.raises(pa.PaError) as ei:
            pa.Operator.with_geometry(mesh, 2, bad, 1.0, 1.0, kind=kind)
        assert ei.value.code == pa.capi.PA_EINVAL
    nan = verts.copy()
    nan[5, 1] = np.nan
    with pytest.raises(pa.PaError) as ei:
        pa.Operator.with_geometry(mesh, 2, nan, 1.0, 1.0)
    assert ei.value.code == pa.capi.PA_EINVAL
    with pytest.raises(pa.PaError) as ei:
        pa.Operator.with_geometry(mesh, 2, verts, 1.0, 1.0, kind=7)
    assert ei.value.code == pa.capi.PA_EINVAL
    with pytest.raises(ValueError):
        pa.Operator.with_geometry(mesh, 2, verts[:-1], 1.0, 1.0)
    op = pa.Operator.with_geometry(mesh, 2, verts, 1.0, 1.0)
    for call in (lambda: op.diagonal(), lambda: op.hierarchy(), lambda: op.rhs((0.0, 0.0, 1.0)),
                 lambda: op.apply_variant(op.empty().zero_(), variant=pa.capi.PA_VARIANT_UNFUSED_SF)):
        with pytest.raises(pa.PaError) as ei:
            call()
        assert ei.value.code == pa.capi.PA_EUNSUPPORTED


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_geometry_full_size_whole_vector(p):
    """The operator sweep's full-size sheared box (~4.2M dofs), the benchmark's launch, with its
    exact vertices given to both trilinear forms: the trilinear map of a parallelepiped is
    the affine map, so both equal the operator the oracle applies to the sweep workload.
    The whole output vs the oracle, FP64 and FP32, over all dofs and each material's nodes."""
    import fullsize
    pa = _pa()
    mesh = fullsize.mesh(p)
    lam, mu = fullsize.lame(p)
    x = fullsize.x_vec(p)
    verts = syn.perturbed_vertices(mesh, amp=0.0)
    print(f"geometry full size whole vector p={p}: oracle", flush=True)
    ref = fullsize.oracle_apply(p)
    for kind in KINDS:
        for dtype in (0, 1):
            op = pa.Operator.with_geometry(mesh, p, verts, lam, mu, kind=kind, dtype=dtype)
            y = _gpu(op, x, pa.PA_UNCONSTRAINED)
            op.close()
            fullsize.check_whole_vector(y, ref, p, dtype, f"geometry kind={kind} p={p} dtype={dtype}")


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_geometry_eighth_box_whole_vector(p):
    """The distorted first 1/8 of the sweep's box (~0.5M dofs, interior vertices moved by up
    to 0.2 of the spacing): both geometry forms, the whole output vs the oracle's quadrature
    sum with per-point Jacobians, FP64 and FP32."""
    import fullsize
    pa = _pa()
    sub = fullsize.eighth(p)
    lam, mu = fullsize.eighth_lame(p)
    print(f"geometry 1/8 box p={p}: oracle", flush=True)
    ref = fullsize.eighth_trilinear_oracle(p)
    x = fullsize.eighth_x(p)
    for kind in KINDS:
        for dtype in (0, 1):
            op = pa.Operator.with_geometry(sub, p, fullsize.eighth_vertices(p), lam, mu, kind=kind, dtype=dtype)
            y = _gpu(op, x, pa.PA_UNCONSTRAINED)
            op.close()
            err = _rel(y, ref)
            print(f"  kind={kind} dtype={dtype}: rel err {err:.2e}", flush=True)
            assert err <= TOL[dtype], err
