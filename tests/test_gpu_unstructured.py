"""GPU parity of the apply on unstructured hexahedral meshes (explicit element-to-node
map) against the oracle (oracle.geometry.UnstructuredOperator): the O-grid cylinder and
boxes written with random element order, orientation and node numbering.

Tolerances (relative, 2-norm over the output): FP64 1e-12, FP32 1e-5, the bars of the
apply in double and single precision.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import geometry

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


def _pa():
    import paper_2601_08374_amd as pa
    return pa


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _gpu(op, x, flags=0):
    tdt = torch.float64 if op.dtype == 0 else torch.float32
    y = op.apply(torch.tensor(x, dtype=tdt, device="cuda"), flags=flags)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def _ogrid(p, seed):
    # several workgroup tiles with a ragged tail at every p
    if p <= 3:
        return syn.ogrid_cylinder(p, n=3, m=2, nz=3, seed=seed)
    if p <= 5:
        return syn.ogrid_cylinder(p, n=2, m=1, nz=2, seed=seed)
    return syn.ogrid_cylinder(p, n=2, m=1, nz=1, seed=seed)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("dtype", [0, 1])
def test_ogrid_parity(p, dtype):
    pa = _pa()
    print(f"unstructured O-grid p={p} dtype={dtype}", flush=True)
    hm = _ogrid(p, seed=p)
    NE = hm.num_elements
    rng = np.random.default_rng(p)
    lam, mu = rng.uniform(0.3, 3.0, NE), rng.uniform(0.3, 3.0, NE)
    ref_op = geometry.UnstructuredOperator(hm, p + 2, lam, mu)
    op = pa.Operator.unstructured(hm, lam, mu, dtype=dtype)
    x = syn.uniform_vector(hm.num_dofs, seed=p)
    for flags, constrained in ((0, True), (pa.PA_UNCONSTRAINED, False)):
        ref = ref_op.apply(x, constrained=constrained)
        assert _rel(_gpu(op, x, flags), ref) <= TOL[dtype], flags


@pytest.mark.parametrize("p", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("renumber", [True, False])
def test_box_as_unstructured_parity(p, renumber):
    """A distorted box with random element order and orientation: parity with the oracle
    and agreement with the structured trilinear operator on the same geometry."""
    pa = _pa()
    mesh = syn.BoxMesh(n=(4, 3, 2) if p <= 3 else (3, 2, 2), L=(1.2, 1.0, 0.8), A=syn.SHEAR_A,
                       clamped_faces=0b001001)
    verts = syn.perturbed_vertices(mesh, amp=0.2, seed=p, interior_only=False)
    hm, node_map, order = syn.box_as_unstructured(mesh, verts, p, seed=10 + p, renumber=renumber,
                                                  shuffle_nodes=not renumber)
    NE = mesh.num_elements
    lam, mu = syn.two_material_lame(NE, seed=p)
    x = syn.uniform_vector(hm.num_dofs, seed=2)
    ref = geometry.UnstructuredOperator(hm, p + 2, lam[order], mu[order]).apply(x, constrained=True)
    y = _gpu(pa.Operator.unstructured(hm, lam[order], mu[order]), x)
    assert _rel(y, ref) <= TOL[0]
    Nb = mesh.num_nodes(p)
    idx = np.concatenate([node_map + c * Nb for c in range(3)])
    xb = np.empty(3 * Nb)
    xb[idx] = x
    yb = _gpu(pa.Operator.with_geometry(mesh, p, verts, lam, mu, kind=pa.PA_GEOM_TRILINEAR), xb)
    assert _rel(y, yb[idx]) <= TOL[0]


@pytest.mark.parametrize("p", [2, 4])
def test_clamped_interior_and_isolated_nodes(p):
    """Clamp flags on element-interior nodes, and nodes that belong to no element."""
    pa = _pa()
    hm = _ogrid(p, seed=3)
    extra = 5
    rng = np.random.default_rng(p)
    cl = rng.random(hm.num_nodes + extra) < 0.2
    hm2 = syn.HexMesh(vertices=hm.vertices, elem_vertices=hm.elem_vertices, p=p, elem_nodes=hm.elem_nodes,
                      num_nodes=hm.num_nodes + extra, clamped=cl)
    NE = hm.num_elements
    lam, mu = rng.uniform(0.5, 2.0, NE), rng.uniform(0.5, 2.0, NE)
    op = pa.Operator.unstructured(hm2, lam, mu)
    ref_op = geometry.UnstructuredOperator(hm2, p + 2, lam, mu)
    x = syn.uniform_vector(hm2.num_dofs, seed=9)
    for flags, constrained in ((0, True), (pa.PA_UNCONSTRAINED, False)):
        assert _rel(_gpu(op, x, flags), ref_op.apply(x, constrained=constrained)) <= TOL[0]


@pytest.mark.parametrize("dtype", [0, 1])
def test_unstructured_add_flag(dtype):
    pa = _pa()
    hm = _ogrid(3, seed=5)
    NE = hm.num_elements
    op = pa.Operator.unstructured(hm, np.full(NE, 1.2), np.full(NE, 0.9), dtype=dtype)
    x = syn.uniform_vector(hm.num_dofs, seed=1)
    y0 = syn.uniform_vector(hm.num_dofs, seed=2)
    tdt = torch.float64 if dtype == 0 else torch.float32
    yt = torch.tensor(y0, dtype=tdt, device="cuda")
    op.apply(torch.tensor(x, dtype=tdt, device="cuda"), yt, flags=pa.PA_ADD)
    ref = y0 + geometry.UnstructuredOperator(hm, 5, 1.2, 0.9).apply(x, constrained=True)
    # a constrained apply with PA_ADD adds the input on clamped rows
    ref[np.tile(hm.clamped, 3)] = (y0 + x)[np.tile(hm.clamped, 3)]
    assert _rel(yt.double().cpu().numpy(), ref) <= TOL[dtype]


def _patch_row_unstructured(hm, x, lam, mu, node, node_elems):
    """The row of A x at one node from the oracle on the elements that contain it."""
    els = node_elems[node]
    sub_nodes, inv = np.unique(hm.elem_nodes[els].ravel(), return_inverse=True)
    sub = syn.HexMesh(vertices=hm.vertices, elem_vertices=hm.elem_vertices[els], p=hm.p,
                      elem_nodes=inv.reshape(len(els), -1).astype(np.int32), num_nodes=len(sub_nodes),
                      clamped=np.zeros(len(sub_nodes), dtype=bool))
    nn = hm.num_nodes
    xs = np.concatenate([x[c * nn + sub_nodes] for c in range(3)])
    ys = geometry.UnstructuredOperator(sub, hm.p + 2, lam[els], mu[els]).apply(xs)
    k = int(np.searchsorted(sub_nodes, node))
    return ys[[k, len(sub_nodes) + k, 2 * len(sub_nodes) + k]]


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_unstructured_full_size_sampled(p):
    """The distorted sheared box at the operator sweep's full size (~4.2M dofs) as an
    unstructured mesh (random element orientations), same launch as the benchmark:
    sampled rows vs the oracle on the elements around each node."""
    pa = _pa()
    print(f"unstructured full size p={p}", flush=True)
    mesh = syn.sheared_box_mesh(p)
    verts = syn.perturbed_vertices(mesh, amp=0.2, seed=17)
    hm, node_map, order = syn.box_as_unstructured(mesh, verts, p, seed=1, permute=False, renumber=False)
    lam, mu = syn.two_material_lame(mesh.num_elements, seed=1)
    op = pa.Operator.unstructured(hm, lam[order], mu[order])
    x = syn.uniform_vector(op.N, seed=0)
    y = _gpu(op, x, pa.PA_UNCONSTRAINED)
    nn = hm.num_nodes
    nodes = np.random.default_rng(6).integers(0, nn, 12)
    want = set(int(n) for n in nodes)
    node_elems = {n: [] for n in want}
    hit = np.isin(hm.elem_nodes, list(want))
    for e, a in zip(*np.nonzero(hit)):
        node_elems[int(hm.elem_nodes[e, a])].append(int(e))
    scale = np.abs(y).max()
    for node in want:
        ref = _patch_row_unstructured(hm, x, lam[order], mu[order], node, node_elems)
        got = y[[node, nn + node, 2 * nn + node]]
        assert np.abs(got - ref).max() <= 50 * TOL[0] * scale, (node, got, ref)


def test_unstructured_errors():
    pa = _pa()
    hm = _ogrid(2, seed=1)
    NE = hm.num_elements

    def make(**kw):
        d = dict(vertices=hm.vertices, elem_vertices=hm.elem_vertices, p=hm.p, elem_nodes=hm.elem_nodes,
                 num_nodes=hm.num_nodes, clamped=hm.clamped)
        d.update(kw)
        return syn.HexMesh(**d)

    def code(h, **kw):
        with pytest.raises(pa.PaError) as ei:
            pa.Operator.unstructured(h, 1.0, 1.0, **kw)
        return ei.value.code

    assert code(hm, q=5) == pa.capi.PA_EUNSUPPORTED
    bad = hm.elem_nodes.copy()
    bad[0, 13] = bad[1, 13]                  # an element-interior node shared by two elements
    assert code(make(elem_nodes=bad)) == pa.capi.PA_EINVAL
    bad = hm.elem_nodes.copy()
    bad[2, 0] = hm.num_nodes                 # node index out of range
    assert code(make(elem_nodes=bad)) == pa.capi.PA_EINVAL
    bad = hm.elem_nodes.copy()
    bad[2, 1] = bad[2, 0]                    # a node listed twice in one element
    assert code(make(elem_nodes=bad)) == pa.capi.PA_EINVAL
    bad = hm.elem_vertices.copy()
    bad[3, 0] = len(hm.vertices)             # vertex index out of range
    assert code(make(elem_vertices=bad)) == pa.capi.PA_EINVAL
    bad = hm.elem_vertices.copy()
    bad[3] = bad[3][[1, 0, 3, 2, 5, 4, 7, 6]]   # mirrored element: det J < 0
    assert code(make(elem_vertices=bad)) == pa.capi.PA_EINVAL
    op = pa.Operator.unstructured(hm, np.full(NE, 1.0), np.full(NE, 1.0))
    for call in (lambda: op.diagonal(), lambda: op.hierarchy(), lambda: op.rhs((0.0, 0.0, 1.0)),
                 lambda: op.apply_variant(op.empty().zero_(), variant=pa.capi.PA_VARIANT_UNFUSED_SF)):
        with pytest.raises(pa.PaError) as ei:
            call()
        assert ei.value.code == pa.capi.PA_EUNSUPPORTED


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_unstructured_full_size_whole_vector(p):
    """The operator sweep's full-size sheared box (~4.2M dofs) with its exact vertices, written
    as an unstructured mesh (elements in random order, each in a random orientation, box node
    numbering): the same operator as the oracle's on the sweep workload.  The whole output
    (mapped back to box nodes) vs the oracle, FP64 and FP32, over all dofs and each
    material's nodes."""
    import fullsize
    pa = _pa()
    mesh = fullsize.mesh(p)
    lam, mu = fullsize.lame(p)
    x = fullsize.x_vec(p)
    verts = syn.perturbed_vertices(mesh, amp=0.0)
    hm, node_map, order = syn.box_as_unstructured(mesh, verts, p, seed=3, permute=True, renumber=False)
    Nn = mesh.num_nodes(p)
    perm = np.concatenate([c * Nn + node_map for c in range(3)])   # unstructured dof -> box dof
    print(f"unstructured full size whole vector p={p}: oracle", flush=True)
    ref = fullsize.oracle_apply(p)
    for dtype in (0, 1):
        op = pa.Operator.unstructured(hm, lam[order], mu[order], dtype=dtype)
        yu = _gpu(op, x[perm], pa.PA_UNCONSTRAINED)
        op.close()
        y = np.empty_like(yu)
        y[perm] = yu
        fullsize.check_whole_vector(y, ref, p, dtype, f"unstructured p={p} dtype={dtype}")


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_unstructured_eighth_box_whole_vector(p):
    """The distorted first 1/8 of the sweep's box (~0.5M dofs) as an unstructured mesh with
    elements and nodes shuffled and every element in a random orientation: the whole output
    (mapped back to box nodes) vs the oracle's quadrature sum on the box, FP64 and FP32."""
    import fullsize
    pa = _pa()
    sub = fullsize.eighth(p)
    lam, mu = fullsize.eighth_lame(p)
    x = fullsize.eighth_x(p)
    hm, node_map, order = syn.box_as_unstructured(sub, fullsize.eighth_vertices(p), p, seed=4, permute=True,
                                                  renumber=False, shuffle_nodes=True)
    Nn = sub.num_nodes(p)
    perm = np.concatenate([c * Nn + node_map for c in range(3)])
    print(f"unstructured 1/8 box p={p}: oracle", flush=True)
    ref = fullsize.eighth_trilinear_oracle(p)
    for dtype in (0, 1):
        op = pa.Operator.unstructured(hm, lam[order], mu[order], dtype=dtype)
        yu = _gpu(op, x[perm], pa.PA_UNCONSTRAINED)
        op.close()
        y = np.empty_like(yu)
        y[perm] = yu
        err = _rel(y, ref)
        print(f"  dtype={dtype}: rel err {err:.2e}", flush=True)
        assert err <= TOL[dtype], err
