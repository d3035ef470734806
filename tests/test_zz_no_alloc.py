"""GPU test of pa_elast_apply_noalloc, the apply whose element-boundary partial sums live in
the library's static per-device scratch array: its output must equal pa_elast_apply_ex's
bit for bit (same kernels, fixed summation order), on consecutive calls whose second input
is smaller than the first (the array then still holds the first call's values), for the
structured kernels (p = 1 tile kernel, p >= 2 element kernel), the unstructured kernel and
the accumulate / constrained forms; operators whose element-boundary buffer exceeds the
array are refused with PA_EINVAL and leave y untouched.
"""
import numpy as np
import pytest

import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pa():
    import paper_2601_08374_amd as pa
    return pa


def _tdt(dtype):
    return torch.float64 if dtype == 0 else torch.float32


def _both(op, x, flags, y0=None):
    """(pa_elast_apply_ex, pa_elast_apply_noalloc) outputs on the same input; y0 seeds y for PA_ADD."""
    ya = op.empty() if y0 is None else y0.clone()
    yb = op.empty() if y0 is None else y0.clone()
    op.apply(x, ya, flags=flags)
    op.apply_noalloc(x, yb, flags=flags)
    torch.cuda.synchronize()
    return ya.cpu().numpy(), yb.cpu().numpy()


def _box_op(mesh, p, dtype, seed=1):
    pa = _pa()
    lam, mu = syn.two_material_lame(mesh.num_elements, seed=seed)
    return pa.Operator(mesh, p, lam, mu, q=p + 2, dtype=dtype)


@pytest.mark.parametrize("dtype", [0, 1])
def test_noalloc_equals_apply_large_then_small(dtype):
    pa = _pa()
    # first call: the full-size sheared box at p = 8 (~4.2M dofs), clamped x- and z+ faces
    big = syn.sheared_box_mesh(8)
    big.clamped_faces = 0b100001
    op1 = _box_op(big, 8, dtype)
    print(f"noalloc p=8 sheared box N={op1.N} dtype={dtype}", flush=True)
    x1 = torch.tensor(syn.uniform_vector(op1.N, seed=0), dtype=_tdt(dtype), device="cuda")
    for flags in (0, pa.PA_UNCONSTRAINED):
        ya, yb = _both(op1, x1, flags)
        assert np.array_equal(ya, yb), flags
        assert np.abs(ya).max() > 0
    # second call: a smaller operator (2x3x2 elements, p = 4); the array still holds the
    # first call's partial sums
    small = syn.BoxMesh(n=(2, 3, 2), L=(0.5, 0.9, 0.4), A=syn.SHEAR_A, clamped_faces=0b000100)
    op2 = _box_op(small, 4, dtype, seed=3)
    print(f"noalloc p=4 small box N={op2.N} dtype={dtype}", flush=True)
    x2 = torch.tensor(syn.uniform_vector(op2.N, seed=5), dtype=_tdt(dtype), device="cuda")
    y0 = torch.tensor(syn.uniform_vector(op2.N, seed=6), dtype=_tdt(dtype), device="cuda")
    for flags, seed_y in ((0, False), (pa.PA_ADD, True), (pa.PA_UNCONSTRAINED | pa.PA_ADD, True)):
        ya, yb = _both(op2, x2, flags, y0 if seed_y else None)
        assert np.array_equal(ya, yb), flags


@pytest.mark.parametrize("dtype", [0, 1])
def test_noalloc_tile_kernel_then_unstructured(dtype):
    pa = _pa()
    # p = 1: the tile kernel on the full-size sheared box (1.38M elements)
    m = syn.sheared_box_mesh(1)
    op1 = _box_op(m, 1, dtype)
    print(f"noalloc p=1 sheared box N={op1.N} dtype={dtype}", flush=True)
    x1 = torch.tensor(syn.uniform_vector(op1.N, seed=0), dtype=_tdt(dtype), device="cuda")
    ya, yb = _both(op1, x1, 0)
    assert np.array_equal(ya, yb)
    # then a smaller unstructured mesh (O-grid around a cylinder, p = 3)
    um = syn.ogrid_cylinder(3, n=3, m=2, nz=3, seed=3)
    lam, mu = syn.two_material_lame(um.num_elements, seed=2)
    op2 = pa.Operator.unstructured(um, lam, mu, dtype=dtype)
    print(f"noalloc unstructured p=3 N={op2.N} dtype={dtype}", flush=True)
    x2 = torch.tensor(syn.uniform_vector(op2.N, seed=4), dtype=_tdt(dtype), device="cuda")
    for flags in (0, pa.PA_UNCONSTRAINED):
        ya, yb = _both(op2, x2, flags)
        assert np.array_equal(ya, yb), flags


def test_noalloc_refuses_oversize_operator():
    pa = _pa()
    # p = 2 on the full-size sheared box in FP64: 103 MiB of element-boundary sums > 64 MiB
    op = _box_op(syn.sheared_box_mesh(2), 2, 0)
    x = torch.tensor(syn.uniform_vector(op.N, seed=0), dtype=torch.float64, device="cuda")
    y = torch.full_like(x, 7.0)
    with pytest.raises(pa.capi.PaError) as ei:
        op.apply_noalloc(x, y)
    assert ei.value.code == pa.capi.PA_EINVAL
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    # the same operator in FP32 (half the bytes) is accepted
    op32 = _box_op(syn.sheared_box_mesh(2), 2, 1)
    x32 = x.float()
    ya, yb = _both(op32, x32, 0)
    assert np.array_equal(ya, yb)
