"""Pins of the unstructured-mesh oracle (oracle.geometry.UnstructuredOperator) and of the
mesh descriptions it is fed (synthetic.hex_high_order_nodes and the two generators).

* the numbering is conforming: every element's trilinear map puts a shared node at the
  same point, and element-interior nodes belong to one element;
* a box written as an unstructured mesh (random element order, random orientation of
  every element, renumbered nodes) gives the box operator permuted: against the affine
  oracle (a different route) and against the distorted-box oracle;
* on the O-grid cylinder (vertices shared by three quadrilaterals of the cross-section):
  the volume is that of the prism over the regular polygon, the energy of u = E x is
  (1/2) V e:C:e, the rows of interior nodes of A (E x) vanish (patch test), rigid
  motions lie in the nullspace, and the matrix is symmetric PSD with six zero modes.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import elasticity, geometry, rules


def _node_coords(hm):
    """Coordinates of every node from every element's map; the spread over elements."""
    D = hm.p + 1
    g = rules.gll_nodes(hm.p)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    V8 = hm.vertices[hm.elem_vertices.astype(np.int64)]
    x = geometry.map_points(V8, xi).reshape(-1, 3)
    en = hm.elem_nodes.ravel().astype(np.int64)
    out = np.zeros((hm.num_nodes, 3))
    out[en] = x
    spread = np.abs(out[en] - x).max()
    return out, spread


def _boundary_nodes(hm):
    D = hm.p + 1
    en = hm.elem_nodes.reshape(-1, D, D, D)
    ev = hm.elem_vertices.reshape(-1, 2, 2, 2)   # [e, c, b, a]
    count, where = {}, {}
    for e in range(hm.num_elements):
        for d in range(3):
            for s in range(2):
                sl_v = [slice(None)] * 3
                sl_v[2 - d] = s
                key = tuple(sorted(ev[e][tuple(sl_v)].ravel()))
                count[key] = count.get(key, 0) + 1
                sl_n = [slice(None)] * 3
                sl_n[2 - d] = s * hm.p
                where[key] = en[e][tuple(sl_n)].ravel()
    b = np.zeros(hm.num_nodes, dtype=bool)
    for key, c in count.items():
        if c == 1:
            b[where[key]] = True
    return b


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_numbering_conforming(p):
    for hm in (syn.ogrid_cylinder(p, seed=1),
               syn.box_as_unstructured(syn.BoxMesh(n=(3, 2, 2)),
                                       syn.perturbed_vertices(syn.BoxMesh(n=(3, 2, 2)), 0.2, 1), p)[0],
               syn.box_as_unstructured(syn.BoxMesh(n=(3, 2, 2)),
                                       syn.perturbed_vertices(syn.BoxMesh(n=(3, 2, 2)), 0.2, 1), p,
                                       renumber=False, shuffle_nodes=True)[0]):
        _, spread = _node_coords(hm)
        assert spread <= 1e-14
        counts = np.bincount(hm.elem_nodes.ravel(), minlength=hm.num_nodes)
        assert counts.min() >= 1
        if p >= 2:
            D = p + 1
            inner = hm.elem_nodes.reshape(-1, D, D, D)[:, 1:p, 1:p, 1:p].ravel()
            assert np.all(counts[inner] == 1)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_box_as_unstructured_matches_box(p):
    mesh = syn.graded_mesh((3, 2, 2), seed=p, L=(1.1, 0.9, 1.2), A=syn.random_rotation(p) @ syn.SHEAR_A,
                           clamped_faces=0b010010)
    NE = mesh.num_elements
    rng = np.random.default_rng(p)
    lam, mu = rng.uniform(0.5, 2.0, NE), rng.uniform(0.5, 2.0, NE)
    for amp in (0.0, 0.2):
        verts = syn.perturbed_vertices(mesh, amp=amp, seed=p, interior_only=False)
        hm, node_map, order = syn.box_as_unstructured(mesh, verts, p, seed=p)
        ref_op = (elasticity.Operator(mesh, p, p + 2, lam, mu) if amp == 0.0 else
                  geometry.TrilinearOperator(mesh, p, p + 2, verts, lam, mu))
        un = geometry.UnstructuredOperator(hm, p + 2, lam[order], mu[order])
        xb = syn.uniform_vector(mesh.num_dofs(p), seed=5)
        Nb = mesh.num_nodes(p)
        idx = np.concatenate([node_map + c * Nb for c in range(3)])
        for constrained in (False, True):
            yb = ref_op.apply(xb, constrained=constrained)
            yu = un.apply(xb[idx], constrained=constrained)
            assert np.linalg.norm(yu - yb[idx]) <= 1e-12 * np.linalg.norm(yb)
        # box numbering kept, nodes relabelled at random
        hm2, node_map2, order2 = syn.box_as_unstructured(mesh, verts, p, seed=p + 7, renumber=False,
                                                         shuffle_nodes=True)
        idx2 = np.concatenate([node_map2 + c * Nb for c in range(3)])
        yu2 = geometry.UnstructuredOperator(hm2, p + 2, lam[order2], mu[order2]).apply(xb[idx2], constrained=True)
        yb2 = ref_op.apply(xb, constrained=True)
        assert np.linalg.norm(yu2 - yb2[idx2]) <= 1e-12 * np.linalg.norm(yb2)


def _polygon_volume(n, R, H):
    k = 4 * n
    return H * 0.5 * k * R * R * np.sin(2 * np.pi / k)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_ogrid_volume_energy_patch(p):
    n, m, nz, R, H = 3, 2, 2, 1.0, 1.5
    hm = syn.ogrid_cylinder(p, n=n, m=m, nz=nz, R=R, H=H, seed=4)
    lam, mu = 1.4, 0.7
    op = geometry.UnstructuredOperator(hm, p + 2, lam, mu)
    V = _polygon_volume(n, R, H)
    assert abs(op.volume() - V) <= 1e-13 * V
    X, _ = _node_coords(hm)
    E = np.random.default_rng(p).uniform(-1, 1, (3, 3))
    u = (X @ E.T).T.ravel()
    eps = 0.5 * (E + E.T)
    want = 0.5 * V * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    r = op.apply(u)
    assert abs(0.5 * u @ r - want) <= 1e-12 * abs(want)
    inner = ~_boundary_nodes(hm)
    assert inner.sum() > 0
    inner3 = np.tile(inner, 3)
    assert np.abs(r[inner3]).max() <= 1e-12 * np.abs(r).max()


@pytest.mark.parametrize("p", [1, 2])
def test_ogrid_nullspace_and_spectrum(p):
    hm = syn.ogrid_cylinder(p, n=2, m=1, nz=1, seed=2)
    op = geometry.UnstructuredOperator(hm, p + 2, 1.0, 1.0)
    X, _ = _node_coords(hm)
    W = np.array([[0.0, 0.4, -0.1], [-0.4, 0.0, 0.6], [0.1, -0.6, 0.0]])
    x = syn.uniform_vector(op.N, seed=1)
    nrm = np.linalg.norm(op.apply(x)) / np.linalg.norm(x)
    for u in ((X @ W.T).T.ravel(), np.concatenate([np.zeros(hm.num_nodes), np.ones(hm.num_nodes),
                                                   np.zeros(hm.num_nodes)])):
        assert np.linalg.norm(op.apply(u)) <= 1e-12 * nrm * np.linalg.norm(u)
    if p == 1:
        A = op.dense()
        assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
        ev = np.linalg.eigvalsh(0.5 * (A + A.T))
        assert ev[0] >= -1e-12 * ev[-1]
        assert np.sum(ev < 1e-10 * ev[-1]) == 6
