"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle scripts.

This module only *describes* workloads: structured box meshes (element counts,
box lengths, an optional global affine map and optional graded node
coordinates, clamped faces), per-element material parameters and random
vectors.  It holds none of the elasticity method's arithmetic: element
Jacobians, basis functions, quadrature, operators and solvers live on each side
of the parity check separately (the HIP library and the oracle).

Conventions (all shared by both sides through this description only):

* Elements are numbered lexicographically with ``ex`` fastest.
* ``clamped_faces`` is a bitmask: bit0 x-, bit1 x+, bit2 y-, bit3 y+, bit4 z-, bit5 z+.
* Random streams use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

FACE_XMIN, FACE_XMAX, FACE_YMIN, FACE_YMAX, FACE_ZMIN, FACE_ZMAX = 0, 1, 2, 3, 4, 5


@dataclasses.dataclass
class BoxMesh:
    """A structured box of n[0] x n[1] x n[2] hexahedra.

    Reference node coordinates along axis ``a`` are ``grade[a]`` (length
    ``n[a]+1``, strictly increasing) or uniform on ``[0, L[a]]``; the physical
    point is ``A @ X + x0`` with ``det(A) > 0``, so every element is an affine
    parallelepiped.
    """

    n: tuple
    L: tuple = (1.0, 1.0, 1.0)
    A: np.ndarray = dataclasses.field(default_factory=lambda: np.eye(3))
    x0: tuple = (0.0, 0.0, 0.0)
    grade: Optional[Sequence[Optional[np.ndarray]]] = None
    clamped_faces: int = 0

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        self.L = tuple(float(v) for v in self.L)
        self.A = np.asarray(self.A, dtype=np.float64).reshape(3, 3)
        self.x0 = tuple(float(v) for v in self.x0)
        if self.grade is not None:
            g = []
            for a in range(3):
                ga = self.grade[a]
                g.append(None if ga is None else np.ascontiguousarray(ga, dtype=np.float64))
            self.grade = tuple(g)

    @property
    def num_elements(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def axis_nodes(self, a: int) -> np.ndarray:
        """Vertex coordinates along reference axis ``a`` (length n[a]+1)."""
        if self.grade is not None and self.grade[a] is not None:
            return np.asarray(self.grade[a], dtype=np.float64)
        return np.linspace(0.0, self.L[a], self.n[a] + 1)

    def num_nodes(self, p: int) -> int:
        return (self.n[0] * p + 1) * (self.n[1] * p + 1) * (self.n[2] * p + 1)

    def num_dofs(self, p: int) -> int:
        return 3 * self.num_nodes(p)


def lame_from_young_poisson(E, nu):
    """Lame parameters of an isotropic material from Young's modulus and Poisson ratio."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def uniform_vector(n: int, seed: int = 0, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


# --------------------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------------------

SHEAR_A = np.array([[1.0, 0.2, 0.2], [0.0, 1.0, 0.2], [0.0, 0.0, 1.0]])


def unit_cube_4(clamped: bool = False) -> BoxMesh:
    """Unit cube, 4x4x4 elements (clamped on x=0 when ``clamped``)."""
    return BoxMesh(n=(4, 4, 4), L=(1.0, 1.0, 1.0), clamped_faces=(1 << FACE_XMIN) if clamped else 0)


def sheared_box_mesh(p: int) -> BoxMesh:
    """Fixed-size (~4.2M dofs) sheared box of the operator sweep.

    The reference box [0,1.25]^2 x [0,1] is split into (120/p,120/p,96/p) cubes
    for p in {1,2,3,4,6,8}; p=5 and p=7 use (24,24,19) and (17,17,14), the
    nearly-cubic counts that keep ~4.2M dofs.  The global map A is a shear with
    0.2 above the diagonal (det A = 1).
    """
    table = {1: (120, 120, 96), 2: (60, 60, 48), 3: (40, 40, 32), 4: (30, 30, 24),
             5: (24, 24, 19), 6: (20, 20, 16), 7: (17, 17, 14), 8: (15, 15, 12)}
    n = table[p]
    return BoxMesh(n=n, L=(1.25, 1.25, 1.0), A=SHEAR_A.copy())


def two_material_lame(num_elements: int, seed: int = 1, E=(1.0, 100.0), nu: float = 0.3):
    """Per-element Lame parameters, material drawn uniformly from two (seeded)."""
    mat = np.random.default_rng(seed).integers(0, 2, num_elements)
    Es = np.where(mat == 0, E[0], E[1])
    return lame_from_young_poisson(Es, np.full(num_elements, nu))


def random_spd_stiffness(num: int, seed: int = 11, lam: float = 1.0, mu: float = 1.0,
                         spread: float = 0.5) -> np.ndarray:
    """[num, 6, 6] symmetric positive definite Voigt stiffnesses: an isotropic matrix
    (lam, mu) plus spread * M M^T / 6 with M ~ U[-1,1]^{6x6} (general anisotropy)."""
    rng = np.random.default_rng(seed)
    base = np.zeros((6, 6))
    base[:3, :3] = lam
    base += np.diag([2 * mu, 2 * mu, 2 * mu, mu, mu, mu])
    M = rng.uniform(-1.0, 1.0, (num, 6, 6))
    return base[None] + spread * np.einsum("nij,nkj->nik", M, M) / 6.0


def quadrature_point_lame(lam_e, mu_e, q: int, seed: int = 13, spread: float = 0.3):
    """Per-point Lame parameters [NE, q^3]: the element values times (1 + spread u),
    u ~ U[-1,1] independently per point (point alpha = qx + q (qy + q qz))."""
    rng = np.random.default_rng(seed)
    lam_e = np.asarray(lam_e, dtype=np.float64)
    mu_e = np.asarray(mu_e, dtype=np.float64)
    n = lam_e.shape[0]
    f1 = 1.0 + spread * rng.uniform(-1.0, 1.0, (n, q ** 3))
    f2 = 1.0 + spread * rng.uniform(-1.0, 1.0, (n, q ** 3))
    return lam_e[:, None] * f1, mu_e[:, None] * f2


def cantilever_mesh(nx: int = 80, ny: int = 8, nz: int = 8, length: float = 8.0) -> BoxMesh:
    """8:1:1 cantilever [0,8]x[0,1]^2 clamped at x=0 (traction goes on x=8)."""
    return BoxMesh(n=(nx, ny, nz), L=(length, 1.0, 1.0), clamped_faces=1 << FACE_XMIN)


def graded_mesh(n, seed: int, L=(1.0, 1.0, 1.0), A=None, clamped_faces: int = 0,
                spread: float = 0.35) -> BoxMesh:
    """A box with random strictly-increasing per-axis vertex coordinates."""
    rng = np.random.default_rng(seed)
    grade = []
    for a in range(3):
        h = rng.uniform(1.0 - spread, 1.0 + spread, n[a])
        x = np.concatenate([[0.0], np.cumsum(h)])
        grade.append(x * (L[a] / x[-1]))
    return BoxMesh(n=n, L=L, A=np.eye(3) if A is None else A, grade=grade, clamped_faces=clamped_faces)


def perturbed_vertices(mesh: BoxMesh, amp: float = 0.2, seed: int = 17, interior_only: bool = True) -> np.ndarray:
    """Vertex positions [(n0+1)(n1+1)(n2+1), 3] of a distorted box: the box vertices
    (A X + x0, vertex (i,j,k) at i + (n0+1)(j + (n1+1)k)) moved by amp times the
    smallest local reference spacing times U[-1,1]^3, on interior vertices only or on
    all of them.  With amp below ~0.25 every element keeps a positive Jacobian."""
    rng = np.random.default_rng(seed)
    ax = [np.asarray(mesh.axis_nodes(a), dtype=np.float64) for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    R = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    # smallest spacing of the reference cells touching each vertex, per axis
    hs = []
    for a in range(3):
        d = np.diff(ax[a])
        h = np.minimum(np.concatenate([[d[0]], d]), np.concatenate([d, [d[-1]]]))
        hs.append(h)
    Hz, Hy, Hx = np.meshgrid(hs[2], hs[1], hs[0], indexing="ij")
    H = np.minimum(np.minimum(Hx, Hy), Hz).ravel()
    dR = amp * H[:, None] * rng.uniform(-1.0, 1.0, R.shape)
    if interior_only:
        n0, n1, n2 = mesh.n
        k, j, i = np.meshgrid(np.arange(n2 + 1), np.arange(n1 + 1), np.arange(n0 + 1), indexing="ij")
        edge = (i == 0) | (i == n0) | (j == 0) | (j == n1) | (k == 0) | (k == n2)
        dR[edge.ravel()] = 0.0
    return (R + dR) @ mesh.A.T + np.asarray(mesh.x0)


# ---------------------------------------------------------------- unstructured hex meshes
# An unstructured hexahedral mesh is described by vertex positions [NV, 3], the 8
# vertices of every element [NE, 8] (local vertex a + 2(b + 2c) at reference corner
# (a, b, c)) and, for order p, the global node of every local node [NE, (p+1)^3]
# (local node ix + D(iy + D iz)).  The helpers below only build such descriptions.

def _cube_rotations():
    """The 24 proper rotations of the reference cube as (perm, flip): new coordinate k
    reads old coordinate perm[k], mirrored when flip[k]."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        sign_p = np.linalg.det(np.eye(3)[list(perm)])
        for flips in itertools.product((0, 1), repeat=3):
            if sign_p * (-1) ** sum(flips) > 0:
                out.append((perm, flips))
    return out


def hex_high_order_nodes(ev: np.ndarray, p: int, num_vertices: Optional[int] = None):
    """Conforming global numbering of the order-p nodes of a hex mesh given only its
    element vertices ev [NE, 8]: vertices first (node = vertex id), then edge-interior,
    face-interior and cell-interior nodes.  Shared edges and faces are numbered in a
    frame fixed by their global vertex ids, so neighbouring elements agree whatever
    their local orientation.  Returns (elem_nodes [NE, D^3] int32, num_nodes)."""
    ev = np.asarray(ev, dtype=np.int64)
    NE = ev.shape[0]
    NV = int(ev.max()) + 1 if num_vertices is None else int(num_vertices)
    D, m = p + 1, p - 1
    out = np.empty((NE, D, D, D), dtype=np.int64)      # [e, iz, iy, ix]
    edges, faces = {}, {}
    base_edge = NV

    def corner(e, a, b, c):
        return ev[e, a + 2 * (b + 2 * c)]

    for e in range(NE):
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    out[e, c * p, b * p, a * p] = corner(e, a, b, c)
    if p == 1:
        return out.reshape(NE, -1).astype(np.int32), NV
    # edges: the three directions, each with 4 positions of the other two corners
    for e in range(NE):
        for d in range(3):
            o1, o2 = [k for k in range(3) if k != d]
            for s1 in range(2):
                for s2 in range(2):
                    lo, hi = [0, 0, 0], [0, 0, 0]
                    lo[o1] = hi[o1] = s1
                    lo[o2] = hi[o2] = s2
                    hi[d] = 1
                    vA, vB = corner(e, *lo), corner(e, *hi)
                    key = (min(vA, vB), max(vA, vB))
                    if key not in edges:
                        edges[key] = len(edges)
                    first = base_edge + edges[key] * m
                    for t in range(1, p):
                        tt = t if vA < vB else p - t
                        idx = [0, 0, 0]
                        idx[o1], idx[o2], idx[d] = s1 * p, s2 * p, t
                        out[e, idx[2], idx[1], idx[0]] = first + tt - 1
    base_face = base_edge + len(edges) * m
    sq = [(0, 0), (1, 0), (1, 1), (0, 1)]           # cyclic corners of a face in its (u, v) frame
    for e in range(NE):
        for d in range(3):
            u_ax, v_ax = [k for k in range(3) if k != d]
            for s in range(2):
                g = []
                for (cu, cv) in sq:
                    idx = [0, 0, 0]
                    idx[d], idx[u_ax], idx[v_ax] = s, cu, cv
                    g.append(corner(e, *idx))
                key = tuple(sorted(g))
                if key not in faces:
                    faces[key] = len(faces)
                first = base_face + faces[key] * m * m
                i0 = int(np.argmin(g))                # canonical origin: the smallest vertex id
                nxt, prv = (i0 + 1) % 4, (i0 + 3) % 4
                i1 = nxt if g[nxt] < g[prv] else prv  # first canonical axis toward the smaller neighbour
                o, a1 = np.array(sq[i0]), np.array(sq[i1])
                du = a1 - o                            # local direction of canonical u
                i2 = prv if i1 == nxt else nxt
                dv = np.array(sq[i2]) - o              # local direction of canonical v
                for vv in range(1, p):
                    for uu in range(1, p):
                        # local (u, v) of the node with canonical (uu, vv)
                        lu = o[0] * p + du[0] * uu + dv[0] * vv
                        lv = o[1] * p + du[1] * uu + dv[1] * vv
                        idx = [0, 0, 0]
                        idx[d], idx[u_ax], idx[v_ax] = s * p, lu, lv
                        out[e, idx[2], idx[1], idx[0]] = first + (uu - 1) + m * (vv - 1)
    base_cell = base_face + len(faces) * m * m
    cells = base_cell + np.arange(NE)[:, None, None, None] * m ** 3
    iz, iy, ix = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    out[:, 1:p, 1:p, 1:p] = cells + (ix + m * (iy + m * iz))[None]
    return out.reshape(NE, -1).astype(np.int32), int(base_cell + NE * m ** 3)


@dataclasses.dataclass
class HexMesh:
    """An unstructured hexahedral mesh of order p (see the conventions above)."""
    vertices: np.ndarray        # [NV, 3]
    elem_vertices: np.ndarray   # [NE, 8] int32
    p: int
    elem_nodes: np.ndarray      # [NE, (p+1)^3] int32
    num_nodes: int
    clamped: np.ndarray         # [num_nodes] bool

    @property
    def num_elements(self) -> int:
        return self.elem_vertices.shape[0]

    @property
    def num_dofs(self) -> int:
        return 3 * self.num_nodes


def box_as_unstructured(mesh: BoxMesh, verts: np.ndarray, p: int, seed: int = 3, permute: bool = True,
                        reorient: bool = True, renumber: bool = True, shuffle_nodes: bool = False):
    """The box mesh with vertex positions verts ([(n0+1)(n1+1)(n2+1), 3], see
    perturbed_vertices) written as an unstructured mesh: elements in a random order
    (permute), each in a random one of the 24 orientations of the cube (reorient), nodes
    numbered by hex_high_order_nodes (renumber; small meshes) or kept in box order,
    optionally relabelled by a random permutation (shuffle_nodes).  Returns (HexMesh,
    node_map, elem_order): node_map[u] = box node (gx + Nx (gy + Ny gz)) of node u and
    elem_order[i] = box element of element i; clamped nodes follow the box's faces."""
    rng = np.random.default_rng(seed)
    n0, n1, n2 = mesh.n
    D = p + 1
    NE = n0 * n1 * n2
    Nx, Ny, Nz = n0 * p + 1, n1 * p + 1, n2 * p + 1
    ez, ey, ex = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    # box numbering of every element's local nodes and vertices
    kz, ky, kx = np.meshgrid(np.arange(D), np.arange(D), np.arange(D), indexing="ij")
    loc = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    cz, cy, cx = np.meshgrid(np.arange(2), np.arange(2), np.arange(2), indexing="ij")
    cor = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    # per rotation: the old local node / corner seen at each new local node / corner
    rots = _cube_rotations()
    PI = np.empty((len(rots), D ** 3), dtype=np.int64)
    PV = np.empty((len(rots), 8), dtype=np.int64)
    for r, (perm, flip) in enumerate(rots):
        old = np.empty_like(loc)
        oc = np.empty_like(cor)
        for k in range(3):
            old[:, perm[k]] = np.where(flip[k], p - loc[:, k], loc[:, k])
            oc[:, perm[k]] = np.where(flip[k], 1 - cor[:, k], cor[:, k])
        PI[r] = old[:, 0] + D * (old[:, 1] + D * old[:, 2])
        PV[r] = oc[:, 0] + 2 * (oc[:, 1] + 2 * oc[:, 2])
    ident = rots.index(((0, 1, 2), (0, 0, 0)))
    order = rng.permutation(NE) if permute else np.arange(NE)
    r_e = rng.integers(len(rots), size=NE) if reorient else np.full(NE, ident)
    gx = (ex[order] * p)[:, None] + loc[None, :, 0]
    gy = (ey[order] * p)[:, None] + loc[None, :, 1]
    gz = (ez[order] * p)[:, None] + loc[None, :, 2]
    box_nodes = gx + Nx * (gy + Ny * gz)                                   # [NE, D^3] in old local order
    box_nodes = np.take_along_axis(box_nodes, PI[r_e], axis=1)
    vx = ex[order][:, None] + cor[None, :, 0]
    vy = ey[order][:, None] + cor[None, :, 1]
    vz = ez[order][:, None] + cor[None, :, 2]
    ev = vx + (n0 + 1) * (vy + (n1 + 1) * vz)
    ev = np.take_along_axis(ev, PV[r_e], axis=1)
    if renumber:
        en, nn = hex_high_order_nodes(ev, p, num_vertices=(n0 + 1) * (n1 + 1) * (n2 + 1))
        node_map = np.full(nn, -1, dtype=np.int64)
        node_map[en.ravel()] = box_nodes.ravel()
    else:
        nn = Nx * Ny * Nz
        if shuffle_nodes:
            new_id = rng.permutation(nn)
            en = new_id[box_nodes].astype(np.int32)
            node_map = np.argsort(new_id)
        else:
            en = box_nodes.astype(np.int32)
            node_map = np.arange(nn)
    g = np.arange(Nx * Ny * Nz)
    gx, gy, gz = g % Nx, (g // Nx) % Ny, g // (Nx * Ny)
    f = mesh.clamped_faces
    cl = (((f & 1) > 0) & (gx == 0)) | (((f & 2) > 0) & (gx == Nx - 1)) | (((f & 4) > 0) & (gy == 0)) | \
         (((f & 8) > 0) & (gy == Ny - 1)) | (((f & 16) > 0) & (gz == 0)) | (((f & 32) > 0) & (gz == Nz - 1))
    hm = HexMesh(vertices=np.asarray(verts, dtype=np.float64), elem_vertices=ev.astype(np.int32), p=p,
                 elem_nodes=en, num_nodes=nn, clamped=cl[node_map])
    return hm, node_map, order


def ogrid_cylinder(p: int, n: int = 4, m: int = 3, nz: int = 4, R: float = 1.0, a: float = 0.4,
                   H: float = 2.0, seed: Optional[int] = None) -> HexMesh:
    """A 5-block O-grid ("butterfly") mesh of a polygonal cylinder: a central n x n block
    of [-a,a]^2 and four n x m blocks out to a regular 4n-gon of radius R, extruded in
    nz layers over [0, H], clamped at z = 0.  Block corners are vertices shared by three
    quadrilaterals of the cross-section (an unstructured topology).  Elements are listed
    in a random order when seed is given."""
    pts, key = [], {}

    def vid(x, y):
        k = (round(x, 12), round(y, 12))
        if k not in key:
            key[k] = len(pts)
            pts.append((x, y))
        return key[k]

    quads = []
    s = np.linspace(-a, a, n + 1)
    for j in range(n):
        for i in range(n):
            quads.append((vid(s[i], s[j]), vid(s[i + 1], s[j]), vid(s[i + 1], s[j + 1]), vid(s[i], s[j + 1])))
    # side blocks: inner edge on the square, outer edge on the polygon, counter-clockwise
    side_in = [((a, -a), (a, a)), ((a, a), (-a, a)), ((-a, a), (-a, -a)), ((-a, -a), (a, -a))]
    for k, (p0, p1) in enumerate(side_in):
        th0 = -np.pi / 4 + k * np.pi / 2
        for i in range(n):
            for r in range(m):
                def point(ii, rr):
                    t = ii / n
                    xi = (1 - t) * np.array(p0) + t * np.array(p1)
                    th = th0 + t * np.pi / 2
                    # polygon vertex angles are multiples of the 4n-gon's step
                    xo = R * np.array([np.cos(th), np.sin(th)])
                    w = rr / m
                    q = (1 - w) * xi + w * xo
                    return vid(q[0], q[1])
                quads.append((point(i, r), point(i, r + 1), point(i + 1, r + 1), point(i + 1, r)))
    P2 = np.array(pts)
    NV2 = len(P2)
    # orient every quadrilateral counter-clockwise
    fixed = []
    for qd in quads:
        x, y = P2[list(qd), 0], P2[list(qd), 1]
        area = 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)
        fixed.append(qd if area > 0 else qd[::-1])
    z = np.linspace(0.0, H, nz + 1)
    V = np.concatenate([np.column_stack([P2, np.full(NV2, zz)]) for zz in z])
    ev = []
    for L in range(nz):
        for (q0, q1, q2, q3) in fixed:
            lo, hi = L * NV2, (L + 1) * NV2
            # local vertices a + 2(b + 2c): (0,0),(1,0),(0,1),(1,1) of the quad's frame
            ev.append((q0 + lo, q1 + lo, q3 + lo, q2 + lo, q0 + hi, q1 + hi, q3 + hi, q2 + hi))
    ev = np.array(ev, dtype=np.int64)
    if seed is not None:
        ev = ev[np.random.default_rng(seed).permutation(len(ev))]
    en, nn = hex_high_order_nodes(ev, p, num_vertices=len(V))
    D = p + 1
    # clamped: every node on a z = 0 face (layer-0 elements whose local iz = 0 face is the bottom)
    cl = np.zeros(nn, dtype=bool)
    enr = en.reshape(-1, D, D, D)
    bottom = np.all(V[ev[:, :4], 2] == 0.0, axis=1)
    cl[enr[bottom, 0].ravel()] = True
    return HexMesh(vertices=V, elem_vertices=ev.astype(np.int32), p=p, elem_nodes=en, num_nodes=nn, clamped=cl)


def random_rotation(seed: int) -> np.ndarray:
    """A random proper rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((3, 3))
    Qm, R = np.linalg.qr(M)
    Qm = Qm @ np.diag(np.sign(np.diag(R)))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] = -Qm[:, 0]
    return Qm


@dataclasses.dataclass
class ServeRequest:
    rid: int
    arrival: float
    n: tuple
    p: int
    E: float
    nu: float
    f: tuple


def serving_stream(num: int = 512, rate: float = 1.0, seed: int = 5, n_lo: int = 4, n_hi: int = 32,
                   ps=(2, 4, 6, 8)):
    """Poisson arrivals of box solves with random sizes, orders and materials."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(num):
        t += rng.exponential(1.0 / rate)
        n = tuple(int(v) for v in rng.integers(n_lo, n_hi + 1, 3))
        p = int(rng.choice(ps))
        E = float(10.0 ** rng.uniform(0.0, 2.0))
        nu = float(rng.uniform(0.2, 0.4))
        f = tuple(float(v) for v in rng.uniform(-1.0, 1.0, 3))
        out.append(ServeRequest(i, t, n, p, E, nu, f))
    return out
