// Apply for linear elements (p = 1): register-resident, one lane per element.
//
// The operator is that of the fused kernel (paper Sec. 4.2, 4.4, 4.5): reference
// gradient, pointwise Voigt stress with w*detJ*lambda, w*detJ*mu and Q = sigma J^{-T}
// (eq. 7), tested against the basis gradients.  With two nodes per axis the whole
// element state fits in registers, so each lane runs an element by itself: no LDS
// (except for the nodal values of the double-precision per-point kernel), no barriers.
// With per-element Lame data every factor of the quadrature sum is a polynomial of
// degree at most one per axis, and the sum collapses to one term per monomial
// (lin_element_closed); per-point Lame data keeps the point loops (lin_element).
//
// A wavefront is a tile of kLinTX x kLinTY element columns (lane = column);
// each lane walks a chunk of lin_chunk() elements up its column, carrying the upper face of
// one element (x values and partial results) in registers into the next (the per-point
// kernels also prefetch the next element's x face and data while they compute).  After
// each element the finished node layer is summed across lanes with shuffles
// (x neighbour, then y neighbour); every node of the layer has one owning
// lane, which writes y itself when all elements touching the node lie in the
// tile, and otherwise stores its partial sum in the tile's slot of the
// skeleton buffer.  pa_lin_skeleton_kernel then adds the (up to 8) tile
// partial sums of every tile-boundary node in a fixed order: no atomics,
// bitwise-reproducible results.
#include "apply_kernel.h"

namespace pa {

template <typename T, int Q>
struct LinTabs {
    T B0[Q], B1[Q];   // linear Lagrange basis at the Gauss-Legendre points: 1 - xi_k, xi_k
    T w[Q];           // Gauss-Legendre weights on [0,1]
    T wzy[Q * Q];     // w[qz] * w[qy]
    T cb[3];          // lin_element_closed: beta_n = 4^(n-2) W0^(3-n) W2^n, W_m = sum_k w[k] (xi_k - 1/2)^m
};

// 12 words of per-element data with 16-byte loads (the rows are 48 or 96 bytes).
__device__ __forceinline__ void load_ed12(const double* p, double (&d)[12]) {
    const double2* v = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const double2 t = v[i];
        d[2 * i] = t.x;
        d[2 * i + 1] = t.y;
    }
}
__device__ __forceinline__ void load_ed12(const float* p, float (&d)[12]) {
    const float4* v = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float4 t = v[i];
        d[4 * i] = t.x;
        d[4 * i + 1] = t.y;
        d[4 * i + 2] = t.z;
        d[4 * i + 3] = t.w;
    }
}

// Slot of boundary node (lx, ly, lz) of tile t (local node coordinates in the tile's node
// box; tz = elements per tile along z) in the tile's face arrays of component c: nodes on an
// x face (lx = 0 or kLinTX) in the x-face array [side][lz][ly], other nodes on a y face in the
// y-face array [side][lz][lx], the remaining ones (lz = 0 or tz) in the z-face array
// [side][ly][lx].  Lanes that handle consecutive nodes along a face then touch consecutive
// words, in the fused kernel and in the skeleton gather.
__device__ __forceinline__ unsigned lin_face_slot(int lz, int ly, int lx, int tz) {
    if (lx == 0 || lx == kLinTX) return ((unsigned)(lx == kLinTX) * (tz + 1) + lz) * (kLinTY + 1) + ly;
    const unsigned ofs_y = 2 * (unsigned)(tz + 1) * (kLinTY + 1);
    if (ly == 0 || ly == kLinTY) return ofs_y + ((unsigned)(ly == kLinTY) * (tz + 1) + lz) * (kLinTX + 1) + lx;
    const unsigned ofs_z = ofs_y + 2 * (unsigned)(tz + 1) * (kLinTX + 1);
    return ofs_z + ((unsigned)(lz != 0) * (kLinTY + 1) + ly) * (kLinTX + 1) + lx;
}
__device__ __forceinline__ size_t lin_slot(int t, int c, int lz, int ly, int lx, int tz) {
    return ((size_t)t * 3 + c) * lin_face_words(tz) + lin_face_slot(lz, ly, lx, tz);
}

// One (qy, qz) column of quadrature points with per-point Lame parameters lq[qx], mq[qx]:
// forward X to the reference gradient, pointwise stress (weights w[qx] * lzy * lq[qx],
// w[qx] * mzy * mq[qx]; lzy, mzy carry w[qz] w[qy] det J) and its two Voigt moments along the
// column, M0 = sum w sigma and M1 = sum w xi sigma, from which lin_project forms the
// backward X channels of Q = sigma J^{-T}.
// Inputs per component c and x-column ix: a = B_y B_z x, b = G_y B_z x, e = B_y G_z x.
//
// With the linear basis in x, B_x(xi) = (1 - xi, xi) and G_x = (-1, 1), so along the
// column the reference gradient is linear in xi: g = (a1 - a0, b0 + xi (b1 - b0),
// e0 + xi (e1 - e0)), and so is the physical gradient, du = D0 + xi D1 (both J^{-T}
// products formed once per column).  On the way back, J^{-1} is constant over the element,
// so the x sums of Q = sigma J^{-T} are J^{-1} applied to the x sums of sigma:
// S0 = sum Q_0 = M0 J^{-1}_0, r_m = (sum (1 - xi) Q_m, sum xi Q_m) = ((M0 - M1) J^{-1}_m, M1 J^{-1}_m).
template <int Q, typename T>
__device__ __forceinline__ void lin_moments(const T (&a)[3][2], const T (&b)[3][2], const T (&e)[3][2],
                                            const T (&Ji)[9], const T lzy, const T mzy, const LinTabs<T, Q>& tb,
                                            T (&M0)[6], T (&M1)[6], const T (&lq)[Q], const T (&mq)[Q]) {
    T D0[3][3], D1[3][3];   // du[c][i] = d u_c / d x_i = D0[c][i] + xi D1[c][i]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T ga = a[c][1] - a[c][0], db = b[c][1] - b[c][0], de = e[c][1] - e[c][0];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            D0[c][i] = Ji[0 * 3 + i] * ga + Ji[1 * 3 + i] * b[c][0] + Ji[2 * 3 + i] * e[c][0];
            D1[c][i] = Ji[1 * 3 + i] * db + Ji[2 * 3 + i] * de;
        }
    }
    // Voigt moments: entries (xx, yy, zz, yz, xz, xy)
#pragma unroll
    for (int v = 0; v < 6; ++v) M0[v] = M1[v] = T(0);
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
        const T xi = tb.B1[qx];
        const T lam = lzy * tb.w[qx] * lq[qx], mu = mzy * tb.w[qx] * mq[qx];
        T du[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < 3; ++i) du[c][i] = fma(xi, D1[c][i], D0[c][i]);
        const T div = du[0][0] + du[1][1] + du[2][2];
        const T ld = lam * div, m2 = mu + mu;
        T sv[6];
        sv[0] = ld + m2 * du[0][0];
        sv[1] = ld + m2 * du[1][1];
        sv[2] = ld + m2 * du[2][2];
        sv[3] = mu * (du[1][2] + du[2][1]);
        sv[4] = mu * (du[0][2] + du[2][0]);
        sv[5] = mu * (du[0][1] + du[1][0]);
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            M0[v] += sv[v];
            M1[v] = fma(xi, sv[v], M1[v]);
        }
    }
}

// The backward X channels from the two Voigt moments: S0 = M0 J^{-1}_0,
// r_m = ((M0 - M1) J^{-1}_m, M1 J^{-1}_m) for m = 1, 2 (linear in the moments).
template <typename T>
__device__ __forceinline__ void lin_project(const T (&M0)[6], const T (&M1)[6], const T (&Ji)[9], T (&S0)[3],
                                            T (&r1)[3][2], T (&r2)[3][2]) {
    // sigma[c][i] as a Voigt index
    constexpr int kV[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T s0 = T(0), R1 = T(0), X1 = T(0), R2 = T(0), X2 = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T m0 = M0[kV[c][i]], m1 = M1[kV[c][i]];
            s0 = fma(m0, Ji[0 * 3 + i], s0);
            R1 = fma(m0, Ji[1 * 3 + i], R1);
            X1 = fma(m1, Ji[1 * 3 + i], X1);
            R2 = fma(m0, Ji[2 * 3 + i], R2);
            X2 = fma(m1, Ji[2 * 3 + i], X2);
        }
        S0[c] = s0;
        r1[c][0] = R1 - X1;
        r1[c][1] = X1;
        r2[c][0] = R2 - X2;
        r2[c][1] = X2;
    }
}

// Per-point material (QPM): mdp points at the element's (lambda, mu) of point 0; point
// alpha, word k is mdp[(2 alpha + k) * ns] (point-major layout, elements contiguous).
template <int Q, typename T>
__device__ __forceinline__ void lin_point_lame(const T* mdp, size_t ns, int qz, int qy, T (&lq)[Q], T (&mq)[Q]) {
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
        const size_t al = qx + Q * (qy + Q * qz);
        lq[qx] = mdp[(2 * al) * ns];
        mq[qx] = mdp[(2 * al + 1) * ns];
    }
}

constexpr int kLinLds = 256;   // lanes per workgroup = LDS column stride

// Compiler barrier: values staged in LDS are re-read after it instead of being
// kept live in registers.
__device__ __forceinline__ void lds_reload_point() { __asm__ volatile("" ::: "memory"); }

// Nodal values of component c, x-column ix of an element in difference form: with a0, a1
// the nodes (iy = 0, 1) of the lower face and b0, b1 those of the upper face, the words
// (a0, a1 - a0, b0 - a0, (b1 - a1) - (b0 - a0)).  Interpolated to (eta, zeta) the node
// values are then bilinear in these four with unit coefficients: B_z x at iy is
// a_iy + zeta (b_iy - a_iy), B_y of it is z0 + eta (z1 - z0), and
// z1 - z0 = (a1 - a0) + zeta ((b1 - a1) - (b0 - a0)).
constexpr int kLinNodeWords = 24;
__device__ __forceinline__ int lin_node_word(int c, int ix, int w) { return (c * 2 + ix) * 4 + w; }

// the difference form of the element with lower x face fa and upper x face fb (word k of a
// face is (c, iy, ix) = (k >> 2, (k >> 1) & 1, k & 1)), handed to put(word, value)
template <typename T, typename F>
__device__ __forceinline__ void lin_node_form(const T (&fa)[12], const T (&fb)[12], F&& put) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int ix = 0; ix < 2; ++ix) {
            const T a0 = fa[c * 4 + ix], a1 = fa[c * 4 + 2 + ix];
            const T dz = fb[c * 4 + ix] - a0;
            put(lin_node_word(c, ix, 0), a0);
            put(lin_node_word(c, ix, 1), a1 - a0);
            put(lin_node_word(c, ix, 2), dz);
            put(lin_node_word(c, ix, 3), (fb[c * 4 + 2 + ix] - a1) - dz);
        }
}

// where an element's difference form is read from: the lane's LDS column (double
// precision, re-read in every column so that it does not hold registers) or registers
struct LinNodesLds {
    static constexpr bool kLds = true;
    static constexpr int kStride = kLinLds;
};
struct LinNodesReg {
    static constexpr bool kLds = false;
    static constexpr int kStride = 1;
};

// Element contribution y_e = K_e x_e of one element with per-point Lame data, added to ya
// (lower face iz = 0) and yb (upper face iz = 1); word k of a face is (c, iy, ix) =
// (k >> 2, (k >> 1) & 1, k & 1).  nd holds the element's nodal values in difference form
// (word w at nd[w * Src::kStride]).  Per (qz, qy) column: the forward Y/Z interpolation
// (four FMAs per x-column), the column's Voigt moments (lin_moments), their projection
// (lin_project), the backward Y sweep (B_y = (1 - eta, eta), G_y = (-1, 1)) and the
// backward Z sweep into the faces.
template <int Q, typename T, typename Src>
__device__ __forceinline__ void lin_element(const T* nd, const T (&d)[12], const LinTabs<T, Q>& tb,
                                            T (&ya)[12], T (&yb)[12], const T* mdp, size_t ns) {
    constexpr int stride = Src::kStride;
    T Ji[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Ji[k] = d[k];
    const T lw = d[9], mw = d[10];
#pragma unroll 1
    for (int qz = 0; qz < Q; ++qz) {
        const T bz0 = tb.B0[qz], bz1 = tb.B1[qz];
#pragma unroll 1
        for (int qy = 0; qy < Q; ++qy) {
            if constexpr (Src::kLds) lds_reload_point();
            const T by0 = tb.B0[qy], by1 = tb.B1[qy];
            const T wzy = tb.wzy[qz * Q + qy];
            // a = B_y B_z x, b = G_y B_z x, e = B_y G_z x at (eta, zeta) = (by1, bz1)
            T a[3][2], b[3][2], e[3][2];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int ix = 0; ix < 2; ++ix) {
                    const T n0 = nd[lin_node_word(c, ix, 0) * stride], ny = nd[lin_node_word(c, ix, 1) * stride];
                    const T nz = nd[lin_node_word(c, ix, 2) * stride], nyz = nd[lin_node_word(c, ix, 3) * stride];
                    const T z0 = fma(bz1, nz, n0);
                    b[c][ix] = fma(bz1, nyz, ny);
                    a[c][ix] = fma(by1, b[c][ix], z0);
                    e[c][ix] = fma(by1, nyz, nz);
                }
            T M0[6], M1[6], lq[Q], mq[Q];
            lin_point_lame<Q, T>(mdp, ns, qz, qy, lq, mq);
            lin_moments<Q, T>(a, b, e, Ji, lw * wzy, mw * wzy, tb, M0, M1, lq, mq);
            // t0 = B_y S0 (sign of G_x by ix) + G_y r1 takes B_z, t2 = B_y r2 takes G_z = (-1, +1)
            T S0[3], r1[3][2], r2[3][2];
            lin_project(M0, M1, Ji, S0, r1, r2);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int iy = 0; iy < 2; ++iy) {
                    const T by = iy ? by1 : by0;
#pragma unroll
                    for (int ix = 0; ix < 2; ++ix) {
                        const int k = c * 4 + iy * 2 + ix;
                        const T t0 = (ix ? by : -by) * S0[c] + (iy ? r1[c][ix] : -r1[c][ix]);
                        const T t2 = by * r2[c][ix];
                        ya[k] += bz0 * t0 - t2;
                        yb[k] += bz1 * t0 + t2;
                    }
                }
        }
    }
}

// One monomial t (bit k = power of s_k, t != 7) of lin_element_closed: the physical gradient
// coefficient Dt = sum_{k: t_k = 0} H_{t + e_k} (x) J^{-1}_k (row k of J^{-1}), its stress with
// the weights lt, mt, and P[k][c] = (sigma J^{-T})[c][k] for the k with t_k = 0.
template <int t, typename T>
__device__ __forceinline__ void lin_monomial(const T (&h)[8][3], const T (&Ji)[9], const T lt, const T mt,
                                             T (&P)[3][3]) {
    T D[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T acc = T(0);
            bool first = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if ((t >> k) & 1) continue;
                const T hv = h[t | (1 << k)][c];
                acc = first ? hv * Ji[k * 3 + j] : fma(hv, Ji[k * 3 + j], acc);
                first = false;
            }
            D[c][j] = acc;
        }
    const T ld = lt * (D[0][0] + D[1][1] + D[2][2]), m2 = mt + mt;
    T S[3][3];
    S[0][0] = fma(m2, D[0][0], ld);
    S[1][1] = fma(m2, D[1][1], ld);
    S[2][2] = fma(m2, D[2][2], ld);
    S[1][2] = S[2][1] = mt * (D[1][2] + D[2][1]);
    S[0][2] = S[2][0] = mt * (D[0][2] + D[2][0]);
    S[0][1] = S[1][0] = mt * (D[0][1] + D[1][0]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if ((t >> k) & 1) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) P[k][c] = fma(S[c][2], Ji[k * 3 + 2], fma(S[c][1], Ji[k * 3 + 1], S[c][0] * Ji[k * 3]));
    }
}

// Element contribution of one element with per-element Lame weights (d[9] = det J lambda,
// d[10] = det J mu), added to ya (lower face) and stored to yb (upper face); fa, fb are the element's
// lower and upper x faces (word k = (c, iy, ix) as above).
//
// In centred coordinates s = xi - 1/2 the basis is prod_k (1/2 + sgn(i_k) s_k), sgn(0) = -1,
// sgn(1) = +1, so the nodal interpolant is u = sum_a 2^(|a|-3) H_a s^a over a in {0,1}^3,
// where H_a = sum_i x_i prod_k sgn(i_k)^(a_k) is the 8-point Walsh-Hadamard transform of the
// nodal values.  J^{-1} and the Lame weights are constant over the element, so the physical
// gradient, the stress and Q = sigma J^{-T} are sums over the monomials t != (1,1,1), and
// the test gradients d phi_i / d xi_k are sums over the monomials with t_k = 0.  The
// quadrature sum of a product of two monomials is a product of the rule's centred 1D
// moments W_m = sum w s^m; the Gauss rule is symmetric, so its odd moments vanish and only
// equal monomials pair up, with weight W0^(3-|t|) W2^|t|.  With the powers of 2 folded in
// (beta_n = 4^(n-2) W0^(3-n) W2^n, LinTabs::cb), the element vector is
//   y_i = sum_a prod_k sgn(i_k)^(a_k) Y_a,   Y_a = sum_{k: a_k = 1} P_{a - e_k}[k],
//   P_t = beta_|t| sigma(Dt) J^{-T},          Dt = sum_{k: t_k = 0} H_{t + e_k} (x) J^{-1}_k:
// the same quadrature sums as the point loops, regrouped, in about a quarter of their
// operations.
template <typename T>
__device__ __forceinline__ void lin_element_closed(const T (&fa)[12], const T (&fb)[12], const T (&d)[12],
                                                   const T (&cb)[3], T (&ya)[12], T (&yb)[12]) {
    // h[a][c], a = ax + 2 ay + 4 az; node i = ix + 2 iy + 4 iz
    T h[8][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (i & 4) ? fb[c * 4 + (i & 3)] : fa[c * 4 + (i & 3)];
#pragma unroll
        for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (!(j & bit)) {
                    const T lo = v[j], hi = v[j | bit];
                    v[j] = hi + lo;
                    v[j | bit] = hi - lo;
                }
#pragma unroll
        for (int a = 0; a < 8; ++a) h[a][c] = v[a];
    }
    T Ji[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Ji[k] = d[k];
    const T l0 = cb[0] * d[9], m0 = cb[0] * d[10];
    const T l1 = cb[1] * d[9], m1 = cb[1] * d[10];
    const T l2 = cb[2] * d[9], m2 = cb[2] * d[10];
    // Y[a][c]; the monomials in an order that lets each H_a die early
    T Y[8][3], P[3][3];
    lin_monomial<0>(h, Ji, l0, m0, P);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Y[1][c] = P[0][c];
        Y[2][c] = P[1][c];
        Y[4][c] = P[2][c];
    }
    lin_monomial<1>(h, Ji, l1, m1, P);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Y[3][c] = P[1][c];
        Y[5][c] = P[2][c];
    }
    lin_monomial<2>(h, Ji, l1, m1, P);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Y[3][c] += P[0][c];
        Y[6][c] = P[2][c];
    }
    lin_monomial<4>(h, Ji, l1, m1, P);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Y[5][c] += P[0][c];
        Y[6][c] += P[1][c];
    }
    lin_monomial<3>(h, Ji, l2, m2, P);
#pragma unroll
    for (int c = 0; c < 3; ++c) Y[7][c] = P[2][c];
    lin_monomial<5>(h, Ji, l2, m2, P);
#pragma unroll
    for (int c = 0; c < 3; ++c) Y[7][c] += P[1][c];
    lin_monomial<6>(h, Ji, l2, m2, P);
#pragma unroll
    for (int c = 0; c < 3; ++c) Y[7][c] += P[0][c];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T v[8];
        v[0] = T(0);
#pragma unroll
        for (int a = 1; a < 8; ++a) v[a] = Y[a][c];
        // y_i = sum_a prod_k sgn(i_k)^(a_k) v_a, one axis at a time
#pragma unroll
        for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (!(j & bit)) {
                    const T lo = v[j], hi = v[j | bit];
                    v[j] = lo - hi;
                    v[j | bit] = lo + hi;
                }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i & 4) yb[c * 4 + (i & 3)] = v[i];
            else ya[c * 4 + (i & 3)] += v[i];
        }
    }
}

// the double-precision per-point kernel keeps the element's nodal values in LDS (its point
// loops need more than 256 VGPRs with them in registers)
template <typename T, bool QPM>
constexpr bool kLinXInLds = QPM && sizeof(T) == 8;

template <int Q, typename T, bool QPM = false>
__global__ void __launch_bounds__(256)
pa_apply_lin_kernel(const T* __restrict__ x, T* __restrict__ y, T* __restrict__ sk, const T* __restrict__ ed,
                    const LinTabs<T, Q> tb, const Geom g, const int TZ, const int add, const T* __restrict__ md) {
    constexpr int TX = kLinTX, TY = kLinTY;
    static_assert(TX * TY == 64 && kLinLds == 256, "one tile per wavefront, four per workgroup");
    const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
    // one tile per wavefront: the tile and everything derived from it are wave-uniform
    const int tile = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (tile >= ntx * nty * ntz) return;   // the whole wavefront leaves together
    const int lane = threadIdx.x & 63;
    const int lx = lane % TX, ly = lane / TX;
    const int tx = tile % ntx, tr = tile / ntx;
    const int ty = tr % nty, tz = tr / nty;
    const int tx0 = tx * TX, ty0 = ty * TY, ez0 = tz * TZ;
    const int tx1 = min(tx0 + TX, g.nx), ty1 = min(ty0 + TY, g.ny), ez1 = min(ez0 + TZ, g.nz);
    const int ex = tx0 + lx, ey = ty0 + ly;
    const bool valid = ex < g.nx && ey < g.ny;
    const bool lastx = ex == tx1 - 1, lasty = ey == ty1 - 1;
    const size_t NN = (size_t)g.Nn;
    // per-component vectors (wave-uniform bases) indexed by 32-bit node numbers (3 Nn < 2^31),
    // and the tile's face arrays: the lanes' addresses are formed where they are used
    const T* const xc[3] = {x, x + NN, x + 2 * NN};
    T* const yc[3] = {y, y + NN, y + 2 * NN};
    const size_t fw = (size_t)lin_face_words(TZ);
    T* const skc[3] = {sk + (size_t)tile * 3 * fw, sk + ((size_t)tile * 3 + 1) * fw, sk + ((size_t)tile * 3 + 2) * fw};
    const unsigned lane_node = (unsigned)ex + (unsigned)g.Nx * (unsigned)ey;   // node (ex, ey, 0)
    const unsigned layer = (unsigned)g.Nx * (unsigned)g.Ny;

    // clamped corner nodes of the column's faces are read as 0 (constrained operator)
    auto load_face = [&](int gz, T (&f)[12]) {
#pragma unroll
        for (int iy = 0; iy < 2; ++iy)
#pragma unroll
            for (int ix = 0; ix < 2; ++ix) {
                const unsigned node = lane_node + layer * (unsigned)gz + (unsigned)ix + (unsigned)g.Nx * (unsigned)iy;
                const bool use = valid && !(g.clamp && clamped_node(g.clamp, ex + ix, ey + iy, gz, g));
#pragma unroll
                for (int c = 0; c < 3; ++c) f[c * 4 + iy * 2 + ix] = use ? xc[c][node] : T(0);
            }
    };
    auto load_data = [&](int ez, T (&d)[12]) {
        if (valid) {
            const unsigned e = (unsigned)ex + (unsigned)g.nx * ((unsigned)ey + (unsigned)g.ny * (unsigned)ez);
            load_ed12(ed + (size_t)e * kEdStride, d);
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) d[k] = T(0);
        }
    };
    // sum node layer gz across lanes and write it: y for nodes whose elements all lie
    // in the tile, the tile's skeleton slot for the others
    auto emit_layer = [&](T (&v)[3][2][2], int gz) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int iy = 0; iy < 2; ++iy) {
                const T t = __shfl_up(v[c][iy][1], 1, TX);
                if (lx > 0) v[c][iy][0] += t;
            }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int ix = 0; ix < 2; ++ix) {
                const T t = __shfl_up(v[c][1][ix], TX, 64);
                if (ly > 0) v[c][0][ix] += t;
            }
        if (!valid) return;
        const bool cz = (gz > ez0 || gz == 0) && (gz < ez1 || gz == g.nz);
#pragma unroll
        for (int iy = 0; iy < 2; ++iy)
#pragma unroll
            for (int ix = 0; ix < 2; ++ix) {
                if ((ix && !lastx) || (iy && !lasty)) continue;   // node owned by another lane
                const int gx = ex + ix, gy = ey + iy;
                const bool cx = (gx > tx0 || gx == 0) && (gx < tx1 || gx == g.nx);
                const bool cy = (gy > ty0 || gy == 0) && (gy < ty1 || gy == g.ny);
                if (cx && cy && cz) {
                    const unsigned node = lane_node + layer * (unsigned)gz + (unsigned)ix + (unsigned)g.Nx * (unsigned)iy;
                    const bool cl = g.clamp && clamped_node(g.clamp, gx, gy, gz, g);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const T val = cl ? xc[c][node] : v[c][iy][ix];
                        T* yp = yc[c] + node;
                        *yp = add ? *yp + val : val;
                    }
                } else {
                    const unsigned slot = lin_face_slot(gz - ez0, gy - ty0, gx - tx0, TZ);
#pragma unroll
                    for (int c = 0; c < 3; ++c) skc[c][slot] = v[c][iy][ix];
                }
            }
    };

    // per-point material of element (ex, ey, ez); lanes past the mesh read element 0 (their
    // element data is zero)
    auto mat_ptr = [&](int ez) -> const T* {
        if constexpr (QPM) return md + (valid ? (size_t)(ex + g.nx * (ey + g.ny * ez)) : (size_t)0);
        else return nullptr;
    };
    T xn[12], dn[12], ya[12];
    auto to_face = [](const T (&f)[12], T (&v)[3][2][2]) {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k >> 2][(k >> 1) & 1][k & 1] = f[k];
    };
#pragma unroll
    for (int k = 0; k < 12; ++k) ya[k] = T(0);
    if constexpr (kLinXInLds<T, QPM>) {
        // the element's nodal values in difference form and the lower x face of the next
        // element in the lane's LDS column; the next element's data is loaded after the
        // current element (two waves per SIMD hide the latency)
        __shared__ T s_x[(kLinNodeWords + 12) * kLinLds];
        T* const col = s_x + threadIdx.x;
        T* const face = col + kLinNodeWords * kLinLds;
        auto store_face = [&](const T (&f)[12]) {
#pragma unroll
            for (int k = 0; k < 12; ++k) face[k * kLinLds] = f[k];
        };
        load_face(ez0, xn);
        store_face(xn);
        load_face(ez0 + 1, xn);
        load_data(ez0, dn);
#pragma unroll 1
        for (int ez = ez0; ez < ez1; ++ez) {
            T d[12], yb[12];
            // lower face from LDS, upper face (xn) from registers
            T fl[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) fl[k] = face[k * kLinLds];
            lin_node_form(fl, xn, [&](int w, T v) { col[w * kLinLds] = v; });
            store_face(xn);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                d[k] = dn[k];
                yb[k] = T(0);
            }
            lin_element<Q, T, LinNodesLds>(col, d, tb, ya, yb, mat_ptr(ez), (size_t)g.NE);
            if (ez + 1 < ez1) {
                load_face(ez + 2, xn);
                load_data(ez + 1, dn);
            }
            T v[3][2][2];
            to_face(ya, v);
            emit_layer(v, ez);
#pragma unroll
            for (int k = 0; k < 12; ++k) ya[k] = yb[k];
        }
    } else if constexpr (QPM) {
        // everything in registers; the next element's data is prefetched
        T xa[12];
        load_face(ez0, xa);
        load_face(ez0 + 1, xn);
        load_data(ez0, dn);
#pragma unroll 1
        for (int ez = ez0; ez < ez1; ++ez) {
            T xb[12], d[12], yb[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                xb[k] = xn[k];
                d[k] = dn[k];
                yb[k] = T(0);
            }
            if (ez + 1 < ez1) {
                load_face(ez + 2, xn);
                load_data(ez + 1, dn);
            }
            T nd[kLinNodeWords];
            lin_node_form(xa, xb, [&](int w, T v) { nd[w] = v; });
            lin_element<Q, T, LinNodesReg>(nd, d, tb, ya, yb, mat_ptr(ez), (size_t)g.NE);
            T v[3][2][2];
            to_face(ya, v);
            emit_layer(v, ez);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                xa[k] = xb[k];
                ya[k] = yb[k];
            }
        }
    } else {
        // per-element data, closed form: the element's upper face and data are loaded at the
        // top of each step (prefetching them one element ahead took more registers than
        // the two waves per SIMD this loop runs at, and measured slower)
        T xa[12];
        load_face(ez0, xa);
#pragma unroll 1
        for (int ez = ez0; ez < ez1; ++ez) {
            T xb[12], d[12], yb[12];
            load_face(ez + 1, xb);
            load_data(ez, d);
            lin_element_closed(xa, xb, d, tb.cb, ya, yb);
            T v[3][2][2];
            to_face(ya, v);
            emit_layer(v, ez);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                xa[k] = xb[k];
                ya[k] = yb[k];
            }
        }
    }
    T v[3][2][2];
    to_face(ya, v);
    emit_layer(v, ez1);
}

// The nodes that more than one tile holds (on an interior tile plane x = 8k, y = 8k or
// z = TZ k), as three sets: (a) every node of the interior x planes, (b) the nodes of the
// interior y planes off the x planes, (c) the nodes of the interior z planes off the x and
// y planes.  Each plane is cut into blocks of 8 x 8 nodes, one wavefront per block, so that
// the lanes of a wavefront read runs of 8 consecutive words in 8 consecutive rows of a
// tile's face array (lanes of a block past the mesh, or on a plane of an earlier set, idle).
struct LinSharedNodes {
    int nxp, nyp, nzp;    // interior tile planes along x, y, z
    int bx, by, bz;       // 8-node blocks along x, y, z
    int64_t la, lb, lc;   // lanes of each set (64 per block)
};

inline LinSharedNodes lin_shared_nodes(const Geom& g, int TZ) {
    LinSharedNodes s;
    s.nxp = (g.nx + kLinTX - 1) / kLinTX - 1;
    s.nyp = (g.ny + kLinTY - 1) / kLinTY - 1;
    s.nzp = (g.nz + TZ - 1) / TZ - 1;
    s.bx = (g.Nx + 7) / 8;
    s.by = (g.Ny + 7) / 8;
    s.bz = (g.Nz + 7) / 8;
    s.la = (int64_t)s.nxp * s.by * s.bz * 64;
    s.lb = (int64_t)s.nyp * s.bx * s.bz * 64;
    s.lc = (int64_t)s.nzp * s.bx * s.by * 64;
    return s;
}

// For every shared tile-boundary node: sum the partial sums of the tiles touching it
// in a fixed order (z, y, x candidates) and write y.
template <typename T>
__global__ void __launch_bounds__(256)
pa_lin_skeleton_kernel(const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ sk, const Geom g,
                       const int TZ, const LinSharedNodes sn, const int add) {
    static_assert(kLinTX == 8 && kLinTY == 8, "node blocks and tile planes share the 8-node spacing");
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // lane (i, j) of an 8 x 8 node block: i along the block's first axis, j along its second
    const int i = (int)(t & 7), j = (int)((t >> 3) & 7);
    int gx, gy, gz;
    if (t < sn.la) {
        // x plane: blocks over (y, z)
        const int b = (int)(t >> 6);
        const int r = b / sn.by;
        gy = 8 * (b % sn.by) + i;
        gz = 8 * (r % sn.bz) + j;
        gx = kLinTX * (r / sn.bz + 1);
        if (gy >= g.Ny || gz >= g.Nz) return;
    } else if (t < sn.la + sn.lb) {
        // y plane: blocks over (x, z), nodes on an x plane excluded
        const int b = (int)((t - sn.la) >> 6);
        const int r = b / sn.bx;
        const int bxi = b % sn.bx;
        gx = 8 * bxi + i;
        gz = 8 * (r % sn.bz) + j;
        gy = kLinTY * (r / sn.bz + 1);
        if (gx >= g.Nx || gz >= g.Nz || (i == 0 && bxi >= 1 && bxi <= sn.nxp)) return;
    } else if (t < sn.la + sn.lb + sn.lc) {
        // z plane: blocks over (x, y), nodes on an x or y plane excluded
        const int b = (int)((t - sn.la - sn.lb) >> 6);
        const int r = b / sn.bx;
        const int bxi = b % sn.bx, byi = r % sn.by;
        gx = 8 * bxi + i;
        gy = 8 * byi + j;
        gz = TZ * (r / sn.by + 1);
        if (gx >= g.Nx || gy >= g.Ny || (i == 0 && bxi >= 1 && bxi <= sn.nxp) ||
            (j == 0 && byi >= 1 && byi <= sn.nyp))
            return;
    } else {
        return;
    }
    const int node = gx + g.Nx * (gy + g.Ny * gz);
    const int gg[3] = {gx, gy, gz}, nn[3] = {g.nx, g.ny, g.nz}, TT[3] = {kLinTX, kLinTY, TZ};
    // per axis the tiles of the elements before (gg-1) and after (gg) the node
    int t_[3][2];
    bool v_[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool lo = gg[a] > 0, hi = gg[a] < nn[a];
        t_[a][0] = lo ? (gg[a] - 1) / TT[a] : 0;
        t_[a][1] = hi ? gg[a] / TT[a] : 0;
        v_[a][0] = lo;
        v_[a][1] = hi && !(lo && t_[a][1] == t_[a][0]);
    }
    const int ntx = (g.nx + kLinTX - 1) / kLinTX, nty = (g.ny + kLinTY - 1) / kLinTY;
    const size_t NN = (size_t)g.Nn;
    const bool cl = g.clamp && clamped_node(g.clamp, gx, gy, gz, g);
    T acc[3] = {T(0), T(0), T(0)};
    if (!cl) {
        // fixed order (z, y, x candidates); every existing tile's loads are issued before the
        // first sum, a tile that does not exist contributes zero
        T v[8][3];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
#pragma unroll
            for (int c = 0; c < 3; ++c) v[k][c] = T(0);
            if (v_[0][kx] && v_[1][ky] && v_[2][kz]) {
                const int tx = t_[0][kx], ty = t_[1][ky], tz = t_[2][kz];
                const int tl = tx + ntx * (ty + nty * tz);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    v[k][c] = sk[lin_slot(tl, c, gz - tz * TZ, gy - ty * kLinTY, gx - tx * kLinTX, TZ)];
            }
        }
        // (an empty asm per value keeps the sums out of the branches above)
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) asm volatile("" : "+v"(v[k][c]));
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += v[k][c];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = x[c * NN + node];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T* yp = y + c * NN + node;
        *yp = add ? *yp + acc[c] : acc[c];
    }
}

template <int Q, typename T, bool QPM = false>
int launch_lin(const ApplyLaunch& L) {
    const Geom& g = L.g;
    if (g.NE == 0) return PA_OK;
    if (L.tab->p != 1 || L.tab->q != Q) return fail(PA_EINVAL, "tables are for p=%d q=%d", L.tab->p, L.tab->q);
    LinTabs<T, Q> tb;
    for (int k = 0; k < Q; ++k) {
        tb.B0[k] = (T)L.tab->B[0 * Q + k];
        tb.B1[k] = (T)L.tab->B[1 * Q + k];
        tb.w[k] = (T)L.tab->w[k];
    }
    // centred moments of the rule (the odd ones vanish: the rule is symmetric about 1/2)
    double W0 = 0.0, W2 = 0.0;
    for (int k = 0; k < Q; ++k) {
        const double s = L.tab->B[Q + k] - 0.5;
        W0 += L.tab->w[k];
        W2 += L.tab->w[k] * s * s;
    }
    tb.cb[0] = (T)(W0 * W0 * W0 / 16.0);
    tb.cb[1] = (T)(W0 * W0 * W2 / 4.0);
    tb.cb[2] = (T)(W0 * W2 * W2);
    for (int qz = 0; qz < Q; ++qz)
        for (int qy = 0; qy < Q; ++qy) tb.wzy[qz * Q + qy] = (T)(L.tab->w[qz] * L.tab->w[qy]);
    const int n[3] = {g.nx, g.ny, g.nz};
    const int tz = lin_chunk(n, lin_wave_slots(sizeof(T) == 8 ? PA_F64 : PA_F32, QPM));
    const int64_t nt = lin_tiles(n, tz);
    const int nb = (int)((nt + 3) / 4);
    hipLaunchKernelGGL((pa_apply_lin_kernel<Q, T, QPM>), dim3(nb), dim3(256), 0, L.stream, (const T*)L.x, (T*)L.y,
                       (T*)L.sk, (const T*)L.ed, tb, g, tz, L.add, (const T*)L.md);
    PA_HIP(hipGetLastError());
    const LinSharedNodes sn = lin_shared_nodes(g, tz);
    const int64_t nsh = sn.la + sn.lb + sn.lc;
    if (nsh > 0) {
        hipLaunchKernelGGL((pa_lin_skeleton_kernel<T>), dim3((unsigned)((nsh + 255) / 256)), dim3(256), 0, L.stream,
                           (const T*)L.x, (T*)L.y, (const T*)L.sk, g, tz, sn, L.add);
        PA_HIP(hipGetLastError());
    }
    return PA_OK;
}

int launch_apply_p1(const ApplyLaunch& L, int q_off, int dtype) {
    // per-point Lame data stays in this kernel (point-major layout, see pa_elast_setup_material);
    // the anisotropic stiffness, non-affine geometry and unstructured meshes go through the
    // sum-factorized kernel
    if (L.kmap) return launch_apply_unstructured<1>(L, q_off, dtype);
    if (L.geo != PA_GEOM_AFFINE) return launch_apply_geometry<1>(L, q_off, dtype);
    if (L.mat == PA_MAT_QP_ISO) {
        if (q_off != 1) return fail(PA_EUNSUPPORTED, "general material data is built for q = p + 2 only");
        if (!L.lin) return fail(PA_EINVAL, "per-point p = 1 data is laid out for the linear-element kernel");
        return dtype == PA_F64 ? launch_lin<3, double, true>(L) : launch_lin<3, float, true>(L);
    }
    if (L.mat != PA_MAT_ELEM_ISO) return launch_apply_material<1>(L, q_off, dtype);
    // small meshes: the sum-factorized kernel (see p1_runs_lin)
    if (!L.lin) return launch_apply_p<1>(L, q_off, dtype);
    if (dtype == PA_F64) {
        switch (q_off) {
            case 0: return launch_lin<2, double>(L);
            case 1: return launch_lin<3, double>(L);
            case 2: return launch_lin<4, double>(L);
        }
    } else {
        switch (q_off) {
            case 0: return launch_lin<2, float>(L);
            case 1: return launch_lin<3, float>(L);
            case 2: return launch_lin<4, float>(L);
        }
    }
    return fail(PA_EUNSUPPORTED, "q = p+1+%d not built", q_off);
}

}  // namespace pa
