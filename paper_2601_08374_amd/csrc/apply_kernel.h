// Fused matrix-free apply of the linear-elasticity operator on affine hexahedra.
//
// Kernel 1 (pa_apply_kernel), per element and per displacement component c
// (paper Sec. 4.2 macro-kernel fusion, Sec. 4.4 sum factorization, Sec. 4.5
// Voigt stress and transposed sweeps):
//   forward X:  u = x B, v = x G on lines (iz,iy) read straight from the
//               L-vector (restriction G; clamped entries read as 0)  -> LDS [2][D][D][Q]
//   forward Y:  (v B, u G, u B)         (lines (iz,qx))               -> LDS [3][D][Q][Q]
//   forward Z:  into a register column per (qx,qy): ref-gradient [c][m][qz]
// then pointwise, in registers: grad = J^{-T} ref-grad, Voigt stress with the
// weighted w*detJ*lambda, w*detJ*mu (eq. 7), Q_{c,m} = sum_i sigma_{c,i} J^{-1}_{m,i};
// then per output component: backward Z (column -> LDS), Y (-> LDS), X on
// lines (iz,iy) (the m-channels that share a 1D factor are summed before the
// next sweep), whose results go straight out: nodes strictly inside the element
// are written to y by their only owner; element-boundary ("skeleton")
// contributions go to a per-element buffer.
// Kernel 2 (pa_skeleton_kernel) sums, for every element-boundary node, the
// contributions of its (up to 8) elements in a fixed order and writes y -- no
// atomics, no separate initialisation of y, bitwise-reproducible results.
//
// From p = 3 on every 1D contraction uses the even-odd decomposition: on the
// symmetric Gauss-Lobatto / Gauss-Legendre point sets B[i][k] = B[D-1-i][Q-1-k]
// and G[i][k] = -G[D-1-i][Q-1-k], so pairs of outputs k, Q-1-k come from the
// sums and differences of mirrored inputs with half-size tables.
//
// gfx950 mapping: the tables are kernel arguments (kernarg segment), so
// contractions read them with scalar loads as wave-uniform SGPR operands; lanes
// map to whole 1D lines (inputs in VGPRs, no per-FMA LDS traffic); LDS only
// transposes between sweeps, with odd row strides against bank conflicts; the
// x lines of component c+1 are loaded while component c is being contracted.
// Several elements share a workgroup at low p to fill 64-wide wavefronts.
//
// Compile-time variants of the same kernel (the pointwise stage and the node
// addressing change, the sweeps do not): MAT selects the material data (per-element
// Lame parameters, per-point Lame parameters, per-element anisotropic Voigt
// stiffness); GEO the element geometry (affine J^{-1} per element, J^{-1} and w det J
// stored per quadrature point, or the trilinear map recomputed per point); UNS an
// unstructured mesh, whose nodes come from an explicit element-to-node map and whose
// element-boundary contributions are summed by pa_uns_gather_kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace pa {

// ---------------------------------------------------------------- even-odd tables
// For M (NI x NO) with M[i][k] = SIGN * M[NI-1-i][NO-1-k]:
//   P[i][k] = (M[i][k] + M[NI-1-i][k]) / 2 (i < NI/2),  P[NI/2][k] = M[NI/2][k] for odd NI;
//   N[i][k] = (M[i][k] - M[NI-1-i][k]) / 2 (i < NI/2);   k < ceil(NO/2).
template <typename T, int NI, int NO>
struct EOTab {
    static constexpr int hI = NI / 2, mI = NI & 1, hO = NO / 2, mO = NO & 1, KO = hO + mO;
    T P[(hI + mI) * KO];
    T N[(hI > 0 ? hI : 1) * KO];
};

template <typename T, int NI, int NO>
inline void fill_eo(EOTab<T, NI, NO>& t, const double* M /* M[i*NO+k] */) {
    using E = EOTab<T, NI, NO>;
    for (int k = 0; k < E::KO; ++k) {
        for (int i = 0; i < E::hI; ++i) {
            t.P[i * E::KO + k] = (T)(0.5 * (M[i * NO + k] + M[(NI - 1 - i) * NO + k]));
            t.N[i * E::KO + k] = (T)(0.5 * (M[i * NO + k] - M[(NI - 1 - i) * NO + k]));
        }
        if (E::mI) t.P[E::hI * E::KO + k] = (T)M[E::hI * NO + k];
    }
}

// out[k] = sum_i in[i] M[i][k] for every k (ADD: out += ...), even-odd form.
template <int SIGN, bool ADD, typename T, int NI, int NO>
__device__ __forceinline__ void eo_contract(const T (&in)[NI], T (&out)[NO], const EOTab<T, NI, NO>& t) {
    using E = EOTab<T, NI, NO>;
    constexpr int hI = E::hI, mI = E::mI, hO = E::hO, mO = E::mO, KO = E::KO;
    T s[hI > 0 ? hI : 1], a[hI > 0 ? hI : 1];
#pragma unroll
    for (int i = 0; i < hI; ++i) {
        s[i] = in[i] + in[NI - 1 - i];
        a[i] = in[i] - in[NI - 1 - i];
    }
#pragma unroll
    for (int k = 0; k < KO; ++k) {
        T sp = T(0), an = T(0);   // symmetric-input part (P) and antisymmetric-input part (N)
        const bool mid = (mO && k == hO);
        if (SIGN > 0 || !mid) {
#pragma unroll
            for (int i = 0; i < hI; ++i) sp = fma(s[i], t.P[i * KO + k], sp);
            if (mI) sp = fma(in[hI], t.P[hI * KO + k], sp);
        }
        if (SIGN < 0 || !mid) {
#pragma unroll
            for (int i = 0; i < hI; ++i) an = fma(a[i], t.N[i * KO + k], an);
        }
        // SIGN > 0: out[k] = sp + an, out[NO-1-k] = sp - an ; SIGN < 0: out[k] = an + sp, out[NO-1-k] = an - sp
        const T ev = SIGN > 0 ? sp : an, od = SIGN > 0 ? an : sp;
        if (mid) {
            if (ADD) out[k] += ev; else out[k] = ev;
        } else {
            if (ADD) { out[k] += ev + od; out[NO - 1 - k] += ev - od; }
            else { out[k] = ev + od; out[NO - 1 - k] = ev - od; }
        }
    }
}

// Plain table M[i][k] (NI x NO) for the low orders, where the even-odd form would
// spend more additions than it saves multiplications.
template <typename T, int NI, int NO>
struct DTab {
    T M[NI * NO];
};

template <typename T, int NI, int NO>
inline void fill_direct(DTab<T, NI, NO>& t, const double* M) {
    for (int i = 0; i < NI * NO; ++i) t.M[i] = (T)M[i];
}

template <int SIGN, bool ADD, typename T, int NI, int NO>
__device__ __forceinline__ void eo_contract(const T (&in)[NI], T (&out)[NO], const DTab<T, NI, NO>& t) {
#pragma unroll
    for (int k = 0; k < NO; ++k) {
        T acc = ADD ? out[k] : T(0);
#pragma unroll
        for (int i = 0; i < NI; ++i) acc = fma(in[i], t.M[i * NO + k], acc);
        out[k] = acc;
    }
}

// Backward (quadrature -> nodal) contraction with the forward even-odd table F of the
// same 1D matrix M (D x Q), read transposed: out[i] = sum_k in[k] M[i][k].  With
// s[k] = in[k] + in[Q-1-k], a[k] = in[k] - in[Q-1-k] (s of the middle point = its input)
// and the symmetry M[D-1-i][Q-1-k] = SIGN M[i][k], the pair i, D-1-i is
//   SIGN > 0: S = sum_k s[k] P[i][k], A = sum_k a[k] N[i][k]; out = S + A, S - A
//   SIGN < 0: S = sum_k s[k] N[i][k], A = sum_k a[k] P[i][k]; out = A + S, A - S
// and an odd D's middle output is the S (SIGN > 0) or A (SIGN < 0) sum alone.  These
// are the numbers of the even-odd form of M^T, so the backward sweeps need no table of
// their own (half the scalar registers the tables take).
template <typename T, int NI, int NO>   // NI = Q inputs, NO = D outputs
struct EOT {
    const EOTab<T, NO, NI>& f;
};

template <int SIGN, bool ADD, typename T, int NI, int NO>
__device__ __forceinline__ void eo_contract(const T (&in)[NI], T (&out)[NO], const EOT<T, NI, NO> tt) {
    using F = EOTab<T, NO, NI>;
    constexpr int hD = F::hI, mD = F::mI, hQ = F::hO, mQ = F::mO, KQ = F::KO;
    const F& t = tt.f;
    T s[KQ], a[hQ > 0 ? hQ : 1];
#pragma unroll
    for (int k = 0; k < hQ; ++k) {
        s[k] = in[k] + in[NI - 1 - k];
        a[k] = in[k] - in[NI - 1 - k];
    }
    if (mQ) s[hQ] = in[hQ];
#pragma unroll
    for (int i = 0; i < hD + mD; ++i) {
        const bool mid = mD && i == hD;
        T S = T(0), A = T(0);
        if (SIGN > 0) {
#pragma unroll
            for (int k = 0; k < KQ; ++k) S = fma(s[k], t.P[i * KQ + k], S);
            if (!mid) {
#pragma unroll
                for (int k = 0; k < hQ; ++k) A = fma(a[k], t.N[i * KQ + k], A);
            }
        } else {
            if (!mid) {
#pragma unroll
                for (int k = 0; k < KQ; ++k) S = fma(s[k], t.N[i * KQ + k], S);
            }
#pragma unroll
            for (int k = 0; k < hQ; ++k) A = fma(a[k], t.P[i * KQ + k], A);
        }
        const T ev = SIGN > 0 ? S : A, od = SIGN > 0 ? A : S;
        if (mid) {
            if (ADD) out[i] += ev; else out[i] = ev;
        } else {
            if (ADD) { out[i] += ev + od; out[NO - 1 - i] += ev - od; }
            else { out[i] = ev + od; out[NO - 1 - i] = ev - od; }
        }
    }
}

// Even-odd tables from p = 3 on (D >= 4: fewer instructions and no scalar-register spills
// of the tables there); plain tables below, where the even-odd form saves no instruction.
template <int NI, int NO>
constexpr bool kEvenOdd = NI >= 4 && NO >= 4;

template <typename T, int NI, int NO, bool EO = kEvenOdd<NI, NO>>
struct TabSel {
    using type = EOTab<T, NI, NO>;
    static void fill(type& t, const double* M) { fill_eo<T, NI, NO>(t, M); }
};
template <typename T, int NI, int NO>
struct TabSel<T, NI, NO, false> {
    using type = DTab<T, NI, NO>;
    static void fill(type& t, const double* M) { fill_direct<T, NI, NO>(t, M); }
};

// Backward tables: plain transposed tables below p = 4; in the even-odd range none (the
// backward sweeps read the forward tables transposed, EOT), except in the collocated form
// (COL), whose backward matrices differ from the forward ones: there they are even-odd
// tables of their own, stored node-major like a forward table and read through EOT.
template <typename T, int D, int Q, bool EO = kEvenOdd<D, Q>, bool COL = false>
struct BackTabs {
    typename TabSel<T, Q, D>::type Bt, Gt;   // quadrature (Q) -> nodal (D)
};
template <typename T, int D, int Q>
struct BackTabs<T, D, Q, true, false> {};
template <typename T, int D, int Q>
struct BackTabs<T, D, Q, true, true> {
    EOTab<T, D, Q> Bb, Gb;   // node-major: Bb[i][j] = the weight of point j's value at node i
};

template <typename T, int D, int Q, bool COL = false>
struct ApplyTabs {
    typename TabSel<T, D, Q>::type Bf, Gf;   // forward: nodal (D) -> quadrature (Q)
    BackTabs<T, D, Q, kEvenOdd<D, Q>, COL> bk;
    T w[Q];
    T x[Q];   // Gauss-Legendre points on [0,1] (trilinear geometry)
};

// Backward operands B^T and G^T of the apply tables.
template <typename T, int D, int Q, bool COL>
__device__ __forceinline__ decltype(auto) back_B(const ApplyTabs<T, D, Q, COL>& t) {
    if constexpr (kEvenOdd<D, Q> && COL) return EOT<T, Q, D>{t.bk.Bb};
    else if constexpr (kEvenOdd<D, Q>) return EOT<T, Q, D>{t.Bf};
    else return (t.bk.Bt);
}
template <typename T, int D, int Q, bool COL>
__device__ __forceinline__ decltype(auto) back_G(const ApplyTabs<T, D, Q, COL>& t) {
    if constexpr (kEvenOdd<D, Q> && COL) return EOT<T, Q, D>{t.bk.Gb};
    else if constexpr (kEvenOdd<D, Q>) return EOT<T, Q, D>{t.Gf};
    else return (t.bk.Gt);
}

template <typename T, int D, int Q>
inline ApplyTabs<T, D, Q> make_tabs(const Tables& t) {
    ApplyTabs<T, D, Q> r;
    TabSel<T, D, Q>::fill(r.Bf, t.B);
    TabSel<T, D, Q>::fill(r.Gf, t.G);
    if constexpr (!kEvenOdd<D, Q>) {
        double Bt[D * Q], Gt[D * Q];
        for (int i = 0; i < D; ++i)
            for (int k = 0; k < Q; ++k) {
                Bt[k * D + i] = t.B[i * Q + k];
                Gt[k * D + i] = t.G[i * Q + k];
            }
        TabSel<T, Q, D>::fill(r.bk.Bt, Bt);
        TabSel<T, Q, D>::fill(r.bk.Gt, Gt);
    }
    for (int k = 0; k < Q; ++k) r.w[k] = (T)t.w[k];
    for (int k = 0; k < Q; ++k) r.x[k] = (T)t.xq[k];
    return r;
}

// Tables of the collocated form (affine elements, per-element Lame data, plain tables).
// J^{-1} and the Lame weights are constant over such an element, so every entry of the
// reference gradient, of the stress and of Q = sigma J^{-T} is a polynomial of degree at
// most p in each coordinate and equals its interpolant through the p+1 Gauss-Lobatto nodes
// per axis.  Substituting that interpolant into the quadrature sums regroups them: the
// pointwise stage runs at the (p+1)^3 nodes (forward tables: the identity for values and
// the nodal differentiation matrix l'_i(x_j) for derivatives; unit weights), and the rule
// enters through the backward tables Mm[j][i] = sum_r w_r l_j(xi_r) l_i(xi_r) and
// Nm[j][i] = sum_r w_r l_j(xi_r) l'_i(xi_r), built from the tables of the requested q.
template <typename T, int D>
inline ApplyTabs<T, D, D, kEvenOdd<D, D>> make_colloc_tabs(const Tables& t) {
    constexpr bool EO = kEvenOdd<D, D>;
    const int Q = t.q;
    // forward [node i][node j]; backward node-major [node i][point j] and point-major [j][i]
    double Bf[D * D], Gf[D * D], Bn[D * D], Gn[D * D], Bt[D * D], Gt[D * D];
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            Bf[i * D + j] = i == j ? 1.0 : 0.0;
            double v = 0.0;
            if (i == j) {
                for (int m = 0; m < D; ++m)
                    if (m != i) v += 1.0 / (t.gll[i] - t.gll[m]);
            } else {
                double num = 1.0, den = 1.0;
                for (int m = 0; m < D; ++m) {
                    if (m == i) continue;
                    den *= t.gll[i] - t.gll[m];
                    if (m != j) num *= t.gll[j] - t.gll[m];
                }
                v = num / den;
            }
            Gf[i * D + j] = v;
            double mm = 0.0, nm = 0.0;   // Mm[j][i], Nm[j][i]
            for (int r = 0; r < Q; ++r) {
                mm += t.w[r] * t.B[j * Q + r] * t.B[i * Q + r];
                nm += t.w[r] * t.B[j * Q + r] * t.G[i * Q + r];
            }
            Bt[j * D + i] = Bn[i * D + j] = mm;
            Gt[j * D + i] = Gn[i * D + j] = nm;
        }
    ApplyTabs<T, D, D, EO> r;
    TabSel<T, D, D>::fill(r.Bf, Bf);
    TabSel<T, D, D>::fill(r.Gf, Gf);
    if constexpr (EO) {
        // node-major, the orientation EOT reads; Mm is symmetric under the mirror i -> D-1-i,
        // j -> D-1-j and Nm antisymmetric, as B and G are
        fill_eo<T, D, D>(r.bk.Bb, Bn);
        fill_eo<T, D, D>(r.bk.Gb, Gn);
    } else {
        TabSel<T, D, D>::fill(r.bk.Bt, Bt);
        TabSel<T, D, D>::fill(r.bk.Gt, Gt);
    }
    for (int k = 0; k < D; ++k) {
        r.w[k] = T(1);
        r.x[k] = (T)t.gll[k];
    }
    return r;
}

// Degrees whose affine per-element apply runs in the collocated form.
template <int P>
constexpr bool kCollocated = true;

// ---------------------------------------------------------------- skeleton numbering
// Element-boundary ("skeleton") local nodes (some index 0 or p), numbered in
// lexicographic (iz, iy, ix) order: full layers iz = 0 and iz = p hold D*D nodes,
// inner layers 4(D-1) nodes (rows iy = 0 and iy = p complete, inner rows ix = 0, p).
template <int D>
struct Skel {
    static constexpr int P = D - 1;
    static constexpr int S = D * D * D - (D - 2) * (D - 2) * (D - 2);
    static constexpr int LAYER = 4 * (D - 1);
    __host__ __device__ __forceinline__ static int index(int ix, int iy, int iz) {
        int base, off;
        if (iz == 0 || iz == P) {
            base = (iz == 0) ? 0 : D * D + (D - 2) * LAYER;
            off = iy * D + ix;
        } else {
            base = D * D + (iz - 1) * LAYER;
            if (iy == 0) off = ix;
            else if (iy == P) off = D + 2 * (D - 2) + ix;
            else off = D + 2 * (iy - 1) + (ix == P ? 1 : 0);
        }
        return base + off;
    }
    __host__ __device__ __forceinline__ static bool interior(int ix, int iy, int iz) {
        return ix > 0 && ix < P && iy > 0 && iy < P && iz > 0 && iz < P;
    }
    // A row (iy, iz) is either entirely on the element boundary ("full": its nodes have
    // consecutive slots from index(0, iy, iz)) or crosses the interior (only its two end
    // nodes are skeleton nodes, at index(0, iy, iz) and index(0, iy, iz) + 1).
    __host__ __device__ __forceinline__ static bool full_row(int iy, int iz) {
        return iy == 0 || iy == P || iz == 0 || iz == P;
    }
    // Slot of node ix of a row from the row's first slot; not called for interior nodes.
    __host__ __device__ __forceinline__ static int row_slot(int s0, bool full, int ix) {
        return full ? s0 + ix : s0 + (ix == P ? 1 : 0);
    }
    // Buffer layout: node-major ([c][s][e]) up to p = 5, so that the skeleton kernel's
    // reads of one slot for consecutive elements are contiguous; element-major
    // ([e][c][s]) from p = 6 on, where an element's slots are many and its face rows
    // long enough to keep the apply kernel's writes contiguous (measured crossover).
    static constexpr bool ELEM_MAJOR = D >= 7;
    __device__ __forceinline__ static size_t offset(int e, int c, int s, int NE) {
        return ELEM_MAJOR ? ((size_t)e * 3 + c) * S + s : ((size_t)c * S + s) * NE + e;
    }
    // offset(e, c, s, NE) - offset(e, c, 0, NE)
    __device__ __forceinline__ static size_t slot_offset(int s, int NE) {
        return ELEM_MAJOR ? (size_t)s : (size_t)(unsigned)s * (unsigned)NE;
    }
};

// LDS layout of one element: Ua[ch][iz][iy][qx] (X-pass output, two channels;
// reused for the backward Y output) and Ra[ch][iz][qy][qx] (Y-pass output, three
// channels; reused for the backward Z output), qx contiguous.  Strides in words.
struct LdsStrides {
    int UY, UZ, UC, UT;   // Ua: iy, iz, channel, element
    int RY, RZ, RC, ST;   // Ra: qy, iz, channel, element
};

// Padded strides, chosen to minimise bank conflicts of the four access
// patterns (X lines, Y lines on Ua, Y lines on Ra, Z columns): each candidate was
// scored by the largest number of lanes that share a bank within every group of 16
// lanes (8-byte words) or 32 lanes (4-byte words), summed over the kernel's LDS
// instructions, with the element footprint capped at 1.25x the unpadded one.
// Other (p, q) use a plain layout with odd row strides.
constexpr LdsStrides lds_strides(int P, int Q, int word) {
    if (Q == P + 2 && word == 8) {
        switch (P) {
            case 2: return {5, 20, 54, 108, 4, 20, 56, 172};
            case 3: return {5, 20, 80, 160, 5, 26, 105, 313};
            case 4: return {7, 35, 174, 351, 6, 38, 188, 574};
            case 5: return {7, 42, 256, 508, 7, 55, 324, 986};
            case 6: return {9, 63, 440, 880, 8, 72, 496, 1488};
            case 7: return {10, 89, 702, 1416, 9, 89, 704, 2120};
            case 8: return {13, 117, 1050, 2100, 10, 106, 948, 2844};
        }
    }
    if (Q == P + 2 && word == 4) {
        switch (P) {
            case 2: return {4, 12, 37, 81, 4, 20, 60, 176};
            case 3: return {5, 20, 80, 176, 5, 26, 103, 313};
            case 4: return {7, 38, 201, 414, 6, 38, 188, 574};
            case 5: return {7, 42, 272, 540, 7, 52, 309, 945};
            case 6: return {9, 72, 494, 988, 8, 72, 496, 1488};
            case 7: return {9, 72, 576, 1152, 9, 85, 676, 2033};
            case 8: return {13, 117, 1050, 2100, 10, 106, 948, 2844};
        }
    }
    // the collocated form (Q = p + 1) in double precision, chosen the same way; at p = 4 and in
    // single precision the padded layouts measured no faster than the plain one
    if (Q == P + 1 && word == 8) {
        switch (P) {
            case 2: return {3, 9, 27, 59, 3, 10, 29, 89};
            case 3: return {5, 20, 79, 158, 4, 20, 76, 228};
        }
    }
    const int D = P + 1, QP = Q | 1;
    return {QP, D * QP, D * D * QP, 2 * D * D * QP, Q, Q * Q, D * Q * Q, 3 * D * Q * Q};
}

// Elements per workgroup: fill 64-lane waves with the E*Q*Q quadrature columns while
// keeping the workgroup's LDS at or below 64 KiB.
template <int P, int Q, typename T>
struct ApplyCfg {
    static constexpr int D = P + 1;
    static constexpr int QQ = Q * Q;
    static constexpr LdsStrides L = lds_strides(P, Q, (int)sizeof(T));
    static constexpr int UT = L.UT, ST = L.ST;
    static_assert(L.UY >= Q && L.UZ >= (D - 1) * L.UY + Q && L.UC >= (D - 1) * (L.UZ + L.UY) + Q &&
                      L.UT >= L.UC + (D - 1) * (L.UZ + L.UY) + Q,
                  "Ua strides overlap");
    static_assert(L.RY >= Q && L.RZ >= (Q - 1) * L.RY + Q && L.RC >= (D - 1) * L.RZ + (Q - 1) * L.RY + Q &&
                      L.ST >= 2 * L.RC + (D - 1) * L.RZ + (Q - 1) * L.RY + Q,
                  "Ra strides overlap");
    static constexpr int LDS_ELEM = ST + UT + kEdStride;
    // Lane utilisation of a sweep over n lines (one lane each) in 64-wide waves.
    static constexpr double util(int n) { return double(n) / (((n + 63) / 64) * 64); }
    // Score of E elements per workgroup: the utilisation of the column passes (forward Z,
    // pointwise, backward Z: the bulk of the work); in single precision also a quarter
    // weight for the mean of the X and Y line passes.  (Measured: the larger workgroups
    // this picks at p = 2, 3 and 8 gain 2-8% in FP32; in FP64 p = 2 was unchanged and
    // p = 3 slower, so FP64 keeps the smallest workgroup with the best column use.)
    static constexpr int pickE() {
        constexpr bool lines = sizeof(T) == 4;
        int bestE = 1;
        double bestU = 0.0;
        for (int E = 1; E * QQ <= 256; ++E) {
            if (E > 1 && E * LDS_ELEM * (int)sizeof(T) > 65536) break;
            const double u = util(E * QQ) + (lines ? 0.25 * 0.5 * (util(E * D * D) + util(E * D * Q)) : 0.0);
            if (u > bestU + (lines ? 0.005 : 0.02)) { bestU = u; bestE = E; }
        }
        return bestE;
    }
    static constexpr int E = pickE();
    static constexpr int NT = ((E * QQ + 63) / 64) * 64;
};

// Consecutive workgroups are dealt round-robin to the 8 XCDs; remap so that each
// XCD receives a contiguous range of element blocks (shared faces stay in one L2).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, k = b >> 3;
    const int start = xcd * per + (xcd < rem ? xcd : rem);
    return start + k;
}

// Material data forms of the pointwise stage: per-element Lame parameters (ed[9],
// ed[10] = detJ lambda, detJ mu), per-quadrature-point Lame parameters (md =
// [NE][Q^3][2] lambda, mu; ed[9] = detJ), or a per-element anisotropic Voigt
// stiffness (md = [NE][21], upper triangle row by row; ed[9] = detJ).
enum : int { kMatElemIso = 0, kMatQpIso = 1, kMatAniso = 2 };

// Element geometry forms: affine (ed[0..8] = J^{-1}, constant per element), trilinear
// with J^{-1} and w det J stored per quadrature point (gd = [NE][10][Q^3]: word
// m*3+i is (J^{-1})_{m,i}, word 9 is w_alpha det J), or trilinear recomputed per
// point from 21 coefficients per element (gd = [NE][21]: vectors a..g of
// x(xi) = x0 + a xi + b eta + c zeta + d xi eta + e xi zeta + f eta zeta + g xi eta zeta).
// The non-affine forms take ed[9], ed[10] = lambda, mu (no det J).
enum : int { kGeoAffine = 0, kGeoQp = 1, kGeoTri = 2 };

// Unstructured kernels that keep the block's element-to-node map in LDS instead of each
// line's node ids in registers: where that raises the number of waves per SIMD (FP64 at
// p = 1 and p = 8; elsewhere the LDS copy measured slower).
template <int P, typename T>
constexpr bool kUnsIdsInLds = sizeof(T) == 8 && (P == 1 || P == 8);

// UNS: unstructured mesh.  Nodes come from the element-to-node map kmap (global node,
// kClampBit on clamped nodes; g.clamp != 0 for a constrained apply), element-interior
// nodes go to y directly and element-boundary nodes to the skeleton entry kpos of
// their (element, slot): entries are stored in the order of the per-node gather lists,
// so pa_uns_gather_kernel reads each node's contributions as one contiguous run.
template <int P, int Q, typename T, int MAT = kMatElemIso, int GEO = kGeoAffine, bool UNS = false, bool COL = false>
__global__ void __launch_bounds__((ApplyCfg<P, Q, T>::NT))
pa_apply_kernel(const T* __restrict__ x, T* __restrict__ y, T* __restrict__ sk, const T* __restrict__ ed,
                const ApplyTabs<T, P + 1, Q, COL> tab, const Geom g, const int add, const T* __restrict__ md,
                const T* __restrict__ gd, const int* __restrict__ kmap, const int* __restrict__ kpos) {
    static_assert(GEO == kGeoAffine || MAT == kMatElemIso, "non-affine geometry takes per-element Lame data");
    static_assert(!UNS || GEO == kGeoTri, "unstructured meshes take the recomputed trilinear geometry");
    using C = ApplyCfg<P, Q, T>;
    using SK = Skel<P + 1>;
    constexpr int D = P + 1, E = C::E, NT = C::NT, QQ = Q * Q;
    constexpr int UT = C::UT, ST = C::ST;
    constexpr int UY = C::L.UY, UZ = C::L.UZ, UC = C::L.UC, RY = C::L.RY, RZ = C::L.RZ, RC = C::L.RC;
    __shared__ T Ra[E * ST];          // Y-pass output | backward Z output
    __shared__ T Ua[E * UT];          // X-pass output | backward Y output
    __shared__ T Es[E * kEdStride];   // per-element PA data of the block
    __shared__ T Cs[MAT == kMatAniso || GEO == kGeoTri ? E * 21 : 1];   // stiffness or trilinear coefficients
    // unstructured: node ids of the element lines in registers, or (KL) the block's map in LDS
    constexpr bool KL = UNS && kUnsIdsInLds<P, T>;
    __shared__ int Ks[KL ? E * D * D * D : 1];

    const int tid = threadIdx.x;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int e0 = blk * E;
    const int ne_blk = g.NE - e0 < E ? g.NE - e0 : E;
    const int cel = tid / QQ, cq = tid % QQ;
    const int cqx = cq % Q, cqy = cq / Q;
    const bool has_col = tid < E * QQ;
    T gq[3][3][Q];   // [component][reference direction][qz]
    const size_t NN = (size_t)g.Nn;

    // x-lines of this thread: line l = (el, iz, iy) of the block, l = tid + j*NT.
    // The first node of each line is computed once; the loads of component c+1
    // are issued right after the X sweep of component c.
    constexpr int NL = E * D * D;
    constexpr int GX = (NL + NT - 1) / NT;
    static_assert(GX * D <= 32, "clamp mask bits");
    int ln_node[GX];       // global node of (ix = 0) of the line (unstructured: 0, KL: its word in Ks), or -1
    int ln_slot[GX];       // skeleton slot of (ix = 0) of the line
    int ln_el[GX];         // element of the line in the block
    int ln_ua[GX];         // word of the line's (qx = 0) in Ua
    unsigned ln_full = 0u; // bit j: the line lies on the element boundary
    unsigned ln_cl = 0u;   // bit j*D + ix: clamped node (read as 0)
    int ln_nodes[UNS && !KL ? GX : 1][UNS && !KL ? D : 1];   // unstructured: every node of the line
    // global node of node ix of line j (the map word without its clamp flag)
    auto uns_node = [&](int j, int ix) -> size_t {
        if constexpr (KL) return (unsigned)Ks[ln_node[j] + ix] & ~kClampBit;
        else return (size_t)ln_nodes[UNS ? j : 0][UNS ? ix : 0];
    };
    // box coordinates of the block's first element (block-uniform)
    const int bx0 = e0 % g.nx, bxr = e0 / g.nx, by0 = bxr % g.ny, bz0 = bxr / g.ny;
    // the lines' node addresses and clamp flags come from the element numbers (from the
    // block's map in LDS when KL), so that the first x loads are in flight while the
    // element data is staged
    auto line_setup = [&]() {
#pragma unroll
    for (int j = 0; j < GX; ++j) {
        ln_node[j] = -1;
        ln_slot[j] = 0;
        ln_el[j] = 0;
        ln_ua[j] = 0;
        const int l = tid + j * NT;
        if (l < NL) {
            const int el = l / (D * D), r = l % (D * D);
            const int iz = r / D, iy = r % D;
            const bool valid = el < ne_blk;
            ln_el[j] = el;
            ln_ua[j] = el * UT + iz * UZ + iy * UY;
            ln_slot[j] = SK::index(0, iy, iz);
            if (SK::full_row(iy, iz)) ln_full |= 1u << j;
            if (KL && valid) {
                ln_node[j] = el * (D * D * D) + D * (iy + D * iz);
                if (g.clamp) {
#pragma unroll
                    for (int ix = 0; ix < D; ++ix)
                        if ((unsigned)Ks[ln_node[j] + ix] & kClampBit) ln_cl |= 1u << (j * D + ix);
                }
            } else if (UNS && valid) {
                ln_node[j] = 0;
                const int* mp = kmap + (size_t)(e0 + el) * (D * D * D) + D * (iy + D * iz);
#pragma unroll
                for (int ix = 0; ix < D; ++ix) {
                    const unsigned v = (unsigned)mp[ix];
                    ln_nodes[UNS && !KL ? j : 0][UNS && !KL ? ix : 0] = (int)(v & ~kClampBit);
                    if (g.clamp && (v & kClampBit)) ln_cl |= 1u << (j * D + ix);
                }
            } else if (valid) {
                // element e0 + el: step from the block's first element (no per-lane division)
                int ex = bx0 + el, ey = by0, ez = bz0;
                while (ex >= g.nx) {
                    ex -= g.nx;
                    if (++ey == g.ny) {
                        ey = 0;
                        ++ez;
                    }
                }
                const int gx0 = ex * P, gy0 = ey * P, gz0 = ez * P;
                ln_node[j] = gx0 + g.Nx * (gy0 + iy + g.Ny * (gz0 + iz));
                if (g.clamp) {
#pragma unroll
                    for (int ix = 0; ix < D; ++ix)
                        if (clamped_node(g.clamp, gx0 + ix, gy0 + iy, gz0 + iz, g)) ln_cl |= 1u << (j * D + ix);
                }
            }
        }
    }
    };
    T xr[GX][D];
    auto line_load = [&](int c) {
#pragma unroll
        for (int j = 0; j < GX; ++j)
#pragma unroll
            for (int ix = 0; ix < D; ++ix)
                xr[j][ix] = (ln_node[j] >= 0 && !((ln_cl >> (j * D + ix)) & 1u))
                                ? x[c * NN + (UNS ? uns_node(j, ix) : (size_t)(ln_node[j] + ix))]
                                : T(0);
    };
    if constexpr (!KL) {
        line_setup();
        line_load(0);
    }
    if constexpr (KL) {
        for (int w = tid; w < E * D * D * D; w += NT)
            Ks[w] = w < ne_blk * (D * D * D) ? kmap[(size_t)e0 * (D * D * D) + w] : 0;
    }
    for (int w = tid; w < E * kEdStride; w += NT)
        Es[w] = w < ne_blk * kEdStride ? ed[(size_t)e0 * kEdStride + w] : T(0);
    if constexpr (MAT == kMatAniso) {
        for (int w = tid; w < E * 21; w += NT) Cs[w] = w < ne_blk * 21 ? md[(size_t)e0 * 21 + w] : T(0);
    }
    if constexpr (GEO == kGeoTri) {
        // slots past the last element repeat element e0 (a regular map; their Lame data is zero)
        for (int w = tid; w < E * 21; w += NT) Cs[w] = gd[(size_t)e0 * 21 + (w < ne_blk * 21 ? w : w % 21)];
    }

    __syncthreads();       // Es, Cs, Ks ready
    if constexpr (KL) {
        line_setup();
        line_load(0);
    }

    // Y-pass line (el, iz, qx) of word w: its offsets in Ua and Ra; when one pass of the
    // workgroup covers all lines, the thread's line is computed once for every sweep
    constexpr bool Y1 = E * D * Q <= NT;
    auto yline = [&](int w, int& ua, int& ra) {
        const int el = w / (D * Q), r = w % (D * Q);
        const int iz = r / Q, qx = r % Q;
        ua = el * UT + iz * UZ + qx;
        ra = el * ST + iz * RZ + qx;
    };
    int y1_ua = 0, y1_ra = 0;
    if constexpr (Y1) yline(tid, y1_ua, y1_ra);
    auto yoffs = [&](int w, int& ua, int& ra) {
        if constexpr (Y1) {
            ua = y1_ua;
            ra = y1_ra;
        } else {
            yline(w, ua, ra);
        }
    };

#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // ---- forward X from the x lines: Ua[el][ch][iz][iy][qx]
#pragma unroll
        for (int j = 0; j < GX; ++j) {
            const int l = tid + j * NT;
            if (l < NL) {
                T u[Q], v[Q];
                eo_contract<1, false>(xr[j], u, tab.Bf);
                eo_contract<-1, false>(xr[j], v, tab.Gf);
                T* uo = Ua + ln_ua[j];
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    uo[k] = u[k];
                    uo[UC + k] = v[k];
                }
            }
        }
        if (c < 2) line_load(c + 1);
        __syncthreads();
        // ---- forward Y: lines (el, iz, qx): s0 = v B (d/dxi), s1 = u G (d/deta), s2 = u B
        for (int w = tid; w < E * D * Q; w += NT) {
            int ua, ra;
            yoffs(w, ua, ra);
            const T* ui = Ua + ua;
            T uv[D], vv[D], s0[Q], s1[Q], s2[Q];
#pragma unroll
            for (int i = 0; i < D; ++i) { uv[i] = ui[i * UY]; vv[i] = ui[UC + i * UY]; }
            eo_contract<1, false>(vv, s0, tab.Bf);
            eo_contract<-1, false>(uv, s1, tab.Gf);
            eo_contract<1, false>(uv, s2, tab.Bf);
            T* so = Ra + ra;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                so[k * RY] = s0[k];
                so[RC + k * RY] = s1[k];
                so[2 * RC + k * RY] = s2[k];
            }
        }
        __syncthreads();
        // ---- forward Z: the thread's own (qx,qy) column
        if (has_col) {
            const T* si = Ra + cel * ST + cqy * RY + cqx;
            T i0[D], i1[D], i2[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                i0[i] = si[i * RZ];
                i1[i] = si[RC + i * RZ];
                i2[i] = si[2 * RC + i * RZ];
            }
            eo_contract<1, false>(i0, gq[c][0], tab.Bf);
            eo_contract<1, false>(i1, gq[c][1], tab.Bf);
            eo_contract<-1, false>(i2, gq[c][2], tab.Gf);
        }
        // the next X sweep writes Ua only; Ra is rewritten after the next barrier
    }

    // ---- pointwise stage: Voigt stress and Q = sigma J^{-T}, in place
    if (has_col) {
        T Ji[9];
        const T* d = Es + cel * kEdStride;
#pragma unroll
        for (int k = 0; k < 9; ++k) Ji[k] = d[k];
        const T lw = d[9], mw = d[10];
        const T wxy = tab.w[cqx] * tab.w[cqy];
        // trilinear geometry: the parts of the Jacobian columns fixed along the column
        // (J[:,0] = A0 + zeta A1, J[:,1] = B0 + zeta B1, J[:,2] = C0)
        T A0[3], A1[3], B0[3], B1[3], C0[3];
        if constexpr (GEO == kGeoTri) {
            const T* gc = Cs + cel * 21;
            const T xi = tab.x[cqx], eta = tab.x[cqy];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T a = gc[i], b = gc[3 + i], c = gc[6 + i], dd = gc[9 + i], ee = gc[12 + i],
                        f = gc[15 + i], gg = gc[18 + i];
                A0[i] = a + dd * eta;
                A1[i] = ee + gg * eta;
                B0[i] = b + dd * xi;
                B1[i] = f + gg * xi;
                C0[i] = c + ee * xi + (f + gg * xi) * eta;
            }
        }
        // columns of the tail block past the last element read element e0 (zero Lame data there)
        const int ce = cel < ne_blk ? cel : 0;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            T W = wxy * tab.w[k];
            if constexpr (GEO == kGeoQp) {
                const T* gp = gd + (size_t)(e0 + ce) * (10 * Q * Q * Q) + cqx + Q * (cqy + Q * k);
#pragma unroll
                for (int w = 0; w < 9; ++w) Ji[w] = gp[w * (Q * Q * Q)];
                W = gp[9 * (Q * Q * Q)];
            } else if constexpr (GEO == kGeoTri) {
                // Ji = adj(J) = det J * J^{-1}; the 1/det J of both J^{-1} factors and the
                // det J of the measure leave W / det J
                const T z = tab.x[k];
                const T j00 = A0[0] + z * A1[0], j10 = A0[1] + z * A1[1], j20 = A0[2] + z * A1[2];
                const T j01 = B0[0] + z * B1[0], j11 = B0[1] + z * B1[1], j21 = B0[2] + z * B1[2];
                const T j02 = C0[0], j12 = C0[1], j22 = C0[2];
                // adj(J)[m][i] = cofactor of J[i][m]
                Ji[0] = j11 * j22 - j12 * j21;
                Ji[1] = j02 * j21 - j01 * j22;
                Ji[2] = j01 * j12 - j02 * j11;
                Ji[3] = j12 * j20 - j10 * j22;
                Ji[4] = j00 * j22 - j02 * j20;
                Ji[5] = j02 * j10 - j00 * j12;
                Ji[6] = j10 * j21 - j11 * j20;
                Ji[7] = j01 * j20 - j00 * j21;
                Ji[8] = j00 * j11 - j01 * j10;
                const T det = j00 * Ji[0] + j01 * Ji[3] + j02 * Ji[6];
                W = W / det;
            }
            T du[3][3];   // du[c][i] = d u_c / d x_i = sum_m Jinv[m][i] ref[c][m]
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    du[cc][i] = Ji[0 * 3 + i] * gq[cc][0][k] + Ji[1 * 3 + i] * gq[cc][1][k] +
                                Ji[2 * 3 + i] * gq[cc][2][k];
            T s[3][3];
            if constexpr (MAT == kMatAniso) {
                // sigma_V = W detJ C eps_V, eps_V = (e_xx, e_yy, e_zz, 2e_yz, 2e_xz, 2e_xy)
                const T* cp = Cs + cel * 21;
                const T ev[6] = {du[0][0], du[1][1], du[2][2], du[1][2] + du[2][1], du[0][2] + du[2][0],
                                 du[0][1] + du[1][0]};
                const T Wd = W * lw;
                T sv[6];
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    T acc = T(0);
#pragma unroll
                    for (int j = 0; j < 6; ++j) {
                        const int a = i < j ? i : j, b = i < j ? j : i;   // packed upper triangle
                        acc += cp[a * 6 - a * (a - 1) / 2 + (b - a)] * ev[j];
                    }
                    sv[i] = Wd * acc;
                }
                s[0][0] = sv[0];
                s[1][1] = sv[1];
                s[2][2] = sv[2];
                s[1][2] = s[2][1] = sv[3];
                s[0][2] = s[2][0] = sv[4];
                s[0][1] = s[1][0] = sv[5];
            } else {
                T lam, mu;
                if constexpr (MAT == kMatQpIso) {
                    const size_t pt = ((size_t)(e0 + ce) * (Q * Q * Q) + cqx + Q * (cqy + Q * k)) * 2;
                    lam = W * lw * md[pt];
                    mu = W * lw * md[pt + 1];
                } else {
                    lam = W * lw;
                    mu = W * mw;
                }
                const T div = du[0][0] + du[1][1] + du[2][2];
                const T ld = lam * div, m2 = mu + mu;
                s[0][0] = ld + m2 * du[0][0];
                s[1][1] = ld + m2 * du[1][1];
                s[2][2] = ld + m2 * du[2][2];
                s[0][1] = s[1][0] = mu * (du[0][1] + du[1][0]);
                s[0][2] = s[2][0] = mu * (du[0][2] + du[2][0]);
                s[1][2] = s[2][1] = mu * (du[1][2] + du[2][1]);
            }
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    gq[cc][m][k] = s[cc][0] * Ji[m * 3 + 0] + s[cc][1] * Ji[m * 3 + 1] + s[cc][2] * Ji[m * 3 + 2];
        }
    }

    // ---- backward sweeps, one output component at a time; results leave from the X sweep
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // backward Z: own column -> Ra[el][m][iz][qy][qx] (the previous Y sweep finished
        // reading Ra before the barrier that preceded the previous X sweep)
        if (has_col) {
            T t0[D], t1[D], t2[D];
            eo_contract<1, false>(gq[c][0], t0, back_B(tab));
            eo_contract<1, false>(gq[c][1], t1, back_B(tab));
            eo_contract<-1, false>(gq[c][2], t2, back_G(tab));
            T* so = Ra + cel * ST + cqy * RY + cqx;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                so[i * RZ] = t0[i];
                so[RC + i * RZ] = t1[i];
                so[2 * RC + i * RZ] = t2[i];
            }
        }
        __syncthreads();
        // backward Y: lines (el, iz, qx): R0 = T0 B^T, R12 = T1 G^T + T2 B^T
        for (int w = tid; w < E * D * Q; w += NT) {
            int ua, ra;
            yoffs(w, ua, ra);
            const T* ti = Ra + ra;
            T a0[Q], a1[Q], a2[Q], r0[D], r12[D];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                a0[k] = ti[k * RY];
                a1[k] = ti[RC + k * RY];
                a2[k] = ti[2 * RC + k * RY];
            }
            eo_contract<1, false>(a0, r0, back_B(tab));
            eo_contract<-1, false>(a1, r12, back_G(tab));
            eo_contract<1, true>(a2, r12, back_B(tab));
            T* ro = Ua + ua;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                ro[i * UY] = r0[i];
                ro[UC + i * UY] = r12[i];
            }
        }
        __syncthreads();
        // backward X on lines (el, iz, iy): y = R0 G^T + R12 B^T, written out directly:
        // element-interior nodes to y (sole owner), boundary nodes to the skeleton buffer
#pragma unroll
        for (int j = 0; j < GX; ++j) {
            const int l = tid + j * NT;
            if (l < NL && ln_node[j] >= 0) {
                const int el = ln_el[j];
                const T* ri = Ua + ln_ua[j];
                T a0[Q], a1[Q], yo[D];
#pragma unroll
                for (int k = 0; k < Q; ++k) { a0[k] = ri[k]; a1[k] = ri[UC + k]; }
                eo_contract<-1, false>(a0, yo, back_G(tab));
                eo_contract<1, true>(a1, yo, back_B(tab));
                const bool full = (ln_full >> j) & 1u;
                T* const skl = sk + SK::offset(e0 + el, c, 0, g.NE);   // slot 0 of (element, c)
#pragma unroll
                for (int ix = 0; ix < D; ++ix) {
                    // the end nodes of a row are always skeleton nodes
                    const bool inner = ix > 0 && ix < P && !full;
                    if constexpr (UNS) {
                        if (inner) {
                            // sole owner; a clamped interior node keeps its input in a constrained apply
                            const size_t o = c * NN + uns_node(j, ix);
                            const T v = ((ln_cl >> (j * D + ix)) & 1u) ? x[o] : yo[ix];
                            y[o] = add ? y[o] + v : v;
                        } else {
                            sk[(size_t)kpos[(size_t)(e0 + el) * SK::S + SK::row_slot(ln_slot[j], full, ix)] * 3 + c] =
                                yo[ix];
                        }
                    } else if (inner) {
                        T* yp = y + c * NN + ln_node[j] + ix;
                        *yp = add ? *yp + yo[ix] : yo[ix];
                    } else {
                        skl[SK::slot_offset(SK::row_slot(ln_slot[j], full, ix), g.NE)] = yo[ix];
                    }
                }
            }
        }
        // the next backward Z writes Ra only; Ua is rewritten after the next barrier
    }
}

// The element-boundary nodes of the box numbered compactly, so that the skeleton kernel's
// lanes all have work: z-layers in order; a layer on element faces (gz % p == 0) holds
// all Nx Ny nodes; any other layer holds, per element slab of rows, the full row
// gy % p == 0 and the nodes gx % p == 0 of the p - 1 rows after it, then the last full row.
struct SkelNodes {
    int full;    // nodes of a face layer: Nx Ny
    int row;     // nodes of one element slab of rows in an inner layer: Nx + (p - 1)(nx + 1)
    int inner;   // nodes of an inner layer: ny row + Nx
    int slab;    // nodes of one element slab of layers: full + (p - 1) inner
    int total;   // nz slab + full
};

inline SkelNodes skel_nodes(const Geom& g, int p) {
    SkelNodes s;
    s.full = g.Nx * g.Ny;
    s.row = g.Nx + (p - 1) * (g.nx + 1);
    s.inner = g.ny * s.row + g.Nx;
    s.slab = s.full + (p - 1) * s.inner;
    s.total = g.nz * s.slab + s.full;
    return s;
}

template <int P>
__host__ __device__ __forceinline__ void skel_node_coords(int t, const SkelNodes& s, const Geom& g, int& gx,
                                                           int& gy, int& gz) {
    const int ez = t / s.slab;
    int r = t - ez * s.slab;
    if (r < s.full) {
        gz = ez * P;
        gy = r / g.Nx;
        gx = r - gy * g.Nx;
        return;
    }
    r -= s.full;
    const int j = r / s.inner;
    r -= j * s.inner;
    gz = ez * P + 1 + j;
    const int ey = r / s.row;
    r -= ey * s.row;
    if (r < g.Nx) {
        gy = ey * P;
        gx = r;
        return;
    }
    r -= g.Nx;
    const int k = r / (g.nx + 1);
    gy = ey * P + 1 + k;
    gx = (r - k * (g.nx + 1)) * P;
}

// Kernel 2: for every element-boundary node, sum the skeleton contributions of its
// elements in a fixed order and write y.
template <int P, typename T>
__global__ void __launch_bounds__(256)
pa_skeleton_kernel(const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ sk, const Geom g,
                   const SkelNodes sn, const int add) {
    using SK = Skel<P + 1>;
    // each XCD takes a contiguous range of nodes, as the apply kernel gave it a contiguous
    // range of elements: most of a node's contributions were written through the same L2
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (t >= sn.total) return;
    int gx, gy, gz;
    skel_node_coords<P>(t, sn, g, gx, gy, gz);
    const int node = gx + g.Nx * (gy + g.Ny * gz);
    const NodeCands nc = node_candidates(g, P, gx, gy, gz);
    const size_t NN = (size_t)g.Nn;
    const bool cl = g.clamp && clamped_node(g.clamp, gx, gy, gz, g);
    T acc[3] = {T(0), T(0), T(0)};
    if (!cl) {
        // fixed summation order (z, y, x candidates).  The loads of every existing candidate
        // are issued before the first sum, so that their latencies overlap; a candidate
        // that does not exist contributes zero.
        T v[8][3];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
#pragma unroll
            for (int c = 0; c < 3; ++c) v[k][c] = T(0);
            if (nc.v[0][kx] && nc.v[1][ky] && nc.v[2][kz]) {
                const int e = nc.e[0][kx] + g.nx * (nc.e[1][ky] + g.ny * nc.e[2][kz]);
                const int s = SK::index(nc.l[0][kx], nc.l[1][ky], nc.l[2][kz]);
#pragma unroll
                for (int c = 0; c < 3; ++c) v[k][c] = sk[SK::offset(e, c, s, g.NE)];
            }
        }
        // (an empty asm per value keeps the sums out of the branches above, which would
        // otherwise wait for each candidate's loads before issuing the next one's)
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

// Unstructured mesh: every non-interior node i sums its skeleton entries [ptr[i],
// ptr[i+1]) (its elements in ascending order) and writes y; a clamped node keeps its
// input in a constrained apply, a node of no element gets 0.
template <typename T>
__global__ void __launch_bounds__(256)
pa_uns_gather_kernel(const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ sk,
                     const int* __restrict__ ptr, const int* __restrict__ nodes, const int n_sk, const size_t NN,
                     const int constrained, const int add) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_sk) return;
    const unsigned v = (unsigned)nodes[i];
    const size_t node = v & ~kClampBit;
    T acc[3] = {T(0), T(0), T(0)};
    if (constrained && (v & kClampBit)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = x[c * NN + node];
    } else {
        const int b = ptr[i], e = ptr[i + 1];
        for (int k = b; k < e; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += sk[(size_t)k * 3 + c];
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T* yp = y + c * NN + node;
        *yp = add ? *yp + acc[c] : acc[c];
    }
}

template <int P, int Q, typename T, int MAT = kMatElemIso, int GEO = kGeoAffine, bool UNS = false, bool COL = false>
int launch_apply_tabs(const ApplyLaunch& L, const ApplyTabs<T, P + 1, Q, COL>& tab) {
    using C = ApplyCfg<P, Q, T>;
    if (L.g.NE == 0 && !UNS) return PA_OK;
    const int nb = (L.g.NE + C::E - 1) / C::E;
    if (nb > 0) {
        hipLaunchKernelGGL((pa_apply_kernel<P, Q, T, MAT, GEO, UNS, COL>), dim3(nb), dim3(C::NT), 0, L.stream,
                           (const T*)L.x, (T*)L.y, (T*)L.sk, (const T*)L.ed, tab, L.g, L.add, (const T*)L.md,
                           (const T*)L.gd, L.kmap, L.kpos);
        PA_HIP(hipGetLastError());
    }
    if constexpr (UNS) {
        if (L.n_sk > 0) {
            hipLaunchKernelGGL((pa_uns_gather_kernel<T>), dim3((L.n_sk + 255) / 256), dim3(256), 0, L.stream,
                               (const T*)L.x, (T*)L.y, (const T*)L.sk, L.sk_ptr, L.sk_node, L.n_sk,
                               (size_t)L.g.Nn, L.g.clamp != 0 ? 1 : 0, L.add);
            PA_HIP(hipGetLastError());
        }
        return PA_OK;
    }
    const SkelNodes sn = skel_nodes(L.g, P);
    const int nb2 = (sn.total + 255) / 256;
    hipLaunchKernelGGL((pa_skeleton_kernel<P, T>), dim3(nb2), dim3(256), 0, L.stream, (const T*)L.x, (T*)L.y,
                       (const T*)L.sk, L.g, sn, L.add);
    PA_HIP(hipGetLastError());
    return PA_OK;
}

template <int P, int Q, typename T, int MAT = kMatElemIso, int GEO = kGeoAffine, bool UNS = false>
int launch_apply_typed(const ApplyLaunch& L) {
    return launch_apply_tabs<P, Q, T, MAT, GEO, UNS>(L, make_tabs<T, P + 1, Q>(*L.tab));
}

// Per-point and anisotropic material forms (q = p + 2 only).
template <int P>
int launch_apply_material(const ApplyLaunch& L, int q_off, int dtype) {
    if (q_off != 1) return fail(PA_EUNSUPPORTED, "general material data is built for q = p + 2 only");
    if (dtype == PA_F64) {
        if (L.mat == PA_MAT_QP_ISO) return launch_apply_typed<P, P + 2, double, kMatQpIso>(L);
        return launch_apply_typed<P, P + 2, double, kMatAniso>(L);
    }
    if (L.mat == PA_MAT_QP_ISO) return launch_apply_typed<P, P + 2, float, kMatQpIso>(L);
    return launch_apply_typed<P, P + 2, float, kMatAniso>(L);
}

// Non-affine (trilinear) geometry forms (q = p + 2 only).
template <int P>
int launch_apply_geometry(const ApplyLaunch& L, int q_off, int dtype) {
    if (q_off != 1) return fail(PA_EUNSUPPORTED, "non-affine geometry is built for q = p + 2 only");
    if (L.mat != PA_MAT_ELEM_ISO) return fail(PA_EUNSUPPORTED, "non-affine geometry takes per-element Lame data");
    if (dtype == PA_F64) {
        if (L.geo == PA_GEOM_QP_DATA) return launch_apply_typed<P, P + 2, double, kMatElemIso, kGeoQp>(L);
        return launch_apply_typed<P, P + 2, double, kMatElemIso, kGeoTri>(L);
    }
    if (L.geo == PA_GEOM_QP_DATA) return launch_apply_typed<P, P + 2, float, kMatElemIso, kGeoQp>(L);
    return launch_apply_typed<P, P + 2, float, kMatElemIso, kGeoTri>(L);
}

// Unstructured meshes (q = p + 2, recomputed trilinear geometry).
template <int P>
int launch_apply_unstructured(const ApplyLaunch& L, int q_off, int dtype) {
    if (q_off != 1) return fail(PA_EUNSUPPORTED, "unstructured meshes are built for q = p + 2 only");
    if (dtype == PA_F64) return launch_apply_typed<P, P + 2, double, kMatElemIso, kGeoTri, true>(L);
    return launch_apply_typed<P, P + 2, float, kMatElemIso, kGeoTri, true>(L);
}

template <int P>
int launch_apply_p(const ApplyLaunch& L, int q_off, int dtype) {
    if (L.kmap) return launch_apply_unstructured<P>(L, q_off, dtype);
    if (L.geo != PA_GEOM_AFFINE) return launch_apply_geometry<P>(L, q_off, dtype);
    if (L.mat != PA_MAT_ELEM_ISO) return launch_apply_material<P>(L, q_off, dtype);
    if constexpr (kCollocated<P>) {
        // the sums of the requested rule (any q the tables were built for), collocated
        if (q_off < 0 || q_off > 2) return fail(PA_EUNSUPPORTED, "q = p+1+%d not built", q_off);
        constexpr bool EO = kEvenOdd<P + 1, P + 1>;
        if (dtype == PA_F64)
            return launch_apply_tabs<P, P + 1, double, kMatElemIso, kGeoAffine, false, EO>(
                L, make_colloc_tabs<double, P + 1>(*L.tab));
        return launch_apply_tabs<P, P + 1, float, kMatElemIso, kGeoAffine, false, EO>(
            L, make_colloc_tabs<float, P + 1>(*L.tab));
    }
    if (dtype == PA_F64) {
        switch (q_off) {
            case 0: return launch_apply_typed<P, P + 1, double>(L);
            case 1: return launch_apply_typed<P, P + 2, double>(L);
            case 2: return launch_apply_typed<P, P + 3, double>(L);
        }
    } else {
        switch (q_off) {
            case 0: return launch_apply_typed<P, P + 1, float>(L);
            case 1: return launch_apply_typed<P, P + 2, float>(L);
            case 2: return launch_apply_typed<P, P + 3, float>(L);
        }
    }
    return fail(PA_EUNSUPPORTED, "q = p+1+%d not built", q_off);
}

}  // namespace pa
