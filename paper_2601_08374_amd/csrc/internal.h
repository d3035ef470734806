// Internal declarations of the paelast HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "paelast.h"

namespace pa {

constexpr int kMaxP = 8;
constexpr int kMaxD = kMaxP + 1;
constexpr int kMaxQ = kMaxP + 3;
constexpr int kEdStride = 12;   // words of per-element PA data: J^{-1} (9), detJ*lambda, detJ*mu, pad

// Thread-local error message; returns `code` for convenient `return fail(...)`.
int fail(int code, const char* fmt, ...);

#define PA_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t _e = (call);                                                      \
        if (_e != hipSuccess) return ::pa::fail(PA_EHIP, "%s failed: %s", #call,   \
                                                hipGetErrorString(_e));             \
    } while (0)

// Host copy of the 1D tables on [0,1]: B[i*q+k] = l_i(x_k), G[i*q+k] = l_i'(x_k), w[k].
struct Tables {
    int p = 0, q = 0;
    double gll[kMaxD];
    double xq[kMaxQ];
    double B[kMaxD * kMaxQ];
    double G[kMaxD * kMaxQ];
    double w[kMaxQ];
};

struct MeshDesc {
    int n[3] = {0, 0, 0};
    double A[9];
    double x0[3];
    uint32_t clamp = 0;
    std::vector<double> vert[3];   // vertex coordinates per axis (n[a]+1)
};

// Geometry of one operator as the kernels see it.
struct Geom {
    int nx, ny, nz;     // elements per axis
    int Nx, Ny, Nz;     // nodes per axis (n*p+1)
    int Nn;             // nodes
    int NE;             // elements
    uint32_t clamp;     // clamped-face mask (0: unconstrained)
};

struct ApplyLaunch {
    Geom g;
    const void* x;
    void* y;
    void* sk;            // skeleton buffer of the operator (element-boundary contributions)
    const void* ed;      // per-element data of the launch dtype
    int mat = PA_MAT_ELEM_ISO;   // PA_MAT_* form of the material data
    const void* md = nullptr;   // per-point Lame parameters or anisotropic stiffness (mat != PA_MAT_ELEM_ISO)
    int geo = PA_GEOM_AFFINE;   // PA_GEOM_* form of the element geometry
    const void* gd = nullptr;   // per-point J^{-1}, w det J or trilinear coefficients (geo != PA_GEOM_AFFINE)
    // unstructured mesh (kmap != nullptr): element-to-node map and skeleton gather lists
    const int* kmap = nullptr;     // [NE][D^3] global node | kClampBit
    const int* sk_ptr = nullptr;   // [n_sk + 1] CSR offsets: node i owns skeleton entries [ptr[i], ptr[i+1])
    const int* kpos = nullptr;     // [NE][S] skeleton entry of (element, slot); entry k holds words 3k..3k+2
    const int* sk_node = nullptr;  // [n_sk] global node | kClampBit of every non-interior node
    int n_sk = 0;
    const Tables* tab;
    int add;             // accumulate into y (y pre-initialised by the caller)
    bool lin = false;    // p = 1: the linear-element kernel (the operator's skeleton buffer is sized for it)
    hipStream_t stream;
};

// Fused apply launchers, one translation unit per degree p.  q_off = q - p - 1.
int launch_apply_p1(const ApplyLaunch&, int q_off, int dtype);
int launch_apply_p2(const ApplyLaunch&, int q_off, int dtype);
int launch_apply_p3(const ApplyLaunch&, int q_off, int dtype);
int launch_apply_p4(const ApplyLaunch&, int q_off, int dtype);
int launch_apply_p5(const ApplyLaunch&, int q_off, int dtype);
int launch_apply_p6(const ApplyLaunch&, int q_off, int dtype);
int launch_apply_p7(const ApplyLaunch&, int q_off, int dtype);
int launch_apply_p8(const ApplyLaunch&, int q_off, int dtype);

// Linear elements (p = 1) run a register-resident kernel in which one wavefront
// covers kLinTX x kLinTY element columns and each lane walks a chunk of lin_chunk()
// elements up its column; only nodes on the faces of such tiles go through the
// skeleton buffer.
constexpr int kLinTX = 8, kLinTY = 8;
// Wavefronts the GPU holds at once for that kernel: 256 CUs x 4 SIMDs x the waves per SIMD
// its registers allow -- four for per-element data in single precision, two otherwise.
inline int lin_wave_slots(int dtype, bool point_data) { return dtype == PA_F32 && !point_data ? 4096 : 2048; }

// z-chunk length for an n[0] x n[1] x n[2] mesh: the smallest length with which all
// (column tile, z-chunk) wavefronts are resident at once -- one round of waves, no tail.
// Small meshes get short chunks (down to one element), so that more wavefronts share the
// work; large ones as few tile faces across z as fill the GPU once.
inline int lin_chunk(const int n[3], int slots) {
    const int64_t nxy = (int64_t)((n[0] + kLinTX - 1) / kLinTX) * ((n[1] + kLinTY - 1) / kLinTY);
    int L = 1;
    while (L < n[2] && nxy * ((n[2] + L - 1) / L) > slots) ++L;
    return L;
}

// Which kernel a p = 1 operator runs: the sum-factorized kernel (kLinNever), the linear-element
// kernel (kLinAlways: per-point Lame data, stored point-major for it), or the linear-element
// kernel on meshes of more than kLinSmallMesh elements (kLinBySize).  The linear-element kernel
// walks each lane's chunk of elements in sequence, which on small meshes leaves most of the GPU
// idle; there the sum-factorized kernel, which spreads an element over nine lanes, is faster
// (measured crossover between 32^3 and 48^3 elements).
enum : int { kLinNever = 0, kLinBySize = 1, kLinAlways = 2 };
constexpr int64_t kLinSmallMesh = 32768;
inline bool p1_runs_lin(const int n[3], int lin_mode) {
    const int64_t NE = (int64_t)n[0] * n[1] * n[2];
    return lin_mode == kLinAlways || (lin_mode == kLinBySize && NE > kLinSmallMesh);
}

// Words per tile and component of the linear-element skeleton buffer: the tile's
// boundary nodes in three face arrays, each contiguous along its face (x faces
// [2][tz+1][TY+1], y faces [2][tz+1][TX+1], z faces [2][TY+1][TX+1]).
constexpr int64_t lin_face_words(int tz) {
    return 2 * (int64_t)(tz + 1) * (kLinTY + 1) + 2 * (int64_t)(tz + 1) * (kLinTX + 1) +
           2 * (int64_t)(kLinTY + 1) * (kLinTX + 1);
}

inline int64_t lin_tiles(const int n[3], int tz) {
    return (int64_t)((n[0] + kLinTX - 1) / kLinTX) * ((n[1] + kLinTY - 1) / kLinTY) * ((n[2] + tz - 1) / tz);
}

// Words of the skeleton buffer of one operator: per element, 3 components x its
// element-boundary nodes; for the linear-element kernel (p = 1, see p1_runs_lin),
// 3 components x the face nodes of every tile.
inline int64_t skeleton_words(int p, const int n[3], int lin_mode, int dtype) {
    if (p == 1 && p1_runs_lin(n, lin_mode)) {
        const int tz = lin_chunk(n, lin_wave_slots(dtype, lin_mode == kLinAlways));
        return lin_tiles(n, tz) * 3 * lin_face_words(tz);
    }
    const int64_t NE = (int64_t)n[0] * n[1] * n[2];
    const int64_t D = p + 1;
    return NE * 3 * (D * D * D - (D - 2) * (D - 2) * (D - 2));
}

// Work arrays of the unfused apply variants (ablation.hip), allocated on first use.
struct AblationBuffers;
void free_ablation(AblationBuffers* b);

// Clamped-node flag in the element-to-node map of an unstructured mesh.
constexpr unsigned kClampBit = 0x80000000u;

inline Geom make_geom(const MeshDesc& m, int p, bool constrained) {
    Geom g;
    g.nx = m.n[0]; g.ny = m.n[1]; g.nz = m.n[2];
    g.Nx = g.nx * p + 1; g.Ny = g.ny * p + 1; g.Nz = g.nz * p + 1;
    g.Nn = g.Nx * g.Ny * g.Nz;
    g.NE = g.nx * g.ny * g.nz;
    g.clamp = constrained ? m.clamp : 0u;
    return g;
}

}  // namespace pa

// Opaque handles of the C ABI.
struct pa_op {
    pa::MeshDesc mesh;
    int p = 0, q = 0, dtype = PA_F64;
    int64_t NE = 0, Nn = 0, N = 0;
    hipStream_t stream = nullptr;
    std::vector<double> lam, mu;     // host copies (used to build solver hierarchies)
    void* ed = nullptr;              // device per-element data [NE][kEdStride] of dtype
    void* sk = nullptr;              // skeleton buffer (skeleton_words) of dtype used by every apply
    size_t sk_bytes = 0;             // its size
    int device = 0;                  // HIP device that holds the operator's memory
    double* d_tab = nullptr;         // device copy of the FP64 tables (B, G, w, bb/bg/gg, sB)
    double* d_vert = nullptr;        // device vertex coordinates, x | y | z
    pa::Tables tab;                  // host copy of the tables (kernel arguments)
    pa_gmg* cached = nullptr;        // hierarchy cached by gmg_pcg_solve
    pa::AblationBuffers* abl = nullptr;   // pa_elast_apply_variant work arrays
    int mat = PA_MAT_ELEM_ISO;       // material data form
    void* md = nullptr;              // device material data of dtype (PA_MAT_QP_ISO, PA_MAT_ANISO)
    bool md_point_major = false;     // md word k of point alpha of element e at (2 alpha + k) NE + e
    bool lin = false;                // p = 1: applies run the linear-element kernel
    std::vector<double> mdata;       // host copy of per-point Lame data [NE][q^3][2] (solver hierarchies)
    int geo = PA_GEOM_AFFINE;        // element geometry form
    void* gd = nullptr;              // device geometry data of dtype (PA_GEOM_QP_DATA, PA_GEOM_TRILINEAR)
    // unstructured mesh (pa_elast_setup_unstructured); kmap == nullptr on the box
    int* kmap = nullptr;             // device [NE][D^3] global node | kClampBit
    int* sk_ptr = nullptr;           // device CSR over the non-interior nodes
    int* kpos = nullptr;
    int* sk_node = nullptr;
    int n_sk = 0;
    pa_solve_opts_t cached_opts;
};
