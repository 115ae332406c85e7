// Internal declarations of the gfx950 hyper-reduced RVE library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "hrom.h"

namespace hrom {

constexpr int kMaxModes = 96;   // m <= 96
constexpr int kGramChunk = 512; // ECM points per partial sum of the basis Gram matrix

// Per-point K-hat record.  FP64 path: the upper 16 x 16 accumulator tiles of
// the augmented contraction over Ghat = [G | I_9 | 0], MT (MT + 1) / 2 tiles of
// 256 entries.  Mixed path: the symmetric matrix [[Kaa, KaF], [KaF^T, KFF]] in
// the order the condensation reads it: indices 0..m-1 modes, 9 macro
// components at mp = 8 ceil(m / 8), lower 8 x 8 blocks (t >= u) in the order
// t (t + 1) / 2 + u, block entry (r, c) at 8 r + c; entries outside the modes
// and the macro components are not written.
__host__ __device__ inline int64_t khat_len(int m, int MT, bool mixed) {
    if (!mixed) return (int64_t)(MT * (MT + 1) / 2) * 256;
    const int MB = (m + 7) / 8 + 2;
    return (int64_t)(MB * (MB + 1) / 2) * 64;
}
constexpr int kMaxTiles = 7;    // ceil((96 + 10) / 16)
constexpr int kQChunk = 64;     // ECM points per phase-A chunk (one per lane)

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Three BF16 levels of an FP64 value: x = hi + mid + lo + O(2^-27 |x|), each
// level the round-to-nearest-even BF16 of what the levels before it leave
// (the remainders formed in FP64).  Products of two such splits keep the six
// level pairs (hh, hm, mh, hl, lh, mm) for FP32-level accuracy.
__device__ __forceinline__ uint16_t bf16_rne_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ void bf16_split3(double x, uint16_t lv[3]) {
    lv[0] = bf16_rne_bits((float)x);
    const double r1 = x - (double)__uint_as_float((uint32_t)lv[0] << 16);
    lv[1] = bf16_rne_bits((float)r1);
    const double r2 = r1 - (double)__uint_as_float((uint32_t)lv[1] << 16);
    lv[2] = bf16_rne_bits((float)r2);
}
__host__ __device__ inline int gb3_halves(int m) { return (m + 31) / 32; }

// Device-side description of one RVE cluster, in the layouts the kernels read.
struct ClusterDev {
    int m, Q, Qpad;        // Qpad: Q rounded up to a multiple of 64
    int MT, MP;            // column tiles of the augmented mode matrix, MP = 16 MT
    int res_t, res_c;      // tile / lane column holding the residual column m + 9
    int64_t first, count;
    int64_t off_a, off_kaa, off_kaf;   // offsets in caller mode-indexed arrays
    int64_t ws_khat;       // element offset of the cluster's tile workspace
    int64_t ws_L;          // element offset of the cluster's factor workspace
    int64_t ws_qs;         // element offset of the cluster's per-ECM-point scalars
    int64_t ws_hist;       // J2: element offset of the cluster's history [count][Qpad][8]
    int variant;           // launch variant of the tangent contraction (autotuned)
    int kin_variant;       // kinematics: 0 four, 1 eight wavefronts per 32-point workgroup
    int cond_variant;      // condensation: 0 three, 1 two wavefronts per SIMD (m <= 80)
    double* Ghat;          // [Qpad][9][MP]  augmented [G | I_9 | 0] (FP64)
    double* GT;            // [Qpad/64][9][m][64]  G, ECM point fastest (FP64)
    double* Gf;            // [9 Qpad/16][KS][64]  A-operand fragments of the kinematics GEMM
    int KS;                // 4 ceil(m / 16) k-steps of the kinematics GEMM (zero beyond m)
    double* w;             // [Qpad] (zero padded)
    int* phase;            // [Qpad]
    uint16_t* Fpk;         // [Qpad][MA][64][8] packed low-precision fragments of G (mixed path)
    uint32_t* Gb3;         // [9 Qpad/16][NH][3][64][4]  BF16 three-level A fragments of the
                           // mixed adjoint GEMM, NH = ceil(m / 32) halves of 32 modes (mixed path)
    // mode basis of the computation: Gram = R^T R of the caller's G in the
    // weighted gradient inner product, Gt = G R^{-1} (every layout above is
    // built from Gt), at = R a
    double* gram;          // [m][m]
    double* gram_part;     // [ceil(Q / kGramChunk)][m][m] partial sums of the Gram matrix
    double* R;             // [m][m] upper triangular
    double* Rinv;          // [m][m] upper triangular
    double* Gt;            // [Q][9][m]
    float* kscale;         // [1] inverse scaling of the low-precision w_q A_q of the last eval
};

struct ClusterGPU;
struct WorkItem;

constexpr size_t kArenaAlign = 256;   // alignment of every buffer carved from a plan's arena

struct Plan {
    // every device buffer of the plan except the grouped-launch tables below
    // is carved from one region: hipMalloc'ed at plan creation (owns_arena),
    // or a static device array for the allocation-free entry point
    char* arena = nullptr;
    size_t arena_bytes = 0;
    bool owns_arena = false;
    int ncl = 0;
    int64_t N = 0;
    int prec = HROM_FP64;
    unsigned flags = 0;
    int device = 0;
    // optional HIP events around the tangent contraction of hrom_eval
    bool profile = false;
    hipEvent_t ev_tan[2] = {nullptr, nullptr};
    std::vector<ClusterDev> cl;
    int64_t a_len = 0, kaa_len = 0, kaf_len = 0, x_len = 0;
    // per-point workspace
    double* Fr = nullptr;      // [9][N] RVE-frame deformation gradient
    double* polar = nullptr;   // [21][N] Fbar (9), eigenvectors V (9), stretches u (3)
    double* Pr = nullptr;      // [9][N]
    double* r = nullptr;       // mode-indexed [m][count] blocks
    void* Khat = nullptr;      // per-cluster tile blocks (double or float)
    void* qs = nullptr;        // per-cluster [count][Qpad][12] tangent scalars (double or float)
    double* L = nullptr;       // per-cluster [count][m][m] factor
    int* piv = nullptr;        // per-cluster [count][m] pivots (LU fallback)
    double* at = nullptr;      // mode-indexed: amplitudes in the plan's mode basis
    double* dt = nullptr;      // mode-indexed: update increment in the plan's mode basis
    int* basis_flag = nullptr; // set when a cluster's mode gradients are linearly dependent
    double* y = nullptr;       // mode-indexed
    double* X = nullptr;       // [9 m][count] blocks, offset 9*off_a
    double* Palg = nullptr;    // [9][N]
    double* Cr = nullptr;      // [81][N]
    double* S = nullptr;       // [9][N] second Piola stress of the push-out
    double* rnorm = nullptr;   // [N]
    double* dU = nullptr;      // [9][N] stretch increment scratch
    double* gr = nullptr;      // [9][N] backward: RVE-frame cotangent
    double* Lam = nullptr;     // [9][N] backward: Linv(sym(F^T g))
    double* lam = nullptr;     // mode-indexed: adjoint solution lambda
    double* rho = nullptr;     // mode-indexed: refinement residual
    int* conv = nullptr;       // [N]: adjoint refinement converged
    double* hr = nullptr;      // [9][N]
    double* gth = nullptr;     // [4][N] per-point theta gradients
    double* gth_part = nullptr;  // [4][kThetaChunks] partial sums of gth
    int64_t khat_len = 0, L_len = 0, qs_len = 0, hist_len = 0;
    bool j2 = false;           // J2 plasticity with history (FP64 plans)
    int nmac = 9;              // macro components condensed (6 with HROM_BIOT6)
    double* hist_n = nullptr;  // J2: committed history, per cluster [count][Qpad][8]
    double* hist_t = nullptr;  // J2: history of the last evaluation
    int stage = 0;             // 0 = nothing, 1 = evaluated, 2 = condensed
    // grouped launches (more than one cluster)
    bool grouped = false;
    int max_m = 0;
    ClusterGPU* cls_dev = nullptr;
    WorkItem* items_tan = nullptr;   // FP64 plans: 4-point tiles, decreasing cost
    int persistent_grid = 512;       // FP64 plans: workgroups of the persistent tangent launch
    int n_tan = 0;
    int* counter = nullptr;          // work-queue head of the persistent tangent launch (FP64)
};

// ---------------------------------------------------------------- kernels
struct PointArgs {
    int64_t N;
    int objective;
    const double* Fbar;
    double* Fr;
    double* polar;
    int* status;
};
void launch_prepare(const PointArgs& a, hipStream_t s);

struct EvalArgs {
    int m, Q, Qpad, MP, MT, KS;
    int64_t first, count, N;
    const double* Ghat;
    const double* Gf;      // kinematics-GEMM fragments [9 Qpad / 16][KS][64]
    const double* w;
    const int* phase;
    const uint16_t* Fpk;
    const double* theta;
    const double* Fr;
    const double* a;       // cluster block [m][count]
    void* qs;              // cluster block [count][Qpad][12] per-ECM-point tangent scalars
    void* Khat;            // cluster block [count][ntiles][256]
    double* r;             // cluster block [m][count]
    double* Pr;            // [9][N]
    int* status;           // [N]
    int qexp;              // ceil(log2 Q): the ECM-weight part of the mixed-mode scaling
    float* kscale_out;     // cluster's inverse scaling of w_q A_q (written by the kinematics)
    const double* hist_n;  // J2: committed state [count][Qpad][8] (cluster block)
    double* hist_t;        // J2: state of this evaluation [count][Qpad][8]
};
int launch_kin(int mixed, int j2, int variant, const EvalArgs& a, hipStream_t s);
int launch_eval_f64(int MT, int variant, int j2, const EvalArgs& a, hipStream_t s);
int launch_eval_mixed(int MT, int prec, bool split, int variant, int j2, const EvalArgs& a, hipStream_t s);

struct CondenseArgs {
    int m, MT, res_t, res_c;
    int mixed;
    int nmac;              // macro components condensed: 9, or 6 (symmetric stretch)
    int64_t first, count, N;
    const void* Khat;
    const double* r;       // cluster block
    const double* Pr;
    double* L;             // cluster block [count][m][m]
    int* piv;              // cluster block [count][m]
    double* y;             // cluster block [m][count]
    double* X;             // cluster block [nmac m][count]
    double* Palg;          // [9][N]
    double* Cr;            // [81][N]
    double* rnorm;         // [N]
    int* status;
    const float* kscale;   // device: inverse of the mixed-mode scaling of w_q A_q
    int variant;           // register condensation: 0 three, 1 two wavefronts per SIMD
    // optional exports (NULL = skip)
    double* outKaa;        // [m*m][count]
    double* outKaF;        // [m*9][count]
    double* outKFF;        // [81][N]
};
int launch_unpack_condense(const CondenseArgs& a, int mode, hipStream_t s);
int launch_condense_reg(const CondenseArgs& a, hipStream_t s);   // m <= 96

struct PushArgs {
    int64_t N;
    int objective;
    const double* polar;
    const double* Palg;
    const double* Cr;
    double* Pbar;
    double* Cbar;
    double* S;
    int* status;
};
void launch_pushout(const PushArgs& a, hipStream_t s);

struct CauchyArgs {
    int64_t N;
    const double* polar;
    const double* Palg;   // [9][N] RVE frame
    const double* Cr;     // [81][N] RVE frame
    double* sigma;        // [9][N]
    double* dsdD;         // [81][N] or null
    int* status;
};
void launch_cauchy(const CauchyArgs& a, hipStream_t s);

struct BiotArgs {
    int64_t N;
    const double* Palg;   // [9][N] RVE frame
    const double* Cr;     // [81][N] RVE frame
    double* T;            // [6][N] Biot stress (Voigt order 11 22 33 12 23 13)
    double* CB;           // [36][N] Biot tangent dT/dgamma (engineering shear), or null
    int* status;
};
void launch_biot(const BiotArgs& a, hipStream_t s);

struct UpdateArgs {
    int m;
    int64_t first, count, N;
    int objective;
    const double* dFbar;   // [9][N] or null
    const double* polar;
    double* dU;            // [9][N]
    const double* y;       // cluster block
    const double* X;       // cluster block [nmac m][count]
    int nmac;              // 9, or 6 (X holds the columns of the basis E6)
    const double* rnorm;
    const int* status;
    double tol;
    double* dt;            // cluster block: amplitude increment in the plan's mode basis
};
void launch_stretch_increment(const UpdateArgs& a, hipStream_t s);
void launch_update(const UpdateArgs& a, hipStream_t s);

struct BackwardArgs {
    int m, Q, Qpad, mixed, objective, with_rho;
    int64_t first, count, N;
    const double* GT;
    const double* Ghat;
    const double* Gf;
    const uint32_t* Gb3;   // mixed plans: BF16 three-level fragments of G
    int MP, MT, KS;
    const double* w;
    const int* phase;
    const double* theta;
    const double* Fr;
    const double* a;       // cluster block
    const double* lam;     // cluster block
    const double* gr;      // [9][N]
    double* hr;            // [9][N]
    double* gth;           // [4][N]
    double* rho;           // cluster block (refinement residual) or null
    int* status;
    const int* conv;       // refinement pass: cluster block [count]; workgroups whose points
                           // have all converged skip the pass
};
int launch_backward_b(const BackwardArgs& a, hipStream_t s);

struct BwPointArgs {
    int64_t N;
    int objective;
    const double* polar;
    const double* S;
    const double* g;
    double* gr;
    double* Lam;
    const double* hr;
    double* gF;
};
void launch_bw_pullback(const BwPointArgs& a, hipStream_t s);
void launch_bw_pushforward(const BwPointArgs& a, hipStream_t s);

struct LambdaArgs {
    int m;
    int64_t first, count, N;
    int nmac;              // 9, or 6 (X holds the columns of the basis E6)
    const double* X;       // cluster block [nmac m][count]
    const double* gr;      // [9][N]
    double* lam;           // cluster block [m][count]
    int* conv;             // cluster block [count] or null: cleared (refinement restarts)
};
void launch_lambda(const LambdaArgs& a, hipStream_t s);

struct RefineArgs {
    int m;
    int64_t first, count;
    const double* L;
    const int* piv;
    int* status;
    const double* rho;     // cluster block
    double* lam;           // cluster block, updated in place
    int* conv;             // cluster block [count]: 1 once the correction fell below tol
    double tol;            // stop when ||dlambda|| <= tol ||lambda||
    double flag_tol;       // after the last step: ||dlambda|| > flag_tol ||lambda|| flags the point
    int last;              // last allowed step
};
constexpr int kRefineSteps = 3;          // cap on adjoint refinement steps
constexpr double kRefineTol = 1e-6;      // stop: relative size of the last correction
constexpr double kRefineFlagTol = 1e-5;  // HROM_PT_NOREFINE above this after the last step
void launch_refine_lambda(const RefineArgs& a, hipStream_t s);

constexpr int kThetaChunks = 256;   // stage-1 partials per theta component
void launch_reduce_theta(int64_t N, const double* gth, double* part, double* out, hipStream_t s);
// J2 history [count][Qpad][8] -> [count][Q][7]
void launch_history_export(const double* src, int Q, int Qpad, int64_t count, double* out,
                           hipStream_t s);
void launch_mark_unconverged(int64_t N, const double* rnorm, double tol, int* status,
                             hipStream_t s);

// mode basis (k_basis.hip)
struct BasisArgs {
    int m, Q;
    const double* G;       // caller's [Q][9][m]
    const double* w;       // caller's [Q]
    double* gram;
    double* gram_part;     // [ceil(Q / kGramChunk)][m][m] partial Gram matrices
    double* R;
    double* Rinv;
    double* Gt;
    int* flag;
};
void launch_basis_build(const BasisArgs& a, hipStream_t s);
enum { MAP_R = 0, MAP_RT = 1, MAP_RINV = 2 };
struct ModeMapArgs {
    int m;
    int64_t first, count;
    const double* T;       // [m][m] (R or R^{-1})
    const double* x;       // cluster block [m][count]
    double* y;             // cluster block [m][count] (MAP_RINV: y -= T x), or null
    double* norm;          // [N] or null: ||T x||_2 per point
};
void launch_mode_map(int kind, const ModeMapArgs& a, hipStream_t s);
void launch_export_basis(const double* R, int m, int64_t count, double* Kaa, double* KaF,
                         hipStream_t s);
int set_basis_attributes();

// plan-time layout builders
struct LayoutArgs {
    int m, Q, Qpad, MT, MP, prec;
    const double* G;
    const double* w;
    const int* phase;
    double* Ghat;
    double* GT;
    double* Gf;
    int KS;
    double* wpad;
    int* phpad;
    uint16_t* Fpk;         // packed mixed-path fragments [Qpad][MA][64][8]
    uint32_t* Gb3;         // mixed adjoint GEMM fragments [9 Qpad/16][NH][3][64][4]
    int split;
};
void launch_build_layouts(const LayoutArgs& a, hipStream_t s);


// ---------------------------------------------------------------- grouped launches
// Several RVE clusters in one launch (the FP64 tangent contraction; every
// other step, and the mixed tangent, launch once per cluster, each at the
// occupancy its mode count allows): a kernel
// body runs on one work item (cluster c, tile `unit` of that cluster); the
// per-cluster constants live in a device array built at plan creation, the
// per-call pointers in GroupCall.
struct ClusterGPU {
    int m, Q, Qpad, MP, MT, KS;
    int64_t first, count, off_a, ws_qs, ws_khat, ws_L;
    const double* Ghat;
    const double* Gf;
    const double* w;
    const int* phase;
    const uint16_t* Fpk;
};

struct WorkItem {
    int c;      // cluster
    int unit;   // tile of the cluster (32 points for the kinematics and the
                // adjoint, 4 or 8 for the tangent contraction)
};

struct GroupCall {
    const ClusterGPU* cls;
    int ncl;
    const WorkItem* items;
    int nitems;
    int* counter;          // work-queue head of the persistent tangent kernel
    int64_t N;
    const double* theta;
    const double* Fr;
    const double* a;
    void* qs;
    void* Khat;
    double* r;
    double* Pr;
    int* status;
};

int launch_tan_persistent(const GroupCall& g, int grid, hipStream_t s);   // FP64
void set_kernel_attributes();

// the r leading left singular vectors of xf^T (xf [P][M] rows) into lam with
// row stride ld, all singular values into sigma (one-sided block Jacobi of the
// empirical cubature, shared by the POD of the clustered training); method 0:
// Householder QR first for tall matrices (M >= 2 Ppad), 1: the sweeps on xf^T
// itself, 2: QR first (M >= Ppad)
int svd_left(int P, int M, const double* xf, int r, double* lam, int ld, double* sigma, double tol,
             int max_sweeps, int* sweeps, double* off_hist, int method, hipStream_t stream);

}  // namespace hrom
