// Mode basis of the computation.  The ROM amplitudes enter the RVE only
// through the span of the mode gradients (Sec. 3.2.1, eq. ROM_assumption), so
// the condensed stress and tangent do not depend on the basis chosen for that
// span.  Every plan works in the basis that is orthonormal in the weighted
// gradient inner product <G_i, G_j> = sum_q w_q G_qi : G_qj:
//   Gram = R^T R (Cholesky, R upper triangular),  Gt = G R^{-1},  at = R a.
// The low-precision contraction then sees well-scaled operands whatever the
// caller's basis (an ill-conditioned basis would otherwise amplify the
// rounding of G into the span), and the FP64 path is unchanged up to
// rounding.  Caller-side arrays stay in the caller's basis: a is mapped in
// (at = R a), the update is mapped out (a -= R^{-1} dt), the residual norm
// and the optional r, Kaa, KaF outputs are taken back with R^T.
#include <hip/hip_runtime.h>

#include "hrom_internal.h"

namespace hrom {

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Gram[i][j] = sum_q w_q sum_I G[q][I][i] G[q][I][j]: partial sums over
// chunks of kGramChunk ECM points (blockIdx.y), one thread per (i, j), then
// the chunks summed in order, so the summation order is fixed
__global__ void __launch_bounds__(256) k_gram_part(const double* G, const double* w, int m, int Q,
                                                   double* part) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * m) return;
    const int i = t / m, j = t % m;
    const int q0 = blockIdx.y * kGramChunk, q1 = min(Q, q0 + kGramChunk);
    double s = 0.0;
    for (int q = q0; q < q1; q++) {
        double sq = 0.0;
#pragma unroll
        for (int I = 0; I < 9; I++)
            sq = fma(G[((int64_t)q * 9 + I) * m + i], G[((int64_t)q * 9 + I) * m + j], sq);
        s = fma(w[q], sq, s);
    }
    part[(int64_t)blockIdx.y * m * m + t] = s;
}

__global__ void __launch_bounds__(256) k_gram_sum(const double* part, int mm, int nchunk, double* gram) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mm) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; c++) s += part[(int64_t)c * mm + t];
    gram[t] = s;
}

// One workgroup: Cholesky Gram = R^T R in LDS (right-looking, column by
// column), then R^{-1} by back substitution of the identity, column k per
// thread.  A pivot at or below 1e-13 of the largest diagonal entry (mode
// gradients linearly dependent in the weighted inner product) sets *flag = 1
// and leaves R, R^{-1} as NaN, so that every later use flags its points.
__global__ void __launch_bounds__(256) k_basis_factor(const double* gram, int m, double* R,
                                                      double* Rinv, int* flag) {
    extern __shared__ double sm[];
    double* A = sm;               // [m][m], upper triangle becomes R
    int& bad = *reinterpret_cast<int*>(sm + m * m);
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    for (int e = t; e < m * m; e += blockDim.x) A[e] = gram[e];
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < m; i++) dmax = fmax(dmax, A[i * m + i]);
    for (int j = 0; j < m; j++) {
        const double d = A[j * m + j];
        if (!(d > 1e-13 * dmax)) {
            if (t == 0) bad = 1;
            break;
        }
        const double rjj = sqrt(d);
        __syncthreads();
        // row j of R: R_jk = A_jk / r_jj for k > j
        for (int k = j + 1 + t; k < m; k += blockDim.x) A[j * m + k] /= rjj;
        __syncthreads();
        if (t == 0) A[j * m + j] = rjj;
        // trailing update of the upper triangle: A_ik -= R_ji R_jk, i <= k
        for (int e = t; e < (m - j - 1) * (m - j - 1); e += blockDim.x) {
            const int i = j + 1 + e / (m - j - 1), k = j + 1 + e % (m - j - 1);
            if (k >= i) A[i * m + k] = fma(-A[j * m + i], A[j * m + k], A[i * m + k]);
        }
        __syncthreads();
    }
    __syncthreads();
    const bool ok = bad == 0;
    if (t == 0 && !ok) *flag = 1;
    for (int e = t; e < m * m; e += blockDim.x) {
        const int i = e / m, k = e % m;
        R[e] = ok ? (k >= i ? A[e] : 0.0) : __builtin_nan("");
    }
    // R^{-1}: column k solves R x = e_k, x_i = 0 for i > k
    for (int k = t; k < m; k += blockDim.x) {
        for (int i = m - 1; i >= 0; i--) {
            double v = 0.0;
            if (i <= k) {
                double s = (i == k) ? 1.0 : 0.0;
                for (int j = i + 1; j <= k; j++) s = fma(-A[i * m + j], Rinv[j * m + k], s);
                v = s / A[i * m + i];
            }
            Rinv[i * m + k] = ok ? v : __builtin_nan("");
        }
    }
}

// Gt[q][I][n] = sum_{j <= n} G[q][I][j] Rinv[j][n]
__global__ void __launch_bounds__(256) k_basis_apply(const double* G, const double* Rinv, int m,
                                                     int Q, double* Gt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)Q * 9 * m) return;
    const int n = (int)(t % m);
    const int64_t row = t / m;
    double s = 0.0;
    for (int j = 0; j <= n; j++) s = fma(G[row * m + j], Rinv[(int64_t)j * m + n], s);
    Gt[t] = s;
}

void launch_basis_build(const BasisArgs& a, hipStream_t s) {
    const int nchunk = (a.Q + kGramChunk - 1) / kGramChunk;
    hipLaunchKernelGGL(k_gram_part, dim3(nblocks((int64_t)a.m * a.m, 256), nchunk), dim3(256), 0, s, a.G, a.w,
                       a.m, a.Q, a.gram_part);
    hipLaunchKernelGGL(k_gram_sum, dim3(nblocks((int64_t)a.m * a.m, 256)), dim3(256), 0, s,
                       (const double*)a.gram_part, a.m * a.m, nchunk, a.gram);
    const size_t lds = sizeof(double) * ((size_t)a.m * a.m + 1);
    hipLaunchKernelGGL(k_basis_factor, dim3(1), dim3(256), lds, s, (const double*)a.gram, a.m, a.R,
                       a.Rinv, a.flag);
    hipLaunchKernelGGL(k_basis_apply, dim3(nblocks((int64_t)a.Q * 9 * a.m, 256)), dim3(256), 0, s,
                       a.G, (const double*)a.Rinv, a.m, a.Q, a.Gt);
}

// ---------------------------------------------------------------- per-point maps
// y = T x for every macro point of a cluster, with T one of
//   MAP_R    (R, upper):          at = R a
//   MAP_RT   (R^T, lower):        r = R^T rt (optionally only ||r||_2)
//   MAP_RINV (R^{-1}, upper):     a -= R^{-1} dt
// as an FP64 MFMA GEMM: workgroup = 64 points, wavefront w = points
// 16 w .. 16 w + 15, every 16-row tile of T against them (16x16x4 MFMA: lane
// (g, c) holds T[16 t + c][4 kb + g] and x[4 kb + g][16 w + c], accumulator
// element e is row 16 t + g + 4 e, point 16 w + c); the k-steps left of an
// upper tile's diagonal (right of a lower tile's) are zero and skipped.  The
// norm sums each lane's squares, then the four lane groups in a fixed order.
template <int KIND, int MA>
__global__ void __launch_bounds__(256) k_mode_map(ModeMapArgs A) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int m = A.m;
    const int64_t p = (int64_t)blockIdx.x * 64 + 16 * wave + c;   // this lane's point (B, D)
    const bool live = p < A.count;
    constexpr int KB = 4 * MA;   // k-steps over the padded modes
    v4d acc[MA];
#pragma unroll
    for (int t = 0; t < MA; t++) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < KB; kb++) {
        const int k = 4 * kb + g;
        const double bx = (live && k < m) ? A.x[(int64_t)k * A.count + p] : 0.0;
#pragma unroll
        for (int t = 0; t < MA; t++) {
            // upper T: tile t has nonzeros only for k >= 16 t; lower: k <= 16 t + 15
            const bool used = (KIND == MAP_RT) ? (4 * kb <= 16 * t + 15) : (4 * kb + 3 >= 16 * t);
            if (used) {
                const int i = 16 * t + c;
                double av = 0.0;
                if (i < m && k < m) av = (KIND == MAP_RT) ? A.T[(int64_t)k * m + i] : A.T[(int64_t)i * m + k];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bx, acc[t], 0, 0, 0);
            }
        }
    }
    double nrm = 0.0;
#pragma unroll
    for (int t = 0; t < MA; t++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int i = 16 * t + g + 4 * e;
            const double v = acc[t][e];
            if (i < m && live) {
                const int64_t o = (int64_t)i * A.count + p;
                if (KIND == MAP_RINV) A.y[o] -= v;
                else if (A.y) A.y[o] = v;
            }
            nrm = fma(v, v, nrm);
        }
    if (A.norm) {
        nrm += __shfl_xor(nrm, 16);
        nrm += __shfl_xor(nrm, 32);
        if (g == 0 && live) A.norm[A.first + p] = sqrt(nrm);
    }
}

template <int KIND>
static void launch_map_t(const ModeMapArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(a.count, 64)), block(256);
    switch ((a.m + 15) / 16) {
        case 1: hipLaunchKernelGGL((k_mode_map<KIND, 1>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_mode_map<KIND, 2>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_mode_map<KIND, 3>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_mode_map<KIND, 4>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_mode_map<KIND, 5>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((k_mode_map<KIND, 6>), grid, block, 0, s, a); break;
    }
}

void launch_mode_map(int kind, const ModeMapArgs& a, hipStream_t s) {
    if (kind == MAP_R) launch_map_t<MAP_R>(a, s);
    else if (kind == MAP_RT) launch_map_t<MAP_RT>(a, s);
    else launch_map_t<MAP_RINV>(a, s);
}

// Exported blocks back to the caller's basis, one workgroup per macro point:
// Kaa <- R^T Kt R, KaF <- R^T KaFt (in place, layouts [m*m][count], [m*9][count]).
__global__ void __launch_bounds__(256) k_export_basis(const double* R, int m, int64_t count,
                                                      double* Kaa, double* KaF) {
    extern __shared__ double sm[];
    double* K = sm;            // [m][m]
    double* Z = sm + m * m;    // [m][m] = Kt R, then scratch for KaF
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    if (Kaa) {
        for (int e = t; e < m * m; e += blockDim.x) K[e] = Kaa[(int64_t)e * count + p];
        __syncthreads();
        for (int e = t; e < m * m; e += blockDim.x) {
            const int i = e / m, k = e % m;
            double s = 0.0;
            for (int j = 0; j <= k; j++) s = fma(K[i * m + j], R[(int64_t)j * m + k], s);
            Z[e] = s;
        }
        __syncthreads();
        for (int e = t; e < m * m; e += blockDim.x) {
            const int i = e / m, k = e % m;
            double s = 0.0;
            for (int j = 0; j <= i; j++) s = fma(R[(int64_t)j * m + i], Z[j * m + k], s);
            Kaa[(int64_t)e * count + p] = s;
        }
        __syncthreads();
    }
    if (KaF) {
        for (int e = t; e < m * 9; e += blockDim.x) Z[e] = KaF[(int64_t)e * count + p];
        __syncthreads();
        for (int e = t; e < m * 9; e += blockDim.x) {
            const int i = e / 9, J = e % 9;
            double s = 0.0;
            for (int j = 0; j <= i; j++) s = fma(R[(int64_t)j * m + i], Z[j * 9 + J], s);
            KaF[(int64_t)e * count + p] = s;
        }
    }
}

void launch_export_basis(const double* R, int m, int64_t count, double* Kaa, double* KaF,
                         hipStream_t s) {
    if (!Kaa && !KaF) return;
    const size_t lds = sizeof(double) * 2 * (size_t)m * m + sizeof(double) * 9 * m;
    hipLaunchKernelGGL(k_export_basis, dim3((unsigned)count), dim3(256), lds, s, R, m, count, Kaa,
                       KaF);
}

int set_basis_attributes() {
    const int m = kMaxModes;
    const int lim_exp = (int)(sizeof(double) * (2 * m * m + 9 * m));
    const int lim_fac = (int)(sizeof(double) * (m * m + 1));
    if (hipFuncSetAttribute((const void*)k_export_basis, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim_exp) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_basis_factor, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim_fac) != hipSuccess)
        return HROM_E_HIP;
    return HROM_OK;
}

}  // namespace hrom
