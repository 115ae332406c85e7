// Clustered training (Sec. 3.4, Box 2) and the POD basis with the
// elastic-inelastic split (Sec. 3.2.1, eqs. SVD_displacement and
// snapshots_displacement).
//
//  * hrom_training_clusters: the macro strain states scaled per component by
//    their root mean square, then Lloyd's k-means: a thread per point finds
//    its nearest centre (the centres in LDS) and counts changed labels; per
//    chunk of 1024 points a thread per centre sums the centre's points in
//    order, and the chunk partials are added in chunk order (every run gives
//    the same bits); the host loop stops when no label changes.
//  * hrom_training_paths: monotonic trajectories Fr = I + t H(c).
//  * hrom_pod: the elastic modes from the snapshots' left singular vectors,
//    the inelastic snapshots without their part in the elastic span, their
//    leading left singular vectors appended (the one-sided Jacobi of the
//    empirical cubature).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "hrom.h"
#include "hrom_internal.h"

namespace hrom {
namespace trn {

constexpr int kMaxD = 8;        // features per point
constexpr int kMaxK = 1024;     // centres

__device__ double block_sum256(double s, double* red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

// per component: the root mean square over the points (1 where it is zero)
__global__ void __launch_bounds__(256) k_rms(const double* E, int64_t N, double* scale) {
    __shared__ double red[4];
    const double* e = E + (int64_t)blockIdx.x * N;
    double s = 0.0;
    for (int64_t g = threadIdx.x; g < N; g += 256) s += e[g] * e[g];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) {
        const double v = sqrt(s / (double)N);
        scale[blockIdx.x] = v > 0.0 ? v : 1.0;
    }
}

__global__ void k_km_init(const double* E, int64_t N, int d, int k, const int32_t* idx, const double* scale,
                          double* C) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * d) return;
    const int c = e / d, j = e % d;
    C[e] = E[(int64_t)j * N + idx[c]] / scale[j];
}

// nearest centre of every point (ties: the lowest index); counts changes
__global__ void __launch_bounds__(256) k_km_assign(const double* E, int64_t N, int d, int k, const double* scale,
                                                   const double* C, int32_t* labels, int* changed) {
    extern __shared__ double sC[];   // k d centres
    for (int e = threadIdx.x; e < k * d; e += 256) sC[e] = C[e];
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int ch = 0;
    if (g < N) {
        double x[kMaxD];
#pragma unroll
        for (int j = 0; j < kMaxD; j++) x[j] = (j < d) ? E[(int64_t)j * N + g] / scale[j] : 0.0;
        double best = INFINITY;
        int bi = 0;
        for (int c = 0; c < k; c++) {
            double d2 = 0.0;
#pragma unroll
            for (int j = 0; j < kMaxD; j++)
                if (j < d) {
                    const double t = x[j] - sC[c * d + j];
                    d2 += t * t;
                }
            if (d2 < best) {
                best = d2;
                bi = c;
            }
        }
        ch = (labels[g] != bi) ? 1 : 0;
        labels[g] = bi;
    }
    // one atomic per wavefront
    const unsigned long long bal = __ballot(ch);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(changed, __popcll(bal));
}

constexpr int kChunk = 1024;     // points per workgroup of the centre update

// per chunk of 1024 points and per centre: the sum of the centre's points
// (normalised) and their count, a thread per centre scanning the chunk in
// order from LDS (the same bits on every run)
__global__ void __launch_bounds__(256) k_km_partial(const double* E, int64_t N, int d, int k, const double* scale,
                                                    const int32_t* labels, double* part) {
    __shared__ int sl[kChunk];
    __shared__ double sx[kMaxD][kChunk];
    const int64_t g0 = (int64_t)blockIdx.x * kChunk;
    const int n = (int)min((int64_t)kChunk, N - g0);
    for (int i = threadIdx.x; i < kChunk; i += 256) {
        sl[i] = (i < n) ? labels[g0 + i] : -1;
        for (int j = 0; j < d; j++) sx[j][i] = (i < n) ? E[(int64_t)j * N + g0 + i] / scale[j] : 0.0;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += 256) {
        double acc[kMaxD];
#pragma unroll
        for (int j = 0; j < kMaxD; j++) acc[j] = 0.0;
        double cnt = 0.0;
        for (int i = 0; i < n; i++) {
            if (sl[i] != c) continue;
            cnt += 1.0;
#pragma unroll
            for (int j = 0; j < kMaxD; j++)
                if (j < d) acc[j] += sx[j][i];
        }
        double* out = part + ((int64_t)blockIdx.x * k + c) * (d + 1);
        for (int j = 0; j < d; j++) out[j] = acc[j];
        out[d] = cnt;
    }
}

// centre c = mean of its points from the chunk partials in chunk order (a
// centre without points stays)
__global__ void k_km_reduce(const double* part, int nchunks, int k, int d, double* C) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * d) return;
    const int c = e / d, j = e % d;
    double s = 0.0, n = 0.0;
    for (int b = 0; b < nchunks; b++) {
        const double* p = part + ((int64_t)b * k + c) * (d + 1);
        s += p[j];
        n += p[d];
    }
    if (n > 0.0) C[e] = s / n;
}

__global__ void k_km_out(const double* C, int k, int d, const double* scale, double* out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < k * d) out[e] = C[e] * scale[e % d];
}

__global__ void k_paths(const double* C, int k, int n_steps, double* Fr) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * n_steps) return;
    const int c = e / n_steps, j = e % n_steps;
    const double t = (double)(j + 1) / (double)n_steps;
    const double* h = C + 6 * c;
    const double H[9] = {h[0], h[3], h[5], h[3], h[1], h[4], h[5], h[4], h[2]};
#pragma unroll
    for (int I = 0; I < 9; I++) Fr[9 * (int64_t)e + I] = ((I % 4 == 0) ? 1.0 : 0.0) + t * H[I];
}

// coefficients of the inelastic snapshots on the elastic modes:
// coef[j][e] = sum_g X[j][g] Phi[g][e] (a workgroup per snapshot)
__global__ void __launch_bounds__(256) k_pod_coef(const double* X, int64_t nd, const double* Phi, int ld,
                                                  int n_el, double* coef) {
    __shared__ double red[4];
    const double* x = X + (int64_t)blockIdx.x * nd;
    for (int e = 0; e < n_el; e++) {
        double s = 0.0;
        for (int64_t g = threadIdx.x; g < nd; g += 256) s += x[g] * Phi[g * ld + e];
        s = block_sum256(s, red);
        if (threadIdx.x == 0) coef[(int64_t)blockIdx.x * n_el + e] = s;
    }
}

// X_mod[j][g] = X[j][g] - sum_e coef[j][e] Phi[g][e]
__global__ void k_pod_sub(const double* X, int64_t nd, int s_in, const double* Phi, int ld, int n_el,
                          const double* coef, double* Xm) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)s_in * nd) return;
    const int64_t j = e / nd, g = e % nd;
    double s = 0.0;
    for (int q = 0; q < n_el; q++) s += coef[j * n_el + q] * Phi[g * ld + q];
    Xm[e] = X[e] - s;
}

}  // namespace trn
}  // namespace hrom

using namespace hrom;
using namespace hrom::trn;

extern "C" {

int hrom_training_clusters(int64_t N, int32_t d, const double* E, int32_t k, const int32_t* init_idx,
                           int32_t max_iter, double* centres, int32_t* labels, int32_t* iters,
                           hipStream_t stream) {
    if (N < 1 || d < 1 || d > kMaxD || k < 1 || k > kMaxK || k > N || max_iter < 1 || !E || !init_idx ||
        !centres || !labels)
        return HROM_E_INVALID;
    double *scale = nullptr, *C = nullptr, *part = nullptr;
    int* changed = nullptr;
    const int nchunks = (int)((N + kChunk - 1) / kChunk);
    if (hipMalloc((void**)&scale, sizeof(double) * d) != hipSuccess) return HROM_E_NOMEM;
    if (hipMalloc((void**)&C, sizeof(double) * k * d) != hipSuccess ||
        hipMalloc((void**)&changed, sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&part, sizeof(double) * (size_t)nchunks * k * (d + 1)) != hipSuccess) {
        (void)hipFree(scale);
        (void)hipFree(C);
        (void)hipFree(changed);
        return HROM_E_NOMEM;
    }
    int rc = HROM_OK, it = 0, hch = 1;
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_rms, dim3(d), dim3(256), 0, stream, E, N, scale);
    hipLaunchKernelGGL(k_km_init, dim3((k * d + 255) / 256), dim3(256), 0, stream, E, N, d, k, init_idx, scale, C);
    if (hipMemsetAsync(labels, 0xff, sizeof(int32_t) * N, stream) != hipSuccess) rc = HROM_E_HIP;
    while (rc == HROM_OK && it < max_iter && hch != 0) {
        if (hipMemsetAsync(changed, 0, sizeof(int), stream) != hipSuccess) {
            rc = HROM_E_HIP;
            break;
        }
        hipLaunchKernelGGL(k_km_assign, dim3(nb), dim3(256), sizeof(double) * k * d, stream, E, N, d, k, scale, C,
                           labels, changed);
        hipLaunchKernelGGL(k_km_partial, dim3(nchunks), dim3(256), 0, stream, E, N, d, k, scale, labels, part);
        hipLaunchKernelGGL(k_km_reduce, dim3((k * d + 255) / 256), dim3(256), 0, stream, part, nchunks, k, d, C);
        it++;
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&hch, changed, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            rc = HROM_E_HIP;
    }
    if (rc == HROM_OK) {
        hipLaunchKernelGGL(k_km_out, dim3((k * d + 255) / 256), dim3(256), 0, stream, C, k, d, scale, centres);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) rc = HROM_E_HIP;
    }
    (void)hipFree(scale);
    (void)hipFree(C);
    (void)hipFree(changed);
    (void)hipFree(part);
    if (iters) *iters = it;
    if (rc == HROM_OK && hch != 0) rc = HROM_E_NOCONV;
    return rc;
}

int hrom_training_paths(int32_t k, const double* centres, int32_t n_steps, double* Fr, hipStream_t stream) {
    if (k < 1 || n_steps < 1 || !centres || !Fr) return HROM_E_INVALID;
    const int n = k * n_steps;
    hipLaunchKernelGGL(k_paths, dim3((n + 255) / 256), dim3(256), 0, stream, centres, k, n_steps, Fr);
    return hipGetLastError() == hipSuccess ? HROM_OK : HROM_E_HIP;
}

int hrom_pod(int32_t nd, int32_t s_el, const double* X_el, int32_t s_in, const double* X_in, int32_t n_el,
             int32_t n_in, double* Phi, double* sigma_el, double* sigma_in, hipStream_t stream) {
    if (nd < 1 || s_el < 1 || s_in < 1 || n_el < 1 || n_in < 0 || n_el > s_el || n_in > s_in || !X_el ||
        !X_in || !Phi || !sigma_el || !sigma_in)
        return HROM_E_INVALID;
    const int ld = n_el + n_in;
    int rc = svd_left(s_el, nd, X_el, n_el, Phi, ld, sigma_el, 0.0, 0, nullptr, nullptr, 0, stream);
    if (rc != HROM_OK) return rc;
    double *coef = nullptr, *Xm = nullptr;
    if (hipMalloc((void**)&coef, sizeof(double) * (size_t)s_in * n_el) != hipSuccess) return HROM_E_NOMEM;
    if (hipMalloc((void**)&Xm, sizeof(double) * (size_t)s_in * nd) != hipSuccess) {
        (void)hipFree(coef);
        return HROM_E_NOMEM;
    }
    hipLaunchKernelGGL(k_pod_coef, dim3(s_in), dim3(256), 0, stream, X_in, (int64_t)nd, Phi, ld, n_el, coef);
    const int64_t tot = (int64_t)s_in * nd;
    hipLaunchKernelGGL(k_pod_sub, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream, X_in, (int64_t)nd,
                       s_in, Phi, ld, n_el, coef, Xm);
    if (hipGetLastError() != hipSuccess) rc = HROM_E_HIP;
    if (rc == HROM_OK)
        rc = svd_left(s_in, nd, Xm, n_in, n_in > 0 ? Phi + n_el : nullptr, ld, sigma_in, 0.0, 0, nullptr, nullptr,
                      0, stream);
    (void)hipStreamSynchronize(stream);
    (void)hipFree(coef);
    (void)hipFree(Xm);
    return rc;
}

}  // extern "C"
