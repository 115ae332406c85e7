// Empirical cubature on the GPU (Sec. 3.3): the training matrix x_f of eq.
// ECM1, the truncated basis lambda of eq. SVDlambda, and the greedy point
// selection with least squares and an NNLS fallback of Box 1.
//
//  * hrom_ecm_training: the force integrand [G_g^T P(F_g); P(F_g)] of every
//    snapshot at every candidate point (one thread per candidate, four
//    snapshots per thread, the mode gradients read candidate-contiguous from
//    a transposed copy), then per row the weighted integral f^k_i and the
//    subtraction of f^k_i / V0.
//  * hrom_ecm_svd: for tall matrices a Householder QR x_f^T = Q R and a
//    second, column-pivoted QR R^T Pi = Q2 R2 first (the sweeps then run on
//    the P x P matrix R2^T); blocked one-sided Jacobi on the swept matrix:
//    per round a tournament of disjoint pairs of 32-column blocks;
//    for each pair the 64 x 64 Gram matrix (partial sums over row chunks,
//    summed in a fixed order), one cyclic Jacobi sweep over it in LDS (a full
//    inner solve cost more time than the extra outer sweep it saves), and the
//    product of the 64 columns with the accumulated rotation.  Sweeps run until every pair is
//    orthogonal to the tolerance relative to the column norms; then the
//    columns are ranked by norm and the leading r, normalised, form lambda.
//    One-sided Jacobi keeps small singular values accurate (a Gram matrix of
//    the whole x_f would square their condition).
//  * hrom_ecm_select: per greedy iteration a scoring kernel over all
//    candidates (the whole GPU; an exact two-pass argmax, lowest index on
//    ties) and a one-workgroup kernel holding a QR factorisation of J_z:
//    append by classical Gram-Schmidt with a second pass when the first
//    loses more than 1 - 1/sqrt(2) of the norm, back substitution, and the
//    Lawson-Hanson active-set NNLS warm-started at the previous weights,
//    removing columns by Givens rotations.  The host launches the pairs in
//    batches and stops at the workgroup's done flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "hrom.h"
#include "hrom_math.h"

namespace hrom {
namespace ecm {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double s) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// x of lane l (l uniform across the wavefront), through two scalar reads
__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// block-wide sum over 256 threads (fixed order); every thread gets the sum
__device__ double block_sum(double s, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    s = wave_sum(s);
    __syncthreads();
    if (lane == 0) red[wave] = s;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

// sum over a workgroup of 1024 threads (fixed order); every thread gets it
__device__ double block_sum1024(double s, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    s = wave_sum(s);
    __syncthreads();
    if (lane == 0) red[wave] = s;
    __syncthreads();
    double t[8];
#pragma unroll
    for (int i = 0; i < 8; i++) t[i] = red[2 * i] + red[2 * i + 1];
    const double u = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    __syncthreads();
    return u;
}

// ------------------------------------------------------------------------
// training matrix
// ------------------------------------------------------------------------
// Gt[(I m + n) M + g] = G[g][I][n]
__global__ void k_gt(const double* __restrict__ G, int nm, int M, double* __restrict__ Gt) {
    __shared__ double t[32][33];
    const int g0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int g = g0 + j, c = c0 + threadIdx.x;
        t[j][threadIdx.x] = (g < M && c < nm) ? G[(int64_t)g * nm + c] : 0.0;
    }
    __syncthreads();
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int c = c0 + j, g = g0 + threadIdx.x;
        if (g < M && c < nm) Gt[(int64_t)c * M + g] = t[threadIdx.x][j];
    }
}

constexpr int kES = 4;   // snapshots per thread

// compressible Neo-Hooke first Piola stress P = mu (F - F^-T) + lam ln J F^-T;
// false if det F <= 0
__device__ inline bool nh_stress(const double* F, double mu, double lam, double* P) {
    double Fi[9];
    const double J = inv3(F, Fi);
    if (!(J > 0.0)) return false;
    const double l = log(J);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            P[3 * i + j] = mu * (F[3 * i + j] - Fi[3 * j + i]) + lam * l * Fi[3 * j + i];
    return true;
}

__global__ void __launch_bounds__(256) k_integrand(const double* __restrict__ Gt, const int32_t* phase,
                                                   const double* theta, int m, int M, int p,
                                                   const double* __restrict__ Fr,
                                                   const double* __restrict__ a,
                                                   double* __restrict__ xf, int* bad) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    const int k0 = blockIdx.y * kES;
    if (g >= M) return;
    const int nk = min(kES, p - k0), nt = m + 9;
    const int ph = phase[g];
    const double mu = theta[2 * ph], lam = theta[2 * ph + 1];
    double F[kES][9];
#pragma unroll
    for (int s = 0; s < kES; s++)
#pragma unroll
        for (int I = 0; I < 9; I++) F[s][I] = (s < nk) ? Fr[9 * (k0 + s) + I] : ((I % 4 == 0) ? 1.0 : 0.0);
    for (int I = 0; I < 9; I++)
        for (int n = 0; n < m; n++) {
            const double gv = Gt[(int64_t)(I * m + n) * M + g];
#pragma unroll
            for (int s = 0; s < kES; s++)
                if (s < nk) F[s][I] += gv * a[(int64_t)(k0 + s) * m + n];
        }
    double P[kES][9];
    int nbad = 0;
#pragma unroll
    for (int s = 0; s < kES; s++) {
        if (s < nk && !nh_stress(F[s], mu, lam, P[s])) {
            nbad++;
#pragma unroll
            for (int I = 0; I < 9; I++) P[s][I] = 0.0;
        }
    }
    if (nbad) atomicAdd(bad, nbad);
    for (int n = 0; n < m; n++) {
        double f[kES];
#pragma unroll
        for (int s = 0; s < kES; s++) f[s] = 0.0;
        for (int I = 0; I < 9; I++) {
            const double gv = Gt[(int64_t)(I * m + n) * M + g];
#pragma unroll
            for (int s = 0; s < kES; s++) f[s] += gv * P[s][I];
        }
#pragma unroll
        for (int s = 0; s < kES; s++)
            if (s < nk) xf[((int64_t)(k0 + s) * nt + n) * M + g] = f[s];
    }
#pragma unroll
    for (int s = 0; s < kES; s++)
        if (s < nk)
#pragma unroll
            for (int I = 0; I < 9; I++) xf[((int64_t)(k0 + s) * nt + m + I) * M + g] = P[s][I];
}

// V0 = sum of the weights (one workgroup)
__global__ void __launch_bounds__(256) k_volume(const double* w, int M, double* V0) {
    __shared__ double red[4];
    double s = 0.0;
    for (int g = threadIdx.x; g < M; g += 256) s += w[g];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *V0 = s;
}

// per row: fint = sum_g w_g x_g, then x_g -= fint / V0 (one workgroup per row)
__global__ void __launch_bounds__(256) k_center(double* xf, const double* w, int M, const double* V0,
                                                double* fint) {
    __shared__ double red[4];
    double* row = xf + (int64_t)blockIdx.x * M;
    double s = 0.0;
    for (int g = threadIdx.x; g < M; g += 256) s += w[g] * row[g];
    s = block_sum(s, red);
    if (threadIdx.x == 0) fint[blockIdx.x] = s;
    const double sub = s / *V0;
    for (int g = threadIdx.x; g < M; g += 256) row[g] -= sub;
}

// ------------------------------------------------------------------------
// one-sided block Jacobi SVD of x_f^T
// ------------------------------------------------------------------------
constexpr int kSB = 32;          // columns per block
constexpr int kSW = 2 * kSB;     // columns per pair
constexpr int kSR = 64;          // rows per LDS tile

__device__ __forceinline__ int pair_col(int2 pr, int c) {
    return c < kSB ? pr.x * kSB + c : pr.y * kSB + (c - kSB);
}

// partial Gram of the 64 columns of pair blockIdx.x over rows chunk blockIdx.y
// a pair is skipped when neither of its blocks changed since the pair was
// last found orthogonal (versions of the blocks then = the recorded ones)
__device__ __forceinline__ bool pair_settled(const int2 pr, const int* ver, const int2* pver, int pi) {
    const int2 v = pver[pi];
    return ver[pr.x] == v.x && ver[pr.y] == v.y;
}

__global__ void __launch_bounds__(256) k_svd_gram(const double* __restrict__ A, int M, const int2* pairs,
                                                  int chunk_rows, int nchunks, double* __restrict__ part,
                                                  const int* ver, const int2* pver, int pbase) {
    // FP64 16x16x4 MFMA: wavefront w forms the four 16 x 16 tiles (w, 0..3) of
    // the 64 x 64 Gram matrix; lane (g, c) = (lane / 16, lane % 16) feeds
    // A[c][g] = T[16 w + c][k0 + g] and B[g][c] = T[16 J + c][k0 + g], and its
    // accumulator element e is D[g + 4 e][c]
    __shared__ double T[kSW][kSR + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
    const int2 pr = pairs[blockIdx.x];
    if (pair_settled(pr, ver, pver, pbase + blockIdx.x)) return;
    const int r0 = blockIdx.y * chunk_rows, r1 = min(M, r0 + chunk_rows);
    v4d acc[4];
#pragma unroll
    for (int J = 0; J < 4; J++) acc[J] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int rb = r0; rb < r1; rb += kSR) {
        for (int e = tid; e < kSW * kSR; e += 256) {
            const int cc = e / kSR, rr = e % kSR, gg = rb + rr;
            T[cc][rr] = (gg < r1) ? A[(int64_t)pair_col(pr, cc) * M + gg] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int k0 = 0; k0 < kSR; k0 += 4) {
            const double a = T[16 * wave + c][k0 + g];
#pragma unroll
            for (int J = 0; J < 4; J++)
                acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, T[16 * J + c][k0 + g], acc[J], 0, 0, 0);
        }
        __syncthreads();
    }
    double* out = part + ((int64_t)blockIdx.x * nchunks + blockIdx.y) * (kSW * kSW);
#pragma unroll
    for (int J = 0; J < 4; J++)
#pragma unroll
        for (int e = 0; e < 4; e++) out[(16 * wave + g + 4 * e) * kSW + 16 * J + c] = acc[J][e];
}

// order-preserving bits of a non-negative double, for atomicMax
__device__ __forceinline__ unsigned long long nonneg_bits(double x) {
    return (unsigned long long)__double_as_longlong(x);
}

// max over p < q of |W_pq| / sqrt(W_pp W_qq) (pairs with a zero column excluded)
__device__ double offdiag(const double (*W)[kSW + 1], double* red) {
    double o = 0.0;
    for (int e = threadIdx.x; e < kSW * kSW; e += 256) {
        const int p = e / kSW, q = e % kSW;
        if (p < q) {
            const double d = W[p][p] * W[q][q];
            if (d > 0.0) o = fmax(o, fabs(W[p][q]) / sqrt(d));
        }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) o = fmax(o, __shfl_xor(o, s, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = o;
    __syncthreads();
    const double t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return t;
}

// eigenvectors of the pair's Gram matrix by cyclic Jacobi (tournament order
// of 32 disjoint rotations per step); records the pair's orthogonality
// before the rotation
__global__ void __launch_bounds__(256) k_svd_rotate(const double* __restrict__ part, int nchunks,
                                                    double tol, int max_inner, double* __restrict__ Vout,
                                                    unsigned long long* offmax, const int2* pairs, int* ver,
                                                    int2* pver, int pbase, int* apply) {
    __shared__ double W[kSW][kSW + 1];
    __shared__ double V[kSW][kSW + 1];
    __shared__ double cs[kSW / 2][2];
    __shared__ int pq[kSW / 2][2];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const int2 pr = pairs[blockIdx.x];
    const int pi = pbase + blockIdx.x;
    if (pair_settled(pr, ver, pver, pi)) {
        if (tid == 0) apply[blockIdx.x] = 0;
        return;
    }
    const double* src = part + (int64_t)blockIdx.x * nchunks * (kSW * kSW);
    for (int e = tid; e < kSW * kSW; e += 256) {
        double s = 0.0;
        for (int ch = 0; ch < nchunks; ch++) s += src[(int64_t)ch * kSW * kSW + e];
        W[e / kSW][e % kSW] = s;
        V[e / kSW][e % kSW] = (e / kSW == e % kSW) ? 1.0 : 0.0;
    }
    __syncthreads();
    // W is symmetric up to rounding of the partial sums: use the upper triangle
    for (int e = tid; e < kSW * kSW; e += 256) {
        const int p = e / kSW, q = e % kSW;
        if (p > q) W[p][q] = W[q][p];
    }
    __syncthreads();
    const double off0 = offdiag(W, red);
    if (tid == 0) atomicMax(offmax, nonneg_bits(off0));
    if (!(off0 > tol)) {
        // orthogonal: record the blocks' versions, nothing to apply
        if (tid == 0) {
            pver[pi] = make_int2(ver[pr.x], ver[pr.y]);
            apply[blockIdx.x] = 0;
        }
        return;
    }
    if (tid == 0) {
        apply[blockIdx.x] = 1;
        ver[pr.x]++;
        ver[pr.y]++;
    }
    // per step each thread takes the rotations k = tid / 64 + 4 i (i < 8) for
    // column (row) tid % 64 and issues all their loads before its first store
    // (disjoint rotations touch disjoint rows and columns)
    constexpr int KT = kSW / 2 / 4;
    const int kb = tid >> 6, li = tid & 63;
    for (int sweep = 0; sweep < max_inner; sweep++) {
        for (int step = 0; step < kSW - 1; step++) {
            if (tid < kSW / 2) {
                // tournament: position 0 fixed, the others rotate
                auto pos = [&](int j) { return j == 0 ? 0 : 1 + (j - 1 + step) % (kSW - 1); };
                int p = pos(tid), q = pos(kSW - 1 - tid);
                if (p > q) { const int t = p; p = q; q = t; }
                const double al = W[p][p], be = W[q][q], ga = W[p][q];
                double c = 1.0, s = 0.0;
                if (ga != 0.0 && fabs(ga) > 1e-17 * sqrt(fabs(al * be))) {
                    const double tau = (be - al) / (2.0 * ga);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                cs[tid][0] = c;
                cs[tid][1] = s;
                pq[tid][0] = p;
                pq[tid][1] = q;
            }
            __syncthreads();
            int p[KT], q[KT];
            double c[KT], s[KT];
#pragma unroll
            for (int i = 0; i < KT; i++) {
                const int k = kb + 4 * i;
                p[i] = pq[k][0];
                q[i] = pq[k][1];
                c[i] = cs[k][0];
                s[i] = cs[k][1];
            }
            {   // rows p, q: W <- J^T W (li = column)
                double wp[KT], wq[KT];
#pragma unroll
                for (int i = 0; i < KT; i++) {
                    wp[i] = W[p[i]][li];
                    wq[i] = W[q[i]][li];
                }
#pragma unroll
                for (int i = 0; i < KT; i++) {
                    W[p[i]][li] = c[i] * wp[i] - s[i] * wq[i];
                    W[q[i]][li] = s[i] * wp[i] + c[i] * wq[i];
                }
            }
            __syncthreads();
            {   // columns p, q: W <- W J, V <- V J (li = row)
                double wp[KT], wq[KT], vp[KT], vq[KT];
#pragma unroll
                for (int i = 0; i < KT; i++) {
                    wp[i] = W[li][p[i]];
                    wq[i] = W[li][q[i]];
                    vp[i] = V[li][p[i]];
                    vq[i] = V[li][q[i]];
                }
#pragma unroll
                for (int i = 0; i < KT; i++) {
                    W[li][p[i]] = c[i] * wp[i] - s[i] * wq[i];
                    W[li][q[i]] = s[i] * wp[i] + c[i] * wq[i];
                    V[li][p[i]] = c[i] * vp[i] - s[i] * vq[i];
                    V[li][q[i]] = s[i] * vp[i] + c[i] * vq[i];
                }
            }
            __syncthreads();
        }
        if (sweep + 1 < max_inner && !(offdiag(W, red) > 0.1 * tol)) break;
    }
    for (int e = tid; e < kSW * kSW; e += 256) Vout[(int64_t)blockIdx.x * kSW * kSW + e] = V[e / kSW][e % kSW];
}

// the pair's 64 columns times its rotation over rows chunk blockIdx.y (1024
// rows, the rotation loaded once), 64 rows per step: FP64 16x16x4 MFMA,
// wavefront w the row tile w against the four column tiles (A[row][c] =
// T[c][row], B[c][c'] = V[c][c']), the result staged in LDS for coalesced
// stores
__global__ void __launch_bounds__(256) k_svd_apply(double* __restrict__ A, int M, const int2* pairs,
                                                   const double* __restrict__ Vin, const int* apply,
                                                   int chunk_rows) {
    __shared__ double T[kSW][kSR + 1];
    __shared__ double Vs[kSW][kSW + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
    if (!apply[blockIdx.x]) return;
    const int2 pr = pairs[blockIdx.x];
    const double* V = Vin + (int64_t)blockIdx.x * kSW * kSW;
    for (int e = tid; e < kSW * kSW; e += 256) Vs[e / kSW][e % kSW] = V[e];
    const int r0 = blockIdx.y * chunk_rows, r1 = min(M, r0 + chunk_rows);
    for (int g0 = r0; g0 < r1; g0 += kSR) {
        for (int e = tid; e < kSW * kSR; e += 256) {
            const int cc = e / kSR, rr = e % kSR, gg = g0 + rr;
            T[cc][rr] = (gg < r1) ? A[(int64_t)pair_col(pr, cc) * M + gg] : 0.0;
        }
        __syncthreads();
        v4d acc[4];
#pragma unroll
        for (int C = 0; C < 4; C++) acc[C] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k0 = 0; k0 < kSW; k0 += 4) {
            const double a = T[k0 + g][16 * wave + c];
#pragma unroll
            for (int C = 0; C < 4; C++)
                acc[C] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Vs[k0 + g][16 * C + c], acc[C], 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int C = 0; C < 4; C++)
#pragma unroll
            for (int e = 0; e < 4; e++) T[16 * C + c][16 * wave + g + 4 * e] = acc[C][e];
        __syncthreads();
        for (int e = tid; e < kSW * kSR; e += 256) {
            const int cc = e / kSR, rr = e % kSR, gg = g0 + rr;
            if (gg < r1) A[(int64_t)pair_col(pr, cc) * M + gg] = T[cc][rr];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_svd_norms(const double* A, int M, double* sig) {
    __shared__ double red[4];
    const double* col = A + (int64_t)blockIdx.x * M;
    double s = 0.0;
    for (int g = threadIdx.x; g < M; g += 256) s += col[g] * col[g];
    s = block_sum(s, red);
    if (threadIdx.x == 0) sig[blockIdx.x] = sqrt(s);
}

// rank of every column by decreasing norm (ties: lower index first)
__global__ void k_svd_rank(const double* sig, int P, int* perm, double* sig_out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P) return;
    const double s = sig[c];
    int rk = 0;
    for (int d = 0; d < P; d++) {
        const double t = sig[d];
        rk += (t > s || (t == s && d < c)) ? 1 : 0;
    }
    perm[rk] = c;
    sig_out[rk] = s;
}

// lam[g][j] = A[perm[j]][g] / sigma_j, j < r (row stride ld)
__global__ void k_svd_extract(const double* A, int M, const int* perm, const double* sig_sorted, int r,
                              double* lam, int ld) {
    __shared__ double t[32][33];
    const int g0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    for (int jj = threadIdx.y; jj < 32; jj += 8) {
        const int j = j0 + jj, g = g0 + threadIdx.x;
        t[jj][threadIdx.x] = (j < r && g < M) ? A[(int64_t)perm[j] * M + g] / sig_sorted[j] : 0.0;
    }
    __syncthreads();
    for (int gg = threadIdx.y; gg < 32; gg += 8) {
        const int g = g0 + gg, j = j0 + threadIdx.x;
        if (g < M && j < r) lam[(int64_t)g * ld + j] = t[threadIdx.x][gg];
    }
}

// ------------------------------------------------------------------------
// Householder QR of x_f^T ahead of the sweeps (tall matrices)
// ------------------------------------------------------------------------
// x_f^T = Q R with Q the product of Householder reflectors, in panels of kQB
// columns applied to the rest of the matrix in the compact WY form
// Q_k = I - V_k T_k V_k^T.  R has the singular values of x_f^T and every
// sweep over it touches P rows in place of M; the left vectors of x_f^T are
// Q times those of R.  Householder QR is backward stable, so the singular
// values keep their absolute accuracy relative to sigma_1.
constexpr int kQB = 32;

// Householder reflector of a column with head x1 and squared tail norm sg:
// H = I - t v v^T with v = (1, sc x_tail) maps the column to b e_1; t = 0
// (H = I) when the tail is zero
__device__ __forceinline__ void reflector(double x1, double sg, double& b, double& t, double& sc) {
    t = 0.0;
    b = x1;
    sc = 0.0;
    if (sg > 0.0) {
        const double nrm = sqrt(x1 * x1 + sg);
        b = (x1 >= 0.0) ? -nrm : nrm;
        t = (b - x1) / b;
        sc = 1.0 / (x1 - b);
    }
}

// Reflector of column j (rows j .. M-1) and its product with the panel
// columns j + 1 .. j + gridDim.x - 1: workgroup b handles column j + b.  Every
// workgroup forms the reflector from column j, which no workgroup of this
// launch writes; workgroup 0 stores v (one at row j, zero above), tau and the
// diagonal entry beta of R.  H = I - tau v v^T maps column j to beta e_j;
// tau = 0 (H = I) when the column is zero below row j.
__global__ void __launch_bounds__(1024) k_qr_col(double* __restrict__ A, int M, int j, double* __restrict__ V,
                                                 double* __restrict__ tau, double* __restrict__ beta) {
    __shared__ double red[16];
    const int tid = threadIdx.x;
    const double* x = A + (int64_t)j * M;
    double* y = A + (int64_t)(j + blockIdx.x) * M;
    const double x1 = x[j], y1 = y[j];
    double s = 0.0;
#pragma unroll 4
    for (int i = j + 1 + tid; i < M; i += 1024) s += x[i] * x[i];
    const double sg = block_sum1024(s, red);
    double t, b, sc;
    reflector(x1, sg, b, t, sc);
    if (blockIdx.x == 0) {
        double* v = V + (int64_t)j * M;
        for (int i = tid; i < M; i += 1024) v[i] = (i < j) ? 0.0 : ((i == j) ? 1.0 : x[i] * sc);
        if (tid == 0) {
            tau[j] = t;
            beta[j] = b;
        }
        return;
    }
    if (t == 0.0) return;
    double d = 0.0;
#pragma unroll 4
    for (int i = j + 1 + tid; i < M; i += 1024) d += x[i] * y[i];
    const double f = t * (y1 + sc * block_sum1024(d, red));
#pragma unroll 4
    for (int i = j + 1 + tid; i < M; i += 1024) y[i] -= f * (x[i] * sc);
    if (tid == 0) y[j] = y1 - f;
}

// Partial products V_p^T X over the rows of chunk blockIdx.y (from row r0 on)
// for a tile of 32 columns of X per blockIdx.x (V_p: the kQB columns of a
// panel, zero above its first row): FP64 16x16x4 MFMA, wavefront w the 16 x 16
// tile (w / 2, w % 2); lane (g, c) feeds A[c][g] = V[k0 + g][16 (w / 2) + c]
// and B[g][c] = X[k0 + g][16 (w % 2) + c], accumulator element e = D[g + 4 e][c]
__global__ void __launch_bounds__(256) k_qr_cross(const double* __restrict__ Vp, const double* __restrict__ X,
                                                  int M, int r0, int ncols, int chunk_rows, int nchunks,
                                                  double* __restrict__ part) {
    __shared__ double Vt[kQB][kSR + 1];
    __shared__ double Xt[kQB][kSR + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
    const int c0 = blockIdx.x * kQB, ti = wave >> 1, tj = wave & 1;
    const int rb0 = r0 + blockIdx.y * chunk_rows, rb1 = min(M, rb0 + chunk_rows);
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    for (int rb = rb0; rb < rb1; rb += kSR) {
        for (int e = tid; e < kQB * kSR; e += 256) {
            const int cc = e / kSR, rr = e % kSR, gg = rb + rr;
            const bool in = gg < rb1;
            Vt[cc][rr] = in ? Vp[(int64_t)cc * M + gg] : 0.0;
            Xt[cc][rr] = (in && c0 + cc < ncols) ? X[(int64_t)(c0 + cc) * M + gg] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int k0 = 0; k0 < kSR; k0 += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Vt[16 * ti + c][k0 + g], Xt[16 * tj + c][k0 + g], acc, 0, 0,
                                                       0);
        __syncthreads();
    }
    double* out = part + ((int64_t)blockIdx.x * nchunks + blockIdx.y) * (kQB * kQB);
#pragma unroll
    for (int e = 0; e < 4; e++) out[(16 * ti + g + 4 * e) * kQB + 16 * tj + c] = acc[e];
}

// Z[k][col] = sum over the chunks in order of the partials of k_qr_cross
__global__ void __launch_bounds__(256) k_qr_zsum(const double* __restrict__ part, int nchunks, int ncols,
                                                 double* __restrict__ Z) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kQB * ncols) return;
    const int k = e / ncols, col = e % ncols;
    const double* src = part + (int64_t)(col / kQB) * nchunks * (kQB * kQB) + k * kQB + col % kQB;
    double s = 0.0;
    for (int ch = 0; ch < nchunks; ch++) s += src[(int64_t)ch * (kQB * kQB)];
    Z[(int64_t)k * ncols + col] = s;
}

// T of the panel's compact WY form (one workgroup of kQB threads) from
// Y = V^T V (row stride ldy) and the panel's tau: T_ii = tau_i,
// T[0:i, i] = -tau_i T[0:i, 0:i] Y[0:i, i]
__global__ void k_qr_tbuild(const double* __restrict__ Y, int ldy, const double* __restrict__ tau,
                            double* __restrict__ T) {
    __shared__ double Ts[kQB][kQB + 1];
    const int r = threadIdx.x;
    for (int k = 0; k < kQB; k++) Ts[r][k] = 0.0;
    __syncthreads();
    for (int i = 0; i < kQB; i++) {
        double s = 0.0;
        if (r < i)
            for (int k = r; k < i; k++) s += Ts[r][k] * Y[k * ldy + i];
        __syncthreads();
        if (r < i) Ts[r][i] = -tau[i] * s;
        if (r == i) Ts[i][i] = tau[i];
        __syncthreads();
    }
    for (int k = 0; k < kQB; k++) T[r * kQB + k] = Ts[r][k];
}

// Wt = T^T Z (trans: the transposed panel, Q_k^T X) or T Z (Q_k X)
__global__ void __launch_bounds__(256) k_qr_tmul(const double* __restrict__ T, const double* __restrict__ Z,
                                                 int ncols, int trans, double* __restrict__ Wt) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kQB * ncols) return;
    const int i = e / ncols, col = e % ncols;
    double s = 0.0;
    for (int k = 0; k < kQB; k++) s += (trans ? T[k * kQB + i] : T[i * kQB + k]) * Z[(int64_t)k * ncols + col];
    Wt[(int64_t)i * ncols + col] = s;
}

// X[:, c] -= V_p Wt[:, c] over the rows of chunk blockIdx.y (from row r0 on)
// for a tile of 32 columns per blockIdx.x: FP64 MFMA with the accumulator
// started at X, wavefront w the rows 16 w .. of every 64-row step against the
// two column tiles (A[c][g] = -V[row][k0 + g], B[g][c] = Wt[k0 + g][col])
__global__ void __launch_bounds__(256) k_qr_update(double* __restrict__ X, const double* __restrict__ Vp, int M,
                                                   int r0, int ncols, int chunk_rows, const double* __restrict__ Wt) {
    __shared__ double Vt[kSR][kQB + 1];
    __shared__ double Ws[kQB][kQB + 1];
    __shared__ double Xt[kQB][kSR + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
    const int c0 = blockIdx.x * kQB;
    for (int e = tid; e < kQB * kQB; e += 256) {
        const int k = e / kQB, cc = e % kQB;
        Ws[k][cc] = (c0 + cc < ncols) ? Wt[(int64_t)k * ncols + c0 + cc] : 0.0;
    }
    const int rb0 = r0 + blockIdx.y * chunk_rows, rb1 = min(M, rb0 + chunk_rows);
    for (int rb = rb0; rb < rb1; rb += kSR) {
        for (int e = tid; e < kQB * kSR; e += 256) {
            const int cc = e / kSR, rr = e % kSR, gg = rb + rr;
            const bool in = gg < rb1;
            Vt[rr][cc] = in ? Vp[(int64_t)cc * M + gg] : 0.0;
            Xt[cc][rr] = (in && c0 + cc < ncols) ? X[(int64_t)(c0 + cc) * M + gg] : 0.0;
        }
        __syncthreads();
        v4d acc[2];
#pragma unroll
        for (int J = 0; J < 2; J++)
#pragma unroll
            for (int e = 0; e < 4; e++) acc[J][e] = Xt[16 * J + c][16 * wave + g + 4 * e];
#pragma unroll
        for (int k0 = 0; k0 < kQB; k0 += 4) {
            const double a = -Vt[16 * wave + c][k0 + g];
#pragma unroll
            for (int J = 0; J < 2; J++)
                acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ws[k0 + g][16 * J + c], acc[J], 0, 0, 0);
        }
        // each wavefront rewrites only the rows it read
#pragma unroll
        for (int J = 0; J < 2; J++)
#pragma unroll
            for (int e = 0; e < 4; e++) Xt[16 * J + c][16 * wave + g + 4 * e] = acc[J][e];
        __syncthreads();
        for (int e = tid; e < kQB * kSR; e += 256) {
            const int cc = e / kSR, rr = e % kSR, gg = rb + rr;
            if (gg < rb1 && c0 + cc < ncols) X[(int64_t)(c0 + cc) * M + gg] = Xt[cc][rr];
        }
        __syncthreads();
    }
}

// ---- second factorisation, with column pivoting, of R^T (Drmac-Veselic
// preconditioning): R^T Pi = Q2 R2, and the sweeps run on X = R2^T, whose
// columns are nearly orthogonal from the start (the pivoted triangle is
// graded), so that the quadratic phase begins within a few sweeps.  With
// R = Pi R2^T Q2^T the left vectors of R are Pi times those of X; Q2 itself
// is never needed.  Matrices here are stored as Ppad columns of P entries.

// B[i][c] = R[i][c]: column i of B is row i of R (zero for the padding)
__global__ void __launch_bounds__(256) k_qr_rtbuild(const double* __restrict__ A, int M, const double* beta, int P,
                                                    int Ppad, double* __restrict__ B) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)Ppad * P) return;
    const int i = (int)(e / P), c = (int)(e % P);
    B[e] = (i >= P || c < i) ? 0.0 : ((c == i) ? beta[i] : A[(int64_t)c * M + i]);
}

// squared norms of the columns of B, the identity permutation
__global__ void __launch_bounds__(256) k_qrcp_init(const double* __restrict__ B, int P, double* nu, int* perm) {
    __shared__ double red[4];
    const double* col = B + (int64_t)blockIdx.x * P;
    double s = 0.0;
    for (int i = threadIdx.x; i < P; i += 256) s += col[i] * col[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        nu[blockIdx.x] = s;
        perm[blockIdx.x] = blockIdx.x;
    }
}

// Step j of the pivoted QR of B (P columns of P entries): the pivot is the
// remaining column (positions j .. P-1, physical columns through perm_in)
// with the largest squared norm of rows j .. P-1 (nu_in, by physical column;
// lowest position on ties), found by every workgroup alike; workgroup b
// takes position j + b after the exchange of positions j and the pivot.
// Workgroup 0 records beta_j (R2's diagonal) and the exchanged permutation;
// the others apply the pivot column's reflector to their column, which no
// workgroup of this launch reads, and record its squared norm over rows
// j + 1 .. (nu_out).  The permutation and the norms alternate between two
// buffers from step to step.
__global__ void __launch_bounds__(256) k_qrcp_col(double* __restrict__ B, int P, int j, const int* __restrict__ perm_in,
                                                  const double* __restrict__ nu_in, int* __restrict__ perm_out,
                                                  double* __restrict__ nu_out, double* __restrict__ beta2) {
    __shared__ double red[4];
    __shared__ double wv[4];
    __shared__ int wi[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double bv = -1.0;
    int bi = INT32_MAX;
    for (int c = j + tid; c < P; c += 256) {
        const double v = nu_in[perm_in[c]];
        if (v > bv) {
            bv = v;
            bi = c;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) {
        wv[wave] = bv;
        wi[wave] = bi;
    }
    __syncthreads();
    double pv = wv[0];
    int cs = wi[0];
    for (int w = 1; w < 4; w++)
        if (wv[w] > pv || (wv[w] == pv && wi[w] < cs)) {
            pv = wv[w];
            cs = wi[w];
        }
    const int xp = perm_in[cs];
    const int pos = j + blockIdx.x;
    const int yp = (pos == j) ? xp : ((pos == cs) ? perm_in[j] : perm_in[pos]);
    const double* x = B + (int64_t)xp * P;
    double* y = B + (int64_t)yp * P;
    const double x1 = x[j], y1 = y[j];
    double s = 0.0;
    for (int i = j + 1 + tid; i < P; i += 256) s += x[i] * x[i];
    const double sg = block_sum(s, red);
    double t, b, sc;
    reflector(x1, sg, b, t, sc);
    if (blockIdx.x == 0) {
        if (tid == 0) beta2[j] = b;
        for (int c = tid; c < P; c += 256) perm_out[c] = (c == j) ? xp : ((c == cs) ? perm_in[j] : perm_in[c]);
        return;
    }
    double f = 0.0;
    if (t != 0.0) {
        double d = 0.0;
        for (int i = j + 1 + tid; i < P; i += 256) d += x[i] * y[i];
        f = t * (y1 + sc * block_sum(d, red));
    }
    double s2 = 0.0;
    for (int i = j + 1 + tid; i < P; i += 256) {
        const double yn = y[i] - f * (x[i] * sc);
        y[i] = yn;
        s2 += yn * yn;
    }
    s2 = block_sum(s2, red);
    if (tid == 0) {
        y[j] = y1 - f;
        nu_out[yp] = s2;
    }
}

// X = R2^T for the sweeps: column i = row i of R2 over the positions,
// (0 .. 0, beta2_i, B[perm[c]][i] for c > i); zero padding columns
__global__ void __launch_bounds__(256) k_qrcp_xbuild(const double* __restrict__ B, int P, int Ppad, const int* perm,
                                                     const double* beta2, double* __restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)Ppad * P) return;
    const int i = (int)(e / P), c = (int)(e % P);
    X[e] = (i >= P || c < i) ? 0.0 : ((c == i) ? beta2[i] : B[(int64_t)perm[c] * P + i]);
}

// inverse of the final permutation
__global__ void __launch_bounds__(256) k_qrcp_iperm(const int* perm, int P, int* iperm) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < P) iperm[perm[c]] = c;
}

// X[j][i] = R-side left vector j: column perm[j] of the swept matrix (MJ rows)
// over sigma_j at its row iperm[i] (i itself without iperm), zero for rows
// i >= MJ (j < r)
__global__ void __launch_bounds__(256) k_qr_xinit(const double* __restrict__ Jm, int MJ, const int* perm,
                                                  const double* sig, const int* iperm, int r, int M,
                                                  double* __restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)r * M) return;
    const int j = (int)(e / M), i = (int)(e % M);
    X[e] = (i < MJ) ? Jm[(int64_t)perm[j] * MJ + (iperm ? iperm[i] : i)] / sig[j] : 0.0;
}

// lam[g][j] = X[j][g] (row stride ld)
__global__ void k_qr_out(const double* __restrict__ X, int M, int r, double* __restrict__ lam, int ld) {
    __shared__ double t[32][33];
    const int g0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    for (int jj = threadIdx.y; jj < 32; jj += 8) {
        const int j = j0 + jj, g = g0 + threadIdx.x;
        t[jj][threadIdx.x] = (j < r && g < M) ? X[(int64_t)j * M + g] : 0.0;
    }
    __syncthreads();
    for (int gg = threadIdx.y; gg < 32; gg += 8) {
        const int g = g0 + gg, j = j0 + threadIdx.x;
        if (g < M && j < r) lam[(int64_t)g * ld + j] = t[threadIdx.x][gg];
    }
}

// ------------------------------------------------------------------------
// Box 1 greedy
// ------------------------------------------------------------------------
constexpr int kMaxRows = 1024;   // r + 1 <= 1024, mt <= r + 1
constexpr int kStepThreads = 512; // workgroup of the one-workgroup step
constexpr int kStepWaves = kStepThreads / 64;

// sum over the step's workgroup (fixed order); every thread gets the sum
__device__ double step_sum(double s, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s = wave_sum(s);
    __syncthreads();
    if (lane == 0) red[wave] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kStepWaves; w++) t += red[w];
    __syncthreads();
    return t;
}

struct State {
    int n;        // selected points (columns of the QR)
    int iters;    // greedy iterations done
    int done;     // 1 once the loop has ended
    int err;      // 0, or an HROM_E_* code
    int navail;   // candidates still available
    int nfree;    // free physical columns of R
    int pad[2];
};

struct SelArgs {
    const double* lam;   // [M][r]
    int M, r, mt;
    double V0;
    double* jn;          // [M] |j_k|
    double* csum;        // [M] sum_i |J_ik|
    uint8_t* avail;      // [M]
    double* Q;           // [mt][r + 1], column c at Q + c (r + 1)
    double* R;           // [mt][mt] by physical column: entry (row i, column pc) at pc mt + i
    double* x;           // [mt] weights by position
    int* zsel;           // [mt] candidate of each position
    int* stamp;          // [mt] iteration that picked the candidate
    int* cmap;           // [mt] physical column of R of each position
    int* cfree;          // [mt] free physical columns
    double* res;         // [r + 1] b - J_z w
    double* pscore;      // [nb] per-workgroup best score
    int* pidx;           // [nb] and its candidate
    int nb;
    int* trace;          // [trace_cap][4]: picked, nnls, dropped, n; or null
    int trace_cap;
    State* st;
};

__global__ void k_sel_prep(SelArgs A) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < A.M) {
        double s = 1.0, t = 1.0;
        for (int j = 0; j < A.r; j++) {
            const double v = A.lam[(int64_t)g * A.r + j];
            s += v * v;
            t += fabs(v);
        }
        A.jn[g] = sqrt(s);
        A.csum[g] = t;
        A.avail[g] = 1;
    }
    if (g <= A.r) A.res[g] = (g == A.r) ? A.V0 : 0.0;
    if (g == 0) {
        A.st->n = 0;
        A.st->iters = 0;
        A.st->done = (A.mt <= 0 || A.M <= 0) ? 1 : 0;
        A.st->err = 0;
        A.st->navail = A.M;
        A.st->nfree = 0;
    }
}

// step 1: score of every available candidate, j_k . r / |j_k|
__global__ void __launch_bounds__(256) k_sel_score(SelArgs A) {
    if (A.st->done) return;
    __shared__ double sres[kMaxRows];
    __shared__ double bs[4];
    __shared__ int bi[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r = A.r;
    for (int j = tid; j <= r; j += 256) sres[j] = A.res[j];
    __syncthreads();
    double best = -INFINITY;
    int bidx = INT32_MAX;
    const int nw = gridDim.x * 4;
    for (int k = blockIdx.x * 4 + wave; k < A.M; k += nw) {
        if (!A.avail[k]) continue;
        const double* lk = A.lam + (int64_t)k * r;
        double s = 0.0;
        for (int j = lane; j < r; j += 64) s += lk[j] * sres[j];
        s = wave_sum(s);
        const double sc = (s + sres[r]) / A.jn[k];
        if (sc > best) {
            best = sc;
            bidx = k;
        }
    }
    if (lane == 0) {
        bs[wave] = best;
        bi[wave] = bidx;
    }
    __syncthreads();
    if (tid == 0) {
        double b = bs[0];
        int i = bi[0];
        for (int w = 1; w < 4; w++)
            if (bs[w] > b || (bs[w] == b && bi[w] < i)) {
                b = bs[w];
                i = bi[w];
            }
        A.pscore[blockIdx.x] = b;
        A.pidx[blockIdx.x] = i;
    }
}

// LDS of the one-workgroup step
struct StepLds {
    double v[kMaxRows];     // column being appended
    double h[kMaxRows];     // its projections
    double h2[kMaxRows];
    double c[kMaxRows];     // Q^T b
    double cw[kMaxRows];    // working copy of c in the back substitution
    double z[kMaxRows];     // least-squares solution by position
    double xw[kMaxRows];    // current weights by position
    double res[kMaxRows];   // residual b - Q Q^T b
    union {
        double D[64][65];        // diagonal block of the back substitution
        double gs[kMaxRows][2];  // Givens (c, s) of a downdate
    };
    int zs[kMaxRows];       // candidate of each position
    int st[kMaxRows];       // its pick stamp
    int cm[kMaxRows];       // physical column of R holding each position
    int cf[kMaxRows];       // free physical columns
    int nfree;
    int zl[kMaxRows];       // NNLS: candidates outside the passive set
    int zst[kMaxRows];      //       their pick stamps
    int zbl[kMaxRows];      //       blocked flags
    double red[kStepWaves];
    double bsc;
    int bidx;
};

// v <- j_k = [lam_k; 1]
__device__ void load_col(const SelArgs& A, int k, StepLds& L) {
    for (int i = threadIdx.x; i <= A.r; i += kStepThreads) L.v[i] = (i < A.r) ? A.lam[(int64_t)k * A.r + i] : 1.0;
    __syncthreads();
}

// sum over columns c < n of Q[c][i] x[c] for row i: 16 columns per step,
// their loads issued together
__device__ __forceinline__ double qrow_dot(const double* Q, int r1, int i, int n, const double* x) {
    double s = 0.0;
    int c = 0;
    for (; c + 16 <= n; c += 16) {
        double q[16];
#pragma unroll
        for (int u = 0; u < 16; u++) q[u] = Q[(int64_t)(c + u) * r1 + i];
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int u = 0; u < 16; u += 2) {
            t0 += q[u] * x[c + u];
            t1 += q[u + 1] * x[c + u + 1];
        }
        s += t0 + t1;
    }
    for (; c < n; c++) s += Q[(int64_t)c * r1 + i] * x[c];
    return s;
}

// h <- Q_n^T v: a wavefront per four columns, its lanes over consecutive rows
// (every load instruction reads whole cache lines; a thread per column read
// 64 lines per instruction), four 64-row chunks of the four columns in flight
// per lane, then fixed-order wavefront sums; v <- v - Q_n h (a thread per row)
__device__ void project(const SelArgs& A, int n, StepLds& L, double* h) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r1 = A.r + 1;
    constexpr int CG = 4;
    for (int c0 = 4 * wave; c0 < n; c0 += 4 * kStepWaves) {
        // columns past n read column c0 and are discarded
        int64_t off[4];
#pragma unroll
        for (int u = 0; u < 4; u++) off[u] = (int64_t)((c0 + u < n) ? c0 + u : c0) * r1;
        double sc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i0 = 0; i0 < r1; i0 += 64 * CG) {
            // rows past r1 read the last row with weight zero
            double qv[CG][4], vv[CG];
#pragma unroll
            for (int k = 0; k < CG; k++) {
                const int i = i0 + 64 * k + lane, ic = min(i, r1 - 1);
                vv[k] = (i < r1) ? L.v[ic] : 0.0;
#pragma unroll
                for (int u = 0; u < 4; u++) qv[k][u] = A.Q[off[u] + ic];
            }
#pragma unroll
            for (int k = 0; k < CG; k++)
#pragma unroll
                for (int u = 0; u < 4; u++) sc[u] += qv[k][u] * vv[k];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) sc[u] = wave_sum(sc[u]);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (c0 + u < n) h[c0 + u] = sc[u];
        }
    }
    __syncthreads();
    for (int i = tid; i < r1; i += kStepThreads) L.v[i] -= qrow_dot(A.Q, r1, i, n, h);
    __syncthreads();
}

// append v as column n of the QR (R's column in a free physical slot);
// returns |v_perp| / |v|
__device__ double qr_append(const SelArgs& A, int n, StepLds& L) {
    const int tid = threadIdx.x, r1 = A.r + 1;
    double s = 0.0;
    for (int i = tid; i < r1; i += kStepThreads) s += L.v[i] * L.v[i];
    const double vn = sqrt(step_sum(s, L.red));
    project(A, n, L, L.h);
    s = 0.0;
    for (int i = tid; i < r1; i += kStepThreads) s += L.v[i] * L.v[i];
    double rho = sqrt(step_sum(s, L.red));
    if (n > 0 && rho < 0.7071067811865476 * vn) {   // second Gram-Schmidt pass
        project(A, n, L, L.h2);
        for (int c = tid; c < n; c += kStepThreads) L.h[c] += L.h2[c];
        s = 0.0;
        for (int i = tid; i < r1; i += kStepThreads) s += L.v[i] * L.v[i];
        rho = sqrt(step_sum(s, L.red));
    }
    const int slot = (L.nfree > 0) ? L.cf[L.nfree - 1] : n;
    const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
    for (int i = tid; i < r1; i += kStepThreads) A.Q[(int64_t)n * r1 + i] = L.v[i] * inv;
    for (int c = tid; c < n; c += kStepThreads) A.R[(int64_t)slot * A.mt + c] = L.h[c];
    __syncthreads();
    if (tid == 0) {
        A.R[(int64_t)slot * A.mt + n] = rho;
        L.cm[n] = slot;
        if (L.nfree > 0) L.nfree--;
    }
    __syncthreads();
    return vn > 0.0 ? rho / vn : 0.0;
}

// res = b - Q_n c with c = Q_n^T b as left by the last qr_solve
__device__ void residual(const SelArgs& A, int n, StepLds& L) {
    const int tid = threadIdx.x, r = A.r, r1 = r + 1;
    for (int i = tid; i < r1; i += kStepThreads) L.res[i] = ((i == r) ? A.V0 : 0.0) - qrow_dot(A.Q, r1, i, n, L.c);
    __syncthreads();
}

// c = Q_n^T b = V0 Q[r][.]; z = R^{-1} c by blocks of 64 rows from the
// bottom: the diagonal block in LDS, solved by wavefront 0 with the solution
// in lane registers (the pivots' reciprocals formed lane-parallel), then the
// rows above updated a thread per row; and
// res = b - Q_n c
__device__ void qr_solve(const SelArgs& A, int n, StepLds& L, bool want_res) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r = A.r, r1 = r + 1, mt = A.mt;
    for (int c = tid; c < n; c += kStepThreads) {
        const double cv = A.V0 * A.Q[(int64_t)c * r1 + r];
        L.c[c] = cv;
        L.cw[c] = cv;
    }
    __syncthreads();
    for (int b1 = n; b1 > 0; b1 -= 64) {
        const int b0 = max(0, b1 - 64), bs = b1 - b0;
        // the diagonal block, lanes over the rows of a column (whole cache lines)
        for (int e = tid; e < 64 * 64; e += kStepThreads) {
            const int ii = e & 63, jj = e >> 6;
            L.D[ii][jj] = (ii < bs && jj < bs && jj >= ii) ? A.R[L.cm[b0 + jj] * mt + b0 + ii] : 0.0;
        }
        __syncthreads();
        if (wave == 0) {
            // lane l holds row b0 + l: its right-hand side, then its solution;
            // the pivots' reciprocals are formed first, one per lane, so that
            // each step of the chain is a product and a broadcast
            double rhs = (lane < bs) ? L.cw[b0 + lane] : 0.0;
            const double dinv = (lane < bs) ? 1.0 / L.D[lane][lane] : 0.0;
            double zl = 0.0;
            // the lane's entries of eight columns read ahead of their steps
            // and the updates selected rather than branched, so that no LDS
            // read waits inside the chain
            for (int i0 = bs - 1; i0 >= 0; i0 -= 8) {
                double dv[8];
#pragma unroll
                for (int u = 0; u < 8; u++) dv[u] = L.D[lane][max(i0 - u, 0)];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int ii = i0 - u;
                    if (ii < 0) break;
                    const double zi = readlane_d(rhs * dinv, ii);
                    zl = (lane == ii) ? zi : zl;
                    rhs = (lane < ii) ? rhs - dv[u] * zi : rhs;
                }
            }
            if (lane < bs) L.z[b0 + lane] = zl;
        }
        __syncthreads();
        // rows above the block: cw_i -= sum_j R[i][j] z_j over the block's
        // columns (a thread per row, so that each load instruction reads
        // consecutive rows of one column; 16 loads in flight)
        for (int i = tid; i < b0; i += kStepThreads) {
            const double* Ri = A.R + i;
            double s0 = 0.0, s1 = 0.0;
            int jj = 0;
            for (; jj + 16 <= bs; jj += 16) {
                double t[16];
#pragma unroll
                for (int u = 0; u < 16; u++) t[u] = Ri[L.cm[b0 + jj + u] * mt];
#pragma unroll
                for (int u = 0; u < 16; u += 2) {
                    s0 += t[u] * L.z[b0 + jj + u];
                    s1 += t[u + 1] * L.z[b0 + jj + u + 1];
                }
            }
            for (; jj < bs; jj++) s0 += Ri[L.cm[b0 + jj] * mt] * L.z[b0 + jj];
            L.cw[i] -= s0 + s1;
        }
        __syncthreads();
    }
    if (want_res) residual(A, n, L);
}

// remove position j from the QR of n columns: Givens rotations on rows
// j .. n-1 restore the triangle of R with column j taken out (R's columns are
// addressed through the position -> physical column map, so no column moves;
// the freed physical column is reused by a later append), Q's columns j ..
// n-1 rotate alike and the last drops; the position arrays shift left
template <int T>   // positions per lane: T >= ceil(mt / 64)
__device__ void qr_remove(const SelArgs& A, int j, int n, StepLds& L) {
    const int tid = threadIdx.x, lane = tid & 63, r1 = A.r + 1, mt = A.mt;
    // the map without position j: chunks of kStepThreads positions from the left,
    // each read completely before it is written (the next chunk reads only
    // positions right of it)
    const int freed = L.cm[j];
    for (int p0 = j; p0 < n - 1; p0 += kStepThreads) {
        int cm_n = 0, zs_n = 0, st_n = 0;
        double xw_n = 0.0;
        const int p = p0 + tid;
        if (p < n - 1) {
            cm_n = L.cm[p + 1];
            zs_n = L.zs[p + 1];
            st_n = L.st[p + 1];
            xw_n = L.xw[p + 1];
        }
        __syncthreads();
        if (p < n - 1) {
            L.cm[p] = cm_n;
            L.zs[p] = zs_n;
            L.st[p] = st_n;
            L.xw[p] = xw_n;
        }
        __syncthreads();
    }
    if (tid == 0) L.cf[L.nfree++] = freed;
    __syncthreads();
    if (tid < 64) {
        // lane owns positions col = lane + 64 t of the new map; cr: the row
        // being finished, nx: the next row, nn: the one after (prefetched).
        // Every load and store is unconditional, so that the compiler can
        // count the memory operations in flight and wait for the prefetch
        // only: lanes past the last position read and write the freed
        // physical column (dead until a later append rewrites it), and lanes
        // left of the pivot write row i of their column, below its diagonal,
        // where no reader of R looks.  Position i sits in slot i / 64, one
        // copy of the step per slot, so the slots left of it drop out
        // pc: element offset of the lane's physical column (< mt * mt, int)
        int pc[T];
#pragma unroll
        for (int t = 0; t < T; t++) {
            const int col = lane + 64 * t;
            pc[t] = ((col < n - 1) ? L.cm[col] : freed) * mt;
        }
        const int rj1 = min(j + 1, n - 1);
        double cr[T], nx[T];
#pragma unroll
        for (int t = 0; t < T; t++) cr[t] = A.R[pc[t] + j];
#pragma unroll
        for (int t = 0; t < T; t++) nx[t] = A.R[pc[t] + rj1];
        // T stores into the freed column after the first rows' loads: every
        // way into a step then has a step's stores and loads issued after the
        // next row's loads, so each step waits for its prefetch alone
#pragma unroll
        for (int t = 0; t < T; t++) A.R[(int64_t)freed * mt + min(j + t, n - 1)] = 0.0;
#pragma unroll
        for (int t0 = 0; t0 < T; t0++) {
            const int ilo = max(j, 64 * t0), ihi = min(n - 1, 64 * t0 + 64);
            for (int i = ilo; i < ihi; i++) {
                const int r2 = min(i + 2, n - 1);
                double nn[T];
#pragma unroll
                for (int t = t0; t < T; t++) nn[t] = A.R[pc[t] + r2];
                const double a = readlane_d(cr[t0], i & 63);
                const double b = readlane_d(nx[t0], i & 63);
                const double rr = sqrt(a * a + b * b);
                const double c = rr > 0.0 ? a / rr : 1.0, s = rr > 0.0 ? b / rr : 0.0;
#pragma unroll
                for (int t = t0; t < T; t++) {
                    A.R[pc[t] + i] = c * cr[t] + s * nx[t];
                    cr[t] = -s * cr[t] + c * nx[t];
                    nx[t] = nn[t];
                }
                if (lane == 0) {
                    L.gs[i][0] = c;
                    L.gs[i][1] = s;
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < r1; i += kStepThreads) {
        // the rows ahead are loaded unconditionally (clamped to the last
        // column, whose value is then never used), so that the waits stay on
        // the oldest of the three loads in flight
        double q = A.Q[(int64_t)j * r1 + i];
        double q1 = A.Q[(int64_t)min(j + 1, n - 1) * r1 + i];
        double q2 = A.Q[(int64_t)min(j + 2, n - 1) * r1 + i];
        for (int t = j; t < n - 1; t++) {
            const double q3 = A.Q[(int64_t)min(t + 3, n - 1) * r1 + i];
            const double c = L.gs[t][0], s = L.gs[t][1];
            A.Q[(int64_t)t * r1 + i] = c * q + s * q1;
            q = -s * q + c * q1;
            q1 = q2;
            q2 = q3;
        }
    }
    __syncthreads();
}

__device__ void finish(const SelArgs& A, int err) {
    if (threadIdx.x == 0) {
        A.st->err = err;
        A.st->done = 1;
    }
}

// steps 1 (argmax of the partial maxima) to 7 of one greedy iteration; T:
// positions per lane of the column removal (8 for mt <= 512, else 16)
template <int T>
__global__ void __launch_bounds__(kStepThreads) k_sel_step(SelArgs A) {
    if (A.st->done) return;
    __shared__ StepLds L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r = A.r, r1 = r + 1;
    // ---- step 1: the best candidate (max score, lowest index on ties)
    {
        double b = -INFINITY;
        int bi = INT32_MAX;
        for (int e = tid; e < A.nb; e += kStepThreads) {
            const double s = A.pscore[e];
            const int i = A.pidx[e];
            if (s > b || (s == b && i < bi)) {
                b = s;
                bi = i;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ob = __shfl_xor(b, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > b || (ob == b && oi < bi)) {
                b = ob;
                bi = oi;
            }
        }
        __shared__ double wb[kStepWaves];
        __shared__ int wi[kStepWaves];
        if (lane == 0) {
            wb[wave] = b;
            wi[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kStepWaves; w++)
                if (wb[w] > b || (wb[w] == b && wi[w] < bi)) {
                    b = wb[w];
                    bi = wi[w];
                }
            if (!(b > -INFINITY)) {
                for (int w = 0; w < kStepWaves; w++)
                    if (wi[w] < bi) bi = wi[w];
            }
            L.bidx = bi;
        }
        __syncthreads();
    }
    const int k = L.bidx;
    int n = A.st->n;
    const int it = A.st->iters;
    if (k == INT32_MAX || k < 0 || k >= A.M) {   // no candidate left
        finish(A, 0);
        return;
    }
    // the selection's state into LDS
    for (int c = tid; c < n; c += kStepThreads) {
        L.zs[c] = A.zsel[c];
        L.st[c] = A.stamp[c];
        L.cm[c] = A.cmap[c];
        L.xw[c] = A.x[c];
    }
    const int nf0 = A.st->nfree;
    for (int c = tid; c < nf0; c += kStepThreads) L.cf[c] = A.cfree[c];
    if (tid == 0) L.nfree = nf0;
    __syncthreads();
    // ---- step 2
    if (tid == 0) A.avail[k] = 0;
    const int navail = A.st->navail - 1;
    // ---- step 3: unrestricted least squares with column k appended
    load_col(A, k, L);
    double rel = qr_append(A, n, L);
    if (!(rel > 1e-12)) {
        finish(A, HROM_E_RANK);
        return;
    }
    if (tid == 0) {
        L.zs[n] = k;
        L.st[n] = it;
    }
    n++;
    __syncthreads();
    qr_solve(A, n, L, false);
    // ---- step 4
    int neg = 0;
    for (int c = tid; c < n; c += kStepThreads) neg |= (L.z[c] < 0.0) ? 1 : 0;
    neg = __syncthreads_or(neg);
    int ndrop = 0;
    if (!neg) {
        for (int c = tid; c < n; c += kStepThreads) L.xw[c] = L.z[c];
        residual(A, n, L);
    } else {
        // ---- steps 5 and 6: Lawson-Hanson NNLS, warm start at the previous
        // weights (positive on the first n - 1 columns) with w_k = 0.  Column k
        // enters the passive set at once -- the method's first outer step, its
        // dual entry j_k . res being its positive score -- and the inner loop
        // starts from the least-squares solution of step 3
        double cmax = 1.0;
        for (int c = tid; c < n; c += kStepThreads) cmax = fmax(cmax, A.csum[L.zs[c]]);
        for (int o = 32; o >= 1; o >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
        if (lane == 0) L.red[wave] = cmax;
        __syncthreads();
        for (int w = 0; w < kStepWaves; w++) cmax = fmax(cmax, L.red[w]);
        __syncthreads();
        const double tol = 1e-13 * cmax * fmax(1.0, fabs(A.V0));
        int nz = 0;
        int tc = k, ts = it;          // the column that entered last
        int guard = 3 * (n + 1) + 10;
        bool ok = false, first = true;
        if (tid == 0) L.xw[n - 1] = 0.0;
        __syncthreads();
        while (guard-- > 0) {
            // inner loop: z is the least-squares solution on the passive set
            while (guard-- > 0) {
                int allpos = 1;
                for (int c = tid; c < n; c += kStepThreads) allpos &= (L.z[c] > 0.0) ? 1 : 0;
                allpos = __syncthreads_and(allpos);
                if (allpos) {
                    for (int c = tid; c < n; c += kStepThreads) L.xw[c] = L.z[c];
                    for (int e = tid; e < nz; e += kStepThreads) L.zbl[e] = 0;
                    __syncthreads();
                    break;
                }
                if (first && !(L.z[n - 1] > 0.0)) {
                    // the entering column's own entry is not positive: set it aside
                    __syncthreads();
                    if (tid == 0) {
                        L.cf[L.nfree++] = L.cm[n - 1];
                        L.zl[nz] = tc;
                        L.zst[nz] = ts;
                        L.zbl[nz] = 1;
                    }
                    n--;
                    nz++;
                    __syncthreads();
                    break;
                }
                first = false;
                // move toward z until the first passive entry reaches zero
                if (tid == 0) {
                    double al = INFINITY;
                    for (int c = 0; c < n; c++)
                        if (!(L.z[c] > 0.0)) al = fmin(al, L.xw[c] / (L.xw[c] - L.z[c]));
                    L.bsc = al;
                }
                __syncthreads();
                const double al = L.bsc;
                for (int c = tid; c < n; c += kStepThreads) {
                    const bool at = !(L.z[c] > 0.0) && (L.xw[c] / (L.xw[c] - L.z[c]) == al);
                    const double nx = L.xw[c] + al * (L.z[c] - L.xw[c]);
                    L.xw[c] = (at || !(nx > 0.0)) ? 0.0 : nx;
                    L.h2[c] = (at || !(nx > 0.0)) ? 1.0 : 0.0;
                }
                __syncthreads();
                for (int c = n - 1; c >= 0; c--) {
                    if (L.h2[c] != 0.0) {
                        if (tid == 0) {
                            L.zl[nz] = L.zs[c];
                            L.zst[nz] = L.st[c];
                            L.zbl[nz] = 0;
                        }
                        nz++;
                        __syncthreads();
                        qr_remove<T>(A, c, n, L);
                        n--;
                    }
                }
                for (int e = tid; e < nz; e += kStepThreads) L.zbl[e] = 0;
                __syncthreads();
                qr_solve(A, n, L, false);
            }
            residual(A, n, L);     // c of the passive set is left by the last solve
            // outer: the dual entry of every non-passive, unblocked candidate
            for (int e = wave; e < nz; e += kStepWaves) {
                double sg = 0.0;
                if (!L.zbl[e]) {
                    const double* lk = A.lam + (int64_t)L.zl[e] * r;
                    for (int j = lane; j < r; j += 64) sg += lk[j] * L.res[j];
                    sg = wave_sum(sg) + L.res[r];
                } else {
                    sg = -INFINITY;
                }
                if (lane == 0) L.h2[e] = sg;
            }
            __syncthreads();
            if (tid == 0) {
                int t = -1;
                double gt = -INFINITY;
                for (int e = 0; e < nz; e++)
                    if (L.h2[e] > gt || (L.h2[e] == gt && t >= 0 && L.zst[e] < L.zst[t])) {
                        gt = L.h2[e];
                        t = e;
                    }
                L.bidx = (t >= 0 && gt > tol) ? t : -1;
            }
            __syncthreads();
            const int te = L.bidx;
            if (te < 0) {
                ok = true;
                break;
            }
            tc = L.zl[te];
            ts = L.zst[te];
            __syncthreads();
            if (tid == 0) {   // remove from the non-passive list
                for (int e = te; e < nz - 1; e++) {
                    L.zl[e] = L.zl[e + 1];
                    L.zst[e] = L.zst[e + 1];
                    L.zbl[e] = L.zbl[e + 1];
                }
            }
            nz--;
            __syncthreads();
            load_col(A, tc, L);
            rel = qr_append(A, n, L);
            if (!(rel > 1e-12)) {
                finish(A, HROM_E_RANK);
                return;
            }
            if (tid == 0) {
                L.zs[n] = tc;
                L.st[n] = ts;
                L.xw[n] = 0.0;
            }
            n++;
            first = true;
            __syncthreads();
            qr_solve(A, n, L, false);
        }
        if (!ok) {
            finish(A, HROM_E_NOCONV);
            return;
        }
        ndrop = nz;
    }
    // ---- step 7
    __syncthreads();
    for (int c = tid; c < n; c += kStepThreads) {
        A.x[c] = L.xw[c];
        A.zsel[c] = L.zs[c];
        A.stamp[c] = L.st[c];
        A.cmap[c] = L.cm[c];
    }
    for (int c = tid; c < L.nfree; c += kStepThreads) A.cfree[c] = L.cf[c];
    for (int i = tid; i < r1; i += kStepThreads) A.res[i] = L.res[i];
    if (tid == 0) {
        A.st->nfree = L.nfree;
        if (A.trace && it < A.trace_cap) {
            A.trace[4 * it + 0] = k;
            A.trace[4 * it + 1] = neg ? 1 : 0;
            A.trace[4 * it + 2] = ndrop;
            A.trace[4 * it + 3] = n;
        }
        A.st->n = n;
        A.st->iters = it + 1;
        A.st->navail = navail;
        if (n >= A.mt || navail <= 0) A.st->done = 1;
    }
}

// the selection in pick order
__global__ void k_sel_finish(SelArgs A, int n, int32_t* z, double* w) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int rk = 0;
    for (int q = 0; q < n; q++) rk += (A.stamp[q] < A.stamp[p]) ? 1 : 0;
    z[rk] = A.zsel[p];
    w[rk] = A.x[p];
}

}  // namespace ecm
}  // namespace hrom

using namespace hrom;
using namespace hrom::ecm;

namespace {

struct Arena {
    void* base = nullptr;
    size_t off = 0, size = 0;
    int alloc(size_t bytes) {
        size = bytes;
        return hipMalloc(&base, bytes) == hipSuccess ? HROM_OK : HROM_E_NOMEM;
    }
    template <typename T>
    T* take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T* p = (T*)((char*)base + off);
        off += sizeof(T) * std::max<size_t>(n, 1);
        return p;
    }
    ~Arena() {
        if (base) (void)hipFree(base);
    }
};

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

int launched() { return hipGetLastError() == hipSuccess ? HROM_OK : HROM_E_HIP; }

}  // namespace

extern "C" {

int hrom_ecm_training(int32_t m, int32_t M, const double* G, const double* w, const int32_t* phase,
                      const double* theta, int32_t p, const double* Fr, const double* a, double* xf,
                      double* fint, int32_t* nbad, hipStream_t stream) {
    if (m < 1 || M < 1 || p < 1 || !G || !w || !phase || !theta || !Fr || !a || !xf || !fint)
        return HROM_E_INVALID;
    const int64_t nm = 9LL * m;
    if (nm * (int64_t)M > (int64_t)1 << 40) return HROM_E_UNSUPPORTED;
    Arena ar;
    const size_t bytes = round256(sizeof(double) * nm * M) + 4096;
    if (ar.alloc(bytes) != HROM_OK) return HROM_E_NOMEM;
    double* Gt = ar.take<double>((size_t)(nm * M));
    double* V0 = ar.take<double>(1);
    int* bad = ar.take<int>(1);
    if (hipMemsetAsync(bad, 0, sizeof(int), stream) != hipSuccess) return HROM_E_HIP;
    hipLaunchKernelGGL(k_gt, dim3((M + 31) / 32, (unsigned)((nm + 31) / 32)), dim3(32, 8), 0, stream, G,
                       (int)nm, M, Gt);
    hipLaunchKernelGGL(k_integrand, dim3((M + 255) / 256, (p + kES - 1) / kES), dim3(256), 0, stream, Gt,
                       phase, theta, m, M, p, Fr, a, xf, bad);
    hipLaunchKernelGGL(k_volume, dim3(1), dim3(256), 0, stream, w, M, V0);
    hipLaunchKernelGGL(k_center, dim3((unsigned)((int64_t)p * (m + 9))), dim3(256), 0, stream, xf, w, M, V0,
                       fint);
    if (launched() != HROM_OK) return HROM_E_HIP;
    int hbad = 0;
    if (hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return HROM_E_HIP;
    if (nbad) *nbad = hbad;
    return HROM_OK;
}

}  // extern "C"

namespace hrom {
// the r leading left singular vectors of xf^T (xf [P][M]) into lam (row
// stride ld), all singular values into sigma; the Jacobi of hrom_ecm_svd
int svd_left(int P, int M, const double* xf, int r, double* lam, int ld, double* sigma, double tol,
             int max_sweeps, int* sweeps, double* off_hist, int method, hipStream_t stream) {
    if (P < 1 || M < 1 || r < 0 || r > P || ld < r || !xf || !sigma || (r > 0 && !lam) || method < 0 ||
        method > 2)
        return HROM_E_INVALID;
    if (!(tol > 0.0)) tol = 1e-13;
    if (max_sweeps <= 0) max_sweeps = 40;
    int nbk = (P + kSB - 1) / kSB;
    if (nbk < 2) nbk = 2;
    if (nbk & 1) nbk++;
    const int Ppad = nbk * kSB, npairs = nbk / 2, nrounds = nbk - 1;
    // QR first: on request (M >= Ppad), or for matrices with at least twice
    // as many rows as padded columns
    if (method == 2 && M < Ppad) return HROM_E_INVALID;
    const bool qr = method == 2 || (method == 0 && M >= 2 * Ppad);
    const int MJ = qr ? P : M;   // rows of the matrix the sweeps run on
    const int chunk_rows = qr ? 256 : 1024, nchunks = (MJ + chunk_rows - 1) / chunk_rows;
    const int qchunk = 1024, qmax = (M + qchunk - 1) / qchunk, npan = (P + kQB - 1) / kQB;
    // tournament schedule: block 0 fixed, the others rotate
    std::vector<int2> sched((size_t)nrounds * npairs);
    for (int t = 0; t < nrounds; t++) {
        auto pos = [&](int j) { return j == 0 ? 0 : 1 + (j - 1 + t) % (nbk - 1); };
        for (int i = 0; i < npairs; i++) {
            int a0 = pos(i), b0 = pos(nbk - 1 - i);
            sched[(size_t)t * npairs + i] = make_int2(std::min(a0, b0), std::max(a0, b0));
        }
    }
    Arena ar;
    size_t bytes = round256(sizeof(double) * (size_t)Ppad * M) + round256(sizeof(int2) * sched.size()) +
                   round256(sizeof(double) * (size_t)npairs * nchunks * kSW * kSW) +
                   round256(sizeof(double) * (size_t)npairs * kSW * kSW) + 2 * round256(sizeof(double) * Ppad) +
                   round256(sizeof(int) * Ppad) + 256 + round256(sizeof(int) * nbk) +
                   round256(sizeof(int2) * sched.size()) + round256(sizeof(int) * npairs) + 4096;
    if (qr)
        bytes += round256(sizeof(double) * (size_t)Ppad * M) + round256(sizeof(double) * (size_t)Ppad * P) +
                 round256(sizeof(double) * (size_t)std::max(r, 1) * M) +
                 round256(sizeof(double) * (size_t)(Ppad / kQB) * qmax * kQB * kQB) +
                 2 * round256(sizeof(double) * (size_t)kQB * Ppad) +
                 round256(sizeof(double) * (size_t)npan * kQB * kQB) + 3 * round256(sizeof(double) * Ppad) +
                 round256(sizeof(double) * (size_t)Ppad * P) + 2 * round256(sizeof(double) * P) +
                 3 * round256(sizeof(int) * P) + 4096;
    if (ar.alloc(bytes) != HROM_OK) return HROM_E_NOMEM;
    double* A = ar.take<double>((size_t)Ppad * M);
    int2* dsched = ar.take<int2>(sched.size());
    double* part = ar.take<double>((size_t)npairs * nchunks * kSW * kSW);
    double* Vb = ar.take<double>((size_t)npairs * kSW * kSW);
    double* sig = ar.take<double>(Ppad);
    double* sig_sorted = ar.take<double>(Ppad);
    int* perm = ar.take<int>(Ppad);
    unsigned long long* offmax = ar.take<unsigned long long>(1);
    int* ver = ar.take<int>(nbk);
    int2* pver = ar.take<int2>(sched.size());
    int* apply = ar.take<int>(npairs);
    double *V = nullptr, *Rm = nullptr, *X = nullptr, *qpart = nullptr, *Z = nullptr, *Wt = nullptr,
           *Tall = nullptr, *tau = nullptr, *beta = nullptr, *Bq = nullptr, *nu[2] = {nullptr, nullptr},
           *beta2 = nullptr;
    int *pm[2] = {nullptr, nullptr}, *iperm = nullptr;
    if (qr) {
        V = ar.take<double>((size_t)Ppad * M);
        Rm = ar.take<double>((size_t)Ppad * P);
        X = ar.take<double>((size_t)std::max(r, 1) * M);
        qpart = ar.take<double>((size_t)(Ppad / kQB) * qmax * kQB * kQB);
        Z = ar.take<double>((size_t)kQB * Ppad);
        Wt = ar.take<double>((size_t)kQB * Ppad);
        Tall = ar.take<double>((size_t)npan * kQB * kQB);
        tau = ar.take<double>(Ppad);
        beta = ar.take<double>(Ppad);
        Bq = ar.take<double>((size_t)Ppad * P);
        nu[0] = ar.take<double>(P);
        nu[1] = ar.take<double>(P);
        beta2 = ar.take<double>(Ppad);
        pm[0] = ar.take<int>(P);
        pm[1] = ar.take<int>(P);
        iperm = ar.take<int>(P);
    }
    if (hipMemcpyAsync(A, xf, sizeof(double) * (size_t)P * M, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
        hipMemsetAsync(A + (size_t)P * M, 0, sizeof(double) * (size_t)(Ppad - P) * M, stream) != hipSuccess ||
        hipMemcpyAsync(dsched, sched.data(), sizeof(int2) * sched.size(), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemsetAsync(ver, 0, sizeof(int) * nbk, stream) != hipSuccess ||
        hipMemsetAsync(pver, 0xff, sizeof(int2) * sched.size(), stream) != hipSuccess)
        return HROM_E_HIP;
    // products V_p^T X, then X -= V_p W with W = T^T (V_p^T X) or T (V_p^T X),
    // over the rows j0 .. of panel pn (V_p is zero above them)
    auto panel_apply = [&](int pn, double* Xc, int ncols, int trans) {
        const int j0 = pn * kQB, qn = (M - j0 + qchunk - 1) / qchunk;
        const double* Vp = V + (size_t)j0 * M;
        const int ct = (ncols + kQB - 1) / kQB;
        hipLaunchKernelGGL(k_qr_cross, dim3(ct, qn), dim3(256), 0, stream, Vp, Xc, M, j0, ncols, qchunk, qn, qpart);
        hipLaunchKernelGGL(k_qr_zsum, dim3((kQB * ncols + 255) / 256), dim3(256), 0, stream, qpart, qn, ncols, Z);
        hipLaunchKernelGGL(k_qr_tmul, dim3((kQB * ncols + 255) / 256), dim3(256), 0, stream,
                           Tall + (size_t)pn * kQB * kQB, Z, ncols, trans, Wt);
        hipLaunchKernelGGL(k_qr_update, dim3(ct, qn), dim3(256), 0, stream, Xc, Vp, M, j0, ncols, qchunk, Wt);
    };
    double* Jm = A;
    if (qr) {
        if (hipMemsetAsync(V, 0, sizeof(double) * (size_t)Ppad * M, stream) != hipSuccess ||
            hipMemsetAsync(tau, 0, sizeof(double) * Ppad, stream) != hipSuccess)
            return HROM_E_HIP;
        for (int pn = 0; pn < npan; pn++) {
            const int j0 = pn * kQB, j1 = std::min(P, j0 + kQB);
            for (int j = j0; j < j1; j++)
                hipLaunchKernelGGL(k_qr_col, dim3(j1 - j), dim3(1024), 0, stream, A, M, j, V, tau, beta);
            // T from Y = V_p^T V_p
            const int qn = (M - j0 + qchunk - 1) / qchunk;
            const double* Vp = V + (size_t)j0 * M;
            hipLaunchKernelGGL(k_qr_cross, dim3(1, qn), dim3(256), 0, stream, Vp, Vp, M, j0, kQB, qchunk, qn, qpart);
            hipLaunchKernelGGL(k_qr_zsum, dim3((kQB * kQB + 255) / 256), dim3(256), 0, stream, qpart, qn, kQB, Z);
            hipLaunchKernelGGL(k_qr_tbuild, dim3(1), dim3(kQB), 0, stream, Z, kQB, tau + j0,
                               Tall + (size_t)pn * kQB * kQB);
            // the trailing columns: A <- Q_p^T A
            if (P > j1) panel_apply(pn, A + (size_t)j1 * M, P - j1, 1);
        }
        // R^T Pi = Q2 R2 by Householder reflectors with column pivoting, one
        // launch per column; the sweeps then run on X = R2^T
        const int64_t nr = (int64_t)Ppad * P;
        const unsigned gr = (unsigned)((nr + 255) / 256);
        hipLaunchKernelGGL(k_qr_rtbuild, dim3(gr), dim3(256), 0, stream, A, M, beta, P, Ppad, Bq);
        hipLaunchKernelGGL(k_qrcp_init, dim3(P), dim3(256), 0, stream, Bq, P, nu[0], pm[0]);
        for (int j = 0; j < P; j++)
            hipLaunchKernelGGL(k_qrcp_col, dim3(P - j), dim3(256), 0, stream, Bq, P, j, pm[j & 1], nu[j & 1],
                               pm[(j + 1) & 1], nu[(j + 1) & 1], beta2);
        const int* pfin = pm[P & 1];
        hipLaunchKernelGGL(k_qrcp_xbuild, dim3(gr), dim3(256), 0, stream, Bq, P, Ppad, pfin, beta2, Rm);
        hipLaunchKernelGGL(k_qrcp_iperm, dim3((P + 255) / 256), dim3(256), 0, stream, pfin, P, iperm);
        if (launched() != HROM_OK) return HROM_E_HIP;
        Jm = Rm;
    }
    int sw = 0;
    bool conv = false;
    for (; sw < max_sweeps && !conv; sw++) {
        if (hipMemsetAsync(offmax, 0, sizeof(unsigned long long), stream) != hipSuccess) return HROM_E_HIP;
        for (int t = 0; t < nrounds; t++) {
            const int2* pr = dsched + (size_t)t * npairs;
            const int pbase = t * npairs;
            hipLaunchKernelGGL(k_svd_gram, dim3(npairs, nchunks), dim3(256), 0, stream, Jm, MJ, pr, chunk_rows,
                               nchunks, part, ver, pver, pbase);
            hipLaunchKernelGGL(k_svd_rotate, dim3(npairs), dim3(256), 0, stream, part, nchunks, tol, 1, Vb,
                               offmax, pr, ver, pver, pbase, apply);
            hipLaunchKernelGGL(k_svd_apply, dim3(npairs, nchunks), dim3(256), 0, stream, Jm, MJ, pr, Vb, apply,
                               chunk_rows);
        }
        if (launched() != HROM_OK) return HROM_E_HIP;
        unsigned long long hb = 0;
        if (hipMemcpyAsync(&hb, offmax, sizeof(hb), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return HROM_E_HIP;
        double off;
        std::memcpy(&off, &hb, sizeof(off));
        if (off_hist) off_hist[sw] = off;
        conv = !(off > tol);
    }
    if (sweeps) *sweeps = sw;
    hipLaunchKernelGGL(k_svd_norms, dim3(P), dim3(256), 0, stream, Jm, MJ, sig);
    hipLaunchKernelGGL(k_svd_rank, dim3((P + 255) / 256), dim3(256), 0, stream, sig, P, perm, sig_sorted);
    if (r > 0) {
        if (qr) {
            // left vectors of x_f^T = Q [Pi U_X; 0]: the rows of X's vectors
            // put back in R's row order, then the panels in reverse order
            const int64_t nx = (int64_t)r * M;
            hipLaunchKernelGGL(k_qr_xinit, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, stream, Jm, MJ, perm,
                               sig_sorted, iperm, r, M, X);
            for (int pn = npan - 1; pn >= 0; pn--) panel_apply(pn, X, r, 0);
            hipLaunchKernelGGL(k_qr_out, dim3((M + 31) / 32, (r + 31) / 32), dim3(32, 8), 0, stream, X, M, r, lam,
                               ld);
        } else {
            hipLaunchKernelGGL(k_svd_extract, dim3((M + 31) / 32, (r + 31) / 32), dim3(32, 8), 0, stream, A, M,
                               perm, sig_sorted, r, lam, ld);
        }
    }
    if (launched() != HROM_OK) return HROM_E_HIP;
    if (hipMemcpyAsync(sigma, sig_sorted, sizeof(double) * P, hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return HROM_E_HIP;
    // numerical rank: sigma_r at or below max(M, P) eps sigma_1 carries no
    // direction of the data
    double sr = 1.0, s1 = 1.0;
    if (r > 0 && (hipMemcpyAsync(&sr, sig_sorted + (r - 1), sizeof(double), hipMemcpyDeviceToHost, stream) !=
                      hipSuccess ||
                  hipMemcpyAsync(&s1, sig_sorted, sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess ||
                  hipStreamSynchronize(stream) != hipSuccess))
        return HROM_E_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return HROM_E_HIP;
    if (!conv) return HROM_E_NOCONV;
    if (!(sr > (double)std::max(M, P) * std::numeric_limits<double>::epsilon() * s1)) return HROM_E_RANK;
    return HROM_OK;
}
}  // namespace hrom

extern "C" {

int hrom_ecm_svd(int32_t P, int32_t M, const double* xf, int32_t r, double* lam, double* sigma, double tol,
                 int32_t max_sweeps, int32_t method, int32_t* sweeps, double* off_hist, hipStream_t stream) {
    return hrom::svd_left(P, M, xf, r, lam, r, sigma, tol, max_sweeps, sweeps, off_hist, method, stream);
}

int hrom_ecm_select(int32_t M, int32_t r, const double* lam, double V0, int32_t mt, int32_t* z, double* w,
                    int32_t* n_sel, int32_t* trace, int32_t trace_cap, int32_t* iters, hipStream_t stream) {
    if (M < 1 || r < 0 || mt < 1 || mt > r + 1 || r + 1 > kMaxRows || !z || !w || (r > 0 && !lam) ||
        !(std::isfinite(V0)))
        return HROM_E_INVALID;
    const int nb = std::min(1024, std::max(1, (M + 15) / 16));
    const int r1 = r + 1;
    Arena ar;
    const size_t bytes = round256(sizeof(double) * (size_t)M) * 2 + round256(M) +
                         round256(sizeof(double) * (size_t)mt * r1) + round256(sizeof(double) * (size_t)mt * mt) +
                         round256(sizeof(double) * mt) + 4 * round256(sizeof(int) * mt) +
                         round256(sizeof(double) * r1) + round256(sizeof(double) * nb) +
                         round256(sizeof(int) * nb) + round256(sizeof(State)) + 4096;
    if (ar.alloc(bytes) != HROM_OK) return HROM_E_NOMEM;
    SelArgs A{};
    A.lam = lam;
    A.M = M;
    A.r = r;
    A.mt = mt;
    A.V0 = V0;
    A.jn = ar.take<double>(M);
    A.csum = ar.take<double>(M);
    A.avail = ar.take<uint8_t>(M);
    A.Q = ar.take<double>((size_t)mt * r1);
    A.R = ar.take<double>((size_t)mt * mt);
    A.x = ar.take<double>(mt);
    A.zsel = ar.take<int>(mt);
    A.stamp = ar.take<int>(mt);
    A.cmap = ar.take<int>(mt);
    A.cfree = ar.take<int>(mt);
    A.res = ar.take<double>(r1);
    A.pscore = ar.take<double>(nb);
    A.pidx = ar.take<int>(nb);
    A.nb = nb;
    A.trace = trace;
    A.trace_cap = trace ? trace_cap : 0;
    A.st = ar.take<State>(1);
    const int gp = std::max(M, r1);
    hipLaunchKernelGGL(k_sel_prep, dim3((gp + 255) / 256), dim3(256), 0, stream, A);
    if (launched() != HROM_OK) return HROM_E_HIP;
    State hs{};
    const int64_t cap = (int64_t)M + 2;
    int64_t launched_iters = 0;
    for (;;) {
        for (int b = 0; b < 32; b++) {
            hipLaunchKernelGGL(k_sel_score, dim3(nb), dim3(256), 0, stream, A);
            if (mt <= 512) hipLaunchKernelGGL(k_sel_step<8>, dim3(1), dim3(kStepThreads), 0, stream, A);
            else hipLaunchKernelGGL(k_sel_step<16>, dim3(1), dim3(kStepThreads), 0, stream, A);
        }
        launched_iters += 32;
        if (launched() != HROM_OK) return HROM_E_HIP;
        if (hipMemcpyAsync(&hs, A.st, sizeof(State), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return HROM_E_HIP;
        if (hs.done) break;
        if (launched_iters > cap) return HROM_E_NOCONV;
    }
    if (hs.n > 0) hipLaunchKernelGGL(k_sel_finish, dim3((hs.n + 255) / 256), dim3(256), 0, stream, A, hs.n, z, w);
    if (launched() != HROM_OK || hipStreamSynchronize(stream) != hipSuccess) return HROM_E_HIP;
    if (n_sel) *n_sel = hs.n;
    if (iters) *iters = hs.iters;
    return hs.err;
}

}  // extern "C"
