// Static condensation of the ROM amplitudes at every macro point
// (Sec. 3.2.3, eq. Biot_Tangent): factor Kaa (Cholesky; LU with partial
// pivoting when a pivot is not positive, Sec. 4: factorise, never invert),
// solve y = Kaa^{-1} r and X = Kaa^{-1} KaF, and form
//   Palg = Pr - KaF^T y,   Cr = KFF - KaF^T X.
// One wavefront per macro point.  The SPD path keeps the point's augmented
// matrix in registers (condense_reg_body below); points with a non-positive
// pivot are finished by the full-matrix LU kernel, whose blocks live in LDS
// with rows distributed over lanes (row i on lane i mod 64).
#include <hip/hip_runtime.h>

#include "hrom_internal.h"

namespace hrom {

struct CondLds {
    int ld;
    double *K, *KaF, *KFF, *B, *Pr, *rv;
    __device__ CondLds(double* sm, int m) {
        ld = m + 1;
        K = sm;                 // [m][ld]
        KaF = K + m * ld;       // [m][9]
        KFF = KaF + 9 * m;      // [81]
        B = KFF + 81;           // [m][10]: r | KaF, overwritten by y | X
        Pr = B + 10 * m;        // [9]
        rv = Pr + 9;            // [m]
    }
};

static size_t cond_lds_bytes(int m) {
    return sizeof(double) * ((size_t)m * (m + 1) + 9 * m + 81 + 10 * m + 9 + m + 1);
}

// Row of accumulator element e held by lane group g inside a 16x16 tile:
// FP64 16x16x4 MFMA interleaves (row g + 4e), the 16-bit MFMAs with FP32
// accumulation keep rows contiguous per lane group (row 4g + e); the column
// is the lane index mod 16 in both.
template <typename TT>
__device__ __forceinline__ int acc_row(int g, int e);
template <>
__device__ __forceinline__ int acc_row<double>(int g, int e) { return g + 4 * e; }
template <>
__device__ __forceinline__ int acc_row<float>(int g, int e) { return 4 * g + e; }

// entry (xi, xk) of the symmetric augmented tangent (indices 0..m-1 modes,
// m..m+8 macro components) from a point's K-hat record
template <typename TT>
__device__ __forceinline__ double khat_at(const TT* kh, int m, int MT, int xi, int xk);

template <>
__device__ __forceinline__ double khat_at<double>(const double* kh, int m, int MT, int xi, int xk) {
    (void)m;
    const int lo = xi < xk ? xi : xk, hi = xi < xk ? xk : xi;
    const int ti = lo >> 4, tj = hi >> 4, rw = lo & 15, cl = hi & 15;
    const int idx = ti * MT - ti * (ti - 1) / 2 + (tj - ti);
    return kh[(int64_t)idx * 256 + (cl + 16 * (rw & 3)) * 4 + (rw >> 2)];
}

template <>
__device__ __forceinline__ double khat_at<float>(const float* kh, int m, int MT, int xi, int xk) {
    (void)MT;
    const int mp = 8 * ((m + 7) / 8);
    const int ci = xi < m ? xi : mp + (xi - m), ck = xk < m ? xk : mp + (xk - m);
    const int r = ci > ck ? ci : ck, c = ci > ck ? ck : ci;
    const int t = r >> 3, u = c >> 3;
    return (double)kh[(int64_t)(t * (t + 1) / 2 + u) * 64 + 8 * (r & 7) + (c & 7)];
}

template <typename TT>
__device__ void unpack_tiles(const CondenseArgs& A, const TT* kh, CondLds& S, bool kaa_only) {
    const int m = A.m, MT = A.MT, lane = threadIdx.x;
    const double ks = (double)*A.kscale;
    for (int e = lane; e < m * m; e += 64) {
        const int i = e / m, k = e % m;
        S.K[i * S.ld + k] = khat_at<TT>(kh, m, MT, i, k) * ks;
    }
    if (kaa_only) return;
    for (int e = lane; e < m * 9; e += 64) S.KaF[e] = khat_at<TT>(kh, m, MT, e / 9, m + e % 9) * ks;
    for (int e = lane; e < 81; e += 64) S.KFF[e] = khat_at<TT>(kh, m, MT, m + e / 9, m + e % 9) * ks;
}

// mode 0: export the raw blocks; 1: full condensation (Cholesky, LU on a
// non-positive pivot); 2: LU condensation of the points already flagged
// HROM_PT_NOT_SPD by the register kernel, every other point is skipped.
template <typename TT>
__global__ void __launch_bounds__(64) k_unpack_condense(CondenseArgs A, int mode) {
    extern __shared__ double sm[];
    const int m = A.m, lane = threadIdx.x;
    const int64_t pl = blockIdx.x;
    const int64_t b = A.first + pl;
    if (mode == 2 && !(A.status[b] & HROM_PT_NOT_SPD)) return;
    const int do_condense = mode;
    CondLds S(sm, m);
    const TT* kh = (const TT*)A.Khat + (int64_t)pl * khat_len(m, A.MT, sizeof(TT) == 4);
    unpack_tiles<TT>(A, kh, S, false);
    for (int i = lane; i < m; i += 64) {
        const double ri = A.r[(int64_t)i * A.count + pl];
        S.rv[i] = ri;
        S.B[i * 10] = ri;
    }
    if (lane < 9) S.Pr[lane] = A.Pr[(int64_t)lane * A.N + b];
    __syncthreads();
    for (int i = lane; i < m; i += 64)
#pragma unroll
        for (int J = 0; J < 9; J++) S.B[i * 10 + 1 + J] = S.KaF[i * 9 + J];

    if (!do_condense) {
        // test exports of the raw blocks
        if (A.outKaa)
            for (int e = lane; e < m * m; e += 64)
                A.outKaa[(int64_t)e * A.count + pl] = S.K[(e / m) * S.ld + (e % m)];
        if (A.outKaF)
            for (int e = lane; e < m * 9; e += 64) A.outKaF[(int64_t)e * A.count + pl] = S.KaF[e];
        if (A.outKFF)
            for (int e = lane; e < 81; e += 64) A.outKFF[(int64_t)e * A.N + b] = S.KFF[e];
        return;
    }
    __syncthreads();

    // ------------------------------------------------ Cholesky, right-looking
    // column j scaled by the pivot, then the trailing update of the lower
    // triangle spread over the 64 lanes in an 8 x 8 pattern (row i = j+1+r+8s,
    // column k = j+1+c+8t <= i): independent read-modify-writes.
    bool spd = (mode != 2);
    const int lr = lane >> 3, lcol = lane & 7;
    for (int j = 0; j < m && spd; j++) {
        const double d = S.K[j * S.ld + j];
        if (!(d > 0.0)) {
            spd = false;
            break;
        }
        const double sd = sqrt(d);
        __syncthreads();
        for (int i = j + 1 + lane; i < m; i += 64) S.K[i * S.ld + j] = S.K[i * S.ld + j] / sd;
        if (lane == 0) S.K[j * S.ld + j] = sd;
        __syncthreads();
        for (int i = j + 1 + lr; i < m; i += 8) {
            const double lij = S.K[i * S.ld + j];
            double* Ki = S.K + i * S.ld;
            for (int k = j + 1 + lcol; k <= i; k += 8) Ki[k] -= lij * S.K[k * S.ld + j];
        }
        __syncthreads();
    }
    int st = 0;
    int* piv = A.piv + pl * m;
    if (spd) {
        // L z = B, then L^T x = z (10 right-hand sides)
        for (int j = 0; j < m; j++) {
            __syncthreads();
            const double rjj = 1.0 / S.K[j * S.ld + j];
            double z[10];
#pragma unroll
            for (int r = 0; r < 10; r++) z[r] = S.B[j * 10 + r] * rjj;
            __syncthreads();
            for (int i = lane; i < m; i += 64) {
                if (i == j) {
#pragma unroll
                    for (int r = 0; r < 10; r++) S.B[j * 10 + r] = z[r];
                } else if (i > j) {
                    const double lij = S.K[i * S.ld + j];
#pragma unroll
                    for (int r = 0; r < 10; r++) S.B[i * 10 + r] -= lij * z[r];
                }
            }
        }
        for (int j = m - 1; j >= 0; j--) {
            __syncthreads();
            const double rjj = 1.0 / S.K[j * S.ld + j];
            double x[10];
#pragma unroll
            for (int r = 0; r < 10; r++) x[r] = S.B[j * 10 + r] * rjj;
            __syncthreads();
            for (int i = lane; i < m; i += 64) {
                if (i == j) {
#pragma unroll
                    for (int r = 0; r < 10; r++) S.B[j * 10 + r] = x[r];
                } else if (i < j) {
                    const double lji = S.K[j * S.ld + i];
#pragma unroll
                    for (int r = 0; r < 10; r++) S.B[i * 10 + r] -= lji * x[r];
                }
            }
        }
        if (lane == 0) piv[0] = -1;   // marks a Cholesky factor
    } else {
        // ------------------------------------------------ LU with partial pivoting
        st |= HROM_PT_NOT_SPD;
        __syncthreads();
        unpack_tiles<TT>(A, kh, S, true);
        for (int i = lane; i < m; i += 64) {
            S.B[i * 10] = S.rv[i];
#pragma unroll
            for (int J = 0; J < 9; J++) S.B[i * 10 + 1 + J] = S.KaF[i * 9 + J];
        }
        __syncthreads();
        for (int j = 0; j < m; j++) {
            // pivot: largest |K[i][j]|, i >= j, smallest index on ties
            double best = -1.0;
            int bi = j;
            for (int i = lane; i < m; i += 64) {
                if (i >= j) {
                    const double v = fabs(S.K[i * S.ld + j]);
                    if (v > best) { best = v; bi = i; }
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off);
                const int oi = __shfl_xor(bi, off);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (lane == 0) piv[j] = bi;
            if (!(best > 0.0)) {
                st |= HROM_PT_NONFINITE;
                break;
            }
            __syncthreads();
            if (bi != j) {
                for (int k = lane; k < m; k += 64) {
                    const double t = S.K[j * S.ld + k];
                    S.K[j * S.ld + k] = S.K[bi * S.ld + k];
                    S.K[bi * S.ld + k] = t;
                }
                if (lane < 10) {
                    const double t = S.B[j * 10 + lane];
                    S.B[j * 10 + lane] = S.B[bi * 10 + lane];
                    S.B[bi * 10 + lane] = t;
                }
            }
            __syncthreads();
            const double pj = S.K[j * S.ld + j];
            for (int i = lane; i < m; i += 64) {
                if (i > j) {
                    const double lij = S.K[i * S.ld + j] / pj;
                    S.K[i * S.ld + j] = lij;
                    for (int k = j + 1; k < m; k++) S.K[i * S.ld + k] -= lij * S.K[j * S.ld + k];
                }
            }
            __syncthreads();
        }
        if (!(st & HROM_PT_NONFINITE)) {
            for (int j = 0; j < m; j++) {   // unit lower
                __syncthreads();
                double z[10];
#pragma unroll
                for (int r = 0; r < 10; r++) z[r] = S.B[j * 10 + r];
                __syncthreads();
                for (int i = lane; i < m; i += 64)
                    if (i > j) {
                        const double lij = S.K[i * S.ld + j];
#pragma unroll
                        for (int r = 0; r < 10; r++) S.B[i * 10 + r] -= lij * z[r];
                    }
            }
            for (int j = m - 1; j >= 0; j--) {
                __syncthreads();
                const double rjj = 1.0 / S.K[j * S.ld + j];
                double x[10];
#pragma unroll
                for (int r = 0; r < 10; r++) x[r] = S.B[j * 10 + r] * rjj;
                __syncthreads();
                for (int i = lane; i < m; i += 64) {
                    if (i == j) {
#pragma unroll
                        for (int r = 0; r < 10; r++) S.B[j * 10 + r] = x[r];
                    } else if (i < j) {
                        const double uij = S.K[i * S.ld + j];
#pragma unroll
                        for (int r = 0; r < 10; r++) S.B[i * 10 + r] -= uij * x[r];
                    }
                }
            }
        }
    }
    __syncthreads();

    // ------------------------------------------------ condensation and outputs
    // Palg = Pr - KaF^T y (outputs 0..8), Cr = KFF - KaF^T X (outputs 9..89):
    // dot products over the modes with four independent partial sums
    bool fin = true;
    for (int o = lane; o < 90; o += 64) {
        const int I = (o < 9) ? o : (o - 9) / 9;
        const int col = (o < 9) ? 0 : 1 + (o - 9) % 9;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int k = 0;
        for (; k + 4 <= m; k += 4) {
            s0 = fma(S.KaF[k * 9 + I], S.B[k * 10 + col], s0);
            s1 = fma(S.KaF[(k + 1) * 9 + I], S.B[(k + 1) * 10 + col], s1);
            s2 = fma(S.KaF[(k + 2) * 9 + I], S.B[(k + 2) * 10 + col], s2);
            s3 = fma(S.KaF[(k + 3) * 9 + I], S.B[(k + 3) * 10 + col], s3);
        }
        for (; k < m; k++) s0 = fma(S.KaF[k * 9 + I], S.B[k * 10 + col], s0);
        const double dot = (s0 + s1) + (s2 + s3);
        if (o < 9) {
            const double v = S.Pr[o] - dot;
            A.Palg[(int64_t)o * A.N + b] = v;
            fin = fin && isfinite(v);
        } else {
            const double v = S.KFF[I * 9 + (col - 1)] - dot;
            A.Cr[(int64_t)(I * 9 + (col - 1)) * A.N + b] = v;
            fin = fin && isfinite(v);
        }
    }
    double rr = 0.0;
    for (int i = lane; i < m; i += 64) {
        rr += S.rv[i] * S.rv[i];
        A.y[(int64_t)i * A.count + pl] = S.B[i * 10];
        if (A.nmac == 6) {
            // the columns of the basis E6 (E11, E22, E33, E12 + E21, E23 + E32, E13 + E31)
            const double* Bi = S.B + i * 10 + 1;
            const double x6[6] = {Bi[0], Bi[4], Bi[8], Bi[1] + Bi[3], Bi[5] + Bi[7], Bi[2] + Bi[6]};
#pragma unroll
            for (int J = 0; J < 6; J++) A.X[((int64_t)i * 6 + J) * A.count + pl] = x6[J];
        } else {
#pragma unroll
            for (int J = 0; J < 9; J++) A.X[((int64_t)i * 9 + J) * A.count + pl] = S.B[i * 10 + 1 + J];
        }
        if (A.L) {
            double* Lrow = A.L + (pl * m + i) * (int64_t)m;
            for (int k = 0; k < m; k++) Lrow[k] = S.K[i * S.ld + k];
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rr += __shfl_xor(rr, off);
    const uint64_t bad = __ballot(!fin);
    if (lane == 0) {
        A.rnorm[b] = sqrt(rr);
        if (bad) st |= HROM_PT_NONFINITE;
        if (st) A.status[b] |= st;
    }
}

int launch_unpack_condense(const CondenseArgs& a, int mode, hipStream_t s) {
    const size_t bytes = cond_lds_bytes(a.m);
    if (bytes > 160 * 1024) return HROM_E_UNSUPPORTED;
    const dim3 grid((unsigned)a.count), block(64);
    if (a.mixed) {
        static bool attr = false;
        if (!attr) {
            hipFuncSetAttribute((const void*)k_unpack_condense<float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            attr = true;
        }
        hipLaunchKernelGGL(k_unpack_condense<float>, grid, block, bytes, s, a, mode);
    } else {
        static bool attr = false;
        if (!attr) {
            hipFuncSetAttribute((const void*)k_unpack_condense<double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            attr = true;
        }
        hipLaunchKernelGGL(k_unpack_condense<double>, grid, block, bytes, s, a, mode);
    }
    return HROM_OK;
}

// ---------------------------------------------------------------- refinement
// lambda <- lambda + Kaa~^{-1} rho with the stored factor of the evaluated
// (low-precision) Kaa~: one step of iterative refinement of the adjoint solve.
// One wavefront per point; x stays in registers (lane l holds rows l and
// l + 64, m <= 96) and x_j reaches every lane by readlane, so the
// substitutions need no LDS and no barrier.  The factor is read from HBM
// (each triangle once per substitution, only the entries a lane uses), the
// loads of sixteen steps (one 128-byte line of a row) issued ahead of their
// dependent updates.

__device__ __forceinline__ double lane_value(double v, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

// x_j of the vector held as (x0 on lane j, x1 on lane j - 64)
__device__ __forceinline__ double row_value(double x0, double x1, int j) {
    return j < 64 ? lane_value(x0, j) : lane_value(x1, j - 64);
}

// four points per workgroup, one per wavefront (no LDS, no barrier: the
// wavefronts are independent)
__global__ void __launch_bounds__(256) k_refine_lambda(RefineArgs A) {
    constexpr int U = 16;
    const int m = A.m, lane = threadIdx.x & 63;
    const int64_t pl = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pl >= A.count) return;
    const int64_t b = A.first + pl;
    if (A.status[b] & (HROM_PT_JNONPOS | HROM_PT_NONFINITE)) return;
    if (A.conv[pl]) return;
    const double* Lg = A.L + pl * (int64_t)m * m;
    const int* piv = A.piv + pl * m;
    const int i0 = lane, i1 = lane + 64;
    const bool h0 = i0 < m, h1 = i1 < m;
    double x0 = h0 ? A.rho[(int64_t)i0 * A.count + pl] : 0.0;
    double x1 = h1 ? A.rho[(int64_t)i1 * A.count + pl] : 0.0;
    const bool chol = (piv[0] < 0);
    if (!chol) {
        // the row interchanges of the LU factor, in order
        for (int j = 0; j < m; j++) {
            const int pj = piv[j];
            if (pj != j) {
                const double xj = row_value(x0, x1, j), xp = row_value(x0, x1, pj);
                if (i0 == j) x0 = xp;
                else if (i0 == pj) x0 = xj;
                if (i1 == j) x1 = xp;
                else if (i1 == pj) x1 = xj;
            }
        }
    }
    // forward: L z = x (unit diagonal for LU); lane i needs L[i][j]
    for (int j0 = 0; j0 < m; j0 += U) {
        double l0[U], l1[U], d[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int jj = min(j0 + u, m - 1);
            // only the entries left of the diagonal are used
            l0[u] = (h0 && jj < i0) ? Lg[(int64_t)i0 * m + jj] : 0.0;
            l1[u] = (h1 && jj < i1) ? Lg[(int64_t)i1 * m + jj] : 0.0;
            d[u] = Lg[(int64_t)jj * m + jj];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int j = j0 + u;
            if (j < m) {
                const double xj = row_value(x0, x1, j);
                const double z = chol ? xj / d[u] : xj;
                if (i0 == j) x0 = z;
                else if (i0 > j) x0 -= l0[u] * z;
                if (i1 == j) x1 = z;
                else if (i1 > j) x1 -= l1[u] * z;
            }
        }
    }
    // backward: L^T x = z (Cholesky, lane i needs L[j][i]) or U x = z (LU,
    // lane i needs U[i][j])
    for (int j0 = m - 1; j0 >= 0; j0 -= U) {
        double l0[U], l1[U], d[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int jj = max(j0 - u, 0);
            const int64_t a0 = chol ? (int64_t)jj * m + i0 : (int64_t)i0 * m + jj;
            const int64_t a1 = chol ? (int64_t)jj * m + i1 : (int64_t)i1 * m + jj;
            // only the entries of rows i < j are used
            l0[u] = (h0 && i0 < jj) ? Lg[a0] : 0.0;
            l1[u] = (h1 && i1 < jj) ? Lg[a1] : 0.0;
            d[u] = Lg[(int64_t)jj * m + jj];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int j = j0 - u;
            if (j >= 0) {
                const double z = row_value(x0, x1, j) / d[u];
                if (i0 == j) x0 = z;
                else if (i0 < j) x0 -= l0[u] * z;
                if (i1 == j) x1 = z;
                else if (i1 < j) x1 -= l1[u] * z;
            }
        }
    }
    double l0 = 0.0, l1 = 0.0;
    if (h0) {
        l0 = A.lam[(int64_t)i0 * A.count + pl] + x0;
        A.lam[(int64_t)i0 * A.count + pl] = l0;
    }
    if (h1) {
        l1 = A.lam[(int64_t)i1 * A.count + pl] + x1;
        A.lam[(int64_t)i1 * A.count + pl] = l1;
    }
    // stopping rule: the correction just applied is below tol of lambda
    double dd = x0 * x0 + x1 * x1, ll = l0 * l0 + l1 * l1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        dd += __shfl_xor(dd, off);
        ll += __shfl_xor(ll, off);
    }
    if (lane == 0) {
        if (dd <= A.tol * A.tol * ll) A.conv[pl] = 1;
        // after the last step a correction still above flag_tol of lambda
        // means lambda is not known to the accuracy of the mixed path
        else if (A.last && !(dd <= A.flag_tol * A.flag_tol * ll)) A.status[b] |= HROM_PT_NOREFINE;
    }
}

void launch_refine_lambda(const RefineArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_lambda, dim3((unsigned)((a.count + 3) / 4)), dim3(256), 0, s, a);
}

}  // namespace hrom


namespace hrom {

// ---------------------------------------------------------------------------
// Register-resident condensation (m <= 96): one wavefront per macro point.
//
// The symmetric augmented matrix
//     M = [[Kaa, KaF, r], [KaF^T, KFF, Pr], [r^T, Pr^T, 0]]
// is eliminated over its m mode pivots (LDL^T, no square roots).  The
// trailing 10 x 10 block is then the Schur complement
//     [[KFF - KaF^T Kaa^-1 KaF, Pr - KaF^T Kaa^-1 r], [., -r^T Kaa^-1 r]],
// i.e. the condensed RVE-frame tangent C_r and the algorithmic stress P_alg
// (Sec. 3.2.3), and the eliminated rows of [KaF | r] hold L^-1 [KaF | r];
// one backward substitution with D L^T gives X = Kaa^-1 KaF and y = Kaa^-1 r
// for the monolithic update.
//
// Index space: modes 0..m-1, identity padding up to mp = 8 ceil(m / 8), the
// nine macro components at mp..mp+8, the residual row at mp+9, zero padding
// to 8 MB.  The 8 x 8 lane grid (lr = lane / 8, lc = lane % 8) owns element
// (8t + lr, 8u + lc) of every lower block t >= u in register M[t(t+1)/2 + u];
// block indices are compile-time constants, so the matrix never leaves the
// register file.  Columns and rows are broadcast through a few LDS words.
// A non-positive pivot flags HROM_PT_NOT_SPD (the LU pass finishes the point).
// ---------------------------------------------------------------------------

__host__ __device__ constexpr int lblk(int t, int u) { return t * (t + 1) / 2 + u; }

// 1 / d for a pivot d > 0: hardware reciprocal refined by two Newton steps
// (a few units in the last place; shorter dependency chain than a division)
__device__ __forceinline__ double recip_pos(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// The register condensation runs one wavefront per workgroup: LDS accesses of
// one wavefront complete in issue order, so exchanging values between its
// lanes needs only a wavefront-scope fence (no hardware barrier)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// block -> point order: workgroups are dispatched round-robin over the eight
// XCDs; give each XCD a contiguous range of points so the component-major
// stores of neighbouring points meet in the same L2
__device__ __forceinline__ int64_t xcd_order(int64_t bid, int64_t n) {
    const int64_t q = n >> 3, rem = n & 7, x = bid & 7;
    return x * q + (x < rem ? x : rem) + (bid >> 3);
}

template <typename TT, int MB>
__device__ void condense_reg_body(const CondenseArgs& A, int64_t pl) {
    constexpr int NB = MB * (MB + 1) / 2;
    constexpr int JB = MB - 2;               // pivot blocks
    const int m = A.m, mp = 8 * JB, MT = A.MT;
    const int lane = threadIdx.x, lr = lane >> 3, lc = lane & 7;
    const int64_t b = A.first + pl;
    const TT* kh = (const TT*)A.Khat + (int64_t)pl * khat_len(m, MT, sizeof(TT) == 4);
    const double ks = (double)*A.kscale;
    __shared__ double cb[8 * MB];            // column / row broadcast
    __shared__ double zb[16];                // right-hand sides of one row

    // ---- gather the lower blocks of M from the K-hat tiles, r and Pr
    auto aug = [&](int i) {   // augmented K-hat index: -1 identity, -2 residual row, -3 zero
        return i < m ? i : (i < mp ? -1 : (i < mp + 9 ? m + i - mp : (i == mp + 9 ? -2 : -3)));
    };
    double M[NB];
    double rr = 0.0;
    // BATCH: all loads of the point are issued first, unconditionally, from
    // addresses inside their arrays (a placeholder address where the element
    // is not read); each loaded value gets an unconditional use (an empty asm
    // statement), so the compiler cannot sink a load into the branch that
    // reads it, where every load waits for the one before.  Only where the
    // loaded values fit the register budget next to the matrix.
    constexpr bool BATCH = sizeof(TT) == 4 ? MB <= 12 : MB <= 9;
    if constexpr (BATCH) {
        TT raw[NB];
        double rraw[MB];
#pragma unroll
        for (int t = 0; t < MB; t++) {
#pragma unroll
            for (int u = 0; u <= t; u++) {
                if constexpr (sizeof(TT) == 4) {
                    raw[lblk(t, u)] = kh[lblk(t, u) * 64 + lane];   // lane order, whole record
                } else {
                    const int xi = aug(8 * t + lr), xk = aug(8 * u + lc);
                    const bool kin = xi >= 0 && xk >= 0;
                    raw[lblk(t, u)] = khat_at<TT>(kh, m, MT, kin ? xi : 0, kin ? xk : 0);
                }
            }
        }
        // the residual row mp + 9 lies in block row JB + 1 (lane row 1): r
        // against the mode columns, Pr against the macro columns
#pragma unroll
        for (int u = 0; u < MB; u++) {
            const int xi = aug(8 * (JB + 1) + lr), xk = aug(8 * u + lc);
            const bool rrow = xi == -2 && xk >= 0, isr = rrow && xk < m;
            const double* rp = isr ? A.r + (int64_t)xk * A.count + pl
                                   : (rrow ? A.Pr + (int64_t)(xk - m) * A.N + b : A.r + pl);
            rraw[u] = *rp;
        }
#pragma unroll
        for (int e = 0; e < NB; e++) asm volatile("" ::"v"(raw[e]));
#pragma unroll
        for (int u = 0; u < MB; u++) asm volatile("" ::"v"(rraw[u]));
#pragma unroll
        for (int t = 0; t < MB; t++) {
#pragma unroll
            for (int u = 0; u <= t; u++) {
                const int i = 8 * t + lr, k = 8 * u + lc;
                const int xi = aug(i), xk = aug(k);
                double v = (xi >= 0 && xk >= 0) ? (double)raw[lblk(t, u)] * ks
                                                 : ((xi == -1 || xk == -1) ? (i == k ? 1.0 : 0.0) : 0.0);
                if (t == JB + 1 && xi == -2 && xk >= 0) {
                    v = rraw[u];
                    if (xk < m) rr = fma(v, v, rr);
                }
                M[lblk(t, u)] = v;
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < MB; t++) {
#pragma unroll
            for (int u = 0; u <= t; u++) {
                const int i = 8 * t + lr, k = 8 * u + lc;
                const int xi = aug(i), xk = aug(k);
                double v = 0.0;
                if (xi >= 0 && xk >= 0) {
                    if constexpr (sizeof(TT) == 4) v = (double)kh[lblk(t, u) * 64 + lane] * ks;
                    else v = khat_at<TT>(kh, m, MT, xi, xk) * ks;
                } else if (xi == -1 || xk == -1) {
                    v = (i == k) ? 1.0 : 0.0;
                } else if (xi == -2 && xk >= 0) {
                    if (xk < m) {
                        v = A.r[(int64_t)xk * A.count + pl];
                        rr = fma(v, v, rr);
                    } else {
                        v = A.Pr[(int64_t)(xk - m) * A.N + b];
                    }
                }
                M[lblk(t, u)] = v;
            }
        }
    }

    // ---- LDL^T elimination of the mp mode pivots (right-looking)
    bool spd = true;
#pragma unroll
    for (int J = 0; J < JB; J++) {
#pragma unroll 1
        for (int jj = 0; jj < 8; jj++) {
            const int j = 8 * J + jj;
            if (lc == jj) {
#pragma unroll
                for (int t = J; t < MB; t++) cb[8 * t + lr] = M[lblk(t, J)];
            }
            wave_sync();
            // a non-positive pivot is only flagged here: the sweep finishes
            // with meaningless values and the point goes to the LU pass
            const double d = cb[j];
            spd = spd && (d > 0.0);
            const double rd = recip_pos(d);
            double ck[MB];
#pragma unroll
            for (int u = J; u < MB; u++) {
                const double v = cb[8 * u + lc];
                ck[u] = (u > J || lc > jj) ? v : 0.0;
            }
#pragma unroll
            for (int t = J; t < MB; t++) {
                const double v = cb[8 * t + lr] * rd;
                const double ci = (t > J || lr > jj) ? v : 0.0;
#pragma unroll
                for (int u = J; u <= t; u++) M[lblk(t, u)] = fma(-ci, ck[u], M[lblk(t, u)]);
            }
            wave_sync();
        }
    }
    if (!spd) {
        if (lane == 0) A.status[b] |= HROM_PT_NOT_SPD;
        return;
    }

    // ---- optional Cholesky factor for the adjoint refinement: L = c / sqrt(d)
    if (A.L) {
        // pivots d_k of the lane's columns: diagonal (k, k) is held by lane (k%8, k%8)
        if (lr == lc) {
#pragma unroll
            for (int u = 0; u < JB; u++) cb[8 * u + lc] = M[lblk(u, u)];
        }
        wave_sync();
        double* Lp = A.L + pl * (int64_t)m * m;
#pragma unroll
        for (int t = 0; t < JB; t++)
#pragma unroll
            for (int u = 0; u <= t; u++) {
                const int i = 8 * t + lr, k = 8 * u + lc;
                if (i < m && k <= i) {
                    const double sk = sqrt(cb[k]);
                    Lp[(int64_t)i * m + k] = (i == k) ? sk : M[lblk(t, u)] / sk;
                }
            }
        wave_sync();
    }
    if (lane == 0) A.piv[pl * m] = -1;

    // ---- backward substitution (D L^T) [X | y] = L^-1 [KaF | r], right-looking
    // right-hand side c = lr in block JB, c = 8 + lr (lr < 2) in block JB + 1
#pragma unroll
    for (int J = JB - 1; J >= 0; J--) {
#pragma unroll 1
        for (int jj = 7; jj >= 0; jj--) {
            const int j = 8 * J + jj;
            if (lr == jj) {
#pragma unroll
                for (int u = 0; u <= J; u++) cb[8 * u + lc] = M[lblk(J, u)];
            }
            if (lc == jj) {
                zb[lr] = M[lblk(JB, J)];
                zb[8 + lr] = M[lblk(JB + 1, J)];
            }
            wave_sync();
            const double rdj = recip_pos(cb[j]);
            const double x0 = zb[lr] * rdj;
            const double x1 = (lr < 2) ? zb[8 + lr] * rdj : 0.0;
            if (lc == jj) {
                M[lblk(JB, J)] = x0;
                M[lblk(JB + 1, J)] = x1;
            }
#pragma unroll
            for (int u = 0; u <= J; u++) {
                const double l = (u < J || lc < jj) ? cb[8 * u + lc] : 0.0;
                M[lblk(JB, u)] = fma(-l, x0, M[lblk(JB, u)]);
                M[lblk(JB + 1, u)] = fma(-l, x1, M[lblk(JB + 1, u)]);
            }
            wave_sync();
        }
    }

    // ---- outputs: y, X (mode-indexed, component-major), P_alg, C_r, rnorm
#pragma unroll
    for (int u = 0; u < JB; u++) {
        const int i = 8 * u + lc;
        if (i < m) {
            A.X[((int64_t)i * 9 + lr) * A.count + pl] = M[lblk(JB, u)];
            if (lr == 0) A.X[((int64_t)i * 9 + 8) * A.count + pl] = M[lblk(JB + 1, u)];
            if (lr == 1) A.y[(int64_t)i * A.count + pl] = M[lblk(JB + 1, u)];
        }
    }
    bool fin = true;
    {
        // C_r rows/cols 0..7: block (JB, JB), full 8 x 8 (symmetric updates)
        const double c0 = M[lblk(JB, JB)];
        A.Cr[(int64_t)(lr * 9 + lc) * A.N + b] = c0;
        fin = fin && isfinite(c0);
        if (lr == 0) {          // row / column 8 of C_r from block (JB + 1, JB)
            const double c8 = M[lblk(JB + 1, JB)];
            A.Cr[(int64_t)(8 * 9 + lc) * A.N + b] = c8;
            A.Cr[(int64_t)(lc * 9 + 8) * A.N + b] = c8;
            fin = fin && isfinite(c8);
            if (lc == 0) {
                const double c88 = M[lblk(JB + 1, JB + 1)];
                A.Cr[(int64_t)80 * A.N + b] = c88;
                fin = fin && isfinite(c88);
            }
        } else if (lr == 1) {   // residual row: P_alg
            const double p0 = M[lblk(JB + 1, JB)];
            A.Palg[(int64_t)lc * A.N + b] = p0;
            fin = fin && isfinite(p0);
            if (lc == 0) {
                const double p8 = M[lblk(JB + 1, JB + 1)];
                A.Palg[(int64_t)8 * A.N + b] = p8;
                fin = fin && isfinite(p8);
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rr += __shfl_xor(rr, off);
    const uint64_t bad = __ballot(!fin);
    if (lane == 0) {
        A.rnorm[b] = sqrt(rr);
        if (bad) A.status[b] |= HROM_PT_NONFINITE;
    }
}

// OCC: wavefronts per SIMD the register budget is cut for (3 lets a few
// bytes spill at the largest blocks, 2 spills nothing); m > 64 always 2
template <typename TT, int MB, int OCC>
__global__ void __launch_bounds__(64, OCC) k_condense_reg(CondenseArgs A) {
    condense_reg_body<TT, MB>(A, xcd_order(blockIdx.x, A.count));
}

template <typename TT>
static void launch_reg_t(const CondenseArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)a.count), block(64);
    const bool o2 = a.variant == 1;
#define HROM_REG(MB_)                                                                          \
    if (o2 || (MB_) > 10) hipLaunchKernelGGL((k_condense_reg<TT, MB_, 2>), grid, block, 0, s, a); \
    else hipLaunchKernelGGL((k_condense_reg<TT, MB_, (MB_) <= 10 ? 3 : 2>), grid, block, 0, s, a);
    switch ((a.m + 7) / 8) {
        case 1: { HROM_REG(3) } break;
        case 2: { HROM_REG(4) } break;
        case 3: { HROM_REG(5) } break;
        case 4: { HROM_REG(6) } break;
        case 5: { HROM_REG(7) } break;
        case 6: { HROM_REG(8) } break;
        case 7: { HROM_REG(9) } break;
        case 8: { HROM_REG(10) } break;
        // m = 65 .. 96: two wavefronts per SIMD
        case 9: { HROM_REG(11) } break;
        case 10: { HROM_REG(12) } break;
        case 11: { HROM_REG(13) } break;
        default: { HROM_REG(14) } break;
    }
#undef HROM_REG
}

// ---------------------------------------------------------------------------
// Six-component (Biot) condensation of objective plans: the RVE is driven by
// the symmetric stretch Ubar (Sec. 3.2.2), so the macro degrees of freedom
// are the six coordinates of Ubar in the basis E6 = {E11, E22, E33, E12 + E21,
// E23 + E32, E13 + E31}: KaU = KaF E6 (m x 6), KUU = E6^T KFF E6, PU = E6^T Pr,
// and six right-hand sides.  The augmented matrix [[Kaa, KaU, r], [., KUU, PU],
// [., ., 0]] then has one trailing 8 x 8 block (six components, the residual
// row at mp + 6, one zero row) instead of two.  Outputs: X6 = Kaa^{-1} KaU
// [6m][count], y, and the symmetric projections of the condensed stress and
// tangent, Palg = sum_k D_k (E6_k : Palg) and Cr = sum_kl D_k (E6_k : Cr :
// E6_l) D_l^T with the dual basis D_k (E11, .., (E12 + E21) / 2, ..), which is
// all that the objective push-out reads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int e6_count(int k) { return k < 3 ? 1 : 2; }
// the row-major 3x3 components of E6_k
__device__ __forceinline__ int e6_comp(int k, int n) {
    switch (k) {
        case 0: return 0;
        case 1: return 4;
        case 2: return 8;
        case 3: return n ? 3 : 1;
        case 4: return n ? 7 : 5;
        default: return n ? 6 : 2;
    }
}

template <typename TT, int MB>
__device__ void condense6_reg_body(const CondenseArgs& A, int64_t pl) {
    constexpr int NB = MB * (MB + 1) / 2;
    constexpr int JB = MB - 1;               // pivot blocks
    const int m = A.m, mp = 8 * JB, MT = A.MT;
    const int lane = threadIdx.x, lr = lane >> 3, lc = lane & 7;
    const int64_t b = A.first + pl;
    const TT* kh = (const TT*)A.Khat + (int64_t)pl * khat_len(m, MT, sizeof(TT) == 4);
    const double ks = (double)*A.kscale;
    __shared__ double cb[8 * MB];
    __shared__ double zb[8];

    double M[NB];
    double rr = 0.0;
    // ---- mode blocks (t, u < JB): the same K-hat entries as the nine-component layout
    {
        TT raw[JB * (JB + 1) / 2];
#pragma unroll
        for (int t = 0; t < JB; t++)
#pragma unroll
            for (int u = 0; u <= t; u++) {
                if constexpr (sizeof(TT) == 4) {
                    raw[lblk(t, u)] = kh[lblk(t, u) * 64 + lane];
                } else {
                    const int i = 8 * t + lr, k = 8 * u + lc;
                    const bool kin = i < m && k < m;
                    raw[lblk(t, u)] = khat_at<TT>(kh, m, MT, kin ? i : 0, kin ? k : 0);
                }
            }
#pragma unroll
        for (int t = 0; t < JB; t++)
#pragma unroll
            for (int u = 0; u <= t; u++) {
                const int i = 8 * t + lr, k = 8 * u + lc;
                double v;
                if (i < m && k < m) v = (double)raw[lblk(t, u)] * ks;
                else v = (i == k) ? 1.0 : 0.0;       // identity padding of the modes
                M[lblk(t, u)] = v;
            }
    }
    // ---- trailing block row JB: KaU, KUU, PU and the residual row
    {
        const int ci = lr;   // 0..5 component, 6 residual, 7 zero
#pragma unroll
        for (int u = 0; u <= JB; u++) {
            const int k = 8 * u + lc;
            double v = 0.0;
            if (u < JB) {
                if (k < m) {
                    if (ci < 6) {
                        for (int n = 0; n < e6_count(ci); n++)
                            v += (double)khat_at<TT>(kh, m, MT, m + e6_comp(ci, n), k);
                        v *= ks;
                    } else if (ci == 6) {
                        v = A.r[(int64_t)k * A.count + pl];
                        rr = fma(v, v, rr);
                    }
                }
            } else {
                const int cj = lc;
                if (ci < 6 && cj < 6) {
                    for (int n = 0; n < e6_count(ci); n++)
                        for (int n2 = 0; n2 < e6_count(cj); n2++)
                            v += (double)khat_at<TT>(kh, m, MT, m + e6_comp(ci, n), m + e6_comp(cj, n2));
                    v *= ks;
                } else if ((ci < 6 && cj == 6) || (ci == 6 && cj < 6)) {
                    const int cc = ci < 6 ? ci : cj;
                    for (int n = 0; n < e6_count(cc); n++) v += A.Pr[(int64_t)e6_comp(cc, n) * A.N + b];
                }
            }
            M[lblk(JB, u)] = v;
        }
    }

    // ---- LDL^T elimination of the mp mode pivots (right-looking)
    bool spd = true;
#pragma unroll
    for (int J = 0; J < JB; J++) {
#pragma unroll 1
        for (int jj = 0; jj < 8; jj++) {
            const int j = 8 * J + jj;
            if (lc == jj) {
#pragma unroll
                for (int t = J; t < MB; t++) cb[8 * t + lr] = M[lblk(t, J)];
            }
            wave_sync();
            const double d = cb[j];
            spd = spd && (d > 0.0);
            const double rd = recip_pos(d);
            double ck[MB];
#pragma unroll
            for (int u = J; u < MB; u++) {
                const double v = cb[8 * u + lc];
                ck[u] = (u > J || lc > jj) ? v : 0.0;
            }
#pragma unroll
            for (int t = J; t < MB; t++) {
                const double v = cb[8 * t + lr] * rd;
                const double ci = (t > J || lr > jj) ? v : 0.0;
#pragma unroll
                for (int u = J; u <= t; u++) M[lblk(t, u)] = fma(-ci, ck[u], M[lblk(t, u)]);
            }
            wave_sync();
        }
    }
    spd = __ballot(!spd) == 0;
    if (!spd) {
        if (lane == 0) A.status[b] |= HROM_PT_NOT_SPD;
        return;
    }
    if (A.L) {
        if (lr == lc) {
#pragma unroll
            for (int u = 0; u < JB; u++) cb[8 * u + lc] = M[lblk(u, u)];
        }
        wave_sync();
        double* Lp = A.L + pl * (int64_t)m * m;
#pragma unroll
        for (int t = 0; t < JB; t++)
#pragma unroll
            for (int u = 0; u <= t; u++) {
                const int i = 8 * t + lr, k = 8 * u + lc;
                if (i < m && k <= i) {
                    const double sk = sqrt(cb[k]);
                    Lp[(int64_t)i * m + k] = (i == k) ? sk : M[lblk(t, u)] / sk;
                }
            }
        wave_sync();
    }
    if (lane == 0) A.piv[pl * m] = -1;

    // ---- backward substitution (D L^T) [X6 | y] = L^-1 [KaU | r]: right-hand
    // side c = lr of block JB
#pragma unroll
    for (int J = JB - 1; J >= 0; J--) {
#pragma unroll 1
        for (int jj = 7; jj >= 0; jj--) {
            const int j = 8 * J + jj;
            if (lr == jj) {
#pragma unroll
                for (int u = 0; u <= J; u++) cb[8 * u + lc] = M[lblk(J, u)];
            }
            if (lc == jj) zb[lr] = M[lblk(JB, J)];
            wave_sync();
            const double x0 = zb[lr] * recip_pos(cb[j]);
            if (lc == jj) M[lblk(JB, J)] = x0;
#pragma unroll
            for (int u = 0; u <= J; u++) {
                const double l = (u < J || lc < jj) ? cb[8 * u + lc] : 0.0;
                M[lblk(JB, u)] = fma(-l, x0, M[lblk(JB, u)]);
            }
            wave_sync();
        }
    }

    // ---- outputs: X6, y; the symmetric projections of P_alg and C_r
#pragma unroll
    for (int u = 0; u < JB; u++) {
        const int i = 8 * u + lc;
        if (i < m) {
            if (lr < 6) A.X[((int64_t)i * 6 + lr) * A.count + pl] = M[lblk(JB, u)];
            else if (lr == 6) A.y[(int64_t)i * A.count + pl] = M[lblk(JB, u)];
        }
    }
    bool fin = true;
    {
        const double v = M[lblk(JB, JB)];   // entry (lr, lc) of the trailing block
        const double dr = lr < 3 ? 1.0 : 0.5, dc = lc < 3 ? 1.0 : 0.5;
        if (lr < 6 && lc < 6) {
            fin = isfinite(v);
            for (int n = 0; n < e6_count(lr); n++)
                for (int n2 = 0; n2 < e6_count(lc); n2++)
                    A.Cr[(int64_t)(9 * e6_comp(lr, n) + e6_comp(lc, n2)) * A.N + b] = v * dr * dc;
        } else if (lr == 6 && lc < 6) {
            fin = isfinite(v);
            for (int n = 0; n < e6_count(lc); n++) A.Palg[(int64_t)e6_comp(lc, n) * A.N + b] = v * dc;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rr += __shfl_xor(rr, off);
    const uint64_t bad = __ballot(!fin);
    if (lane == 0) {
        A.rnorm[b] = sqrt(rr);
        if (bad) A.status[b] |= HROM_PT_NONFINITE;
    }
}

template <typename TT, int MB, int OCC>
__global__ void __launch_bounds__(64, OCC) k_condense6_reg(CondenseArgs A) {
    condense6_reg_body<TT, MB>(A, xcd_order(blockIdx.x, A.count));
}

template <typename TT>
static void launch_reg6_t(const CondenseArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)a.count), block(64);
    const bool o2 = a.variant == 1;
#define HROM_REG6(MB_)                                                                          \
    if (o2 || (MB_) > 10) hipLaunchKernelGGL((k_condense6_reg<TT, MB_, 2>), grid, block, 0, s, a); \
    else hipLaunchKernelGGL((k_condense6_reg<TT, MB_, (MB_) <= 10 ? 3 : 2>), grid, block, 0, s, a);
    switch ((a.m + 7) / 8) {
        case 1: { HROM_REG6(2) } break;
        case 2: { HROM_REG6(3) } break;
        case 3: { HROM_REG6(4) } break;
        case 4: { HROM_REG6(5) } break;
        case 5: { HROM_REG6(6) } break;
        case 6: { HROM_REG6(7) } break;
        case 7: { HROM_REG6(8) } break;
        case 8: { HROM_REG6(9) } break;
        case 9: { HROM_REG6(10) } break;
        case 10: { HROM_REG6(11) } break;
        case 11: { HROM_REG6(12) } break;
        default: { HROM_REG6(13) } break;
    }
#undef HROM_REG6
}

int launch_condense_reg(const CondenseArgs& a, hipStream_t s) {
    if (a.m < 1 || a.m > 96) return HROM_E_UNSUPPORTED;
    if (a.count == 0) return HROM_OK;
    if (a.nmac == 6) {
        if (a.mixed) launch_reg6_t<float>(a, s);
        else launch_reg6_t<double>(a, s);
        return HROM_OK;
    }
    if (a.mixed) launch_reg_t<float>(a, s);
    else launch_reg_t<double>(a, s);
    return HROM_OK;
}

}  // namespace hrom

namespace hrom {
// dynamic-LDS limits, set once before any launch (also before graph capture)
void set_kernel_attributes() {
    const int lim = 160 * 1024;
    hipFuncSetAttribute((const void*)k_unpack_condense<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void*)k_unpack_condense<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void*)k_refine_lambda, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}
}  // namespace hrom
