// Adjoint backward through the converged ROM state.  With the RVE-frame
// cotangent g_r and the adjoint solution lambda = Kaa^{-T} KaF g_r, every ECM
// point is re-evaluated (F_q and the tangent are recomputed, never stored):
//   v_q   = g_r - G_q lambda
//   h_r  += w_q A_q v_q                               (= Cr^T g_r)
//   dmu_p  += w_q v_q : (F_q - F_q^{-T}),  dlam_p += w_q v_q : (ln J_q F_q^{-T})
// for the phase p of q.  Optionally the refinement residual
//   rho = sum_q G_q^T (w_q A_q v_q)  (= KaF g_r - Kaa lambda)
// of the adjoint system is accumulated with the same operator.
// One wavefront per macro point, lane = ECM point.
#include <hip/hip_runtime.h>

#include "hrom_internal.h"

namespace hrom {

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// (A : v)_ij = mu v_ij + (mu - lam ln J) (Fi v Fi)_ji + lam Fi_ji tr(Fi v)
template <typename T>
__device__ __forceinline__ void nh_apply(const T* Fi, T mu, T la, T ell, const T* v, T* Av) {
    T FiV[9], FVF[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            FiV[3 * i + j] = Fi[3 * i] * v[j] + Fi[3 * i + 1] * v[3 + j] + Fi[3 * i + 2] * v[6 + j];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            FVF[3 * i + j] = FiV[3 * i] * Fi[j] + FiV[3 * i + 1] * Fi[3 + j] + FiV[3 * i + 2] * Fi[6 + j];
    const T tr = FiV[0] + FiV[4] + FiV[8];
    const T cm = mu - la * ell;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            Av[3 * i + j] = mu * v[3 * i + j] + cm * FVF[3 * j + i] + la * Fi[3 * j + i] * tr;
}

__global__ void __launch_bounds__(256) k_backward_q(BackwardArgs A) {
    __shared__ double s_a[4][kMaxModes];
    __shared__ double s_l[4][kMaxModes];
    __shared__ double s_v[4][9 * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t pl = (int64_t)blockIdx.x * 4 + wave;
    const bool valid = pl < A.count;
    if (!valid) pl = A.count - 1;
    const int64_t b = A.first + pl;
    const int m = A.m;
    for (int k = lane; k < m; k += 64) {
        s_a[wave][k] = A.a[(int64_t)k * A.count + pl];
        s_l[wave][k] = A.lam[(int64_t)k * A.count + pl];
    }
    double Fr[9], gr[9];
#pragma unroll
    for (int I = 0; I < 9; I++) {
        Fr[I] = A.Fr[I * A.N + b];
        gr[I] = A.gr[I * A.N + b];
    }
    const double mu0 = A.theta[0], la0 = A.theta[1], mu1 = A.theta[2], la1 = A.theta[3];
    double h[9], gt[4];
#pragma unroll
    for (int I = 0; I < 9; I++) h[I] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++) gt[i] = 0.0;
    double rho0 = 0.0, rho1 = 0.0;
    int bits = 0;
    __syncthreads();
    for (int q0 = 0; q0 < A.Qpad; q0 += 64) {
        const int q = q0 + lane;
        double F[9], v[9];
#pragma unroll
        for (int I = 0; I < 9; I++) {
            F[I] = Fr[I];
            v[I] = gr[I];
        }
        const double* gt_ = A.GT + (int64_t)(q0 >> 6) * 9 * m * 64 + lane;
        for (int k = 0; k < m; k++) {
            const double ak = s_a[wave][k], lk = s_l[wave][k];
#pragma unroll
            for (int I = 0; I < 9; I++) {
                const double gv = gt_[(int64_t)(I * m + k) * 64];
                F[I] = fma(ak, gv, F[I]);
                v[I] = fma(-lk, gv, v[I]);
            }
        }
        const double wq = A.w[q];
        const int p = A.phase[q];
        const double mu = p ? mu1 : mu0, la = p ? la1 : la0;
        const double c00 = F[4] * F[8] - F[5] * F[7];
        const double c01 = F[5] * F[6] - F[3] * F[8];
        const double c02 = F[3] * F[7] - F[4] * F[6];
        const double J = F[0] * c00 + F[1] * c01 + F[2] * c02;
        const bool ok = (q < A.Q) && (J > 0.0);
        if (q < A.Q && !(J > 0.0)) bits |= HROM_PT_JNONPOS;
        double Fi[9];
        {
            const double id = 1.0 / J;
            Fi[0] = c00 * id;
            Fi[3] = c01 * id;
            Fi[6] = c02 * id;
            Fi[1] = (F[2] * F[7] - F[1] * F[8]) * id;
            Fi[4] = (F[0] * F[8] - F[2] * F[6]) * id;
            Fi[7] = (F[1] * F[6] - F[0] * F[7]) * id;
            Fi[2] = (F[1] * F[5] - F[2] * F[4]) * id;
            Fi[5] = (F[2] * F[3] - F[0] * F[5]) * id;
            Fi[8] = (F[0] * F[4] - F[1] * F[3]) * id;
        }
        const double ell = ok ? log(J) : 0.0;
        double Av[9];
        if (A.mixed) {
            float Fif[9], vf[9], Avf[9];
#pragma unroll
            for (int k = 0; k < 9; k++) {
                Fif[k] = (float)Fi[k];
                vf[k] = (float)v[k];
            }
            nh_apply<float>(Fif, (float)mu, (float)la, (float)ell, vf, Avf);
#pragma unroll
            for (int k = 0; k < 9; k++) Av[k] = (double)Avf[k];
        } else {
            nh_apply<double>(Fi, mu, la, ell, v, Av);
        }
        double dmu = 0.0, dla = 0.0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                dmu = fma(v[3 * i + j], F[3 * i + j] - Fi[3 * j + i], dmu);
                dla = fma(v[3 * i + j], ell * Fi[3 * j + i], dla);
            }
        const double wo = ok ? wq : 0.0;
#pragma unroll
        for (int I = 0; I < 9; I++) h[I] = fma(wo, Av[I], h[I]);
        const double wm = p ? 0.0 : wo, wi = p ? wo : 0.0;
        gt[0] = fma(wm, dmu, gt[0]);
        gt[1] = fma(wm, dla, gt[1]);
        gt[2] = fma(wi, dmu, gt[2]);
        gt[3] = fma(wi, dla, gt[3]);
        if (A.with_rho) {
#pragma unroll
            for (int I = 0; I < 9; I++) s_v[wave][I * 64 + lane] = wo * Av[I];
            __syncthreads();
            const double* gh = A.Ghat + (int64_t)q0 * 9 * A.MP;
            for (int qq = 0; qq < 64; qq++) {
#pragma unroll
                for (int I = 0; I < 9; I++) {
                    const double sv = s_v[wave][I * 64 + qq];
                    const double* row = gh + (int64_t)(qq * 9 + I) * A.MP;
                    if (lane < m) rho0 = fma(sv, row[lane], rho0);
                    if (lane + 64 < m) rho1 = fma(sv, row[lane + 64], rho1);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int I = 0; I < 9; I++)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) h[I] += __shfl_xor(h[I], off);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) gt[i] += __shfl_xor(gt[i], off);
    const uint64_t bad = __ballot(bits);
    if (!valid) return;
    const bool failed = (A.status[b] & (HROM_PT_JNONPOS | HROM_PT_NONFINITE)) || bad;
    if (lane < 9) {
        double v = 0.0;
#pragma unroll
        for (int I = 0; I < 9; I++) v = (lane == I) ? h[I] : v;
        A.hr[(int64_t)lane * A.N + b] = failed ? 0.0 : v;
    }
    if (lane < 4) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < 4; i++) v = (lane == i) ? gt[i] : v;
        A.gth[(int64_t)lane * A.N + b] = failed ? 0.0 : v;
    }
    if (A.with_rho) {
        if (lane < m) A.rho[(int64_t)lane * A.count + pl] = failed ? 0.0 : rho0;
        if (lane + 64 < m) A.rho[(int64_t)(lane + 64) * A.count + pl] = failed ? 0.0 : rho1;
    }
    if (lane == 0 && bad) A.status[b] |= HROM_PT_JNONPOS;
}

int launch_backward_q(const BackwardArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_backward_q, dim3(nblocks(a.count, 4)), dim3(256), 0, s, a);
    return HROM_OK;
}

}  // namespace hrom
