// Adjoint backward through the converged ROM state.  With the RVE-frame
// cotangent g_r and the adjoint solution lambda = Kaa^{-T} KaF g_r, every ECM
// point is re-evaluated (F_q and the tangent are recomputed, never stored):
//   v_q   = g_r - G_q lambda
//   h_r  += w_q A_q v_q                               (= Cr^T g_r)
//   dmu_p  += w_q v_q : (F_q - F_q^{-T}),  dlam_p += w_q v_q : (ln J_q F_q^{-T})
// for the phase p of q.  Optionally the refinement residual
//   rho = sum_q G_q^T (w_q A_q v_q)  (= KaF g_r - Kaa lambda)
// of the adjoint system is accumulated with the same operator.
#include <hip/hip_runtime.h>

#include "hrom_internal.h"

namespace hrom {

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



// Point-batched form of the adjoint re-evaluation: sixteen macro points per
// workgroup; F_q - Fr = G a and G lambda are two GEMMs with the cluster's G
// as the shared operand (FP64 MFMA, N = the 16 points); the law and its
// adjoint run one (point, ECM point) pair per thread; the refinement
// residual rho = G^T (w A v) is a third FP64 GEMM.  Per-point sums over the
// ECM points (h_r, dL/dtheta) reduce in a fixed order.
struct BwLds {
    double sA[kMaxModes + 4][16];
    double sL[kMaxModes + 4][16];
    double sF[16 * 9][17];
    double sV[16 * 9][17];
    double sU[9][16];
    double sG[9][16];
    int sbits[16];
};

__device__ void bw_body(const BackwardArgs& A, int64_t p0, BwLds& Ls) {
    constexpr int PT = 16, QC = 16;
    auto& sA = Ls.sA;
    auto& sL = Ls.sL;
    auto& sF = Ls.sF;
    auto& sV = Ls.sV;
    auto& sU = Ls.sU;
    auto& sG = Ls.sG;
    auto& sbits = Ls.sbits;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, c = lane & 15;
    const int m = A.m, KS = A.KS, MP = A.MP, MT = A.MT;
    const int np = (int)min((int64_t)PT, A.count - p0);
    if (tid < PT) sbits[tid] = 0;
    for (int e = tid; e < 4 * KS * PT; e += 256) {
        const int k = e / PT, p = e % PT;
        const bool in = (k < m && p < np);
        sA[k][p] = in ? A.a[(int64_t)k * A.count + p0 + p] : 0.0;
        sL[k][p] = in ? A.lam[(int64_t)k * A.count + p0 + p] : 0.0;
    }
    for (int e = tid; e < 9 * PT; e += 256) {
        const int I = e / PT, p = e % PT;
        const int64_t b = A.first + p0 + p;
        sU[I][p] = (p < np) ? A.Fr[(int64_t)I * A.N + b] : ((I % 4 == 0) ? 1.0 : 0.0);
        sG[I][p] = (p < np) ? A.gr[(int64_t)I * A.N + b] : 0.0;
    }
    const double mu0 = A.theta[0], la0 = A.theta[1], mu1 = A.theta[2], la1 = A.theta[3];
    double h[9], gt[4];
#pragma unroll
    for (int I = 0; I < 9; I++) h[I] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++) gt[i] = 0.0;
    v4d racc[8];
#pragma unroll
    for (int t = 0; t < 8; t++) racc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    __syncthreads();

    for (int q0 = 0; q0 < A.Qpad; q0 += QC) {
        double gr[9][8];
        if (A.with_rho) {
            const double* gh = A.Ghat + (int64_t)(q0 * 9 + 36 * wave + g) * MP + c;
#pragma unroll
            for (int j = 0; j < 9; j++)
#pragma unroll
                for (int t = 0; t < 8; t++)
                    if (t < MT) gr[j][t] = gh[(int64_t)(4 * j) * MP + 16 * t];
        }
        const int rt0 = (q0 / 16) * 9;
        for (int t = wave; t < 9; t += 4) {
            const double* gf = A.Gf + ((int64_t)(rt0 + t) * KS) * 64 + lane;
            double af[24];
#pragma unroll
            for (int s2 = 0; s2 < 24; s2++)
                if (s2 < KS) af[s2] = gf[(int64_t)s2 * 64];
            v4d accF = v4d{0.0, 0.0, 0.0, 0.0}, accL = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s2 = 0; s2 < 24; s2++)
                if (s2 < KS) {
                    accF = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s2], sA[4 * s2 + g][c], accF, 0, 0, 0);
                    accL = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s2], sL[4 * s2 + g][c], accL, 0, 0, 0);
                }
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = 16 * t + g + 4 * e;
                sF[row][c] = accF[e] + sU[row % 9][c];
                sV[row][c] = sG[row % 9][c] - accL[e];
            }
        }
        __syncthreads();
        {
            const int p = tid >> 4, qq = tid & 15, q = q0 + qq;
            double F[9], v[9];
#pragma unroll
            for (int I = 0; I < 9; I++) {
                F[I] = sF[qq * 9 + I][p];
                v[I] = sV[qq * 9 + I][p];
            }
            const double wq = A.w[q];
            const int ph = A.phase[q];
            const double mu = ph ? mu1 : mu0, la = ph ? la1 : la0;
            double Fi[9];
            const double c00 = F[4] * F[8] - F[5] * F[7];
            const double c01 = F[5] * F[6] - F[3] * F[8];
            const double c02 = F[3] * F[7] - F[4] * F[6];
            const double J = F[0] * c00 + F[1] * c01 + F[2] * c02;
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
            const bool live = (q < A.Q) && (p < np);
            const bool ok = live && (J > 0.0);
            if (live && !(J > 0.0)) atomicOr(&sbits[p], HROM_PT_JNONPOS);
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
            const double wo = ok ? wq : 0.0;
            double dmu = 0.0, dla = 0.0;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    dmu = fma(v[3 * i + j], F[3 * i + j] - Fi[3 * j + i], dmu);
                    dla = fma(v[3 * i + j], ell * Fi[3 * j + i], dla);
                }
#pragma unroll
            for (int I = 0; I < 9; I++) h[I] = fma(wo, Av[I], h[I]);
            const double wm = ph ? 0.0 : wo, wi = ph ? wo : 0.0;
            gt[0] = fma(wm, dmu, gt[0]);
            gt[1] = fma(wm, dla, gt[1]);
            gt[2] = fma(wi, dmu, gt[2]);
            gt[3] = fma(wi, dla, gt[3]);
            if (A.with_rho) {
#pragma unroll
                for (int I = 0; I < 9; I++) sV[qq * 9 + I][p] = wo * Av[I];
            }
        }
        __syncthreads();
        if (A.with_rho) {
#pragma unroll
            for (int j = 0; j < 9; j++) {
                const double bv = sV[36 * wave + 4 * j + g][c];
#pragma unroll
                for (int t = 0; t < 8; t++)
                    if (t < MT) racc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(gr[j][t], bv, racc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // per-point sums over the 16 threads of the point (lanes 16p' .. 16p'+15
    // of a wave hold point p = tid >> 4): fixed butterfly within 16 lanes
#pragma unroll
    for (int I = 0; I < 9; I++)
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) h[I] += __shfl_xor(h[I], off);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) gt[i] += __shfl_xor(gt[i], off);
    {
        const int p = tid >> 4, sub = tid & 15;
        if (p < np) {
            const int64_t b = A.first + p0 + p;
            const bool failed = (A.status[b] & (HROM_PT_JNONPOS | HROM_PT_NONFINITE)) || sbits[p];
            double v = 0.0;
#pragma unroll
            for (int I = 0; I < 9; I++) v = (sub == I) ? h[I] : v;
            if (sub < 9) A.hr[(int64_t)sub * A.N + b] = failed ? 0.0 : v;
            double u = 0.0;
#pragma unroll
            for (int i = 0; i < 4; i++) u = (sub == 9 + i) ? gt[i] : u;
            if (sub >= 9 && sub < 13) A.gth[(int64_t)(sub - 9) * A.N + b] = failed ? 0.0 : u;
        }
    }
    if (A.with_rho) {
        double* red = &sF[0][0];
#pragma unroll
        for (int t = 0; t < 8; t++) {
            if (t >= MT) break;
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 4; e++) red[(wave * 16 + g + 4 * e) * 16 + c] = racc[t][e];
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int rr = g + 4 * e;
                    const double v = ((red[(0 * 16 + rr) * 16 + c] + red[(1 * 16 + rr) * 16 + c]) +
                                      red[(2 * 16 + rr) * 16 + c]) + red[(3 * 16 + rr) * 16 + c];
                    const int row = 16 * t + rr;
                    if (c < np && row < m) {
                        const bool failed = sbits[c] != 0;
                        A.rho[(int64_t)row * A.count + p0 + c] = failed ? 0.0 : v;
                    }
                }
            }
        }
    }
    __syncthreads();
    if (tid < np && sbits[tid]) A.status[A.first + p0 + tid] |= HROM_PT_JNONPOS;
}

__global__ void __launch_bounds__(256) k_backward_b(BackwardArgs A) {
    __shared__ BwLds Ls;
    bw_body(A, (int64_t)blockIdx.x * 16, Ls);
}

// adjoint re-evaluation of every cluster in one launch (16-point tiles)
__global__ void __launch_bounds__(256) k_backward_grouped(GroupCall G) {
    __shared__ BwLds Ls;
    const WorkItem w = G.items[blockIdx.x];
    const ClusterGPU& C = G.cls[w.c];
    BackwardArgs A;
    A.m = C.m; A.Q = C.Q; A.Qpad = C.Qpad; A.mixed = G.mixed; A.objective = G.objective;
    A.with_rho = G.with_rho; A.first = C.first; A.count = C.count; A.N = G.N;
    A.GT = nullptr; A.Ghat = C.Ghat; A.Gf = C.Gf; A.MP = C.MP; A.MT = C.MT; A.KS = C.KS;
    A.w = C.w; A.phase = C.phase; A.theta = G.theta; A.Fr = G.Fr; A.a = G.a + C.off_a;
    A.lam = G.lam + C.off_a; A.gr = G.gr; A.hr = G.hr; A.gth = G.gth;
    A.rho = G.rho ? G.rho + C.off_a : nullptr; A.status = G.status;
    bw_body(A, (int64_t)w.unit * 16, Ls);
}

int launch_backward_grouped(const GroupCall& g, hipStream_t s) {
    hipLaunchKernelGGL(k_backward_grouped, dim3(g.nitems), dim3(256), 0, s, g);
    return HROM_OK;
}

int launch_backward_b(const BackwardArgs& a, hipStream_t s) {
    if (a.MT > 8) return HROM_E_UNSUPPORTED;
    hipLaunchKernelGGL(k_backward_b, dim3((unsigned)((a.count + 15) / 16)), dim3(256), 0, s, a);
    return HROM_OK;
}

}  // namespace hrom
