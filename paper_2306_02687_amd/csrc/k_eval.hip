// Evaluation of the hyper-reduced RVE at every macro point (Sec. 3.2.1 and
// 3.3), in two kernels.
//
// k_kin -- kinematics, material law and residual, sixteen macro points per
// workgroup.  The reduced kinematics F_q - Fr = sum_m a_m G_qm of all points
// of the workgroup is one GEMM with the cluster's G as the shared operand
// (rows: ECM point x tensor row, K: modes, N: the 16 points) on FP64 MFMA;
// the Neo-Hooke stress P_q runs one (point, ECM point) pair per thread; the
// residual and homogenised stress rhat = Ghat^T (w P) = [r; Pr] is a second
// FP64 GEMM (K: ECM point x tensor row).  The tangent of every ECM point
// leaves as 12 scalars (F_q^{-1}, w mu, w (mu - lam ln J), w lam).
//
// k_eval_f64 / k_eval_mixed -- the tangent contraction
//   Khat = sum_q Ghat_q^T (w_q A_q) Ghat_q,   Ghat_q = [G_q | I_9 | 0],
// whose blocks are Kaa, KaF and KFF, one macro point per wavefront, four per
// workgroup, accumulated over the ECM points into upper-triangular 16x16
// tiles held in registers.
#include <hip/hip_runtime.h>

#include "hrom_internal.h"
#include "hrom_j2.h"

namespace hrom {

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ __forceinline__ double inv3d(const double* A, double* B) {
    const double c00 = A[4] * A[8] - A[5] * A[7];
    const double c01 = A[5] * A[6] - A[3] * A[8];
    const double c02 = A[3] * A[7] - A[4] * A[6];
    const double d = A[0] * c00 + A[1] * c01 + A[2] * c02;
    const double id = 1.0 / d;
    B[0] = c00 * id;
    B[3] = c01 * id;
    B[6] = c02 * id;
    B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return d;
}

// Row I = (i, j) of the Neo-Hooke tangent scaled by the ECM weight,
//   W[I][(k,l)] = c0 d_ik d_jl + c1 Fi_li Fi_jk + c2 Fi_ji Fi_lk
// with c0 = w mu, c1 = w (mu - lam ln J), c2 = w lam, Fi = F^{-1}.
template <int I, typename T>
__device__ __forceinline__ void tangent_row(const T* Fi, T c0, T c1, T c2, T* W) {
    constexpr int i = I / 3, j = I % 3;
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int l = 0; l < 3; l++) {
            T v = c1 * Fi[3 * l + i] * Fi[3 * j + k] + c2 * Fi[3 * j + i] * Fi[3 * l + k];
            if (k == i && l == j) v += c0;
            W[3 * k + l] = v;
        }
}


// ============================================================== kinematics
// 32 macro points per workgroup of NW = 4 or 8 wavefronts, ECM points in
// rounds of 16.  Every FP64 MFMA operand of G is used for two 16-point column
// tiles.  Per round:
//   F - F_r = G a      144 rows (ECM point, component) x 32 points; wave w takes
//                      row tiles w (+ NW ...) < 8, waves 0..3 a k-range of row
//                      tile 8 (partial sums added in a fixed order)
//   law                thread = 8 / NW (point, ECM point) pairs: w P, tangent
//                      scalars (w P overwrites F in place)
//   r += G^T (w P)     the round's 36 k-steps in four k-ranges of nine, one
//                      per wave w % 4 (eight waves: waves w and w + 4 split
//                      the mode tiles by parity); fixed-order sum over the four
//                      k-ranges at the end, so that both workgroup shapes give
//                      bitwise the same r
//   Pbar_r += w P      fixed-order sum over the round's ECM points
// With four wavefronts and m <= 64 the workgroup holds about 73 KB of LDS, so
// two workgroups share a CU and the matrix phases of one overlap the material
// law of the other.
constexpr int kKinPT = 32;
// weights and phases of a round's ECM points, staged through LDS up to four
// mode tiles; with more the workgroup would outgrow half the CU's LDS
// (80 KiB at six tiles), and the law reads them from memory itself
template <int AR>
constexpr bool kin_stage_w() { return AR <= 64; }
template <int AR, bool W = kin_stage_w<AR>()>
struct KinLdsW {};
template <int AR>
struct KinLdsW<AR, true> {
    double sWq[16];
    int sPh[16];
};
template <int AR>   // rows of the mode amplitudes (>= 16 ceil(m / 16))
struct KinLds : KinLdsW<AR> {
    double sA[AR][kKinPT];
    double sF[16 * 9][kKinPT + 1];   // F of the round, then w P in place
    double sF8[4][16][kKinPT + 1];
    double sU[9][kKinPT];
    int sbits[kKinPT];
};

// the 32 macro points p0 .. p0+31 of the cluster described by A; MA = ceil(m / 16);
// J2: small-strain J2 plasticity with history in place of Neo-Hooke (the
// history and the law in FP64 on both paths; the mixed path stores the nine
// tangent scalars in FP32)
template <bool MIXED, int MA, int NW, int AR, bool J2 = false>
__device__ void kin_body(const EvalArgs& A, int64_t p0, KinLds<AR>& L) {
    constexpr int PT = kKinPT, QC = 16, NT = 64 * NW;
    static_assert(AR >= 16 * MA, "mode amplitude rows");
    static_assert(NW == 4 || NW == 8, "four or eight wavefronts");
    auto& sA = L.sA;
    auto& sF = L.sF;
    auto& sWP = L.sF;
    auto& sF8 = L.sF8;
    auto& sU = L.sU;
    auto& sbits = L.sbits;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, c = lane & 15;
    const int m = A.m, MP = A.MP;
    constexpr int KS = 4 * MA;   // k-steps of the G a GEMM (the plan pads them to whole mode tiles)
    const int np = (int)min((int64_t)PT, A.count - p0);
    if (tid < PT) sbits[tid] = 0;
    __syncthreads();
    for (int e = tid; e < 4 * KS * PT; e += NT) {
        const int k = e / PT, p = e % PT;
        double v = 0.0;
        if (k < m && p < np) {
            v = A.a[(int64_t)k * A.count + p0 + p];
            if (!isfinite(v)) {
                atomicOr(&sbits[p], HROM_PT_NONFINITE);
                v = 0.0;
            }
        }
        sA[k][p] = v;
    }
    for (int e = tid; e < 9 * PT; e += NT) {
        const int I = e / PT, p = e % PT;
        sU[I][p] = (p < np) ? A.Fr[(int64_t)I * A.N + A.first + p0 + p] : ((I % 4 == 0) ? 1.0 : 0.0);
    }
    const double mu0 = A.theta[0], la0 = A.theta[1], mu1 = A.theta[2], la1 = A.theta[3];
    // mixed path: w_q A_q leaves scaled by the power of two 2^(qexp + 4 - e),
    // 2^(e - 1) <= max |theta| < 2^e, so that its entries are O(16) whatever the
    // units of the moduli (FP16 range); the condensation divides it out
    float wscale = 1.0f;
    if (MIXED) {
        // J2 plans: theta = per phase (mu, lam, sy0, H), the moduli at 0, 1, 4, 5
        const double mx = J2 ? fmax(fmax(fabs(A.theta[0]), fabs(A.theta[1])), fmax(fabs(A.theta[4]), fabs(A.theta[5])))
                             : fmax(fmax(fabs(mu0), fabs(la0)), fmax(fabs(mu1), fabs(la1)));
        const int e = (mx > 0.0 && isfinite(mx)) ? ilogb(mx) + 1 : 0;
        wscale = ldexpf(1.0f, A.qexp + 4 - e);
    }
    if (blockIdx.x == 0 && tid == 0 && A.kscale_out) *A.kscale_out = 1.0f / wscale;
    v4d racc[MA][2];
#pragma unroll
    for (int t = 0; t < MA; t++) racc[t][0] = racc[t][1] = v4d{0.0, 0.0, 0.0, 0.0};
    // Pbar_r (I = e / 32, point e % 32) for the entries e = tid + NT h < 288
    constexpr int NPB = (9 * PT + NT - 1) / NT;
    double pacc[NPB];
#pragma unroll
    for (int h = 0; h < NPB; h++) pacc[h] = 0.0;
    const int klo = wave * (KS / 4);   // k-range of row tile 8 (waves 0..3)
    const int v = wave & 3;                        // k-range of the residual GEMM
    const int js = 9 * v;                          // k-steps js .. js + 8
    const int tpar = (NW == 8) ? (wave >> 2) : 0;  // mode-tile parity (eight waves)
    auto holds = [&](int t) { return NW == 4 || (t & 1) == tpar; };
    __syncthreads();

    for (int q0 = 0; q0 < A.Qpad; q0 += QC) {
        const int rt0 = (q0 / 16) * 9;
        // weights and phases of the round's ECM points, loaded ahead of the
        // GEMM and handed to the law through LDS (where it has room for them)
        constexpr bool WS = kin_stage_w<AR>();
        double wnext = 0.0;
        int phnext = 0;
        if (WS && tid < QC) {
            wnext = A.w[q0 + tid];
            phnext = A.phase[q0 + tid];
        }
        // ---- F - Fr: row tiles wave, wave + NW, ... < 8
#pragma unroll
        for (int h = 0; h < 8 / NW; h++) {
            const int rt = wave + NW * h;
            const double* gf = A.Gf + ((int64_t)(rt0 + rt) * KS) * 64 + lane;
            double af[4 * MA];
#pragma unroll
            for (int s2 = 0; s2 < 4 * MA; s2++)
                af[s2] = gf[(int64_t)s2 * 64];
            v4d a0 = v4d{0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
            for (int s2 = 0; s2 < KS; s2++) {
                a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s2], sA[4 * s2 + g][c], a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s2], sA[4 * s2 + g][16 + c], a1, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = 16 * rt + g + 4 * e;   // FP64 MFMA accumulator rows interleave
                sF[row][c] = a0[e] + sU[row % 9][c];
                sF[row][16 + c] = a1[e] + sU[row % 9][16 + c];
            }
        }
        // ---- row tile 8: a k-range per wave 0..3
        if (wave < 4) {
            const double* gf = A.Gf + ((int64_t)(rt0 + 8) * KS) * 64 + lane;
            v4d a0 = v4d{0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
            for (int s = 0; s < KS / 4; s++) {   // k-steps klo .. klo + KS / 4 - 1
                const int s2 = klo + s;
                const double av = gf[(int64_t)s2 * 64];
                a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sA[4 * s2 + g][c], a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sA[4 * s2 + g][16 + c], a1, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; e++) {
                sF8[wave][g + 4 * e][c] = a0[e];
                sF8[wave][g + 4 * e][16 + c] = a1[e];
            }
        }
        if constexpr (WS) {
            if (tid < QC) {
                L.sWq[tid] = wnext;
                L.sPh[tid] = phnext;
            }
        }
        __syncthreads();
        // ---- rows 128..143 of F: fixed-order sum of the four k-range partials
        for (int e = tid; e < 16 * PT; e += NT) {
            const int r = e >> 5, p = e & 31;
            sF[128 + r][p] = ((sF8[0][r][p] + sF8[1][r][p]) + (sF8[2][r][p] + sF8[3][r][p])) + sU[(128 + r) % 9][p];
        }
        __syncthreads();
        // ---- material law: thread = (point p, ECM point q0 + qq), 8 / NW per thread
#pragma unroll 1
        for (int h = 0; h < 8 / NW; h++) {
            const int e2 = tid + NT * h;
            const int p = e2 >> 4, qq = e2 & 15, q = q0 + qq;
            double F[9];
#pragma unroll
            for (int I = 0; I < 9; I++) F[I] = sF[qq * 9 + I][p];
            double wq;
            int ph;
            if constexpr (WS) {
                wq = L.sWq[qq];
                ph = L.sPh[qq];
            } else {
                wq = A.w[q];
                ph = A.phase[q];
            }
            if constexpr (J2) {
                // theta = per phase (mu, lam, sy0, H); committed state in, new state out
                const double* mp = A.theta + 4 * ph;
                const bool live = (q < A.Q) && (p < np);
                const int64_t ho = ((p0 + p) * A.Qpad + q) * 8;
                double hn[7], sig[9], t[9], ht[7];
#pragma unroll
                for (int k = 0; k < 7; k++) hn[k] = live ? A.hist_n[ho + k] : 0.0;
                j2_update(F, mp[0], mp[1], mp[2], mp[3], hn, sig, t, ht);
#pragma unroll
                for (int I = 0; I < 9; I++) sWP[qq * 9 + I][p] = live ? wq * sig[I] : 0.0;
                if (p < np) {
                    const int64_t off = ((p0 + p) * A.Qpad + q) * 12;
                    if constexpr (MIXED) {
                        // (w kappa, w 2 mu th, w 2 mu thb) scaled like the Neo-Hooke scalars, then n
                        const float ws = wscale;
                        float* o = (float*)A.qs + off;
                        v4f v0 = v4f{(float)(wq * t[0]) * ws, (float)(wq * t[1]) * ws, (float)(wq * t[2]) * ws,
                                     (float)t[3]};
                        v4f v1 = v4f{(float)t[4], (float)t[5], (float)t[6], (float)t[7]};
                        v4f v2 = v4f{(float)t[8], 0.f, 0.f, 0.f};
                        if (!live) v0 = v1 = v2 = v4f{0.f, 0.f, 0.f, 0.f};
                        *(v4f*)(o) = v0;
                        *(v4f*)(o + 4) = v1;
                        *(v4f*)(o + 8) = v2;
                    } else {
                        double* o = (double*)A.qs + off;
#pragma unroll
                        for (int k = 0; k < 3; k++) o[k] = live ? wq * t[k] : 0.0;
#pragma unroll
                        for (int k = 3; k < 12; k++) o[k] = (live && k < 9) ? t[k] : 0.0;
                    }
                    if (live) {
#pragma unroll
                        for (int k = 0; k < 7; k++) A.hist_t[ho + k] = ht[k];
                    }
                }
                continue;
            }
            const double mu = ph ? mu1 : mu0, la = ph ? la1 : la0;
            double Fi[9];
            const double J = inv3d(F, Fi);
            const bool live = (q < A.Q) && (p < np);
            const bool ok = live && (J > 0.0);
            if (live && !(J > 0.0)) atomicOr(&sbits[p], HROM_PT_JNONPOS);
            const double ell = ok ? log(J) : 0.0;
            // w P over the same slots the thread read F from
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++)
                    sWP[qq * 9 + 3 * i + j][p] =
                        ok ? wq * (mu * (F[3 * i + j] - Fi[3 * j + i]) + la * ell * Fi[3 * j + i]) : 0.0;
            if (p < np) {
                const double c0 = ok ? wq * mu : 0.0;
                const double c1 = ok ? wq * (mu - la * ell) : 0.0;
                const double c2 = ok ? wq * la : 0.0;
                const int64_t off = ((p0 + p) * A.Qpad + q) * 12;
                if (MIXED) {
                    const float ws = wscale;
                    float* o = (float*)A.qs + off;
                    v4f v0 = v4f{(float)Fi[0], (float)Fi[1], (float)Fi[2], (float)Fi[3]};
                    v4f v1 = v4f{(float)Fi[4], (float)Fi[5], (float)Fi[6], (float)Fi[7]};
                    v4f v2 = v4f{(float)Fi[8], (float)c0 * ws, (float)c1 * ws, (float)c2 * ws};
                    if (!ok) v0 = v1 = v2 = v4f{0.f, 0.f, 0.f, 0.f};
                    *(v4f*)(o) = v0;
                    *(v4f*)(o + 4) = v1;
                    *(v4f*)(o + 8) = v2;
                } else {
                    double* o = (double*)A.qs + off;
#pragma unroll
                    for (int k = 0; k < 9; k++) o[k] = ok ? Fi[k] : 0.0;
                    o[9] = c0;
                    o[10] = c1;
                    o[11] = c2;
                }
            }
        }
        __syncthreads();
        // ---- r += G^T (w P): this wave's k-steps of the round, the mode tiles
        for (int jj = 0; jj < 9; jj++) {
            const int j = js + jj;
            const double b0 = sWP[4 * j + g][c], b1 = sWP[4 * j + g][16 + c];
            const double* gh = A.Ghat + (int64_t)(q0 * 9 + 4 * j + g) * MP + c;
#pragma unroll
            for (int t = 0; t < MA; t++)
                if (holds(t)) {
                    const double av = gh[16 * t];
                    racc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, racc[t][0], 0, 0, 0);
                    racc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, racc[t][1], 0, 0, 0);
                }
        }
        // ---- Pbar_r += sum over the round's ECM points of w P
#pragma unroll
        for (int h = 0; h < NPB; h++) {
            const int e2 = tid + NT * h;
            if (e2 < 9 * PT) {
                const int I = e2 >> 5, p = e2 & 31;
                double sp = 0.0;
#pragma unroll
                for (int qq = 0; qq < QC; qq++) sp += sWP[qq * 9 + I][p];
                pacc[h] += sp;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int h = 0; h < NPB; h++) {
        const int e2 = tid + NT * h;
        if (e2 < 9 * PT && (e2 & 31) < np)
            A.Pr[(int64_t)(e2 >> 5) * A.N + A.first + p0 + (e2 & 31)] = pacc[h];
    }
    // fixed-order sum of the four k-range partials of r through LDS (sF reused)
    double* red = &sF[0][0];
#pragma unroll
    for (int t = 0; t < MA; t++) {
        if (holds(t)) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                red[(v * 16 + g + 4 * e) * PT + c] = racc[t][0][e];
                red[(v * 16 + g + 4 * e) * PT + 16 + c] = racc[t][1][e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 512 / NT; h++) {
            const int e2 = tid + NT * h;   // 16 rows x 32 points
            const int rr = e2 >> 5, p = e2 & 31;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < 4; w++) sum += red[(w * 16 + rr) * PT + p];
            const int row = 16 * t + rr;
            if (p < np && row < m) A.r[(int64_t)row * A.count + p0 + p] = sum;
        }
        __syncthreads();
    }
    if (tid < np && sbits[tid]) A.status[A.first + p0 + tid] |= sbits[tid];
}

template <bool MIXED, int MA, bool J2>
__global__ void __launch_bounds__(256, 2) k_kin(EvalArgs A) {
    __shared__ KinLds<16 * MA> L;
    kin_body<MIXED, MA, 4, 16 * MA, J2>(A, (int64_t)blockIdx.x * kKinPT, L);
}

// the same 32 points per workgroup on eight wavefronts (row tiles w and
// w + 8, the k-range partials of the ninth tile unchanged: the same bits)
template <bool MIXED, int MA, bool J2>
__global__ void __launch_bounds__(512, 1) k_kin8(EvalArgs A) {
    __shared__ KinLds<16 * MA> L;
    kin_body<MIXED, MA, 8, 16 * MA, J2>(A, (int64_t)blockIdx.x * kKinPT, L);
}

template <bool MIXED, bool J2, bool W8>
static void launch_kin_t(const EvalArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(a.count, kKinPT)), block(W8 ? 512 : 256);
#define HROM_KIN(MA_)                                                                  \
    if constexpr (W8) hipLaunchKernelGGL((k_kin8<MIXED, MA_, J2>), grid, block, 0, s, a); \
    else hipLaunchKernelGGL((k_kin<MIXED, MA_, J2>), grid, block, 0, s, a);
    switch ((a.m + 15) / 16) {
        case 1: { HROM_KIN(1) } break;
        case 2: { HROM_KIN(2) } break;
        case 3: { HROM_KIN(3) } break;
        case 4: { HROM_KIN(4) } break;
        case 5: { HROM_KIN(5) } break;
        default: { HROM_KIN(6) } break;
    }
#undef HROM_KIN
}

// variant 0: four wavefronts per workgroup (two workgroups per CU), 1: eight
int launch_kin(int mixed, int j2, int variant, const EvalArgs& a, hipStream_t s) {
    if ((a.m + 15) / 16 > 6) return HROM_E_UNSUPPORTED;
    const bool w8 = variant == 1;
    if (j2 && mixed) w8 ? launch_kin_t<true, true, true>(a, s) : launch_kin_t<true, true, false>(a, s);
    else if (j2) w8 ? launch_kin_t<false, true, true>(a, s) : launch_kin_t<false, true, false>(a, s);
    else if (mixed) w8 ? launch_kin_t<true, false, true>(a, s) : launch_kin_t<true, false, false>(a, s);
    else w8 ? launch_kin_t<false, false, true>(a, s) : launch_kin_t<false, false, false>(a, s);
    return HROM_OK;
}

// ============================================================== FP64 tangent
// the W row of tensor row I, then its products with the mode tiles; J2: the
// tangent from the nine scalars s (Neo-Hooke: F^{-1} = s, c0..c2)
template <int I, int MT, bool J2>
__device__ __forceinline__ void row_step_f64(const double* Fi, double c0, double c1, double c2,
                                             const double (&Gc)[MT][9], v4d* acc) {
    double W[9];
    if constexpr (J2) j2_tangent_row<I>(Fi, W);
    else tangent_row<I>(Fi, c0, c1, c2, W);
    double Bv[MT];
#pragma unroll
    for (int t = 0; t < MT; t++) {
        double s = 0.0;
#pragma unroll
        for (int J = 0; J < 9; J++) s = fma(W[J], Gc[t][J], s);
        Bv[t] = s;
    }
    int idx = 0;
#pragma unroll
    for (int ti = 0; ti < MT; ti++)
#pragma unroll
        for (int tj = ti; tj < MT; tj++) {
            acc[idx] = __builtin_amdgcn_mfma_f64_16x16x4f64(Gc[ti][I], Bv[tj], acc[idx], 0, 0, 0);
            idx++;
        }
}

// FP64: the tangent product T_q = (w_q A_q) Ghat_q is formed on the vector
// ALUs straight into the B operand of the FP64 MFMA; the contraction index is
// k = (ECM point, tensor row), lane group g taking ECM point q0 + 4 qb + g.
template <int MT>
__device__ __forceinline__ void load_ghat(const double* gh, int MP, double (&Gc)[MT][9]) {
#pragma unroll
    for (int t = 0; t < MT; t++)
#pragma unroll
        for (int J = 0; J < 9; J++) Gc[t][J] = gh[J * MP + 16 * t];
}

template <int MT, bool J2 = false>
__device__ __forceinline__ void tangent_block_f64(const double* st, int qq, const double (&Gc)[MT][9],
                                                  v4d* acc) {
    double Fi[9];
#pragma unroll
    for (int k = 0; k < 9; k++) Fi[k] = st[k * 64 + qq];
    const double c0 = st[9 * 64 + qq], c1 = st[10 * 64 + qq], c2 = st[11 * 64 + qq];
    row_step_f64<0, MT, J2>(Fi, c0, c1, c2, Gc, acc);
    row_step_f64<1, MT, J2>(Fi, c0, c1, c2, Gc, acc);
    row_step_f64<2, MT, J2>(Fi, c0, c1, c2, Gc, acc);
    row_step_f64<3, MT, J2>(Fi, c0, c1, c2, Gc, acc);
    row_step_f64<4, MT, J2>(Fi, c0, c1, c2, Gc, acc);
    row_step_f64<5, MT, J2>(Fi, c0, c1, c2, Gc, acc);
    row_step_f64<6, MT, J2>(Fi, c0, c1, c2, Gc, acc);
    row_step_f64<7, MT, J2>(Fi, c0, c1, c2, Gc, acc);
    row_step_f64<8, MT, J2>(Fi, c0, c1, c2, Gc, acc);
}

// the 4 macro points pl0 .. pl0+3 of the cluster, one per wavefront
template <int MT, bool PFREQ = true, bool J2 = false>
__device__ void tan_f64_body(const EvalArgs& A, int64_t pl0, double (*s_st)[12 * 64]) {
    constexpr int NT = MT * (MT + 1) / 2;
    constexpr bool PF = PFREQ && (MT <= 5);   // register budget of the double buffer
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    int64_t pl = pl0 + wave;
    const bool valid = pl < A.count;
    if (!valid) pl = A.count - 1;
    const int MP = A.MP;
    double* st = s_st[wave];
    const double* qsp = (const double*)A.qs + (pl * A.Qpad) * 12;
    v4d acc[NT];
#pragma unroll
    for (int i = 0; i < NT; i++) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};

    for (int q0 = 0; q0 < A.Qpad; q0 += 64) {
        {
            const double* src = qsp + (int64_t)(q0 + lane) * 12;
#pragma unroll
            for (int k = 0; k < 12; k++) st[k * 64 + lane] = src[k];
        }
        __syncthreads();
        if (PF) {
            // two register buffers: the next ECM point's Ghat rows load while
            // the current one is contracted
            double GA[MT][9], GB[MT][9];
            load_ghat<MT>(A.Ghat + (int64_t)(q0 + g) * 9 * MP + c, MP, GA);
            for (int qb = 0; qb < 16; qb += 2) {
                load_ghat<MT>(A.Ghat + (int64_t)(q0 + 4 * (qb + 1) + g) * 9 * MP + c, MP, GB);
                tangent_block_f64<MT, J2>(st, 4 * qb + g, GA, acc);
                if (qb + 2 < 16)
                    load_ghat<MT>(A.Ghat + (int64_t)(q0 + 4 * (qb + 2) + g) * 9 * MP + c, MP, GA);
                tangent_block_f64<MT, J2>(st, 4 * (qb + 1) + g, GB, acc);
            }
        } else {
            for (int qb = 0; qb < 16; qb++) {
                double Gc[MT][9];
                load_ghat<MT>(A.Ghat + (int64_t)(q0 + 4 * qb + g) * 9 * MP + c, MP, Gc);
                tangent_block_f64<MT, J2>(st, 4 * qb + g, Gc, acc);
            }
        }
        __syncthreads();
    }
    if (!valid) return;
    double* kh = (double*)A.Khat + (int64_t)pl * NT * 256 + lane * 4;
#pragma unroll
    for (int i = 0; i < NT; i++) *(v4d*)(kh + i * 256) = acc[i];
}

template <int MT, bool PF, bool J2>
__global__ void __launch_bounds__(256, 1) k_eval_f64(EvalArgs A) {
    __shared__ double s_st[4][12 * 64];
    tan_f64_body<MT, PF, J2>(A, (int64_t)blockIdx.x * 4, s_st);
}

template <bool PF, bool J2>
static int launch_f64_t(int MT, const EvalArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(a.count, 4)), block(256);
    switch (MT) {
        case 2: hipLaunchKernelGGL((k_eval_f64<2, PF, J2>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_eval_f64<3, PF, J2>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_eval_f64<4, PF, J2>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_eval_f64<5, PF, J2>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_eval_f64<6, PF, J2>), grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL((k_eval_f64<7, PF, J2>), grid, block, 0, s, a); break;
        default: return HROM_E_UNSUPPORTED;
    }
    return HROM_OK;
}

// variant bit 1: G double-buffering off (the FP64 kernel has one occupancy);
// j2: the J2 plasticity tangent rows
int launch_eval_f64(int MT, int variant, int j2, const EvalArgs& a, hipStream_t s) {
    if (j2) return (variant & 2) ? launch_f64_t<false, true>(MT, a, s) : launch_f64_t<true, true>(MT, a, s);
    return (variant & 2) ? launch_f64_t<false, false>(MT, a, s) : launch_f64_t<true, false>(MT, a, s);
}

// ============================================================== mixed tangent
// Low-precision operand types: fragments are carried as 16-bit patterns, two
// per dword; conversions round to nearest even.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

template <int PREC>
struct Pk;

template <>
struct Pk<HROM_MIXED_BF16> {
    // (x0, x1) -> one dword, x0 in the low half
    static __device__ __forceinline__ uint32_t pack(float x0, float x1) {
        typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
        typedef float v2f __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f{x0, x1}), v2bf));
    }
    // x minus the value in the low / high half of h, as one dot2 with the
    // packed factor (-1, 0) or (0, -1); x - round(x) is exact in FP32 and so
    // is the dot2 result.  The factor sits in a scalar register: folded into an
    // inline constant it reaches the hardware with its halves swapped.
    template <uint32_t V>
    static __device__ __forceinline__ uint32_t in_sgpr() {
        uint32_t r;
        asm("s_mov_b32 %0, %1" : "=s"(r) : "n"(V));
        return r;
    }
    static __device__ __forceinline__ float res_lo(uint32_t h, float x) {
        typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(v2bf, h),
                                               __builtin_bit_cast(v2bf, in_sgpr<0x0000BF80u>()), x, false);
    }
    static __device__ __forceinline__ float res_hi(uint32_t h, float x) {
        typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(v2bf, h),
                                               __builtin_bit_cast(v2bf, in_sgpr<0xBF800000u>()), x, false);
    }
    // per-lane form: x - lo(h) where f = (-1, 0), x where f = 0 (f a register)
    static __device__ __forceinline__ uint32_t g1_factor() { return 0x0000BF80u; }
    static __device__ __forceinline__ float res_lo_if(uint32_t h, float x, uint32_t f) {
        typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(v2bf, h), __builtin_bit_cast(v2bf, f), x, false);
    }
    static constexpr uint32_t one = 0x3F80u;
    static __device__ __forceinline__ v4f mfma(v4u32 a, v4u32 b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                       __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
    }
};

template <>
struct Pk<HROM_MIXED_FP16> {
    static __device__ __forceinline__ uint32_t pack(float x0, float x1) {
        typedef _Float16 v2h __attribute__((ext_vector_type(2)));
        typedef float v2f __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f{x0, x1}), v2h));
    }
    // x minus the value in the low / high half of h (exact in FP32; the
    // FP16 dot2 is not exact for subnormal halves)
    static __device__ __forceinline__ float res_lo(uint32_t h, float x) {
        return x - (float)__builtin_bit_cast(_Float16, (unsigned short)(h & 0xFFFFu));
    }
    static __device__ __forceinline__ float res_hi(uint32_t h, float x) {
        return x - (float)__builtin_bit_cast(_Float16, (unsigned short)(h >> 16));
    }
    // per-lane form: f = 1.0f (bits) or 0: x - lo(h) or x, one FMA
    static __device__ __forceinline__ uint32_t g1_factor() { return 0x3F800000u; }
    static __device__ __forceinline__ float res_lo_if(uint32_t h, float x, uint32_t f) {
        return fmaf(-(float)__builtin_bit_cast(_Float16, (unsigned short)(h & 0xFFFFu)), __uint_as_float(f), x);
    }
    static constexpr uint32_t one = 0x3C00u;
    static __device__ __forceinline__ v4f mfma(v4u32 a, v4u32 b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a),
                                                      __builtin_bit_cast(v8h, b), c, 0, 0, 0);
    }
};

// Mixed path: tangent contraction on BF16/FP16 MFMA (16x16x32, FP32
// accumulation), one macro point per wavefront.  Per ECM point q, with
// W_q = w_q A_q (9 x 9, FP32, scaled by a power of two) and the mode tiles G_t:
//   T_t  = W_q G_t          one MFMA per mode tile,
//   Kaa += G_ti^T T_tj      one MFMA per upper tile pair (T re-split into hi/lo),
//   KaF += G_t^T W_q        one MFMA per mode tile,
//   KFF += W_q              one MFMA against a constant identity fragment.
// Every operand is carried as hi + lo and all three split products
// hi*hi + lo*hi + hi*lo of the nine-component contraction share the 32 k-slots
// of one MFMA: the components sit in the accumulator rows 0,1 | 4,5 | 8,9 |
// 12,13,14 of the four lane groups, so lane group g holds rows 4g + e of T and
// its k-slots pair (G parts) x (W or T parts) as
//   groups 0..2: Gh.Th(a) Gh.Th(b) Gl.Th(a) Gl.Th(b) Gh.Tl(a) Gh.Tl(b) [g1: Gh.Tl(8)] 0
//   group 3:     same for a = 6, b = 7, then Gh.Th(8) Gl.Th(8)
// The one term that does not fit its own lane group, Tl(8), is formed in
// group 1 itself: its lanes read the W row of component 8 for their otherwise
// unused accumulator row 6, so row 6 of T is a copy of component 8 (ignored on
// output).  W is built once per ECM point in LDS by the whole wavefront (16 ECM
// points per round) rather than per lane.
// Record per point: Kaa upper tiles [MA(MA+1)/2][256], KaF tiles [MA][256]
// (row = mode, column = accumulator row of the component), KFF tile [256].
constexpr int kCQ = 16;   // ECM points per LDS round
// LDS records of one round: per ECM point the 36 records (component K, lane
// group g) at 4 K + g, then one zero record read by the lanes that carry no
// tensor row
constexpr int kWR = 37;

__device__ __forceinline__ int comp_pos(int K) { return K < 6 ? 4 * (K >> 1) + (K & 1) : 6 + K; }
__device__ __forceinline__ int pos_comp(int r) {
    const int g = r >> 2, e = r & 3;
    if (g < 3) return e < 2 ? 2 * g + e : -1;
    return e < 3 ? 6 + e : -1;
}

// the four lane records (lane groups 0..3) of W row KI, from w[J] = W[KI][J]
template <int PREC, bool SPLIT>
__device__ __forceinline__ void w_records(const float* w, v4u32* rec) {
    uint32_t h[5], l[5];
#pragma unroll
    for (int p = 0; p < 4; p++) {
        h[p] = Pk<PREC>::pack(w[2 * p], w[2 * p + 1]);
        l[p] = SPLIT ? Pk<PREC>::pack(Pk<PREC>::res_lo(h[p], w[2 * p]), Pk<PREC>::res_hi(h[p], w[2 * p + 1])) : 0u;
    }
    h[4] = Pk<PREC>::pack(w[8], w[8]);
    l[4] = SPLIT ? Pk<PREC>::pack(Pk<PREC>::res_lo(h[4], w[8]), 0.f) : 0u;
    rec[0] = v4u32{h[0], h[0], l[0], 0u};
    rec[1] = v4u32{h[1], h[1], l[1], l[4]};
    rec[2] = v4u32{h[2], h[2], l[2], 0u};
    rec[3] = v4u32{h[3], h[3], l[3], h[4]};
}

// T tile (accumulator rows 4g + e) -> K-step B operand.  Row 4g + 2 is
// component 8 in groups 1 and 3 (zero in groups 0, 2); g1 = 1 in group 1:
// its last dword becomes (Tl(8), Tl(8)), that of group 3 (Th(8), Th(8)).
template <int PREC, bool SPLIT>
__device__ __forceinline__ v4u32 t_operand(v4f T, uint32_t g1) {
    const uint32_t hA = Pk<PREC>::pack(T[0], T[1]);
    const uint32_t lA = SPLIT ? Pk<PREC>::pack(Pk<PREC>::res_lo(hA, T[0]), Pk<PREC>::res_hi(hA, T[1])) : 0u;
    const uint32_t h8 = Pk<PREC>::pack(T[2], T[2]);
    const float x8 = SPLIT ? Pk<PREC>::res_lo_if(h8, T[2], g1) : (g1 ? 0.f : T[2]);
    return v4u32{hA, hA, lA, Pk<PREC>::pack(x8, x8)};
}

// NP macro points per wavefront (1 or 2): with two, both points' products
// take the same mode fragments, so each fragment is fetched once for two
// points (half the fragment traffic through the CU's load path).
template <int MA, int PREC, bool SPLIT, bool PF, int NP = 1, bool J2 = false>
__device__ void tan_mixed_body(const EvalArgs& A, int64_t pl0, v4u32 (*s_w)[kCQ * kWR]) {
    constexpr int NA = MA * (MA + 1) / 2;
    constexpr int QR = kCQ / NP;   // ECM points per LDS round
    constexpr int kUnrollQ = 2;   // ECM points per unrolled step (4 with two points spills)
    static_assert(NP == 1 || NP == 2, "one or two points per wavefront");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    int64_t pl[NP];
    bool valid[NP];
#pragma unroll
    for (int pp = 0; pp < NP; pp++) {
        pl[pp] = pl0 + NP * wave + pp;
        valid[pp] = pl[pp] < A.count;
        if (!valid[pp]) pl[pp] = A.count - 1;
    }
    v4u32* sw = s_w[wave];
    // W builder of this lane: point pb, ECM point qq of the round, row set u
    const int pb = (NP == 1) ? 0 : lane / (4 * QR), qq = (lane >> 2) & (QR - 1), u = lane & 3;
    const float* qsp = (const float*)A.qs + ((pb == 0 ? pl[0] : pl[NP - 1]) * A.Qpad) * 12;
    const v4u32* fp = (const v4u32*)A.Fpk + lane;
    // the zero record of every ECM point slot
    if (lane < kCQ) sw[lane * kWR + 36] = v4u32{0u, 0u, 0u, 0u};
    // this lane's record: row c of W (component pos_comp(c); row 6 takes
    // component 8 as well, see above), else the zero record
    const int rcomp = (c == 6) ? 8 : pos_comp(c);
    const int wrec = (rcomp >= 0) ? 4 * rcomp + g : 36;
    const uint32_t in_g1 = (g == 1) ? Pk<PREC>::g1_factor() : 0u;   // see t_operand
    // identity fragment: G[J][column c] = 1 for J = component of accumulator row c
    v4u32 Ip;
    {
        const int K = pos_comp(c);
        const int a = (g < 3) ? 2 * g : 6, b = a + 1;
        const uint32_t ha = (K == a) ? Pk<PREC>::one : 0u, hb = (K == b) ? Pk<PREC>::one : 0u;
        const uint32_t h8 = (K == 8) ? Pk<PREC>::one : 0u;
        Ip = v4u32{ha | (hb << 16), 0u, ha | (hb << 16), (g == 1 || g == 3) ? h8 : 0u};
    }
    v4f acc[NP][NA], accF[NP][MA], accFF[NP];
#pragma unroll
    for (int pp = 0; pp < NP; pp++) {
        accFF[pp] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NA; i++) acc[pp][i] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < MA; i++) accF[pp][i] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // Per ECM point: the T products first, then the KaF and KFF products (their
    // matrix time covers the latency of T), then per mode tile tj the hi/lo
    // split of T_tj followed at once by the Kaa products of column tj, so the
    // split of the next tile overlaps the products of this one.
    v4u32 Gc[MA];
#pragma unroll
    for (int t = 0; t < MA; t++) Gc[t] = fp[t * 64];
    // the tangent scalars of the lane's ECM point, one round ahead
    v4f xn0, xn1, xn2;
    {
        const v4f* src = (const v4f*)(qsp + (int64_t)qq * 12);
        xn0 = src[0];
        xn1 = src[1];
        xn2 = src[2];
    }
    for (int q0 = 0; q0 < A.Qpad; q0 += QR) {
        const v4f x0 = xn0, x1 = xn1, x2 = xn2;
        {
            const int qn = (q0 + QR < A.Qpad) ? q0 + QR : q0;
            const v4f* src = (const v4f*)(qsp + (int64_t)(qn + qq) * 12);
            xn0 = src[0];
            xn1 = src[1];
            xn2 = src[2];
        }
        // ---- W rows of this round: lane (pb, qq, u < 3) builds the rows
        // (i, j) = (u, 0..2) of W_{q0+qq} of point pb; the lanes u = 3 build none
        if constexpr (J2) {
            // J2 tangent rows (i, j) = (u, 0..2) from the scalars
            // (w kappa, w 2 mu th, w 2 mu thb, n xx yy zz xy yz xz):
            //   W[(i,j)][(k,l)] = w kappa d_ij d_kl + w 2 mu th (sym(d_ik d_jl) - d_ij d_kl / 3)
            //                     - w 2 mu thb n_ij n_kl
            const float a0 = x0[0], a1 = x0[1], a2 = x0[2];
            const float nv[6] = {x0[3], x1[0], x1[1], x1[2], x1[3], x2[0]};
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const float nij = (u == 0) ? nv[j2_slot(0, j)] : ((u == 1) ? nv[j2_slot(1, j)] : nv[j2_slot(2, j)]);
                float w[9];
#pragma unroll
                for (int k = 0; k < 3; k++)
#pragma unroll
                    for (int l = 0; l < 3; l++) {
                        float v = -a2 * nij * nv[j2_slot(k, l)];
                        if (u == j && k == l) v += a0 - a1 * (1.0f / 3.0f);
                        if (u == k && j == l) v += 0.5f * a1;
                        if (u == l && j == k) v += 0.5f * a1;
                        w[3 * k + l] = v;
                    }
                v4u32 rec[4];
                w_records<PREC, SPLIT>(w, rec);
                if (u < 3) {
                    v4u32* dst = sw + (pb * QR + qq) * kWR + 4 * (3 * u + j);
#pragma unroll
                    for (int gg = 0; gg < 4; gg++) dst[gg] = rec[gg];
                }
            }
        } else {
            const float F[9] = {x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3], x2[0]};
            const float c0 = x2[1], c1 = x2[2], c2 = x2[3];
            // W[(i,j)][(k,l)] = c1 F(l,i) F(j,k) + c2 F(j,i) F(l,k) + c0 [k = i][l = j]:
            // with i the lane's own index only F(., i) and the diagonal term
            // need a per-lane choice, once per round
            float fc[3], col[3], d[3];
#pragma unroll
            for (int t = 0; t < 3; t++) {
                fc[t] = (u == 0) ? F[3 * t] : ((u == 1) ? F[3 * t + 1] : F[3 * t + 2]);   // F(t, i)
                col[t] = c1 * fc[t];
                d[t] = (t == u) ? c0 : 0.f;
            }
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const float sji = c2 * fc[j];
                float w[9];
#pragma unroll
                for (int k = 0; k < 3; k++)
#pragma unroll
                    for (int l = 0; l < 3; l++)
                        w[3 * k + l] = fmaf(col[l], F[3 * j + k],
                                            fmaf(sji, F[3 * l + k], (l == j) ? d[k] : 0.f));
                v4u32 rec[4];
                w_records<PREC, SPLIT>(w, rec);
                if (u < 3) {
                    v4u32* dst = sw + (pb * QR + qq) * kWR + 4 * (3 * u + j);
#pragma unroll
                    for (int gg = 0; gg < 4; gg++) dst[gg] = rec[gg];
                }
            }
        }
        // ---- contraction over the round (LDS traffic of one wavefront is in order)
        v4u32 Wq[NP];
#pragma unroll
        for (int pp = 0; pp < NP; pp++) Wq[pp] = sw[pp * QR * kWR + wrec];
#pragma unroll(kUnrollQ)
        for (int qi = 0; qi < QR; qi++) {
            const int q = q0 + qi;
            v4u32 Wn[NP];
#pragma unroll
            for (int pp = 0; pp < NP; pp++) Wn[pp] = sw[(pp * QR + (qi + 1 < QR ? qi + 1 : qi)) * kWR + wrec];
            v4u32 Gn[MA];
            if (PF) {
                const int qn = (q + 1 < A.Qpad) ? q + 1 : q;
#pragma unroll
                for (int t = 0; t < MA; t++) Gn[t] = fp[((int64_t)qn * MA + t) * 64];
            }
            // point by point, so that one point's T is live at a time
#pragma unroll
            for (int pp = 0; pp < NP; pp++) {
                v4f T[MA];
#pragma unroll
                for (int t = 0; t < MA; t++) T[t] = Pk<PREC>::mfma(Wq[pp], Gc[t], v4f{0.f, 0.f, 0.f, 0.f});
                accFF[pp] = Pk<PREC>::mfma(Wq[pp], Ip, accFF[pp]);
                // KFa = sum_q T_q (W_q is symmetric): the T tiles summed in FP32
                // (accumulator row 4g + 3 carries no component and is skipped)
#pragma unroll
                for (int t = 0; t < MA; t++)
#pragma unroll
                    for (int e = 0; e < 3; e++) accF[pp][t][e] += T[t][e];
#pragma unroll
                for (int tj = 0; tj < MA; tj++) {
                    const v4u32 B = t_operand<PREC, SPLIT>(T[tj], in_g1);
#pragma unroll
                    for (int ti = 0; ti <= tj; ti++) {
                        const int idx = ti * MA - ti * (ti - 1) / 2 + (tj - ti);
                        acc[pp][idx] = Pk<PREC>::mfma(Gc[ti], B, acc[pp][idx]);
                    }
                }
            }
            if (PF) {
#pragma unroll
                for (int t = 0; t < MA; t++) Gc[t] = Gn[t];
            } else {
                const int qn = (q + 1 < A.Qpad) ? q + 1 : q;
#pragma unroll
                for (int t = 0; t < MA; t++) Gc[t] = fp[((int64_t)qn * MA + t) * 64];
            }
#pragma unroll
            for (int pp = 0; pp < NP; pp++) Wq[pp] = Wn[pp];
        }
    }
    // record in the condensation's order: lower 8 x 8 blocks of the augmented
    // matrix (modes, then the components at mp), entry (r, c) of block (t, u)
    // at 64 (t (t + 1) / 2 + u) + 8 (r % 8) + c % 8; each symmetric pair comes
    // from one accumulator entry (upper Kaa, the KaF tiles, KFF with I >= J)
    const int m = A.m, mp = 8 * ((m + 7) / 8);
    const int Kc = pos_comp(c);
#pragma unroll
    for (int pp = 0; pp < NP; pp++) {
        if (!valid[pp]) continue;
        float* kh = (float*)A.Khat + pl[pp] * khat_len(m, 0, true);
        auto put = [&](int r, int cc, float v) {   // r >= cc
            const int t = r >> 3, uu = cc >> 3;
            float* blk = kh + (t * (t + 1) / 2 + uu) * 64;
            blk[8 * (r & 7) + (cc & 7)] = v;
            if (t == uu) blk[8 * (cc & 7) + (r & 7)] = v;
        };
        int idx = 0;
#pragma unroll
        for (int ti = 0; ti < MA; ti++)
#pragma unroll
            for (int tj = ti; tj < MA; tj++, idx++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int R = 16 * ti + 4 * g + e, C = 16 * tj + c;
                    if (R < m && C < m && R <= C) put(C, R, acc[pp][idx][e]);
                }
#pragma unroll
        for (int t = 0; t < MA; t++)
#pragma unroll
            for (int e = 0; e < 3; e++) {
                // sum of T tiles: component row 4 g + e, mode column 16 t + c
                const int KI = pos_comp(4 * g + e), k = 16 * t + c;
                if (KI >= 0 && k < m) put(mp + KI, k, accF[pp][t][e]);
            }
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int KI = pos_comp(4 * g + e);
            if (KI >= 0 && Kc >= 0 && KI >= Kc) put(mp + KI, mp + Kc, accFF[pp][e]);
        }
    }
}

// OCC4: ask for four wavefronts per SIMD (register cap 128; one point per
// wavefront fits three without asking);
// NP: macro points per wavefront
template <int MA, int PREC, bool SPLIT, bool PF, bool OCC4, int NP, bool J2 = false>
__global__ void __launch_bounds__(256, (OCC4 && MA <= 4 && NP == 1) ? 4 : 2) k_eval_mixed(EvalArgs A) {
    __shared__ v4u32 s_w[4][kCQ * kWR];
    tan_mixed_body<MA, PREC, SPLIT, PF, NP, J2>(A, (int64_t)blockIdx.x * (4 * NP), s_w);
}

// J2 plans: one launch shape (one point per wavefront, no prefetch)
template <int PREC>
static int launch_mixed_j2(const EvalArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(a.count, 4)), block(256);
    switch ((a.m + 15) / 16) {
        case 1: hipLaunchKernelGGL((k_eval_mixed<1, PREC, true, false, false, 1, true>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_eval_mixed<2, PREC, true, false, false, 1, true>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_eval_mixed<3, PREC, true, false, false, 1, true>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_eval_mixed<4, PREC, true, false, false, 1, true>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_eval_mixed<5, PREC, true, false, false, 1, true>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_eval_mixed<6, PREC, true, false, false, 1, true>), grid, block, 0, s, a); break;
        default: return HROM_E_UNSUPPORTED;
    }
    return HROM_OK;
}

template <int PREC, bool SPLIT, bool PF, bool OCC4, int NP>
static int launch_mixed_t(const EvalArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(a.count, 4 * NP)), block(256);
    switch ((a.m + 15) / 16) {
        case 1: hipLaunchKernelGGL((k_eval_mixed<1, PREC, SPLIT, PF, OCC4, NP>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_eval_mixed<2, PREC, SPLIT, PF, OCC4, NP>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_eval_mixed<3, PREC, SPLIT, PF, OCC4, NP>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_eval_mixed<4, PREC, SPLIT, PF, OCC4, NP>), grid, block, 0, s, a); break;
        // two points per wavefront do not fit the register file beyond m = 64
        case 5: hipLaunchKernelGGL((k_eval_mixed<5, PREC, SPLIT, PF, OCC4, 1>), dim3(nblocks(a.count, 4)), block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_eval_mixed<6, PREC, SPLIT, PF, OCC4, 1>), dim3(nblocks(a.count, 4)), block, 0, s, a); break;
        default: return HROM_E_UNSUPPORTED;
    }
    return HROM_OK;
}

template <int PREC, bool SPLIT>
static int launch_mixed_v(int variant, const EvalArgs& a, hipStream_t s) {
    switch (variant) {
        case 0: return launch_mixed_t<PREC, SPLIT, true, false, 1>(a, s);
        case 1: return launch_mixed_t<PREC, SPLIT, true, true, 1>(a, s);
        case 2: return launch_mixed_t<PREC, SPLIT, false, false, 1>(a, s);
        case 3: return launch_mixed_t<PREC, SPLIT, false, true, 1>(a, s);
        case 4: return launch_mixed_t<PREC, SPLIT, false, false, 2>(a, s);
        default: return launch_mixed_t<PREC, SPLIT, true, false, 2>(a, s);
    }
}

// variants 0..3: bit 0 three wavefronts per SIMD instead of two, bit 1 no
// prefetch; 4, 5: two macro points per wavefront (without, with prefetch)
// (mixed plans require split operands: plan creation rejects single-term ones)
int launch_eval_mixed(int MT, int prec, bool split, int variant, int j2, const EvalArgs& a, hipStream_t s) {
    (void)MT;
    if (!split) return HROM_E_UNSUPPORTED;
    if (j2) {
        if (prec == HROM_MIXED_BF16) return launch_mixed_j2<HROM_MIXED_BF16>(a, s);
        if (prec == HROM_MIXED_FP16) return launch_mixed_j2<HROM_MIXED_FP16>(a, s);
        return HROM_E_INVALID;
    }
    if (prec == HROM_MIXED_BF16) return launch_mixed_v<HROM_MIXED_BF16, true>(variant, a, s);
    if (prec == HROM_MIXED_FP16) return launch_mixed_v<HROM_MIXED_FP16, true>(variant, a, s);
    return HROM_E_INVALID;
}

// ============================================================== grouped launches
__device__ inline EvalArgs group_eval_args(const GroupCall& G, int c, size_t tsz) {
    const ClusterGPU& C = G.cls[c];
    EvalArgs A;
    A.m = C.m; A.Q = C.Q; A.Qpad = C.Qpad; A.MP = C.MP; A.MT = C.MT; A.KS = C.KS;
    A.first = C.first; A.count = C.count; A.N = G.N;
    A.Ghat = C.Ghat; A.Gf = C.Gf; A.w = C.w; A.phase = C.phase; A.Fpk = C.Fpk;
    A.theta = G.theta; A.Fr = G.Fr; A.a = G.a + C.off_a;
    A.qs = (char*)G.qs + tsz * (size_t)C.ws_qs;
    A.Khat = (char*)G.Khat + tsz * (size_t)C.ws_khat;
    A.r = G.r + C.off_a; A.Pr = G.Pr; A.status = G.status;
    A.qexp = 0;
    A.kscale_out = nullptr;
    A.hist_n = nullptr;
    A.hist_t = nullptr;
    return A;
}

__global__ void k_reset_counter(int* counter) { *counter = 0; }

// FP64 plans: one persistent launch for the tangent contraction of every
// cluster: the workgroups pull 4-point tiles from a work queue sorted by
// decreasing cost (largest m first), so the uneven clusters balance over the
// CUs.  Every workgroup leaves when the queue is exhausted.
__global__ void __launch_bounds__(256, 1) k_tan_persistent(GroupCall G) {
    __shared__ int s_item;
    __shared__ double s_st[4][12 * 64];
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(G.counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= G.nitems) break;
        const WorkItem w = G.items[it];
        const int64_t pl0 = (int64_t)w.unit * 4;
        const EvalArgs A = group_eval_args(G, w.c, sizeof(double));
        switch (A.MT) {
            case 2: tan_f64_body<2>(A, pl0, s_st); break;
            case 3: tan_f64_body<3>(A, pl0, s_st); break;
            case 4: tan_f64_body<4>(A, pl0, s_st); break;
            case 5: tan_f64_body<5>(A, pl0, s_st); break;
            case 6: tan_f64_body<6>(A, pl0, s_st); break;
            default: tan_f64_body<7>(A, pl0, s_st); break;
        }
        __syncthreads();
    }
}

int launch_tan_persistent(const GroupCall& g, int grid, hipStream_t s) {
    if (g.nitems == 0) return HROM_OK;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, g.counter);
    hipLaunchKernelGGL(k_tan_persistent, dim3(grid), dim3(256), 0, s, g);
    return HROM_OK;
}

}  // namespace hrom
