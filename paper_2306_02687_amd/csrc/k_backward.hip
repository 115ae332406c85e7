// Adjoint backward through the converged ROM state.  With the RVE-frame
// cotangent g_r and the adjoint solution lambda = Kaa^{-T} KaF g_r, every ECM
// point is re-evaluated (F_q and the tangent are recomputed, never stored):
//   v_q   = g_r - G_q lambda
//   h_r  += w_q A_q v_q                               (= Cr^T g_r)
//   dmu_p  += w_q v_q : (F_q - F_q^{-T}),  dlam_p += w_q v_q : (ln J_q F_q^{-T})
// for the phase p of q.  Optionally the refinement residual
//   rho = sum_q G_q^T (w_q A_q v_q)  (= KaF g_r - Kaa lambda)
// of the adjoint system is accumulated with the same operator (for mixed
// plans in FP64: the residual of their iterative refinement).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "hrom_internal.h"

namespace hrom {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f bf16_mfma(v4u32 a, v4u32 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
}

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

// The law and its adjoint at one (point, ECM point) pair in precision T: F^-1
// and ln J of F_q, A v, and the contractions v : dP/dmu = v : (F - F^-T),
// v : dP/dlam = v : (ln J F^-T).  ok: J > 0 (else Av, dmu, dla are not used).
// FP32 (the mixed pass): reciprocal of J to one ulp, the library log.
template <typename T>
__device__ __forceinline__ bool pair_law(const T* F, const T* v, T mu, T la, T* Av, T& dmu, T& dla) {
    const T c00 = F[4] * F[8] - F[5] * F[7];
    const T c01 = F[5] * F[6] - F[3] * F[8];
    const T c02 = F[3] * F[7] - F[4] * F[6];
    const T J = F[0] * c00 + F[1] * c01 + F[2] * c02;
    T id;
    if constexpr (std::is_same<T, float>::value) id = __builtin_amdgcn_rcpf(J);
    else id = 1.0 / J;
    T Fi[9];
    Fi[0] = c00 * id;
    Fi[3] = c01 * id;
    Fi[6] = c02 * id;
    Fi[1] = (F[2] * F[7] - F[1] * F[8]) * id;
    Fi[4] = (F[0] * F[8] - F[2] * F[6]) * id;
    Fi[7] = (F[1] * F[6] - F[0] * F[7]) * id;
    Fi[2] = (F[1] * F[5] - F[2] * F[4]) * id;
    Fi[5] = (F[2] * F[3] - F[0] * F[5]) * id;
    Fi[8] = (F[0] * F[4] - F[1] * F[3]) * id;
    const bool ok = J > T(0);
    const T ell = ok ? log(J) : T(0);
    nh_apply<T>(Fi, mu, la, ell, v, Av);
    T sm = T(0), sl = T(0);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            sm = fma(v[3 * i + j], F[3 * i + j] - Fi[3 * j + i], sm);
            sl = fma(v[3 * i + j], Fi[3 * j + i], sl);
        }
    dmu = sm;
    dla = ell * sl;
    return ok;
}



// Point-batched form of the adjoint re-evaluation: 32 macro points per
// workgroup of NW = 4 or 8 wavefronts; F_q - Fr = G a and G lambda are GEMMs
// with the cluster's G as the shared operand, the law and its adjoint run per
// (point, ECM point) pair (eight waves: one pair per thread; four waves: the
// pairs (p, s) and (p, s + 8) of one point per thread); the refinement
// residual rho = G^T (w A v) is a third FP64 GEMM in four k-ranges.  Per-point
// sums over the ECM points (h_r, dL/dtheta) reduce in a fixed order.
// FP64 operator: FP64 MFMA (two 16-point column tiles), wave w taking row
// tiles w (+ NW ...) < 8 of the round's 144 rows (ECM point, component) and
// waves 0..3 one of the four products (F or G lambda, column tile) of tile 8.
// Mixed path (its law evaluates A v in FP32 and F_q, v_q sit in LDS as FP32,
// so that four wavefronts fit two workgroups per CU): both GEMMs on BF16
// MFMA with G, a and lambda split into three BF16 levels each (six level
// pairs per mode, FP32 accumulation: FP32-level results at a fifth of the
// FP64 matrix time); waves 0, 1 form F, waves 2, 3 G lambda, each for all 32
// points over alternate row tiles, with its a or lambda fragments built once
// in registers.
constexpr int kBwPT = 32;
template <int AR, typename LT>
struct BwLds {
    double sA[AR][kBwPT];
    double sL[AR][kBwPT];
    LT sF[16 * 9][kBwPT + 1];
    LT sV[16 * 9][kBwPT + 1];
    double sU[9][kBwPT];
    double sG[9][kBwPT];
    double sWq[16];
    int sPh[16];
    int sbits[kBwPT];
};

template <int MA, bool MIXED, bool RHO, int NW, int AR, typename LT>
__device__ void bw_body(const BackwardArgs& A, int64_t p0, BwLds<AR, LT>& Ls) {
    constexpr int PT = kBwPT, QC = 16, NT = 64 * NW;
    static_assert(NW == 4 || NW == 8, "four or eight wavefronts");
    static_assert(MIXED || AR >= 16 * MA, "mode amplitude rows");
    static_assert(!MIXED || NW == 4, "the mixed pass runs with four wavefronts");
    auto& sA = Ls.sA;
    auto& sL = Ls.sL;
    auto& sF = Ls.sF;
    auto& sV = Ls.sV;
    auto& sU = Ls.sU;
    auto& sG = Ls.sG;
    auto& sbits = Ls.sbits;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, c = lane & 15;
    const int m = A.m, MP = A.MP;
    constexpr int KS = 4 * MA;   // k-steps of the G a GEMM (the plan pads them to whole mode tiles)
    const int np = (int)min((int64_t)PT, A.count - p0);
    if (RHO) {
        // refinement pass: nothing to do once every point of the workgroup has converged
        if (tid < PT) sbits[tid] = (tid < np && !A.conv[p0 + tid]) ? 1 : 0;
        __syncthreads();
        int live = 0;
#pragma unroll 1
        for (int p = 0; p < PT; p++) live |= sbits[p];
        if (!live) return;
        __syncthreads();
    }
    if (tid < PT) sbits[tid] = 0;
    if constexpr (!MIXED) {
        for (int e = tid; e < 4 * KS * PT; e += NT) {
            const int k = e / PT, p = e % PT;
            const bool in = (k < m && p < np);
            sA[k][p] = in ? A.a[(int64_t)k * A.count + p0 + p] : 0.0;
            sL[k][p] = in ? A.lam[(int64_t)k * A.count + p0 + p] : 0.0;
        }
    }
    // mixed pass: this wave's B fragments, lane (g, c) holding the three BF16
    // levels of modes 32 h + 8 g .. + 7 of point 16 pt + c (a for waves 0, 1,
    // lambda for waves 2, 3; zero beyond m and beyond the workgroup's points)
    constexpr int NH = MIXED ? (MA + 1) / 2 : 1;
    v4u32 Bf[2][NH][3];
    if constexpr (MIXED) {
        const double* src = (wave >> 1) ? A.lam : A.a;
#pragma unroll
        for (int pt = 0; pt < 2; pt++)
#pragma unroll
            for (int hh = 0; hh < NH; hh++) {
                uint32_t wd[3][4];
#pragma unroll
                for (int d = 0; d < 4; d++) {
                    wd[0][d] = wd[1][d] = wd[2][d] = 0u;
#pragma unroll
                    for (int ii = 0; ii < 2; ii++) {
                        const int k = 32 * hh + 8 * g + 2 * d + ii, p = 16 * pt + c;
                        const double v = (k < m && p < np) ? src[(int64_t)k * A.count + p0 + p] : 0.0;
                        uint16_t lv[3];
                        bf16_split3(v, lv);
#pragma unroll
                        for (int L = 0; L < 3; L++) wd[L][d] |= (uint32_t)lv[L] << (16 * ii);
                    }
                }
#pragma unroll
                for (int L = 0; L < 3; L++) Bf[pt][hh][L] = v4u32{wd[L][0], wd[L][1], wd[L][2], wd[L][3]};
            }
    }
    for (int e = tid; e < 9 * PT; e += NT) {
        const int I = e / PT, p = e % PT;
        const int64_t b = A.first + p0 + p;
        sU[I][p] = (p < np) ? A.Fr[(int64_t)I * A.N + b] : ((I % 4 == 0) ? 1.0 : 0.0);
        sG[I][p] = (p < np) ? A.gr[(int64_t)I * A.N + b] : 0.0;
    }
    const double mu0 = A.theta[0], la0 = A.theta[1], mu1 = A.theta[2], la1 = A.theta[3];
    // law pairs of this thread: (point pp, ECM points qa + 8 h)
    constexpr int NPAIR = 8 / NW, LPP = 16 / NPAIR;   // pairs per thread, lanes per point
    const int pp = tid / LPP, qa = tid % LPP;
    double h[9], gt[4];
#pragma unroll
    for (int I = 0; I < 9; I++) h[I] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++) gt[i] = 0.0;
    // rho GEMM: wave w takes the mode tiles of parity w & 1 over the k-range
    // w >> 1 (18 of the round's 36 k-steps)
    static_assert(!RHO || NW == 4, "the rho pass runs with four wavefronts");
    const int tpar = wave & 1, krange = wave >> 1;
    constexpr int RT = RHO ? (MA + 1) / 2 : 1;
    v4d racc[RT][2];
#pragma unroll
    for (int u = 0; u < RT; u++) racc[u][0] = racc[u][1] = v4d{0.0, 0.0, 0.0, 0.0};
    __syncthreads();

    for (int q0 = 0; q0 < A.Qpad; q0 += QC) {
        const int rt0 = (q0 / 16) * 9;
        // weights and phases of the round's ECM points: loaded here, stored to
        // LDS after the GEMMs (their latency hidden behind the products)
        double wnext = 0.0;
        int phnext = 0;
        if (tid < QC) {
            wnext = A.w[q0 + tid];
            phnext = A.phase[q0 + tid];
        }
        if constexpr (MIXED) {
            // F (waves 0, 1) or G lambda (waves 2, 3) over row tiles of the
            // parity of the wave; per output tile the six level pairs of every
            // mode half, the small products first and the hi * hi ones last
            const bool isF = wave < 2;
            // the next row tile's fragments are loaded while this one's
            // products run (the last tile reloads itself)
            v4u32 Af[NH][3];
            {
                const v4u32* ga = reinterpret_cast<const v4u32*>(A.Gb3) + ((int64_t)(rt0 + (wave & 1)) * NH * 3) * 64 + lane;
#pragma unroll
                for (int hh = 0; hh < NH; hh++)
#pragma unroll
                    for (int L = 0; L < 3; L++) Af[hh][L] = ga[(hh * 3 + L) * 64];
            }
            for (int rt = wave & 1; rt < 9; rt += 2) {
                const int rn = (rt + 2 < 9) ? rt + 2 : rt;
                const v4u32* gn = reinterpret_cast<const v4u32*>(A.Gb3) + ((int64_t)(rt0 + rn) * NH * 3) * 64 + lane;
                v4u32 An[NH][3];
#pragma unroll
                for (int hh = 0; hh < NH; hh++)
#pragma unroll
                    for (int L = 0; L < 3; L++) An[hh][L] = gn[(hh * 3 + L) * 64];
                v4f acc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
                for (int hh = 0; hh < NH; hh++)
#pragma unroll
                    for (int pt = 0; pt < 2; pt++) {
                        acc[pt] = bf16_mfma(Af[hh][0], Bf[pt][hh][2], acc[pt]);
                        acc[pt] = bf16_mfma(Af[hh][2], Bf[pt][hh][0], acc[pt]);
                        acc[pt] = bf16_mfma(Af[hh][1], Bf[pt][hh][1], acc[pt]);
                        acc[pt] = bf16_mfma(Af[hh][0], Bf[pt][hh][1], acc[pt]);
                        acc[pt] = bf16_mfma(Af[hh][1], Bf[pt][hh][0], acc[pt]);
                    }
#pragma unroll
                for (int hh = 0; hh < NH; hh++)
#pragma unroll
                    for (int pt = 0; pt < 2; pt++) acc[pt] = bf16_mfma(Af[hh][0], Bf[pt][hh][0], acc[pt]);
                // accumulator element e: row 4 g + e of the tile, point 16 pt + c
#pragma unroll
                for (int pt = 0; pt < 2; pt++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const int row = 16 * rt + 4 * g + e, col = 16 * pt + c;
                        if (isF) sF[row][col] = (LT)((double)acc[pt][e] + sU[row % 9][col]);
                        else sV[row][col] = (LT)(sG[row % 9][col] - (double)acc[pt][e]);
                    }
#pragma unroll
                for (int hh = 0; hh < NH; hh++)
#pragma unroll
                    for (int L = 0; L < 3; L++) Af[hh][L] = An[hh][L];
            }
        } else {
#pragma unroll
        for (int hh = 0; hh < 8 / NW; hh++) {
            const int rt = wave + NW * hh;
            const double* gf = A.Gf + ((int64_t)(rt0 + rt) * KS) * 64 + lane;
            double af[4 * MA];
#pragma unroll
            for (int s2 = 0; s2 < 4 * MA; s2++)
                af[s2] = gf[(int64_t)s2 * 64];
            v4d f0 = v4d{0.0, 0.0, 0.0, 0.0}, f1 = f0, l0 = f0, l1 = f0;
#pragma unroll
            for (int s2 = 0; s2 < KS; s2++)
                {
                    f0 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s2], sA[4 * s2 + g][c], f0, 0, 0, 0);
                    f1 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s2], sA[4 * s2 + g][16 + c], f1, 0, 0, 0);
                    l0 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s2], sL[4 * s2 + g][c], l0, 0, 0, 0);
                    l1 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s2], sL[4 * s2 + g][16 + c], l1, 0, 0, 0);
                }
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = 16 * rt + g + 4 * e;   // FP64 MFMA accumulator rows interleave
                sF[row][c] = (LT)(f0[e] + sU[row % 9][c]);
                sF[row][16 + c] = (LT)(f1[e] + sU[row % 9][16 + c]);
                sV[row][c] = (LT)(sG[row % 9][c] - l0[e]);
                sV[row][16 + c] = (LT)(sG[row % 9][16 + c] - l1[e]);
            }
        }
        if (wave < 4) {
            // row tile 8: wave 0 / 1 the F columns 0..15 / 16..31, wave 2 / 3 G lambda
            const double* gf = A.Gf + ((int64_t)(rt0 + 8) * KS) * 64 + lane;
            const int col = 16 * (wave & 1) + c;
            const bool isF = wave < 2;
            v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s2 = 0; s2 < KS; s2++)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(gf[(int64_t)s2 * 64],
                                                               isF ? sA[4 * s2 + g][col] : sL[4 * s2 + g][col],
                                                               acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = 128 + g + 4 * e;
                if (isF) sF[row][col] = (LT)(acc[e] + sU[row % 9][col]);
                else sV[row][col] = (LT)(sG[row % 9][col] - acc[e]);
            }
        }
        }
        if (tid < QC) {
            Ls.sWq[tid] = wnext;
            Ls.sPh[tid] = phnext;
        }
        __syncthreads();
#pragma unroll 1
        for (int k2 = 0; k2 < NPAIR; k2++) {
            const int p = pp, qq = qa + LPP * k2, q = q0 + qq;
            const double wq = Ls.sWq[qq];
            const int ph = Ls.sPh[qq];
            const bool live = (q < A.Q) && (p < np);
            using CT = typename std::conditional<MIXED, float, double>::type;
            CT F[9], v[9], Av[9], dmu, dla;
#pragma unroll
            for (int I = 0; I < 9; I++) {
                F[I] = (CT)sF[qq * 9 + I][p];
                v[I] = (CT)sV[qq * 9 + I][p];
            }
            const double mu = ph ? mu1 : mu0, la = ph ? la1 : la0;
            const bool ok = pair_law<CT>(F, v, (CT)mu, (CT)la, Av, dmu, dla) && live;
            if (live && !ok) atomicOr(&sbits[p], HROM_PT_JNONPOS);
            const double wo = ok ? wq : 0.0;
            if constexpr (RHO) {
                // the refinement pass needs only rho; h and dL/dtheta come from
                // the pass that follows it
#pragma unroll
                for (int I = 0; I < 9; I++) sV[qq * 9 + I][p] = (LT)(wo * (double)Av[I]);
            } else {
#pragma unroll
                for (int I = 0; I < 9; I++) h[I] = fma(wo, (double)Av[I], h[I]);
                const double wm = ph ? 0.0 : wo, wi = ph ? wo : 0.0;
                gt[0] = fma(wm, (double)dmu, gt[0]);
                gt[1] = fma(wm, (double)dla, gt[1]);
                gt[2] = fma(wi, (double)dmu, gt[2]);
                gt[3] = fma(wi, (double)dla, gt[3]);
            }
        }
        __syncthreads();
        if constexpr (RHO) {
            for (int j = 18 * krange; j < 18 * krange + 18; j++) {
                const double b0 = (double)sV[4 * j + g][c], b1 = (double)sV[4 * j + g][16 + c];
                const double* gh = A.Ghat + (int64_t)(q0 * 9 + 4 * j + g) * MP + c;
#pragma unroll
                for (int u = 0; u < RT; u++) {
                    const int t = 2 * u + tpar;
                    if (t < MA) {
                        const double av = gh[16 * t];
                        racc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, racc[u][0], 0, 0, 0);
                        racc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, racc[u][1], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        }
    }
    // per-point sums over the LPP threads of the point (consecutive lanes of a
    // wave): fixed butterfly
    if constexpr (!RHO) {
#pragma unroll
        for (int I = 0; I < 9; I++)
#pragma unroll
            for (int off = LPP / 2; off > 0; off >>= 1) h[I] += __shfl_xor(h[I], off);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int off = LPP / 2; off > 0; off >>= 1) gt[i] += __shfl_xor(gt[i], off);
        if (pp < np) {
            const int64_t b = A.first + p0 + pp;
            const bool failed = (A.status[b] & (HROM_PT_JNONPOS | HROM_PT_NONFINITE)) || sbits[pp];
            // outputs 0..8 = h_r, 9..12 = dL/dtheta, written by the point's lanes
#pragma unroll
            for (int o0 = 0; o0 < 13; o0 += LPP) {
                const int o = o0 + qa;
                double val = 0.0;
#pragma unroll
                for (int I = 0; I < 9; I++) val = (o == I) ? h[I] : val;
#pragma unroll
                for (int i = 0; i < 4; i++) val = (o == 9 + i) ? gt[i] : val;
                if (o < 9) A.hr[(int64_t)o * A.N + b] = failed ? 0.0 : val;
                else if (o < 13) A.gth[(int64_t)(o - 9) * A.N + b] = failed ? 0.0 : val;
            }
        }
    }
    if constexpr (RHO) {
        // fixed-order sum of the two k-range partials of rho through LDS
        double* red = reinterpret_cast<double*>(&sF[0][0]);
#pragma unroll
        for (int t = 0; t < MA; t++) {
            __syncthreads();
            if ((t & 1) == tpar) {
                const int u = t >> 1;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    red[(krange * 16 + g + 4 * e) * PT + c] = racc[u][0][e];
                    red[(krange * 16 + g + 4 * e) * PT + 16 + c] = racc[u][1][e];
                }
            }
            __syncthreads();
#pragma unroll
            for (int k2 = 0; k2 < 512 / NT; k2++) {
                const int e2 = tid + NT * k2;   // 16 rows x 32 points
                const int rr = e2 >> 5, p = e2 & 31;
                double sum = 0.0;
#pragma unroll
                for (int w = 0; w < 2; w++) sum += red[(w * 16 + rr) * PT + p];
                const int row = 16 * t + rr;
                if (p < np && row < m) A.rho[(int64_t)row * A.count + p0 + p] = sbits[p] ? 0.0 : sum;
            }
        }
    }
    __syncthreads();
    if (tid < np && sbits[tid]) A.status[A.first + p0 + tid] |= HROM_PT_JNONPOS;
}

// one launch per cluster: the mixed path with four wavefronts (two workgroups
// per CU), the FP64 path with eight; the refinement pass (the accurate
// operator of a mixed plan: FP64 law, FP64 staging) with four
template <int MA, bool MIXED, bool RHO>
__global__ void __launch_bounds__((MIXED || RHO) ? 256 : 512, MIXED ? 2 : 1) k_backward_b(BackwardArgs A) {
    __shared__ BwLds<MIXED ? 1 : 16 * MA, typename std::conditional<MIXED, float, double>::type> Ls;
    bw_body<MA, MIXED, RHO, (MIXED || RHO) ? 4 : 8>(A, (int64_t)blockIdx.x * kBwPT, Ls);
}

template <bool MIXED, bool RHO>
static int launch_bw_t(const BackwardArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.count + kBwPT - 1) / kBwPT)), block((MIXED || RHO) ? 256 : 512);
    switch ((a.m + 15) / 16) {
        case 1: hipLaunchKernelGGL((k_backward_b<1, MIXED, RHO>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_backward_b<2, MIXED, RHO>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_backward_b<3, MIXED, RHO>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_backward_b<4, MIXED, RHO>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_backward_b<5, MIXED, RHO>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_backward_b<6, MIXED, RHO>), grid, block, 0, s, a); break;
        default: return HROM_E_UNSUPPORTED;
    }
    return HROM_OK;
}

int launch_backward_b(const BackwardArgs& a, hipStream_t s) {
    // the refinement pass exists for the low-precision tangents only; its
    // residual uses the FP64 operator (FP64 law and staging), so that the
    // refined adjoint converges to the FP64 solution
    if (a.with_rho) return a.mixed ? launch_bw_t<false, true>(a, s) : HROM_E_INVALID;
    if (a.mixed) return launch_bw_t<true, false>(a, s);
    return launch_bw_t<false, false>(a, s);
}

}  // namespace hrom
