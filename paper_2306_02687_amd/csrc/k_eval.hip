// Evaluation of the hyper-reduced RVE at every macro point (Sec. 3.2.1 and
// 3.3): per ECM point q the reduced kinematics F_q = Fr + sum_m a_m G_qm, the
// Neo-Hooke stress P_q and tangent A_q, and the ECM sums
//   Khat = sum_q Ghat_q^T (w_q A_q) Ghat_q,   Ghat_q = [G_q | I_9 | 0]
// whose blocks are Kaa (modes x modes), KaF (modes x macro), KFF
// (macro x macro); the FP64 kernel also carries the column w_q P_q, giving
// the residual r and the homogenised stress Pr in the same contraction.
//
// Work layout: a workgroup of 4 wavefronts evaluates 4 macro points of one
// cluster, one point per wavefront.  Each wavefront loops over the ECM points
// in chunks of 64:
//   phase A (lane = ECM point): kinematics and material law, with G read in
//            the [chunk][9][m][64] layout (coalesced); per-point scalars of
//            the tangent go to LDS;
//   phase B (MFMA): the contraction over k = (ECM point, tensor row), into
//            upper-triangular 16x16 tiles of Khat held in registers.
// G (shared by every point of the cluster) is streamed from L2; nothing of
// size Q leaves the chip.
#include <hip/hip_runtime.h>

#include "hrom_internal.h"

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

template <int I, int MT>
__device__ __forceinline__ void row_step_f64(const double* Fi, double c0, double c1, double c2,
                                             double wPI, const double (&Gc)[MT][9], bool res_lane,
                                             int res_t, v4d* acc) {
    double W[9];
    tangent_row<I>(Fi, c0, c1, c2, W);
    double Bv[MT];
#pragma unroll
    for (int t = 0; t < MT; t++) {
        double s = 0.0;
#pragma unroll
        for (int J = 0; J < 9; J++) s = fma(W[J], Gc[t][J], s);
        Bv[t] = (res_lane && t == res_t) ? wPI : s;
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

// ============================================================== FP64
template <int MT>
__global__ void __launch_bounds__(256, 1) k_eval_f64(EvalArgs A) {
    constexpr int NT = MT * (MT + 1) / 2;
    constexpr int NS = 21;   // LDS scalars per ECM point: Fi (9), c0, c1, c2, w P (9)
    __shared__ double s_st[4][NS * 64];
    __shared__ double s_a[4][kMaxModes];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    int64_t pl = (int64_t)blockIdx.x * 4 + wave;
    const bool valid = pl < A.count;
    if (!valid) pl = A.count - 1;
    const int64_t b = A.first + pl;
    const int m = A.m, MP = A.MP;
    double* st = s_st[wave];
    int bits = 0;
    for (int k = lane; k < m; k += 64) {
        const double ak = A.a[(int64_t)k * A.count + pl];
        if (!isfinite(ak)) bits |= HROM_PT_NONFINITE;
        s_a[wave][k] = ak;
    }
    double Fr[9];
#pragma unroll
    for (int I = 0; I < 9; I++) Fr[I] = A.Fr[I * A.N + b];
    const double mu0 = A.theta[0], la0 = A.theta[1], mu1 = A.theta[2], la1 = A.theta[3];
    v4d acc[NT];
#pragma unroll
    for (int i = 0; i < NT; i++) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
    const bool res_lane = (c == A.res_c);
    __syncthreads();

    for (int q0 = 0; q0 < A.Qpad; q0 += 64) {
        // ---------------- phase A: lane = ECM point q0 + lane
        {
            const int q = q0 + lane;
            double F[9];
#pragma unroll
            for (int I = 0; I < 9; I++) F[I] = Fr[I];
            const double* gt = A.GT + (int64_t)(q0 >> 6) * 9 * m * 64 + lane;
            for (int k = 0; k < m; k++) {
                const double ak = s_a[wave][k];
#pragma unroll
                for (int I = 0; I < 9; I++) F[I] = fma(ak, gt[(int64_t)(I * m + k) * 64], F[I]);
            }
            const double wq = A.w[q];
            const int ph = A.phase[q];
            const double mu = ph ? mu1 : mu0, la = ph ? la1 : la0;
            double Fi[9];
            const double J = inv3d(F, Fi);
            double c0 = 0.0, c1 = 0.0, c2 = 0.0, wP[9];
            const bool ok = (q < A.Q) && (J > 0.0);
            if (q < A.Q && !(J > 0.0)) bits |= HROM_PT_JNONPOS;
            const double ell = ok ? log(J) : 0.0;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++)
                    wP[3 * i + j] = ok ? wq * (mu * (F[3 * i + j] - Fi[3 * j + i]) + la * ell * Fi[3 * j + i])
                                       : 0.0;
            if (ok) {
                c0 = wq * mu;
                c1 = wq * (mu - la * ell);
                c2 = wq * la;
            }
#pragma unroll
            for (int k = 0; k < 9; k++) st[k * 64 + lane] = ok ? Fi[k] : 0.0;
            st[9 * 64 + lane] = c0;
            st[10 * 64 + lane] = c1;
            st[11 * 64 + lane] = c2;
#pragma unroll
            for (int k = 0; k < 9; k++) st[(12 + k) * 64 + lane] = wP[k];
        }
        __syncthreads();
        // ---------------- phase B: MFMA over k = (ECM point, row I); lane group g
        // takes ECM point q0 + 4 qb + g, all 16 lanes of a group share it.
        for (int qb = 0; qb < 16; qb++) {
            const int qq = 4 * qb + g;
            const double* gh = A.Ghat + (int64_t)(q0 + qq) * 9 * MP + c;
            double Gc[MT][9];
#pragma unroll
            for (int t = 0; t < MT; t++)
#pragma unroll
                for (int J = 0; J < 9; J++) Gc[t][J] = gh[J * MP + 16 * t];
            double Fi[9];
#pragma unroll
            for (int k = 0; k < 9; k++) Fi[k] = st[k * 64 + qq];
            const double c0 = st[9 * 64 + qq], c1 = st[10 * 64 + qq], c2 = st[11 * 64 + qq];
            const double* wp = st + 12 * 64 + qq;
            row_step_f64<0, MT>(Fi, c0, c1, c2, wp[0 * 64], Gc, res_lane, A.res_t, acc);
            row_step_f64<1, MT>(Fi, c0, c1, c2, wp[1 * 64], Gc, res_lane, A.res_t, acc);
            row_step_f64<2, MT>(Fi, c0, c1, c2, wp[2 * 64], Gc, res_lane, A.res_t, acc);
            row_step_f64<3, MT>(Fi, c0, c1, c2, wp[3 * 64], Gc, res_lane, A.res_t, acc);
            row_step_f64<4, MT>(Fi, c0, c1, c2, wp[4 * 64], Gc, res_lane, A.res_t, acc);
            row_step_f64<5, MT>(Fi, c0, c1, c2, wp[5 * 64], Gc, res_lane, A.res_t, acc);
            row_step_f64<6, MT>(Fi, c0, c1, c2, wp[6 * 64], Gc, res_lane, A.res_t, acc);
            row_step_f64<7, MT>(Fi, c0, c1, c2, wp[7 * 64], Gc, res_lane, A.res_t, acc);
            row_step_f64<8, MT>(Fi, c0, c1, c2, wp[8 * 64], Gc, res_lane, A.res_t, acc);
        }
        __syncthreads();
    }

    // status of the point: OR over lanes
    const uint64_t bad_j = __ballot(bits & HROM_PT_JNONPOS);
    const uint64_t bad_n = __ballot(bits & HROM_PT_NONFINITE);
    if (!valid) return;
    if (lane == 0 && (bad_j | bad_n))
        A.status[b] |= (bad_j ? HROM_PT_JNONPOS : 0) | (bad_n ? HROM_PT_NONFINITE : 0);
    double* kh = (double*)A.Khat + (int64_t)pl * NT * 256 + lane * 4;
#pragma unroll
    for (int i = 0; i < NT; i++) *(v4d*)(kh + i * 256) = acc[i];
    // residual column m + 9: r (rows < m) and Pr (rows m .. m+8)
    if (res_lane) {
#pragma unroll
        for (int ti = 0; ti < MT; ti++) {
            const int idx = ti * MT - ti * (ti - 1) / 2 + (MT - 1 - ti);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = 16 * ti + g + 4 * e;   // FP64 MFMA accumulator rows interleave
                const double v = acc[idx][e];
                if (row < m) A.r[(int64_t)row * A.count + pl] = v;
                else if (row < m + 9) A.Pr[(int64_t)(row - m) * A.N + b] = v;
            }
        }
    }
}

int launch_eval_f64(int MT, const EvalArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(a.count, 4)), block(256);
    switch (MT) {
        case 2: hipLaunchKernelGGL(k_eval_f64<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_eval_f64<3>, grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_eval_f64<4>, grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL(k_eval_f64<5>, grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL(k_eval_f64<6>, grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL(k_eval_f64<7>, grid, block, 0, s, a); break;
        default: return HROM_E_UNSUPPORTED;
    }
    return HROM_OK;
}

// ============================================================== mixed
// Low-precision operand types.  bf16 fragments are carried as 16-bit
// patterns; the conversion rounds to nearest even.
typedef short v4s __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned short v4u __attribute__((ext_vector_type(4)));

template <int PREC>
struct LP;

template <>
struct LP<HROM_MIXED_BF16> {
    static __device__ __forceinline__ unsigned short cvt(float x) {
        uint32_t u = __float_as_uint(x);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (unsigned short)(u >> 16);
    }
    static __device__ __forceinline__ float back(unsigned short h) {
        return __uint_as_float(((uint32_t)h) << 16);
    }
    static __device__ __forceinline__ v4f mfma16(v4u a, v4u b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, a),
                                                         __builtin_bit_cast(v4s, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ v4f mfma32(v4u a0, v4u a1, v4u b0, v4u b1, v4f c) {
        typedef unsigned short v8u __attribute__((ext_vector_type(8)));
        const v8u a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
        const v8u b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                       __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
    }
};

template <>
struct LP<HROM_MIXED_FP16> {
    static __device__ __forceinline__ unsigned short cvt(float x) {
        return __builtin_bit_cast(unsigned short, (_Float16)x);
    }
    static __device__ __forceinline__ float back(unsigned short h) {
        return (float)__builtin_bit_cast(_Float16, h);
    }
    static __device__ __forceinline__ v4f mfma16(v4u a, v4u b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, a),
                                                     __builtin_bit_cast(v4h, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ v4f mfma32(v4u a0, v4u a1, v4u b0, v4u b1, v4f c) {
        typedef unsigned short v8u __attribute__((ext_vector_type(8)));
        const v8u a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
        const v8u b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a),
                                                      __builtin_bit_cast(v8h, b), c, 0, 0, 0);
    }
};

template <int PREC>
__device__ __forceinline__ void split4(const float* x, v4u& hi, v4u& lo) {
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const unsigned short h = LP<PREC>::cvt(x[e]);
        hi[e] = h;
        lo[e] = LP<PREC>::cvt(x[e] - LP<PREC>::back(h));
    }
}

// Mixed path.  Kinematics, stress, residual and homogenised stress in FP64;
// the tangent A_q in FP32; the contraction Khat = sum_q Ghat_q^T (w_q A_q) Ghat_q
// on BF16/FP16 MFMA with FP32 accumulation, in two chained steps per ECM point:
//   T_q = (w_q A_q) Ghat_q       16x16x16 MFMA, rows I of T come out in the
//                                accumulator layout (lane (g,c): rows 4g..4g+3,
//                                column c), which is the B-operand layout of
//   Khat += Ghat^T [T_q0 ; T_q1] 16x16x32 MFMA over a pair of ECM points.
// With SPLIT every operand x is carried as hi + lo (both low precision) and
// each product as hi*hi + lo*hi + hi*lo.
template <int MT, int PREC, bool SPLIT>
__global__ void __launch_bounds__(256, 1) k_eval_mixed(EvalArgs A) {
    constexpr int NT = MT * (MT + 1) / 2;
    constexpr int QC = 32;   // ECM points per chunk
    __shared__ float s_W[4][QC * 81];
    __shared__ double s_wP[4][9 * QC];
    __shared__ double s_a[4][kMaxModes];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    int64_t pl = (int64_t)blockIdx.x * 4 + wave;
    const bool valid = pl < A.count;
    if (!valid) pl = A.count - 1;
    const int64_t b = A.first + pl;
    const int m = A.m, MP = A.MP;
    int bits = 0;
    for (int k = lane; k < m; k += 64) {
        const double ak = A.a[(int64_t)k * A.count + pl];
        if (!isfinite(ak)) bits |= HROM_PT_NONFINITE;
        s_a[wave][k] = ak;
    }
    double Fr[9];
#pragma unroll
    for (int I = 0; I < 9; I++) Fr[I] = A.Fr[I * A.N + b];
    const double mu0 = A.theta[0], la0 = A.theta[1], mu1 = A.theta[2], la1 = A.theta[3];
    const float wscale = A.wscale;
    v4f acc[NT];
#pragma unroll
    for (int i = 0; i < NT; i++) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
    double Pacc[9];
#pragma unroll
    for (int I = 0; I < 9; I++) Pacc[I] = 0.0;
    double racc0 = 0.0, racc1 = 0.0;   // residual of modes lane and lane + 64
    float* sW = s_W[wave];
    double* swP = s_wP[wave];
    __syncthreads();

    for (int q0 = 0; q0 < A.Qpad; q0 += QC) {
        // ---------------- phase A: lanes 0..31 = ECM points q0 .. q0+31
        if (lane < QC) {
            const int q = q0 + lane;
            double F[9];
#pragma unroll
            for (int I = 0; I < 9; I++) F[I] = Fr[I];
            const double* gt = A.GT + (int64_t)(q >> 6) * 9 * m * 64 + (q & 63);
            for (int k = 0; k < m; k++) {
                const double ak = s_a[wave][k];
#pragma unroll
                for (int I = 0; I < 9; I++) F[I] = fma(ak, gt[(int64_t)(I * m + k) * 64], F[I]);
            }
            const double wq = A.w[q];
            const int ph = A.phase[q];
            const double mu = ph ? mu1 : mu0, la = ph ? la1 : la0;
            double Fi[9];
            const double J = inv3d(F, Fi);
            const bool ok = (q < A.Q) && (J > 0.0);
            if (q < A.Q && !(J > 0.0)) bits |= HROM_PT_JNONPOS;
            const double ell = ok ? log(J) : 0.0;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    const double v = ok ? wq * (mu * (F[3 * i + j] - Fi[3 * j + i]) + la * ell * Fi[3 * j + i])
                                        : 0.0;
                    swP[(3 * i + j) * QC + lane] = v;
                    Pacc[3 * i + j] += v;
                }
            // FP32 tangent, scaled by a power of two for the low-precision range
            float Fif[9];
#pragma unroll
            for (int k = 0; k < 9; k++) Fif[k] = ok ? (float)Fi[k] : 0.f;
            const float c0 = ok ? (float)(wq * mu) * wscale : 0.f;
            const float c1 = ok ? (float)(wq * (mu - la * ell)) * wscale : 0.f;
            const float c2 = ok ? (float)(wq * la) * wscale : 0.f;
            float* wr = sW + lane * 81;
            float Wrow[9];
            tangent_row<0>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[0 * 9 + J2] = Wrow[J2];
            tangent_row<1>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[1 * 9 + J2] = Wrow[J2];
            tangent_row<2>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[2 * 9 + J2] = Wrow[J2];
            tangent_row<3>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[3 * 9 + J2] = Wrow[J2];
            tangent_row<4>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[4 * 9 + J2] = Wrow[J2];
            tangent_row<5>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[5 * 9 + J2] = Wrow[J2];
            tangent_row<6>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[6 * 9 + J2] = Wrow[J2];
            tangent_row<7>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[7 * 9 + J2] = Wrow[J2];
            tangent_row<8>(Fif, c0, c1, c2, Wrow);
#pragma unroll
            for (int J2 = 0; J2 < 9; J2++) wr[8 * 9 + J2] = Wrow[J2];
        }
        __syncthreads();
        // ---------------- phase R: FP64 residual, lane = mode
        {
            const double* gh = A.Ghat + (int64_t)q0 * 9 * MP;
            for (int qq = 0; qq < QC; qq++) {
#pragma unroll
                for (int I = 0; I < 9; I++) {
                    const double wp = swP[I * QC + qq];
                    const double* row = gh + (int64_t)(qq * 9 + I) * MP;
                    if (lane < m) racc0 = fma(wp, row[lane], racc0);
                    if (lane + 64 < m) racc1 = fma(wp, row[lane + 64], racc1);
                }
            }
        }
        // ---------------- phase B: chained MFMA over pairs of ECM points
        for (int qp = 0; qp < QC / 2; qp++) {
            v4u Gh[2][MT], Gl[2][MT], Th[2][MT], Tl[2][MT];
#pragma unroll
            for (int s2 = 0; s2 < 2; s2++) {
                const int qq = 2 * qp + s2;
                const int q = q0 + qq;
                // W fragment: lane (g, c) holds W[I = c][J = 4g + e]
                float wv[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int J2 = 4 * g + e;
                    wv[e] = (c < 9 && J2 < 9) ? sW[qq * 81 + c * 9 + J2] : 0.f;
                }
                v4u Wh, Wl;
                split4<PREC>(wv, Wh, Wl);
                const v4u* fh = (const v4u*)(A.Fhi) + ((int64_t)q * MT) * 64 + lane;
                const v4u* fl = (const v4u*)(A.Flo) + ((int64_t)q * MT) * 64 + lane;
#pragma unroll
                for (int t = 0; t < MT; t++) {
                    Gh[s2][t] = fh[t * 64];
                    if (SPLIT) Gl[s2][t] = fl[t * 64];
                }
#pragma unroll
                for (int t = 0; t < MT; t++) {
                    v4f T = v4f{0.f, 0.f, 0.f, 0.f};
                    T = LP<PREC>::mfma16(Wh, Gh[s2][t], T);
                    if (SPLIT) {
                        T = LP<PREC>::mfma16(Wl, Gh[s2][t], T);
                        T = LP<PREC>::mfma16(Wh, Gl[s2][t], T);
                    }
                    float tv[4] = {T[0], T[1], T[2], T[3]};
                    split4<PREC>(tv, Th[s2][t], Tl[s2][t]);
                }
            }
            int idx = 0;
#pragma unroll
            for (int ti = 0; ti < MT; ti++)
#pragma unroll
                for (int tj = ti; tj < MT; tj++) {
                    acc[idx] = LP<PREC>::mfma32(Gh[0][ti], Gh[1][ti], Th[0][tj], Th[1][tj], acc[idx]);
                    if (SPLIT) {
                        acc[idx] = LP<PREC>::mfma32(Gl[0][ti], Gl[1][ti], Th[0][tj], Th[1][tj], acc[idx]);
                        acc[idx] = LP<PREC>::mfma32(Gh[0][ti], Gh[1][ti], Tl[0][tj], Tl[1][tj], acc[idx]);
                    }
                    idx++;
                }
        }
        __syncthreads();
    }

    // homogenised stress: fixed-order butterfly over the 64 lanes
#pragma unroll
    for (int I = 0; I < 9; I++) {
        double v = Pacc[I];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        Pacc[I] = v;
    }
    const uint64_t bad_j = __ballot(bits & HROM_PT_JNONPOS);
    const uint64_t bad_n = __ballot(bits & HROM_PT_NONFINITE);
    if (!valid) return;
    if (lane == 0 && (bad_j | bad_n))
        A.status[b] |= (bad_j ? HROM_PT_JNONPOS : 0) | (bad_n ? HROM_PT_NONFINITE : 0);
    if (lane < 9) {
        double v = 0.0;
#pragma unroll
        for (int I = 0; I < 9; I++) v = (lane == I) ? Pacc[I] : v;
        A.Pr[(int64_t)lane * A.N + b] = v;
    }
    if (lane < m) A.r[(int64_t)lane * A.count + pl] = racc0;
    if (lane + 64 < m) A.r[(int64_t)(lane + 64) * A.count + pl] = racc1;
    float* kh = (float*)A.Khat + (int64_t)pl * NT * 256 + lane * 4;
#pragma unroll
    for (int i = 0; i < NT; i++) *(v4f*)(kh + i * 256) = acc[i];
}

template <int PREC, bool SPLIT>
static int launch_mixed_t(int MT, const EvalArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(a.count, 4)), block(256);
    switch (MT) {
        case 2: hipLaunchKernelGGL((k_eval_mixed<2, PREC, SPLIT>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_eval_mixed<3, PREC, SPLIT>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_eval_mixed<4, PREC, SPLIT>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_eval_mixed<5, PREC, SPLIT>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_eval_mixed<6, PREC, SPLIT>), grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL((k_eval_mixed<7, PREC, SPLIT>), grid, block, 0, s, a); break;
        default: return HROM_E_UNSUPPORTED;
    }
    return HROM_OK;
}

int launch_eval_mixed(int MT, int prec, bool split, const EvalArgs& a, hipStream_t s) {
    if (prec == HROM_MIXED_BF16)
        return split ? launch_mixed_t<HROM_MIXED_BF16, true>(MT, a, s)
                     : launch_mixed_t<HROM_MIXED_BF16, false>(MT, a, s);
    if (prec == HROM_MIXED_FP16)
        return split ? launch_mixed_t<HROM_MIXED_FP16, true>(MT, a, s)
                     : launch_mixed_t<HROM_MIXED_FP16, false>(MT, a, s);
    return HROM_E_INVALID;
}

}  // namespace hrom
