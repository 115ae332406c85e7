// Small-strain J2 (von Mises) plasticity with linear isotropic hardening at
// one ECM point, FP64: the material of the paper's Example 1 (Sec. 5), an
// elastic-plastic matrix (initial yield stress sy0, hardening modulus H) with
// elastic inclusions.  State per ECM point (Sec. 4: internal variables only
// at the hyper integration points): the plastic strain (tensor components
// xx, yy, zz, xy, yz, xz) and the equivalent plastic strain alpha.
//
// Radial return: with d = dev(eps) - eps_p (eps = sym(F) - I), the trial
// deviatoric stress is 2 mu d; it yields when 2 mu |d| exceeds
// sqrt(2/3) (sy0 + H alpha).  Then the plastic multiplier is
// g = (2 mu |d| - sqrt(2/3)(sy0 + H alpha)) / (2 mu + 2 H / 3) along
// n = d / |d|, and the consistent tangent is
//   kappa 1x1 + 2 mu th (I_sym - 1x1 / 3) - 2 mu thb n x n,
//   th = 1 - g / |d|,  thb = 1 / (1 + H / (3 mu)) - g / |d|.
// The tangent leaves as nine scalars (kappa, 2 mu th, 2 mu thb, n), from
// which the contraction rebuilds its rows.
#pragma once

#include <hip/hip_runtime.h>

namespace hrom {

// tensor-component index of the symmetric pair (i, j) in (xx, yy, zz, xy, yz, xz)
__host__ __device__ constexpr int j2_slot(int i, int j) {
    return i == j ? i : ((i + j == 1) ? 3 : ((i + j == 3) ? 4 : 5));
}

// F (3x3 row-major), material (mu, lam, sy0, H), committed state hn[7];
// returns sigma (3x3 row-major, symmetric), tangent scalars t[9] and the new
// state ht[7]
__device__ inline void j2_update(const double* F, double mu, double lam, double sy0, double H,
                                 const double* hn, double* sig, double* t, double* ht) {
    const double e[6] = {F[0] - 1.0, F[4] - 1.0, F[8] - 1.0, 0.5 * (F[1] + F[3]),
                         0.5 * (F[5] + F[7]), 0.5 * (F[2] + F[6])};
    const double vol = e[0] + e[1] + e[2];
    double d[6];
#pragma unroll
    for (int k = 0; k < 6; k++) d[k] = e[k] - (k < 3 ? vol / 3.0 : 0.0) - hn[k];
    // tensor norm: the off-diagonal components count twice
    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] +
                      2.0 * (d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
    const double dn = sqrt(dd);
    const double r23 = sqrt(2.0 / 3.0);
    const double over = 2.0 * mu * dn - r23 * (sy0 + H * hn[6]);
    double g = 0.0, inv = 0.0;
    if (over > 0.0) {
        g = over / (2.0 * mu + 2.0 * H / 3.0);
        inv = 1.0 / dn;
    }
    const double kappa = lam + 2.0 * mu / 3.0;
    const double keep = 1.0 - g * inv;   // share of the trial deviator kept
    double s[6];
#pragma unroll
    for (int k = 0; k < 6; k++) s[k] = 2.0 * mu * keep * d[k];
    sig[0] = kappa * vol + s[0];
    sig[4] = kappa * vol + s[1];
    sig[8] = kappa * vol + s[2];
    sig[1] = sig[3] = s[3];
    sig[5] = sig[7] = s[4];
    sig[2] = sig[6] = s[5];
    t[0] = kappa;
    t[1] = 2.0 * mu * keep;
    t[2] = (g > 0.0) ? 2.0 * mu * (1.0 / (1.0 + H / (3.0 * mu)) - g * inv) : 0.0;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const double nk = d[k] * inv;
        t[3 + k] = nk;
        ht[k] = hn[k] + g * nk;
    }
    ht[6] = hn[6] + r23 * g;
}

// Row I = (i, j) of the J2 tangent (scaled by the ECM weight), from the nine
// scalars wt = (w kappa, w 2 mu th, w 2 mu thb, n):
//   W[I][(k, l)] = w kappa d_ij d_kl + w 2 mu th (sym(d_ik d_jl) - d_ij d_kl / 3)
//                  - w 2 mu thb n_ij n_kl
template <int I, typename T>
__device__ __forceinline__ void j2_tangent_row(const T* wt, T* W) {
    constexpr int i = I / 3, j = I % 3;
    const T nij = wt[3 + j2_slot(i, j)];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int l = 0; l < 3; l++) {
            T v = -wt[2] * nij * wt[3 + j2_slot(k, l)];
            if (i == j && k == l) v += wt[0] - wt[1] / T(3);
            if (i == k && j == l) v += T(0.5) * wt[1];
            if (i == l && j == k) v += T(0.5) * wt[1];
            W[3 * k + l] = v;
        }
}

}  // namespace hrom
