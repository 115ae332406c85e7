// Per-macro-point kernels: polar split, push-out to the macro frame, the
// monolithic update, the backward pull-back / push-forward, reductions and
// the plan-time layout builder.  One thread per macro point (or per
// (mode, point) pair); all per-point arrays are component-major [k][N], so
// consecutive threads touch consecutive addresses.
#include <hip/hip_runtime.h>

#include "hrom_internal.h"
#include "hrom_math.h"

namespace hrom {

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- polar split
// Fbar = Rbar Ubar (Sec. 3.2.2): eigen-decomposition of C = Fbar^T Fbar,
// Ubar = V diag(sqrt c) V^T.  The RVE frame sees Fr = Ubar (objective) or
// Fr = Fbar (direct).  Non-finite input or det Fbar <= 0 flags the point and
// substitutes the identity so that no NaN leaves the point.
__global__ void __launch_bounds__(256) k_prepare(PointArgs A) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.N) return;
    const int64_t N = A.N;
    double F[9];
    int st = 0;
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        F[k] = A.Fbar[k * N + b];
        fin = fin && isfinite(F[k]);
    }
    if (!fin) st |= HROM_PT_NONFINITE;
    if (fin && A.objective && !(det3(F) > 0.0)) st |= HROM_PT_JNONPOS;
    if (st) {
#pragma unroll
        for (int k = 0; k < 9; k++) F[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    double V[9], u[3], U[9];
    if (A.objective) {
        double C[9], c[3];
        tmul3(F, F, C);
        eigsym3(C, V, c);
#pragma unroll
        for (int i = 0; i < 3; i++) u[i] = sqrt(c[i]);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                U[3 * i + j] = V[3 * i] * u[0] * V[3 * j] + V[3 * i + 1] * u[1] * V[3 * j + 1] +
                               V[3 * i + 2] * u[2] * V[3 * j + 2];
    } else {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            U[k] = F[k];
            V[k] = (k % 4 == 0) ? 1.0 : 0.0;
        }
        u[0] = u[1] = u[2] = 1.0;
    }
#pragma unroll
    for (int k = 0; k < 9; k++) {
        A.Fr[k * N + b] = U[k];
        A.polar[k * N + b] = F[k];
        A.polar[(9 + k) * N + b] = V[k];
    }
#pragma unroll
    for (int k = 0; k < 3; k++) A.polar[(18 + k) * N + b] = u[k];
    A.status[b] = st;
}

void launch_prepare(const PointArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare, dim3(nblocks(a.N, 256)), dim3(256), 0, s, a);
}

__device__ __forceinline__ void load_polar(const double* polar, int64_t N, int64_t b, double* F,
                                           double* V, double* u) {
#pragma unroll
    for (int k = 0; k < 9; k++) {
        F[k] = polar[k * N + b];
        V[k] = polar[(9 + k) * N + b];
    }
#pragma unroll
    for (int k = 0; k < 3; k++) u[k] = polar[(18 + k) * N + b];
}

// ---------------------------------------------------------------- push-out
// Biot stress T = sym(Palg_r) (eq. workconjugacy), second Piola S from
// Ubar S + S Ubar = 2 T, Pbar = Fbar S; tangent column k along E_k:
// dU = Linv(E_k^T F + F^T E_k), dT = sym(Cr dU),
// dS = Linv(2 dT - dU S - S dU), Cbar e_k = E_k S + F dS.
// One thread per (column k, macro point); the nine column threads of a point
// are neighbours in one wavefront, so the point's tangent entries are fetched
// once per wavefront; the k = 0 thread also writes Pbar, S.
__global__ void __launch_bounds__(256) k_pushout(PushArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = A.N;
    if (t >= 9 * N) return;
    const int64_t b = t / 9;
    const int kc = (int)(t - 9 * b);
    double Pa[9];
#pragma unroll
    for (int k = 0; k < 9; k++) Pa[k] = A.Palg[k * N + b];
    bool fin = true;
    if (!A.objective) {
        if (kc == 0) {
#pragma unroll
            for (int k = 0; k < 9; k++) {
                A.Pbar[k * N + b] = Pa[k];
                fin = fin && isfinite(Pa[k]);
            }
        }
#pragma unroll
        for (int I = 0; I < 9; I++) {
            const double v = A.Cr[(9 * I + kc) * N + b];
            A.Cbar[(9 * I + kc) * N + b] = v;
            fin = fin && isfinite(v);
        }
        if (!fin) atomicOr(&A.status[b], HROM_PT_NONFINITE);
        return;
    }
    double F[9], V[9], u[3];
    load_polar(A.polar, N, b, F, V, u);
    double T2[9], S[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) T2[3 * i + j] = Pa[3 * i + j] + Pa[3 * j + i];
    lyap_solve(V, u, T2, S);
    if (kc == 0) {
        double P[9];
        mul3(F, S, P);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            A.Pbar[k * N + b] = P[k];
            A.S[k * N + b] = S[k];
            fin = fin && isfinite(P[k]);
        }
    }
    const int ka = kc / 3, kb = kc % 3;   // E_k = e_ka (x) e_kb
    double dC[9], dU[9];
    // (E_k^T F)_ij = delta_{i kb} F_{ka j};  dC = E_k^T F + F^T E_k
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            dC[3 * i + j] = (i == kb ? F[3 * ka + j] : 0.0) + (j == kb ? F[3 * ka + i] : 0.0);
    lyap_solve(V, u, dC, dU);
    double dP[9];
#pragma unroll
    for (int I = 0; I < 9; I++) {
        double s = 0.0;
#pragma unroll
        for (int J = 0; J < 9; J++) s = fma(A.Cr[(9 * I + J) * N + b], dU[J], s);
        dP[I] = s;
    }
    double B[9], t1[9], t2[9], dS[9], FdS[9];
    mul3(dU, S, t1);
    mul3(S, dU, t2);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            B[3 * i + j] = (dP[3 * i + j] + dP[3 * j + i]) - t1[3 * i + j] - t2[3 * i + j];
    lyap_solve(V, u, B, dS);
    mul3(F, dS, FdS);
#pragma unroll
    for (int I = 0; I < 9; I++) {
        const int i = I / 3, j = I % 3;
        const double v = (i == ka ? S[3 * kb + j] : 0.0) + FdS[I];
        A.Cbar[(9 * I + kc) * N + b] = v;
        fin = fin && isfinite(v);
    }
    if (!fin) atomicOr(&A.status[b], HROM_PT_NONFINITE);
}

void launch_pushout(const PushArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_pushout, dim3(nblocks(9 * a.N, 256)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------- Updated-Lagrangian output
// Cauchy stress and the tangent dsigma/dD of App. A from the RVE-frame
// algorithmic stress and condensed tangent.  The Biot relation (eq.
// biotstress) T = J/2 (R^T sigma F^-T + F^-1 sigma R) reads, for the rotated
// stress Z = R^T sigma R and F = R U,  Z U^-1 + U^-1 Z = (2/J) T, i.e.
// U Z + Z U = (2/J) U T U: one symmetric Lyapunov solve in the eigenbasis of
// U, then sigma = R Z R^T.  Tangent column (k, l): stretch rate
// Udot = sym(R^T E_kl F) (constant rotation over the step), dT = sym(Cr Udot),
// dsigma = the same Biot inversion of dT.  One thread per (column, point),
// the nine columns of a point neighbours as in the push-out; the column-0
// thread also writes sigma.
__global__ void __launch_bounds__(256) k_cauchy(CauchyArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = A.N;
    if (t >= 9 * N) return;
    const int64_t b = t / 9;
    const int kc = (int)(t - 9 * b);
    double F[9], V[9], u[3];
    load_polar(A.polar, N, b, F, V, u);
    double U[9], Ui[9], R[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            U[3 * i + j] = V[3 * i] * u[0] * V[3 * j] + V[3 * i + 1] * u[1] * V[3 * j + 1] +
                           V[3 * i + 2] * u[2] * V[3 * j + 2];
            Ui[3 * i + j] = V[3 * i] / u[0] * V[3 * j] + V[3 * i + 1] / u[1] * V[3 * j + 1] +
                            V[3 * i + 2] / u[2] * V[3 * j + 2];
        }
    mul3(F, Ui, R);
    const double c2J = 2.0 / (u[0] * u[1] * u[2]);   // 2 / J, J = det U
    // sigma = R Z R^T with U Z + Z U = (2/J) U T U
    auto biot_to_cauchy = [&](const double* T, double* sig) {
        double a1[9], B[9], Z[9], RZ[9];
        mul3(U, T, a1);
        mul3(a1, U, B);
#pragma unroll
        for (int k = 0; k < 9; k++) B[k] *= c2J;
        lyap_solve(V, u, B, Z);
        mul3(R, Z, RZ);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                sig[3 * i + j] = RZ[3 * i] * R[3 * j] + RZ[3 * i + 1] * R[3 * j + 1] + RZ[3 * i + 2] * R[3 * j + 2];
    };
    bool fin = true;
    if (kc == 0) {
        double T[9], sig[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                T[3 * i + j] = 0.5 * (A.Palg[(3 * i + j) * N + b] + A.Palg[(3 * j + i) * N + b]);
        biot_to_cauchy(T, sig);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            A.sigma[k * N + b] = sig[k];
            fin = fin && isfinite(sig[k]);
        }
    }
    if (A.dsdD) {
        const int ka = kc / 3, kb = kc % 3;
        // Udot_ij = R_{ka i} F_{kb j}, symmetrised
        double dU[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                dU[3 * i + j] = 0.5 * (R[3 * ka + i] * F[3 * kb + j] + R[3 * ka + j] * F[3 * kb + i]);
        double dP[9];
#pragma unroll
        for (int I = 0; I < 9; I++) {
            double acc = 0.0;
#pragma unroll
            for (int J = 0; J < 9; J++) acc = fma(A.Cr[(9 * I + J) * N + b], dU[J], acc);
            dP[I] = acc;
        }
        double dT[9], dsig[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) dT[3 * i + j] = 0.5 * (dP[3 * i + j] + dP[3 * j + i]);
        biot_to_cauchy(dT, dsig);
#pragma unroll
        for (int I = 0; I < 9; I++) {
            A.dsdD[(9 * I + kc) * N + b] = dsig[I];
            fin = fin && isfinite(dsig[I]);
        }
    }
    if (!fin) atomicOr(&A.status[b], HROM_PT_NONFINITE);
}

// Biot stress and tangent in Voigt form from the RVE-frame condensed state
// (Sec. 3.2.2 eq. workconjugacy: the Biot stress T = sym(Palg_r) is work
// conjugate to Ubar; Sec. 3.2.3 eq. Biot_Tangent): T_k = D_k : Palg and
// CB_kl = D_k : Cr : D_l with the dual basis D = (E11, E22, E33,
// (E12 + E21) / 2, (E23 + E32) / 2, (E13 + E31) / 2), i.e. dT_k / dgamma_l
// with engineering shear strains gamma = (U11, U22, U33, 2 U12, 2 U23, 2 U13).
// One thread per (row k of CB, point); row 0 also writes T.
__global__ void __launch_bounds__(256) k_biot(BiotArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = A.N;
    if (t >= 6 * N) return;
    const int64_t b = t / 6;
    const int k = (int)(t - 6 * b);
    constexpr int c0[6] = {0, 4, 8, 1, 5, 2}, c1[6] = {0, 4, 8, 3, 7, 6};
    constexpr double dw[6] = {1.0, 1.0, 1.0, 0.5, 0.5, 0.5};
    bool fin = true;
    if (k == 0) {
#pragma unroll
        for (int l = 0; l < 6; l++) {
            const double v = (l < 3) ? A.Palg[(int64_t)c0[l] * N + b]
                                     : 0.5 * (A.Palg[(int64_t)c0[l] * N + b] + A.Palg[(int64_t)c1[l] * N + b]);
            A.T[(int64_t)l * N + b] = v;
            fin = fin && isfinite(v);
        }
    }
    if (A.CB) {
#pragma unroll
        for (int l = 0; l < 6; l++) {
            double v = 0.0;
            // D_k : Cr : D_l, D_k = sum of its components with weight dw
            for (int n = 0; n < (k < 3 ? 1 : 2); n++)
                for (int n2 = 0; n2 < (l < 3 ? 1 : 2); n2++)
                    v += A.Cr[(int64_t)(9 * (n ? c1[k] : c0[k]) + (n2 ? c1[l] : c0[l])) * N + b];
            v *= dw[k] * dw[l];
            A.CB[(int64_t)(6 * k + l) * N + b] = v;
            fin = fin && isfinite(v);
        }
    }
    if (!fin) atomicOr(&A.status[b], HROM_PT_NONFINITE);
}

void launch_biot(const BiotArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_biot, dim3(nblocks(6 * a.N, 256)), dim3(256), 0, s, a);
}

void launch_cauchy(const CauchyArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_cauchy, dim3(nblocks(9 * a.N, 256)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------- update
// linearised macro stretch increment dU = Linv(dF^T F + F^T dF) (objective)
// or dF (direct); zero when no increment is given (pure micro Newton step).
__global__ void __launch_bounds__(256) k_stretch_increment(UpdateArgs A) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.N) return;
    const int64_t N = A.N;
    double dU[9];
    if (!A.dFbar) {
#pragma unroll
        for (int k = 0; k < 9; k++) dU[k] = 0.0;
    } else if (!A.objective) {
#pragma unroll
        for (int k = 0; k < 9; k++) dU[k] = A.dFbar[k * N + b];
    } else {
        double F[9], V[9], u[3], dF[9], a1[9], dC[9];
        load_polar(A.polar, N, b, F, V, u);
#pragma unroll
        for (int k = 0; k < 9; k++) dF[k] = A.dFbar[k * N + b];
        tmul3(dF, F, a1);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) dC[3 * i + j] = a1[3 * i + j] + a1[3 * j + i];
        lyap_solve(V, u, dC, dU);
    }
#pragma unroll
    for (int k = 0; k < 9; k++) A.dU[k * N + b] = dU[k];
}

void launch_stretch_increment(const UpdateArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_stretch_increment, dim3(nblocks(a.N, 256)), dim3(256), 0, s, a);
}

// Increment of the amplitudes in the plan's mode basis, dt = y + X dU
// (Sec. 3.2.3; the caller's a then moves by R^{-1} dt), one thread per (group
// of kModesPerThread modes, point): the point's dU is read once for the
// group.  Points flagged as failed get dt = 0; without an increment (pure
// micro Newton step) so do converged points (rnorm < tol): they are frozen.
constexpr int kModesPerThread = 4;
__global__ void __launch_bounds__(256) k_update(UpdateArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ng = (A.m + kModesPerThread - 1) / kModesPerThread;
    if (t >= (int64_t)ng * A.count) return;
    const int kg = (int)(t / A.count);
    const int64_t pl = t - (int64_t)kg * A.count;
    const int64_t b = A.first + pl;
    const bool frozen = (A.status[b] & (HROM_PT_JNONPOS | HROM_PT_NONFINITE)) ||
                        (!A.dFbar && !(A.rnorm[b] >= A.tol));
    double dU[9];
#pragma unroll
    for (int J = 0; J < 9; J++) dU[J] = frozen ? 0.0 : A.dU[J * A.N + b];
    // six-component plans: the coordinates of the (symmetric) increment in the
    // dual basis of E6, (dU11, dU22, dU33, dU12, dU23, dU13)
    const double d6[6] = {dU[0], dU[4], dU[8], 0.5 * (dU[1] + dU[3]), 0.5 * (dU[5] + dU[7]),
                          0.5 * (dU[2] + dU[6])};
#pragma unroll
    for (int kk = 0; kk < kModesPerThread; kk++) {
        const int k = kg * kModesPerThread + kk;
        if (k < A.m) {
            double s = 0.0;
            if (!frozen) {
                s = A.y[(int64_t)k * A.count + pl];
                if (A.nmac == 6) {
#pragma unroll
                    for (int J = 0; J < 6; J++) s = fma(A.X[((int64_t)k * 6 + J) * A.count + pl], d6[J], s);
                } else {
#pragma unroll
                    for (int J = 0; J < 9; J++) s = fma(A.X[((int64_t)k * 9 + J) * A.count + pl], dU[J], s);
                }
            }
            A.dt[(int64_t)k * A.count + pl] = s;
        }
    }
}

void launch_update(const UpdateArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)((a.m + kModesPerThread - 1) / kModesPerThread) * a.count;
    hipLaunchKernelGGL(k_update, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------- backward
// pull-back of the macro cotangent: Lam = Linv(sym(F^T g)), g_r = 2 Lam
__global__ void __launch_bounds__(256) k_bw_pullback(BwPointArgs A) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.N) return;
    const int64_t N = A.N;
    double g[9];
#pragma unroll
    for (int k = 0; k < 9; k++) g[k] = A.g[k * N + b];
    if (!A.objective) {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            A.gr[k * N + b] = g[k];
            A.Lam[k * N + b] = 0.5 * g[k];
        }
        return;
    }
    double F[9], V[9], u[3], Ftg[9], H[9], Lam[9];
    load_polar(A.polar, N, b, F, V, u);
    tmul3(F, g, Ftg);
    sym3(Ftg, H);
    lyap_solve(V, u, H, Lam);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        A.Lam[k * N + b] = Lam[k];
        A.gr[k * N + b] = 2.0 * Lam[k];
    }
}

void launch_bw_pullback(const BwPointArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_bw_pullback, dim3(nblocks(a.N, 256)), dim3(256), 0, s, a);
}

// dL/dFbar = g S + 2 F Linv(sym(h_r) - Lam S - S Lam)
__global__ void __launch_bounds__(256) k_bw_pushforward(BwPointArgs A) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.N) return;
    const int64_t N = A.N;
    double h[9];
#pragma unroll
    for (int k = 0; k < 9; k++) h[k] = A.hr[k * N + b];
    if (!A.objective) {
#pragma unroll
        for (int k = 0; k < 9; k++) A.gF[k * N + b] = h[k];
        return;
    }
    double F[9], V[9], u[3], S[9], Lam[9], g[9], M[9], t1[9], t2[9], Z[9], FZ[9], gS[9];
    load_polar(A.polar, N, b, F, V, u);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        S[k] = A.S[k * N + b];
        Lam[k] = A.Lam[k * N + b];
        g[k] = A.g[k * N + b];
    }
    mul3(Lam, S, t1);
    mul3(S, Lam, t2);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            M[3 * i + j] = 0.5 * (h[3 * i + j] + h[3 * j + i]) - t1[3 * i + j] - t2[3 * i + j];
    lyap_solve(V, u, M, Z);
    mul3(F, Z, FZ);
    mul3(g, S, gS);
#pragma unroll
    for (int k = 0; k < 9; k++) A.gF[k * N + b] = gS[k] + 2.0 * FZ[k];
}

void launch_bw_pushforward(const BwPointArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_bw_pushforward, dim3(nblocks(a.N, 256)), dim3(256), 0, s, a);
}

// adjoint solve with the stored factor: lambda = Kaa^{-T} KaF g_r = X g_r, one
// thread per (group of kModesPerThread modes, point)
__global__ void __launch_bounds__(256) k_lambda(LambdaArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ng = (A.m + kModesPerThread - 1) / kModesPerThread;
    if (t >= (int64_t)ng * A.count) return;
    const int kg = (int)(t / A.count);
    const int64_t pl = t - (int64_t)kg * A.count;
    const int64_t b = A.first + pl;
    if (kg == 0 && A.conv) A.conv[pl] = 0;
    double gr[9];
#pragma unroll
    for (int J = 0; J < 9; J++) gr[J] = A.gr[J * A.N + b];
    const double g6[6] = {gr[0], gr[4], gr[8], 0.5 * (gr[1] + gr[3]), 0.5 * (gr[5] + gr[7]),
                          0.5 * (gr[2] + gr[6])};
#pragma unroll
    for (int kk = 0; kk < kModesPerThread; kk++) {
        const int k = kg * kModesPerThread + kk;
        if (k < A.m) {
            double s = 0.0;
            if (A.nmac == 6) {
#pragma unroll
                for (int J = 0; J < 6; J++) s = fma(A.X[((int64_t)k * 6 + J) * A.count + pl], g6[J], s);
            } else {
#pragma unroll
                for (int J = 0; J < 9; J++) s = fma(A.X[((int64_t)k * 9 + J) * A.count + pl], gr[J], s);
            }
            A.lam[(int64_t)k * A.count + pl] = s;
        }
    }
}

void launch_lambda(const LambdaArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)((a.m + kModesPerThread - 1) / kModesPerThread) * a.count;
    hipLaunchKernelGGL(k_lambda, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------- reductions
// dL/dtheta: fixed-order sum over points (bitwise reproducible).  Stage 1:
// block (j, c) takes the contiguous chunk j of component c, thread t sums its
// points t, t + 256, ... of the chunk in order, then a fixed tree; stage 2:
// one block per component adds the kThetaChunks partials by the same tree.
__device__ __forceinline__ double block_tree_sum(double v, double* s) {
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    return s[0];
}

__global__ void __launch_bounds__(256) k_reduce_theta_chunks(int64_t N, const double* gth, double* part) {
    __shared__ double s[256];
    const int j = blockIdx.x, c = blockIdx.y, t = threadIdx.x;
    const int64_t ch = (N + kThetaChunks - 1) / kThetaChunks;
    const int64_t b0 = (int64_t)j * ch, b1 = b0 + ch < N ? b0 + ch : N;
    double acc = 0.0;
    for (int64_t b = b0 + t; b < b1; b += 256) acc += gth[c * N + b];
    const double tot = block_tree_sum(acc, s);
    if (t == 0) part[c * kThetaChunks + j] = tot;
}

__global__ void __launch_bounds__(256) k_reduce_theta(const double* part, double* out) {
    __shared__ double s[256];
    const int c = blockIdx.x;
    const double tot = block_tree_sum(part[c * kThetaChunks + threadIdx.x], s);
    if (threadIdx.x == 0) out[c] = tot;
}

void launch_reduce_theta(int64_t N, const double* gth, double* part, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_theta_chunks, dim3(kThetaChunks, 4), dim3(256), 0, s, N, gth, part);
    hipLaunchKernelGGL(k_reduce_theta, dim3(4), dim3(256), 0, s, (const double*)part, out);
}

__global__ void __launch_bounds__(256) k_history_export(const double* src, int Q, int Qpad,
                                                        int64_t count, double* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count * Q * 7) return;
    const int k = (int)(t % 7);
    const int64_t pq = t / 7;
    const int q = (int)(pq % Q);
    const int64_t b = pq / Q;
    out[t] = src[(b * Qpad + q) * 8 + k];
}

void launch_history_export(const double* src, int Q, int Qpad, int64_t count, double* out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_history_export, dim3(nblocks(count * Q * 7, 256)), dim3(256), 0, s, src,
                       Q, Qpad, count, out);
}

__global__ void __launch_bounds__(256) k_mark_unconverged(int64_t N, const double* rnorm, double tol, int* status) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N) return;
    if (!(rnorm[b] < tol)) status[b] |= HROM_PT_NOCONV;
}

void launch_mark_unconverged(int64_t N, const double* rnorm, double tol, int* status,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_mark_unconverged, dim3(nblocks(N, 256)), dim3(256), 0, s, N, rnorm, tol,
                       status);
}

// ---------------------------------------------------------------- plan-time layouts
__device__ __forceinline__ uint16_t to_bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16_bits(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}
__device__ __forceinline__ uint16_t to_f16_bits(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float from_f16_bits(uint16_t h) {
    return (float)__builtin_bit_cast(_Float16, h);
}

// One thread per (q, row J, column n) of the augmented mode matrix
// Ghat_q = [G_q | I_9 | 0] (9 x MP).
__global__ void __launch_bounds__(256) k_build_ghat(LayoutArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)A.Qpad * 9 * A.MP;
    if (t >= tot) return;
    const int n = (int)(t % A.MP);
    const int J = (int)((t / A.MP) % 9);
    const int q = (int)(t / (9 * (int64_t)A.MP));
    double v = 0.0;
    if (q < A.Q) {
        if (n < A.m) v = A.G[((int64_t)q * 9 + J) * A.m + n];
        else if (n < A.m + 9) v = (n - A.m == J) ? 1.0 : 0.0;
    }
    A.Ghat[t] = v;
    if (n < A.m) {
        // GT[(q/64)][J][n][q%64]
        A.GT[(((int64_t)(q >> 6) * 9 + J) * A.m + n) * 64 + (q & 63)] = (q < A.Q) ? v : 0.0;
    }
    if (J == 0 && n == 0) A.phpad[q] = (q < A.Q) ? A.phase[q] : 0;
}

// Packed MFMA fragments of the mode gradients for the mixed tangent: ECM point
// q, mode tile t, lane (g, c) holds 8 low-precision values for mode column
// n = 16 t + c, one per k-slot of a 16x16x32 MFMA.  The nine tensor
// components are spread over the four lane groups as (0,1), (2,3), (4,5),
// (6,7,8); with a, b (and d = 8 in group 3) the group's components the slots
// are
//   groups 0..2: Gh[a] Gh[b] Gl[a] Gl[b] Gh[a] Gh[b] (group 1: Gh[8]) 0
//   group 3:     Gh[a] Gh[b] Gl[a] Gl[b] Gh[a] Gh[b] Gh[8] Gl[8]
// (hi part Gh and rounded remainder Gl; Gl = 0 without the split).  Paired
// with the matching W or T slots, one MFMA forms all three split products
// hi*hi + lo*hi + hi*lo of the nine-component contraction.
__global__ void __launch_bounds__(256) k_build_frags(LayoutArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int MA = (A.m + 15) / 16;
    const int64_t tot = (int64_t)A.Qpad * MA * 64 * 8;
    if (t >= tot) return;
    const int s = (int)(t & 7);
    const int lane = (int)((t >> 3) & 63);
    const int tile = (int)((t >> 9) % MA);
    const int q = (int)((t >> 9) / MA);
    const int g = lane >> 4, c = lane & 15;
    const int n = 16 * tile + c;
    const int a = (g < 3) ? 2 * g : 6, b = a + 1;
    int comp = -1, lo = 0;
    switch (s) {
        case 0: case 4: comp = a; break;
        case 1: case 5: comp = b; break;
        case 2: comp = a; lo = 1; break;
        case 3: comp = b; lo = 1; break;
        case 6: comp = (g == 1 || g == 3) ? 8 : -1; break;
        default: comp = (g == 3) ? 8 : -1; lo = 1; break;
    }
    double v = 0.0;
    if (comp >= 0 && q < A.Q && n < A.m) v = A.G[((int64_t)q * 9 + comp) * A.m + n];
    uint16_t bits;
    if (A.prec == HROM_MIXED_BF16) {
        const uint16_t hi = to_bf16_bits((float)v);
        bits = lo ? (A.split ? to_bf16_bits((float)(v - (double)from_bf16_bits(hi))) : 0) : hi;
    } else {
        const uint16_t hi = to_f16_bits((float)v);
        bits = lo ? (A.split ? to_f16_bits((float)(v - (double)from_f16_bits(hi))) : 0) : hi;
    }
    A.Fpk[t] = bits;
}

// A-operand fragments of the kinematics GEMM (FP64 16x16x4 MFMA): row tile
// rt, k-step s, lane (g, c) holds G[q][I][k] with 9 q + I = 16 rt + c and
// k = 4 s + g (zero beyond m and beyond Q).
__global__ void __launch_bounds__(256) k_build_gf(LayoutArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntile = (int64_t)A.Qpad * 9 / 16;
    if (t >= ntile * A.KS * 64) return;
    const int lane = (int)(t & 63);
    const int s = (int)((t >> 6) % A.KS);
    const int64_t rt = (t >> 6) / A.KS;
    const int64_t row = rt * 16 + (lane & 15);
    const int q = (int)(row / 9), I = (int)(row % 9);
    const int k = 4 * s + (lane >> 4);
    A.Gf[t] = (q < A.Q && k < A.m) ? A.G[((int64_t)q * 9 + I) * A.m + k] : 0.0;
}

// A-operand fragments of the mixed adjoint GEMM (BF16 16x16x32 MFMA, FP32
// accumulation): row tile rt, half h (modes 32 h ..), level L of the
// three-level BF16 split, lane (g, c), dword d holds the levels L of
// G[q][I][k] and G[q][I][k + 1] (low half first) with 9 q + I = 16 rt + c and
// k = 32 h + 8 g + 2 d (zero beyond m and beyond Q).
__global__ void __launch_bounds__(256) k_build_gb3(LayoutArgs A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int NH = gb3_halves(A.m);
    const int64_t ntile = (int64_t)A.Qpad * 9 / 16;
    if (t >= ntile * NH * 3 * 256) return;
    const int d = (int)(t & 3), lane = (int)((t >> 2) & 63);
    const int L = (int)((t >> 8) % 3);
    const int h = (int)((t >> 8) / 3 % NH);
    const int64_t rt = (t >> 8) / 3 / NH;
    const int64_t row = rt * 16 + (lane & 15);
    const int q = (int)(row / 9), I = (int)(row % 9);
    uint32_t word = 0;
#pragma unroll
    for (int ii = 0; ii < 2; ii++) {
        const int k = 32 * h + 8 * (lane >> 4) + 2 * d + ii;
        const double v = (q < A.Q && k < A.m) ? A.G[((int64_t)q * 9 + I) * A.m + k] : 0.0;
        uint16_t lv[3];
        bf16_split3(v, lv);
        word |= (uint32_t)lv[L] << (16 * ii);
    }
    A.Gb3[t] = word;
}

// Weights of the volume averages (Sec. 2 and 3.3): w_q / V0 with V0 = sum_q
// w_q (summed in order), so that the ECM sums are averages over the RVE
// whatever measure the caller's weights add up to.
__global__ void __launch_bounds__(256) k_normalize_w(const double* w, int Q, int Qpad, double* wpad) {
    __shared__ double V0;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < Q; q++) s += w[q];
        V0 = s;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < Qpad; q += blockDim.x) wpad[q] = (q < Q) ? w[q] / V0 : 0.0;
}

void launch_build_layouts(const LayoutArgs& a, hipStream_t s) {
    const int64_t n1 = (int64_t)a.Qpad * 9 * a.MP;
    hipLaunchKernelGGL(k_build_ghat, dim3(nblocks(n1, 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_normalize_w, dim3(1), dim3(256), 0, s, a.w, a.Q, a.Qpad, a.wpad);
    const int64_t n3 = (int64_t)a.Qpad * 9 / 16 * a.KS * 64;
    hipLaunchKernelGGL(k_build_gf, dim3(nblocks(n3, 256)), dim3(256), 0, s, a);
    if (a.prec != HROM_FP64) {
        const int64_t n2 = (int64_t)a.Qpad * ((a.m + 15) / 16) * 512;
        hipLaunchKernelGGL(k_build_frags, dim3(nblocks(n2, 256)), dim3(256), 0, s, a);
        const int64_t n4 = (int64_t)a.Qpad * 9 / 16 * gb3_halves(a.m) * 3 * 256;
        hipLaunchKernelGGL(k_build_gb3, dim3(nblocks(n4, 256)), dim3(256), 0, s, a);
    }
}

}  // namespace hrom
