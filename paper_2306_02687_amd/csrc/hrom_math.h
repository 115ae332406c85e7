// Small per-point tensor algebra for the gfx950 kernels (double precision).
// 3x3 tensors are row-major arrays, index 3 i + j.
#pragma once

#include <hip/hip_runtime.h>

namespace hrom {

__device__ __forceinline__ double det3(const double* A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// B = A^{-1} from the cofactors; returns det A
__device__ __forceinline__ double inv3(const double* A, double* B) {
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

__device__ __forceinline__ void mul3(const double* A, const double* B, double* C) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// C = A^T B
__device__ __forceinline__ void tmul3(const double* A, const double* B, double* C) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            C[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}

__device__ __forceinline__ void sym3(const double* A, double* S) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) S[3 * i + j] = 0.5 * (A[3 * i + j] + A[3 * j + i]);
}

// Eigen-decomposition of a symmetric 3x3 matrix S = V diag(e) V^T by cyclic
// Jacobi rotations applied in place (rows/columns p, q of the working copy).
__device__ inline void eigsym3(const double* S, double* V, double* e) {
    double a00 = S[0], a11 = S[4], a22 = S[8];
    double a01 = 0.5 * (S[1] + S[3]), a02 = 0.5 * (S[2] + S[6]), a12 = 0.5 * (S[5] + S[7]);
#pragma unroll
    for (int i = 0; i < 9; i++) V[i] = (i == 0 || i == 4 || i == 8) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 32; sweep++) {
        const double off = a01 * a01 + a02 * a02 + a12 * a12;
        const double dia = a00 * a00 + a11 * a11 + a22 * a22;
        if (off == 0.0 || off <= 1e-34 * dia) break;
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const int p = (r == 2) ? 1 : 0;
            const int q = (r == 0) ? 1 : 2;
            double& apq = (r == 0) ? a01 : (r == 1 ? a02 : a12);
            if (apq == 0.0) continue;
            double& app = (p == 0) ? a00 : a11;
            double& aqq = (q == 1) ? a11 : a22;
            const double th = (aqq - app) / (2.0 * apq);
            const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0);
            const double s = t * c;
            // couplings a_kp, a_kq of the remaining index k = 3 - p - q
            double* pkp;
            double* pkq;
            if (r == 0) { pkp = &a02; pkq = &a12; }        // (p,q) = (0,1), k = 2
            else if (r == 1) { pkp = &a01; pkq = &a12; }   // (p,q) = (0,2), k = 1
            else { pkp = &a01; pkq = &a02; }               // (p,q) = (1,2), k = 0
            const double kp = *pkp, kq = *pkq;
            *pkp = c * kp - s * kq;
            *pkq = s * kp + c * kq;
            app -= t * apq;
            aqq += t * apq;
            apq = 0.0;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const double vp = V[3 * i + p], vq = V[3 * i + q];
                V[3 * i + p] = c * vp - s * vq;
                V[3 * i + q] = s * vp + c * vq;
            }
        }
    }
    e[0] = a00;
    e[1] = a11;
    e[2] = a22;
}

// Z solving U Z + Z U = B for symmetric B, with U = V diag(u) V^T:
// (V^T Z V)_ij = (V^T B V)_ij / (u_i + u_j).
__device__ inline void lyap_solve(const double* V, const double* u, const double* B, double* Z) {
    double T[9], M[9];
    tmul3(V, B, T);   // V^T B
    mul3(T, V, M);    // V^T B V
    const double h00 = 0.5 / u[0], h11 = 0.5 / u[1], h22 = 0.5 / u[2];
    const double h01 = 1.0 / (u[0] + u[1]), h02 = 1.0 / (u[0] + u[2]), h12 = 1.0 / (u[1] + u[2]);
    M[0] *= h00; M[4] *= h11; M[8] *= h22;
    M[1] *= h01; M[3] *= h01;
    M[2] *= h02; M[6] *= h02;
    M[5] *= h12; M[7] *= h12;
    // Z = V M V^T
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            T[3 * i + j] = V[3 * i] * M[j] + V[3 * i + 1] * M[3 + j] + V[3 * i + 2] * M[6 + j];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            Z[3 * i + j] = T[3 * i] * V[3 * j] + T[3 * i + 1] * V[3 * j + 1] + T[3 * i + 2] * V[3 * j + 2];
}

}  // namespace hrom
