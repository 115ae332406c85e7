/*
 * hrom_oracle.c -- plain FP64 CPU oracle of the hyper-reduced RVE evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU path: it is written from the paper (Lange, Huetter, Kiefer,
 * "A monolithic hyper ROM FE2 method with clustered training at finite
 * deformations", arXiv 2306.02687) and the compressible Neo-Hooke law, as
 * plain loops in double precision, one macro point at a time (OpenMP only
 * distributes independent macro points over threads).
 *
 * Notation (paper -> here): ROM amplitudes u~ -> a (m of them), hyper
 * integration points / weights (z~, w~) -> the Q ECM points with weights w,
 * element ROM modes -> mode gradients G[q][I][m] (3x3 tensors flattened
 * row-major, I = 3 i + j), macro stretch U -> Ubar, reduced residual r~ -> r,
 * reduced stiffness k~ -> Kaa, dr~/dU -> KaF, dSigma/du~ -> KFa = KaF^T,
 * dSigma/dU -> KFF.  Tangent convention: A[I][J] = dP_I / dF_J.
 *
 * Step map (each function cites the passage it follows):
 *   polar split of Fbar ............ Sec. 3.2.2, eq. (ploar_decomp); the
 *                                    eigen route of the appendix
 *   reduced kinematics ............. Sec. 3.2.1, eq. (ROM_assumption)
 *   Neo-Hooke P, A at ECM points ... material law of the workload
 *   ECM sums r, Kaa, KaF, KFF, P ... Sec. 3.2.1 eqs. (ROMintforce),
 *                                    (ROMstiffness), Sec. 3.3 (ECM sums over
 *                                    the reference domain, constant weights)
 *   Cholesky / LU of Kaa ........... Sec. 4 (factorise, never invert)
 *   condensation ................... Sec. 3.2.3 (algorithmic stress,
 *                                    eq. Biot_Tangent)
 *   monolithic update .............. Sec. 3.2.3 (increment of u~)
 *   push-out to the macro frame .... Sec. 3.2.2 eqs. (workconjugacy),
 *                                    (biotstress) in second-Piola form
 *   adjoint backward ............... derivative of the converged map
 *   Cauchy stress and tangent ...... Sec. 3.2.2 eq. (biotstress), App. A
 *                                    eqs. (tangent_continuum),
 *                                    (d_Cauchy_d_Biot), (dUdot_dd)
 *   J2 plasticity at ECM points .... Sec. 5 Example 1 (elastic-plastic
 *                                    matrix with initial yield stress and
 *                                    linear hardening, elastic inclusions);
 *                                    state only at the hyper integration
 *                                    points (Sec. 4)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PT_JNONPOS 1
#define ORC_PT_NOT_SPD 2
#define ORC_PT_NOCONV 4
#define ORC_PT_NONFINITE 8

/* ------------------------------------------------------------------ */
/* 3x3 helpers (row-major, A[3*i+j])                                   */
/* ------------------------------------------------------------------ */
static void m3_mul(const double *A, const double *B, double *C) /* C = A B */
{
    double T[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}

static void m3_tmul(const double *A, const double *B, double *C) /* C = A^T B */
{
    double T[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[3 * k + i] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}

static void m3_transpose(const double *A, double *B)
{
    double T[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) T[3 * i + j] = A[3 * j + i];
    memcpy(B, T, sizeof T);
}

static void m3_sym(const double *A, double *S) /* S = (A + A^T) / 2 */
{
    double T[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) T[3 * i + j] = 0.5 * (A[3 * i + j] + A[3 * j + i]);
    memcpy(S, T, sizeof T);
}

static double m3_det(const double *A)
{
    return A[0] * (A[4] * A[8] - A[5] * A[7])
         - A[1] * (A[3] * A[8] - A[5] * A[6])
         + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse by the adjugate */
static void m3_inv(const double *A, double *B)
{
    double d = m3_det(A);
    double T[9];
    T[0] = (A[4] * A[8] - A[5] * A[7]) / d;
    T[1] = (A[2] * A[7] - A[1] * A[8]) / d;
    T[2] = (A[1] * A[5] - A[2] * A[4]) / d;
    T[3] = (A[5] * A[6] - A[3] * A[8]) / d;
    T[4] = (A[0] * A[8] - A[2] * A[6]) / d;
    T[5] = (A[2] * A[3] - A[0] * A[5]) / d;
    T[6] = (A[3] * A[7] - A[4] * A[6]) / d;
    T[7] = (A[1] * A[6] - A[0] * A[7]) / d;
    T[8] = (A[0] * A[4] - A[1] * A[3]) / d;
    memcpy(B, T, sizeof T);
}

/*
 * Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations:
 * S = V diag(lam) V^T, columns of V are eigenvectors.
 */
static void sym3_eig(const double *S, double *V, double *lam)
{
    double A[9];
    memcpy(A, S, sizeof A);
    for (int i = 0; i < 9; i++) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    static const int PQ[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int sweep = 0; sweep < 64; sweep++) {
        double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-34 * dia || off == 0.0) break;
        for (int r = 0; r < 3; r++) {
            int p = PQ[r][0], q = PQ[r][1];
            double apq = A[3 * p + q];
            if (apq == 0.0) continue;
            /* rotation J (identity except the (p,q) plane) with A' = J^T A J
               and A'_pq = 0: tan(phi) = t solves t^2 + 2 theta t - 1 = 0 */
            double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
            double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            double J[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
            J[3 * p + p] = c;
            J[3 * q + q] = c;
            J[3 * p + q] = s;
            J[3 * q + p] = -s;
            double T[9];
            m3_tmul(J, A, T);
            m3_mul(T, J, A);
            A[3 * p + q] = A[3 * q + p] = 0.0;
            m3_mul(V, J, V);
        }
    }
    lam[0] = A[0];
    lam[1] = A[4];
    lam[2] = A[8];
}

/* ------------------------------------------------------------------ */
/* Polar split  Fbar = Rbar Ubar  (Sec. 3.2.2, eq. ploar_decomp), by   */
/* the eigen route of the appendix: C = Fbar^T Fbar = V diag(c) V^T,   */
/* Ubar = V diag(sqrt c) V^T, Rbar = Fbar Ubar^{-1}.                   */
/* ------------------------------------------------------------------ */
typedef struct {
    double F[9];  /* macro deformation gradient */
    double U[9];  /* right stretch */
    double R[9];  /* rotation */
    double V[9];  /* eigenvectors of U (columns) */
    double u[3];  /* principal stretches */
} polar_t;

static void polar_split(const double *F, polar_t *P)
{
    double C[9], c[3];
    memcpy(P->F, F, 9 * sizeof(double));
    m3_tmul(F, F, C);
    sym3_eig(C, P->V, c);
    double Ui[9];
    for (int i = 0; i < 3; i++) P->u[i] = sqrt(c[i]);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0, si = 0.0;
            for (int k = 0; k < 3; k++) {
                s += P->V[3 * i + k] * P->u[k] * P->V[3 * j + k];
                si += P->V[3 * i + k] / P->u[k] * P->V[3 * j + k];
            }
            P->U[3 * i + j] = s;
            Ui[3 * i + j] = si;
        }
    m3_mul(F, Ui, P->R);
}

/* Linv(B): the symmetric Z with Ubar Z + Z Ubar = B, for symmetric B,
   solved in the eigenbasis of Ubar: (V^T Z V)_ij = (V^T B V)_ij / (u_i + u_j). */
static void lyap_inv(const polar_t *P, const double *B, double *Z)
{
    double T[9], Bt[9];
    m3_tmul(P->V, B, T);
    m3_mul(T, P->V, Bt);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) Bt[3 * i + j] /= (P->u[i] + P->u[j]);
    m3_mul(P->V, Bt, T);
    double Vt[9];
    m3_transpose(P->V, Vt);
    m3_mul(T, Vt, Z);
}

/* linearised stretch increment dU = Linv(dF^T F + F^T dF) */
static void stretch_increment(const polar_t *P, const double *dF, double *dU)
{
    double a[9], b[9], dC[9];
    m3_tmul(dF, P->F, a);
    m3_tmul(P->F, dF, b);
    for (int i = 0; i < 9; i++) dC[i] = a[i] + b[i];
    lyap_inv(P, dC, dU);
}

/* ------------------------------------------------------------------ */
/* Compressible Neo-Hooke:  W = mu/2 (I1 - 3) - mu ln J + lam/2 (ln J)^2 */
/*   P_ij    = mu (F_ij - Finv_ji) + lam lnJ Finv_ji                    */
/*   A_ijkl  = mu d_ik d_jl + (mu - lam lnJ) Finv_li Finv_jk            */
/*             + lam Finv_ji Finv_lk                                    */
/* ------------------------------------------------------------------ */
static int neo_hooke(const double *F, double mu, double lam, double *P, double *A,
                     double *Jout, double *ell_out, double *Finv_out)
{
    double J = m3_det(F);
    if (Jout) *Jout = J;
    if (!(J > 0.0)) return -1;
    double Fi[9];
    m3_inv(F, Fi);
    double ell = log(J);
    if (ell_out) *ell_out = ell;
    if (Finv_out) memcpy(Finv_out, Fi, sizeof Fi);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            P[3 * i + j] = mu * (F[3 * i + j] - Fi[3 * j + i]) + lam * ell * Fi[3 * j + i];
    if (A) {
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                for (int k = 0; k < 3; k++)
                    for (int l = 0; l < 3; l++) {
                        double v = (mu - lam * ell) * Fi[3 * l + i] * Fi[3 * j + k]
                                 + lam * Fi[3 * j + i] * Fi[3 * l + k];
                        if (i == k && j == l) v += mu;
                        A[9 * (3 * i + j) + (3 * k + l)] = v;
                    }
    }
    return 0;
}

static int all_finite(const double *x, int n)
{
    for (int i = 0; i < n; i++)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Evaluate the hyper-reduced RVE at one macro point, in the RVE frame  */
/* (Sec. 3.2.1 eqs. ROM_assumption, ROMintforce, ROMstiffness; Sec. 3.3 */
/* ECM sums with constant weights on the reference domain).             */
/*   F_q  = Fr + sum_m a_m G_qm                                         */
/*   r    = sum_q w_q G_q^T P_q          Pr  = sum_q w_q P_q             */
/*   Kaa  = sum_q G_q^T (w_q A_q) G_q    KaF = sum_q w_q G_q^T A_q       */
/*   KFF  = sum_q w_q A_q                                               */
/* The weights sum to the RVE measure V0; every ECM sum is divided by  */
/* V0 (the volume averages of Sec. 2 and 3.3), i.e. the weights enter  */
/* as w_q / V0.  The workloads have V0 = 1.                             */
/* ------------------------------------------------------------------ */
typedef struct {
    int m, Q;
    const double *G;   /* [Q][9][m] */
    const double *w;   /* [Q] */
    const int *phase;  /* [Q] */
    double theta[4];   /* mu0, lam0, mu1, lam1 */
    double V0;         /* sum of the weights, in order */
    int j2;            /* material: 0 Neo-Hooke (theta), 1 J2 plasticity (mat) */
    double mat[8];     /* J2: per phase (mu, lam, sigma_y0, H) */
} rve_t;

/* ------------------------------------------------------------------ */
/* Small-strain J2 (von Mises) plasticity with linear isotropic         */
/* hardening, the material of the paper's Example 1 (Sec. 5): an        */
/* elastic-plastic matrix with initial yield stress sigma_y0 and        */
/* hardening modulus H, elastic inclusions (sigma_y0 beyond reach).      */
/* Strain eps = sym(F) - I; state per ECM point h = (eps_p[6], alpha)   */
/* with eps_p ordered xx, yy, zz, xy, yz, xz and alpha the equivalent   */
/* plastic strain.  Radial return (a textbook algorithm, restated):     */
/*   s_tr = 2 mu (dev eps - eps_p_n),  f = |s_tr| - sqrt(2/3) (sy0 +     */
/*   H alpha_n);  f <= 0: elastic;  else dgam = f / (2 mu + 2 H / 3),    */
/*   n = s_tr / |s_tr|, s = s_tr - 2 mu dgam n, eps_p += dgam n,        */
/*   alpha += sqrt(2/3) dgam.  sigma = kappa tr(eps) I + s, kappa =      */
/*   lam + 2 mu / 3.  Consistent tangent dsigma/deps:                   */
/*   kappa 1x1 + 2 mu th (I_sym - 1x1 / 3) - 2 mu thb n x n,            */
/*   th = 1 - 2 mu dgam / |s_tr|, thb = 1 / (1 + H / (3 mu)) - (1 - th). */
/* As a function of F: P = sigma (symmetric), A[9I+J] = dsigma_I/dF_J.   */
/* ------------------------------------------------------------------ */
static const int kVoigt[9] = {0, 3, 5, 3, 1, 4, 5, 4, 2};   /* (i, j) -> eps_p slot */

static void j2_law(const double *F, const double *mp, const double *hn, double *P, double *A,
                   double *ht)
{
    const double mu = mp[0], lam = mp[1], sy0 = mp[2], H = mp[3];
    const double kappa = lam + 2.0 * mu / 3.0;
    double eps[9], ep[9], s_tr[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            eps[3 * i + j] = 0.5 * (F[3 * i + j] + F[3 * j + i]) - (i == j ? 1.0 : 0.0);
            ep[3 * i + j] = hn[kVoigt[3 * i + j]];
        }
    const double tr = eps[0] + eps[4] + eps[8];
    double nrm2 = 0.0;
    for (int I = 0; I < 9; I++) {
        const double dev = eps[I] - ((I % 4 == 0) ? tr / 3.0 : 0.0);
        s_tr[I] = 2.0 * mu * (dev - ep[I]);
        nrm2 += s_tr[I] * s_tr[I];
    }
    const double nrm = sqrt(nrm2);
    const double f = nrm - sqrt(2.0 / 3.0) * (sy0 + H * hn[6]);
    double dgam = 0.0, th = 1.0, thb = 0.0, n[9] = {0};
    if (f > 0.0) {
        dgam = f / (2.0 * mu + 2.0 * H / 3.0);
        for (int I = 0; I < 9; I++) n[I] = s_tr[I] / nrm;
        th = 1.0 - 2.0 * mu * dgam / nrm;
        thb = 1.0 / (1.0 + H / (3.0 * mu)) - (1.0 - th);
    }
    for (int I = 0; I < 9; I++)
        P[I] = ((I % 4 == 0) ? kappa * tr : 0.0) + s_tr[I] - 2.0 * mu * dgam * n[I];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++) {
                    const double d_ij = (i == j), d_kl = (k == l);
                    const double isym = 0.5 * ((i == k) * (j == l) + (i == l) * (j == k));
                    A[9 * (3 * i + j) + 3 * k + l] = kappa * d_ij * d_kl
                        + 2.0 * mu * th * (isym - d_ij * d_kl / 3.0)
                        - 2.0 * mu * thb * n[3 * i + j] * n[3 * k + l];
                }
    if (ht) {
        for (int v = 0; v < 6; v++) ht[v] = hn[v];
        for (int i = 0; i < 3; i++)
            for (int j = i; j < 3; j++) ht[kVoigt[3 * i + j]] = hn[kVoigt[3 * i + j]] + dgam * n[3 * i + j];
        ht[6] = hn[6] + sqrt(2.0 / 3.0) * dgam;
    }
}

static int eval_point(const rve_t *c, const double *Fr, const double *a,
                      double *r, double *Pr, double *Kaa, double *KaF, double *KFF,
                      const double *hn, double *ht)
{
    const int m = c->m, Q = c->Q;
    int status = 0;
    memset(r, 0, sizeof(double) * m);
    memset(Pr, 0, sizeof(double) * 9);
    memset(Kaa, 0, sizeof(double) * m * m);
    memset(KaF, 0, sizeof(double) * m * 9);
    memset(KFF, 0, sizeof(double) * 81);
    double *T = (double *)malloc(sizeof(double) * 9 * m);
    for (int q = 0; q < Q; q++) {
        const double *Gq = c->G + (size_t)q * 9 * m;
        const double wq = c->w[q] / c->V0;
        const double mu = c->theta[2 * c->phase[q]], lam = c->theta[2 * c->phase[q] + 1];
        double F[9], P[9], A[81], J;
        for (int I = 0; I < 9; I++) {
            double s = Fr[I];
            for (int k = 0; k < m; k++) s += a[k] * Gq[I * m + k];
            F[I] = s;
        }
        if (c->j2) {
            j2_law(F, c->mat + 4 * c->phase[q], hn + 7 * (size_t)q, P, A, ht ? ht + 7 * (size_t)q : NULL);
        } else if (neo_hooke(F, mu, lam, P, A, &J, NULL, NULL) != 0) {
            status |= ORC_PT_JNONPOS;
            continue;
        }
        for (int I = 0; I < 9; I++) Pr[I] += wq * P[I];
        for (int k = 0; k < m; k++) {
            double s = 0.0;
            for (int I = 0; I < 9; I++) s += Gq[I * m + k] * P[I];
            r[k] += wq * s;
        }
        for (int I = 0; I < 81; I++) KFF[I] += wq * A[I];
        /* T = (w_q A_q) G_q, then Kaa += G_q^T T and KaF += G_q^T (w_q A_q) */
        for (int I = 0; I < 9; I++)
            for (int k = 0; k < m; k++) {
                double s = 0.0;
                for (int J2 = 0; J2 < 9; J2++) s += A[9 * I + J2] * Gq[J2 * m + k];
                T[I * m + k] = wq * s;
            }
        for (int k = 0; k < m; k++) {
            for (int n = 0; n < m; n++) {
                double s = 0.0;
                for (int I = 0; I < 9; I++) s += Gq[I * m + k] * T[I * m + n];
                Kaa[k * m + n] += s;
            }
            for (int J2 = 0; J2 < 9; J2++) {
                double s = 0.0;
                for (int I = 0; I < 9; I++) s += Gq[I * m + k] * A[9 * I + J2];
                KaF[k * 9 + J2] += wq * s;
            }
        }
    }
    free(T);
    return status;
}

/* ------------------------------------------------------------------ */
/* Dense factorisations (Sec. 4: LU / Cholesky with right-hand sides,   */
/* never an explicit inverse).                                          */
/* ------------------------------------------------------------------ */
/* Cholesky K = L L^T in place (lower triangle of L); returns -1 on a   */
/* non-positive pivot.                                                  */
static int cholesky(int m, double *L)
{
    for (int j = 0; j < m; j++) {
        double d = L[j * m + j];
        for (int k = 0; k < j; k++) d -= L[j * m + k] * L[j * m + k];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        L[j * m + j] = d;
        for (int i = j + 1; i < m; i++) {
            double s = L[i * m + j];
            for (int k = 0; k < j; k++) s -= L[i * m + k] * L[j * m + k];
            L[i * m + j] = s / d;
        }
    }
    return 0;
}

static void chol_solve(int m, const double *L, double *x) /* L L^T x = b */
{
    for (int i = 0; i < m; i++) {
        double s = x[i];
        for (int k = 0; k < i; k++) s -= L[i * m + k] * x[k];
        x[i] = s / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; i--) {
        double s = x[i];
        for (int k = i + 1; k < m; k++) s -= L[k * m + i] * x[k];
        x[i] = s / L[i * m + i];
    }
}

/* LU with partial pivoting in place; piv[i] = row swapped into i */
static int lu_factor(int m, double *A, int *piv)
{
    for (int j = 0; j < m; j++) {
        int p = j;
        for (int i = j + 1; i < m; i++)
            if (fabs(A[i * m + j]) > fabs(A[p * m + j])) p = i;
        piv[j] = p;
        if (A[p * m + j] == 0.0) return -1;
        if (p != j)
            for (int k = 0; k < m; k++) {
                double t = A[j * m + k];
                A[j * m + k] = A[p * m + k];
                A[p * m + k] = t;
            }
        for (int i = j + 1; i < m; i++) {
            A[i * m + j] /= A[j * m + j];
            for (int k = j + 1; k < m; k++) A[i * m + k] -= A[i * m + j] * A[j * m + k];
        }
    }
    return 0;
}

static void lu_solve(int m, const double *A, const int *piv, double *x)
{
    for (int j = 0; j < m; j++)
        if (piv[j] != j) {
            double t = x[j];
            x[j] = x[piv[j]];
            x[piv[j]] = t;
        }
    for (int i = 0; i < m; i++) {
        double s = x[i];
        for (int k = 0; k < i; k++) s -= A[i * m + k] * x[k];
        x[i] = s;
    }
    for (int i = m - 1; i >= 0; i--) {
        double s = x[i];
        for (int k = i + 1; k < m; k++) s -= A[i * m + k] * x[k];
        x[i] = s / A[i * m + i];
    }
}

/* ------------------------------------------------------------------ */
/* Static condensation (Sec. 3.2.3):                                    */
/*   y = Kaa^{-1} r,  X = Kaa^{-1} KaF                                  */
/*   algorithmic stress  Palg = Pr - KFa y                              */
/*   condensed tangent   Cr   = KFF - KFa X      (eq. Biot_Tangent)     */
/* ------------------------------------------------------------------ */
static int condense_point(int m, const double *Kaa, const double *KaF, const double *KFF,
                          const double *r, const double *Pr, double *y, double *X,
                          double *Palg, double *Cr)
{
    int status = 0;
    double *L = (double *)malloc(sizeof(double) * m * m);
    int *piv = (int *)malloc(sizeof(int) * m);
    double *col = (double *)malloc(sizeof(double) * m);
    memcpy(L, Kaa, sizeof(double) * m * m);
    int use_lu = 0;
    if (cholesky(m, L) != 0) {
        status |= ORC_PT_NOT_SPD;
        memcpy(L, Kaa, sizeof(double) * m * m);
        if (lu_factor(m, L, piv) != 0) status |= ORC_PT_NONFINITE;
        use_lu = 1;
    }
    memcpy(y, r, sizeof(double) * m);
    if (use_lu) lu_solve(m, L, piv, y); else chol_solve(m, L, y);
    for (int J = 0; J < 9; J++) {
        for (int k = 0; k < m; k++) col[k] = KaF[k * 9 + J];
        if (use_lu) lu_solve(m, L, piv, col); else chol_solve(m, L, col);
        for (int k = 0; k < m; k++) X[k * 9 + J] = col[k];
    }
    for (int I = 0; I < 9; I++) {
        double s = Pr[I];
        for (int k = 0; k < m; k++) s -= KaF[k * 9 + I] * y[k];
        Palg[I] = s;
        for (int J = 0; J < 9; J++) {
            double t = KFF[9 * I + J];
            for (int k = 0; k < m; k++) t -= KaF[k * 9 + I] * X[k * 9 + J];
            Cr[9 * I + J] = t;
        }
    }
    free(L);
    free(piv);
    free(col);
    return status;
}

/* ------------------------------------------------------------------ */
/* Push-out from the RVE frame (which sees only Ubar) to the macro      */
/* frame (Sec. 3.2.2 eqs. workconjugacy, biotstress, in second-Piola    */
/* form): the Biot stress T = sym(Palg_r) is work conjugate to Ubar;    */
/* Ubar S + S Ubar = 2 T gives the second Piola stress S and            */
/* Pbar = Fbar S.  Tangent column k (direction E_k):                    */
/*   dC = E_k^T F + F^T E_k,  dU = Linv(dC),  dT = sym(Cr : dU),        */
/*   dS = Linv(2 dT - dU S - S dU),  Cbar e_k = E_k S + F dS.           */
/* ------------------------------------------------------------------ */
static void push_out(const polar_t *P, const double *Palg, const double *Cr,
                     double *Pbar, double *Cbar, double *S_out)
{
    double T[9], S[9], twoT[9];
    m3_sym(Palg, T);
    for (int i = 0; i < 9; i++) twoT[i] = 2.0 * T[i];
    lyap_inv(P, twoT, S);
    if (S_out) memcpy(S_out, S, sizeof S);
    m3_mul(P->F, S, Pbar);
    for (int k = 0; k < 9; k++) {
        double E[9] = {0};
        E[k] = 1.0;
        double dU[9], dP[9], dT[9], B[9], dS[9], t1[9], t2[9];
        stretch_increment(P, E, dU);
        for (int I = 0; I < 9; I++) {
            double s = 0.0;
            for (int J = 0; J < 9; J++) s += Cr[9 * I + J] * dU[J];
            dP[I] = s;
        }
        m3_sym(dP, dT);
        m3_mul(dU, S, t1);
        m3_mul(S, dU, t2);
        for (int i = 0; i < 9; i++) B[i] = 2.0 * dT[i] - t1[i] - t2[i];
        lyap_inv(P, B, dS);
        m3_mul(E, S, t1);
        m3_mul(P->F, dS, t2);
        for (int I = 0; I < 9; I++) Cbar[9 * I + k] = t1[I] + t2[I];
    }
}

/* ------------------------------------------------------------------ */
/* Updated-Lagrangian output (Sec. 3.2.2 eq. biotstress, App. A).       */
/* The Biot stress of the macro point is T = sym(R^T Pbar) = sym(Palg_r) */
/* (the RVE sees Ubar, so Pbar = Rbar Palg_r).  Eq. (biotstress) links it */
/* to the Cauchy stress sigma by the linear map                          */
/*   T_kl = J/2 (R_ik sigma_ij Finv_lj + Finv_ki sigma_ij R_jl),         */
/* whose 9 x 9 matrix is LU-factorised and solved (never inverted, as    */
/* the appendix advises).  App. A: dsigma/dD = dsigma/dT : C^B : dUdot/dD */
/* with C^B = dT/dUdot the condensed tangent restricted to symmetric     */
/* stretch rates and symmetrised, C^B = sym o Cr o sym, and              */
/* dUdot/dD ~ R_ki F_lj (constant rotation over the step).  Output       */
/* sigma[3 i + j], dsdD[9 (3 i + j) + 3 k + l] = dsigma_ij / dD_kl.      */
/* ------------------------------------------------------------------ */
static int cauchy_out(const polar_t *P, const double *Palg, const double *Cr, double *sig,
                      double *dsdD)
{
    const double J = m3_det(P->F);
    double Fi[9], M[81], T[9];
    int piv[9];
    m3_inv(P->F, Fi);
    for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++)
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++)
                    M[9 * (3 * k + l) + 3 * i + j] =
                        0.5 * J * (P->R[3 * i + k] * Fi[3 * l + j] + Fi[3 * k + i] * P->R[3 * j + l]);
    if (lu_factor(9, M, piv) != 0) return ORC_PT_NONFINITE;
    m3_sym(Palg, T);
    memcpy(sig, T, sizeof T);
    lu_solve(9, M, piv, sig);
    for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) {
            /* stretch rate of a unit D_kl: Udot_ij = R_ki F_lj, symmetrised */
            double Ud[9], dU[9], dP[9], dT[9];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) Ud[3 * i + j] = P->R[3 * k + i] * P->F[3 * l + j];
            m3_sym(Ud, dU);
            for (int I = 0; I < 9; I++) {
                double acc = 0.0;
                for (int Jc = 0; Jc < 9; Jc++) acc += Cr[9 * I + Jc] * dU[Jc];
                dP[I] = acc;
            }
            m3_sym(dP, dT);
            lu_solve(9, M, piv, dT);
            for (int I = 0; I < 9; I++) dsdD[9 * I + 3 * k + l] = dT[I];
        }
    return (all_finite(sig, 9) && all_finite(dsdD, 81)) ? 0 : ORC_PT_NONFINITE;
}

/* ------------------------------------------------------------------ */
/* One full evaluate + condense (+ push-out) at one macro point.        */
/* ------------------------------------------------------------------ */
typedef struct {
    double *r, *Pr, *Kaa, *KaF, *KFF, *y, *X, Palg[9], Cr[81], Pbar[9], Cbar[81], S[9];
    polar_t P;
    double rnorm;
} work_t;

static void work_alloc(work_t *W, int m)
{
    W->r = (double *)calloc(m, sizeof(double));
    W->Pr = (double *)calloc(9, sizeof(double));
    W->Kaa = (double *)calloc((size_t)m * m, sizeof(double));
    W->KaF = (double *)calloc((size_t)m * 9, sizeof(double));
    W->KFF = (double *)calloc(81, sizeof(double));
    W->y = (double *)calloc(m, sizeof(double));
    W->X = (double *)calloc((size_t)m * 9, sizeof(double));
}

static void work_free(work_t *W)
{
    free(W->r); free(W->Pr); free(W->Kaa); free(W->KaF); free(W->KFF); free(W->y); free(W->X);
}

/* objective: 1 = RVE sees Ubar (default), 0 = RVE sees Fbar directly */
static int point_eval(const rve_t *c, int objective, const double *Fbar, const double *a, work_t *W,
                      const double *hn, double *ht)
{
    int status = 0;
    const double *Fr;
    if (!all_finite(Fbar, 9) || !all_finite(a, c->m)) return ORC_PT_NONFINITE;
    if (objective) {
        /* a proper polar split F = R U with det R = +1 needs det F > 0 */
        if (!(m3_det(Fbar) > 0.0)) return ORC_PT_JNONPOS;
        polar_split(Fbar, &W->P);
        Fr = W->P.U;
    } else {
        Fr = Fbar;
    }
    status |= eval_point(c, Fr, a, W->r, W->Pr, W->Kaa, W->KaF, W->KFF, hn, ht);
    if (status & ORC_PT_JNONPOS) return status;
    status |= condense_point(c->m, W->Kaa, W->KaF, W->KFF, W->r, W->Pr, W->y, W->X, W->Palg, W->Cr);
    double s = 0.0;
    for (int k = 0; k < c->m; k++) s += W->r[k] * W->r[k];
    W->rnorm = sqrt(s);
    if (objective) {
        push_out(&W->P, W->Palg, W->Cr, W->Pbar, W->Cbar, W->S);
    } else {
        memcpy(W->Pbar, W->Palg, sizeof W->Pbar);
        memcpy(W->Cbar, W->Cr, sizeof W->Cbar);
    }
    if (!all_finite(W->Pbar, 9) || !all_finite(W->Cbar, 81)) status |= ORC_PT_NONFINITE;
    return status;
}

/* monolithic update a <- a - (y + X dFr)   (Sec. 3.2.3) */
static void update_point(const rve_t *c, int objective, const work_t *W, const double *dFbar, double *a)
{
    const int m = c->m;
    double dFr[9] = {0};
    if (dFbar) {
        if (objective) stretch_increment(&W->P, dFbar, dFr);
        else memcpy(dFr, dFbar, sizeof dFr);
    }
    for (int k = 0; k < m; k++) {
        double s = W->y[k];
        for (int J = 0; J < 9; J++) s += W->X[k * 9 + J] * dFr[J];
        a[k] -= s;
    }
}

/* ================================================================== */
/* Exported batch entry points (row-major AoS arrays, one macro point  */
/* per row).  Status codes per point as defined above.                 */
/* ================================================================== */

static rve_t make_rve(int m, int Q, const double *G, const double *w, const int *phase,
                      const double *theta)
{
    rve_t c;
    c.m = m; c.Q = Q; c.G = G; c.w = w; c.phase = phase;
    for (int i = 0; i < 4; i++) c.theta[i] = theta[i];
    c.V0 = 0.0;
    for (int q = 0; q < Q; q++) c.V0 += w[q];
    c.j2 = 0;
    for (int i = 0; i < 8; i++) c.mat[i] = 0.0;
    return c;
}

int orc_neo_hooke(int64_t N, const double *F, double mu, double lam, double *P, double *A)
{
    int bad = 0;
    for (int64_t b = 0; b < N; b++)
        if (neo_hooke(F + 9 * b, mu, lam, P + 9 * b, A ? A + 81 * b : NULL, NULL, NULL, NULL) != 0) bad++;
    return bad;
}

/* Neo-Hooke strain energy, for the energy-consistency pins */
int orc_neo_hooke_energy(int64_t N, const double *F, double mu, double lam, double *Wout)
{
    for (int64_t b = 0; b < N; b++) {
        const double *Fb = F + 9 * b;
        double J = m3_det(Fb), I1 = 0.0;
        for (int i = 0; i < 9; i++) I1 += Fb[i] * Fb[i];
        double l = log(J);
        Wout[b] = 0.5 * mu * (I1 - 3.0) - mu * l + 0.5 * lam * l * l;
    }
    return 0;
}

int orc_polar(int64_t N, const double *F, double *U, double *R, double *V, double *u)
{
    for (int64_t b = 0; b < N; b++) {
        polar_t P;
        polar_split(F + 9 * b, &P);
        if (U) memcpy(U + 9 * b, P.U, sizeof P.U);
        if (R) memcpy(R + 9 * b, P.R, sizeof P.R);
        if (V) memcpy(V + 9 * b, P.V, sizeof P.V);
        if (u) memcpy(u + 3 * b, P.u, sizeof P.u);
    }
    return 0;
}

/* raw RVE-frame blocks at given (Fr, a): no polar split, no condensation */
int orc_eval(int m, int Q, const double *G, const double *w, const int *phase, const double *theta,
             int64_t N, const double *Fr, const double *a, double *r, double *Pr, double *Kaa,
             double *KaF, double *KFF, int *status)
{
    rve_t c = make_rve(m, Q, G, w, phase, theta);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < N; b++) {
        status[b] = eval_point(&c, Fr + 9 * b, a + (size_t)m * b, r + (size_t)m * b, Pr + 9 * b,
                               Kaa + (size_t)m * m * b, KaF + (size_t)9 * m * b, KFF + 81 * b,
                               NULL, NULL);
    }
    return 0;
}

/* full evaluate + condense (+ push-out): Pbar = algorithmic stress, Cbar = condensed tangent */
int orc_point_eval(int m, int Q, const double *G, const double *w, const int *phase,
                   const double *theta, int objective, int64_t N, const double *Fbar,
                   const double *a, double *Pbar, double *Cbar, double *rnorm, double *y,
                   double *X, double *Palg_r, double *Cr, int *status)
{
    rve_t c = make_rve(m, Q, G, w, phase, theta);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < N; b++) {
        work_t W;
        work_alloc(&W, m);
        int st = point_eval(&c, objective, Fbar + 9 * b, a + (size_t)m * b, &W, NULL, NULL);
        memcpy(Pbar + 9 * b, W.Pbar, sizeof W.Pbar);
        memcpy(Cbar + 81 * b, W.Cbar, sizeof W.Cbar);
        if (rnorm) rnorm[b] = W.rnorm;
        if (y) memcpy(y + (size_t)m * b, W.y, sizeof(double) * m);
        if (X) memcpy(X + (size_t)9 * m * b, W.X, sizeof(double) * 9 * m);
        if (Palg_r) memcpy(Palg_r + 9 * b, W.Palg, sizeof W.Palg);
        if (Cr) memcpy(Cr + 81 * b, W.Cr, sizeof W.Cr);
        status[b] = st;
        work_free(&W);
    }
    return 0;
}

/*
 * Micro Newton at fixed Fbar (ROM amplitudes only): repeat
 *   evaluate + condense; stop when ||r||_2 < tol; else a <- a - y,
 * at most max_it evaluations.  Reports Pbar, Cbar of the last evaluation.
 */
int orc_newton(int m, int Q, const double *G, const double *w, const int *phase,
               const double *theta, int objective, int64_t N, const double *Fbar, double *a,
               double tol, int max_it, double *Pbar, double *Cbar, double *rnorm, int *iters,
               int *status)
{
    rve_t c = make_rve(m, Q, G, w, phase, theta);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < N; b++) {
        work_t W;
        work_alloc(&W, m);
        double *ab = a + (size_t)m * b;
        int st = 0, nev = 0, conv = 0;
        for (int it = 0; it < max_it; it++) {
            st = point_eval(&c, objective, Fbar + 9 * b, ab, &W, NULL, NULL);
            nev++;
            if (st & (ORC_PT_JNONPOS | ORC_PT_NONFINITE)) break;
            if (W.rnorm < tol) { conv = 1; break; }
            if (it + 1 < max_it) update_point(&c, objective, &W, NULL, ab);
        }
        if (!conv) st |= ORC_PT_NOCONV;
        memcpy(Pbar + 9 * b, W.Pbar, sizeof W.Pbar);
        memcpy(Cbar + 81 * b, W.Cbar, sizeof W.Cbar);
        rnorm[b] = W.rnorm;
        if (iters) iters[b] = nev;
        status[b] = st;
        work_free(&W);
    }
    return 0;
}

/*
 * Monolithic iterations (Sec. 3.2.3): for k = 0..K-1, evaluate + condense
 * at (Fbar_k, a_k), record Pbar_k, Cbar_k, then a_{k+1} = a_k - (y + X dFr_k)
 * and Fbar_{k+1} = Fbar_k + dFbar_k.  Outputs are [K][N][...].
 */
int orc_monolithic(int m, int Q, const double *G, const double *w, const int *phase,
                   const double *theta, int objective, int64_t N, const double *Fbar0,
                   const double *dFbar, int K, double *a, double *Pbar, double *Cbar,
                   double *rnorm, int *status)
{
    rve_t c = make_rve(m, Q, G, w, phase, theta);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < N; b++) {
        work_t W;
        work_alloc(&W, m);
        double F[9];
        memcpy(F, Fbar0 + 9 * b, sizeof F);
        double *ab = a + (size_t)m * b;
        int st_all = 0;
        for (int k = 0; k < K; k++) {
            int st = point_eval(&c, objective, F, ab, &W, NULL, NULL);
            st_all |= st;
            memcpy(Pbar + ((size_t)k * N + b) * 9, W.Pbar, sizeof W.Pbar);
            memcpy(Cbar + ((size_t)k * N + b) * 81, W.Cbar, sizeof W.Cbar);
            rnorm[(size_t)k * N + b] = W.rnorm;
            const double *dF = dFbar + ((size_t)k * N + b) * 9;
            update_point(&c, objective, &W, dF, ab);
            for (int i = 0; i < 9; i++) F[i] += dF[i];
        }
        status[b] = st_all;
        work_free(&W);
    }
    return 0;
}

/*
 * Adjoint backward at a converged state (a solves r(a) = 0 at Fbar).
 * Loss cotangent g = dL/dPbar (per point).  Pull-back to the RVE frame
 * g_r = 2 Linv(sym(F^T g)); adjoint solve lambda = Kaa^{-T} KaF g_r = X g_r;
 * with v_q = g_r - G_q lambda:
 *   h_r        = sum_q w_q A_q v_q                   (= Cr^T g_r)
 *   dL/dmu_p   = sum_{q in p} w_q v_q : (F_q - F_q^{-T})
 *   dL/dlam_p  = sum_{q in p} w_q v_q : (ln J_q F_q^{-T})
 * and dL/dFbar = g S + 2 F Linv(sym(h_r) - Lam S - S Lam), Lam = g_r / 2.
 * gtheta receives the sum over points in index order.
 */
int orc_backward(int m, int Q, const double *G, const double *w, const int *phase,
                 const double *theta, int objective, int64_t N, const double *Fbar,
                 const double *a, const double *g, double *gF, double *gtheta_pt,
                 double *gtheta, int *status)
{
    rve_t c = make_rve(m, Q, G, w, phase, theta);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < N; b++) {
        work_t W;
        work_alloc(&W, m);
        const double *ab = a + (size_t)m * b;
        const double *gb = g + 9 * b;
        int st = point_eval(&c, objective, Fbar + 9 * b, ab, &W, NULL, NULL);
        double Fr[9], gr[9], Lam[9];
        if (objective) {
            double FtG[9], H[9];
            memcpy(Fr, W.P.U, sizeof Fr);
            m3_tmul(W.P.F, gb, FtG);
            m3_sym(FtG, H);
            lyap_inv(&W.P, H, Lam);
            for (int i = 0; i < 9; i++) gr[i] = 2.0 * Lam[i];
        } else {
            memcpy(Fr, Fbar + 9 * b, sizeof Fr);
            memcpy(gr, gb, sizeof gr);
        }
        double *lambda = (double *)malloc(sizeof(double) * m);
        for (int k = 0; k < m; k++) {
            double s = 0.0;
            for (int J = 0; J < 9; J++) s += W.X[k * 9 + J] * gr[J];
            lambda[k] = s;
        }
        double hr[9] = {0}, gt[4] = {0};
        for (int q = 0; q < Q; q++) {
            const double *Gq = G + (size_t)q * 9 * m;
            const int p = phase[q];
            const double mu = theta[2 * p], lam = theta[2 * p + 1];
            double F[9], v[9], P[9], A[81], J, ell, Fi[9];
            for (int I = 0; I < 9; I++) {
                double s = Fr[I], t = gr[I];
                for (int k = 0; k < m; k++) {
                    s += ab[k] * Gq[I * m + k];
                    t -= Gq[I * m + k] * lambda[k];
                }
                F[I] = s;
                v[I] = t;
            }
            if (neo_hooke(F, mu, lam, P, A, &J, &ell, Fi) != 0) { st |= ORC_PT_JNONPOS; continue; }
            for (int I = 0; I < 9; I++) {
                double s = 0.0;
                for (int J2 = 0; J2 < 9; J2++) s += A[9 * I + J2] * v[J2];
                hr[I] += w[q] / c.V0 * s;
            }
            double dmu = 0.0, dlam = 0.0;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    dmu += v[3 * i + j] * (F[3 * i + j] - Fi[3 * j + i]);
                    dlam += v[3 * i + j] * ell * Fi[3 * j + i];
                }
            gt[2 * p] += w[q] / c.V0 * dmu;
            gt[2 * p + 1] += w[q] / c.V0 * dlam;
        }
        double gFb[9];
        if (objective) {
            double M[9], hs[9], t1[9], t2[9], N2[9], FN[9], gS[9];
            m3_sym(hr, hs);
            m3_mul(Lam, W.S, t1);
            m3_mul(W.S, Lam, t2);
            for (int i = 0; i < 9; i++) M[i] = hs[i] - t1[i] - t2[i];
            lyap_inv(&W.P, M, N2);
            m3_mul(W.P.F, N2, FN);
            m3_mul(gb, W.S, gS);
            for (int i = 0; i < 9; i++) gFb[i] = gS[i] + 2.0 * FN[i];
        } else {
            memcpy(gFb, hr, sizeof gFb);
        }
        memcpy(gF + 9 * b, gFb, sizeof gFb);
        memcpy(gtheta_pt + 4 * b, gt, sizeof gt);
        status[b] = st;
        free(lambda);
        work_free(&W);
    }
    for (int i = 0; i < 4; i++) gtheta[i] = 0.0;
    for (int64_t b = 0; b < N; b++)
        for (int i = 0; i < 4; i++) gtheta[i] += gtheta_pt[4 * b + i];
    return 0;
}

/* Cauchy stress and Updated-Lagrangian tangent from the RVE-frame
   algorithmic stress Palg_r and condensed tangent Cr at Fbar */
int orc_cauchy(int64_t N, const double *Fbar, const double *Palg_r, const double *Cr, double *sigma,
               double *dsdD, int *status)
{
    for (int64_t b = 0; b < N; b++) {
        polar_t P;
        polar_split(Fbar + 9 * b, &P);
        status[b] = cauchy_out(&P, Palg_r + 9 * b, Cr + 81 * b, sigma + 9 * b, dsdD + 81 * b);
    }
    return 0;
}

/* linearised stretch increment, exported for the update pins */
int orc_stretch_increment(int64_t N, const double *F, const double *dF, double *dU)
{
    for (int64_t b = 0; b < N; b++) {
        polar_t P;
        polar_split(F + 9 * b, &P);
        stretch_increment(&P, dF + 9 * b, dU + 9 * b);
    }
    return 0;
}


/* ================================================================== */
/* J2 plasticity entry points (Sec. 5 Example 1 material, state at the  */
/* hyper integration points).  mat[8] = per phase (mu, lam, sigma_y0,    */
/* H); history per macro point [Q][7] (eps_p xx yy zz xy yz xz, alpha): */
/* hist_n is the committed state of the last converged increment,       */
/* hist_t receives the state of the evaluation (the caller commits it).  */
/* ================================================================== */
int orc_j2_law(int64_t N, const double *F, const double *mp, const double *hn, double *P,
               double *A, double *ht)
{
    for (int64_t b = 0; b < N; b++)
        j2_law(F + 9 * b, mp, hn + 7 * b, P + 9 * b, A + 81 * b, ht + 7 * b);
    return 0;
}

static rve_t make_rve_j2(int m, int Q, const double *G, const double *w, const int *phase,
                         const double *mat)
{
    const double th0[4] = {0.0, 0.0, 0.0, 0.0};
    rve_t c = make_rve(m, Q, G, w, phase, th0);
    c.j2 = 1;
    for (int i = 0; i < 8; i++) c.mat[i] = mat[i];
    return c;
}

int orc_j2_eval(int m, int Q, const double *G, const double *w, const int *phase,
                const double *mat, int64_t N, const double *Fr, const double *a,
                const double *hist_n, double *r, double *Pr, double *Kaa, double *KaF,
                double *KFF, double *hist_t, int *status)
{
    rve_t c = make_rve_j2(m, Q, G, w, phase, mat);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < N; b++)
        status[b] = eval_point(&c, Fr + 9 * b, a + (size_t)m * b, r + (size_t)m * b, Pr + 9 * b,
                               Kaa + (size_t)m * m * b, KaF + (size_t)9 * m * b, KFF + 81 * b,
                               hist_n + (size_t)7 * Q * b, hist_t + (size_t)7 * Q * b);
    return 0;
}

/*
 * Micro Newton at fixed Fbar with the committed history hist_n (every
 * evaluation returns from it); hist_t gets the history of the last
 * evaluation, i.e. of the converged state.
 */
int orc_j2_newton(int m, int Q, const double *G, const double *w, const int *phase,
                  const double *mat, int objective, int64_t N, const double *Fbar, double *a,
                  const double *hist_n, double tol, int max_it, double *Pbar, double *Cbar,
                  double *rnorm, int *iters, int *status, double *hist_t)
{
    rve_t c = make_rve_j2(m, Q, G, w, phase, mat);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < N; b++) {
        work_t W;
        work_alloc(&W, m);
        double *ab = a + (size_t)m * b;
        const double *hn = hist_n + (size_t)7 * Q * b;
        double *ht = hist_t + (size_t)7 * Q * b;
        int st = 0, nev = 0, conv = 0;
        for (int it = 0; it < max_it; it++) {
            st = point_eval(&c, objective, Fbar + 9 * b, ab, &W, hn, ht);
            nev++;
            if (st & (ORC_PT_JNONPOS | ORC_PT_NONFINITE)) break;
            if (W.rnorm < tol) { conv = 1; break; }
            if (it + 1 < max_it) update_point(&c, objective, &W, NULL, ab);
        }
        if (!conv) st |= ORC_PT_NOCONV;
        memcpy(Pbar + 9 * b, W.Pbar, sizeof W.Pbar);
        memcpy(Cbar + 81 * b, W.Cbar, sizeof W.Cbar);
        rnorm[b] = W.rnorm;
        if (iters) iters[b] = nev;
        status[b] = st;
        work_free(&W);
    }
    return 0;
}

/* ================================================================== */
/* Biot form of the condensed RVE-frame state (Sec. 3.2.2 eq.           */
/* workconjugacy: the Biot stress, the symmetric part of the RVE-frame  */
/* stress, is work conjugate to the stretch; Sec. 3.2.3 eq.             */
/* Biot_Tangent on symmetric stretch increments).  Voigt order          */
/* (11, 22, 33, 12, 23, 13) with engineering shear strains              */
/* gamma = (U11, U22, U33, 2 U12, 2 U23, 2 U13): a stretch increment is */
/* dU = sum_l dgamma_l D_l with D = (E11, E22, E33, (E12 + E21) / 2,     */
/* (E23 + E32) / 2, (E13 + E31) / 2), the stress T_k = D_k : Palg and   */
/* the tangent CB_kl = dT_k / dgamma_l = D_k : Cr : D_l.                */
/* ================================================================== */
static void voigt_dual(int k, double *D)
{
    static const int ii[6] = {0, 1, 2, 0, 1, 0}, jj[6] = {0, 1, 2, 1, 2, 2};
    memset(D, 0, sizeof(double) * 9);
    if (k < 3) {
        D[3 * ii[k] + jj[k]] = 1.0;
    } else {
        D[3 * ii[k] + jj[k]] = 0.5;
        D[3 * jj[k] + ii[k]] = 0.5;
    }
}

int orc_biot(int64_t N, const double *Palg_r, const double *Cr, double *T, double *CB)
{
    double D[6][9];
    for (int k = 0; k < 6; k++) voigt_dual(k, D[k]);
    for (int64_t b = 0; b < N; b++) {
        const double *P = Palg_r + 9 * b, *C = Cr + 81 * b;
        for (int k = 0; k < 6; k++) {
            double s = 0.0;
            for (int I = 0; I < 9; I++) s += D[k][I] * P[I];
            T[6 * b + k] = s;
            for (int l = 0; l < 6; l++) {
                double t = 0.0;
                for (int I = 0; I < 9; I++)
                    for (int J = 0; J < 9; J++) t += D[k][I] * C[9 * I + J] * D[l][J];
                CB[36 * b + 6 * k + l] = t;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Training integrand of the empirical cubature (Sec. 3.3, eq. ECM1 and */
/* the training matrix below it).  For snapshot k, given as the RVE-    */
/* frame macro input Fr^k and its converged mode coefficients a^k, and  */
/* for every candidate (full-integration) point g, the integrand is the */
/* point's force vector: the mode forces G_g^T P(F_g) (m values) and    */
/* the nine first Piola stress components P(F_g), with                  */
/* F_g = Fr^k + G_g a^k.  Layout f[k][i][g], i < m + 9.  Returns the    */
/* number of (k, g) pairs with det F_g <= 0 (their entries are zero).   */
/* ------------------------------------------------------------------ */
int orc_ecm_integrand(int m, int M, const double *G, const int *phase, const double *theta,
                      int p, const double *Fr, const double *a, double *f)
{
    const int nt = m + 9;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int k = 0; k < p; k++) {
        double *fk = f + (size_t)k * nt * M;
        for (int g = 0; g < M; g++) {
            const double *Gg = G + (size_t)g * 9 * m;
            double F[9], P[9];
            for (int I = 0; I < 9; I++) {
                double s = Fr[9 * k + I];
                for (int n = 0; n < m; n++) s += a[(size_t)m * k + n] * Gg[I * m + n];
                F[I] = s;
            }
            if (neo_hooke(F, theta[2 * phase[g]], theta[2 * phase[g] + 1], P, NULL, NULL, NULL,
                          NULL) != 0) {
                bad++;
                for (int i = 0; i < nt; i++) fk[(size_t)i * M + g] = 0.0;
                continue;
            }
            for (int n = 0; n < m; n++) {
                double s = 0.0;
                for (int I = 0; I < 9; I++) s += Gg[I * m + n] * P[I];
                fk[(size_t)n * M + g] = s;
            }
            for (int I = 0; I < 9; I++) fk[(size_t)(m + I) * M + g] = P[I];
        }
    }
    return bad;
}
