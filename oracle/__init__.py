"""FP64 CPU oracle of the hyper-reduced RVE evaluation (test infrastructure).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path
(the HIP library and its binding) never imports, links or calls it.

The arithmetic lives in ``hrom_oracle.c`` (plain C loops in double precision,
one macro point at a time); this module only marshals numpy arrays into it.
Every array is a row-major numpy array in its natural shape:
``G[Q, 9, m]``, ``Fbar[N, 3, 3]`` (or ``[N, 9]``), ``a[N, m]``.

Every function here is pinned by tests against facts that do not come from
the oracle itself (``tests/test_oracle_pins.py``, ``tests/test_oracle_j2.py``,
``tests/test_oracle_ecm.py``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hrom_oracle.c")
# HROM_ORACLE_LIB: load another build of the same source (e.g. the sanitizer
# build of check_sanitizers.sh) instead of the default one
_LIB = os.environ.get("HROM_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))

PT_JNONPOS, PT_NOT_SPD, PT_NOCONV, PT_NONFINITE = 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, d = C.c_int64, C.c_int, C.c_double
        L.orc_neo_hooke.argtypes = [i64, P, d, d, P, P]
        L.orc_neo_hooke_energy.argtypes = [i64, P, d, d, P]
        L.orc_polar.argtypes = [i64, P, P, P, P, P]
        L.orc_eval.argtypes = [i32, i32, P, P, P, P, i64, P, P, P, P, P, P, P, P]
        L.orc_point_eval.argtypes = [i32, i32, P, P, P, P, i32, i64, P, P, P, P, P, P, P,
                                     P, P, P]
        L.orc_newton.argtypes = [i32, i32, P, P, P, P, i32, i64, P, P, d, i32, P, P, P, P, P]
        L.orc_monolithic.argtypes = [i32, i32, P, P, P, P, i32, i64, P, P, i32, P, P, P, P, P]
        L.orc_backward.argtypes = [i32, i32, P, P, P, P, i32, i64, P, P, P, P, P, P, P]
        L.orc_stretch_increment.argtypes = [i64, P, P, P]
        L.orc_cauchy.argtypes = [i64, P, P, P, P, P, P]
        L.orc_j2_law.argtypes = [i64, P, P, P, P, P, P]
        L.orc_biot.argtypes = [i64, P, P, P, P]
        L.orc_ecm_integrand.argtypes = [i32, i32, P, P, P, i32, P, P, P]
        L.orc_j2_eval.argtypes = [i32, i32, P, P, P, P, i64, P, P, P, P, P, P, P, P, P, P]
        L.orc_j2_newton.argtypes = [i32, i32, P, P, P, P, i32, i64, P, P, P, d, i32, P, P, P,
                                    P, P, P]
        _lib = L
    return _lib


def _f64(x, shape=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if shape is not None:
        x = x.reshape(shape)
    return x


def _p(x):
    return None if x is None else x.ctypes.data_as(C.c_void_p)


def _cluster_args(cl, theta):
    G = _f64(cl.G)
    w = _f64(cl.w)
    ph = np.ascontiguousarray(cl.phase, dtype=np.int32)
    th = _f64(theta, (4,))
    return (G, w, ph, th)


def neo_hooke(F, mu, lam):
    """Neo-Hooke first Piola stress P[N,9] and tangent A[N,9,9] = dP/dF."""
    F = _f64(F)
    N = F.size // 9
    F = F.reshape(N, 9)
    P = np.zeros((N, 9))
    A = np.zeros((N, 9, 9))
    bad = lib().orc_neo_hooke(N, _p(F), mu, lam, _p(P), _p(A))
    if bad:
        raise ValueError("det F <= 0 at %d points" % bad)
    return P, A


def neo_hooke_energy(F, mu, lam):
    F = _f64(F)
    N = F.size // 9
    W = np.zeros(N)
    lib().orc_neo_hooke_energy(N, _p(F.reshape(N, 9)), mu, lam, _p(W))
    return W


def polar(F):
    """Polar split F = R U: returns (U, R, V, u) with U = V diag(u) V^T."""
    F = _f64(F)
    N = F.size // 9
    U, R, V = (np.zeros((N, 3, 3)) for _ in range(3))
    u = np.zeros((N, 3))
    lib().orc_polar(N, _p(F.reshape(N, 9)), _p(U), _p(R), _p(V), _p(u))
    return U, R, V, u


def stretch_increment(F, dF):
    F = _f64(F)
    N = F.size // 9
    dF = _f64(dF, (N, 9))
    dU = np.zeros((N, 3, 3))
    lib().orc_stretch_increment(N, _p(F.reshape(N, 9)), _p(dF), _p(dU))
    return dU


def eval_blocks(cl, theta, Fr, a):
    """Raw RVE-frame blocks at given (Fr, a): dict of r, Pr, Kaa, KaF, KFF, status."""
    G, w, ph, th = _cluster_args(cl, theta)
    Fr = _f64(Fr)
    N = Fr.size // 9
    a = _f64(a, (N, cl.m))
    m = cl.m
    out = dict(r=np.zeros((N, m)), Pr=np.zeros((N, 9)), Kaa=np.zeros((N, m, m)),
               KaF=np.zeros((N, m, 9)), KFF=np.zeros((N, 9, 9)),
               status=np.zeros(N, dtype=np.int32))
    lib().orc_eval(m, cl.Q, _p(G), _p(w), _p(ph), _p(th), N, _p(Fr.reshape(N, 9)), _p(a),
                   _p(out["r"]), _p(out["Pr"]), _p(out["Kaa"]), _p(out["KaF"]),
                   _p(out["KFF"]), _p(out["status"]))
    return out


def point_eval(cl, theta, Fbar, a, objective=True):
    """One evaluate + condense (+ push-out) at given (Fbar, a)."""
    G, w, ph, th = _cluster_args(cl, theta)
    Fbar = _f64(Fbar)
    N = Fbar.size // 9
    a = _f64(a, (N, cl.m))
    m = cl.m
    o = dict(Pbar=np.zeros((N, 9)), Cbar=np.zeros((N, 9, 9)), rnorm=np.zeros(N),
             y=np.zeros((N, m)), X=np.zeros((N, m, 9)), Palg_r=np.zeros((N, 9)),
             Cr=np.zeros((N, 9, 9)), status=np.zeros(N, dtype=np.int32))
    lib().orc_point_eval(m, cl.Q, _p(G), _p(w), _p(ph), _p(th), int(objective), N,
                         _p(Fbar.reshape(N, 9)), _p(a), _p(o["Pbar"]), _p(o["Cbar"]),
                         _p(o["rnorm"]), _p(o["y"]), _p(o["X"]), _p(o["Palg_r"]), _p(o["Cr"]),
                         _p(o["status"]))
    return o


def cauchy(Fbar, Palg_r, Cr):
    """Cauchy stress sigma [N, 9] and the Updated-Lagrangian tangent
    dsigma/dD [N, 9, 9] from the RVE-frame algorithmic stress and condensed
    tangent at Fbar (eq. biotstress, App. A); also the per-point status."""
    Fbar = _f64(Fbar)
    N = Fbar.size // 9
    Pa = _f64(Palg_r, (N, 9))
    Cr = _f64(Cr, (N, 81))
    sig, dsdD = np.zeros((N, 9)), np.zeros((N, 9, 9))
    st = np.zeros(N, dtype=np.int32)
    lib().orc_cauchy(N, _p(Fbar.reshape(N, 9)), _p(Pa), _p(Cr), _p(sig), _p(dsdD), _p(st))
    return sig, dsdD, st


def newton(cl, theta, Fbar, a0=None, tol=1e-10, max_it=25, objective=True):
    """Micro Newton to ||r||_2 < tol; returns dict with a, Pbar, Cbar, rnorm, iters, status."""
    G, w, ph, th = _cluster_args(cl, theta)
    Fbar = _f64(Fbar)
    N = Fbar.size // 9
    a = np.zeros((N, cl.m)) if a0 is None else _f64(a0, (N, cl.m)).copy()
    o = dict(a=a, Pbar=np.zeros((N, 9)), Cbar=np.zeros((N, 9, 9)), rnorm=np.zeros(N),
             iters=np.zeros(N, dtype=np.int32), status=np.zeros(N, dtype=np.int32))
    lib().orc_newton(cl.m, cl.Q, _p(G), _p(w), _p(ph), _p(th), int(objective), N,
                     _p(Fbar.reshape(N, 9)), _p(a), float(tol), int(max_it), _p(o["Pbar"]),
                     _p(o["Cbar"]), _p(o["rnorm"]), _p(o["iters"]), _p(o["status"]))
    return o


def monolithic(cl, theta, Fbar0, dFbar, a0=None, objective=True):
    """K monolithic iterations; dFbar[K, N, 3, 3].  Outputs Pbar[K,N,9], Cbar[K,N,9,9]."""
    G, w, ph, th = _cluster_args(cl, theta)
    Fbar0 = _f64(Fbar0)
    N = Fbar0.size // 9
    dF = _f64(dFbar)
    K = dF.shape[0]
    dF = dF.reshape(K, N, 9)
    a = np.zeros((N, cl.m)) if a0 is None else _f64(a0, (N, cl.m)).copy()
    o = dict(a=a, Pbar=np.zeros((K, N, 9)), Cbar=np.zeros((K, N, 9, 9)),
             rnorm=np.zeros((K, N)), status=np.zeros(N, dtype=np.int32))
    lib().orc_monolithic(cl.m, cl.Q, _p(G), _p(w), _p(ph), _p(th), int(objective), N,
                         _p(Fbar0.reshape(N, 9)), _p(dF), K, _p(a), _p(o["Pbar"]),
                         _p(o["Cbar"]), _p(o["rnorm"]), _p(o["status"]))
    return o


def backward(cl, theta, Fbar, a, g, objective=True):
    """Adjoint gradients at a converged state: (dL/dFbar[N,9], dL/dtheta[4], per-point[N,4])."""
    G, w, ph, th = _cluster_args(cl, theta)
    Fbar = _f64(Fbar)
    N = Fbar.size // 9
    a = _f64(a, (N, cl.m))
    g = _f64(g, (N, 9))
    gF = np.zeros((N, 9))
    gpt = np.zeros((N, 4))
    gth = np.zeros(4)
    st = np.zeros(N, dtype=np.int32)
    lib().orc_backward(cl.m, cl.Q, _p(G), _p(w), _p(ph), _p(th), int(objective), N,
                       _p(Fbar.reshape(N, 9)), _p(a), _p(g), _p(gF), _p(gpt), _p(gth), _p(st))
    return dict(gF=gF, gtheta=gth, gtheta_pt=gpt, status=st)


# ---------------------------------------------------------------- J2 plasticity
# Material of the paper's Example 1 (Sec. 5): mat[8] = per phase (mu, lambda,
# initial yield stress sigma_y0, linear hardening modulus H); history per
# (macro point, ECM point) = (eps_p xx yy zz xy yz xz, alpha).

def j2_law(F, mp, hn=None):
    """Pointwise J2 return map: sigma[N,9], tangent dsigma/dF [N,9,9], new history [N,7]."""
    F = _f64(F)
    N = F.size // 9
    hn = np.zeros((N, 7)) if hn is None else _f64(hn, (N, 7))
    P, A, ht = np.zeros((N, 9)), np.zeros((N, 9, 9)), np.zeros((N, 7))
    lib().orc_j2_law(N, _p(F.reshape(N, 9)), _p(_f64(mp, (4,))), _p(hn), _p(P), _p(A), _p(ht))
    return P, A, ht


def j2_eval(cl, mat, Fr, a, hist_n=None):
    """Raw RVE-frame blocks with J2 at ECM points; hist_n / hist_t [N, Q, 7]."""
    G, w, ph, _ = _cluster_args(cl, np.zeros(4))
    Fr = _f64(Fr)
    N = Fr.size // 9
    a = _f64(a, (N, cl.m))
    m, Q = cl.m, cl.Q
    hn = np.zeros((N, Q, 7)) if hist_n is None else _f64(hist_n, (N, Q, 7))
    out = dict(r=np.zeros((N, m)), Pr=np.zeros((N, 9)), Kaa=np.zeros((N, m, m)),
               KaF=np.zeros((N, m, 9)), KFF=np.zeros((N, 9, 9)), hist=np.zeros((N, Q, 7)),
               status=np.zeros(N, dtype=np.int32))
    lib().orc_j2_eval(m, Q, _p(G), _p(w), _p(ph), _p(_f64(mat, (8,))), N, _p(Fr.reshape(N, 9)),
                      _p(a), _p(hn), _p(out["r"]), _p(out["Pr"]), _p(out["Kaa"]), _p(out["KaF"]),
                      _p(out["KFF"]), _p(out["hist"]), _p(out["status"]))
    return out


def j2_newton(cl, mat, Fbar, a0=None, hist_n=None, tol=1e-10, max_it=25, objective=True):
    """Micro Newton at fixed Fbar from the committed history hist_n; the
    returned 'hist' is the state of the converged evaluation (to commit)."""
    G, w, ph, _ = _cluster_args(cl, np.zeros(4))
    Fbar = _f64(Fbar)
    N = Fbar.size // 9
    a = np.zeros((N, cl.m)) if a0 is None else _f64(a0, (N, cl.m)).copy()
    hn = np.zeros((N, cl.Q, 7)) if hist_n is None else _f64(hist_n, (N, cl.Q, 7))
    o = dict(a=a, Pbar=np.zeros((N, 9)), Cbar=np.zeros((N, 9, 9)), rnorm=np.zeros(N),
             iters=np.zeros(N, dtype=np.int32), status=np.zeros(N, dtype=np.int32),
             hist=np.zeros((N, cl.Q, 7)))
    lib().orc_j2_newton(cl.m, cl.Q, _p(G), _p(w), _p(ph), _p(_f64(mat, (8,))), int(objective), N,
                        _p(Fbar.reshape(N, 9)), _p(a), _p(hn), float(tol), int(max_it),
                        _p(o["Pbar"]), _p(o["Cbar"]), _p(o["rnorm"]), _p(o["iters"]),
                        _p(o["status"]), _p(o["hist"]))
    return o


def j2_path(cl, mat, Fbar_path, tol=1e-10, max_it=25, objective=True):
    """Load path of macro states Fbar_path[K, N, 3, 3]: at each state a micro
    Newton from the previous amplitudes and the committed history, then the
    converged history is committed.  Returns the list of per-state results."""
    Fp = _f64(Fbar_path)
    K = Fp.shape[0]
    N = Fp[0].size // 9
    a, hist = np.zeros((N, cl.m)), np.zeros((N, cl.Q, 7))
    out = []
    for k in range(K):
        o = j2_newton(cl, mat, Fp[k], a0=a, hist_n=hist, tol=tol, max_it=max_it,
                      objective=objective)
        a, hist = o["a"], o["hist"]
        out.append(o)
    return out


def biot(Palg_r, Cr):
    """Biot stress T[N, 6] (Voigt 11 22 33 12 23 13) and tangent CB[N, 6, 6] =
    dT/dgamma (engineering shear) from the RVE-frame Palg_r[N, 9], Cr[N, 9, 9]."""
    Palg_r = _f64(Palg_r)
    N = Palg_r.size // 9
    Cr = _f64(Cr, (N, 81))
    T, CB = np.zeros((N, 6)), np.zeros((N, 6, 6))
    lib().orc_biot(N, _p(Palg_r.reshape(N, 9)), _p(Cr), _p(T), _p(CB))
    return T, CB


# ---------------------------------------------------------------------------
# Empirical cubature (Sec. 3.3): training matrix, SVD basis and the greedy
# point selection of Box 1.  Library primitives serve as steps: numpy's SVD
# (eq. SVDlambda) and numpy.linalg.lstsq (Box 1, step 3).  The NNLS of step 5
# is the Lawson-Hanson active-set method written out below: scipy 1.15's
# nnls returns non-optimal results on some small problems (the optimality
# conditions fail), so it cannot serve as a step.
# ---------------------------------------------------------------------------
def nnls(A, b, tol=None):
    """argmin ||A x - b|| over x >= 0 by the active-set method of Lawson and
    Hanson (Solving Least Squares Problems, 1974, ch. 23), from x = 0.

    Outer loop: the dual vector g = A^T (b - A x); stop when no inactive
    index has g_j > tol, else make the index of the largest g_j passive.
    Inner loop: z = least squares on the passive columns; if every passive
    z_j > 0 take x = z, else move x toward z until the first passive entry
    reaches zero (step alpha = min x_j / (x_j - z_j) over z_j <= 0) and make
    the entries that reached zero inactive.  An index whose own solution
    entry is not positive right after it became passive is set aside until
    x changes (the guard against cycling on rounding)."""
    A = _f64(A)
    b = _f64(b)
    n = A.shape[1]
    if tol is None:
        tol = 1e-13 * max(1.0, np.abs(A).sum(axis=0).max()) * max(1.0, np.linalg.norm(b))
    x = np.zeros(n)
    P = np.zeros(n, dtype=bool)
    blocked = np.zeros(n, dtype=bool)
    for _ in range(3 * n + 10):
        g = A.T @ (b - A @ x)
        g[P | blocked] = -np.inf
        t = int(np.argmax(g)) if n else 0
        if n == 0 or not g[t] > tol:
            return x
        P[t] = True
        first = True
        while True:
            z = np.zeros(n)
            z[P] = np.linalg.lstsq(A[:, P], b, rcond=None)[0]
            if np.all(z[P] > 0):
                x = z
                blocked[:] = False
                break
            if first and z[t] <= 0:
                P[t] = False
                blocked[t] = True
                break
            first = False
            qi = np.flatnonzero(P & (z <= 0))
            ratio = x[qi] / (x[qi] - z[qi])
            alpha = ratio.min()
            x = x + alpha * (z - x)
            hit = np.zeros(n, dtype=bool)
            hit[qi[ratio == alpha]] = True          # the entries that reached zero
            hit |= P & (x <= 0)
            x[hit] = 0.0
            P &= ~hit
            blocked[:] = False
    raise RuntimeError("nnls: no convergence")


def ecm_integrand(cl, theta, Fr, a):
    """Force integrand f[p, m + 9, M] of every snapshot at every candidate
    point: mode forces G_g^T P(F_g), then the nine components of P(F_g),
    F_g = Fr^k + G_g a^k (C routine orc_ecm_integrand)."""
    G, _, ph, th = _cluster_args(cl, theta)
    Fr = _f64(Fr)
    p = Fr.size // 9
    a = _f64(a, (p, cl.m))
    f = np.zeros((p, cl.m + 9, cl.Q))
    bad = lib().orc_ecm_integrand(cl.m, cl.Q, _p(G), _p(ph), _p(th), p, _p(Fr.reshape(p, 9)),
                                  _p(a), _p(f))
    if bad:
        raise ValueError("det F <= 0 at %d (snapshot, point) pairs" % bad)
    return f


def ecm_training_matrix(f, w):
    """Training matrix x_f (Sec. 3.3, the matrix after eq. ECM1): row (k, i),
    column g holds f^{kg}_i - f^k_i / V0, where f^k_i = sum_g w_g f^{kg}_i is
    the fully integrated value and V0 = sum_g w_g.  Returns x_f[p (m+9), M]
    and the integrals f^k_i as a vector of p (m+9)."""
    f = _f64(f)
    p, nt, M = f.shape
    w = _f64(w, (M,))
    V0 = w.sum()
    fint = f.reshape(p * nt, M) @ w
    xf = f.reshape(p * nt, M) - fint[:, None] / V0
    return xf, fint


def ecm_basis(xf, r):
    """Eq. SVDlambda: x_f^T = lambda sigma v^T.  Returns the first r columns
    of lambda (M x r, orthonormal, singular values in decreasing order) and
    all singular values."""
    U, s, _ = np.linalg.svd(_f64(xf).T, full_matrices=False)
    return np.ascontiguousarray(U[:, :r]), s


def ecm_greedy(lam, V0, mt):
    """Box 1: greedy selection of at most mt points with non-negative weights.

    J = [lambda 1]^T ((r + 1) x M), b = [0 ... 0 V0].  Readings: the residual
    of step 7 is b - J_z w (the start value r = b and the maximised positive
    correlation of step 1 fix its sign); ties of step 1 go to the lowest
    index; points that the NNLS of step 5 gives zero weight leave the
    selection for good (the excluded set); the loop also ends when no
    candidate is left.  Returns (z, w, info) with z the selected indices in
    selection order (dropped ones removed), w their weights and info a dict
    with per-iteration records: 'picked', 'nnls' (bool), 'dropped' (lists)
    and 'gap' (relative gap between the best and second best score)."""
    lam = _f64(lam)
    M, r = lam.shape
    J = np.vstack([lam.T, np.ones((1, M))])
    b = np.zeros(r + 1)
    b[-1] = V0
    jn = np.sqrt((J * J).sum(axis=0))
    avail = np.ones(M, dtype=bool)
    z, w = [], np.zeros(0)
    res = b.copy()
    info = dict(picked=[], nnls=[], dropped=[], gap=[])
    while len(z) < mt and avail.any():
        s = (J.T @ res) / jn                                   # step 1
        s[~avail] = -np.inf
        k = int(np.argmax(s))
        s2 = np.partition(s[avail], -2)[-2] if avail.sum() > 1 else -np.inf
        info["gap"].append(float((s[k] - s2) / max(abs(s[k]), 1e-300)))
        z.append(k)                                            # step 2
        avail[k] = False
        Jz = J[:, z]
        w = np.linalg.lstsq(Jz, b, rcond=None)[0]              # step 3
        used = bool((w < 0).any())                             # step 4
        drop = []
        if used:
            w = nnls(Jz, b)                                    # step 5
            keep = w > 0                                       # step 6
            drop = [z[i] for i in range(len(z)) if not keep[i]]
            z = [z[i] for i in range(len(z)) if keep[i]]
            w = w[keep]
        res = b - J[:, z] @ w                                  # step 7
        info["picked"].append(k)
        info["nnls"].append(used)
        info["dropped"].append(drop)
    return np.array(z, dtype=np.int64), w, info


# ---------------------------------------------------------------------------
# Clustered training (Sec. 3.4, Box 2) and the POD basis (Sec. 3.2.1,
# eqs. SVD_displacement and snapshots_displacement).
# ---------------------------------------------------------------------------
def kmeans(X, C0, max_iter=100):
    """Lloyd's k-means (Box 2, step 3).  X [N, d] points, C0 [k, d] initial
    centres.  Each iteration assigns every point to its nearest centre
    (squared Euclidean distance; ties to the lowest centre index), then moves
    every centre to the mean of its points (a centre without points stays).
    Stops when no assignment changes.  Returns (centres, labels, iterations)."""
    X = _f64(X)
    C = _f64(C0).copy()
    N, k = X.shape[0], C.shape[0]
    labels = np.full(N, -1, dtype=np.int64)
    for it in range(1, max_iter + 1):
        d2 = ((X[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
        new = d2.argmin(axis=1)
        changed = int((new != labels).sum())
        labels = new
        for c in range(k):
            sel = labels == c
            if sel.any():
                C[c] = X[sel].mean(axis=0)
        if changed == 0:
            return C, labels, it
    return C, labels, max_iter


def pod_split(X_el, X_inel, n_el, n_inel):
    """Eq. SVD_displacement with the elastic-inelastic split: the first n_el
    left singular vectors of the elastic snapshots X_el [nd, s_el] form
    Phi_el; the inelastic snapshots lose their part in span Phi_el
    (eq. snapshots_displacement: X_inel - Phi_el Phi_el^T X_inel) and the
    first n_inel left singular vectors of the rest form Phi_inel.
    Returns (Phi [nd, n_el + n_inel], sigma_el, sigma_inel)."""
    X_el = _f64(X_el)
    X_inel = _f64(X_inel)
    U, s_el, _ = np.linalg.svd(X_el, full_matrices=False)
    Phi_el = U[:, :n_el]
    X_mod = X_inel - Phi_el @ (Phi_el.T @ X_inel)
    V, s_in, _ = np.linalg.svd(X_mod, full_matrices=False)
    return np.hstack([Phi_el, V[:, :n_inel]]), s_el, s_in


def training_clusters(E, k, init_idx, max_iter=100):
    """Box 2, steps 2 and 3: every strain component scaled by its root mean
    square over the points (the normalisation of the strain values), Lloyd's
    k-means started from the points init_idx, the centres returned in strain
    units.  E [N, d]; returns (centres [k, d], labels, iterations)."""
    E = _f64(E)
    s = np.sqrt((E * E).mean(axis=0))
    s[s == 0.0] = 1.0
    Xn = E / s
    C, labels, it = kmeans(Xn, Xn[np.asarray(init_idx)], max_iter)
    return C * s, labels, it


def training_paths(centres, n_steps):
    """Monotonic training trajectories from the cluster centres: for centre c
    (Voigt strain xx yy zz xy yz xz, tensor shear components) and step
    j = 1 .. n_steps the RVE-frame macro input Fr = I + (j / n_steps) H(c),
    H symmetric.  Returns Fr [k n_steps, 9] (centre-major)."""
    C = _f64(centres)
    k = C.shape[0]
    out = np.zeros((k, n_steps, 3, 3))
    for c in range(k):
        H = np.array([[C[c, 0], C[c, 3], C[c, 5]],
                      [C[c, 3], C[c, 1], C[c, 4]],
                      [C[c, 5], C[c, 4], C[c, 2]]])
        for j in range(n_steps):
            out[c, j] = np.eye(3) + (j + 1) / n_steps * H
    return out.reshape(k * n_steps, 9)
