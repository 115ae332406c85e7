"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is a closed form,
an invariant, a central finite difference of a different oracle output, a
brute-force equality, or a special case that reduces to a textbook formula.
Each test names the passage it follows.
"""
import copy

import numpy as np
import pytest

from hrom_inputs import (THETA_REF, make_cluster, make_increments, make_macro_points,
                         perturbed_theta, zipf_counts)

RNG = np.random.default_rng(12345)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def rotate_stress(Qr, P):
    return Qr @ P


def rotate_tangent(Qr, C):
    # C_{ijkl} -> Q_ip Q_kr C_{pjrl}
    C4 = C.reshape(3, 3, 3, 3)
    return np.einsum("ip,kr,pjrl->ijkl", Qr, Qr, C4).reshape(9, 9)


@pytest.fixture(scope="module")
def small():
    cl = make_cluster(8, 32, 1000)
    F, R, H = make_macro_points(16, 1001)
    return cl, F, R, H


# ---------------------------------------------------------------- generators
def test_generator_weights_and_zero_mean():
    """ECM weights sum to the RVE measure V0 = 1 (Sec. 3.3, volume exactness);
    mode gradients have zero weighted mean (zero-mean fluctuations, Sec. 2)."""
    for (m, Q, s) in [(8, 32, 1), (64, 512, 2), (96, 576, 3)]:
        cl = make_cluster(m, Q, s)
        assert abs(cl.w.sum() - 1.0) < 1e-14
        assert np.all(cl.w > 0)
        mean = np.tensordot(cl.w, cl.G, axes=(0, 0))
        assert np.abs(mean).max() < 1e-16 * Q
        assert 0.15 < cl.phase.mean() < 0.45
        assert cl.G.shape == (Q, 9, m)


def test_zipf_split():
    c = zipf_counts(262144, 8, 1.1)
    assert sum(c) == 262144
    assert c == sorted(c, reverse=True)
    p = np.array([(k + 1) ** -1.1 for k in range(8)])
    assert np.abs(np.array(c) / 262144 - p / p.sum()).max() < 1e-5


# ---------------------------------------------------------------- Neo-Hooke
def test_neo_hooke_closed_form_uniaxial(orc):
    """Uniaxial stretch F = diag(s,1,1): P11 = mu (s - 1/s) + lam ln(s)/s,
    P22 = P33 = lam ln s, shear components zero.  P(I) = 0."""
    mu, lam = 1.3, 2.1
    for s in [0.7, 1.0, 1.25, 2.0]:
        F = np.diag([s, 1.0, 1.0])
        P, _ = orc.neo_hooke(F, mu, lam)
        P = P.reshape(3, 3)
        ref = np.diag([mu * (s - 1 / s) + lam * np.log(s) / s, lam * np.log(s), lam * np.log(s)])
        assert np.abs(P - ref).max() < 1e-14


def test_neo_hooke_stress_is_energy_derivative(orc):
    """P = dW/dF for W = mu/2 (I1 - 3) - mu ln J + lam/2 (ln J)^2 (central FD)."""
    mu, lam = 10.0, 15.0
    F = np.eye(3) + 0.2 * RNG.standard_normal((3, 3))
    P, _ = orc.neo_hooke(F, mu, lam)
    h = 1e-6
    fd = np.zeros(9)
    for k in range(9):
        E = np.zeros(9)
        E[k] = h
        fd[k] = (orc.neo_hooke_energy(F.ravel() + E, mu, lam)[0]
                 - orc.neo_hooke_energy(F.ravel() - E, mu, lam)[0]) / (2 * h)
    assert rel(P[0], fd) < 1e-8


def test_neo_hooke_tangent_fd_and_symmetry(orc):
    """A = dP/dF by central FD; A major-symmetric (hyperelastic)."""
    mu, lam = 1.0, 1.5
    F = np.eye(3) + 0.3 * RNG.standard_normal((3, 3))
    if np.linalg.det(F) <= 0:
        F[0] *= -1
    _, A = orc.neo_hooke(F, mu, lam)
    A = A[0]
    h = 1e-6
    fd = np.zeros((9, 9))
    for k in range(9):
        E = np.zeros(9)
        E[k] = h
        Pp, _ = orc.neo_hooke(F.ravel() + E, mu, lam)
        Pm, _ = orc.neo_hooke(F.ravel() - E, mu, lam)
        fd[:, k] = (Pp[0] - Pm[0]) / (2 * h)
    assert rel(A, fd) < 1e-8
    assert np.abs(A - A.T).max() < 1e-13


def test_neo_hooke_small_strain_limit(orc):
    """At F = I the tangent is isotropic linear elasticity
    mu (d_ik d_jl + d_il d_jk) + lam d_ij d_kl."""
    mu, lam = 10.0, 15.0
    _, A = orc.neo_hooke(np.eye(3), mu, lam)
    d = np.eye(3)
    ref = (mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d))
           + lam * np.einsum("ij,kl->ijkl", d, d))
    assert np.abs(A[0] - ref.reshape(9, 9)).max() < 1e-14


def test_theta_linearity(orc):
    """At fixed F, P is linear in (mu, lam): dP/dmu = F - F^-T, dP/dlam = lnJ F^-T."""
    F = np.eye(3) + 0.2 * RNG.standard_normal((3, 3))
    P1, _ = orc.neo_hooke(F, 1.0, 0.0)
    P2, _ = orc.neo_hooke(F, 0.0, 1.0)
    P3, _ = orc.neo_hooke(F, 2.5, 3.5)
    assert np.abs(2.5 * P1 + 3.5 * P2 - P3).max() < 1e-13
    Fi = np.linalg.inv(F)
    assert np.abs(P1[0] - (F - Fi.T).ravel()).max() < 1e-13
    assert np.abs(P2[0] - (np.log(np.linalg.det(F)) * Fi.T).ravel()).max() < 1e-13


# ---------------------------------------------------------------- polar split
def test_polar_recovers_generator(orc):
    """Fbar = R (I + H), H symmetric and small: the polar split (Sec. 3.2.2)
    must return U = I + H and the generator's R."""
    F, R, H = make_macro_points(64, 77, amp=0.2)
    U, Rr, V, u = orc.polar(F)
    assert np.abs(U - (np.eye(3) + H)).max() < 1e-13
    assert np.abs(Rr - R).max() < 1e-13
    assert np.abs(np.einsum("nji,njk->nik", Rr, Rr) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(Rr) - 1).max() < 1e-13


def test_stretch_increment(orc):
    """For dF = R dH (dH symmetric) the linearised stretch increment is dH
    exactly; in general it matches the FD of the polar stretch."""
    F, R, H = make_macro_points(8, 78, amp=0.1)
    dH = 0.01 * RNG.standard_normal((8, 3, 3))
    dH = dH + dH.transpose(0, 2, 1)
    dU = orc.stretch_increment(F, R @ dH)
    assert np.abs(dU - dH).max() < 1e-14
    dF = RNG.standard_normal((8, 3, 3))
    h = 1e-6
    Up = orc.polar(F + h * dF)[0]
    Um = orc.polar(F - h * dF)[0]
    assert rel(orc.stretch_increment(F, dF), (Up - Um) / (2 * h)) < 1e-8


# ---------------------------------------------------------------- evaluation blocks
def test_eval_zero_state(orc, small):
    """F_r = I and a = 0: every ECM point is undeformed, so r = 0 and P = 0 exactly."""
    cl, _, _, _ = small
    o = orc.eval_blocks(cl, THETA_REF, np.eye(3)[None], np.zeros((1, cl.m)))
    assert np.all(o["r"] == 0.0) and np.all(o["Pr"] == 0.0)
    assert o["status"][0] == 0


def _fd_blocks(orc, cl, Fr, a, h=1e-6):
    m = cl.m
    dr_da = np.zeros((m, m))
    dP_da = np.zeros((9, m))
    for k in range(m):
        e = np.zeros(m)
        e[k] = h
        op = orc.eval_blocks(cl, THETA_REF, Fr, a + e)
        om = orc.eval_blocks(cl, THETA_REF, Fr, a - e)
        dr_da[:, k] = (op["r"][0] - om["r"][0]) / (2 * h)
        dP_da[:, k] = (op["Pr"][0] - om["Pr"][0]) / (2 * h)
    dr_dF = np.zeros((m, 9))
    dP_dF = np.zeros((9, 9))
    for k in range(9):
        e = np.zeros(9)
        e[k] = h
        op = orc.eval_blocks(cl, THETA_REF, Fr.ravel() + e, a)
        om = orc.eval_blocks(cl, THETA_REF, Fr.ravel() - e, a)
        dr_dF[:, k] = (op["r"][0] - om["r"][0]) / (2 * h)
        dP_dF[:, k] = (op["Pr"][0] - om["Pr"][0]) / (2 * h)
    return dr_da, dr_dF, dP_da, dP_dF


def test_eval_blocks_are_derivatives(orc, small):
    """Kaa = dr/da (eq. ROMstiffness), KaF = dr/dF_r, KFa = dP/da, KFF = dP/dF_r
    at fixed a, all by central FD; Kaa = Kaa^T, KFa = KaF^T, KFF major-symmetric."""
    cl, F, _, _ = small
    U = orc.polar(F[:1])[0][0]
    a = 0.05 * RNG.standard_normal(cl.m)
    o = orc.eval_blocks(cl, THETA_REF, U, a)
    Kaa, KaF, KFF = o["Kaa"][0], o["KaF"][0], o["KFF"][0]
    dr_da, dr_dF, dP_da, dP_dF = _fd_blocks(orc, cl, U, a)
    assert rel(Kaa, dr_da) < 1e-8
    assert rel(KaF, dr_dF) < 1e-8
    assert rel(KaF.T, dP_da) < 1e-8
    assert rel(KFF, dP_dF) < 1e-8
    assert np.abs(Kaa - Kaa.T).max() < 1e-14 * np.abs(Kaa).max()
    assert np.abs(KFF - KFF.T).max() < 1e-14 * np.abs(KFF).max()


def _rve_energy(orc, cl, Fr, a, theta=THETA_REF):
    """sum_q w_q W(F_q): the RVE energy on the reference domain (Sec. 3.3)."""
    Fq = Fr.reshape(1, 9) + np.einsum("qim,m->qi", cl.G, a)
    Wq = np.zeros(cl.Q)
    for p in (0, 1):
        sel = cl.phase == p
        Wq[sel] = orc.neo_hooke_energy(Fq[sel], theta[2 * p], theta[2 * p + 1])
    return float(cl.w @ Wq)


def test_residual_and_stress_are_energy_gradients(orc, small):
    """Galerkin residual r = dW/da (eq. ROMintforce) and homogenised stress
    P_r = dW/dF_r (eq. homogenization_Stress) of the RVE energy, by central FD."""
    cl, F, _, _ = small
    U = orc.polar(F[1:2])[0][0]
    a = 0.05 * RNG.standard_normal(cl.m)
    o = orc.eval_blocks(cl, THETA_REF, U, a)
    h = 1e-6
    fr = np.array([(_rve_energy(orc, cl, U, a + h * e) - _rve_energy(orc, cl, U, a - h * e))
                   / (2 * h) for e in np.eye(cl.m)])
    fp = np.array([(_rve_energy(orc, cl, U.ravel() + h * e, a)
                    - _rve_energy(orc, cl, U.ravel() - h * e, a)) / (2 * h) for e in np.eye(9)])
    assert rel(o["r"][0], fr) < 1e-7
    assert rel(o["Pr"][0], fp) < 1e-7


def test_hyper_equals_full_integration_with_zero_weights(orc):
    """ECM sum over a subset z~ of the full points (Sec. 3.3) equals, bitwise,
    the full-integration sum with the weights outside z~ set to zero."""
    full = make_cluster(6, 40, 31)
    sub_idx = np.sort(RNG.choice(40, size=12, replace=False))
    w_hyper = np.zeros(40)
    w_hyper[sub_idx] = RNG.uniform(0.5, 1.5, 12)
    w_hyper /= w_hyper.sum()
    zero_w = copy.copy(full)
    zero_w.w = w_hyper
    hyper = copy.copy(full)
    hyper.Q = 12
    hyper.G = np.ascontiguousarray(full.G[sub_idx])
    hyper.w = np.ascontiguousarray(w_hyper[sub_idx])
    hyper.phase = np.ascontiguousarray(full.phase[sub_idx])
    F, _, _ = make_macro_points(4, 32)
    a = 0.05 * RNG.standard_normal((4, 6))
    o1 = orc.eval_blocks(zero_w, THETA_REF, F, a)
    o2 = orc.eval_blocks(hyper, THETA_REF, F, a)
    for k in ("r", "Pr", "Kaa", "KaF", "KFF"):
        assert np.array_equal(o1[k], o2[k]), k


def test_ecm_sums_invariant_to_point_order_and_weight_measure(orc):
    """The ECM sums are sums over an unordered set of points (Sec. 3.3):
    permuting the points (with their weights, gradients and phases) changes
    the blocks only by rounding; and they are averages over the RVE (Sec. 2):
    weights that add up to another measure V0 = 2.5 give the same blocks, and
    the same condensed stress and tangent."""
    cl = make_cluster(6, 40, 33)
    F, _, _ = make_macro_points(4, 34)
    a = 0.05 * RNG.standard_normal((4, 6))
    o = orc.eval_blocks(cl, THETA_REF, F, a)
    perm = RNG.permutation(40)
    pc = copy.copy(cl)
    pc.G = np.ascontiguousarray(cl.G[perm])
    pc.w = np.ascontiguousarray(cl.w[perm])
    pc.phase = np.ascontiguousarray(cl.phase[perm])
    op = orc.eval_blocks(pc, THETA_REF, F, a)
    for k in ("r", "Pr", "Kaa", "KaF", "KFF"):
        assert rel(op[k], o[k]) < 1e-14, k
    # a permutation that is not the identity does change the summation order
    assert any(not np.array_equal(op[k], o[k]) for k in ("r", "Kaa"))
    sc = copy.copy(cl)
    sc.w = 2.5 * cl.w
    os_ = orc.eval_blocks(sc, THETA_REF, F, a)
    for k in ("r", "Pr", "Kaa", "KaF", "KFF"):
        assert rel(os_[k], o[k]) < 1e-15, k
    n1 = orc.newton(cl, THETA_REF, F)
    n2 = orc.newton(sc, THETA_REF, F)
    assert rel(n2["Pbar"], n1["Pbar"]) < 1e-14 and rel(n2["Cbar"], n1["Cbar"]) < 1e-14


# ---------------------------------------------------------------- condensation + Newton
def test_single_phase_reduces_to_neo_hooke(orc, small):
    """A single-phase RVE with zero-mean mode gradients has a* = 0 and returns
    the pointwise law: Pbar = P_NH(Fbar), Cbar = A_NH(Fbar), in both frames."""
    cl, F, _, _ = small
    one = copy.copy(cl)
    one.phase = np.zeros_like(cl.phase)
    P, A = orc.neo_hooke(F, THETA_REF[0], THETA_REF[1])
    for objective in (True, False):
        o = orc.newton(one, THETA_REF, F, objective=objective)
        assert np.abs(o["a"]).max() < 1e-15
        assert rel(o["Pbar"], P) < 1e-13
        assert rel(o["Cbar"], A) < 1e-13


def test_objectivity(orc, small):
    """P(Q F) = Q P(F) and C(Q F)_ijkl = Q_ip Q_kr C(F)_pjrl: the RVE sees
    only the stretch (Sec. 3.2.2)."""
    cl, F, R, _ = small
    o = orc.newton(cl, THETA_REF, F)
    Qr = make_macro_points(1, 99, amp=0.0, max_angle=2.5)[1][0]
    o2 = orc.newton(cl, THETA_REF, Qr[None] @ F)
    for b in range(F.shape[0]):
        assert rel(o2["Pbar"][b].reshape(3, 3), rotate_stress(Qr, o["Pbar"][b].reshape(3, 3))) < 1e-12
        assert rel(o2["Cbar"][b], rotate_tangent(Qr, o["Cbar"][b])) < 1e-12


def test_condensed_tangent_major_symmetric_and_schur_psd(orc, small):
    """Cbar is the Hessian of the macro energy, hence major-symmetric; the
    Schur complement KFF - Cr is positive semi-definite (SPD Kaa)."""
    cl, F, _, _ = small
    o = orc.newton(cl, THETA_REF, F)
    C = o["Cbar"]
    assert np.abs(C - C.transpose(0, 2, 1)).max() < 1e-12 * np.abs(C).max()
    pe = orc.point_eval(cl, THETA_REF, F, o["a"])
    blocks = orc.eval_blocks(cl, THETA_REF, orc.polar(F)[0], o["a"])
    for b in range(F.shape[0]):
        D = blocks["KFF"][b] - pe["Cr"][b]
        ev = np.linalg.eigvalsh(0.5 * (D + D.T))
        assert ev.min() > -1e-12 * np.abs(ev).max()


@pytest.mark.parametrize("objective", [True, False])
def test_condensed_tangent_is_derivative_of_converged_stress(orc, small, objective):
    """Cbar = dPbar/dFbar through the converged ROM state (eq. Biot_Tangent),
    by central FD of the Newton-converged stress."""
    cl, F, _, _ = small
    h = 1e-6
    for b in range(2):
        o = orc.newton(cl, THETA_REF, F[b:b + 1], tol=1e-14, objective=objective)
        fd = np.zeros((9, 9))
        for k in range(9):
            e = np.zeros(9)
            e[k] = h
            op = orc.newton(cl, THETA_REF, F[b].ravel() + e, tol=1e-14, objective=objective)
            om = orc.newton(cl, THETA_REF, F[b].ravel() - e, tol=1e-14, objective=objective)
            fd[:, k] = (op["Pbar"][0] - om["Pbar"][0]) / (2 * h)
        assert rel(o["Cbar"][0], fd) < 1e-8


def test_newton_quadratic_convergence(orc, small):
    """Exact tangent Kaa => quadratic convergence ||r_{k+1}|| <= c ||r_k||^2."""
    cl, F, _, _ = small
    a = np.zeros((F.shape[0], cl.m))
    norms = []
    for _ in range(4):
        pe = orc.point_eval(cl, THETA_REF, F, a)
        norms.append(pe["rnorm"].copy())
        a = a - pe["y"]
    norms = np.array(norms)
    assert (norms[1] / norms[0] ** 2).max() < 10.0
    assert (norms[2] / norms[1] ** 2).max() < 10.0
    assert norms[3].max() < 1e-14


def test_algorithmic_stress_matches_converged_stress(orc, small):
    """P_alg = P - KFa Kaa^{-1} r predicts the converged stress to O(|r|^2)."""
    cl, F, _, _ = small
    a0 = np.zeros((F.shape[0], cl.m))
    pe = orc.point_eval(cl, THETA_REF, F, a0)
    conv = orc.newton(cl, THETA_REF, F, tol=1e-14)
    err_alg = np.abs(pe["Pbar"] - conv["Pbar"]).max()
    r0 = pe["rnorm"].max()
    assert err_alg < 50 * r0 ** 2


def test_monolithic_update_first_order(orc, small):
    """a_{k+1} = a_k - Kaa^{-1}(r + KaF dU) (Sec. 3.2.3) predicts the converged
    a*(Fbar + dFbar) to second order in |dFbar|."""
    cl, F, R, _ = small
    base = orc.newton(cl, THETA_REF, F[:4], tol=1e-14)
    dH = RNG.standard_normal((4, 3, 3))
    dH = dH + dH.transpose(0, 2, 1)
    errs = []
    for s in (1e-2, 5e-3):
        dF = (R[:4] @ (s * dH))[None]
        mono = orc.monolithic(cl, THETA_REF, F[:4], dF, a0=base["a"])
        target = orc.newton(cl, THETA_REF, F[:4] + dF[0], a0=base["a"], tol=1e-14)
        errs.append(np.abs(mono["a"] - target["a"]).max())
    assert 3.0 < errs[0] / errs[1] < 5.0


# ---------------------------------------------------------------- adjoint
def _loss(orc, cl, theta, F, target, objective=True):
    o = orc.newton(cl, theta, F, tol=1e-14, objective=objective)
    return float(((o["Pbar"] - target) ** 2).sum()), o


@pytest.mark.parametrize("objective", [True, False])
def test_adjoint_matches_finite_differences(orc, small, objective):
    """dL/dtheta and dL/dFbar of L = sum ||Pbar - Pbar*||^2 through the
    converged micro state, vs central FD with h = 1e-6."""
    cl, F, _, _ = small
    F = F[:3]
    th_star, _ = perturbed_theta(5)
    target = orc.newton(cl, th_star, F, tol=1e-14, objective=objective)["Pbar"]
    L0, o = _loss(orc, cl, THETA_REF, F, target, objective)
    g = 2.0 * (o["Pbar"] - target)
    bw = orc.backward(cl, THETA_REF, F, o["a"], g, objective=objective)
    h = 1e-6
    fd_th = np.zeros(4)
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        fd_th[k] = (_loss(orc, cl, THETA_REF + e, F, target, objective)[0]
                    - _loss(orc, cl, THETA_REF - e, F, target, objective)[0]) / (2 * h)
    assert rel(bw["gtheta"], fd_th) < 1e-6
    fd_F = np.zeros((3, 9))
    for b in range(3):
        for k in range(9):
            Fp = F.reshape(3, 9).copy()
            Fm = Fp.copy()
            Fp[b, k] += h
            Fm[b, k] -= h
            fd_F[b, k] = (_loss(orc, cl, THETA_REF, Fp, target, objective)[0]
                          - _loss(orc, cl, THETA_REF, Fm, target, objective)[0]) / (2 * h)
    assert rel(bw["gF"], fd_F) < 1e-6
    # dL/dFbar = Cbar^T g (the adjoint is the transpose of the tangent)
    assert rel(bw["gF"], np.einsum("nij,ni->nj", o["Cbar"], g)) < 1e-12


# ---------------------------------------------------------------- status flags
def test_status_flags(orc, small):
    cl, F, _, _ = small
    o = orc.newton(cl, THETA_REF, np.diag([-1.0, 1.0, 1.0])[None])
    assert o["status"][0] & orc.PT_JNONPOS
    Fn = F[:1].copy()
    Fn[0, 0, 0] = np.nan
    assert orc.newton(cl, THETA_REF, Fn)["status"][0] & orc.PT_NONFINITE
    o = orc.newton(cl, THETA_REF, F[:2], tol=1e-30, max_it=1)
    assert np.all(o["status"] & orc.PT_NOCONV)
    bad = copy.copy(cl)
    th = THETA_REF.copy()
    th[0] = th[2] = -1.0
    o = orc.point_eval(bad, th, F[:2], np.zeros((2, cl.m)))
    assert np.all(o["status"] & orc.PT_NOT_SPD)
    # the LU fallback still solves Kaa y = r
    blocks = orc.eval_blocks(bad, th, orc.polar(F[:2])[0], np.zeros((2, cl.m)))
    for b in range(2):
        res = blocks["Kaa"][b] @ o["y"][b] - blocks["r"][b]
        assert np.abs(res).max() < 1e-12 * max(np.abs(blocks["r"][b]).max(), 1e-300)


# ---------------------------------------------------------------- Updated-Lagrangian output
def _homogeneous_rve_frame(orc, F, mu, lam):
    """RVE-frame inputs of a homogeneous Neo-Hooke point: Palg_r = P(Ubar),
    Cr = A(Ubar) (no fluctuation modes)."""
    U, _, _, _ = orc.polar(F)
    P, A = orc.neo_hooke(U.reshape(-1, 3, 3), mu, lam)
    return P, A


def test_cauchy_equals_neo_hooke_cauchy_stress(orc):
    """Homogeneous states, rotation included: the Cauchy stress obtained from
    the Biot stress by eq. (biotstress) equals the textbook Neo-Hooke Cauchy
    stress sigma = mu/J (F F^T - I) + lam ln J / J I."""
    mu, lam = 10.0, 15.0
    F, _, _ = make_macro_points(16, 8100, amp=0.2, max_angle=1.2)
    Pa, Cr = _homogeneous_rve_frame(orc, F, mu, lam)
    sig, dsdD, st = orc.cauchy(F, Pa, Cr)
    assert not st.any()
    for b in range(16):
        J = np.linalg.det(F[b])
        ref = mu / J * (F[b] @ F[b].T - np.eye(3)) + lam * np.log(J) / J * np.eye(3)
        assert np.abs(sig[b].reshape(3, 3) - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
        # sigma symmetric, so is every column of the tangent
        assert np.abs(dsdD[b].reshape(3, 3, 9) - dsdD[b].reshape(3, 3, 9).transpose(1, 0, 2)).max() < 1e-12


def test_cauchy_tangent_is_lame_at_identity(orc):
    """At F = I (R = U = I, J = 1, sigma = 0) the Updated-Lagrangian tangent
    of App. A reduces to isotropic linear elasticity."""
    mu, lam = 10.0, 15.0
    F = np.eye(3)[None]
    Pa, Cr = _homogeneous_rve_frame(orc, F, mu, lam)
    sig, dsdD, _ = orc.cauchy(F, Pa, Cr)
    d = np.eye(3)
    ref = (mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d))
           + lam * np.einsum("ij,kl->ijkl", d, d))
    assert np.abs(sig).max() < 1e-14
    assert np.abs(dsdD[0] - ref.reshape(9, 9)).max() < 1e-13


def test_cauchy_tangent_pure_dilation(orc):
    """F = s I: the Biot map is T = s^2 sigma, the stretch rate is Udot = s D
    and C^B = sym A(sI) sym with A = mu d_ik d_jl + (mu - lam ln J)/s^2
    d_il d_jk + lam/s^2 d_ij d_kl, so dsigma/dD = C^B / s (derived by hand
    from the appendix's product rule)."""
    mu, lam = 1.3, 2.2
    d = np.eye(3)
    Isym = 0.5 * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d))
    for s in [0.8, 1.1, 1.5]:
        F = s * np.eye(3)[None]
        Pa, Cr = _homogeneous_rve_frame(orc, F, mu, lam)
        sig, dsdD, _ = orc.cauchy(F, Pa, Cr)
        ell = np.log(s ** 3)
        CB = (mu + (mu - lam * ell) / s ** 2) * Isym + lam / s ** 2 * np.einsum("ij,kl->ijkl", d, d)
        assert np.abs(dsdD[0] - (CB / s).reshape(9, 9)).max() < 1e-13


def test_cauchy_rotation_covariance(orc):
    """A superposed rotation Q leaves the RVE-frame state unchanged and
    rotates the outputs: sigma(Q F) = Q sigma Q^T and the tangent transforms
    as a fourth-order tensor.  Random RVE-frame states (not homogeneous)."""
    rng = np.random.default_rng(8200)
    F, _, _ = make_macro_points(8, 8201, amp=0.15, max_angle=0.8)
    Pa = rng.standard_normal((8, 9))
    Cr = rng.standard_normal((8, 9, 9))
    Cr = Cr + Cr.transpose(0, 2, 1)
    Q = make_macro_points(8, 8202, amp=0.0, max_angle=2.0)[1]
    s1, c1, _ = orc.cauchy(F, Pa, Cr)
    s2, c2, _ = orc.cauchy(Q @ F, Pa, Cr)
    for b in range(8):
        q = Q[b]
        assert np.abs(s2[b].reshape(3, 3) - q @ s1[b].reshape(3, 3) @ q.T).max() < 1e-12
        rot = np.einsum("ia,jb,kc,ld,abcd->ijkl", q, q, q, q, c1[b].reshape(3, 3, 3, 3))
        assert np.abs(c2[b].reshape(3, 3, 3, 3) - rot).max() < 1e-11 * max(1.0, np.abs(rot).max())


# ---------------------------------------------------------------- Biot form
def _stretch_from_gamma(g):
    """Symmetric stretch from Voigt coordinates with engineering shear."""
    U = np.diag(g[:3]).astype(float)
    for k, (i, j) in zip(range(3, 6), ((0, 1), (1, 2), (0, 2))):
        U[i, j] = U[j, i] = 0.5 * g[k]
    return U


def test_biot_form_conjugacy_fd_and_symmetry(orc, small):
    """T (Voigt) and CB from the condensed RVE-frame state: T . dgamma equals
    sym(Palg) : dU for a symmetric stretch increment; CB equals central
    differences of the Newton-converged T in the engineering strains (direct
    frame, Fbar = U symmetric); CB is symmetric."""
    cl, _, _, H = small
    n = 3
    g0 = np.stack([np.r_[1 + H[b][0, 0], 1 + H[b][1, 1], 1 + H[b][2, 2],
                         2 * H[b][0, 1], 2 * H[b][1, 2], 2 * H[b][0, 2]] for b in range(n)])
    U0 = np.array([_stretch_from_gamma(g) for g in g0])
    o = orc.newton(cl, THETA_REF, U0, objective=False, tol=1e-14)
    T, CB = orc.biot(o["Pbar"], o["Cbar"])
    # conjugacy
    dg = RNG.standard_normal((n, 6))
    for b in range(n):
        dU = _stretch_from_gamma(dg[b])
        Ts = 0.5 * (o["Pbar"][b].reshape(3, 3) + o["Pbar"][b].reshape(3, 3).T)
        assert abs(T[b] @ dg[b] - np.sum(Ts * dU)) < 1e-14 * max(1.0, np.abs(T[b]).max())
    # finite differences of T in gamma
    h = 1e-6
    for l in range(6):
        e = np.zeros(6)
        e[l] = h
        Up = np.array([_stretch_from_gamma(g + e) for g in g0])
        Um = np.array([_stretch_from_gamma(g - e) for g in g0])
        Tp, _ = orc.biot(orc.newton(cl, THETA_REF, Up, objective=False, tol=1e-14)["Pbar"],
                         np.zeros((n, 81)))
        Tm, _ = orc.biot(orc.newton(cl, THETA_REF, Um, objective=False, tol=1e-14)["Pbar"],
                         np.zeros((n, 81)))
        assert rel((Tp - Tm) / (2 * h), CB[:, :, l]) < 1e-8, l
    assert np.abs(CB - np.transpose(CB, (0, 2, 1))).max() < 1e-12 * np.abs(CB).max()


def test_biot_form_single_phase_is_voigt_neo_hooke(orc, small):
    """One phase: CB is the Voigt matrix D_k : A_NH(U) : D_l of the pointwise
    Neo-Hooke tangent; at U = I it is the isotropic Lame matrix."""
    cl, _, _, H = small
    one = copy.copy(cl)
    one.phase = np.zeros_like(cl.phase)
    mu, lam = THETA_REF[:2]
    o = orc.newton(one, THETA_REF, np.eye(3)[None], objective=False)
    _, CB = orc.biot(o["Pbar"], o["Cbar"])
    C0 = lam * np.ones((3, 3)) + 2 * mu * np.eye(3)
    ref = np.zeros((6, 6))
    ref[:3, :3] = C0
    ref[3:, 3:] = mu * np.eye(3)
    assert np.abs(CB[0] - ref).max() < 1e-13
