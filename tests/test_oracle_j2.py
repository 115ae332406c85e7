"""Pins of the oracle's J2 plasticity (the material of the paper's Example 1,
Sec. 5, with state at the hyper integration points, Sec. 4), CPU only.

* pure shear: the textbook closed form of linear isotropic hardening
  (elastic to tau_y = sigma_y0 / sqrt(3), then slope mu H / (3 mu + H)), in
  one step and in many committed steps (radial loading is path independent);
* elastic unloading from a plastic state along the elastic slope, with the
  plastic strain kept;
* a purely volumetric strain never yields (bulk response kappa tr eps);
* below yield the law is isotropic linear elasticity with the history kept;
* the consistent tangent equals central differences of the return map at
  fixed committed history, elastic and plastic, and is major-symmetric;
* an RVE of one plastic phase with zero-mean mode gradients has a* = 0 and
  returns the pointwise law (stress, tangent and history) along a load-unload
  path, in both frames of the macro deformation gradient;
* the condensed tangent of a two-phase RVE equals central differences of the
  Newton-converged macro stress at fixed committed history.
"""
import copy

import numpy as np
import pytest

from hrom_inputs import MAT_J2, make_cluster, make_load_path, make_macro_points

MU, LAM, SY0, HH = MAT_J2[:4]
RNG = np.random.default_rng(2468)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def shear_F(gam):
    F = np.eye(3)
    F[0, 1] = F[1, 0] = 0.5 * gam   # sym(F) - I = gam / 2 (e_xy + e_yx)
    return F


def tau_closed_form(gam):
    gy = SY0 / (np.sqrt(3.0) * MU)
    if gam <= gy:
        return MU * gam
    ep = (MU * gam - SY0 / np.sqrt(3.0)) / (2.0 * MU + 2.0 * HH / 3.0)
    return MU * gam - 2.0 * MU * ep


def test_pure_shear_closed_form_one_step_and_path(orc):
    mp = MAT_J2[:4]
    gams = np.linspace(0.0, 0.08, 41)[1:]
    # one step from the virgin state
    P, _, _ = orc.j2_law(np.array([shear_F(g) for g in gams]), mp)
    tau = np.array([tau_closed_form(g) for g in gams])
    assert rel(P[:, 1], tau) < 1e-13 and rel(P[:, 3], tau) < 1e-13
    assert np.abs(P[:, [0, 2, 4, 5, 6, 7, 8]]).max() < 1e-15
    # the same path in committed steps
    h = np.zeros((1, 7))
    for g, t in zip(gams, tau):
        P1, _, h = orc.j2_law(shear_F(g)[None], mp, h)
        assert abs(P1[0, 1] - t) < 1e-13 * max(abs(t), 1e-3)
    # the hardening slope past yield and the plastic strain at the end
    g1, g2 = 0.06, 0.07
    slope = (tau_closed_form(g2) - tau_closed_form(g1)) / (g2 - g1)
    assert abs(slope - MU * HH / (3 * MU + HH)) < 1e-12
    ep = (MU * gams[-1] - SY0 / np.sqrt(3.0)) / (2.0 * MU + 2.0 * HH / 3.0)
    assert abs(h[0, 3] - ep) < 1e-14 and abs(h[0, 6] - 2.0 / np.sqrt(3.0) * ep) < 1e-14


def test_elastic_unloading_keeps_plastic_strain(orc):
    mp = MAT_J2[:4]
    _, _, h = orc.j2_law(shear_F(0.06)[None], mp)
    t1 = tau_closed_form(0.06)
    for g in (0.055, 0.04, 0.03):
        P, A, h2 = orc.j2_law(shear_F(g)[None], mp, h)
        assert abs(P[0, 1] - (t1 - MU * (0.06 - g))) < 1e-14
        assert np.array_equal(h2, h)                       # no further plastic flow
    # tangent in the elastic range: d sigma_xy / d gamma = mu (F_xy = F_yx = gamma / 2)
    _, A, _ = orc.j2_law(shear_F(0.04)[None], mp, h)
    assert abs(0.5 * (A[0, 1, 1] + A[0, 1, 3]) - MU) < 1e-15


def test_volumetric_strain_never_yields(orc):
    mp = MAT_J2[:4]
    kappa = LAM + 2.0 * MU / 3.0
    for ev in (0.001, 0.05, 0.3):
        F = (1.0 + ev / 3.0) * np.eye(3)
        P, _, h = orc.j2_law(F[None], mp)
        assert np.abs(h).max() == 0.0
        assert abs(P[0, 0] - kappa * ev) < 1e-14 * max(1.0, kappa * ev)


def test_elastic_range_is_isotropic_elasticity(orc):
    mp = MAT_J2[:4]
    h0 = np.zeros((1, 7))
    h0[0, :6] = 1e-4 * RNG.standard_normal(6)
    h0[0, 6] = 0.02                                       # hardened: larger elastic range
    E = 1e-4 * RNG.standard_normal((3, 3))
    F = np.eye(3) + E
    P, A, h = orc.j2_law(F[None], mp, h0)
    eps = 0.5 * (E + E.T)
    epn = np.array([[h0[0, 0], h0[0, 3], h0[0, 5]], [h0[0, 3], h0[0, 1], h0[0, 4]],
                    [h0[0, 5], h0[0, 4], h0[0, 2]]])
    sig = LAM * np.trace(eps) * np.eye(3) + 2.0 * MU * (eps - epn)
    # F - I loses about four digits of E ~ 1e-4 to rounding
    assert rel(P[0], sig.ravel()) < 1e-11
    assert np.array_equal(h, h0)
    Ci = np.zeros((9, 9))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    Ci[3 * i + j, 3 * k + l] = LAM * (i == j) * (k == l) + MU * (
                        (i == k) * (j == l) + (i == l) * (j == k))
    assert rel(A[0], Ci) < 1e-14


@pytest.mark.parametrize("scale", [0.003, 0.03])
def test_tangent_equals_central_differences(orc, scale):
    """scale 0.003: elastic states; 0.03: plastic states (both from a
    committed, hardened history)."""
    mp = MAT_J2[:4]
    n = 6
    F = np.eye(3)[None] + scale * RNG.standard_normal((n, 3, 3))
    h0 = np.zeros((n, 7))
    h0[:, :3] = 1e-3 * RNG.standard_normal((n, 3))
    h0[:, :3] -= h0[:, :3].mean(axis=1, keepdims=True)    # deviatoric plastic strain
    h0[:, 6] = 0.004
    P0, A, h1 = orc.j2_law(F, mp, h0)
    plastic = np.any(h1 != h0, axis=1)
    assert plastic.all() if scale > 0.01 else not plastic.any()
    eps = 1e-7
    for J in range(9):
        dF = np.zeros((n, 9))
        dF[:, J] = eps
        Pp, _, _ = orc.j2_law(F.reshape(n, 9) + dF, mp, h0)
        Pm, _, _ = orc.j2_law(F.reshape(n, 9) - dF, mp, h0)
        fd = (Pp - Pm) / (2 * eps)
        assert rel(fd, A[:, :, J]) < 1e-7, J
    assert np.abs(A - np.transpose(A, (0, 2, 1))).max() < 1e-14 * np.abs(A).max()


@pytest.mark.parametrize("objective", [False, True])
def test_single_phase_rve_reduces_to_point_law(orc, objective):
    cl = make_cluster(6, 40, 4300)
    one = copy.copy(cl)
    one.phase = np.zeros_like(cl.phase)
    N = 4
    path = make_load_path(N, 4301, amp=0.03)
    res = orc.j2_path(one, MAT_J2, path, objective=objective)
    h = np.zeros((N, 7))
    yielded = False
    for k, o in enumerate(res):
        assert np.all(o["status"] == 0)
        assert np.abs(o["a"]).max() < 1e-14
        # point law at the RVE frame of the macro state
        Fr = orc.polar(path[k])[0] if objective else path[k].reshape(N, 9)
        P, A, h = orc.j2_law(Fr, MAT_J2[:4], h)
        yielded |= bool(np.any(h[:, 6] > 0))
        assert rel(o["hist"], np.repeat(h[:, None, :], cl.Q, axis=1)) < 1e-13
        if not objective:
            assert rel(o["Pbar"], P) < 1e-13 and rel(o["Cbar"], A) < 1e-12
    assert yielded


def test_condensed_tangent_equals_fd_of_converged_stress(orc):
    """Two phases (plastic matrix, elastic inclusions), direct frame, at a
    plastic state of a load path: Cbar = d Pbar / d Fbar at fixed committed
    history, by central differences of the Newton-converged Pbar."""
    cl = make_cluster(8, 48, 4400)
    N = 3
    path = make_load_path(N, 4401, amp=0.03, levels=(0.5, 1.0))
    res = orc.j2_path(cl, MAT_J2, path, tol=1e-14, objective=False)
    hist_n = res[0]["hist"]                                  # committed before the last state
    assert np.any(res[1]["hist"][:, :, 6] > hist_n[:, :, 6])   # the last state yields further
    o = res[1]
    eps = 1e-7
    F = path[1].reshape(N, 9)
    for J in range(9):
        dF = np.zeros((N, 9))
        dF[:, J] = eps
        Pp = orc.j2_newton(cl, MAT_J2, F + dF, a0=o["a"], hist_n=hist_n, tol=1e-14,
                           objective=False)["Pbar"]
        Pm = orc.j2_newton(cl, MAT_J2, F - dF, a0=o["a"], hist_n=hist_n, tol=1e-14,
                           objective=False)["Pbar"]
        fd = (Pp - Pm) / (2 * eps)
        assert rel(fd, o["Cbar"][:, :, J]) < 1e-6, J
