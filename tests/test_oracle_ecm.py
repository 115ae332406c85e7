"""Pins of the empirical-cubature oracle (Sec. 3.3: eq. ECM1, the training
matrix, eq. SVDlambda and the greedy of Box 1) against facts that do not come
from the oracle itself:

* the integrand is the gradient of the stored energy: its mode rows are
  d/da W(Fr + G_g a) and its stress rows dW/dF (central differences of the
  Neo-Hooke energy);
* its weighted sum is the residual r and the stress P_r of the (already
  pinned) evaluation, also for weights that do not sum to one;
* the full quadrature solves J w = b exactly for every truncation (the mean
  subtraction of the training matrix makes x_f w_full = 0);
* a rule selected from polynomial integrands on a grid integrates every
  polynomial of the training degree exactly (a square nonsingular system at
  the end of the loop);
* step 1 starts at r = b, so the first pick is the row of lambda with the
  smallest norm; the second pick follows from the residual b - J_z w and
  differs from the one the opposite sign would give;
* every NNLS result satisfies the Karush-Kuhn-Tucker conditions, and on tiny
  problems equals the best non-negative solution over all subsets;
* the selection is invariant under any rotation lambda -> lambda O (it depends
  only on the truncated subspace) and equivariant under a permutation of the
  candidates; mt = 1 picks the first candidate with weight V0.
"""
import itertools

import numpy as np
import pytest

from hrom_inputs import THETA_REF, make_cluster, make_macro_points


def _snapshots(orc, m, M, p, seed, amp=0.05):
    cl = make_cluster(m, M, seed)
    F, _, _ = make_macro_points(p, seed + 1, amp=amp)
    ref = orc.newton(cl, THETA_REF, F, tol=1e-12, objective=False)
    assert int(ref["status"].max()) == 0
    return cl, F.reshape(p, 9), ref["a"]


def test_integrand_is_energy_gradient(orc):
    cl, Fr, a = _snapshots(orc, 6, 40, 3, 8100)
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    assert f.shape == (3, 6 + 9, 40)
    h = 1e-6
    rng = np.random.default_rng(8102)
    for k, g in [(0, 0), (1, 17), (2, 39)]:
        mu, lam = THETA_REF[2 * cl.phase[g]], THETA_REF[2 * cl.phase[g] + 1]
        Gg = cl.G[g]                                    # [9, m]

        def W_of_a(av):
            return orc.neo_hooke_energy(Fr[k] + Gg @ av, mu, lam)[0]

        def W_of_F(Fv):
            return orc.neo_hooke_energy(Fv, mu, lam)[0]
        for n in range(cl.m):
            e = np.zeros(cl.m)
            e[n] = h
            fd = (W_of_a(a[k] + e) - W_of_a(a[k] - e)) / (2 * h)
            assert abs(fd - f[k, n, g]) < 1e-8 * max(1.0, abs(fd))
        Fg = Fr[k] + Gg @ a[k]
        for I in rng.permutation(9)[:5]:
            e = np.zeros(9)
            e[I] = h
            fd = (W_of_F(Fg + e) - W_of_F(Fg - e)) / (2 * h)
            assert abs(fd - f[k, cl.m + I, g]) < 1e-8 * max(1.0, abs(fd))


def test_integrand_sums_to_residual_and_stress(orc):
    cl, Fr, a = _snapshots(orc, 8, 64, 4, 8200)
    cl.w = cl.w * 3.7                                   # V0 = 3.7
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    xf, fint = orc.ecm_training_matrix(f, cl.w)
    blocks = orc.eval_blocks(cl, THETA_REF, Fr, a)      # sums w_g / V0 (.)
    V0 = cl.w.sum()
    fi = fint.reshape(4, cl.m + 9)
    assert np.allclose(fi[:, :cl.m] / V0, blocks["r"], rtol=0, atol=1e-13)
    assert np.allclose(fi[:, cl.m:] / V0, blocks["Pr"], rtol=0, atol=1e-13)
    # training matrix rows: integrand minus the integral over V0
    assert np.allclose(xf, f.reshape(4 * (cl.m + 9), -1) - fint[:, None] / V0, atol=0)


def test_full_quadrature_solves_every_truncation(orc):
    cl, Fr, a = _snapshots(orc, 8, 300, 6, 8300)
    cl.w = cl.w * 0.25
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    xf, _ = orc.ecm_training_matrix(f, cl.w)
    assert np.abs(xf @ cl.w).max() < 1e-14 * np.abs(xf).max() * 300
    lam, s = orc.ecm_basis(xf, 60)
    assert np.all(np.diff(s) <= 0)
    assert np.allclose(lam.T @ lam, np.eye(60), atol=1e-13)
    for r in (1, 10, 60):
        J = np.vstack([lam[:, :r].T, np.ones((1, 300))])
        b = np.zeros(r + 1)
        b[-1] = cl.w.sum()
        assert np.linalg.norm(J @ cl.w - b) < 1e-13


def _poly_problem(M, d, V0=2.0):
    """Monomials x^0 .. x^d on an M-point grid of [0, 1] with trapezoid
    weights scaled to V0 (the integrand rows of one snapshot)."""
    x = np.linspace(0.0, 1.0, M)
    w = np.full(M, 1.0 / (M - 1))
    w[0] = w[-1] = 0.5 / (M - 1)
    w *= V0
    f = np.stack([x ** j for j in range(d + 1)])[None]     # [1, d + 1, M]
    return x, w, f


@pytest.mark.parametrize("d", [3, 6, 9])
def test_polynomial_rule_is_exact(orc, d):
    M = 401
    x, w, f = _poly_problem(M, d)
    xf, _ = orc.ecm_training_matrix(f, w)
    lam, s = orc.ecm_basis(xf, d)          # rank d: the constant row is zero
    assert s[d] < 1e-12 * s[0]
    z, wt, info = orc.ecm_greedy(lam, w.sum(), d + 1)
    assert len(z) == d + 1 and np.all(wt > 0)
    assert len(set(z.tolist())) == d + 1
    for j in range(d + 1):
        exact = (w * x ** j).sum()
        assert abs((wt * x[z] ** j).sum() - exact) < 1e-11 * max(1.0, abs(exact))


def _random_basis(M, r, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M, r)) * np.linspace(1.0, 3.0, M)[:, None]
    q, _ = np.linalg.qr(X)
    return q


def test_first_and_second_pick(orc):
    M, r, V0 = 200, 12, 1.5
    lam = _random_basis(M, r, 8400)
    z, w, info = orc.ecm_greedy(lam, V0, 2)
    k1 = int(np.argmin((lam * lam).sum(axis=1)))
    assert info["picked"][0] == k1
    J = np.vstack([lam.T, np.ones((1, M))])
    b = np.zeros(r + 1)
    b[-1] = V0
    jn = np.sqrt((J * J).sum(axis=0))
    j1 = J[:, k1]
    w1 = (j1 @ b) / (j1 @ j1)                # one-column least squares
    res = b - j1 * w1
    s = (J.T @ res) / jn
    s[k1] = -np.inf
    assert info["picked"][1] == int(np.argmax(s))
    s_wrong = (J.T @ (-res)) / jn            # the opposite sign of step 7
    s_wrong[k1] = -np.inf
    assert int(np.argmax(s_wrong)) != info["picked"][1]


def _kkt(J, b, w, tol):
    g = J.T @ (b - J @ w)
    assert np.all(w >= 0)
    assert np.all(g[w == 0] <= tol)
    assert np.all(np.abs(g[w > 0]) <= tol)


def test_nnls_steps_satisfy_kkt(orc):
    cl, Fr, a = _snapshots(orc, 12, 1024, 8, 8500)
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    xf, _ = orc.ecm_training_matrix(f, cl.w)
    mt = 96
    lam, _ = orc.ecm_basis(xf, mt - 1)
    V0 = cl.w.sum()
    M, r = lam.shape
    J = np.vstack([lam.T, np.ones((1, M))])
    b = np.zeros(r + 1)
    b[-1] = V0
    z, w, info = orc.ecm_greedy(lam, V0, mt)
    assert sum(info["nnls"]) >= 10, "the case must exercise the NNLS fallback"
    # replay the selection and check every NNLS step
    sel = []
    for k, used, drop in zip(info["picked"], info["nnls"], info["dropped"]):
        sel.append(k)
        if used:
            Jz = J[:, sel]
            assert np.linalg.lstsq(Jz, b, rcond=None)[0].min() < 0
            wn = orc.nnls(Jz, b)
            _kkt(Jz, b, wn, 1e-12)
            assert sorted(drop) == sorted(sel[i] for i in range(len(sel)) if wn[i] == 0)
            sel = [sel[i] for i in range(len(sel)) if wn[i] > 0]
    assert sel == z.tolist()
    assert len(z) == mt
    assert np.linalg.norm(J[:, z] @ w - b) < 1e-12


def test_nnls_equals_brute_force_on_tiny_problems(orc):
    """The oracle's NNLS: on problems whose unconstrained solution has a
    negative entry, its result is the best non-negative solution over all
    subsets of the columns (each subset solved by least squares).  scipy
    1.15's nnls fails this on the ninth problem of this seed."""
    rng = np.random.default_rng(8550)
    done = 0
    while done < 60:
        rows, n = int(rng.integers(4, 9)), int(rng.integers(2, 7))
        n = min(n, rows)
        A = rng.standard_normal((rows, n))
        bb = rng.standard_normal(rows)
        if np.linalg.lstsq(A, bb, rcond=None)[0].min() >= 0:
            continue
        wn = orc.nnls(A, bb)
        _kkt(A, bb, wn, 1e-12)
        best = np.linalg.norm(bb)                   # the empty subset
        for size in range(1, n + 1):
            for S in itertools.combinations(range(n), size):
                ws = np.linalg.lstsq(A[:, S], bb, rcond=None)[0]
                if np.all(ws >= 0):
                    best = min(best, np.linalg.norm(A[:, S] @ ws - bb))
        assert abs(np.linalg.norm(A @ wn - bb) - best) < 1e-12
        done += 1


def test_rotation_invariance_and_permutation(orc):
    M, r, V0 = 250, 14, 1.0
    lam = _random_basis(M, r, 8600)
    z, w, info = orc.ecm_greedy(lam, V0, r + 1)
    assert min(info["gap"]) > 1e-8
    O, _ = np.linalg.qr(np.random.default_rng(8601).standard_normal((r, r)))
    z2, w2, _ = orc.ecm_greedy(lam @ O, V0, r + 1)
    assert z2.tolist() == z.tolist()
    assert np.allclose(w2, w, rtol=1e-10, atol=0)
    perm = np.random.default_rng(8602).permutation(M)
    z3, w3, _ = orc.ecm_greedy(lam[perm], V0, r + 1)
    inv = np.argsort(perm)
    assert [int(perm[i]) for i in z3] == z.tolist()
    assert np.allclose(w3, w, rtol=1e-10, atol=0)
    assert inv[perm[0]] == 0


def test_single_point_rule(orc):
    lam = np.zeros((7, 0))
    z, w, _ = orc.ecm_greedy(lam, 2.5, 1)
    assert z.tolist() == [0] and np.allclose(w, [2.5])


def test_pipeline_on_neo_hooke_snapshots(orc):
    cl, Fr, a = _snapshots(orc, 8, 512, 6, 8700)
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    xf, fint = orc.ecm_training_matrix(f, cl.w)
    mt = 48
    lam, s = orc.ecm_basis(xf, mt - 1)
    z, w, info = orc.ecm_greedy(lam, cl.w.sum(), mt)
    assert len(z) == mt and np.all(w > 0)
    assert abs(w.sum() - cl.w.sum()) < 1e-13
    # the selected rule integrates the training forces to the truncation level:
    # ||x_f w|| is bounded by the discarded singular values times ||w||
    err = np.linalg.norm(xf[:, z] @ w)
    assert err <= s[mt - 1] * np.linalg.norm(w) * 1.0001
