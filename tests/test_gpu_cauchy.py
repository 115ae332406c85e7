"""GPU parity of the Updated-Lagrangian output (Cauchy stress and the App. A
tangent dsigma/dD) against the oracle.

The GPU inverts the Biot relation by a Lyapunov solve in the eigenbasis of
Ubar; the oracle LU-factorises the 9 x 9 Biot map.  Both start from the
condensed RVE-frame state of the same (Fbar, a).  Bars: 1e-12 relative per
point (FP64 path), 1e-5 (mixed BF16 / FP16 paths, hi/lo split).
"""
import numpy as np
import pytest

from hrom_inputs import THETA_REF, make_cluster, make_macro_points
from tests._util import log_case, rel_err_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAR = {0: 1e-12, 1: 1e-5, 2: 1e-5}


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    P.load()
    return P


def _state(P, cls_counts, precision, F, a_list, objective=True):
    from paper_2306_02687_amd import solve
    plan = P.Plan([solve.upload_cluster(c, n) for c, n in cls_counts], precision=precision,
                  objective=objective, split=precision != 0)
    st = plan.status()
    plan.eval(solve.theta_dev(THETA_REF), solve.points_to_soa(F), solve.modes_to_dev(plan, a_list), st)
    Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(plan.N, dtype=torch.float64, device="cuda")
    plan.condense(Pb, Cb, rn, st)
    return plan, st


def _oracle(orc, cl, F, a):
    o = orc.point_eval(cl, THETA_REF, F, a)
    sig, dsdD, st = orc.cauchy(F, o["Palg_r"], o["Cr"])
    assert not st.any() and not o["status"].any()
    return sig, dsdD


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("m,Q,N", [(8, 32, 7), (13, 37, 5), (64, 512, 6), (96, 100, 3)])
def test_cauchy_vs_oracle(P, orc, precision, m, Q, N):
    """Random (Fbar, a) with rotations; sigma [9][N] and dsdD [81][N]."""
    log_case("cauchy", precision, m, Q, N)
    cl = make_cluster(m, Q, 7000 + m)
    F, _, _ = make_macro_points(N, 7100 + m, amp=0.08, max_angle=1.0)
    a = 0.02 * np.random.default_rng(7200 + m).standard_normal((N, m))
    plan, st = _state(P, [(cl, N)], precision, F, [a])
    sig, dsdD = plan.zeros_points(9), plan.zeros_points(81)
    plan.cauchy(sig, dsdD, st)
    torch.cuda.synchronize()
    assert int(st.max().item()) == 0
    ref_s, ref_c = _oracle(orc, cl, F, a)
    es = rel_err_points(sig.cpu().numpy().T, ref_s).max()
    ec = rel_err_points(dsdD.cpu().numpy().T, ref_c.reshape(N, 81)).max()
    print("cauchy", precision, m, Q, "sigma", es, "tangent", ec, flush=True)
    assert es < BAR[precision] and ec < BAR[precision]
    # sigma without the tangent: same bits
    sig2 = plan.zeros_points(9)
    plan.cauchy(sig2, None, st)
    torch.cuda.synchronize()
    assert torch.equal(sig, sig2)
    plan.close()


def test_cauchy_several_clusters(P, orc):
    """A plan of three clusters: every cluster's points vs the oracle."""
    log_case("cauchy_multi")
    shapes = [(8, 48, 5), (24, 144, 4), (80, 480, 3)]
    cls = [make_cluster(m, Q, 7300 + m) for m, Q, _ in shapes]
    Ns = [n for _, _, n in shapes]
    F, _, _ = make_macro_points(sum(Ns), 7400, amp=0.08, max_angle=1.0)
    rng = np.random.default_rng(7401)
    a_list = [0.02 * rng.standard_normal((n, c.m)) for c, n in zip(cls, Ns)]
    plan, st = _state(P, list(zip(cls, Ns)), 0, F, a_list)
    sig, dsdD = plan.zeros_points(9), plan.zeros_points(81)
    plan.cauchy(sig, dsdD, st)
    torch.cuda.synchronize()
    first = 0
    for c, n, a in zip(cls, Ns, a_list):
        ref_s, ref_c = _oracle(orc, c, F[first:first + n], a)
        assert rel_err_points(sig.cpu().numpy().T[first:first + n], ref_s).max() < BAR[0]
        assert rel_err_points(dsdD.cpu().numpy().T[first:first + n], ref_c.reshape(n, 81)).max() < BAR[0]
        first += n
    plan.close()


def test_cauchy_call_order_and_mode(P):
    """Before a condense: HROM_E_ORDER; a plan without the objective split:
    HROM_E_UNSUPPORTED (the Biot route needs Rbar, Ubar)."""
    from paper_2306_02687_amd import binding as B, solve
    log_case("cauchy_errors")
    cl = make_cluster(8, 32, 7500)
    plan = P.Plan([solve.upload_cluster(cl, 4)], precision=0)
    sig = plan.zeros_points(9)
    with pytest.raises(B.HromError, match="-3"):
        plan.cauchy(sig, None, plan.status())
    plan.close()
    F, _, _ = make_macro_points(4, 7501)
    plan, st = _state(P, [(cl, 4)], 0, F, [np.zeros((4, 8))], objective=False)
    with pytest.raises(B.HromError, match="-5"):
        plan.cauchy(plan.zeros_points(9), None, st)
    plan.close()


def test_cauchy_headline_workload_sample(P, orc):
    """131072 points, m = 64, Q = 512, BF16 split, after one evaluate +
    condense at random amplitudes: 32 sampled points vs the oracle."""
    log_case("cauchy_fullsize")
    N, m, Q = 131072, 64, 512
    cl = make_cluster(m, Q, 4000)
    F, _, _ = make_macro_points(N, 7600, amp=0.05)
    a = 0.01 * np.random.default_rng(7601).standard_normal((N, m))
    plan, st = _state(P, [(cl, N)], 1, F, [a])
    sig, dsdD = plan.zeros_points(9), plan.zeros_points(81)
    plan.cauchy(sig, dsdD, st)
    torch.cuda.synchronize()
    assert int(st.max().item()) == 0
    idx = np.sort(np.random.default_rng(7602).choice(N, 32, replace=False))
    ref_s, ref_c = _oracle(orc, cl, F[idx], a[idx])
    es = rel_err_points(sig.cpu().numpy().T[idx], ref_s).max()
    ec = rel_err_points(dsdD.cpu().numpy().T[idx], ref_c.reshape(32, 81)).max()
    print("cauchy fullsize sigma", es, "tangent", ec, flush=True)
    assert es < BAR[1] and ec < BAR[1]
    plan.close()


def test_cauchy_failure_isolation(P):
    """A non-finite macro point keeps its NONFINITE flag through hrom_cauchy
    and leaves every other point's sigma and dsigma/dD bitwise unchanged."""
    log_case("cauchy_isolation")
    m, Q, N = 13, 37, 6
    cl = make_cluster(m, Q, 7700)
    F, _, _ = make_macro_points(N, 7701, amp=0.08, max_angle=1.0)
    a = 0.02 * np.random.default_rng(7702).standard_normal((N, m))
    outs = []
    for bad in (False, True):
        Fb = F.copy()
        if bad:
            Fb[2, 1, 1] = np.nan
        plan, st = _state(P, [(cl, N)], 0, Fb, [a])
        sig, dsdD = plan.zeros_points(9), plan.zeros_points(81)
        plan.cauchy(sig, dsdD, st)
        torch.cuda.synchronize()
        outs.append((sig.cpu().numpy(), dsdD.cpu().numpy(), st.cpu().numpy()))
        plan.close()
    (s0, c0, st0), (s1, c1, st1) = outs
    assert not st0.any()
    assert st1[2] & 8 and not np.delete(st1, 2).any()
    keep = [b for b in range(N) if b != 2]
    assert np.array_equal(s0[:, keep], s1[:, keep]) and np.array_equal(c0[:, keep], c1[:, keep])
    assert np.isfinite(s1).all() and np.isfinite(c1).all()
