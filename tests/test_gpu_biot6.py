"""Six-component (Biot) condensation of objective plans (HROM_BIOT6): the
RVE is driven by the symmetric stretch, so only the six coordinates of Ubar
are condensed (KaU = KaF E6, six right-hand sides).  It must give the
nine-component plan's macro stress and tangent, the same monolithic updates
and adjoint, against the oracle (1e-12 FP64, 1e-5 mixed, 1e-10 / 1e-6 on
gradients), including the LU path and mode counts that use every trailing
block layout; hrom_biot returns the Biot stress and tangent of either kind of
plan (oracle's orc_biot, 1e-12)."""
import numpy as np
import pytest

from hrom_inputs import (THETA_REF, make_cluster, make_increments, make_macro_points,
                         perturbed_theta)
from tests._util import log_case, rel_err_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    P.load()
    return P


def _newton(dev, cl, N, F, precision, biot6, tol=1e-12):
    from paper_2306_02687_amd import solve
    plan = dev.Plan([solve.upload_cluster(cl, N)], precision=precision, biot6=biot6)
    st = solve.newton(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F), tol=tol)
    torch.cuda.synchronize()
    return plan, st


@pytest.mark.parametrize("m,Q", [(8, 48), (13, 37), (24, 144), (64, 512), (96, 192)])
def test_biot6_newton_equals_nine_component_and_oracle(dev, orc, m, Q):
    from paper_2306_02687_amd import solve
    log_case("biot6 newton", m, Q)
    N = 6
    cl = make_cluster(m, Q, 7000 + m)
    F, _, _ = make_macro_points(N, 7001, amp=0.05)
    ref = orc.newton(cl, THETA_REF, F, tol=1e-12)
    for precision, bar in ((0, 1e-12), (1, 1e-5)):
        p9, s9 = _newton(dev, cl, N, F, precision, False)
        p6, s6 = _newton(dev, cl, N, F, precision, True)
        assert int(s6.status.max()) == 0 and s6.iters == s9.iters
        for st in (s9, s6):
            eP = rel_err_points(solve.soa_to_points(st.Pbar), ref["Pbar"])
            eC = rel_err_points(solve.soa_to_points(st.Cbar), ref["Cbar"].reshape(N, -1))
            assert eP.max() < bar and eC.max() < bar
        d = rel_err_points(solve.soa_to_points(s6.Cbar), solve.soa_to_points(s9.Cbar)).max()
        print(f"biot6 m {m} prec {precision}: Cbar vs nine-component {d:.2e}", flush=True)
        assert d < (1e-13 if precision == 0 else 1e-6)
        # Biot outputs of both plans against the oracle's Biot form at the same state
        for plan, st in ((p9, s9), (p6, s6)):
            T = plan.zeros_points(6)
            CB = plan.zeros_points(36)
            plan.biot(T, CB, st.status)
            torch.cuda.synchronize()
            o = orc.point_eval(cl, THETA_REF, F, solve.modes_from_dev(plan, st.a)[0])
            Tr, CBr = orc.biot(o["Palg_r"], o["Cr"])
            assert rel_err_points(solve.soa_to_points(T), Tr).max() < bar
            assert rel_err_points(solve.soa_to_points(CB), CBr.reshape(N, -1)).max() < bar
        p9.close()
        p6.close()


def test_biot6_monolithic_iterations(dev, orc):
    from paper_2306_02687_amd import solve
    log_case("biot6 monolithic")
    N, m, Q, K = 8, 32, 256, 4
    cl = make_cluster(m, Q, 7100)
    F, R, _ = make_macro_points(N, 7101, amp=0.05)
    dF = make_increments(R, K, 7102, amp=0.005)
    plan = dev.Plan([solve.upload_cluster(cl, N)], biot6=True)
    st, out = solve.monolithic(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F),
                               [solve.points_to_soa(x) for x in dF])
    ref = orc.monolithic(cl, THETA_REF, F, dF)
    for k, (Pb, Cb, _) in enumerate(out):
        eP = rel_err_points(solve.soa_to_points(Pb), ref["Pbar"][k])
        eC = rel_err_points(solve.soa_to_points(Cb), ref["Cbar"][k].reshape(N, -1))
        assert eP.max() < 1e-12 and eC.max() < 1e-12, k
    a = solve.modes_from_dev(plan, st.a)[0]
    assert np.abs(a - ref["a"]).max() < 1e-12 * max(1.0, np.abs(ref["a"]).max())
    plan.close()


@pytest.mark.parametrize("precision,refine,bar", [(0, False, 1e-10), (1, True, 1e-6),
                                                  (2, False, 1e-6)])
def test_biot6_adjoint(dev, orc, precision, refine, bar):
    from paper_2306_02687_amd import solve
    log_case("biot6 adjoint", precision, refine)
    N, m, Q = 6, 48, 384
    cl = make_cluster(m, Q, 5000)
    F, _, _ = make_macro_points(N, 5001, amp=0.05)
    th_star, _ = perturbed_theta(5002)
    target = orc.newton(cl, th_star, F, tol=1e-14)["Pbar"]
    plan = dev.Plan([solve.upload_cluster(cl, N)], precision=precision, refine=refine, biot6=True)
    th = solve.theta_dev(THETA_REF)
    st = solve.newton(plan, th, solve.points_to_soa(F), tol=1e-12)
    g = 2.0 * (st.Pbar - solve.points_to_soa(target))
    gF = plan.zeros_points(9)
    gth = torch.zeros(4, dtype=torch.float64, device="cuda")
    plan.backward(th, st.a, g.contiguous(), gF, gth, st.status)
    torch.cuda.synchronize()
    ref_o = orc.newton(cl, THETA_REF, F, tol=1e-14)
    ref = orc.backward(cl, THETA_REF, F, ref_o["a"], 2.0 * (ref_o["Pbar"] - target))
    egF = rel_err_points(solve.soa_to_points(gF), ref["gF"])
    egt = np.linalg.norm(gth.cpu().numpy() - ref["gtheta"]) / np.linalg.norm(ref["gtheta"])
    print(f"biot6 adjoint prec {precision}: dL/dF {egF.max():.2e} dL/dtheta {egt:.2e}", flush=True)
    assert egF.max() < bar and egt < bar
    assert int(st.status.max()) == 0
    plan.close()


def test_biot6_lu_path(dev, orc):
    """Negative shear moduli: every point takes the LU pass, which writes the
    six E6 columns of X; Pbar and Cbar of one evaluate + condense vs the
    oracle (1e-10) and the monolithic update vs the nine-component plan."""
    from paper_2306_02687_amd import solve
    log_case("biot6 LU")
    m, Q, N = 24, 144, 6
    cl = make_cluster(m, Q, 5200)
    F, R, _ = make_macro_points(N, 5201, amp=0.05)
    a = 0.01 * np.random.default_rng(5202).standard_normal((N, m))
    th_np = THETA_REF.copy()
    th_np[0] = th_np[2] = -1.0
    dF = make_increments(R, 1, 5203, amp=0.005)[0]
    ref = orc.point_eval(cl, th_np, F, a)
    outs = []
    for biot6 in (False, True):
        plan = dev.Plan([solve.upload_cluster(cl, N)], biot6=biot6)
        ad = solve.modes_to_dev(plan, [a])
        st = plan.status()
        plan.eval(solve.theta_dev(th_np), solve.points_to_soa(F), ad, st)
        Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
        rn = torch.zeros(N, dtype=torch.float64, device="cuda")
        plan.condense(Pb, Cb, rn, st)
        plan.update(solve.points_to_soa(dF), ad, st)
        torch.cuda.synchronize()
        assert np.all(st.cpu().numpy() == 2)
        assert rel_err_points(solve.soa_to_points(Pb), ref["Pbar"]).max() < 1e-10
        assert rel_err_points(solve.soa_to_points(Cb), ref["Cbar"].reshape(N, -1)).max() < 1e-10
        outs.append(solve.modes_from_dev(plan, ad)[0])
        plan.close()
    assert np.abs(outs[1] - outs[0]).max() < 1e-12 * np.abs(outs[0]).max()
