"""Launch variants change speed only: every variant of the tangent
contraction, the kinematics (four or eight wavefronts per workgroup) and the
register condensation (register budget of three or two wavefronts per SIMD)
gives bitwise-identical results, also in the six-component condensation; the
autotuner picks one of each and caches the choice."""
import numpy as np
import pytest

from hrom_inputs import THETA_REF, make_cluster, make_macro_points
from tests._util import log_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,split,m,Q", [(0, False, 32, 256), (1, True, 64, 512),
                                                 (2, True, 24, 144)])
def test_variants_identical_and_autotune(precision, split, m, Q, tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    from paper_2306_02687_amd import solve, tune
    log_case("variants", precision, split, m, Q)
    N = 24
    cl = make_cluster(m, Q, 900 + m)
    F, _, _ = make_macro_points(N, 901, amp=0.05)
    a = [0.02 * np.random.default_rng(2).standard_normal((N, m))]
    plan = P.Plan([solve.upload_cluster(cl, N)], precision=precision, split=split)
    th, Fd, ad = solve.theta_dev(THETA_REF), solve.points_to_soa(F), solve.modes_to_dev(plan, a)
    outs = []
    for v in range(P.Plan.num_variants()):
        plan.set_variant(v)
        st = plan.status()
        Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
        rn = torch.zeros(N, dtype=torch.float64, device="cuda")
        plan.eval(th, Fd, ad, st)
        plan.condense(Pb, Cb, rn, st)
        torch.cuda.synchronize()
        outs.append((Pb, Cb))
    plan.set_variant(0)
    for kind in (P.binding.VK_KIN, P.binding.VK_CONDENSE):
        for v in range(1, P.Plan.num_kernel_variants(kind)):
            plan.set_kernel_variant(kind, v)
            st = plan.status()
            Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
            rn = torch.zeros(N, dtype=torch.float64, device="cuda")
            plan.eval(th, Fd, ad, st)
            plan.condense(Pb, Cb, rn, st)
            torch.cuda.synchronize()
            outs.append((Pb, Cb))
            plan.set_kernel_variant(kind, 0)
    for Pb, Cb in outs[1:]:
        assert torch.equal(Pb, outs[0][0]) and torch.equal(Cb, outs[0][1])
    path = str(tmp_path / "tune.json")
    r1 = tune.autotune(plan, th, Fd, ad, path=path)
    r2 = tune.autotune(plan, th, Fd, ad, path=path)
    assert not r1["cached"] and r2["cached"] and r1["variant"] == r2["variant"]
    assert r1["kin"] == r2["kin"] and r1["cond"] == r2["cond"]
    print("variant times", r1["ms"], flush=True)
    plan.close()


@pytest.mark.parametrize("m", [8, 64, 96])
def test_condense_variants_biot6(m):
    """The six-component condensation at both register budgets: bitwise equal."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    from paper_2306_02687_amd import solve
    log_case("biot6 condense variants", m)
    N = 16
    cl = make_cluster(m, 3 * m, 930 + m)
    F, _, _ = make_macro_points(N, 931, amp=0.05)
    plan = P.Plan([solve.upload_cluster(cl, N)], precision=1, split=True, biot6=True)
    th, Fd = solve.theta_dev(THETA_REF), solve.points_to_soa(F)
    ad = solve.modes_to_dev(plan, [0.02 * np.random.default_rng(3).standard_normal((N, m))])
    outs = []
    for v in range(P.Plan.num_kernel_variants(P.binding.VK_CONDENSE)):
        plan.set_kernel_variant(P.binding.VK_CONDENSE, v)
        st = plan.status()
        Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
        rn = torch.zeros(N, dtype=torch.float64, device="cuda")
        plan.eval(th, Fd, ad, st)
        plan.condense(Pb, Cb, rn, st)
        torch.cuda.synchronize()
        outs.append((Pb, Cb))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    plan.close()
