"""Launch variants of the tangent contraction change speed only: every
variant gives bitwise-identical results; the autotuner picks one and caches it."""
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
    for Pb, Cb in outs[1:]:
        assert torch.equal(Pb, outs[0][0]) and torch.equal(Cb, outs[0][1])
    path = str(tmp_path / "tune.json")
    r1 = tune.autotune(plan, th, Fd, ad, path=path)
    r2 = tune.autotune(plan, th, Fd, ad, path=path)
    assert not r1["cached"] and r2["cached"] and r1["variant"] == r2["variant"]
    print("variant times", r1["ms"], flush=True)
    plan.close()
