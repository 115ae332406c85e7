"""Batched uneven RVE clusters (m in {8..96}, Q = 6 m, Zipf split) in one plan:
the tangent contraction of every cluster in cost-ordered tile launches (FP64:
one persistent work-queue launch), the other steps once per cluster; and a HIP
graph capturing 10 monolithic iterations."""
import numpy as np
import pytest

from hrom_inputs import THETA_REF, make_cluster, make_increments, make_macro_points, zipf_counts
from tests._util import log_case, rel_err_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MS = [8, 16, 24, 32, 48, 64, 80, 96]


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    P.load()
    return P


def batched_case(total, seed=3000):
    counts = zipf_counts(total, len(MS), 1.1)
    cls = [make_cluster(m, 6 * m, seed + i) for i, m in enumerate(MS)]
    F, R, _ = make_macro_points(total, seed + 100, amp=0.05)
    return cls, counts, F, R


def plan_for(P, cls, counts, precision=0, split=False):
    from paper_2306_02687_amd import solve
    return P.Plan([solve.upload_cluster(c, n) for c, n in zip(cls, counts)],
                  precision=precision, split=split)


@pytest.mark.parametrize("precision,split,tol", [(0, False, 1e-12), (1, True, 1e-5),
                                                 (2, True, 1e-5)])
def test_batched_newton_vs_oracle(P, orc, precision, split, tol):
    """All eight cluster shapes in one plan, Newton-converged Pbar, Cbar per
    cluster vs the oracle."""
    from paper_2306_02687_amd import solve
    log_case("batched_newton", precision, split)
    cls, counts, F, _ = batched_case(96)
    plan = plan_for(P, cls, counts, precision, split)
    st = solve.newton(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F), tol=1e-10)
    torch.cuda.synchronize()
    Pb = st.Pbar.cpu().numpy().T
    Cb = st.Cbar.cpu().numpy().T
    first = 0
    worst = (0.0, 0.0)
    for c, n in zip(cls, counts):
        ref = orc.newton(c, THETA_REF, F[first:first + n], tol=1e-10)
        eP = rel_err_points(Pb[first:first + n], ref["Pbar"]).max()
        eC = rel_err_points(Cb[first:first + n], ref["Cbar"].reshape(n, -1)).max()
        worst = (max(worst[0], eP), max(worst[1], eC))
        first += n
    print("batched", precision, split, "iters", st.iters, "Pbar", worst[0], "Cbar", worst[1],
          flush=True)
    assert worst[0] < tol and worst[1] < tol
    assert int(st.status.cpu().numpy().max()) == 0
    plan.close()


@pytest.mark.parametrize("precision,split", [(0, False), (1, True)])
def test_batched_matches_single_cluster_plans(P, precision, split):
    """The multi-cluster launches (FP64: one persistent tangent launch over a
    work queue; mixed: 8-point tiles for m <= 64 and 4-point tiles above, all
    clusters in two launches) give bitwise the numbers of one plan per cluster
    (every launch shape keeps the same arithmetic order); ragged tile tails in
    every cluster."""
    from paper_2306_02687_amd import solve
    log_case("batched_vs_single", precision, split)
    cls, counts, F, _ = batched_case(64, seed=3500)
    rng = np.random.default_rng(1)
    a_list = [0.02 * rng.standard_normal((n, c.m)) for c, n in zip(cls, counts)]
    th = solve.theta_dev(THETA_REF)
    plan = plan_for(P, cls, counts, precision, split)
    st = plan.status()
    Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(plan.N, dtype=torch.float64, device="cuda")
    plan.eval(th, solve.points_to_soa(F), solve.modes_to_dev(plan, a_list), st)
    plan.condense(Pb, Cb, rn, st)
    first = 0
    for c, n, a in zip(cls, counts, a_list):
        p1 = plan_for(P, [c], [n], precision, split)
        st1 = p1.status()
        Pb1, Cb1 = p1.zeros_points(9), p1.zeros_points(81)
        rn1 = torch.zeros(n, dtype=torch.float64, device="cuda")
        p1.eval(th, solve.points_to_soa(F[first:first + n]), solve.modes_to_dev(p1, [a]), st1)
        p1.condense(Pb1, Cb1, rn1, st1)
        torch.cuda.synchronize()
        assert torch.equal(Cb[:, first:first + n], Cb1), c.m
        assert torch.equal(Pb[:, first:first + n], Pb1), c.m
        first += n
        p1.close()
    plan.close()


@pytest.mark.parametrize("precision,split", [(0, False), (1, True)])
def test_graph_of_ten_monolithic_iterations(P, orc, precision, split):
    """A HIP graph capturing 10 monolithic iterations (evaluate, condense,
    update with dFbar_k) over the batched clusters: every replay equals the
    eager sequence bitwise; FP64 also matches the oracle's iterations."""
    from paper_2306_02687_amd import solve
    log_case("graph", precision, split)
    K = 10
    cls, counts, F, R = batched_case(80, seed=3700)
    dF = make_increments(R, K, 3800, amp=0.005)
    Fk = [F]
    for k in range(K - 1):
        Fk.append(Fk[-1] + dF[k])
    plan = plan_for(P, cls, counts, precision, split)
    th = solve.theta_dev(THETA_REF)
    Fd = [solve.points_to_soa(x) for x in Fk]
    dFd = [solve.points_to_soa(x) for x in dF]
    a = plan.zeros_modes()
    st = plan.status()
    Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(plan.N, dtype=torch.float64, device="cuda")
    outP = [plan.zeros_points(9) for _ in range(K)]
    outC = [plan.zeros_points(81) for _ in range(K)]

    def iterations():
        for k in range(K):
            plan.eval(th, Fd[k], a, st)
            plan.condense(outP[k], outC[k], rn, st)
            plan.update(dFd[k], a, st)

    a.zero_()
    iterations()
    torch.cuda.synchronize()
    eagerP = [x.clone() for x in outP]
    eagerC = [x.clone() for x in outC]
    eager_a = a.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        a.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            iterations()
    torch.cuda.synchronize()
    for rep in range(3):
        a.zero_()
        for x in outP + outC:
            x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(K):
            assert torch.equal(outP[k], eagerP[k]) and torch.equal(outC[k], eagerC[k]), (rep, k)
        assert torch.equal(a, eager_a)
        # eager work between the replays
        plan.eval(th, Fd[0], plan.zeros_modes(), plan.status())
        torch.cuda.synchronize()
    if precision == 0:
        first = 0
        for c, n in zip(cls, counts):
            ref = orc.monolithic(c, THETA_REF, F[first:first + n], dF[:, first:first + n])
            for k in range(K):
                e = rel_err_points(eagerC[k][:, first:first + n].cpu().numpy().T,
                                   ref["Cbar"][k].reshape(n, -1)).max()
                assert e < 1e-12, (c.m, k, e)
            first += n
    plan.close()
