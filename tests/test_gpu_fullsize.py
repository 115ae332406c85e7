"""Full-size workloads in the launch configuration the benchmark times.

Every test runs the whole workload on the GPU and checks a seeded sample of
macro points against the oracle, which computes those points one by one.
Results that sum over all points (dL/dtheta) are checked through linearity:
with the cotangent non-zero only on the sample, the full-size launch must give
the oracle's gradient over the sample, and exactly zero dL/dFbar elsewhere.
Bars: 1e-12 (FP64 path), 1e-5 (mixed path, hi/lo split) relative per point.
"""
import numpy as np
import pytest

from hrom_inputs import (THETA_REF, make_cluster, make_increments, make_macro_points,
                         perturbed_theta, zipf_counts)
from tests._util import log_case, rel_err_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAR = {0: 1e-12, 1: 1e-5, 2: 1e-5}
BAR_GRAD = {0: 1e-10, 1: 1e-5, 2: 1e-5}


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    P.load()
    return P


def sample(N, seed, k):
    return np.sort(np.random.default_rng(seed).choice(N, size=k, replace=False))


def tuned_plan(P, clusters_counts, precision):
    """Plan with the launch variant the benchmark's autotuner picks."""
    from paper_2306_02687_amd import solve, tune
    plan = P.Plan([solve.upload_cluster(c, n) for c, n in clusters_counts], precision=precision,
                  split=precision != 0)
    return plan, tune


@pytest.mark.parametrize("precision", [1, 2, 0])
def test_headline_workload_newton_and_adjoint(P, orc, precision):
    """131072 points, m = 64, Q = 512: Newton-converged Pbar, Cbar and the
    adjoint on 48 sampled points vs the oracle."""
    from paper_2306_02687_amd import solve
    log_case("fullsize_headline", precision)
    N, m, Q = 131072, 64, 512
    cl = make_cluster(m, Q, 4000)
    F, _, _ = make_macro_points(N, 4001, amp=0.05)
    plan, tune = tuned_plan(P, [(cl, N)], precision)
    th = solve.theta_dev(THETA_REF)
    Fd = solve.points_to_soa(F)
    st = solve.State(plan)
    tune.autotune(plan, th, Fd, st.a, use_cache=False)
    st = solve.newton(plan, th, Fd, tol=1e-12, max_it=8)
    torch.cuda.synchronize()
    assert int(st.status.max().item()) == 0
    idx = sample(N, 4002, 48)
    a_gpu = solve.modes_from_dev(plan, st.a)[0][idx]
    Pb = st.Pbar.cpu().numpy().T[idx]
    Cb = st.Cbar.cpu().numpy().T[idx]
    # the condensed outputs at the GPU's amplitudes, and the converged map
    at_a = orc.point_eval(cl, THETA_REF, F[idx], a_gpu)
    conv = orc.newton(cl, THETA_REF, F[idx], tol=1e-13)
    e1 = max(rel_err_points(Pb, at_a["Pbar"]).max(),
             rel_err_points(Cb, at_a["Cbar"].reshape(len(idx), -1)).max())
    e2 = max(rel_err_points(Pb, conv["Pbar"]).max(),
             rel_err_points(Cb, conv["Cbar"].reshape(len(idx), -1)).max())
    # adjoint with the cotangent on the sample only
    th_star, _ = perturbed_theta(4003)
    target = orc.newton(cl, th_star, F[idx], tol=1e-13)["Pbar"]
    gs = 2.0 * (conv["Pbar"] - target)
    g = np.zeros((N, 9))
    g[idx] = gs
    gF = plan.zeros_points(9)
    gth = torch.zeros(4, dtype=torch.float64, device="cuda")
    plan.backward(th, st.a, solve.points_to_soa(g), gF, gth, st.status)
    torch.cuda.synchronize()
    ref = orc.backward(cl, THETA_REF, F[idx], conv["a"], gs)
    gF_h = gF.cpu().numpy().T
    egF = rel_err_points(gF_h[idx], ref["gF"]).max()
    egt = np.linalg.norm(gth.cpu().numpy() - ref["gtheta"]) / np.linalg.norm(ref["gtheta"])
    off = np.ones(N, bool)
    off[idx] = False
    print("prec", precision, "iters", st.iters, "at a", e1, "converged", e2, "gF", egF,
          "gtheta", egt, flush=True)
    assert e1 < BAR[precision] and e2 < BAR[precision]
    assert egF < BAR_GRAD[precision] and egt < BAR_GRAD[precision]
    assert not np.any(gF_h[off])
    plan.close()


def test_monolithic_workload_fp64(P, orc):
    """65536 points, m = 32, Q = 256, five monolithic iterations: every
    iteration's Pbar, Cbar on a seeded subset of 1024 points vs the oracle."""
    from paper_2306_02687_amd import solve
    log_case("fullsize_monolithic")
    N, K = 65536, 5
    cl = make_cluster(32, 256, 2100)
    F, R, _ = make_macro_points(N, 2101, amp=0.05)
    dF = make_increments(R, K, 2102, amp=0.005)
    plan = P.Plan([solve.upload_cluster(cl, N)], precision=P.FP64)
    _, outs = solve.monolithic(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F),
                               [solve.points_to_soa(d) for d in dF])
    torch.cuda.synchronize()
    idx = sample(N, 2103, 1024)
    ref = orc.monolithic(cl, THETA_REF, F[idx], dF[:, idx])
    worst = 0.0
    for k, (Pb, Cb, _) in enumerate(outs):
        eP = rel_err_points(Pb.cpu().numpy().T[idx], ref["Pbar"][k]).max()
        eC = rel_err_points(Cb.cpu().numpy().T[idx], ref["Cbar"][k].reshape(len(idx), -1)).max()
        worst = max(worst, eP, eC)
    print("monolithic fullsize worst", worst, flush=True)
    assert worst < BAR[0]
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_workload_graph(P, orc, precision):
    """262144 points over the eight clusters (Zipf split): a HIP graph of ten
    monolithic iterations, replayed once, with the launch variants the
    benchmark's autotuner picks (per cluster for the mixed plan); eight sampled
    points per cluster vs the oracle after every iteration."""
    from paper_2306_02687_amd import solve, tune
    log_case("fullsize_batched", precision)
    MS = [8, 16, 24, 32, 48, 64, 80, 96]
    K, total = 10, 262144
    counts = zipf_counts(total, len(MS), 1.1)
    cls = [make_cluster(m, 6 * m, 3900 + i) for i, m in enumerate(MS)]
    F, R, _ = make_macro_points(total, 3950, amp=0.05)
    dF = make_increments(R, K, 3951, amp=0.005)
    plan = P.Plan([solve.upload_cluster(c, n) for c, n in zip(cls, counts)],
                  precision=precision, split=precision != 0)
    th = solve.theta_dev(THETA_REF)
    Fk = [F]
    for k in range(K - 1):
        Fk.append(Fk[-1] + dF[k])
    Fd = [solve.points_to_soa(x) for x in Fk]
    dFd = [solve.points_to_soa(x) for x in dF]
    a = plan.zeros_modes()
    tune.autotune(plan, th, Fd[0], a, use_cache=False)
    st = plan.status()
    rn = torch.zeros(plan.N, dtype=torch.float64, device="cuda")
    outP = [plan.zeros_points(9) for _ in range(K)]
    outC = [plan.zeros_points(81) for _ in range(K)]

    def iterations():
        for k in range(K):
            plan.eval(th, Fd[k], a, st)
            plan.condense(outP[k], outC[k], rn, st)
            plan.update(dFd[k], a, st)

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        iterations()   # warm-up outside the capture
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            iterations()
    torch.cuda.synchronize()
    a.zero_()
    st.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    assert int(st.max().item()) == 0
    first, worst = 0, 0.0
    for c, n, ci in zip(cls, counts, range(len(cls))):
        loc = sample(n, 3952 + ci, 8)
        idx = first + loc
        ref = orc.monolithic(c, THETA_REF, F[idx], dF[:, idx])
        for k in range(K):
            eP = rel_err_points(outP[k].cpu().numpy().T[idx], ref["Pbar"][k]).max()
            eC = rel_err_points(outC[k].cpu().numpy().T[idx], ref["Cbar"][k].reshape(8, -1)).max()
            worst = max(worst, eP, eC)
        first += n
    print("batched fullsize", precision, "worst", worst, flush=True)
    assert worst < BAR[precision]
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_adjoint_workload(P, orc, precision):
    """65536 points, m = 48, Q = 384, theta* perturbed by 10 %: dL/dFbar and
    dL/dtheta of L = sum over 32 sampled points of ||Pbar - Pbar*||^2 vs the
    oracle's adjoint."""
    from paper_2306_02687_amd import solve
    log_case("fullsize_adjoint", precision)
    N, m, Q = 65536, 48, 384
    cl = make_cluster(m, Q, 5100)
    F, _, _ = make_macro_points(N, 5101, amp=0.05)
    plan = P.Plan([solve.upload_cluster(cl, N)], precision=precision, split=precision != 0)
    th = solve.theta_dev(THETA_REF)
    st = solve.newton(plan, th, solve.points_to_soa(F), tol=1e-12, max_it=8)
    idx = sample(N, 5102, 32)
    th_star, _ = perturbed_theta(5103)
    target = orc.newton(cl, th_star, F[idx], tol=1e-13)["Pbar"]
    g = np.zeros((N, 9))
    g[idx] = 2.0 * (st.Pbar.cpu().numpy().T[idx] - target)
    gF = plan.zeros_points(9)
    gth = torch.zeros(4, dtype=torch.float64, device="cuda")
    plan.backward(th, st.a, solve.points_to_soa(g), gF, gth, st.status)
    torch.cuda.synchronize()
    conv = orc.newton(cl, THETA_REF, F[idx], tol=1e-13)
    ref = orc.backward(cl, THETA_REF, F[idx], conv["a"], 2.0 * (conv["Pbar"] - target))
    egF = rel_err_points(gF.cpu().numpy().T[idx], ref["gF"]).max()
    egt = np.linalg.norm(gth.cpu().numpy() - ref["gtheta"]) / np.linalg.norm(ref["gtheta"])
    print("adjoint fullsize", precision, "gF", egF, "gtheta", egt, flush=True)
    assert int(st.status.max().item()) == 0
    assert egF < BAR_GRAD[precision] and egt < BAR_GRAD[precision]
    plan.close()


def test_j2_example1_sizes_load_path(P, orc):
    """J2 plasticity at the sizes of the paper's Example 1 hyper ROM (8 modes,
    250 ECM points) over 262144 macro points: a load-unload path of four
    macro states, device-side Newton and a commit at each; 128 sampled points
    against the oracle's path (Pbar, Cbar and committed history, 1e-12; the
    stress error of a point is taken relative to its largest stress along the
    path, since unloading leaves small stresses whose own relative error is
    rounding amplified by cancellation)."""
    from hrom_inputs import MAT_J2, make_load_path
    from paper_2306_02687_amd import solve
    log_case("fullsize_j2")
    N, m, Q = 262144, 8, 250
    cl = make_cluster(m, Q, 4900)
    levels = (0.5, 1.0, 0.6, 0.2)
    path = make_load_path(N, 4901, amp=0.03, levels=levels)
    idx = sample(N, 4902, 128)
    plan = P.Plan([solve.upload_cluster(cl, N)], j2=True)
    th = solve.theta_dev(MAT_J2)
    a = plan.zeros_modes()
    st = plan.status()
    Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(N, dtype=torch.float64, device="cuda")
    ref = orc.j2_path(cl, MAT_J2, path[:, idx], tol=1e-10)
    for k in range(len(levels)):
        plan.newton(th, solve.points_to_soa(path[k]), a, Pb, Cb, rn, st, tol=1e-10, max_it=8)
        plan.commit()
        torch.cuda.synchronize()
        assert int(st.max().item()) == 0
        Pg = Pb.cpu().numpy().T[idx]
        Cg = Cb.cpu().numpy().T[idx]
        hg = plan.history(0)[0][torch.from_numpy(idx).cuda()].cpu().numpy()
        peak = np.max([np.linalg.norm(r["Pbar"], axis=1) for r in ref], axis=0)
        eP = np.linalg.norm(Pg - ref[k]["Pbar"], axis=1) / peak
        eC = rel_err_points(Cg, ref[k]["Cbar"].reshape(len(idx), -1))
        eh = np.abs(hg - ref[k]["hist"]).max() / np.abs(ref[k]["hist"]).max()
        print(f"j2 full size state {k}: Pbar {eP.max():.2e} Cbar {eC.max():.2e} hist {eh:.2e} "
              f"alpha max {ref[k]['hist'][:, :, 6].max():.3e}", flush=True)
        assert eP.max() < 1e-12 and eC.max() < 1e-12 and eh < 1e-12
    plan.close()
