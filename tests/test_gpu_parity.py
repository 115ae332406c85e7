"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: 1e-12 relative (per point, Frobenius) for the FP64 path; 1e-5 for the
mixed path on Pbar and Cbar.  Inputs come from the seeded generators only.
"""
import copy

import numpy as np
import pytest

from hrom_inputs import (THETA_REF, make_cluster, make_increments, make_macro_points,
                         perturbed_theta)
from tests._util import log_case, rel_err_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOLMIX = 1e-5
TOLGRAD = 1e-6   # adjoint gradients of the mixed path (the finite-difference target)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    P.load()
    return P


def make_plan(P, cls_counts, precision=0, objective=True, split=None, refine=False):
    from paper_2306_02687_amd import solve
    specs = [solve.upload_cluster(cl, n) for cl, n in cls_counts]
    return P.Plan(specs, precision=precision, objective=objective, split=split, refine=refine)


def run_eval(P, plan, theta, F, a_list, blocks=True):
    from paper_2306_02687_amd import solve
    th = solve.theta_dev(theta)
    Fd = solve.points_to_soa(F)
    ad = solve.modes_to_dev(plan, a_list)
    st = plan.status()
    out = {}
    if blocks:
        r = plan.zeros_modes()
        Pr = plan.zeros_points(9)
        Kaa = torch.zeros(plan.kaa_len, dtype=torch.float64, device="cuda")
        KaF = torch.zeros(plan.kaf_len, dtype=torch.float64, device="cuda")
        KFF = plan.zeros_points(81)
        plan.eval(th, Fd, ad, st, r=r, Pr=Pr, Kaa=Kaa, KaF=KaF, KFF=KFF)
        out.update(r=r, Pr=Pr, Kaa=Kaa, KaF=KaF, KFF=KFF)
    else:
        plan.eval(th, Fd, ad, st)
    Pbar, Cbar = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(plan.N, dtype=torch.float64, device="cuda")
    plan.condense(Pbar, Cbar, rn, st)
    torch.cuda.synchronize()
    out.update(Pbar=Pbar, Cbar=Cbar, rnorm=rn, status=st)
    return out


def unpack_cluster_blocks(plan, t, kind_off, per_point):
    x = t.cpu().numpy()
    res = []
    for c, cl in enumerate(plan.clusters):
        sz = per_point(cl.m)
        blk = x[kind_off[c]: kind_off[c] + sz * cl.count].reshape(sz, cl.count)
        res.append(blk.T.copy())
    return res


SHAPES = [(8, 32, 6), (13, 37, 5), (32, 256, 9), (64, 512, 4), (96, 100, 3)]


@pytest.mark.parametrize("m,Q,N", SHAPES)
@pytest.mark.parametrize("objective", [True, False])
def test_eval_blocks_fp64(dev, orc, m, Q, N, objective):
    """r, Pr, Kaa, KaF, KFF at random (Fbar, a) vs the oracle, <= 1e-12."""
    log_case("eval_blocks_fp64", m, Q, N, objective)
    cl = make_cluster(m, Q, 100 + m)
    F, _, _ = make_macro_points(N, 200 + m, amp=0.1)
    a = 0.03 * np.random.default_rng(m).standard_normal((N, m))
    plan = make_plan(dev, [(cl, N)], objective=objective)
    o = run_eval(dev, plan, THETA_REF, F, [a])
    Fr = orc.polar(F)[0] if objective else F
    ref = orc.eval_blocks(cl, THETA_REF, Fr, a)
    r = unpack_cluster_blocks(plan, o["r"], plan.off_a, lambda m_: m_)[0]
    Kaa = unpack_cluster_blocks(plan, o["Kaa"], plan.off_kaa, lambda m_: m_ * m_)[0]
    KaF = unpack_cluster_blocks(plan, o["KaF"], plan.off_kaf, lambda m_: 9 * m_)[0]
    Pr = o["Pr"].cpu().numpy().T
    KFF = o["KFF"].cpu().numpy().T
    errs = dict(r=rel_err_points(r, ref["r"]), Pr=rel_err_points(Pr, ref["Pr"]),
                Kaa=rel_err_points(Kaa, ref["Kaa"].reshape(N, -1)),
                KaF=rel_err_points(KaF, ref["KaF"].reshape(N, -1)),
                KFF=rel_err_points(KFF, ref["KFF"].reshape(N, -1)))
    print({k: float(v.max()) for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v.max() < TOL64, (k, v.max())
    assert np.all(o["status"].cpu().numpy() == 0)
    plan.close()


@pytest.mark.parametrize("m,Q,N", SHAPES)
@pytest.mark.parametrize("objective", [True, False])
def test_condense_fp64(dev, orc, m, Q, N, objective):
    """Pbar (algorithmic), Cbar, ||r|| at random a vs the oracle, <= 1e-12."""
    log_case("condense_fp64", m, Q, N, objective)
    cl = make_cluster(m, Q, 300 + m)
    F, _, _ = make_macro_points(N, 400 + m, amp=0.1)
    a = 0.03 * np.random.default_rng(m + 1).standard_normal((N, m))
    plan = make_plan(dev, [(cl, N)], objective=objective)
    o = run_eval(dev, plan, THETA_REF, F, [a], blocks=False)
    ref = orc.point_eval(cl, THETA_REF, F, a, objective=objective)
    eP = rel_err_points(o["Pbar"].cpu().numpy().T, ref["Pbar"])
    eC = rel_err_points(o["Cbar"].cpu().numpy().T, ref["Cbar"].reshape(N, -1))
    eR = rel_err_points(o["rnorm"].cpu().numpy()[:, None], ref["rnorm"][:, None])
    print("Pbar", eP.max(), "Cbar", eC.max(), "rnorm", eR.max(), flush=True)
    assert eP.max() < TOL64 and eC.max() < TOL64 and eR.max() < TOL64
    plan.close()


def test_newton_small_workload(dev, orc):
    """256 points, m = 8, Q = 32: Newton from a = 0 to ||r|| < 1e-10, then Pbar, Cbar."""
    from paper_2306_02687_amd import solve
    log_case("newton_fp64_small")
    cl = make_cluster(8, 32, 1000)
    F, _, _ = make_macro_points(256, 1001, amp=0.05)
    plan = make_plan(dev, [(cl, 256)])
    st = solve.newton(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F), tol=1e-10)
    torch.cuda.synchronize()
    ref = orc.newton(cl, THETA_REF, F, tol=1e-10)
    eP = rel_err_points(st.Pbar.cpu().numpy().T, ref["Pbar"])
    eC = rel_err_points(st.Cbar.cpu().numpy().T, ref["Cbar"].reshape(256, -1))
    a = solve.modes_from_dev(plan, st.a)[0]
    ea = np.abs(a - ref["a"]).max()
    print("iters", st.iters, int(ref["iters"].max()), "Pbar", eP.max(), "Cbar", eC.max(), "a", ea,
          flush=True)
    assert st.iters == int(ref["iters"].max())
    assert eP.max() < TOL64 and eC.max() < TOL64 and ea < 1e-12
    assert np.all(st.status.cpu().numpy() == 0)
    # the device-side fixed-count Newton (no host sync) gives the same result
    st2 = solve.State(plan)
    plan.newton(solve.theta_dev(THETA_REF), solve.points_to_soa(F), st2.a, st2.Pbar, st2.Cbar,
                st2.rnorm, st2.status, tol=1e-10, max_it=6)
    torch.cuda.synchronize()
    assert torch.equal(st2.Pbar, st.Pbar) and torch.equal(st2.Cbar, st.Cbar)
    plan.close()


def test_monolithic_iterations(dev, orc):
    """m = 32, Q = 256: five monolithic iterations (evaluate, condense, update
    with dFbar), outputs compared after every iteration."""
    from paper_2306_02687_amd import solve
    log_case("monolithic_fp64")
    N = 48
    cl = make_cluster(32, 256, 2000)
    F, R, _ = make_macro_points(N, 2001, amp=0.05)
    dF = make_increments(R, 5, 2002, amp=0.005)
    plan = make_plan(dev, [(cl, N)])
    _, outs = solve.monolithic(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F),
                               [solve.points_to_soa(d) for d in dF])
    torch.cuda.synchronize()
    ref = orc.monolithic(cl, THETA_REF, F, dF)
    for k, (Pb, Cb, rn) in enumerate(outs):
        eP = rel_err_points(Pb.cpu().numpy().T, ref["Pbar"][k])
        eC = rel_err_points(Cb.cpu().numpy().T, ref["Cbar"][k].reshape(N, -1))
        print("iter", k, "Pbar", eP.max(), "Cbar", eC.max(), flush=True)
        assert eP.max() < TOL64 and eC.max() < TOL64


@pytest.mark.parametrize("precision,split", [(1, True), (2, True)])
@pytest.mark.parametrize("amp", [0.01, 0.05, 0.2])
def test_mixed_vs_oracle(dev, orc, precision, split, amp):
    """m = 64, Q = 512 mixed path: Newton-converged Pbar, Cbar vs the FP64 oracle."""
    from paper_2306_02687_amd import solve
    log_case("mixed", precision, split, amp)
    N = 8
    cl = make_cluster(64, 512, 4000)
    F, _, _ = make_macro_points(N, 4001 + int(amp * 1000), amp=amp)
    plan = make_plan(dev, [(cl, N)], precision=precision, split=split)
    st = solve.newton(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F), tol=1e-10)
    torch.cuda.synchronize()
    ref = orc.newton(cl, THETA_REF, F, tol=1e-10)
    eP = rel_err_points(st.Pbar.cpu().numpy().T, ref["Pbar"])
    eC = rel_err_points(st.Cbar.cpu().numpy().T, ref["Cbar"].reshape(N, -1))
    print("prec", precision, "split", split, "amp", amp, "iters", st.iters, "Pbar", eP.max(),
          "Cbar", eC.max(), flush=True)
    assert np.all(st.status.cpu().numpy() == 0)
    assert eP.max() < TOLMIX and eC.max() < TOLMIX
    plan.close()


@pytest.mark.parametrize("precision,split,refine", [(0, False, False), (2, True, False),
                                                    (1, True, False), (1, True, True),
                                                    (2, True, True)])
def test_backward_vs_oracle(dev, orc, precision, split, refine):
    """Adjoint gradients dL/dFbar, dL/dtheta of L = sum ||Pbar - Pbar*||^2 at
    the converged state (m = 48, Q = 384) vs the oracle's adjoint."""
    from paper_2306_02687_amd import solve
    log_case("backward", precision)
    N = 6
    cl = make_cluster(48, 384, 5000)
    F, _, _ = make_macro_points(N, 5001, amp=0.05)
    th_star, _ = perturbed_theta(5002)
    target = orc.newton(cl, th_star, F, tol=1e-14)["Pbar"]
    plan = make_plan(dev, [(cl, N)], precision=precision, split=split, refine=refine)
    th = solve.theta_dev(THETA_REF)
    st = solve.newton(plan, th, solve.points_to_soa(F), tol=1e-12)
    g = 2.0 * (st.Pbar - solve.points_to_soa(target))
    gF = plan.zeros_points(9)
    gth = torch.zeros(4, dtype=torch.float64, device="cuda")
    plan.backward(th, st.a, g.contiguous(), gF, gth, st.status)
    torch.cuda.synchronize()
    a_conv = solve.modes_from_dev(plan, st.a)[0]
    ref_o = orc.newton(cl, THETA_REF, F, tol=1e-14)
    gref = 2.0 * (ref_o["Pbar"] - target)
    ref = orc.backward(cl, THETA_REF, F, ref_o["a"], gref)
    egF = rel_err_points(gF.cpu().numpy().T, ref["gF"])
    egt = np.linalg.norm(gth.cpu().numpy() - ref["gtheta"]) / np.linalg.norm(ref["gtheta"])
    print("prec", precision, "split", split, "refine", refine, "gF", egF.max(), "gtheta", egt,
          "a", np.abs(a_conv - ref_o["a"]).max(), flush=True)
    bound = 1e-10 if precision == 0 else TOLGRAD
    assert egF.max() < bound and egt < bound
    assert int(st.status.max().item()) == 0
    plan.close()


@pytest.mark.parametrize("m,Q", [(72, 150), (80, 160), (96, 192)])
@pytest.mark.parametrize("precision,split,refine", [(2, True, True), (1, True, True), (1, True, False),
                                                    (2, True, False)])
def test_backward_beyond_64_modes(dev, orc, m, Q, precision, split, refine):
    """The adjoint with more modes than lanes, up to the largest supported m,
    vs the oracle's adjoint: refined (rows 64.. of the refinement solve on a
    wavefront's second register set) and unrefined (the re-evaluation's
    BF16 three-level GEMMs over three halves of 32 modes, the last one
    partly filled at m = 72, 80)."""
    from paper_2306_02687_amd import solve
    log_case("backward_refined", m, Q, precision, split, refine)
    N = 3
    cl = make_cluster(m, Q, 5100 + m)
    F, _, _ = make_macro_points(N, 5101, amp=0.05)
    th_star, _ = perturbed_theta(5102)
    target = orc.newton(cl, th_star, F, tol=1e-14)["Pbar"]
    plan = make_plan(dev, [(cl, N)], precision=precision, split=split, refine=refine)
    th = solve.theta_dev(THETA_REF)
    st = solve.newton(plan, th, solve.points_to_soa(F), tol=1e-12)
    g = 2.0 * (st.Pbar - solve.points_to_soa(target))
    gF = plan.zeros_points(9)
    gth = torch.zeros(4, dtype=torch.float64, device="cuda")
    plan.backward(th, st.a, g.contiguous(), gF, gth, st.status)
    torch.cuda.synchronize()
    assert int(st.status.max().item()) == 0
    ref_o = orc.newton(cl, THETA_REF, F, tol=1e-14)
    ref = orc.backward(cl, THETA_REF, F, ref_o["a"], 2.0 * (ref_o["Pbar"] - target))
    egF = rel_err_points(gF.cpu().numpy().T, ref["gF"])
    egt = np.linalg.norm(gth.cpu().numpy() - ref["gtheta"]) / np.linalg.norm(ref["gtheta"])
    print("m", m, "prec", precision, "refine", refine, "gF", egF.max(), "gtheta", egt, flush=True)
    assert egF.max() < TOLGRAD and egt < TOLGRAD
    plan.close()


def test_backward_refined_lu_path(dev, orc):
    """An indefinite Kaa (negative shear moduli) at a state that is not an
    equilibrium (random a): every point takes the LU factor.  FP64: the
    adjoint matches the oracle's at the same state to 1e-10.  Mixed (BF16 and
    FP16 split): no accuracy is claimed for points flagged NOT_SPD, and at
    such a non-equilibrium state the forward Palg = Pr - KaF^T y carries the
    error of y from the low-precision factor (large at the one point of this
    input whose Kaa is ill-conditioned); the adjoint refinement runs the row
    interchanges and both substitutions of the LU factor and must not make any
    point worse, keep all but that point within 1e-5, and set no status bit
    beyond NOT_SPD (and NOREFINE, if its corrections do not settle)."""
    from paper_2306_02687_amd import solve
    log_case("backward_refined_lu")
    m, Q, N = 24, 144, 6
    cl = make_cluster(m, Q, 5200)
    F, _, _ = make_macro_points(N, 5201, amp=0.05)
    a = 0.01 * np.random.default_rng(5202).standard_normal((N, m))
    th_np = THETA_REF.copy()
    th_np[0] = th_np[2] = -1.0
    g = 0.1 * np.random.default_rng(5203).standard_normal((N, 9))
    ref = orc.backward(cl, th_np, F, a, g)
    assert np.all(ref["status"] == 2)

    def adjoint_errors(precision, refine):
        plan = make_plan(dev, [(cl, N)], precision=precision, refine=refine)
        th = solve.theta_dev(th_np)
        a_dev = solve.modes_to_dev(plan, [a])
        st = plan.status()
        plan.eval(th, solve.points_to_soa(F), a_dev, st)
        Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
        rn = torch.zeros(N, dtype=torch.float64, device="cuda")
        plan.condense(Pb, Cb, rn, st)
        gF = plan.zeros_points(9)
        gth = torch.zeros(4, dtype=torch.float64, device="cuda")
        plan.backward(th, a_dev, solve.points_to_soa(g), gF, gth, st)
        torch.cuda.synchronize()
        s = st.cpu().numpy()
        egF = rel_err_points(gF.cpu().numpy().T, ref["gF"])
        plan.close()
        with np.printoptions(linewidth=200, precision=2):
            print("LU path prec", precision, "refine", refine, "status", s, "gF", egF, flush=True)
        return s, egF

    s, egF = adjoint_errors(0, False)
    assert np.all(s == 2) and egF.max() < 1e-10
    for precision in (1, 2):
        s, e_plain = adjoint_errors(precision, False)
        assert np.all(s == 2)
        s, e_ref = adjoint_errors(precision, True)
        assert np.all((s == 2) | (s == 2 + 16))
        assert np.all(e_ref <= 1.01 * e_plain + 1e-12)
        assert np.sort(e_ref)[N - 2] < TOLMIX


def test_clusters_in_one_plan_match_single_plans(dev, orc):
    """Several clusters of different (m, Q) in one plan give bitwise the same
    results as one plan per cluster, and match the oracle."""
    log_case("multi_cluster")
    shapes = [(8, 48, 5), (16, 96, 3), (24, 144, 4)]
    cls = [make_cluster(m, Q, 3000 + m) for m, Q, _ in shapes]
    Ns = [n for _, _, n in shapes]
    F, _, _ = make_macro_points(sum(Ns), 3100, amp=0.05)
    a_list = [0.02 * np.random.default_rng(i).standard_normal((n, c.m)) for i, (c, n) in
              enumerate(zip(cls, Ns))]
    plan = make_plan(dev, list(zip(cls, Ns)))
    o = run_eval(dev, plan, THETA_REF, F, a_list, blocks=False)
    first = 0
    for c, n, a in zip(cls, Ns, a_list):
        p1 = make_plan(dev, [(c, n)])
        o1 = run_eval(dev, p1, THETA_REF, F[first:first + n], [a], blocks=False)
        assert torch.equal(o["Pbar"][:, first:first + n], o1["Pbar"])
        assert torch.equal(o["Cbar"][:, first:first + n], o1["Cbar"])
        ref = orc.point_eval(c, THETA_REF, F[first:first + n], a)
        assert rel_err_points(o1["Pbar"].cpu().numpy().T, ref["Pbar"]).max() < TOL64
        first += n
        p1.close()
    plan.close()


@pytest.mark.parametrize("precision,split,refine", [(0, False, False), (1, True, False),
                                                    (2, True, True)])
def test_backward_clusters_in_one_plan(dev, orc, precision, split, refine):
    """Adjoint of a plan holding several clusters vs the oracle's adjoint
    cluster by cluster; dL/dtheta sums over all points.  On the FP64 path
    dL/dFbar also equals that of one plan per cluster bitwise."""
    from paper_2306_02687_amd import solve
    log_case("backward_multi", precision, split, refine)
    shapes = [(8, 48, 5), (24, 144, 4), (48, 288, 3)]
    cls = [make_cluster(m, Q, 3200 + m) for m, Q, _ in shapes]
    Ns = [n for _, _, n in shapes]
    F, _, _ = make_macro_points(sum(Ns), 3300, amp=0.05)
    th_star, _ = perturbed_theta(3301)
    th = solve.theta_dev(THETA_REF)

    def adjoint(cls_counts, Fp, target):
        plan = make_plan(dev, cls_counts, precision=precision, split=split, refine=refine)
        st = solve.newton(plan, th, solve.points_to_soa(Fp), tol=1e-12)
        g = 2.0 * (st.Pbar - solve.points_to_soa(target))
        gF = plan.zeros_points(9)
        gth = torch.zeros(4, dtype=torch.float64, device="cuda")
        plan.backward(th, st.a, g.contiguous(), gF, gth, st.status)
        torch.cuda.synchronize()
        assert int(st.status.max().item()) == 0
        plan.close()
        return gF.cpu(), gth.cpu().numpy()

    targets, refs, first = [], [], 0
    for c, n in zip(cls, Ns):
        Fc = F[first:first + n]
        tgt = orc.newton(c, th_star, Fc, tol=1e-14)["Pbar"]
        conv = orc.newton(c, THETA_REF, Fc, tol=1e-14)
        refs.append(orc.backward(c, THETA_REF, Fc, conv["a"], 2.0 * (conv["Pbar"] - tgt)))
        targets.append(tgt)
        first += n
    gF, gth = adjoint(list(zip(cls, Ns)), F, np.concatenate(targets))
    egF = rel_err_points(gF.numpy().T, np.concatenate([r["gF"] for r in refs]))
    gth_ref = sum(r["gtheta"] for r in refs)
    egt = np.linalg.norm(gth - gth_ref) / np.linalg.norm(gth_ref)
    print("backward multi", precision, split, refine, "gF", egF.max(), "gtheta", egt, flush=True)
    bound = 1e-10 if precision == 0 else TOLGRAD
    assert egF.max() < bound and egt < bound
    if precision == 0:
        first = 0
        for c, n, tgt in zip(cls, Ns, targets):
            gF1, _ = adjoint([(c, n)], F[first:first + n], tgt)
            assert torch.equal(gF[:, first:first + n], gF1)
            first += n


def test_status_flags_and_isolation(dev, orc):
    """Failed points are flagged and do not disturb their neighbours."""
    log_case("status_flags")
    cl = make_cluster(8, 32, 77)
    F, _, _ = make_macro_points(8, 78, amp=0.05)
    Fb = F.copy()
    Fb[1, 0, 0] = np.nan                 # non-finite input
    Fb[2] = np.diag([-1.0, 1.0, 1.0])    # det Fbar <= 0
    plan = make_plan(dev, [(cl, 8)])
    a = [np.zeros((8, 8))]
    o = run_eval(dev, plan, THETA_REF, Fb, a, blocks=False)
    st = o["status"].cpu().numpy()
    assert st[1] & 8 and st[2] & 1
    good = [0, 3, 4, 5, 6, 7]
    ref = orc.point_eval(cl, THETA_REF, F[good], np.zeros((6, 8)))
    assert rel_err_points(o["Pbar"].cpu().numpy().T[good], ref["Pbar"]).max() < TOL64
    assert np.all(st[good] == 0)
    # an indefinite Kaa (negative shear moduli) takes the LU path
    th = THETA_REF.copy()
    th[0] = th[2] = -1.0
    o = run_eval(dev, plan, th, F, a, blocks=False)
    st = o["status"].cpu().numpy()
    assert np.all(st & 2)
    ref = orc.point_eval(cl, th, F, np.zeros((8, 8)))
    assert rel_err_points(o["Pbar"].cpu().numpy().T, ref["Pbar"]).max() < 1e-10
    plan.close()


def test_determinism(dev):
    """Same inputs twice: bitwise identical outputs (no float atomics)."""
    log_case("determinism")
    cl = make_cluster(32, 256, 9)
    F, _, _ = make_macro_points(12, 10, amp=0.05)
    a = [0.02 * np.random.default_rng(0).standard_normal((12, 32))]
    for prec in (0, 1):
        plan = make_plan(dev, [(cl, 12)], precision=prec, split=True)
        o1 = run_eval(dev, plan, THETA_REF, F, a, blocks=False)
        o2 = run_eval(dev, plan, THETA_REF, F, a, blocks=False)
        assert torch.equal(o1["Pbar"], o2["Pbar"]) and torch.equal(o1["Cbar"], o2["Cbar"])
        plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_weights_of_any_measure(dev, orc, precision):
    """ECM weights that add up to V0 = 2.5 instead of 1: the sums are volume
    averages (divided by V0), so the converged Pbar, Cbar equal those of the
    normalised weights and the oracle's with the same weights."""
    from paper_2306_02687_amd import solve
    log_case("weights measure", precision)
    N = 8
    cl = make_cluster(16, 96, 6300)
    F, _, _ = make_macro_points(N, 6301, amp=0.05)
    sc = copy.copy(cl)
    sc.w = 2.5 * cl.w
    out = []
    for c in (cl, sc):
        plan = make_plan(dev, [(c, N)], precision=precision)
        st = solve.newton(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F), tol=1e-12)
        out.append((solve.soa_to_points(st.Pbar), solve.soa_to_points(st.Cbar)))
        assert int(st.status.max().item()) == 0
        plan.close()
    ref = orc.newton(sc, THETA_REF, F, tol=1e-12)
    bar = TOL64 if precision == 0 else TOLMIX
    assert rel_err_points(out[1][0], ref["Pbar"]).max() < bar
    assert rel_err_points(out[1][1], ref["Cbar"].reshape(N, -1)).max() < bar
    assert rel_err_points(out[1][0], out[0][0]).max() < bar
    assert rel_err_points(out[1][1], out[0][1]).max() < bar
