"""GPU parity of the J2 plasticity path (the Example 1 material of Sec. 5,
history at the ECM points, Sec. 4) against the FP64 oracle, bar 1e-12.

* raw blocks r, Pr, Kaa, KaF, KFF and the evaluated history at random states
  from a nonzero committed history (taken from the oracle's load path and
  installed on the GPU by running the same path);
* a load-unload path of macro states with micro Newton and commits, two
  clusters in one plan, both frames: Pbar, Cbar and the committed history at
  every state;
* the same path and blocks on the mixed BF16 / FP16 path (law, history,
  residual and condensation in FP64, the tangent contraction in split
  low-precision MFMA): Pbar and the history within 1e-9 (the Newton tolerance),
  Cbar and the raw tangent blocks within 1e-5, r and Pr within 1e-12;
* the device-side hrom_newton and the host loop agree bitwise on J2;
* call rules: commit before any evaluation, backward on a J2 plan, commit or
  history on a plan without J2.
"""
import numpy as np
import pytest

from hrom_inputs import MAT_J2, make_cluster, make_load_path, make_macro_points
from tests._util import log_case, rel_err_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    P.load()
    return P


def _plan(dev, cls_counts, objective=True, precision=0):
    from paper_2306_02687_amd import solve
    return dev.Plan([solve.upload_cluster(c, n) for c, n in cls_counts], objective=objective,
                    j2=True, precision=precision)


# per precision: bars of (Pbar, Cbar, history)
BARS = {0: (TOL64, TOL64, TOL64), 1: (1e-9, 1e-5, 1e-9), 2: (1e-9, 1e-5, 1e-9)}


def _run_path(dev, plan, path, tol=1e-10):
    """Newton + commit at every state of the path (host loop); per state:
    Pbar, Cbar, committed history, status."""
    from paper_2306_02687_amd import solve
    th = solve.theta_dev(MAT_J2)
    st = solve.State(plan)
    out = []
    for Fk in path:
        st = solve.newton(plan, th, solve.points_to_soa(Fk), state=st, tol=tol, max_it=25)
        plan.commit()
        hist = [h.cpu().numpy() for h in plan.history(0)]
        out.append((solve.soa_to_points(st.Pbar), solve.soa_to_points(st.Cbar), hist,
                    st.status.cpu().numpy().copy()))
    return out


@pytest.mark.parametrize("objective,precision", [(True, 0), (False, 0), (True, 1), (False, 2)])
def test_j2_load_path_two_clusters(dev, orc, objective, precision):
    log_case("j2 path", objective, precision)
    shapes = [(8, 64, 7), (13, 37, 5)]
    cls = [make_cluster(m, Q, 4500 + m) for m, Q, _ in shapes]
    Ns = [n for _, _, n in shapes]
    N = sum(Ns)
    path = make_load_path(N, 4510, amp=0.03)
    plan = _plan(dev, list(zip(cls, Ns)), objective=objective, precision=precision)
    # every converged state is only as close to the solution as |Kaa^-1| tol
    # (small near plastic flow); the FP64 path retraces the oracle's iterates,
    # the mixed one does not, so both sides of a mixed comparison converge to
    # 1e-12 (the condensed stress is second order in that error, the history
    # first order)
    tol = 1e-10 if precision == 0 else 1e-12
    got = _run_path(dev, plan, path, tol=tol)
    bP, bC, bh = BARS[precision]
    first = 0
    refs = []
    for c, n in zip(cls, Ns):
        refs.append(orc.j2_path(c, MAT_J2, path[:, first:first + n], tol=tol,
                                objective=objective))
        first += n
    yielded = False
    for k in range(len(path)):
        Pg, Cg, hg, sg = got[k]
        assert np.all(sg == 0), sg
        first = 0
        for ci, (c, n) in enumerate(zip(cls, Ns)):
            ref = refs[ci][k]
            eP = rel_err_points(Pg[first:first + n], ref["Pbar"])
            eC = rel_err_points(Cg[first:first + n], ref["Cbar"].reshape(n, -1))
            eh = np.abs(hg[ci] - ref["hist"]).max() / max(np.abs(ref["hist"]).max(), 1e-300)
            yielded |= bool(ref["hist"][:, :, 6].max() > 0)
            print(f"j2 prec {precision} state {k} cluster {ci}: Pbar {eP.max():.2e} Cbar {eC.max():.2e} "
                  f"hist {eh:.2e} alpha max {ref['hist'][:, :, 6].max():.3e}", flush=True)
            assert eP.max() < bP and eC.max() < bC and eh < bh
            first += n
    assert yielded
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_j2_blocks_from_committed_history(dev, orc, precision):
    """Raw blocks and the evaluated history at random amplitudes, starting
    from the history committed after two states of a load path."""
    from paper_2306_02687_amd import solve
    log_case("j2 blocks", precision)
    m, Q, N = 16, 96, 6
    cl = make_cluster(m, Q, 4600)
    path = make_load_path(N, 4601, amp=0.03, levels=(0.6, 1.0))
    plan = _plan(dev, [(cl, N)], objective=False, precision=precision)
    tol = 1e-10 if precision == 0 else 1e-12
    _run_path(dev, plan, path, tol=tol)
    ref_path = orc.j2_path(cl, MAT_J2, path, tol=tol, objective=False)
    hist_n = ref_path[-1]["hist"]
    assert hist_n[:, :, 6].max() > 0
    F = path[-1] + 0.01 * np.random.default_rng(4602).standard_normal((N, 3, 3))
    a = 0.02 * np.random.default_rng(4603).standard_normal((N, m))
    ad = solve.modes_to_dev(plan, [a])
    st = plan.status()
    r = plan.zeros_modes()
    Pr = plan.zeros_points(9)
    Kaa = torch.zeros(plan.kaa_len, dtype=torch.float64, device="cuda")
    KaF = torch.zeros(plan.kaf_len, dtype=torch.float64, device="cuda")
    KFF = plan.zeros_points(81)
    plan.eval(solve.theta_dev(MAT_J2), solve.points_to_soa(F), ad, st, r=r, Pr=Pr, Kaa=Kaa,
              KaF=KaF, KFF=KFF)
    torch.cuda.synchronize()
    ref = orc.j2_eval(cl, MAT_J2, F, a, hist_n)
    assert np.all(st.cpu().numpy() == 0)
    got = dict(r=r.cpu().numpy().reshape(m, N).T, Pr=Pr.cpu().numpy().T,
               Kaa=Kaa.cpu().numpy().reshape(m * m, N).T, KaF=KaF.cpu().numpy().reshape(m * 9, N).T,
               KFF=KFF.cpu().numpy().T)
    for k in ("r", "Pr", "Kaa", "KaF", "KFF"):
        e = rel_err_points(got[k], ref[k].reshape(N, -1))
        print("j2 block", precision, k, e.max(), flush=True)
        bar = TOL64 if (precision == 0 or k in ("r", "Pr")) else 1e-5
        assert e.max() < bar, k
    # the committed history came from a path converged to 1e-10 on either path
    hb = TOL64 if precision == 0 else 1e-9
    ht = plan.history(1)[0].cpu().numpy()
    assert np.abs(ht - ref["hist"]).max() < hb * np.abs(ref["hist"]).max()
    assert np.any(ref["hist"] != hist_n)                         # this state flows further
    # the committed history is untouched by the evaluation
    hn = plan.history(0)[0].cpu().numpy()
    assert np.abs(hn - hist_n).max() < hb * np.abs(hist_n).max()
    plan.close()


def test_j2_device_newton_equals_host_loop(dev):
    from paper_2306_02687_amd import solve
    log_case("j2 device newton")
    cl = make_cluster(8, 64, 4700)
    N = 32
    path = make_load_path(N, 4701, amp=0.03, levels=(0.7, 1.0))
    th = solve.theta_dev(MAT_J2)
    plan1 = _plan(dev, [(cl, N)])
    plan2 = _plan(dev, [(cl, N)])
    a1, a2 = plan1.zeros_modes(), plan2.zeros_modes()
    for Fk in path:
        Fd = solve.points_to_soa(Fk)
        st1 = solve.newton(plan1, th, Fd, state=solve.State(plan1, a1), tol=1e-10, max_it=8,
                           early_exit=False)
        plan1.commit()
        Pb, Cb = plan2.zeros_points(9), plan2.zeros_points(81)
        rn = torch.zeros(N, dtype=torch.float64, device="cuda")
        st2 = plan2.status()
        plan2.newton(th, Fd, a2, Pb, Cb, rn, st2, tol=1e-10, max_it=8)
        plan2.commit()
        torch.cuda.synchronize()
        assert torch.equal(st1.Pbar, Pb) and torch.equal(st1.Cbar, Cb)
        assert torch.equal(plan1.history(0)[0], plan2.history(0)[0])
    plan1.close()
    plan2.close()


def test_j2_call_rules(dev):
    import ctypes
    from paper_2306_02687_amd import binding as B
    from paper_2306_02687_amd import solve
    log_case("j2 call rules")
    cl = make_cluster(8, 32, 4800)
    N = 4
    plan = _plan(dev, [(cl, N)])
    L = B.load()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.hrom_commit(plan._h, s) == -3                      # no evaluation yet
    F, _, _ = make_macro_points(N, 4801, amp=0.01)
    st = solve.newton(plan, solve.theta_dev(MAT_J2), solve.points_to_soa(F), tol=1e-10)
    gF = plan.zeros_points(9)
    gth = torch.zeros(8, dtype=torch.float64, device="cuda")
    rc = L.hrom_backward(plan._h, B._ptr(solve.theta_dev(MAT_J2)), B._ptr(st.a),
                         B._ptr(st.Pbar), B._ptr(gF), B._ptr(gth), B._ptr(st.status), s)
    assert rc == -5
    plan.close()
    plain = dev.Plan([solve.upload_cluster(cl, N)])
    assert L.hrom_commit(plain._h, s) == -5
    out = torch.zeros(N * 32 * 7, dtype=torch.float64, device="cuda")
    assert L.hrom_history(plain._h, 0, B._ptr(out), s) == -5
    plain.close()
