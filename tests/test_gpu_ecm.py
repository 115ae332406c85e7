"""GPU parity of the empirical cubature (Sec. 3.3: eq. ECM1, eq. SVDlambda,
Box 1) against the oracle.

Each side runs its own chain from the same seeded candidates and snapshots:
training matrix -> truncated basis -> greedy selection.

* Training matrix x_f and the integrals f^k: element by element, at sizes
  ragged against the 256-candidate workgroups and the four snapshots per
  thread, with V0 != 1.
* Basis: every singular value within 1e-12 sigma_1, lambda orthonormal, and
  the largest principal angle between the two truncated subspaces within a
  bound set by the singular-value gap at the truncation.
* Selection: the per-iteration record (picked candidate, NNLS used, points
  dropped, selection size) equal to the oracle's, the selected indices equal,
  weights within 1e-9 of the oracle's; on cases that run the NNLS fallback
  tens of times.  Where a decision is a near-tie at rounding level (the
  oracle's score gap below 1e-8) the comparison stops there and both results
  must be valid.
* Edge cases: one point (r = 0), the exactness of polynomial rules, and the
  argument checks.
* The workload of the paper's second example (30 modes, 500 points) over
  32768 candidates and 60 snapshots: x_f sampled against the oracle's
  integrand, all singular values and the subspace against numpy's SVD, the
  first 60 greedy iterations against the oracle's, and the final rule exact
  on the truncated system with non-negative weights summing to V0.
"""
import numpy as np
import pytest

from hrom_inputs import THETA_REF, WORKLOADS, make_cluster, make_snapshots
from tests._util import log_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    P.load()
    return P


def _cuda(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def _gpu_training(cl, Fr, a):
    from paper_2306_02687_amd import binding as B
    return B.ecm_training(_cuda(cl.G), _cuda(cl.w), _cuda(cl.phase, torch.int32),
                          _cuda(THETA_REF), _cuda(Fr), _cuda(a))


def _max_angle(L1, L2):
    """sin of the largest principal angle between span L1 and span L2
    (orthonormal columns): the norm of the part of L2 outside span L1."""
    return float(np.linalg.norm(L2 - L1 @ (L1.T @ L2), 2))


@pytest.mark.parametrize("m,M,p", [(8, 1000, 6), (12, 1024, 8), (30, 777, 5)])
def test_training_matrix(dev, orc, m, M, p):
    log_case("ecm training", m, M, p)
    cl = make_cluster(m, M, 9000 + m)
    cl.w = cl.w * 2.5
    Fr, a = make_snapshots(p, m, 9100 + m)
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    xf_o, fint_o = orc.ecm_training_matrix(f, cl.w)
    xf, fint, nbad = _gpu_training(cl, Fr, a)
    assert nbad == 0
    scale = np.abs(f.reshape(p * (m + 9), M)).max(axis=1)
    err = (np.abs(xf.cpu().numpy() - xf_o).max(axis=1) / scale).max()
    errf = (np.abs(fint.cpu().numpy() - fint_o) / (scale * cl.w.sum())).max()
    print(f"training m {m} M {M} p {p}: x_f {err:.2e} fint {errf:.2e}", flush=True)
    assert err < 1e-13 and errf < 1e-13


def _chains(dev, orc, m, M, p, mt, seed, method=0):
    """Oracle and GPU chains from the same inputs."""
    from paper_2306_02687_amd import binding as B
    cl = make_cluster(m, M, seed)
    Fr, a = make_snapshots(p, m, seed + 1)
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    xf_o, _ = orc.ecm_training_matrix(f, cl.w)
    lam_o, s_o = orc.ecm_basis(xf_o, mt - 1)
    xf, _, _ = _gpu_training(cl, Fr, a)
    lam, sig, sweeps, _ = B.ecm_svd(xf, mt - 1, method=method)
    return cl, xf_o, lam_o, s_o, lam, sig, sweeps


# method 1: sweeps on x_f^T itself; 2: Householder QR first, sweeps on R
@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("m,M,p,r", [(8, 1000, 6, 40), (6, 2100, 5, 60), (12, 1024, 8, 95),
                                     (16, 2500, 12, 250), (8, 150, 4, 40)])
def test_svd_basis(dev, orc, m, M, p, r, method):
    log_case("ecm svd", m, M, p, r, method)
    cl, xf_o, lam_o, s_o, lam, sig, sweeps = _chains(dev, orc, m, M, p, r + 1, 9200 + m, method)
    sig = sig.cpu().numpy()
    lam = lam.cpu().numpy()
    es = np.abs(sig - s_o).max() / s_o[0]
    orth = np.abs(lam.T @ lam - np.eye(r)).max()
    ang = _max_angle(lam_o, lam)
    gap = (s_o[r - 1] - s_o[r]) / s_o[0]
    bound = 1e-14 / gap
    print(f"svd P {len(s_o)} M {M} r {r} method {method}: sweeps {sweeps} sigma {es:.2e} orth {orth:.2e} "
          f"angle {ang:.2e} (gap {gap:.2e}, bound {bound:.2e})", flush=True)
    assert es < 1e-12 and orth < 1e-12
    assert ang < bound


def _compare_selection(info_o, trace, z_o, w_o, z, w):
    """Compare the per-iteration records; returns the iterations compared."""
    n_it = len(info_o["picked"])
    for i in range(min(n_it, len(trace))):
        rec_o = (info_o["picked"][i], int(info_o["nnls"][i]), len(info_o["dropped"][i]))
        rec = (int(trace[i][0]), int(trace[i][1]), int(trace[i][2]))
        if rec != rec_o:
            # a rounding-level near-tie of the oracle's own decision
            assert info_o["gap"][i] < 1e-8, (i, rec, rec_o, info_o["gap"][i])
            return i
    assert len(trace) == n_it
    assert z.tolist() == z_o.tolist()
    assert np.abs(w - w_o).max() < 1e-9 * np.abs(w_o).max()
    return n_it


@pytest.mark.parametrize("m,M,p,mt", [(12, 1024, 8, 96), (8, 2048, 10, 96), (6, 777, 4, 40),
                                      (16, 1500, 6, 128)])
def test_selection_pipeline(dev, orc, m, M, p, mt):
    from paper_2306_02687_amd import binding as B
    log_case("ecm selection", m, M, p, mt)
    cl, xf_o, lam_o, s_o, lam, sig, _ = _chains(dev, orc, m, M, p, mt, 9300 + m)
    V0 = float(cl.w.sum())
    z_o, w_o, info_o = orc.ecm_greedy(lam_o, V0, mt)
    z, w, info = B.ecm_select(lam, V0, mt, trace_cap=4 * M)
    trace = info["trace"].cpu().numpy()
    z, w = z.cpu().numpy(), w.cpu().numpy()
    n_cmp = _compare_selection(info_o, trace, z_o, w_o, z, w)
    print(f"selection m {m} M {M} mt {mt}: iters {info['iters']} (oracle {len(info_o['picked'])}) "
          f"NNLS {int(trace[:, 1].sum())} dropped {int(trace[:, 2].sum())} compared {n_cmp} "
          f"w err {np.abs(w - w_o).max() if len(w) == len(w_o) else -1:.2e}", flush=True)
    assert sum(info_o["nnls"]) == 0 or trace[:, 1].sum() > 0
    # the GPU rule on its own basis: exact, non-negative, volume V0
    lamc = lam.cpu().numpy()
    J = np.vstack([lamc.T, np.ones((1, M))])
    b = np.zeros(mt)
    b[-1] = V0
    assert len(z) == mt and np.all(w > 0)
    assert np.linalg.norm(J[:, z] @ w - b) < 1e-10 * V0
    assert abs(w.sum() - V0) < 1e-12 * V0


def test_selection_past_256_points_against_stored_oracle(dev):
    """300 points (the step kernel's position arrays and the triangular solve
    past 256 positions): the record of the stored oracle run, written by
    tests/golden/make_ecm_golden.py from the same seeded inputs."""
    import json
    import os
    from paper_2306_02687_amd import binding as B
    path = os.path.join(os.path.dirname(__file__), "golden", "ecm_m16_M2048_p20_mt300.json")
    ref = json.load(open(path))
    c = ref["case"]
    log_case("ecm stored oracle", c)
    cl = make_cluster(c["m"], c["M"], c["seed"])
    Fr, a = make_snapshots(c["p"], c["m"], c["seed"] + 1)
    xf, _, _ = _gpu_training(cl, Fr, a)
    lam, sig, _, _ = B.ecm_svd(xf, c["mt"] - 1)
    s_o = np.array(ref["sigma"])
    assert np.abs(sig.cpu().numpy() - s_o).max() < 1e-12 * s_o[0]
    z, w, info = B.ecm_select(lam, float(cl.w.sum()), c["mt"], trace_cap=8 * c["M"])
    trace = info["trace"].cpu().numpy()
    info_o = dict(picked=ref["picked"], nnls=ref["nnls"], gap=ref["gap"],
                  dropped=[[0] * d for d in ref["dropped"]])
    n_cmp = _compare_selection(info_o, trace, np.array(ref["z"]), np.array(ref["w"]),
                               z.cpu().numpy(), w.cpu().numpy())
    print(f"stored oracle: iterations {len(ref['picked'])} compared {n_cmp} "
          f"NNLS {int(trace[:, 1].sum())}", flush=True)


def test_selection_maximum_size(dev, orc):
    """The largest selection the step kernel holds: r + 1 = 1024 rows and
    mt = 1024 points (every position array and the triangular solve at full
    length).  The first 100 iterations equal the oracle's; the final rule is
    exact on its truncated system with positive weights summing to V0, and the
    last NNLS (if any) meets the optimality conditions."""
    from paper_2306_02687_amd import binding as B
    log_case("ecm maximum size")
    m, M, p, mt = 16, 6000, 48, 1024
    cl, xf_o, lam_o, s_o, lam, sig, _ = _chains(dev, orc, m, M, p, mt, 9900)
    V0 = float(cl.w.sum())
    z, w, info = B.ecm_select(lam, V0, mt, trace_cap=8 * M)
    trace = info["trace"].cpu().numpy()
    z_o, w_o, info_o = orc.ecm_greedy(lam_o, V0, 100)
    # the spectrum is dense at the truncation (relative gap ~1e-7), so the two
    # truncated subspaces differ by up to ~1e-13 / gap and so may the scores
    gap = (s_o[mt - 2] - s_o[mt - 1]) / s_o[0]
    tie = max(1e-8, 1e-13 / gap)
    for i in range(len(info_o["picked"])):
        rec_o = (info_o["picked"][i], int(info_o["nnls"][i]), len(info_o["dropped"][i]))
        rec = tuple(int(v) for v in trace[i][:3])
        if rec != rec_o:
            assert info_o["gap"][i] < tie, (i, rec, rec_o, info_o["gap"][i], tie)
            break
    z, w = z.cpu().numpy(), w.cpu().numpy()
    lamc = lam.cpu().numpy()
    J = np.vstack([lamc.T, np.ones((1, M))])
    b = np.zeros(mt)
    b[-1] = V0
    print(f"maximum size: iterations {info['iters']} NNLS {int(trace[:, 1].sum())} "
          f"dropped {int(trace[:, 2].sum())} residual {np.linalg.norm(J[:, z] @ w - b):.2e}", flush=True)
    # the removal path of the instance for more than 512 points runs here
    assert int(trace[:, 2].sum()) > 0
    assert len(z) == mt and len(set(z.tolist())) == mt and np.all(w > 0)
    assert np.linalg.norm(J[:, z] @ w - b) < 1e-9 * V0
    assert abs(w.sum() - V0) < 1e-11 * V0


def test_selection_edge_cases(dev, orc):
    from paper_2306_02687_amd import binding as B
    log_case("ecm edge cases")
    # one point: J = 1^T, the first candidate with weight V0
    lam0 = torch.zeros((13, 0), dtype=torch.float64, device="cuda")
    z, w, info = B.ecm_select(lam0, 2.5, 1)
    assert z.tolist() == [0] and w.cpu().tolist() == [2.5]
    # polynomial integrands on a grid: the rule integrates degree d exactly
    M, d = 401, 7
    x = np.linspace(0.0, 1.0, M)
    wq = np.full(M, 1.0 / (M - 1))
    wq[0] = wq[-1] = 0.5 / (M - 1)
    f = np.stack([x ** j for j in range(d + 1)])
    fint = f @ wq
    xfh = f - fint[:, None] / wq.sum()
    xfh[0] = 0.0        # the constant integrand: zero up to the rounding of two sums
    xf = _cuda(xfh)
    lam, sig, _, rc = B.ecm_svd(xf, d)
    zt, wt, _ = B.ecm_select(lam, wq.sum(), d + 1)
    zt, wt = zt.cpu().numpy(), wt.cpu().numpy()
    for j in range(d + 1):
        assert abs((wt * x[zt] ** j).sum() - fint[j]) < 1e-11
    # truncation beyond the rank: the constant row adds nothing, rank d
    _, _, _, rc = B.ecm_svd(xf, d + 1, check=False)
    assert rc == B.E_RANK
    # argument checks (nothing launched)
    lam5 = torch.zeros((10, 5), dtype=torch.float64, device="cuda")
    assert B.ecm_select(lam5, 1.0, 7, check=False)[2]["rc"] == -1        # mt > r + 1
    big = torch.zeros((4, 1024), dtype=torch.float64, device="cuda")
    assert B.ecm_select(big, 1.0, 3, check=False)[2]["rc"] == -1         # r + 1 > 1024
    assert B.ecm_svd(xf, d + 2, check=False)[3] == -1                    # r > P
    assert B.ecm_svd(xf, d, method=3, check=False)[3] == -1              # no such method
    wide = torch.ones((40, 50), dtype=torch.float64, device="cuda")
    assert B.ecm_svd(wide, 4, method=2, check=False)[3] == -1            # QR needs M >= Ppad = 64


def test_paper_example_sizes(dev, orc):
    """30 modes, 500 points, 32768 candidates, 60 snapshots."""
    from paper_2306_02687_amd import binding as B
    wl = WORKLOADS["ecm"]
    m, M, p, mt = wl["m"], wl["M"], wl["p"], wl["mt"]
    log_case("ecm example sizes", m, M, p, mt)
    cl = make_cluster(m, M, wl["seed"])
    Fr, a = make_snapshots(p, m, wl["seed"] + 1, amp=wl["amp"])
    xf, fint, nbad = _gpu_training(cl, Fr, a)
    assert nbad == 0
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    xf_o, fint_o = orc.ecm_training_matrix(f, cl.w)
    del f
    rng = np.random.default_rng(6100)
    rows = rng.choice(p * (m + 9), 64, replace=False)
    xs = xf[torch.from_numpy(rows).cuda()].cpu().numpy()
    scale = np.abs(xf_o[rows]).max(axis=1) + np.abs(fint_o[rows]) / cl.w.sum()
    assert (np.abs(xs - xf_o[rows]).max(axis=1) / scale).max() < 1e-13
    lam, sig, sweeps, _ = B.ecm_svd(xf, mt - 1)
    lam_o, s_o = orc.ecm_basis(xf_o, mt - 1)
    sig = sig.cpu().numpy()
    es = np.abs(sig - s_o).max() / s_o[0]
    lamc = lam.cpu().numpy()
    ang = _max_angle(lam_o, lamc)
    gap = (s_o[mt - 2] - s_o[mt - 1]) / s_o[0]
    V0 = float(cl.w.sum())
    z, w, info = B.ecm_select(lam, V0, mt, trace_cap=4 * mt + 4096)
    trace = info["trace"].cpu().numpy()
    z_o, w_o, info_o = orc.ecm_greedy(lam_o, V0, 60)
    de = np.abs(sig - s_o)
    imax = int(np.argmax(de))
    print(f"sigma error: max at {imax} of {len(s_o)}: sigma_i/sigma_1 {s_o[imax] / s_o[0]:.2e}, "
          f"rel to sigma_i {de[imax] / s_o[imax]:.2e}; top-{mt} max rel to sigma_i "
          f"{(de[:mt] / s_o[:mt]).max():.2e}", flush=True)
    print(f"example sizes: sweeps {sweeps} sigma {es:.2e} angle {ang:.2e} gap {gap:.2e} "
          f"iters {info['iters']} NNLS {int(trace[:, 1].sum())} dropped {int(trace[:, 2].sum())}",
          flush=True)
    # rounding of the Jacobi columns: every sweep updates a column in each of
    # its rounds by 64-term sums, relative error ~ sweeps * rounds * 64 eps
    nb = -(-(p * (m + 9)) // 32)
    nb += nb & 1
    sig_bound = max(1e-12, sweeps * (nb - 1) * 64 * np.finfo(float).eps)
    assert es < sig_bound and ang < 1e-14 / gap
    # the first 60 iterations as the oracle's (its loop ends at 60 points)
    for i in range(len(info_o["picked"])):
        rec_o = (info_o["picked"][i], int(info_o["nnls"][i]), len(info_o["dropped"][i]))
        rec = tuple(int(v) for v in trace[i][:3])
        if rec != rec_o:
            assert info_o["gap"][i] < 1e-8, (i, rec, rec_o)
            break
    z, w = z.cpu().numpy(), w.cpu().numpy()
    J = np.vstack([lamc.T, np.ones((1, M))])
    b = np.zeros(mt)
    b[-1] = V0
    assert len(z) == mt and len(set(z.tolist())) == mt and np.all(w > 0)
    assert np.linalg.norm(J[:, z] @ w - b) < 1e-10 * V0
    assert abs(w.sum() - V0) < 1e-12 * V0
