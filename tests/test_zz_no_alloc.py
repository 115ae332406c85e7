"""The allocation-free entry point hrom_newton_noalloc against the plan path.

hrom_newton_noalloc builds the same plan as hrom_plan_create inside the
library's static device scratch and runs the same kernels as hrom_newton, so
its results must equal those of plan + hrom_newton bitwise, for two calls in
a row (the second smaller, reusing the scratch that the first left behind),
and a request larger than the scratch must be rejected with nothing written.
"""
import numpy as np
import pytest

from hrom_inputs import THETA_REF, make_cluster, make_macro_points
from tests._util import log_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_02687_amd as P
    P.load()
    return P


def _solve_both(P, cls_counts, precision, split, seed, max_it=6, tol=1e-10):
    from paper_2306_02687_amd import binding as B
    from paper_2306_02687_amd import solve
    specs = [solve.upload_cluster(cl, n) for cl, n in cls_counts]
    N = sum(n for _, n in cls_counts)
    F, _, _ = make_macro_points(N, seed, amp=0.05)
    Fd = solve.points_to_soa(F)
    th = solve.theta_dev(THETA_REF)
    # plan path
    plan = P.Plan(specs, precision=precision, split=split)
    a_ref = plan.zeros_modes()
    st_ref = plan.status()
    P_ref, C_ref = plan.zeros_points(9), plan.zeros_points(81)
    rn_ref = torch.zeros(N, dtype=torch.float64, device="cuda")
    plan.newton(th, Fd, a_ref, P_ref, C_ref, rn_ref, st_ref, tol=tol, max_it=max_it)
    torch.cuda.synchronize()
    plan.close()
    # allocation-free path: outputs pre-filled with garbage to see that every entry is written
    a = torch.zeros_like(a_ref)
    st = torch.full_like(st_ref, 77)
    Pb = torch.full_like(P_ref, np.nan)
    Cb = torch.full_like(C_ref, np.nan)
    rn = torch.full_like(rn_ref, np.nan)
    B.newton_noalloc(specs, th, Fd, a, Pb, Cb, rn, st, precision=precision, split=split,
                     tol=tol, max_it=max_it)
    torch.cuda.synchronize()
    return (a_ref, P_ref, C_ref, rn_ref, st_ref), (a, Pb, Cb, rn, st)


def _assert_bitwise(ref, got):
    for x, y, name in zip(ref, got, ("a", "Pbar", "Cbar", "rnorm", "status")):
        assert torch.equal(x, y), name


def test_noalloc_equals_plan_twice_second_smaller(lib):
    # call 1: two clusters, FP64, 256 points
    log_case("noalloc call 1: FP64, clusters (8,32)x200 + (13,37)x56")
    ref, got = _solve_both(lib, [(make_cluster(8, 32, 1000), 200), (make_cluster(13, 37, 1001), 56)],
                           0, False, 1002)
    _assert_bitwise(ref, got)
    assert float(got[3].max()) < 1e-10 and int(got[4].max()) == 0
    # call 2: smaller, one cluster, BF16 with split operands, reusing the scratch
    log_case("noalloc call 2: BF16 split, cluster (6,20)x100")
    ref, got = _solve_both(lib, [(make_cluster(6, 20, 1003), 100)], 1, True, 1004)
    _assert_bitwise(ref, got)
    assert float(got[3].max()) < 1e-10 and int(got[4].max()) == 0


def test_noalloc_rejects_requests_beyond_the_scratch(lib):
    from paper_2306_02687_amd import binding as B
    from paper_2306_02687_amd import solve
    log_case("noalloc oversize request (64,512)x131072 must be rejected")
    cl = make_cluster(64, 512, 1005)
    N = 131072
    spec = solve.upload_cluster(cl, N)
    F = torch.zeros((9, N), dtype=torch.float64, device="cuda")
    F[0] = F[4] = F[8] = 1.0
    th = solve.theta_dev(THETA_REF)
    a = torch.zeros(64 * N, dtype=torch.float64, device="cuda")
    Pb = torch.full((9, N), 5.0, dtype=torch.float64, device="cuda")
    Cb = torch.full((81, 1), 5.0, dtype=torch.float64, device="cuda")   # never touched
    rn = torch.full((N,), 5.0, dtype=torch.float64, device="cuda")
    st = torch.full((N,), 3, dtype=torch.int32, device="cuda")
    rc = B.newton_noalloc([spec], th, F, a, Pb, Cb, rn, st, check=False)
    torch.cuda.synchronize()
    assert rc == B.E_SCRATCH
    assert bool((Pb == 5.0).all()) and bool((rn == 5.0).all()) and bool((st == 3).all())
    assert bool((a == 0.0).all())
    assert B.noalloc_scratch_bytes() == 64 << 20
