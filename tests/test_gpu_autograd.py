"""GPU: the converged map as a torch.autograd.Function against the oracle's adjoint.

L = sum ||Pbar - Pbar*||^2 with targets from perturbed material parameters;
gradients through torch.autograd must equal the oracle's adjoint to the FP64
bar, also when the plan is used by another solve between forward and backward
(the backward then rebuilds the stored factorisation).
"""
import numpy as np
import pytest

from hrom_inputs import THETA_REF, make_cluster, make_macro_points, perturbed_theta
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


@pytest.mark.parametrize("interleave", [False, True])
def test_autograd_matches_oracle_adjoint(dev, orc, interleave):
    from paper_2306_02687_amd import solve
    from paper_2306_02687_amd.autograd import hrom_pbar
    log_case("autograd", interleave)
    N = 12
    cl = make_cluster(16, 96, 6100)
    F, _, _ = make_macro_points(N, 6101, amp=0.05)
    th_star, _ = perturbed_theta(6102)
    target = orc.newton(cl, th_star, F, tol=1e-14)["Pbar"]
    plan = dev.Plan([solve.upload_cluster(cl, N)], precision=dev.FP64)
    th = solve.theta_dev(THETA_REF).requires_grad_(True)
    Fd = solve.points_to_soa(F).requires_grad_(True)
    Pbar, Cbar, a, status = hrom_pbar(plan, th, Fd, tol=1e-13)
    if interleave:
        # another solve on the same plan at different deformations
        F2, _, _ = make_macro_points(N, 6103, amp=0.1)
        hrom_pbar(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F2), tol=1e-13)
    loss = ((Pbar - solve.points_to_soa(target)) ** 2).sum()
    gth, gF = torch.autograd.grad(loss, (th, Fd))
    torch.cuda.synchronize()
    ref_o = orc.newton(cl, THETA_REF, F, tol=1e-14)
    ref = orc.backward(cl, THETA_REF, F, ref_o["a"], 2.0 * (ref_o["Pbar"] - target))
    egF = rel_err_points(gF.cpu().numpy().T, ref["gF"])
    egt = np.linalg.norm(gth.cpu().numpy() - ref["gtheta"]) / np.linalg.norm(ref["gtheta"])
    eP = rel_err_points(Pbar.detach().cpu().numpy().T, ref_o["Pbar"])
    print("autograd interleave", interleave, "P", eP.max(), "gF", egF.max(), "gtheta", egt,
          flush=True)
    assert int(status.cpu().max()) == 0
    assert eP.max() < 1e-12 and egF.max() < 1e-10 and egt < 1e-10
    plan.close()
