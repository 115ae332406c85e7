"""GPU parity of the clustered training (Sec. 3.4, Box 2) and the POD basis
with the elastic-inelastic split (Sec. 3.2.1) against the oracle.

* k-means on normalised strain states: labels identical to the oracle's,
  centres within 1e-13 of the strain scale, the same iteration count; at
  20000 points (ragged against 256-point workgroups) and at the workload's
  262144 points in 30 clusters.
* Trajectories: Fr = I + t H(c) equal to the oracle's bitwise.
* POD: singular values within 1e-12 sigma_1, the elastic span and the whole
  basis within principal angles set by the singular-value gaps, the basis
  orthonormal; at 3000 and 16384 degrees of freedom.
* Argument checks.
"""
import numpy as np
import pytest

from hrom_inputs import WORKLOADS, init_indices, make_pod_snapshots, make_strain_field
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


def _angle(L1, L2):
    return float(np.linalg.norm(L2 - L1 @ (L1.T @ L2), 2))


@pytest.mark.parametrize("N,k,groups", [(20000, 12, 8), (WORKLOADS["training"]["N"],
                                                          WORKLOADS["training"]["k"], 12)])
def test_clusters_vs_oracle(dev, orc, N, k, groups):
    from paper_2306_02687_amd import binding as B
    log_case("training clusters", N, k)
    E = make_strain_field(N, 9500 + k, n_groups=groups)
    idx = init_indices(N, k, 9501 + k)
    C_o, lab_o, it_o = orc.training_clusters(E, k, idx, max_iter=2000)
    C, lab, it, rc = B.training_clusters(_cuda(E.T), k, _cuda(idx, torch.int32), max_iter=2000)
    lab = lab.cpu().numpy()
    C = C.cpu().numpy()
    scale = np.sqrt((E * E).mean(axis=0))
    err = (np.abs(C - C_o) / scale).max()
    print(f"clusters N {N} k {k}: iterations {it} (oracle {it_o}) labels differing "
          f"{int((lab != lab_o).sum())} centres {err:.2e}", flush=True)
    assert rc == 0 and it == it_o and it < 2000
    assert (lab == lab_o).all()
    assert err < 1e-13


def test_paths_vs_oracle(dev, orc):
    from paper_2306_02687_amd import binding as B
    log_case("training paths")
    C = make_strain_field(7, 9600)
    F_o = orc.training_paths(C, 5)
    F = B.training_paths(_cuda(C), 5).cpu().numpy()
    assert np.array_equal(F, F_o)


@pytest.mark.parametrize("nd,s_el,s_in,n_el,n_in", [(3000, 30, 80, 6, 10), (
    WORKLOADS["training"]["nd"], WORKLOADS["training"]["s_el"], WORKLOADS["training"]["s_in"],
    WORKLOADS["training"]["n_el"], WORKLOADS["training"]["n_inel"])])
def test_pod_vs_oracle(dev, orc, nd, s_el, s_in, n_el, n_in):
    from paper_2306_02687_amd import binding as B
    log_case("pod", nd, s_el, s_in, n_el, n_in)
    X_el, X_in, L, P = make_pod_snapshots(nd, s_el, s_in, 9700 + nd, n_in=max(n_in, 12))
    Phi_o, se_o, si_o = orc.pod_split(X_el, X_in, n_el, n_in)
    Phi, se, si, rc = B.pod(_cuda(X_el.T), _cuda(X_in.T), n_el, n_in)
    assert rc == 0
    Phi, se, si = Phi.cpu().numpy(), se.cpu().numpy(), si.cpu().numpy()
    e_el = np.abs(se - se_o).max() / se_o[0]
    e_in = np.abs(si[:n_in + 1] - si_o[:n_in + 1]).max() / si_o[0]
    orth = np.abs(Phi.T @ Phi - np.eye(n_el + n_in)).max()
    a_el = _angle(Phi_o[:, :n_el], Phi[:, :n_el])
    a_all = _angle(Phi_o, Phi)
    gap_el = (se_o[n_el - 1] - se_o[n_el]) / se_o[0]
    gap_in = (si_o[n_in - 1] - si_o[n_in]) / si_o[0]
    print(f"pod nd {nd}: sigma_el {e_el:.2e} sigma_in {e_in:.2e} orth {orth:.2e} angle elastic "
          f"{a_el:.2e} (gap {gap_el:.2e}) whole {a_all:.2e} (gap {gap_in:.2e})", flush=True)
    assert e_el < 1e-12 and e_in < 1e-12 and orth < 1e-12
    assert a_el < 1e-14 / gap_el
    assert a_all < 1e-14 / min(gap_el, gap_in)


def test_argument_checks(dev):
    from paper_2306_02687_amd import binding as B
    log_case("training arguments")
    E9 = torch.zeros((9, 100), dtype=torch.float64, device="cuda")        # d > 8
    idx = torch.arange(4, dtype=torch.int32, device="cuda")
    assert B.training_clusters(E9, 4, idx, check=False)[3] == -1
    E = torch.zeros((6, 3), dtype=torch.float64, device="cuda")           # k > N
    assert B.training_clusters(E, 4, idx, check=False)[3] == -1
    X = torch.zeros((5, 40), dtype=torch.float64, device="cuda")
    assert B.pod(X, X, 6, 2, check=False)[3] == -1                         # n_el > s_el
