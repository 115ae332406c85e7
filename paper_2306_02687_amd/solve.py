"""Host-side drivers over the C ABI: layouts, micro Newton, monolithic iterations.

These functions only move data between the caller's natural shapes and the
ABI layouts (on the host, with numpy) and sequence the library calls; the
arithmetic of the method runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def upload_cluster(cl, count: int, device="cuda") -> B.ClusterSpec:
    """Generator cluster (numpy G[Q,9,m], w[Q], phase[Q]) -> device ClusterSpec."""
    return B.ClusterSpec(
        G=torch.from_numpy(np.ascontiguousarray(cl.G, dtype=np.float64)).to(device),
        w=torch.from_numpy(np.ascontiguousarray(cl.w, dtype=np.float64)).to(device),
        phase=torch.from_numpy(np.ascontiguousarray(cl.phase, dtype=np.int32)).to(device),
        count=int(count))


def points_to_soa(x, device="cuda"):
    """[N, ...] per-point array -> [k, N] component-major device tensor."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    return torch.from_numpy(np.ascontiguousarray(x.reshape(N, -1).T)).to(device)


def soa_to_points(t, shape=None):
    x = t.detach().cpu().numpy().T.copy()
    return x if shape is None else x.reshape((x.shape[0],) + tuple(shape))


def modes_to_dev(plan: B.Plan, a_list, device="cuda"):
    """Per-cluster [count_c, m_c] arrays -> the mode-indexed 1-D device array."""
    out = np.zeros(plan.a_len)
    for c, (cl, a) in enumerate(zip(plan.clusters, a_list)):
        blk = np.asarray(a, dtype=np.float64).reshape(cl.count, cl.m).T
        out[plan.off_a[c]: plan.off_a[c] + cl.m * cl.count] = blk.ravel()
    return torch.from_numpy(out).to(device)


def modes_from_dev(plan: B.Plan, t):
    x = t.detach().cpu().numpy()
    res = []
    for c, cl in enumerate(plan.clusters):
        blk = x[plan.off_a[c]: plan.off_a[c] + cl.m * cl.count].reshape(cl.m, cl.count)
        res.append(blk.T.copy())
    return res


def theta_dev(theta, device="cuda"):
    return torch.tensor(np.asarray(theta, dtype=np.float64), device=device)


class State:
    """Device buffers of one solve: a, Pbar, Cbar, rnorm, status."""

    def __init__(self, plan: B.Plan, a=None):
        self.a = plan.zeros_modes() if a is None else a
        self.Pbar = plan.zeros_points(9)
        self.Cbar = plan.zeros_points(81)
        self.rnorm = torch.zeros(plan.N, dtype=torch.float64, device=self.a.device)
        self.status = plan.status()
        self.iters = 0


def newton(plan: B.Plan, theta, Fbar, state: State | None = None, tol=1e-10, max_it=25,
           early_exit=True) -> State:
    """Micro Newton at fixed Fbar: eval + condense; stop when every point has
    ||r||_2 < tol; else update (converged points frozen).  At most max_it
    evaluations; unconverged points get PT_NOCONV."""
    st = State(plan) if state is None else state
    for it in range(max_it):
        plan.eval(theta, Fbar, st.a, st.status)
        plan.condense(st.Pbar, st.Cbar, st.rnorm, st.status)
        st.iters = it + 1
        if early_exit:
            rn = st.rnorm.cpu().numpy()
            stt = st.status.cpu().numpy()
            ok = (stt & (B.PT_JNONPOS | B.PT_NONFINITE)) != 0
            if np.all((rn < tol) | ok):
                break
        if it + 1 < max_it:
            plan.update(None, st.a, st.status, tol=tol)
    rn = st.rnorm.cpu().numpy()
    if np.any(~(rn < tol)):
        stt = st.status.cpu().numpy()
        stt[~(rn < tol)] |= B.PT_NOCONV
        st.status.copy_(torch.from_numpy(stt))
    return st


def monolithic(plan: B.Plan, theta, Fbar0, dFbar_list, state: State | None = None):
    """K monolithic iterations: eval + condense at (Fbar_k, a_k), record
    (Pbar_k, Cbar_k), update with dFbar_k, Fbar_{k+1} = Fbar_k + dFbar_k.
    Fbar0 and dFbar_k are [9, N] device tensors."""
    st = State(plan) if state is None else state
    F = Fbar0.clone()
    out = []
    for dF in dFbar_list:
        plan.eval(theta, F, st.a, st.status)
        plan.condense(st.Pbar, st.Cbar, st.rnorm, st.status)
        out.append((st.Pbar.clone(), st.Cbar.clone(), st.rnorm.clone()))
        plan.update(dF, st.a, st.status)
        F += dF
    return st, out
