"""Seeded generators for the synthetic RVE clusters and macro load states.

Shapes and distributions follow the synthetic workloads of the hyper-reduced
RVE evaluation (monolithic hyper ROM FE2, Sec. 3.2-3.3 of the paper): an RVE
cluster is described by its ECM points (weights ``w``), the mode gradients
``G`` of its ROM modes at those points and a phase label per point; every
macro Gauss point carries a macro deformation gradient ``Fbar``.

Readings of the workload text:

* ``N(0, 0.05)`` means standard deviation 0.05.
* Draw order per cluster: weights, then mode gradients, then phases, all from
  one ``numpy.random.default_rng(seed)`` (PCG64).
* The weighted mean of each mode gradient is subtracted with the normalised
  weights, so ``sum_q w_q G_qm = 0`` holds to rounding (zero-mean fluctuation
  gradients, the periodic-fluctuation property of Sec. 2).
* Macro loads ``Fbar = R (I + H)`` with ``H`` symmetric; draws are taken in
  blocks: all six upper-triangle entries of every point, then every rotation
  axis (normalised standard-normal 3-vector), then every angle.
* Monolithic-iteration increments ``dFbar = R dH`` with symmetric ``dH`` keep
  the polar split exact (``Ubar`` moves from ``I + H`` to ``I + H + dH``).

Arrays use the natural numpy shapes: ``G[Q, 9, m]`` (3x3 tensors flattened
row-major, index ``3 i + j``), ``Fbar[N, 3, 3]``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# (mu_matrix, lambda_matrix, mu_inclusion, lambda_inclusion)
THETA_REF = np.array([1.0, 1.5, 10.0, 15.0], dtype=np.float64)
# J2 plasticity of the paper's Example 1 (Sec. 5): matrix E = 1, nu = 0.3,
# sigma_y0 = 0.01 E, hardening modulus h = 0.016 E; elastic inclusions E = 10,
# nu = 0.3 (a yield stress beyond reach).  Per phase (mu, lambda, sigma_y0, H)
# with mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu)).
MAT_J2 = np.array([1.0 / 2.6, 0.3 / 0.52, 0.01, 0.016,
                   10.0 / 2.6, 3.0 / 0.52, 1.0e30, 0.0], dtype=np.float64)
# high phase contrast (soft matrix, stiff inclusions): the mode-space stiffness
# is ill-conditioned through the material rather than through the basis
THETA_CONTRAST = np.array([1.0e-3, 1.5e-3, 10.0, 15.0], dtype=np.float64)


@dataclass
class Cluster:
    """One RVE cluster: ECM weights, mode gradients and phase labels."""

    m: int
    Q: int
    G: np.ndarray      # [Q, 9, m] float64
    w: np.ndarray      # [Q] float64, sums to 1 (the RVE measure V0)
    phase: np.ndarray  # [Q] int32, 0 = matrix, 1 = inclusion
    seed: int


def make_cluster(m: int, Q: int, seed: int, g_std: float = 0.05,
                 p_incl: float = 0.3) -> Cluster:
    """Draw one RVE cluster (weights, mode gradients, phase map)."""
    if m < 1 or Q < 1:
        raise ValueError("m and Q must be positive")
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, size=Q)
    w = w / w.sum()
    G = rng.normal(0.0, g_std, size=(Q, 9, m))
    # remove the weighted mean of every (component, mode) over the ECM points
    mean = np.tensordot(w, G, axes=(0, 0))          # [9, m]
    G = G - mean[None, :, :]
    phase = (rng.random(Q) < p_incl).astype(np.int32)
    return Cluster(m=m, Q=Q, G=np.ascontiguousarray(G), w=w, phase=phase, seed=seed)


def make_cluster_illcond(m: int, Q: int, seed: int, cond_modes: float = 100.0,
                         soft_modes: int = 0, g_std: float = 0.05,
                         p_incl: float = 0.3) -> Cluster:
    """An RVE cluster whose mode gradients span the same kind of space as
    ``make_cluster``'s but in an ill-conditioned basis: ``G = G0 M`` with
    ``G0`` drawn as in ``make_cluster(m, Q, seed)`` and ``M = U diag(s) V^T``,
    ``U, V`` random orthogonal (QR of standard-normal matrices with the signs
    of R's diagonal fixed) and ``s`` geometric from 1 down to
    ``1 / cond_modes``.  The mode-space stiffness then has a condition number
    of about ``cond_modes**2`` times that of ``G0``'s (real POD mode gradients
    are far from orthogonal in the weighted gradient inner product).  The
    mixing draws come from ``default_rng(seed + 7919)`` after ``G0``'s.

    With ``soft_modes = k > 0`` the last k columns of ``G0`` are first
    localised in the matrix phase: set to zero at the inclusion points and
    re-centred with the weighted mean over the matrix points only (so that
    ``sum_q w_q G_qm = 0`` still holds).  With a soft matrix and stiff
    inclusions those modes are soft, and the mode-space stiffness is
    ill-conditioned through the material, whatever the basis."""
    base = make_cluster(m, Q, seed, g_std=g_std, p_incl=p_incl)
    G0 = base.G.copy()
    if soft_modes > 0:
        mat = base.phase == 0
        wm = np.where(mat, base.w, 0.0)
        cols = slice(m - soft_modes, m)
        Gs = np.where(mat[:, None, None], G0[:, :, cols], 0.0)
        mean = np.tensordot(wm, Gs, axes=(0, 0)) / wm.sum()
        G0[:, :, cols] = np.where(mat[:, None, None], Gs - mean[None], 0.0)
    rng = np.random.default_rng(seed + 7919)

    def orth(n):
        q, r = np.linalg.qr(rng.standard_normal((n, n)))
        return q * np.sign(np.diag(r))[None, :]

    U, V = orth(m), orth(m)
    s = np.geomspace(1.0, 1.0 / cond_modes, m) if m > 1 else np.ones(1)
    M = (U * s[None, :]) @ V.T
    G = np.ascontiguousarray(np.einsum("qim,mn->qin", G0, M))
    return Cluster(m=m, Q=Q, G=G, w=base.w, phase=base.phase, seed=seed)


def _rotations(rng: np.random.Generator, n: int, max_angle: float) -> np.ndarray:
    axis = rng.standard_normal((n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    ang = rng.uniform(-max_angle, max_angle, size=n)
    K = np.zeros((n, 3, 3))
    K[:, 0, 1], K[:, 0, 2] = -axis[:, 2], axis[:, 1]
    K[:, 1, 0], K[:, 1, 2] = axis[:, 2], -axis[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -axis[:, 1], axis[:, 0]
    s = np.sin(ang)[:, None, None]
    c = np.cos(ang)[:, None, None]
    return np.eye(3)[None] + s * K + (1.0 - c) * (K @ K)


def _sym_from_upper(u6: np.ndarray) -> np.ndarray:
    n = u6.shape[0]
    H = np.zeros((n, 3, 3))
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for k, (i, j) in enumerate(iu):
        H[:, i, j] = u6[:, k]
        H[:, j, i] = u6[:, k]
    return H


def make_macro_points(N: int, seed: int, amp: float = 0.05,
                      max_angle: float = 0.3):
    """Draw ``N`` macro deformation gradients ``Fbar = R (I + H)``.

    Returns ``(Fbar, R, H)``, each ``[N, 3, 3]``.
    """
    rng = np.random.default_rng(seed)
    H = _sym_from_upper(rng.uniform(-amp, amp, size=(N, 6)))
    R = _rotations(rng, N, max_angle)
    Fbar = R @ (np.eye(3)[None] + H)
    return np.ascontiguousarray(Fbar), R, H


def make_increments(R: np.ndarray, n_iter: int, seed: int,
                    amp: float = 0.005) -> np.ndarray:
    """Monolithic-iteration increments ``dFbar_k = R dH_k``: ``[n_iter, N, 3, 3]``."""
    rng = np.random.default_rng(seed)
    N = R.shape[0]
    out = np.empty((n_iter, N, 3, 3))
    for k in range(n_iter):
        dH = _sym_from_upper(rng.uniform(-amp, amp, size=(N, 6)))
        out[k] = R @ dH
    return out


def make_load_path(N: int, seed: int, amp: float = 0.03, levels=(0.25, 0.5, 0.75, 1.0, 0.6, 0.2),
                   max_angle: float = 0.3):
    """A load-unload path of macro states ``Fbar_k = R (I + t_k H)``, ``[K, N, 3, 3]``,
    with ``H`` symmetric U(-amp, amp) and ``R`` drawn as in ``make_macro_points``,
    ``t_k`` the given levels (rising, then falling)."""
    _, R, H = make_macro_points(N, seed, amp=amp, max_angle=max_angle)
    t = np.asarray(levels, dtype=np.float64)
    return np.ascontiguousarray(R[None] @ (np.eye(3)[None, None] + t[:, None, None, None] * H[None]))


def zipf_counts(total: int, n: int, s: float) -> list[int]:
    """Deterministic largest-remainder split of ``total`` in proportion k^-s."""
    p = np.array([(k + 1) ** (-s) for k in range(n)])
    p /= p.sum()
    raw = p * total
    base = np.floor(raw).astype(np.int64)
    rem = total - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    return [int(x) for x in base]


def make_snapshots(p: int, m: int, seed: int, amp: float = 0.05, a_std: float = 0.02):
    """Training snapshots for the empirical cubature: RVE-frame macro inputs
    ``Fr = I + H`` (``H`` symmetric, entries uniform in +-amp), ``[p, 9]``,
    and mode coefficients ``a ~ N(0, a_std^2)``, ``[p, m]``."""
    rng = np.random.default_rng(seed)
    H = _sym_from_upper(rng.uniform(-amp, amp, size=(p, 6)))
    Fr = (np.eye(3)[None] + H).reshape(p, 9)
    a = rng.normal(0.0, a_std, size=(p, m))
    return np.ascontiguousarray(Fr), np.ascontiguousarray(a)


def make_strain_field(N: int, seed: int, n_groups: int = 12, amp: float = 0.05,
                      spread: float = 0.15):
    """Macro strain states ``[N, 6]`` (Voigt xx yy zz xy yz xz) standing in
    for the surrogate macro simulation of the clustered training: ``n_groups``
    loading directions (normal, unit length), each point one of them (uniform
    draw) scaled by ``amp`` times U(0.2, 1) and perturbed by ``spread`` times
    ``amp`` times a standard normal vector."""
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n_groups, 6))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    g = rng.integers(0, n_groups, size=N)
    t = rng.uniform(0.2, 1.0, size=N)
    E = amp * (t[:, None] * D[g] + spread * rng.standard_normal((N, 6)))
    return np.ascontiguousarray(E)


def init_indices(N: int, k: int, seed: int):
    """``k`` distinct point indices for the initial k-means centres."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=k, replace=False)).astype(np.int32)


def make_pod_snapshots(nd: int, s_el: int, s_in: int, seed: int, n_in: int = 12,
                       yield_frac: float = 0.5):
    """Displacement snapshots ``[nd, s]`` with the structure of the POD
    training: elastic snapshots ``X_el = L E`` (``L`` a random ``[nd, 6]``
    response to the six unit strains, ``E`` random strain states) and
    inelastic ones ``X_inel = L E' + P g(E')``, where ``P`` is a random
    ``[nd, n_in]`` block and ``g`` takes the part of ``n_in`` random
    projections of ``E'`` beyond a threshold (zero below it).  Returns
    ``(X_el, X_inel, L, P)``."""
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((nd, 6)) / np.sqrt(nd)
    P = rng.standard_normal((nd, n_in)) / np.sqrt(nd)
    E = rng.uniform(-1.0, 1.0, size=(6, s_el))
    E2 = rng.uniform(-1.0, 1.0, size=(6, s_in))
    A = rng.standard_normal((n_in, 6))
    proj = A @ E2
    g = np.sign(proj) * np.maximum(np.abs(proj) - yield_frac, 0.0)
    return (np.ascontiguousarray(L @ E), np.ascontiguousarray(L @ E2 + P @ g),
            np.ascontiguousarray(L), np.ascontiguousarray(P))


def perturbed_theta(seed: int, rel: float = 0.1):
    """Target parameters ``theta* = theta (1 + rel s)`` with seeded signs ``s``."""
    rng = np.random.default_rng(seed)
    s = np.where(rng.random(4) < 0.5, -1.0, 1.0)
    return THETA_REF * (1.0 + rel * s), s


# The five synthetic workloads: sizes, ROM mode count m and ECM point count Q.
WORKLOADS = {
    "fp64_small": dict(N=256, m=8, Q=32, amp=0.05, seed=1000),
    "fp64_scale": dict(N=65536, m=32, Q=256, amp=0.05, seed=2000, iters=5,
                       inc_amp=0.005),
    "batched": dict(N=262144, ms=[8, 16, 24, 32, 48, 64, 80, 96], q_per_m=6,
                    zipf_s=1.1, amp=0.05, seed=3000, iters=10, inc_amp=0.005),
    "mixed": dict(N=131072, m=64, Q=512, amps=[0.01, 0.05, 0.2], seed=4000),
    "adjoint": dict(N=65536, m=48, Q=384, amp=0.05, seed=5000, rel=0.1),
    # empirical cubature: M candidate points, p training snapshots (30
    # trajectories x 2 load levels), mt selected points (Sec. 3.3, the sizes
    # of the paper's second example: 30 modes, 500 points)
    "ecm": dict(m=30, M=32768, p=60, mt=500, amp=0.05, seed=6000),
    # clustered training: the macro strain states of 262144 points in 30
    # clusters (the paper's first two examples); POD of 16384-dof snapshots
    "training": dict(N=262144, k=30, n_groups=12, seed=7000, nd=16384, s_el=60, s_in=240,
                     n_el=6, n_inel=24),
}
