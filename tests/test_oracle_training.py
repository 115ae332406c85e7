"""Pins of the clustered-training oracle (Sec. 3.4, Box 2) and of the POD
basis with the elastic-inelastic split (Sec. 3.2.1, eqs. SVD_displacement and
snapshots_displacement):

* k-means: the closed form of a one-dimensional two-cluster case; recovery of
  well-separated blobs (labels up to the blob order, centres = blob means);
  at convergence every centre is the mean of its points and every point is
  nearest to its own centre; the within-cluster sum of squares does not
  increase from one iteration to the next; the normalised clustering does not
  change when a strain component is given other units;
* trajectories: Fr = I + t H(c), symmetric, linear in t, ending at the centre;
* POD: the elastic modes span the exact response space of rank-6 elastic
  snapshots, the modes are orthonormal with the inelastic ones orthogonal to
  the elastic ones, the inelastic snapshots are reproduced exactly once
  n_inel reaches the rank of their non-elastic part, and otherwise the
  residual is the root sum of squares of the discarded singular values
  (Eckart-Young).
"""
import numpy as np

from hrom_inputs import init_indices, make_pod_snapshots, make_strain_field


def test_kmeans_one_dimensional_closed_form(orc):
    X = np.array([[-3.0], [-2.0], [-1.0], [1.0], [2.0], [3.0]])
    C, lab, it = orc.kmeans(X, np.array([[-3.0], [3.0]]))
    assert np.allclose(C, [[-2.0], [2.0]]) and lab.tolist() == [0, 0, 0, 1, 1, 1]


def test_kmeans_recovers_separated_blobs(orc):
    rng = np.random.default_rng(8800)
    centres = np.array([[0.0, 0.0], [10.0, 0.0], [0.0, 10.0]])
    truth = rng.integers(0, 3, size=300)
    X = centres[truth] + rng.normal(0.0, 0.5, size=(300, 2))
    init = np.array([np.flatnonzero(truth == c)[0] for c in range(3)])
    C, lab, it = orc.kmeans(X, X[init])
    assert (lab == truth).all()
    for c in range(3):
        assert np.allclose(C[c], X[truth == c].mean(axis=0), rtol=0, atol=1e-14)


def _inertia(X, C, lab):
    return float(((X - C[lab]) ** 2).sum())


def test_kmeans_fixed_point_and_monotone(orc):
    E = make_strain_field(4000, 8810, n_groups=6)
    idx = init_indices(4000, 8, 8811)
    C, lab, it = orc.kmeans(E, E[idx], max_iter=200)
    assert it < 200
    for c in range(8):
        assert np.allclose(C[c], E[lab == c].mean(axis=0), rtol=0, atol=1e-15)
    d2 = ((E[:, None, :] - C[None]) ** 2).sum(axis=2)
    assert (d2[np.arange(4000), lab] <= d2.min(axis=1) + 1e-18).all()
    prev = np.inf
    for n in range(1, it + 1):
        Cn, labn, _ = orc.kmeans(E, E[idx], max_iter=n)
        # the assignment of iteration n against the centres it produced
        J = _inertia(E, Cn, labn)
        assert J <= prev * (1 + 1e-12)
        prev = J


def test_normalised_clustering_unit_invariance(orc):
    E = make_strain_field(3000, 8820)
    idx = init_indices(3000, 10, 8821)
    C1, lab1, _ = orc.training_clusters(E, 10, idx)
    S = np.array([1.0, 1.0, 1.0, 1000.0, 1.0, 0.01])
    C2, lab2, _ = orc.training_clusters(E * S, 10, idx)
    assert (lab1 == lab2).all()
    assert np.allclose(C2, C1 * S, rtol=1e-12, atol=0)


def test_training_paths(orc):
    C = np.array([[0.01, -0.02, 0.005, 0.003, -0.004, 0.002]])
    F = orc.training_paths(C, 4).reshape(4, 3, 3)
    H = F[-1] - np.eye(3)
    assert np.allclose(H, H.T, atol=0)
    assert np.allclose([H[0, 0], H[1, 1], H[2, 2], H[0, 1], H[1, 2], H[0, 2]], C[0], atol=1e-17)
    for j in range(4):
        assert np.allclose(F[j] - np.eye(3), (j + 1) / 4 * H, atol=1e-17)


def test_pod_split(orc):
    X_el, X_in, L, P = make_pod_snapshots(400, 30, 80, 8830, n_in=10)
    Phi, s_el, s_in = orc.pod_split(X_el, X_in, 6, 10)
    assert np.allclose(Phi.T @ Phi, np.eye(16), atol=1e-13)
    Ql, _ = np.linalg.qr(L)
    el = Phi[:, :6]
    assert np.linalg.norm(el - Ql @ (Ql.T @ el), 2) < 1e-13     # span Phi_el = span L
    assert s_el[6] < 1e-13 * s_el[0]                              # rank 6
    assert np.abs(Phi[:, 6:].T @ el).max() < 1e-13
    rec = X_in - Phi @ (Phi.T @ X_in)
    assert np.linalg.norm(rec) < 1e-12 * np.linalg.norm(X_in)    # rank of P g(E') <= 10
    Phi5, _, s5 = orc.pod_split(X_el, X_in, 6, 5)
    rec5 = X_in - Phi5 @ (Phi5.T @ X_in)
    assert abs(np.linalg.norm(rec5) - np.sqrt((s5[5:] ** 2).sum())) < 1e-12 * np.linalg.norm(X_in)
