"""Thin ctypes binding of ``libhrom.so`` (the C ABI declared in include/hrom.h).

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of the library.  Tensors are torch CUDA tensors (device memory and
streams are torch's), in the layouts of the C ABI: per-point arrays are
component-major ``[k, N]`` float64, mode-indexed arrays are 1-D with one
``[m_c, count_c]`` block per cluster.

The library must have been built (``python -m paper_2306_02687_amd.build``);
loading raises if it is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# HROM_LIB: load another build of the library (e.g. the host-sanitizer build
# of oracle/check_sanitizers.sh) instead of the in-tree one
LIB_PATH = os.environ.get("HROM_LIB", os.path.join(_HERE, "libhrom.so"))

HROM_OK = 0
PT_JNONPOS, PT_NOT_SPD, PT_NOCONV, PT_NONFINITE, PT_NOREFINE = 1, 2, 4, 8, 16
FP64, MIXED_BF16, MIXED_FP16 = 0, 1, 2
OBJECTIVE, SPLIT, REFINE, J2, BIOT6 = 1, 2, 4, 8, 16
OFF_A, OFF_KAA, OFF_KAF = 0, 1, 2
VK_TANGENT, VK_KIN, VK_CONDENSE = 0, 1, 2

EXPORTED = ("hrom_plan_create", "hrom_plan_destroy", "hrom_plan_offset", "hrom_eval",
            "hrom_condense", "hrom_update", "hrom_newton", "hrom_backward", "hrom_strerror",
            "hrom_num_variants", "hrom_plan_set_variant", "hrom_plan_profile",
            "hrom_plan_tangent_ms", "hrom_cauchy", "hrom_newton_noalloc",
            "hrom_noalloc_scratch_bytes", "hrom_commit", "hrom_history", "hrom_biot",
            "hrom_ecm_training", "hrom_ecm_svd", "hrom_ecm_select", "hrom_training_clusters",
            "hrom_training_paths", "hrom_pod", "hrom_num_kernel_variants",
            "hrom_plan_set_kernel_variant")
E_SCRATCH, E_NOCONV, E_RANK = -6, -7, -8


class HromError(RuntimeError):
    pass


class _Cluster(C.Structure):
    _fields_ = [("m", C.c_int32), ("Q", C.c_int32), ("G", C.c_void_p), ("w", C.c_void_p),
                ("phase", C.c_void_p), ("first", C.c_int64), ("count", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libhrom.so and declare the C signatures (raises if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HromError(f"{path} not found: build it with `python -m paper_2306_02687_amd.build`")
    L = C.CDLL(path)
    P, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.hrom_plan_create.argtypes = [C.POINTER(P), C.POINTER(_Cluster), i32, i64, i32, C.c_uint32]
    L.hrom_plan_create.restype = C.c_int
    L.hrom_plan_destroy.argtypes = [P]
    L.hrom_plan_offset.argtypes = [P, i32, i32]
    L.hrom_plan_offset.restype = i64
    L.hrom_eval.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
    L.hrom_condense.argtypes = [P, P, P, P, P, P]
    L.hrom_update.argtypes = [P, P, d, P, P, P]
    L.hrom_newton.argtypes = [P, P, P, P, d, i32, P, P, P, P, P]
    L.hrom_backward.argtypes = [P, P, P, P, P, P, P, P]
    L.hrom_cauchy.argtypes = [P, P, P, P, P]
    L.hrom_num_variants.argtypes = []
    L.hrom_num_variants.restype = i32
    L.hrom_plan_set_variant.argtypes = [P, i32, i32]
    L.hrom_num_kernel_variants.argtypes = [i32]
    L.hrom_num_kernel_variants.restype = i32
    L.hrom_plan_set_kernel_variant.argtypes = [P, i32, i32, i32]
    L.hrom_plan_profile.argtypes = [P, i32]
    L.hrom_plan_tangent_ms.argtypes = [P, C.POINTER(C.c_float)]
    L.hrom_newton_noalloc.argtypes = [C.POINTER(_Cluster), i32, i64, i32, C.c_uint32, P, P, P, d,
                                      i32, P, P, P, P, P]
    L.hrom_newton_noalloc.restype = C.c_int
    L.hrom_noalloc_scratch_bytes.argtypes = []
    L.hrom_noalloc_scratch_bytes.restype = C.c_size_t
    L.hrom_commit.argtypes = [P, P]
    L.hrom_biot.argtypes = [P, P, P, P, P]
    L.hrom_history.argtypes = [P, i32, P, P]
    L.hrom_ecm_training.argtypes = [i32, i32, P, P, P, P, i32, P, P, P, P, C.POINTER(i32), P]
    L.hrom_ecm_svd.argtypes = [i32, i32, P, i32, P, P, d, i32, i32, C.POINTER(i32), P, P]
    L.hrom_ecm_select.argtypes = [i32, i32, P, d, i32, P, P, C.POINTER(i32), P, i32,
                                  C.POINTER(i32), P]
    L.hrom_training_clusters.argtypes = [i64, i32, P, i32, P, i32, P, P, C.POINTER(i32), P]
    L.hrom_training_paths.argtypes = [i32, P, i32, P, P]
    L.hrom_pod.argtypes = [i32, i32, P, i32, P, i32, i32, P, P, P, P]
    L.hrom_strerror.argtypes = [C.c_int]
    L.hrom_strerror.restype = C.c_char_p
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != HROM_OK:
        raise HromError(f"{what}: {load().hrom_strerror(rc).decode()} ({rc})")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise HromError("expected a contiguous CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


@dataclass
class ClusterSpec:
    """One RVE cluster on the device: G [Q,9,m], w [Q] float64, phase [Q] int32."""
    G: torch.Tensor
    w: torch.Tensor
    phase: torch.Tensor
    count: int

    @property
    def m(self):
        return int(self.G.shape[2])

    @property
    def Q(self):
        return int(self.G.shape[0])


def _cluster_array(clusters):
    arr = (_Cluster * len(clusters))()
    first = 0
    for i, c in enumerate(clusters):
        for t, dt in ((c.G, torch.float64), (c.w, torch.float64), (c.phase, torch.int32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise HromError("cluster arrays must be contiguous CUDA tensors "
                                "(G, w float64; phase int32)")
        arr[i] = _Cluster(c.m, c.Q, c.G.data_ptr(), c.w.data_ptr(), c.phase.data_ptr(),
                          first, c.count)
        first += c.count
    return arr


def _flags(objective, split, refine, j2=False, biot6=False):
    return ((OBJECTIVE if objective else 0) | (SPLIT if split else 0) | (REFINE if refine else 0)
            | (J2 if j2 else 0) | (BIOT6 if biot6 else 0))


def newton_noalloc(clusters, theta, Fbar, a, Pbar, Cbar, rnorm, status, precision: int = FP64,
                   objective: bool = True, split: bool = False, refine: bool = False,
                   tol: float = 1e-10, max_it: int = 6, stream=None, check: bool = True) -> int:
    """hrom_newton_noalloc: plan + micro Newton with every buffer in the
    library's static device scratch (no device allocation).  Returns the C
    return code when check is False, else raises on failure."""
    arr = _cluster_array(list(clusters))
    N = sum(c.count for c in clusters)
    rc = load().hrom_newton_noalloc(arr, len(clusters), N, precision,
                                    _flags(objective, split, refine), _ptr(theta), _ptr(Fbar),
                                    _ptr(a), float(tol), int(max_it), _ptr(Pbar), _ptr(Cbar),
                                    _ptr(rnorm), _ptr(status), _stream(stream))
    if check:
        _check(rc, "hrom_newton_noalloc")
    return rc


def noalloc_scratch_bytes() -> int:
    return int(load().hrom_noalloc_scratch_bytes())


def ecm_training(G, w, phase, theta, Fr, a, stream=None):
    """hrom_ecm_training: training matrix x_f [p (m + 9), M] and the integrals
    fint [p (m + 9)] from the candidates (G [M, 9, m], w [M] float64, phase [M]
    int32), theta [4] and the snapshots Fr [p, 9], a [p, m].  Returns
    (xf, fint, nbad)."""
    M, _, m = G.shape
    p = Fr.shape[0]
    xf = torch.empty((p * (m + 9), M), dtype=torch.float64, device=G.device)
    fint = torch.empty(p * (m + 9), dtype=torch.float64, device=G.device)
    nbad = C.c_int32(0)
    _check(load().hrom_ecm_training(m, M, _ptr(G), _ptr(w), _ptr(phase), _ptr(theta), p, _ptr(Fr),
                                    _ptr(a), _ptr(xf), _ptr(fint), C.byref(nbad), _stream(stream)),
           "hrom_ecm_training")
    return xf, fint, nbad.value


SVD_AUTO, SVD_DIRECT, SVD_QR = 0, 1, 2


def ecm_svd(xf, r, tol=0.0, max_sweeps=0, stream=None, check=True, history=None, method=SVD_AUTO):
    """hrom_ecm_svd: the r leading left singular vectors of x_f^T, lam [M, r],
    and all singular values sigma [P].  Returns (lam, sigma, sweeps, rc); a
    list passed as history receives the largest relative off-diagonal Gram
    entry of every sweep.  method: SVD_DIRECT sweeps x_f^T itself, SVD_QR
    sweeps the factor R of a Householder QR first, SVD_AUTO picks QR for tall
    matrices."""
    P, M = xf.shape
    lam = torch.empty((M, max(r, 0)), dtype=torch.float64, device=xf.device)
    sigma = torch.empty(P, dtype=torch.float64, device=xf.device)
    sweeps = C.c_int32(0)
    nh = max_sweeps if max_sweeps > 0 else 40
    hist = (C.c_double * nh)()
    rc = load().hrom_ecm_svd(P, M, _ptr(xf), r, _ptr(lam) if r > 0 else None, _ptr(sigma),
                             float(tol), int(max_sweeps), int(method), C.byref(sweeps),
                             C.cast(hist, C.c_void_p), _stream(stream))
    if check:
        _check(rc, "hrom_ecm_svd")
    if history is not None:
        history.extend(hist[:sweeps.value])
    return lam, sigma, sweeps.value, rc


def ecm_select(lam, V0, mt, trace_cap=0, stream=None, check=True):
    """hrom_ecm_select: Box 1 greedy on lam [M, r].  Returns (z, w, info) with
    z [n] int32 candidate indices in pick order, w [n] weights and info a dict
    of iters, rc and (trace_cap > 0) trace [iters, 4]: picked, nnls, dropped, n."""
    M, r = lam.shape
    dev = lam.device
    z = torch.zeros(max(mt, 1), dtype=torch.int32, device=dev)
    w = torch.zeros(max(mt, 1), dtype=torch.float64, device=dev)
    trace = torch.zeros((trace_cap, 4), dtype=torch.int32, device=dev) if trace_cap else None
    n, it = C.c_int32(0), C.c_int32(0)
    rc = load().hrom_ecm_select(M, r, _ptr(lam) if r > 0 else None, float(V0), int(mt), _ptr(z),
                                _ptr(w), C.byref(n), _ptr(trace), int(trace_cap), C.byref(it),
                                _stream(stream))
    if check:
        _check(rc, "hrom_ecm_select")
    info = dict(iters=it.value, rc=rc)
    if trace is not None:
        info["trace"] = trace[:min(it.value, trace_cap)]
    return z[:n.value], w[:n.value], info


class Plan:
    """A plan for N macro points partitioned into RVE clusters (in order)."""

    def __init__(self, clusters, precision: int = FP64, objective: bool = True,
                 split: bool | None = None, refine: bool = False, j2: bool = False,
                 biot6: bool = False):
        """split defaults to True for the mixed precisions (which require it);
        j2 selects J2 plasticity with history (theta of 8 values); biot6 the
        six-component condensation of the symmetric stretch."""
        L = load()
        if split is None:
            split = precision != FP64
        self.clusters = list(clusters)
        self.N = sum(c.count for c in self.clusters)
        arr = _cluster_array(self.clusters)
        flags = _flags(objective, split, refine, j2, biot6)
        h = C.c_void_p()
        torch.cuda.synchronize()
        _check(L.hrom_plan_create(C.byref(h), arr, len(self.clusters), self.N, precision, flags),
               "hrom_plan_create")
        self._h = h
        # Counts the calls that change the plan's stored state (eval, update,
        # newton); an adjoint taken later checks it to know whether the state
        # of its forward solve is still the stored one.
        self.generation = 0
        self.precision = precision
        self.objective = objective
        self.split = split
        self.j2 = j2
        self.a_len = int(L.hrom_plan_offset(h, len(self.clusters), OFF_A))
        self.off_a = [int(L.hrom_plan_offset(h, i, OFF_A)) for i in range(len(self.clusters))]
        self.off_kaa = [int(L.hrom_plan_offset(h, i, OFF_KAA)) for i in range(len(self.clusters))]
        self.off_kaf = [int(L.hrom_plan_offset(h, i, OFF_KAF)) for i in range(len(self.clusters))]
        self.kaa_len = int(L.hrom_plan_offset(h, len(self.clusters), OFF_KAA))
        self.kaf_len = int(L.hrom_plan_offset(h, len(self.clusters), OFF_KAF))

    def close(self):
        if getattr(self, "_h", None):
            load().hrom_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ allocation helpers
    def _dev(self):
        return self.clusters[0].G.device

    def zeros_points(self, k):
        return torch.zeros((k, self.N), dtype=torch.float64, device=self._dev())

    def zeros_modes(self):
        return torch.zeros(self.a_len, dtype=torch.float64, device=self._dev())

    def status(self):
        return torch.zeros(self.N, dtype=torch.int32, device=self._dev())

    def set_variant(self, variant: int, cluster: int = -1):
        _check(load().hrom_plan_set_variant(self._h, int(cluster), int(variant)),
               "hrom_plan_set_variant")

    def set_kernel_variant(self, kind: int, variant: int, cluster: int = -1):
        """Launch variant of the kinematics (VK_KIN), the condensation
        (VK_CONDENSE) or the tangent (VK_TANGENT) of one cluster or all."""
        _check(load().hrom_plan_set_kernel_variant(self._h, int(kind), int(cluster), int(variant)),
               "hrom_plan_set_kernel_variant")

    @staticmethod
    def num_kernel_variants(kind: int) -> int:
        return int(load().hrom_num_kernel_variants(int(kind)))

    def profile(self, enable: bool = True):
        """Record HIP events around the tangent contraction of every eval."""
        _check(load().hrom_plan_profile(self._h, 1 if enable else 0), "hrom_plan_profile")

    def tangent_ms(self) -> float:
        """Duration of the last recorded tangent launch (waits for it)."""
        v = C.c_float()
        _check(load().hrom_plan_tangent_ms(self._h, C.byref(v)), "hrom_plan_tangent_ms")
        return float(v.value)

    @staticmethod
    def num_variants() -> int:
        return int(load().hrom_num_variants())

    # ------------------------------------------------------------ entry points
    def eval(self, theta, Fbar, a, status, r=None, Pr=None, Kaa=None, KaF=None, KFF=None,
             stream=None):
        self.generation += 1
        _check(load().hrom_eval(self._h, _ptr(theta), _ptr(Fbar), _ptr(a), _ptr(r), _ptr(Pr),
                                _ptr(Kaa), _ptr(KaF), _ptr(KFF), _ptr(status), _stream(stream)),
               "hrom_eval")

    def condense(self, Pbar, Cbar, rnorm, status, stream=None):
        _check(load().hrom_condense(self._h, _ptr(Pbar), _ptr(Cbar), _ptr(rnorm), _ptr(status),
                                    _stream(stream)), "hrom_condense")

    def update(self, dFbar, a, status, tol=0.0, stream=None):
        self.generation += 1
        _check(load().hrom_update(self._h, _ptr(dFbar), float(tol), _ptr(a), _ptr(status),
                                  _stream(stream)), "hrom_update")

    def newton(self, theta, Fbar, a, Pbar, Cbar, rnorm, status, tol=1e-10, max_it=6,
               stream=None):
        self.generation += 1
        _check(load().hrom_newton(self._h, _ptr(theta), _ptr(Fbar), _ptr(a), float(tol),
                                  int(max_it), _ptr(Pbar), _ptr(Cbar), _ptr(rnorm), _ptr(status),
                                  _stream(stream)), "hrom_newton")

    def cauchy(self, sigma, dsdD, status, stream=None):
        """Cauchy stress [9][N] and Updated-Lagrangian tangent [81][N] (or None)
        of the last condensed state."""
        _check(load().hrom_cauchy(self._h, _ptr(sigma), _ptr(dsdD), _ptr(status), _stream(stream)),
               "hrom_cauchy")

    def biot(self, T, CB, status, stream=None):
        """Biot stress T [6][N] and tangent CB [36][N] (or None), Voigt order."""
        _check(load().hrom_biot(self._h, _ptr(T), _ptr(CB), _ptr(status), _stream(stream)),
               "hrom_biot")

    def commit(self, stream=None):
        """J2 plans: the history of the last evaluation becomes the committed one."""
        _check(load().hrom_commit(self._h, _stream(stream)), "hrom_commit")

    def history(self, which: int = 0, stream=None):
        """J2 plans: committed (0) or last-evaluated (1) history as a list of
        per-cluster [count, Q, 7] tensors."""
        n = sum(c.count * c.Q * 7 for c in self.clusters)
        out = torch.empty(n, dtype=torch.float64, device=self._dev())
        _check(load().hrom_history(self._h, int(which), _ptr(out), _stream(stream)), "hrom_history")
        res, off = [], 0
        for c in self.clusters:
            k = c.count * c.Q * 7
            res.append(out[off:off + k].view(c.count, c.Q, 7))
            off += k
        return res

    def backward(self, theta, a, gPbar, gFbar, gtheta, status, stream=None):
        _check(load().hrom_backward(self._h, _ptr(theta), _ptr(a), _ptr(gPbar), _ptr(gFbar),
                                    _ptr(gtheta), _ptr(status), _stream(stream)), "hrom_backward")


def training_clusters(E, k, init_idx, max_iter=100, stream=None, check=True):
    """hrom_training_clusters: E [d, N] strain states (component-major),
    init_idx [k] int32.  Returns (centres [k, d], labels [N] int32, iters, rc)."""
    d, N = E.shape
    centres = torch.empty((k, d), dtype=torch.float64, device=E.device)
    labels = torch.empty(N, dtype=torch.int32, device=E.device)
    it = C.c_int32(0)
    rc = load().hrom_training_clusters(N, d, _ptr(E), k, _ptr(init_idx), int(max_iter), _ptr(centres),
                                       _ptr(labels), C.byref(it), _stream(stream))
    if check:
        _check(rc, "hrom_training_clusters")
    return centres, labels, it.value, rc


def training_paths(centres, n_steps, stream=None):
    """hrom_training_paths: Fr [k n_steps, 9] from centres [k, 6]."""
    k = centres.shape[0]
    Fr = torch.empty((k * n_steps, 9), dtype=torch.float64, device=centres.device)
    _check(load().hrom_training_paths(k, _ptr(centres), int(n_steps), _ptr(Fr), _stream(stream)),
           "hrom_training_paths")
    return Fr


def pod(X_el, X_in, n_el, n_in, stream=None, check=True):
    """hrom_pod: X_el [s_el, nd], X_in [s_in, nd] snapshots (one per row).
    Returns (Phi [nd, n_el + n_in], sigma_el, sigma_in, rc)."""
    s_el, nd = X_el.shape
    s_in = X_in.shape[0]
    Phi = torch.empty((nd, n_el + n_in), dtype=torch.float64, device=X_el.device)
    sel = torch.empty(s_el, dtype=torch.float64, device=X_el.device)
    sin = torch.empty(s_in, dtype=torch.float64, device=X_el.device)
    rc = load().hrom_pod(nd, s_el, _ptr(X_el), s_in, _ptr(X_in), int(n_el), int(n_in), _ptr(Phi),
                         _ptr(sel), _ptr(sin), _stream(stream))
    if check:
        _check(rc, "hrom_pod")
    return Phi, sel, sin, rc
