#!/usr/bin/env python3
"""Benchmark of the hyper-reduced RVE evaluation on one MI355X.

One step = one pass of the whole hot path over every macro point of the
workload: polar split, reduced kinematics, Neo-Hooke stress and tangent at
every ECM point, the ECM sums (r, Kaa, KaF, KFF, Pbar), Cholesky
condensation with the objective push-out (Pbar_alg, Cbar), the adjoint
backward (dL/dFbar, dL/dtheta) and the monolithic update of the ROM
amplitudes.  Inputs are resident in HBM before the timed region.

Default workload: 131,072 macro points, m = 64 ROM modes, Q = 512 ECM points,
mixed precision (BF16 MFMA with hi/lo split operands, FP32 tangent, FP64
kinematics / residual / factorisation / condensation).  The same step on the
plain FP64 path is timed beside it; one JSON line goes to stdout.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision bf16|fp16|fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RVE point-evals/s (m=64,Q=512) mixed vs FP64 at 1e-5 rel; % MFMA roofline"
PEAK = {"bf16": 2.5e15, "fp16": 2.5e15, "fp64": 78.6e12}
PREC = {"fp64": 0, "bf16": 1, "fp16": 2}
HBM_PEAK = 8.0e12
# Updated-Lagrangian output per point: reads the polar split (21), Palg_r (9)
# and Cr (81) doubles, writes sigma (9) and dsigma/dD (81)
CAUCHY_BYTES_PER_POINT = 8 * (21 + 9 + 81 + 9 + 81)


def eval_flops_per_point(m: int, Q: int) -> float:
    """Algorithmic flops of the evaluation kernel per macro point (FMA = 2):
    Kaa = G^T (wA) G: 18 Q m^2; T = (wA) G: 162 Q m; kinematics F_q and the
    residual r: 36 Q m; Neo-Hooke P and A: about 600 per ECM point."""
    return 18.0 * Q * m * m + 162.0 * Q * m + 36.0 * Q * m + 600.0 * Q


def step_flops_per_point(m: int, Q: int) -> float:
    """Whole step: evaluation + factor/solves (m^3/3 + 20 m^2) + adjoint
    re-evaluation (F_q, G lambda: 36 Q m; A v and dtheta: ~300 Q)."""
    return eval_flops_per_point(m, Q) + m ** 3 / 3.0 + 20.0 * m * m + 36.0 * Q * m + 300.0 * Q


def tangent_flops_per_point(m, Q):
    """Algorithmic flops of the tangent contraction per macro point (Sec. 3.2.1,
    eq. ROMstiffness), per ECM point: T_q = (w_q A_q) G_q (162 m) and
    Kaa += G_q^T T_q (18 m^2).  KaF = sum_q T_q^T needs no product of its own
    (A_q is major-symmetric) and KFF = sum_q w_q A_q is a sum, so neither is
    counted, even though the kernel forms them on the matrix cores."""
    return 18.0 * Q * m * m + 162.0 * Q * m


def read_traffic(kernel_tag: str, variant: int):
    """HBM bytes per launch of the given launch variant from a committed
    counter summary (lines ``traffic_bytes_per_launch[variant=v]: X``), if present."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch\[variant=%d\]:\s*([0-9.eE+]+)" % int(variant), txt)
    return float(m.group(1)) if m else None


def read_cauchy_traffic(m, Q):
    """HBM bytes per launch of the Updated-Lagrangian output kernel from its
    committed counter summary, if present."""
    path = os.path.join(ROOT, "profiles", f"cauchy_m{m}_q{Q}_traffic.md")
    if not os.path.exists(path):
        return None
    m_ = re.search(r"traffic_bytes_per_launch\[k_cauchy\]:\s*([0-9.eE+]+)", open(path).read())
    return float(m_.group(1)) if m_ else None


def build_inputs(N, m, Q, amp, seed):
    from hrom_inputs import make_cluster, make_macro_points
    cl = make_cluster(m, Q, seed)
    F, _, _ = make_macro_points(N, seed + 1, amp=amp)
    return cl, F


def run_gpu(prec_name, cl, F, N, steps, warmup, split=True, refine=False, biot6=False):
    import torch

    import paper_2306_02687_amd as P
    from hrom_inputs import THETA_REF
    from paper_2306_02687_amd import solve

    from paper_2306_02687_amd import tune

    plan = P.Plan([solve.upload_cluster(cl, N)], precision=PREC[prec_name], split=split,
                  refine=refine and prec_name != "fp64", biot6=biot6)
    th = solve.theta_dev(THETA_REF)
    Fd = solve.points_to_soa(F)
    st = solve.State(plan)
    tuned = tune.autotune(plan, th, Fd, st.a, use_cache=False)
    plan.profile(True)
    tan_ms = []
    # bring the ROM state near convergence (untimed set-up)
    for _ in range(2):
        plan.eval(th, Fd, st.a, st.status)
        plan.condense(st.Pbar, st.Cbar, st.rnorm, st.status)
        plan.update(None, st.a, st.status, tol=0.0)
    g = torch.from_numpy(np.random.default_rng(7).standard_normal((9, N)) * 1e-2).cuda()
    gF = plan.zeros_points(9)
    gth = torch.zeros(4, dtype=torch.float64, device="cuda")

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        plan.eval(th, Fd, st.a, st.status)
        if ev is not None:
            ev[1].record()
        plan.condense(st.Pbar, st.Cbar, st.rnorm, st.status)
        plan.backward(th, st.a, g, gF, gth, st.status)
        plan.update(None, st.a, st.status, tol=0.0)
        if ev is not None:
            # every launch of the step is queued: waiting for the tangent's
            # end event leaves the GPU busy with the rest of the step
            tan_ms.append(plan.tangent_ms())

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    eval_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    # one more forward for the accuracy comparison
    plan.eval(th, Fd, st.a, st.status)
    plan.condense(st.Pbar, st.Cbar, st.rnorm, st.status)
    # Updated-Lagrangian output of the condensed state (not part of the step):
    # ten launches between two events on the launch stream
    sig, dsdD = plan.zeros_points(9), plan.zeros_points(81)
    plan.cauchy(sig, dsdD, st.status)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        plan.cauchy(sig, dsdD, st.status)
    e1.record()
    torch.cuda.synchronize()
    cauchy_ms = e0.elapsed_time(e1) / 10
    del sig, dsdD
    out = dict(wall=wall, eval_ms=eval_ms, tan_ms=float(np.mean(tan_ms)), cauchy_ms=cauchy_ms,
               a=st.a.clone(),
               Pbar=st.Pbar.clone(),
               Cbar=st.Cbar.clone(), status=int(st.status.max().item()),
               variant=tuned["variant"], kin_variant=tuned["kin"], cond_variant=tuned["cond"],
               tune_ms={str(k): v for k, v in tuned["ms"].items()})
    plan.close()
    del st
    torch.cuda.empty_cache()
    return out


def cpu_baseline(cl, F, budget_s=12.0):
    """The oracle (plain C, OpenMP over points) on a bounded sample of the same
    workload: per point one evaluate + condense + adjoint backward."""
    import oracle
    from hrom_inputs import THETA_REF
    rng = np.random.default_rng(11)
    g = rng.standard_normal((F.shape[0], 9)) * 1e-2
    a = np.zeros((F.shape[0], cl.m))
    n0 = 32
    t = time.perf_counter()
    oracle.backward(cl, THETA_REF, F[:n0], a[:n0], g[:n0])
    dt = time.perf_counter() - t
    n = int(min(F.shape[0], max(n0, budget_s / max(dt, 1e-6) * n0)))
    t = time.perf_counter()
    oracle.backward(cl, THETA_REF, F[:n], a[:n], g[:n])
    dt = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return n, dt, threads


def host_cpu():
    """CPU model, logical CPU count and lscpu's socket/core/thread lines of the
    host the oracle ran on."""
    info = {"model": None, "logical_cpus": os.cpu_count()}
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                info["model"] = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keep = ("Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU max MHz", "NUMA node(s)")
        info["lscpu"] = {k.strip(): v.strip() for k, v in
                         (ln.split(":", 1) for ln in out.splitlines() if ":" in ln)
                         if k.strip() in keep}
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def run_batched(args, N=262144, precision="bf16"):
    """Eight uneven RVE clusters (m in {8..96}, Q = 6 m, Zipf(1.1) split of the
    macro points), one HIP graph of 10 monolithic iterations (evaluate,
    condense, update with dFbar_k), mixed and FP64.  Returns the result line."""
    import torch

    import paper_2306_02687_amd as P
    from hrom_inputs import THETA_REF, make_cluster, make_increments, make_macro_points, zipf_counts
    from paper_2306_02687_amd import solve, tune

    K = 10
    ms = [8, 16, 24, 32, 48, 64, 80, 96]
    counts = zipf_counts(N, len(ms), 1.1)
    cls = [make_cluster(m, 6 * m, 3000 + i) for i, m in enumerate(ms)]
    F, R, _ = make_macro_points(N, 3100, amp=0.05)
    dF = make_increments(R, K, 3200, amp=0.005)
    Fk = [F]
    for k in range(K - 1):
        Fk.append(Fk[-1] + dF[k])
    Fd = [solve.points_to_soa(x) for x in Fk]
    dFd = [solve.points_to_soa(x) for x in dF]
    del Fk
    th = solve.theta_dev(THETA_REF)
    res = {}
    for name, prec, split in (("mixed", PREC[precision], True), ("fp64", 0, False)):
        print(f"[bench] batched {name}", file=sys.stderr, flush=True)
        plan = P.Plan([solve.upload_cluster(c, n) for c, n in zip(cls, counts)],
                      precision=prec, split=split)
        a = plan.zeros_modes()
        st = plan.status()
        Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
        rn = torch.zeros(N, dtype=torch.float64, device="cuda")
        tuned = tune.autotune(plan, th, Fd[0], a, use_cache=False)

        def iterations():
            for k in range(K):
                plan.eval(th, Fd[k], a, st)
                plan.condense(Pb, Cb, rn, st)
                plan.update(dFd[k], a, st)

        iterations()   # eager warm-up
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                iterations()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps // 5, 2))
        a.zero_()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            a.zero_()
            g.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[name] = dict(ms_per_graph=dt * 1e3, value=N * K / dt, variant=tuned["variant"],
                         Cbar=Cb.cpu().numpy(), Pbar=Pb.cpu().numpy(),
                         status=int(st.max().item()))
        plan.close()
        torch.cuda.empty_cache()
    eC = (np.linalg.norm(res["mixed"]["Cbar"] - res["fp64"]["Cbar"], axis=0)
          / np.linalg.norm(res["fp64"]["Cbar"], axis=0))
    line = {"metric": "RVE point-evals/s, batched uneven clusters, graph of 10 monolithic iterations",
            "value": res["mixed"]["value"], "unit": "point-evals/s", "n_gpus": 1,
            "ms_per_graph": res["mixed"]["ms_per_graph"], "higher_is_better": True,
            "dtype": f"{precision} MFMAx3 split + fp32 tangent + fp64", "data": "synthetic",
            "config": {"workload": f"{N} macro points over 8 clusters m={ms}, Q=6m, Zipf(1.1) "
                                   f"counts {counts}, 10 monolithic iterations in one HIP graph"},
            "fp64": {"value": res["fp64"]["value"], "ms_per_graph": res["fp64"]["ms_per_graph"]},
            "speedup_mixed_over_fp64": res["fp64"]["ms_per_graph"] / res["mixed"]["ms_per_graph"],
            "mixed_vs_fp64_Cbar_rel_err_max": float(eC.max()),
            "variants": {"mixed": res["mixed"]["variant"], "fp64": res["fp64"]["variant"]},
            "status_max": max(res["mixed"]["status"], res["fp64"]["status"])}
    return line


def run_adjoint(N=65536, m=48, Q=384, precision="bf16", refine=True, newton_its=4):
    """Forward + backward at the adjoint workload's shape: a device-side micro
    Newton of newton_its evaluations (evaluate + condense + update) from a = 0,
    then the adjoint backward of L = sum ||Pbar - Pbar*||^2; ms of each part."""
    import torch

    import paper_2306_02687_amd as P
    from hrom_inputs import THETA_REF, make_cluster, make_macro_points
    from paper_2306_02687_amd import solve

    cl = make_cluster(m, Q, 5000)
    F, _, _ = make_macro_points(N, 5001, amp=0.05)
    Fd = solve.points_to_soa(F)
    plan = P.Plan([solve.upload_cluster(cl, N)], precision=PREC[precision],
                  refine=refine and precision != "fp64")
    th = solve.theta_dev(THETA_REF)
    a = plan.zeros_modes()
    st = plan.status()
    Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(N, dtype=torch.float64, device="cuda")
    target = torch.zeros_like(Pb)
    gF = plan.zeros_points(9)
    gth = torch.zeros(4, dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    times = []
    for rep in range(3):
        a.zero_()
        ev[0].record()
        plan.newton(th, Fd, a, Pb, Cb, rn, st, tol=0.0, max_it=newton_its)
        ev[1].record()
        g = 2.0 * (Pb - target)
        plan.backward(th, a, g, gF, gth, st)
        ev[2].record()
        torch.cuda.synchronize()
        times.append((ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])))
    fwd, bwd = times[-1]
    out = {"workload": f"{N} macro points, m={m}, Q={Q}, {precision}"
                       f"{' split, adjoint refinement' if precision != 'fp64' and refine else ''}: "
                       f"{newton_its} Newton evaluations + one adjoint backward",
           "forward_ms": fwd, "backward_ms": bwd,
           "point_evals_per_s": N * newton_its / (fwd * 1e-3),
           "status_max": int((st & ~4).max().item())}
    plan.close()
    torch.cuda.empty_cache()
    return out


def run_monolithic(N=65536, m=32, Q=256, precision="fp64", iters=5):
    """Five monolithic iterations (evaluate + condense + update with dFbar_k)
    at the FP64-at-scale workload's shape; ms per iteration."""
    import torch

    import paper_2306_02687_amd as P
    from hrom_inputs import THETA_REF, make_cluster, make_increments, make_macro_points
    from paper_2306_02687_amd import solve

    cl = make_cluster(m, Q, 2000)
    F, R, _ = make_macro_points(N, 2001, amp=0.05)
    dF = make_increments(R, iters, 2002, amp=0.005)
    Fd = solve.points_to_soa(F)
    dFd = [solve.points_to_soa(x) for x in dF]
    plan = P.Plan([solve.upload_cluster(cl, N)], precision=PREC[precision])
    th = solve.theta_dev(THETA_REF)
    a = plan.zeros_modes()
    st = plan.status()
    Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(N, dtype=torch.float64, device="cuda")

    def run():
        Fk = Fd.clone()
        for k in range(iters):
            plan.eval(th, Fk, a, st)
            plan.condense(Pb, Cb, rn, st)
            plan.update(dFd[k], a, st)
            Fk += dFd[k]

    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.zero_()
    e0.record()
    run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out = {"workload": f"{N} macro points, m={m}, Q={Q}, {precision}, {iters} monolithic iterations",
           "ms_per_iteration": ms / iters, "point_evals_per_s": N * iters / (ms * 1e-3),
           "status_max": int(st.max().item())}
    plan.close()
    torch.cuda.empty_cache()
    return out


def oracle_errors(m=64, Q=512, n=12, amps=(0.01, 0.05, 0.2), precision="bf16"):
    """Newton-converged Pbar, Cbar of the mixed path against the FP64 oracle
    on n points of the headline shape at each strain amplitude."""
    import oracle
    from hrom_inputs import THETA_REF, make_cluster, make_macro_points
    import paper_2306_02687_amd as P
    from paper_2306_02687_amd import solve

    cl = make_cluster(m, Q, 4000)
    out = {}
    for amp in amps:
        F, _, _ = make_macro_points(n, 4001 + int(amp * 1000), amp=amp)
        ref = oracle.newton(cl, THETA_REF, F, tol=1e-10)
        plan = P.Plan([solve.upload_cluster(cl, n)], precision=PREC[precision])
        st = solve.newton(plan, solve.theta_dev(THETA_REF), solve.points_to_soa(F), tol=1e-10)
        Pg, Cg = solve.soa_to_points(st.Pbar), solve.soa_to_points(st.Cbar)
        plan.close()
        eP = np.linalg.norm(Pg - ref["Pbar"], axis=1) / np.linalg.norm(ref["Pbar"], axis=1)
        eC = (np.linalg.norm(Cg - ref["Cbar"].reshape(n, 81), axis=1)
              / np.linalg.norm(ref["Cbar"].reshape(n, 81), axis=1))
        out[str(amp)] = {"Pbar_max": float(eP.max()), "Cbar_max": float(eC.max())}
    return out


def run_j2(args, quiet=False, precision="fp64"):
    """J2 plasticity (the Example 1 material) at the sizes of the paper's
    Example 1 hyper ROM, m = 8 modes, Q = 250 ECM points, over 262144 macro
    points: a load-unload path of macro states; per state a fixed-count
    device-side micro Newton (evaluate + condense + update) and a commit of
    the history.  precision: fp64, or bf16 / fp16 (split tangent
    contraction; the law, the history and the residual in FP64)."""
    import torch

    import paper_2306_02687_amd as P
    from hrom_inputs import MAT_J2, make_cluster, make_load_path
    from paper_2306_02687_amd import solve

    N = args.N if (args.N != 131072 and args.workload == "j2") else 262144
    m, Q, its = 8, 250, 4
    levels = (0.25, 0.5, 0.75, 1.0, 0.6, 0.2)
    cl = make_cluster(m, Q, 4900)
    path = make_load_path(N, 4901, amp=0.03, levels=levels)
    Fk = [solve.points_to_soa(x) for x in path]
    del path
    plan = P.Plan([solve.upload_cluster(cl, N)], j2=True, precision=PREC[precision])
    plan.profile(True)
    th = solve.theta_dev(MAT_J2)
    a = plan.zeros_modes()
    st = plan.status()
    Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(N, dtype=torch.float64, device="cuda")

    def run_path():
        for F in Fk:
            plan.newton(th, F, a, Pb, Cb, rn, st, tol=0.0, max_it=its)
            plan.commit()

    a.zero_()
    run_path()   # warm-up (also yields the material)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 5)
    t0 = time.perf_counter()
    for _ in range(reps):
        a.zero_()
        run_path()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    evals = N * its * len(levels)
    line = {"metric": "RVE point-evals/s, J2 plasticity with history (Example 1 material)",
            "value": evals / dt, "unit": "point-evals/s", "n_gpus": 1,
            "ms_per_path": dt * 1e3, "higher_is_better": True, "dtype": precision,
            "data": "synthetic",
            "config": {"workload": f"{N} macro points, m={m} ROM modes, Q={Q} ECM points, "
                                   f"load-unload path of {len(levels)} macro states, {its} "
                                   f"Newton evaluations per state, commit after each"},
            # tol 0: every point runs the fixed count (NOCONV, bit 4, set by design)
            "status_max": int((st & ~4).max().item())}
    plan.close()
    torch.cuda.empty_cache()
    if quiet:
        return {k: line[k] for k in ("value", "ms_per_path", "status_max")} | {
            "workload": line["config"]["workload"]}
    print(json.dumps(line), flush=True)


def svd_sweep_flops(P, M):
    """FP64 flops of one sweep of the blocked one-sided Jacobi SVD: every pair
    of 32-column blocks forms its 64 x 64 Gram matrix over the M rows and
    multiplies its 64 columns by the 64 x 64 rotation (2 * 64 * 64 * M each)."""
    nb = max(2, -(-P // 32))
    nb += nb & 1
    pairs_per_sweep = (nb - 1) * (nb // 2)
    return pairs_per_sweep * 2 * (2.0 * 64 * 64 * M)


def svd_flops(P, M, r, sweeps):
    """FP64 flops of hrom_ecm_svd with the library's automatic method: for
    M >= 2 Ppad the Householder QR (2 M P^2 - 2 P^3 / 3), the pivoted QR of
    the P x P factor (4 P^3 / 3), the sweeps over P rows and Q applied to the
    r leading vectors (4 M P r - 2 P^2 r); else the sweeps over the M rows."""
    nb = max(2, -(-P // 32))
    nb += nb & 1
    if M >= 2 * 32 * nb:
        return (2.0 * M * P * P - 2.0 * P ** 3 / 3 + 4.0 * P ** 3 / 3 + sweeps * svd_sweep_flops(P, P)
                + 4.0 * M * P * r - 2.0 * P * P * r)
    return sweeps * svd_sweep_flops(P, M)


def run_ecm(args, quiet=False):
    """The offline stage end to end on the GPU (Box 2 with the empirical
    cubature of Sec. 3.3 and the POD of Sec. 3.2.1), at the sizes of the
    paper's second example, 30 modes and 500 points: the macro strain states
    of 262144 points clustered into 30 training directions (Lloyd's k-means on
    normalised strains), two load levels per direction (60 snapshots), each
    converged by the library's own full-integration Newton over 32768
    candidate points (FP64), then the training matrix, the SVD basis and the
    Box 1 greedy; and the POD with the elastic-inelastic split of 60 + 240
    synthetic 16384-dof displacement snapshots."""
    import torch

    import paper_2306_02687_amd as P
    from hrom_inputs import (THETA_REF, WORKLOADS, init_indices, make_cluster, make_pod_snapshots,
                             make_strain_field)
    from paper_2306_02687_amd import binding as B
    from paper_2306_02687_amd import solve

    wl, wt = WORKLOADS["ecm"], WORKLOADS["training"]
    m, M, mt = wl["m"], wl["M"], wl["mt"]
    Nm, k, n_steps = wt["N"], wt["k"], 2
    p = k * n_steps

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t) * 1e3

    E = torch.from_numpy(make_strain_field(Nm, wt["seed"], n_groups=wt["n_groups"]).T.copy()).cuda()
    idx = torch.from_numpy(init_indices(Nm, k, wt["seed"] + 1)).cuda()
    B.training_clusters(E[:, :4096].contiguous(), 4, idx[:4] % 4096, check=False)   # warm-up
    (C, labels, km_iters, _), t_km = timed(lambda: B.training_clusters(E, k, idx, max_iter=2000))
    Fr_rows, t_paths = timed(lambda: B.training_paths(C, n_steps))
    cl = make_cluster(m, M, wl["seed"])
    spec = solve.upload_cluster(cl, p)
    plan = P.Plan([spec], objective=False)
    th = solve.theta_dev(THETA_REF)
    Fd = Fr_rows.t().contiguous()
    st, t_newton = timed(lambda: solve.newton(plan, th, Fd, tol=1e-12, max_it=25))
    status = int(st.status.max().item())
    a = st.a.t().contiguous()
    plan.close()
    phase = spec.phase.to(torch.int32).contiguous()
    V0 = float(cl.w.sum())
    B.ecm_training(spec.G, spec.w, phase, th, Fr_rows, a)                  # warm-up (code load)
    (xf, fint, nbad), t_tr = timed(lambda: B.ecm_training(spec.G, spec.w, phase, th, Fr_rows, a))
    hist = []
    (lam, sig, sweeps, _), t_svd = timed(lambda: B.ecm_svd(xf, mt - 1, history=hist))
    (z, w, info), t_sel = timed(lambda: B.ecm_select(lam, V0, mt, trace_cap=8 * mt))
    tr = info["trace"].cpu().numpy()
    X_el, X_in, _, _ = make_pod_snapshots(wt["nd"], wt["s_el"], wt["s_in"], wt["seed"] + 2,
                                          n_in=wt["n_inel"])
    Xe = torch.from_numpy(X_el.T.copy()).cuda()
    Xi = torch.from_numpy(X_in.T.copy()).cuda()
    (Phi, _, _, _), t_pod = timed(lambda: B.pod(Xe, Xi, wt["n_el"], wt["n_inel"]))
    Prows = p * (m + 9)
    flops = svd_flops(Prows, M, mt - 1, sweeps)
    sig_h = sig.cpu().numpy()
    res = {"kmeans_ms": t_km, "kmeans_iterations": km_iters, "paths_ms": t_paths,
           "newton_snapshots_ms": t_newton, "training_ms": t_tr, "svd_ms": t_svd, "select_ms": t_sel,
           "ecm_total_ms": t_tr + t_svd + t_sel, "pod_ms": t_pod,
           "svd_sweeps": sweeps, "svd_off_history": [float("%.3g" % v) for v in hist],
           "svd_tflops": flops / (t_svd * 1e-3) / 1e12,
           "svd_frac_of_fp64_peak": flops / (t_svd * 1e-3) / 78.6e12,
           "greedy_iterations": info["iters"], "nnls_calls": int(tr[:, 1].sum()),
           "points_dropped": int(tr[:, 2].sum()), "selected": int(len(z)),
           "sum_w_minus_V0": float(w.sum().item() - V0),
           "sigma_ratio_at_truncation": float(sig_h[mt - 2] / sig_h[0]),
           "status_max": status, "nbad": nbad,
           "workload": f"{Nm} macro strain states -> {k} k-means directions x {n_steps} load levels "
                       f"= {p} snapshots (Newton-converged over {M} candidate points, m={m}); "
                       f"x_f {Prows} x {M}; {mt} points selected; POD of {wt['s_el']} + "
                       f"{wt['s_in']} snapshots of {wt['nd']} dofs into {wt['n_el']} + "
                       f"{wt['n_inel']} modes"}
    if quiet:
        return res
    line = {"metric": "offline stage time (k-means + training paths + ECM selection + POD)",
            "value": t_km + t_paths + res["ecm_total_ms"] + t_pod, "unit": "ms", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": res["workload"]}, "detail": res}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="mixed", choices=["mixed", "batched", "j2", "ecm"],
                    help="mixed: the headline (m=64, Q=512) step; batched: uneven clusters; "
                         "j2: J2 plasticity path at the Example 1 sizes")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "fp64"])
    ap.add_argument("--condense", default="biot6", choices=["biot6", "nine"],
                    help="biot6: condense the six coordinates of the symmetric stretch (the "
                         "Biot form, same Pbar and Cbar); nine: all nine components of Fr")
    ap.add_argument("--refine", action="store_true",
                    help="mixed plans: iterative refinement of the adjoint solve")
    ap.add_argument("--N", type=int, default=131072)
    ap.add_argument("--m", type=int, default=64)
    ap.add_argument("--Q", type=int, default=512)
    ap.add_argument("--amp", type=float, default=0.05)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no FP16 / batched / adjoint / monolithic / J2 legs)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe > 0:
        import torch
        n = int(args.copy_probe * 2 ** 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_launch": 8 * n,
                          "copy_probe_bytes_written_per_launch": 8 * n}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hyper-reduced RVE evaluation is "
              "sharded by macro points across GPUs with no exchange but a 4-value "
              "theta-gradient all-reduce; no multi-GPU figure is produced here.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "batched":
        print(json.dumps(run_batched(args, N=args.N if args.N != 131072 else 262144,
                                     precision=args.precision)), flush=True)
        return
    if args.workload == "j2":
        run_j2(args, precision=args.precision)
        return
    if args.workload == "ecm":
        run_ecm(args)
        return
    N, m, Q = args.N, args.m, args.Q
    print(f"[bench] building inputs N={N} m={m} Q={Q}", file=sys.stderr, flush=True)
    cl, F = build_inputs(N, m, Q, args.amp, 4000)

    split = args.precision != "fp64"
    print(f"[bench] timing {args.precision} (split={split})", file=sys.stderr, flush=True)
    biot6 = args.condense == "biot6"
    res = run_gpu(args.precision, cl, F, N, args.steps, args.warmup, split=split,
                  refine=args.refine, biot6=biot6)
    ms_step = res["wall"] / args.steps * 1e3
    value = N / (ms_step * 1e-3)
    fl_tan = tangent_flops_per_point(m, Q) * N
    achieved = fl_tan / (res["tan_ms"] * 1e-3)
    peak = PEAK[args.precision]
    tag = f"tangent_{args.precision}_m{m}_q{Q}"
    traffic = read_traffic(tag, res["variant"])

    fp64 = None
    if args.precision != "fp64" and not args.skip_fp64:
        print("[bench] timing fp64 reference path", file=sys.stderr, flush=True)
        ref = run_gpu("fp64", cl, F, N, max(2, args.steps // 2), 1, biot6=biot6)
        ms64 = ref["wall"] / max(2, args.steps // 2) * 1e3
        P1, P0 = res["Pbar"].cpu().numpy(), ref["Pbar"].cpu().numpy()
        C1, C0 = res["Cbar"].cpu().numpy(), ref["Cbar"].cpu().numpy()
        eP = np.linalg.norm(P1 - P0, axis=0) / np.maximum(np.linalg.norm(P0, axis=0), 1e-300)
        eC = np.linalg.norm(C1 - C0, axis=0) / np.maximum(np.linalg.norm(C0, axis=0), 1e-300)
        fp64 = {"value": N / (ms64 * 1e-3), "ms_per_step": ms64, "eval_ms": ref["eval_ms"],
                "eval_tflops": eval_flops_per_point(m, Q) * N / (ref["eval_ms"] * 1e-3) / 1e12,
                "eval_frac_of_fp64_peak": eval_flops_per_point(m, Q) * N
                / (ref["eval_ms"] * 1e-3) / PEAK["fp64"],
                "speedup_mixed_over_fp64": ms64 / ms_step,
                "mixed_vs_fp64_rel_err_max": {"Pbar": float(eP.max()), "Cbar": float(eC.max())},
                "mixed_vs_fp64_rel_err_median": {"Pbar": float(np.median(eP)),
                                                 "Cbar": float(np.median(eC))}}

    cpu = None
    if not args.skip_cpu:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        n, dt, thr = cpu_baseline(cl, F)
        cpu = {"value": n / dt, "unit": "point-evals/s", "cores": thr, "kind": "oracle",
               "host": host_cpu(),
               "sample": f"{n} of the {N} macro points, one evaluate + condense + adjoint "
                         f"backward each (plain C, FP64, OpenMP over points)"}

    extras = None
    if not args.no_extras and args.precision != "fp64":
        extras = {}
        other = "fp16" if args.precision == "bf16" else "bf16"
        print(f"[bench] extra: {other} at the headline shape", file=sys.stderr, flush=True)
        r2 = run_gpu(other, cl, F, N, args.steps, args.warmup, split=True, biot6=biot6)
        ms2 = r2["wall"] / args.steps * 1e3
        extras[other] = {"ms_per_step": ms2, "value": N / (ms2 * 1e-3),
                         "tangent_ms": r2["tan_ms"],
                         "frac": tangent_flops_per_point(m, Q) * N / (r2["tan_ms"] * 1e-3) / PEAK[other],
                         "status_max": r2["status"]}
        del r2
        print("[bench] extra: oracle errors at three amplitudes", file=sys.stderr, flush=True)
        extras["oracle_errors_" + args.precision] = oracle_errors(precision=args.precision)
        print("[bench] extra: batched clusters", file=sys.stderr, flush=True)
        b = run_batched(args, precision=args.precision)
        extras["batched"] = {k: b[k] for k in ("value", "ms_per_graph", "fp64",
                                               "speedup_mixed_over_fp64",
                                               "mixed_vs_fp64_Cbar_rel_err_max", "status_max")}
        extras["batched"]["workload"] = b["config"]["workload"]
        print("[bench] extra: adjoint workload", file=sys.stderr, flush=True)
        extras["adjoint_48_384"] = {"mixed": run_adjoint(precision=args.precision),
                                    "fp64": run_adjoint(precision="fp64")}
        print("[bench] extra: FP64 monolithic iterations at (32, 256)", file=sys.stderr, flush=True)
        extras["monolithic_32_256"] = run_monolithic()
        print("[bench] extra: J2 plasticity path", file=sys.stderr, flush=True)
        extras["j2_8_250"] = run_j2(args, quiet=True)
        extras["j2_8_250_" + args.precision] = run_j2(args, quiet=True, precision=args.precision)
        extras["offline_ecm_m30_500_of_32768"] = run_ecm(args, quiet=True)

    line = {
        "metric": METRIC, "value": value, "unit": "point-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision if args.precision == "fp64" else
        f"{args.precision} MFMA{'x3 split' if split else ''} + fp32 tangent + fp64",
        "data": "synthetic",
        "config": {"workload": f"hyper-reduced RVE, {N} macro points, m={m} ROM modes, "
                               f"Q={Q} ECM points, one cluster, strain amplitude {args.amp}",
                   "N": N, "m": m, "Q": Q, "precision": args.precision, "split": split,
                   "step": "eval + condense + adjoint backward + update",
                   "condense": "six coordinates of the symmetric stretch (Biot form)" if biot6
                   else "nine components"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "kernel": "tangent contraction (k_eval_mixed / k_eval_f64)",
                     "kernel_ms": res["tan_ms"], "flops_per_point": tangent_flops_per_point(m, Q),
                     "eval_ms": res["eval_ms"],
                     "eval_tflops": eval_flops_per_point(m, Q) * N / (res["eval_ms"] * 1e-3) / 1e12},
        "step_tflops": step_flops_per_point(m, Q) * N / (ms_step * 1e-3) / 1e12,
        "ul_output": {"kernel": "k_cauchy: Cauchy stress and App. A tangent of the condensed state",
                      "ms": res["cauchy_ms"], "bound": "hbm",
                      "bytes_per_point": CAUCHY_BYTES_PER_POINT,
                      "achieved_GBs": CAUCHY_BYTES_PER_POINT * N / (res["cauchy_ms"] * 1e-3) / 1e9,
                      "frac": CAUCHY_BYTES_PER_POINT * N / (res["cauchy_ms"] * 1e-3) / HBM_PEAK,
                      "traffic": read_cauchy_traffic(m, Q)},
        "status_max": res["status"],
        "tuned_variant": res["variant"], "tuned_kin_variant": res["kin_variant"],
        "tuned_condense_variant": res["cond_variant"], "variant_eval_ms": res["tune_ms"],
        "fp64": fp64,
        "cpu_baseline": cpu,
        "other_workloads": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
