"""Benchmark: tensor entries solved per second for sum_k A_k x_k X = B on one
MI355X, with the roofline of the dominant kernel and the CPU oracle beside it.

One step = the whole FP64 hot path on one right-hand side: sylt_schur_factor
(device Schur factors + eigenvalue-sum separation + plan) and sylt_solve
(U^* transform chain, triangular sweep, U transform chain).  The default
workload is N = 7, n_k = 19 (893,871,739 complex128 entries, 14.3 GB per
tensor); inputs are seeded synthetic tensors already resident in HBM when the
timed region starts.  The mixed-precision solve (FP32 transforms, FP64 sweep,
FP64 residual, iterative refinement to a 1e-12 relative residual) is timed on
the same inputs and reported beside it, and so is the time evolution of
Theorem 1 (sylt_evolve at t = 0.1), the sweep of a plan with normal A_k
(Remark 1), and the advection-diffusion example of Section 5.3.

Prints ONE JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C3b]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TF = 78.6     # MI355X FP64 vector (= FP64 matrix) peak


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3b")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-evolve", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--phase-reps", type=int, default=3)
    return ap.parse_args()


def source_digest(relpath):
    import hashlib
    with open(os.path.join(ROOT, relpath), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_counters(kernel, workload):
    """Counter figures of `kernel` at `workload` from the committed summary
    (profiles/kernel_traffic.txt): HBM bytes per launch (FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for a copy of known
    size), the matrix-core busy fraction and the L2 hit rate.  None if absent
    or if the kernel's source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "kernel_traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
        if f.get("kernel") != kernel or f.get("workload") != workload:
            continue
        if f.get("source_sha256") != source_digest(f.get("source", "")):
            return None
        out = {"traffic": float(f["hbm_bytes_per_launch"])}
        if "mfma_busy" in f:
            out["mfma_busy"] = float(f["mfma_busy"])
        if "l2_hit" in f:
            out["l2_hit"] = float(f["l2_hit"])
        return out
    return None


def roofline_entry(kernel, flops, bytes_alg, ms_total, launches, matrix_core, workload, source):
    """Roofline of one kernel over `launches` launches: the binding roof of its
    algorithmic work (FP64 arithmetic or HBM), achieved = algorithmic work per
    launch / average launch duration."""
    t = ms_total * 1e-3
    t_hbm = bytes_alg / (HBM_PEAK_GBS * 1e9)
    t_fp = flops / (FP64_VECTOR_PEAK_TF * 1e12)
    counters = measured_counters(kernel, workload)
    traffic = counters["traffic"] if counters else None
    if t_fp >= t_hbm:
        ach = flops / t / 1e12
        out = {"kernel": kernel, "bound": "mfma" if matrix_core else "alu",
               "achieved": round(ach, 3), "peak": FP64_VECTOR_PEAK_TF, "unit": "TFLOP/s",
               "frac": round(ach / FP64_VECTOR_PEAK_TF, 4)}
    else:
        ach = bytes_alg / t / 1e9
        out = {"kernel": kernel, "bound": "hbm", "achieved": round(ach, 1),
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)}
    out["traffic"] = traffic
    out["alg_bytes_per_launch"] = bytes_alg / launches
    out["alg_flops_per_launch"] = flops / launches
    out["avg_launch_ms"] = round(ms_total / launches, 4)
    out["launches"] = launches
    if traffic is not None:
        out["traffic_over_alg_bytes"] = round(traffic / (bytes_alg / launches), 2)
    if matrix_core and counters and "mfma_busy" in counters:
        # measured matrix-core busy fraction beside the algorithmic frac above
        out["mfma_busy_measured"] = counters["mfma_busy"]
    if counters and "l2_hit" in counters:
        out["l2_hit_measured"] = counters["l2_hit"]
    return out


def time_events(fn, reps, torch):
    """Average milliseconds per call of fn() on the current stream (HIP events)."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(w, A, B_host, sample_fraction=1.0 / 32, sweep_entries=1 << 23):
    """The oracle (never tuned) on a bounded sample of the same workload: every
    mode product of both transform chains over 1/32 of the fibres, and the
    first 2^23 entries of the literal sweep; each phase's rate is scaled to the
    full tensor (the sweep by its exact multiply-subtract count,
    n_tot (sum n - N)/2, against the sample's)."""
    import numpy as np

    import oracle

    U, T = oracle.factors(A)
    n = list(w.n)
    ntot = w.ntot
    t_tr = 0.0
    for k in range(len(n)):
        nfib = ntot // n[k]
        f1 = max(1, int(nfib * sample_fraction))
        for adj in (True, False):
            t0 = time.perf_counter()
            oracle.mode_product_fibres_inplace(n, k, U[k], B_host, 0, f1, adj)
            t_tr += (time.perf_counter() - t0) * (nfib / f1)
    t0 = time.perf_counter()
    steps = oracle.sweep_inplace(n, T, B_host, sweep_entries)
    t_sw = time.perf_counter() - t0
    total_steps = ntot * (sum(n) - len(n)) // 2
    # per-entry overhead and per-step cost are not separated: scale by steps
    t_sw_full = t_sw * (total_steps / max(1, steps))
    t_full = t_tr + t_sw_full
    return {
        "value": ntot / t_full,
        "unit": "entries/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"oracle C loops at N={len(n)}, n={n[0]}: both transform chains over "
                   f"1/{int(round(1 / sample_fraction))} of the fibres of every mode "
                   f"(OpenMP) + the first {sweep_entries} entries of the literal "
                   f"single-threaded sweep ({steps} multiply-subtracts), each phase "
                   f"scaled to the full tensor"),
        "est_full_solve_s": round(t_full, 2),
        "transform_s_est": round(t_tr, 2),
        "sweep_s_est": round(t_sw_full, 2),
    }


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_full_runs(names, sylt, torch):
    """The oracle run in full (not sampled) on the small workloads, phase by
    phase with a monotonic clock: Schur factors (LAPACK), forward chain,
    literal sweep, backward chain.  The device's plan + solve of the same
    inputs is timed beside it."""
    import numpy as np

    import oracle
    import sylt_workloads as wl

    out = {}
    for name in names:
        w = wl.WORKLOADS[name]
        n = list(w.n)
        A = wl.coefficient_matrices(w.n, w.seed)
        B = wl.rhs(w)
        t = {}
        t0 = time.perf_counter()
        U, T = oracle.factors(A)
        t["factors_s"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        C = oracle.transform(n, U, B, True)
        t["forward_s"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        Y, _ = oracle.sweep(n, T, C)
        t["sweep_s"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        X = oracle.transform(n, U, Y, False)
        t["backward_s"] = time.perf_counter() - t0
        total = sum(t.values())
        A_dev = [torch.from_numpy(a).cuda() for a in A]
        Bd = torch.from_numpy(B).cuda()
        Xd = torch.empty_like(Bd)

        def step():
            plan = sylt.Plan.factor(n, A_dev)
            sylt.solve(plan, Bd, out=Xd)
            return plan
        plans = [step()]  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            plans.append(step())
        e1.record()
        e1.synchronize()
        gpu_ms = e0.elapsed_time(e1) / reps
        for pl in plans:
            pl.destroy()
        err = float(np.max(np.abs(Xd.cpu().numpy() - X)) / np.max(np.abs(X)))
        out[name] = {"n": n, "entries": w.ntot, **{k: round(v, 4) for k, v in t.items()},
                     "oracle_total_s": round(total, 4),
                     "oracle_entries_per_s": round(w.ntot / total, 1),
                     "device_ms": round(gpu_ms, 3), "relmax_device_vs_oracle": err}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no "
              f"multi-GPU path -- run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import sylt_workloads as wl
    from paper_2412_15840_amd import sylt

    w = wl.WORKLOADS[args.workload]
    n = list(w.n)
    ntot = w.ntot
    torch.cuda.set_device(0)
    log(f"workload {w.name} n={n} ntot={ntot}: generating inputs")
    A = wl.coefficient_matrices(w.n, w.seed)
    A_dev = [torch.from_numpy(a).cuda() for a in A]
    B_host = torch.empty(ntot, dtype=torch.complex128, pin_memory=True)
    wl.rhs(w, out=B_host.numpy())
    Bd = B_host.cuda()
    Xd = torch.empty_like(Bd)
    torch.cuda.synchronize()
    log("inputs resident; warmup")

    def step():
        plan = sylt.Plan.factor(n, A_dev)
        sylt.solve(plan, Bd, out=Xd)
        return plan

    for _ in range(args.warmup):
        step().destroy()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    s = torch.cuda.current_stream()
    # one event per step boundary; the plans are destroyed after the timed
    # region (their teardown is not part of a solve)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    plans = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(s)
    for i in range(args.steps):
        plans.append(step())
        ev[i + 1].record(s)
    ev[-1].synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    ms_per_step = ev[0].elapsed_time(ev[-1]) / args.steps
    for pl in plans:
        pl.destroy()
    del plans
    value = ntot / (ms_per_step * 1e-3)
    step_stats = {"mean_ms": round(ms_per_step, 3),
                  "median_ms": round(float(np.median(step_ms)), 3),
                  "min_ms": round(float(np.min(step_ms)), 3),
                  "max_ms": round(float(np.max(step_ms)), 3)}
    log(f"{ms_per_step:.2f} ms/step ({wall:.2f} s wall) -> {value:.4g} entries/s; {step_stats}")

    # ---------------------------------------------------------- phases
    plan = sylt.Plan.factor(n, A_dev)
    desc = plan.describe()
    Yd = Bd.clone()
    reps = args.phase_reps
    t_fwd = time_events(lambda: sylt.transform(plan, Yd, sylt.TO_SCHUR), reps, torch)
    t_sw = time_events(lambda: sylt.sweep(plan, Yd, sylt.OP_N), reps, torch)
    t_bwd = time_events(lambda: sylt.transform(plan, Yd, sylt.FROM_SCHUR), reps, torch)
    del Yd
    t_plan = time_events(lambda: sylt.Plan.factor(n, A_dev).destroy(), 2, torch)
    sum_n = sum(n)
    Nm = len(n)
    # algorithmic work per entry (one read and one write of the tensor per
    # phase: a transform chain is one phase however many passes it takes)
    tr_flops = 8.0 * ntot * sum_n
    tr_bytes = 32.0 * ntot
    sw_flops = 8.0 * ntot * (sum_n - Nm) / 2 + ntot * (2 * (Nm - 1) + 8)
    sw_bytes = 32.0 * ntot
    n_pass = len(desc["transform_passes"])
    n_lvl = desc["sweep"]["tile_levels"]
    t_tr = 0.5 * (t_fwd + t_bwd)
    kernels = {
        "transform_pass": {
            "launches_per_call": n_pass, "ms_per_call": round(t_tr, 3),
            "avg_launch_ms": round(t_tr / n_pass, 4),
            "tflops": tr_flops / (t_tr * 1e-3) / 1e12, "gbs_alg": tr_bytes / (t_tr * 1e-3) / 1e9},
        "sweep_tile": {
            "launches_per_call": n_lvl, "ms_per_call": round(t_sw, 3),
            "avg_launch_ms": round(t_sw / n_lvl, 4),
            "tflops": sw_flops / (t_sw * 1e-3) / 1e12, "gbs_alg": sw_bytes / (t_sw * 1e-3) / 1e9},
    }
    # roofline of both hot kernels; the dominant one (largest time per solve)
    # is the headline roofline object
    tr_kernel = ("transform_mfma_kernel<double2,%d>" % n[0]
                 if all(v == n[0] for v in n) else "transform_pass_kernel")
    sw_kernel = "sweep_tile_kernel<double2,false,%d,%s>" % (
        len([v for v in n if v > 1]), "true" if desc["sweep"]["local_solve"] == "pencil" else "false")
    roof_tr = roofline_entry(tr_kernel, tr_flops, tr_bytes, t_tr, n_pass, True, w.name,
                             "paper_2412_15840_amd/csrc/transform.hip")
    roof_sw = roofline_entry(sw_kernel, sw_flops, sw_bytes, t_sw, n_lvl, False, w.name,
                             "paper_2412_15840_amd/csrc/sweep.hip")
    roof = roof_sw if t_sw >= 2 * t_tr else roof_tr
    kernels["transform_pass"]["roofline"] = roof_tr
    kernels["sweep_tile"]["roofline"] = roof_sw
    # whole-solve roofline: max(algorithmic bytes / HBM peak, flops / FP64 peak)
    t_hbm = (2 * tr_bytes + sw_bytes) / (HBM_PEAK_GBS * 1e9)
    t_fp = (2 * tr_flops + sw_flops) / (FP64_VECTOR_PEAK_TF * 1e12)
    solve_roof = {"t_hbm_ms": round(t_hbm * 1e3, 3), "t_fp64_ms": round(t_fp * 1e3, 3),
                  "binding_roof_frac": round(max(t_hbm, t_fp) / (ms_per_step * 1e-3), 4),
                  "hbm_alg_frac": round(t_hbm / (ms_per_step * 1e-3), 4)}
    phases = {"plan_ms": round(t_plan, 3), "transform_fwd_ms": round(t_fwd, 3),
              "sweep_ms": round(t_sw, 3), "transform_bwd_ms": round(t_bwd, 3)}
    log(f"phases {phases}")

    # ---------------------------------------------------------- mixed form
    mixed = None
    if not args.no_mixed:
        X64 = Xd  # FP64 solution of the last timed step
        Xm = torch.empty_like(Bd)
        ws = torch.empty(plan.workspace_bytes("mixed"), dtype=torch.uint8, device="cuda")
        _, info = sylt.solve(plan, Bd, precision="mixed", out=Xm, workspace=ws, info=True)
        torch.cuda.synchronize()
        reps_m = max(1, min(args.steps, 2))
        t_m = time_events(lambda: sylt.solve(plan, Bd, precision="mixed", out=Xm, workspace=ws),
                          reps_m, torch)
        err = float(((Xm - X64).abs().max() / X64.abs().max()).item())
        mixed = {"ms": round(t_m, 3), "iterations": info["iterations"],
                 "phase_ms": {"transforms": round(info["ms_transform"], 3),
                              "sweeps": round(info["ms_sweep"], 3),
                              "residuals": round(info["ms_residual"], 3)},
                 "rel_residual": info["rel_residual"],
                 "speedup_vs_fp64": round((t_fwd + t_sw + t_bwd) / t_m, 4),
                 "max_rel_diff_vs_fp64": err, "entries_per_s": ntot / (t_m * 1e-3)}
        log(f"mixed {mixed}")
        del ws, Xm

    # ---------------------------------------------------------- evolution
    # Theorem 1 at t = 0.1 (sylt_evolve) on the same plan, with X(0) = B (any
    # seeded input times the same); algorithmic work: four transform chains
    # (B, X(0), exp(tT), back), the Kronecker-sum apply, the sweep
    evolve = None
    if not args.no_evolve:
        Xe = torch.empty_like(Bd)
        ws_e = torch.empty(2 * ntot * 16, dtype=torch.uint8, device="cuda")
        sylt.evolve(plan, 0.1, Bd, Bd, out=Xe, workspace=ws_e)
        torch.cuda.synchronize()
        t_e = time_events(lambda: sylt.evolve(plan, 0.1, Bd, Bd, out=Xe, workspace=ws_e),
                          max(1, min(args.steps, 2)), torch)
        ev_flops = 4 * tr_flops + 8.0 * ntot * sum_n + sw_flops
        t_e_fp = ev_flops / (FP64_VECTOR_PEAK_TF * 1e12)
        evolve = {"t": 0.1, "ms": round(t_e, 3), "entries_per_s": ntot / (t_e * 1e-3),
                  "t_fp64_ms": round(t_e_fp * 1e3, 3),
                  "binding_roof_frac": round(t_e_fp / (t_e * 1e-3), 4)}
        log(f"evolve {evolve}")
        del Xe, ws_e

    # ---------------------------------------------------------- normal A_k
    # Remark 1: with normal A_k the plan's sweep is one Hadamard pass (read and
    # write the tensor: 32 B per entry), timed at the same shape
    normal = None
    if not args.no_evolve:
        An = [torch.from_numpy(a).cuda() for a in wl.normal_coefficient_matrices(w.n, w.seed)]
        plan_n = sylt.Plan.factor(n, An)
        if plan_n.describe()["sweep"]["diagonal"]:
            Yn = Bd.clone()
            t_n = time_events(lambda: sylt.sweep(plan_n, Yn, sylt.OP_N), reps, torch)
            gbs = 32.0 * ntot / (t_n * 1e-3) / 1e9
            normal = {"sweep_ms": round(t_n, 3), "gbs_alg": round(gbs, 1),
                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                      "speedup_vs_tiled_sweep": round(t_sw / t_n, 2)}
            del Yn
        plan_n.destroy()
        log(f"normal {normal}")

    # ---------------------------------------------------------- Section 5.3
    # the advection-diffusion example at the paper's size (N = 6, 16 Hermite
    # nodes per axis, t = 1): plan (device Schur) + sylt_evolve, and the max
    # error against the exact solution (1 + e^t) exp(-x.x)
    advdif = None
    if not args.no_evolve:
        xh, Ah, Bh6, X0h = wl.advection_diffusion(6)
        A6 = [torch.from_numpy(a).cuda() for a in Ah]
        B6, X06 = torch.from_numpy(Bh6).cuda(), torch.from_numpy(X0h).cuda()
        X6 = torch.empty_like(B6)

        def advdif_run():
            p6 = sylt.Plan.factor([16] * 6, A6)
            sylt.evolve(p6, 1.0, B6, X06, out=X6)
            return p6

        advdif_run().destroy()
        torch.cuda.synchronize()
        t_a = time_events(lambda: advdif_run().destroy(), 3, torch)
        err = float(np.max(np.abs(X6.cpu().numpy() - wl.advection_diffusion_exact(xh, 6, 1.0))))
        advdif = {"N": 6, "nodes": 16, "t": 1.0, "ms": round(t_a, 3), "max_error_vs_exact": err,
                  "paper_matlab_s": 25.73, "paper_max_error": 9.6811e-14}
        log(f"advection-diffusion {advdif}")

    # ---------------------------------------------------------- Section 5.1
    # the mixed-extent shape n = (2, 9, 33, 74, 231) (10,153,836 entries):
    # plan (device Schur, global-memory kernel for 74 and 231) + FP64 solve,
    # with the usual synthetic coefficients and right-hand side
    large = None
    if not args.no_large and args.workload != "E1":
        wE = wl.WORKLOADS["E1"]
        AE = [torch.from_numpy(a).cuda() for a in wl.coefficient_matrices(wE.n, wE.seed)]
        BE = torch.from_numpy(wl.rhs(wE)).cuda()
        XE = torch.empty_like(BE)

        def large_run():
            pE = sylt.Plan.factor(list(wE.n), AE)
            sylt.solve(pE, BE, out=XE)
            return pE

        large_run().destroy()
        torch.cuda.synchronize()
        t_l = time_events(lambda: large_run().destroy(), 3, torch)
        pE = sylt.Plan.factor(list(wE.n), AE)
        YE = BE.clone()
        t_lp = time_events(lambda: sylt.Plan.factor(list(wE.n), AE).destroy(), 2, torch)
        t_lf = time_events(lambda: sylt.transform(pE, YE, sylt.TO_SCHUR), reps, torch)
        t_ls = time_events(lambda: sylt.sweep(pE, YE, sylt.OP_N), reps, torch)
        pE.destroy()
        trE = 8.0 * wE.ntot * sum(wE.n)
        large = {"n": list(wE.n), "ntot": wE.ntot, "ms_per_step": round(t_l, 3),
                 "entries_per_s": wE.ntot / (t_l * 1e-3), "plan_ms": round(t_lp, 3),
                 "transform_ms": round(t_lf, 3), "sweep_ms": round(t_ls, 3),
                 "transform_tflops": round(trE / (t_lf * 1e-3) / 1e12, 3),
                 "paper_matlab_s": 27.64}
        log(f"large extent {large}")
        del AE, BE, XE, YE

    # ---------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu:
        log("timing the oracle on a bounded sample")
        Bh = B_host.numpy()
        cpu = cpu_baseline(w, A, Bh)
        cpu["cpu_model"] = cpu_model()
        cpu["nproc"] = os.cpu_count()
        log(f"cpu {cpu}")
        log("the oracle in full on the small workloads")
        cpu["full_runs"] = oracle_full_runs(["C1", "C2", "C5"], sylt, torch)
        log(f"oracle full runs {cpu['full_runs']}")

    line = {
        "metric": "tensor entries solved/s (FP64 Schur/Bartels-Stewart solve, N=7 n=19)",
        "value": value, "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "step_ms": step_stats,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.description}", "n": n, "entries": ntot,
                   "seed": w.seed, "parallelism": "1 GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "solve_roofline": solve_roof,
        "phases": phases, "kernels": kernels, "mixed": mixed, "evolve": evolve,
        "normal_sweep": normal, "advection_diffusion": advdif, "large_extent": large,
        "plan": {"transform_passes": [p["extents"] for p in desc["transform_passes"]],
                 "sweep_block": desc["sweep"]["block"], "sweep_tile_levels": n_lvl,
                 "sep": desc["sep"]},
        "paper_context": {"matlab_laptop_s": 1470.51, "entries_per_s": 6.08e5,
                          "note": "MATLAB on a 2020 MacBook Pro, unshifted complex randn A (Table 1)"},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
