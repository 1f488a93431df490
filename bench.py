"""Benchmark of the fine kinetic propagator on one MI355X.

A step = one pass of the whole hot path over one batch: all 32 parareal
slices of the large Sod workload (Nx=2048, 48^3 velocities on [-10,10]^3,
eps=1e-3, zero-gradient ends) are lifted from their moments, advanced by one
slice span (188 IMEX steps: a three-step pass from the lift, 61 three-step
passes over f, and the last two steps evaluated on the moments, exactly, from
weighted sums of the last stored field) and projected back to moments, all
slices batched in one launch per pass (7.25e9 phase-space cells per buffer).  Prints one JSON line:
phase-space updates/s, the roofline of the dominant kernel (the three-step
relax pass) under both byte models, the CPU oracle timed on a bounded sample,
and secondary sections: the smooth periodic workload (Nx=512, 32^3, 64 slices)
at its three Knudsen numbers, parareal against the serial fine solve at the
baseline configurations and on small latency-bound cases, the exterior-force,
second-order, uneven-batch and adjoint paths.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--workload sod_large|smooth_periodic] [--no-cpu-baseline] [--no-parareal]
       [--extras smooth,parareal,parareal_large,force,order2,uneven,adjoint]
       [--copy-calibration]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BGK phase-space updates/s (Nx*Nv^3*steps) + parareal vs serial-fine speedup"
HBM_PEAK_GBS = 8000.0
TRAFFIC_SUMMARY = {
    ("sod_large", "three"): os.path.join(ROOT, "profiles", "k_step3x_sod_large_traffic.md"),
    ("smooth_periodic", "three"): os.path.join(ROOT, "profiles",
                                               "k_step3x_smooth_periodic_traffic.md"),
    ("smooth_periodic", "two"): os.path.join(ROOT, "profiles",
                                             "k_step2x2_smooth_periodic_traffic.md"),
}
# sources of the step kernels whose counters the traffic summaries record
KERNEL_SRCS = [os.path.join(ROOT, "paper_2502_02704_amd", "csrc", n)
               for n in ("kinetic.hip", "bgk_internal.h")]
TILE_CACHE = os.path.join(ROOT, "paper_2502_02704_amd", "tiles.json")


def log(msg):
    """Progress of the run on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """First 16 hex digits of the SHA-256 of the step kernels' sources
    (concatenated in order)."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def conserved(W):
    """Conserved moments (rho, rho u, E) of primitive (rho, u, theta) rows."""
    import numpy as np
    return np.column_stack([W[:, 0], W[:, 0:1] * W[:, 1:4],
                            0.5 * W[:, 0] * (W[:, 1:4] ** 2).sum(1) + 1.5 * W[:, 0] * W[:, 4]])


def slice_moments(wk, B):
    """Conserved moments of the 64 slices: phase-shifted copies of the smooth
    periodic profile (what a parareal iterate hands to the fine solver)."""
    import numpy as np
    p = wk.problem
    x = p.x_centres()
    V = np.empty((B, p.nx, 5))
    for b in range(B):
        s = np.sin(2 * np.pi * (x + b / B))
        rho, u = 1 + 0.2 * s, 0.1 * s
        V[b] = np.column_stack([rho, rho * u, 0 * x, 0 * x, 0.5 * rho * u * u + 1.5 * rho])
    return V


def workload_batch(name, eps=None):
    """(workload, conserved slice moments [B][nx][5], span) of a benchmark batch."""
    import numpy as np
    from paper_2502_02704_amd import workloads as wl
    if name == "sod_large":
        wk = wl.c3_sod_large()
        V = np.stack([conserved(w) for w in wl.c3_slice_states(wk)])
    else:
        wk = wl.c2_smooth_periodic(eps=1e-2 if eps is None else eps)
        V = slice_moments(wk, wk.n_slices)
    return wk, V, wk.T / wk.n_slices


def steps_on_moments(n):
    """Steps of a propagation with three steps per pass that are evaluated on
    the moments only (not written out as f): after a three-step first pass
    from the lift when n = 2 mod 3, else after a two-step one."""
    if n < 4:
        return 0
    return 2 if n >= 5 and n % 3 == 2 else (n - 2) % 3


def traffic_from_profile(workload, which):
    """HBM bytes per launch of the three- or two-step pass from the committed
    rocprofv3 counter summary of this workload, if it was taken on the
    current kernel source; else None."""
    path = TRAFFIC_SUMMARY.get((workload, which))
    if path is None:
        return None
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", txt, flags=re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wk, V, span, n_sample=20, reps=3):
    """The oracle, built for this host (-O3 -march=native, no fast-math, in
    a temporary directory), on a bounded sample of the same workload: one
    slice lifted, advanced `n_sample` steps of the slice's step size and
    projected; median of `reps` runs on every OpenMP thread, and one run on
    one thread over a single step."""
    import statistics
    import tempfile
    import oracle
    from oracle import build as obuild
    p = wk.problem
    n, dt = oracle.n_steps(p, span)
    sample = n_sample * dt
    tmp = tempfile.mkdtemp(prefix="oracle_native_")
    oracle.use_library(obuild.build_native(os.path.join(tmp, "liboracle_native.so")))
    try:
        assert oracle.n_steps(p, sample)[0] == n_sample
        cores = oracle.get_threads()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.fine_propagate_moments(p, V[0], sample)
            ts.append(time.perf_counter() - t0)
        el = statistics.median(ts)
        oracle.set_threads(1)
        try:
            t1 = time.perf_counter()
            oracle.fine_propagate_moments(p, V[0], dt)
            el1 = time.perf_counter() - t1
        finally:
            oracle.set_threads(cores)
    finally:
        oracle.use_library(None)
    return {"value": p.cells * n_sample / el, "unit": "updates/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"slice 0 of {V.shape[0]}: lift + {n_sample} of its {n} IMEX steps + "
                       f"projection, {p.nx}x{p.nv[0]}^3, median of {reps} runs "
                       f"({', '.join(f'{t:.1f}' for t in ts)} s)"),
            "build": "gcc -O3 -march=native -fopenmp (no -ffast-math), built on this host",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "value_1_thread": p.cells / el1,
            "sample_1_thread": f"lift + 1 step + projection of slice 0, {el1:.1f} s"}


def parareal_row(torch, bgk, name, p, W0np, N, T, E, coarse, lift_order, k_cap, reps,
                 baseline_config, warm_each=True):
    """Parareal (Algorithm 2) against the serial chained fine solve with the
    same kernels and the same launch machinery (captured graphs on both
    sides).  Error = max over slices, cells and components of
    |U_parareal - U_serial| (conserved moments); K runs from 1 until the error
    reaches 1e-6 or K = k_cap.  Wall-clock: median of `reps` runs (after a
    warm-up run per K, or with warm_each False one warm-up at K = k_cap, which
    captures every iteration's graph)."""
    import numpy as np

    def timed(fn, warm=True):
        if warm:
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return out, float(np.median(ts))

    W0 = torch.from_numpy(W0np).cuda()
    run_par = lambda K: bgk.parareal_iterate(p, W0, N, T, K, 0.0, E=E, coarse=coarse,
                                             lift_order=lift_order)
    ref, t_serial = timed(lambda: bgk.serial_fine(p, W0, N, T, E=E, lift_order=lift_order))
    ref = ref.cpu().numpy()
    res = {"workload": name, "baseline_config": baseline_config, "coarse": coarse,
           "lift_order": lift_order, "slices": N, "serial_fine_ms": round(t_serial * 1e3, 4),
           "K": []}
    if not warm_each:
        run_par(k_cap)
    chosen = None
    for K in range(1, k_cap + 1):
        (V, err, kd), t_par = timed(lambda: run_par(K), warm=warm_each)
        e = float(np.max(np.abs(V.cpu().numpy() - ref)))
        res["K"].append({"K": K, "ms": round(t_par * 1e3, 4), "err_vs_fine": e,
                         "speedup": round(t_serial / t_par, 3)})
        if not warm_each:
            log(f"parareal {name} K={K}: {t_par * 1e3:.1f} ms, err {e:.3g}")
        if e <= 1e-6:
            chosen = res["K"][-1]
            break
    bgk.check_status()
    res["K_at_1e-6"] = chosen["K"] if chosen else None
    res["speedup_at_1e-6"] = chosen["speedup"] if chosen else None
    if chosen is None:
        res["err_at_K_cap"] = res["K"][-1]["err_vs_fine"]
        res["speedup_at_K_cap"] = res["K"][-1]["speedup"]
    return res


def parareal_small(torch, bgk, wl, reps=5):
    """The small Sod configuration (64 x 16^3, 8 slices) with the Euler and
    Navier-Stokes coarse models and the order-one lifting, and reduced
    smooth periodic cases (64 x 16^3, 16 slices; not baseline configurations)
    and the two-beam exterior-force test: where one slice's step is
    launch-latency bound, the only regime where one GPU can gain."""
    sod = wl.c1_sod_small()
    s4 = wl.c2_smooth_periodic(eps=1e-4, nx=64, nv=16, n_slices=16)
    s2 = wl.c2_smooth_periodic(eps=1e-2, nx=64, nv=16, n_slices=16)
    fk = wl.c6_two_beam_force()
    cases = [(sod, None, "euler", 0, True), (sod, None, "cns", 0, True),
             (sod, None, "cns", 1, True),
             (s4, None, "euler", 0, False), (s4, None, "cns", 0, False),
             (s2, None, "euler", 0, False), (s2, None, "cns", 0, False),
             (s2, None, "cns", 1, False)]
    out = [parareal_row(torch, bgk, w.name, w.problem, w.W0, w.n_slices, w.T, E, coarse, lo,
                        w.n_slices, reps, base) for w, E, coarse, lo, base in cases]
    out.append(parareal_row(torch, bgk, fk.name, fk.problem, fk.U0(), fk.n_slices, fk.T, fk.E,
                            "euler", 0, fk.n_slices, reps, False))
    return out


def parareal_large(torch, bgk, wl, k_cap_smooth=8, k_cap_sod=6):
    """Parareal at the full baseline sizes, where one slice's fine step is
    bandwidth bound: the smooth periodic workload (512 x 32^3, 64 slices) at
    eps = 1, 1e-2, 1e-4 with the Euler coarse model, at eps = 1e-2 and 1e-4
    also with the Navier-Stokes coarse model and the order-one lifting (at
    eps = 1 that model is outside its regime: the lifted states leave the
    physical set), and the large Sod workload (2048 x 48^3, 32 slices,
    K <= 6), Euler coarse model.  Reported as measured (a slowdown is
    expected: each iteration moves about as many bytes as the serial solve)."""
    out = []
    for eps in (1.0, 1e-2, 1e-4):
        w = wl.c2_smooth_periodic(eps=eps)
        models = [("euler", 0)] + ([("cns", 1)] if eps < 1.0 else [])
        for coarse, lo in models:
            try:
                out.append(parareal_row(torch, bgk, w.name, w.problem, w.W0, w.n_slices, w.T,
                                        None, coarse, lo, k_cap_smooth, 2, True,
                                        warm_each=False))
            except bgk.BgkError as e:
                # a model outside its regime reports a non-physical state
                bgk.status()
                out.append({"workload": w.name, "baseline_config": True, "coarse": coarse,
                            "lift_order": lo, "error": str(e)})
        bgk.free_workspaces()
        torch.cuda.empty_cache()
    w = wl.c3_sod_large()
    out.append(parareal_row(torch, bgk, w.name, w.problem, w.W0, w.n_slices, w.T, None,
                            "euler", 0, k_cap_sod, 1, True, warm_each=False))
    bgk.free_workspaces()
    torch.cuda.empty_cache()
    return out


def force_throughput(torch, bgk, wl, reps=5):
    """The exterior-force path on the two-beam test grid (Nx=100,
    256x16x16 velocities, eps=1e-5): all 20 slices of the first parareal
    iteration batched, lift + 21 steps (one per pass, with the v_x Rusanov
    transport, lanes on v_x columns) + projection.  Updates/s of the whole
    call and HBM rate of the one-step kernel (16 algorithmic bytes per
    update, 8 for the lifted first step)."""
    import numpy as np
    wk = wl.c6_two_beam_force()
    p, N = wk.problem, wk.n_slices
    W = wk.U0()
    V1 = np.column_stack([W[:, 0], W[:, 0:1] * W[:, 1:4],
                          0.5 * W[:, 0] * (W[:, 1:4] ** 2).sum(1) + 1.5 * W[:, 0] * W[:, 4]])
    V = torch.from_numpy(np.stack([V1] * N)).cuda()
    span = wk.T / N
    n, _ = bgk.n_steps(p, span, E=wk.E)
    E = torch.from_numpy(wk.E).cuda()
    bgk.fine_propagate_moments(p, V, span, E=E)
    torch.cuda.synchronize()
    bgk.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        bgk.fine_propagate_moments(p, V, span, E=E)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    ms, launches, upd, by = bgk.prof_read(bgk.PROF_ONE_STEP)
    bgk.prof_enable(False)
    bgk.check_status()
    return {"workload": wk.name + f"_slices{N}", "steps": n,
            "updates_per_s": N * p.cells * n / el, "ms_per_call": round(el * 1e3, 3),
            "step_kernel_GBs": round(by / (ms * 1e-3) / 1e9, 1),
            "step_kernel_avg_us": round(ms * 1e3 / max(launches, 1), 2)}


def uneven_throughput(torch, bgk, wl, span=0.1, reps=3):
    """The uneven multi-instance batch (seeded Riemann problems with Nx in
    [128, 1024], Nv in [16, 32], eps in [1e-4, 1]) advanced together: every
    instance's first step alone, then per round one two-step pass over the
    instances with two or more steps left and one step for those with one
    left (the library's built-in setting; instances with odd Nv on padded
    copies), and, for comparison, one step per launch.  Instances 7, 15 and
    29 are left out: their cold states are not
    resolved on their velocity grids (theta / dv^2 = 0.11, 0.29, 0.33) and
    their temperatures collapse within the span, in the oracle too."""
    insts = [w for q, w in enumerate(wl.c5_uneven()) if q not in (7, 15, 29)]
    probs = [w.problem for w in insts]
    fs = [bgk.lift(w.problem, torch.from_numpy(w.W0).cuda()) for w in insts]
    spans = [span] * len(insts)
    outs, steps = bgk.fine_step_batched(probs, fs, spans)
    note = None
    if bgk.status() != bgk.OK:
        # a state went non-physical over the whole span: time the short one
        note = f"non-physical state flagged over span {span}; timed over 0.01"
        span = 0.01
        spans = [span] * len(insts)
        outs, steps = bgk.fine_step_batched(probs, fs, spans)
        bgk.check_status()
    n_upd = sum(p.cells * n for p, n in zip(probs, steps))

    def timed():
        bgk.fine_step_batched(probs, fs, spans, outs)
        torch.cuda.synchronize()
        bgk.prof_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            bgk.fine_step_batched(probs, fs, spans, outs)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        kinds = {name: bgk.prof_read(kind) for name, kind in
                 (("three_step_pass", bgk.PROF_THREE_STEP), ("two_step_pass", bgk.PROF_TWO_STEP),
                  ("one_step", bgk.PROF_ONE_STEP))}
        bgk.prof_enable(False)
        bgk.check_status()
        return el, kinds

    el, kinds = timed()
    line = {"workload": f"uneven_{len(insts)}_instances", "span": span,
            "steps_min_max": [min(steps), max(steps)],
            "cells": sum(p.cells for p in probs), "updates_per_s": n_upd / el,
            "ms_per_call": round(el * 1e3, 3)}
    if note:
        line["note"] = note
    for name, (ms, launches, upd, by) in kinds.items():
        if launches:
            line[name + "_GBs"] = round(by / (ms * 1e-3) / 1e9, 1)
            line[name + "_avg_us"] = round(ms * 1e3 / launches, 2)
            line[name + "_launches"] = launches
    # the fused passes together: algorithmic bytes over their kernel time
    f_ms = sum(kinds[k][0] for k in ("three_step_pass", "two_step_pass"))
    f_by = sum(kinds[k][3] for k in ("three_step_pass", "two_step_pass"))
    if f_ms > 0:
        line["fused_passes_GBs"] = round(f_by / (f_ms * 1e-3) / 1e9, 1)
    bgk.set_step_fusion(1)
    try:
        el1, _ = timed()
    finally:
        bgk.set_step_fusion(3)
    line["one_step_per_launch_updates_per_s"] = n_upd / el1
    return line


def adjoint_timing(torch, bgk, wl, reps=3):
    """Gradients of the final-time density misfit with respect to the initial
    density and log eps through the fine solve (Nx=256, 24^3 velocities,
    393 steps, checkpoints every 16 steps): forward and backward wall-clock,
    median of `reps` after a warm-up."""
    import numpy as np
    wk, rho0, eps_t, _ = wl.c4_adjoint()
    p = wk.problem
    n, _ = bgk.n_steps(p, wk.T)
    r0 = torch.tensor(rho0, dtype=torch.float64, device="cuda", requires_grad=True)
    le = torch.tensor(np.log(p.eps), dtype=torch.float64, device="cuda", requires_grad=True)
    with torch.no_grad():
        target = bgk.kinetic_density(r0.detach(), torch.tensor(np.log(eps_t), dtype=torch.float64,
                                                               device="cuda"), p, T=wk.T)

    def once():
        r0.grad, le.grad = None, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho = bgk.kinetic_density(r0, le, p, T=wk.T, ckpt_every=16)
        loss = 0.5 * (1.0 / p.nx) * torch.sum((rho - target) ** 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1

    once()
    ts = [once() for _ in range(reps)]
    bgk.check_status()
    fw = float(np.median([t[0] for t in ts]))
    bw = float(np.median([t[1] for t in ts]))
    n_ck = (n + 15) // 16
    return {"workload": f"adjoint_nx{p.nx}_nv{p.nv[0]}", "steps": n, "checkpoint_every": 16,
            "checkpoint_bytes": n_ck * p.cells * 8, "forward_ms": round(fw * 1e3, 2),
            "backward_ms": round(bw * 1e3, 2), "backward_over_forward": round(bw / fw, 2),
            "forward_updates_per_s": p.cells * n / fw}


def second_order_throughput(torch, bgk, V, p, span, reps=2):
    """The second-order (van Leer limited) fine transport on the benchmark
    batch: one step per pass (16 algorithmic bytes per update)."""
    n, _ = bgk.n_steps(p, span)
    bgk.fine_propagate_moments(p, V, span, fine_order=2)
    torch.cuda.synchronize()
    bgk.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        bgk.fine_propagate_moments(p, V, span, fine_order=2)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    ms, launches, upd, by = bgk.prof_read(bgk.PROF_ONE_STEP)
    bgk.prof_enable(False)
    bgk.check_status()
    B = V.shape[0]
    return {"workload": f"smooth_periodic_nx{p.nx}_nv{p.nv[0]}_slices{B}", "steps": n,
            "updates_per_s": B * p.cells * n / el, "ms_per_call": round(el * 1e3, 3),
            "step_kernel_GBs": round(by / (ms * 1e-3) / 1e9, 1),
            "step_kernel_avg_us": round(ms * 1e3 / max(launches, 1), 2)}


def time_batch(torch, bgk, p, V, span, steps, warmup):
    """Times `steps` calls of the batched propagation (lift, fine steps,
    projection) of the slices V after `warmup` calls, with the step kernels'
    launches bracketed by HIP events on their stream.  Returns (seconds,
    {kind: (ms, launches, updates, bytes)})."""
    Vd = torch.from_numpy(V).cuda()
    for _ in range(warmup):
        bgk.fine_propagate_moments(p, Vd, span)
    bgk.check_status()
    torch.cuda.synchronize()
    bgk.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = bgk.fine_propagate_moments(p, Vd, span)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kinds = {k: bgk.prof_read(kind) for k, kind in
             (("three", bgk.PROF_THREE_STEP), ("two", bgk.PROF_TWO_STEP),
              ("all", bgk.PROF_ALL))}
    bgk.prof_enable(False)
    bgk.check_status()
    assert out is None or torch.isfinite(out).all().item()
    return elapsed, kinds


def roofline_of(workload, kinds, updates_per_step, steps, elapsed):
    """Roofline of the dominant kernel, the three-step relax pass (or the
    two-step pass where no three-step pass ran), from the HIP-event timing.
    `frac` uses the pass's own algorithmic bytes: one read and one write of f
    per pass (16 B per cell per pass: 16/3 B per phase-space update with
    three steps per pass, 8 with two); `frac_at_16B_per_update` prices the
    same updates at one read and one write of f per IMEX step."""
    which = "three" if kinds["three"][1] else "two"
    k_ms, k_launches, k_upd, k_bytes = kinds[which]
    a_ms, a_launches, a_upd, a_bytes = kinds["all"]
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    per_launch_alg = k_bytes / max(k_launches, 1)
    pass_ups = k_upd / (k_ms * 1e-3)
    traffic = traffic_from_profile(workload, which)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "frac_basis": ("algorithmic bytes of the pass: one read and one write of f per "
                           f"{'three' if which == 'three' else 'two'}-step pass "
                           f"({k_bytes / max(k_upd, 1.0):.3f} B per phase-space update)"),
            "frac_at_16B_per_update": round(pass_ups * 16.0 / (HBM_PEAK_GBS * 1e9), 4),
            "traffic_over_alg_bytes": (round(traffic / per_launch_alg, 4) if traffic else None),
            "kernel": ("k_step3x relax passes (three IMEX steps per pass over f)"
                       if which == "three" else
                       "k_step2x2 relax passes (two IMEX steps per pass over f)"),
            "launches": k_launches, "avg_launch_us": round(k_ms * 1e3 / max(k_launches, 1), 2),
            "alg_bytes_per_launch": per_launch_alg,
            "alg_bytes_per_update": round(k_bytes / max(k_upd, 1.0), 3),
            "pass_updates_per_s": pass_ups,
            "all_step_kernels": {
                "launches": a_launches,
                "avg_launch_us": round(a_ms * 1e3 / max(a_launches, 1), 2),
                "achieved": round(a_bytes / (a_ms * 1e-3) / 1e9, 1),
                "alg_bytes_per_update": round(a_bytes / max(a_upd, 1.0), 3),
                "share_of_wall_clock": round(a_ms * 1e-3 / elapsed, 4)}}


def pow2_ceil(n):
    v = 1
    while v < n:
        v <<= 1
    return v


def tile_entry(path, arch, p, B, fuse=3):
    """The tile-file entry of this grid class (velocity grid, nx and batch
    rounded up to powers of two, steps per pass) for `arch`, or None."""
    if not os.path.exists(path):
        return None
    for e in json.load(open(path)).get("entries", []):
        if (e["arch"] == arch and e["nv"] == list(p.nv) and e["nx_bucket"] == pow2_ceil(p.nx)
                and e["batch_bucket"] == pow2_ceil(B) and e["steps_per_pass"] == fuse):
            return e
    return None


def tuned_tiles(torch, bgk, p, B, cache):
    """Tiles of the grid class from the tile file, else measured now by
    bgk_autotune (and the file rewritten).  Returns a description for the
    bench line."""
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    e = tile_entry(cache, arch, p, B)
    if e is not None:
        bgk.load_tiles(cache)
        return {"source": "autotune (tile file)", "elems": e["elems"], "chunk": e["chunk"],
                "pair": e["pair"], "arch": arch}
    t0 = time.perf_counter()
    el, ch, pr = bgk.autotune(p, B)
    took = time.perf_counter() - t0
    if os.path.exists(cache):
        bgk.load_tiles(cache)  # keep the file's other entries
    bgk.save_tiles(cache)
    log(f"autotuned {p.nx}x{p.nv} x{B}: elems {el}, chunk {ch}, pair {pr} ({took:.1f} s)")
    return {"source": "autotune (measured in this run)", "elems": el, "chunk": ch, "pair": pr,
            "arch": arch, "autotune_s": round(took, 2)}


def batch_line(torch, bgk, name, steps, warmup, eps=None, cache=None):
    """Throughput and roofline of one benchmark batch, with autotuned tiles
    when a tile file path is given (and the built-in choice timed beside
    them)."""
    wk, V, span = workload_batch(name, eps)
    p = wk.problem
    B = V.shape[0]
    n_fine, _ = bgk.n_steps(p, span)
    virt = steps_on_moments(n_fine)
    updates_per_step = B * p.cells * n_fine
    tiles = None
    if cache:
        tiles = tuned_tiles(torch, bgk, p, B, cache)
        # the built-in choice on the same batch: a plan without tuned shapes
        with bgk.Plan():
            el_h, _ = time_batch(torch, bgk, p, V, span, max(1, min(steps, 2)), 1)
        tiles["builtin_ms_per_step"] = round(el_h / max(1, min(steps, 2)) * 1e3, 2)
    elapsed, kinds = time_batch(torch, bgk, p, V, span, steps, warmup)
    if tiles is not None:
        tiles["tuned_ms_per_step"] = round(elapsed / steps * 1e3, 2)
    cfg = {"workload": f"{wk.name.split('_eps')[0]}_slices{B}", "nx": p.nx, "nv": list(p.nv),
           "v_box": [p.v_lo[0], p.v_hi[0]], "slices_batched": B,
           "fine_steps_per_slice": n_fine, "steps_applied_to_f": n_fine - virt,
           "last_steps_on_moments": virt, "eps": p.eps,
           "bc": "periodic" if p.bc == 1 else "neumann", "updates_per_step": updates_per_step,
           "updates_per_step_applied_to_f": B * p.cells * (n_fine - virt)}
    line = {"value": updates_per_step * steps / elapsed,
            "value_steps_applied_to_f": B * p.cells * (n_fine - virt) * steps / elapsed,
            "ms_per_step": elapsed / steps * 1e3, "config": cfg,
            "roofline": roofline_of(name, kinds, updates_per_step, steps, elapsed)}
    if tiles is not None:
        line["tiles"] = tiles
    return line, wk, V, span


def smooth_section(torch, bgk, steps=5, warmup=1, cache=None):
    """The smooth periodic workload (64 slices of 512 x 32^3, 25 steps per
    slice, the last two evaluated on the moments) at its three Knudsen
    numbers (autotuned tiles), and with two steps per pass at eps = 1e-2 for
    comparison."""
    out = []
    for eps in (1.0, 1e-2, 1e-4):
        line, _, _, _ = batch_line(torch, bgk, "smooth_periodic", steps, warmup, eps,
                                   cache=cache if eps == 1e-2 else None)
        line["config"]["eps"] = eps
        out.append(line)
    bgk.set_step_fusion(2)
    try:
        two, _, _, _ = batch_line(torch, bgk, "smooth_periodic", 3, 1, 1e-2)
        two["steps_per_pass"] = 2
        two["roofline"]["traffic"] = traffic_from_profile("smooth_periodic", "two")
        out.append(two)
    finally:
        bgk.set_step_fusion(3)
    bgk.free_workspaces()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sod_large", choices=["sod_large", "smooth_periodic"])
    ap.add_argument("--eps", type=float, default=None,
                    help="Knudsen number of the smooth periodic main line (default 1e-2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parareal", action="store_true",
                    help="skip every section after the main line (same as --extras '')")
    ap.add_argument("--extras", default="smooth,parareal,parareal_large,force,order2,uneven,adjoint",
                    help="comma list of the extra sections: smooth, parareal, parareal_large, "
                         "force, order2, uneven, adjoint")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--tile-cache", default=TILE_CACHE,
                    help="JSON file of autotuned tiles (read, and written when a grid class "
                         "is tuned in this run)")
    ap.add_argument("--builtin-tiles", action="store_true",
                    help="time the built-in tile choice only (no autotuning)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel directly instead of replaying captured HIP "
                         "graphs (counter-collection runs)")
    ap.add_argument("--only", default="",
                    help="run only these extra sections (comma list, as --extras), without "
                         "the main line or the CPU baseline (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding the "
              "slices over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_02704_amd import bgk
    from paper_2502_02704_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.no_graphs:
        bgk.set_graphs(False)
    cache = None if args.builtin_tiles else args.tile_cache
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only:
        only = {x for x in args.only.split(",") if x}
        line = {"metric": METRIC, "only": sorted(only)}
        sections = {"smooth": ("smooth_periodic", lambda: smooth_section(torch, bgk, cache=cache)),
                    "parareal": ("parareal", lambda: parareal_small(torch, bgk, wl)),
                    "parareal_large": ("parareal_baseline_sizes",
                                       lambda: parareal_large(torch, bgk, wl)),
                    "force": ("exterior_force", lambda: force_throughput(torch, bgk, wl)),
                    "uneven": ("uneven_batch", lambda: uneven_throughput(torch, bgk, wl)),
                    "adjoint": ("adjoint", lambda: adjoint_timing(torch, bgk, wl))}
        for name in sorted(only):
            if name == "order2":
                wk2, V2, span2 = workload_batch("smooth_periodic")
                line["second_order_fine"] = second_order_throughput(
                    torch, bgk, torch.from_numpy(V2).cuda(), wk2.problem, span2)
            else:
                key, fn = sections[name]
                line[key] = fn()
            log(f"{name} done")
        print(json.dumps(line), flush=True)
        return
    main_line, wk, V_np, span = batch_line(torch, bgk, args.workload, args.steps, args.warmup,
                                           args.eps, cache=cache)
    log(f"main line {main_line['config']['workload']}: {main_line['value']:.4g} updates/s, "
        f"{main_line['ms_per_step']:.1f} ms per step")
    bgk.free_workspaces()
    torch.cuda.empty_cache()


    line = {"metric": METRIC, "value": main_line["value"], "unit": "updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_line["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": main_line["config"],
            "value_steps_applied_to_f": main_line["value_steps_applied_to_f"],
            "roofline": main_line["roofline"]}
    if "tiles" in main_line:
        line["tiles"] = main_line["tiles"]
    extras = set() if args.no_parareal else {x for x in args.extras.split(",") if x}
    if "smooth" in extras and args.workload == "sod_large":
        line["smooth_periodic"] = smooth_section(torch, bgk, cache=cache)
        log("smooth periodic section done")
    if "parareal" in extras:
        line["parareal"] = parareal_small(torch, bgk, wl)
        log("parareal, small cases done")
    if "parareal_large" in extras:
        line["parareal_baseline_sizes"] = parareal_large(torch, bgk, wl)
        log("parareal, baseline sizes done")
    if "force" in extras:
        line["exterior_force"] = force_throughput(torch, bgk, wl)
        log("exterior force done")
    if "order2" in extras:
        wk2, V2, span2 = workload_batch("smooth_periodic")
        line["second_order_fine"] = second_order_throughput(
            torch, bgk, torch.from_numpy(V2).cuda(), wk2.problem, span2)
        bgk.free_workspaces()
        torch.cuda.empty_cache()
        log("second-order section done")
    if "uneven" in extras:
        line["uneven_batch"] = uneven_throughput(torch, bgk, wl)
        log("uneven batch done")
    if "adjoint" in extras:
        line["adjoint"] = adjoint_timing(torch, bgk, wl)
        log("adjoint done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wk, V_np, span)
        log("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
