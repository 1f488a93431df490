"""Benchmark of the fine kinetic propagator on one MI355X.

A step = one pass of the whole hot path over one batch: every one of the 64
parareal slices of the smooth periodic workload (Nx=512, 32^3 velocities on
[-8,8]^3, eps=1e-2) is lifted from its moments, advanced by one slice (25 IMEX
steps, three per pass over f where possible) and projected back to moments,
all slices batched in one launch per pass.  The call returns moments only, so
the last two steps are evaluated on their moments (from weighted sums of the
23rd field, by linearity of the transport) rather than written out as f: a
two-step pass from the lift, then seven three-step passes.  Prints one JSON line: phase-space
updates/s, the roofline of the dominant kernel (the three-step relax pass; the
two-step pass is timed beside it), the CPU oracle timed on a bounded sample,
and the parareal vs serial-fine speedup on small workloads where one slice's
step is latency bound.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--eps E]
       [--no-cpu-baseline] [--no-parareal] [--extras parareal,force,order2,uneven,adjoint]
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
    "three": os.path.join(ROOT, "profiles", "k_step3x_smooth_periodic_traffic.md"),
    "two": os.path.join(ROOT, "profiles", "k_step2x2_smooth_periodic_traffic.md"),
}
KERNEL_SRC = os.path.join(ROOT, "paper_2502_02704_amd", "csrc", "kinetic.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


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


def traffic_from_profile(which):
    """HBM bytes per launch of the three- or two-step pass from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source;
    else None."""
    path = TRAFFIC_SUMMARY[which]
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


def cpu_baseline(wk, V, span, budget_s=12.0, max_slices=64):
    """The oracle as it stands, on slices of the same batch until the budget
    is spent (at least one slice)."""
    import oracle
    p = wk.problem
    n, _ = oracle.n_steps(p, span)
    t0 = time.perf_counter()
    done = 0
    while done < max_slices:
        oracle.fine_propagate_moments(p, V[done], span)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    upd = done * p.cells * n
    cores = oracle.get_threads()
    # the same oracle on one thread, one slice
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.fine_propagate_moments(p, V[0], span)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    return {"value": upd / el, "unit": "updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{done} of {V.shape[0]} slices (lift + {n} IMEX steps + projection "
                      f"each, {p.nx}x{p.nv[0]}^3), {el:.1f} s",
            "value_1_thread": p.cells * n / el1}


def parareal_speedup(torch, bgk, wl, reps=5):
    """Parareal vs the serial chained fine solve with the same kernels and the
    same launch machinery (captured graphs on both sides), on small workloads
    where one slice's step is launch-latency bound -- the only regime where
    one GPU can gain (larger slices are bandwidth bound, and parareal then
    does more fine work than the serial solve).  Error = max over slices,
    cells and components of |U_parareal - U_serial| (conserved moments);
    reports the smallest K reaching 1e-6."""
    import numpy as np

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return out, float(np.median(ts))

    sod = wl.c1_sod_small()
    s4 = wl.c2_smooth_periodic(eps=1e-4, nx=64, nv=16, n_slices=16)
    s2 = wl.c2_smooth_periodic(eps=1e-2, nx=64, nv=16, n_slices=16)
    fk = wl.c6_two_beam_force()
    cases = [(sod.name, sod.problem, sod.W0, sod.n_slices, sod.T, None, "euler"),
             (s4.name, s4.problem, s4.W0, s4.n_slices, s4.T, None, "euler"),
             (s4.name, s4.problem, s4.W0, s4.n_slices, s4.T, None, "cns"),
             (s2.name, s2.problem, s2.W0, s2.n_slices, s2.T, None, "euler"),
             (s2.name, s2.problem, s2.W0, s2.n_slices, s2.T, None, "cns"),
             (fk.name, fk.problem, fk.U0(), fk.n_slices, fk.T, fk.E, "euler")]
    cases = [c + (0,) for c in cases]
    # the multiscale variant: Navier-Stokes coarse model with the order-one
    # (Chapman-Enskog) lifting, against the serial chain with the same lifting
    cases.append((s2.name, s2.problem, s2.W0, s2.n_slices, s2.T, None, "cns", 1))
    out = []
    for name, p, W0np, N, T, E, coarse, lo in cases:
        W0 = torch.from_numpy(W0np).cuda()
        ref, t_serial = timed(lambda: bgk.serial_fine(p, W0, N, T, E=E, lift_order=lo))
        ref = ref.cpu().numpy()
        res = {"workload": name, "coarse": coarse, "lift_order": lo, "slices": N,
               "serial_fine_ms": round(t_serial * 1e3, 4), "K": []}
        chosen = None
        for K in range(1, N + 1):
            (V, err, kd), t_par = timed(lambda: bgk.parareal_iterate(p, W0, N, T, K, 0.0, E=E,
                                                                     coarse=coarse,
                                                                     lift_order=lo))
            e = float(np.max(np.abs(V.cpu().numpy() - ref)))
            res["K"].append({"K": K, "ms": round(t_par * 1e3, 4), "err_vs_fine": e,
                             "speedup": round(t_serial / t_par, 3)})
            if e <= 1e-6:
                chosen = res["K"][-1]
                break
        res["K_at_1e-6"] = chosen["K"] if chosen else None
        res["speedup_at_1e-6"] = chosen["speedup"] if chosen else None
        out.append(res)
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


def uneven_throughput(torch, bgk, wl, span=0.01, reps=3):
    """The uneven multi-instance batch (seeded Riemann problems with Nx in
    [128, 1024], Nv in [16, 32], eps in [1e-4, 1]) advanced together: every
    instance's first step alone, then per round one two-step pass over the
    instances with two or more steps left and one step for those with one
    left (the library's built-in setting), and, for comparison, one step per
    launch.  Instances 7, 15 and 29 are left out: their cold states are not
    resolved on their velocity grids (theta / dv^2 = 0.11, 0.29, 0.33) and
    their temperatures collapse within the span, in the oracle too."""
    insts = [w for q, w in enumerate(wl.c5_uneven()) if q not in (7, 15, 29)]
    probs = [w.problem for w in insts]
    fs = [bgk.lift(w.problem, torch.from_numpy(w.W0).cuda()) for w in insts]
    spans = [span] * len(insts)
    outs, steps = bgk.fine_step_batched(probs, fs, spans)
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
                 (("two_step_pass", bgk.PROF_TWO_STEP), ("one_step", bgk.PROF_ONE_STEP))}
        bgk.prof_enable(False)
        bgk.check_status()
        return el, kinds

    el, kinds = timed()
    line = {"workload": f"uneven_{len(insts)}_instances", "span": span,
            "steps_min_max": [min(steps), max(steps)],
            "cells": sum(p.cells for p in probs), "updates_per_s": n_upd / el,
            "ms_per_call": round(el * 1e3, 3)}
    for name, (ms, launches, upd, by) in kinds.items():
        if launches:
            line[name + "_GBs"] = round(by / (ms * 1e-3) / 1e9, 1)
            line[name + "_avg_us"] = round(ms * 1e3 / launches, 2)
            line[name + "_launches"] = launches
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parareal", action="store_true",
                    help="skip every section after the main line (same as --extras '')")
    ap.add_argument("--extras", default="parareal,force,order2,uneven,adjoint",
                    help="comma list of the extra sections: parareal, force, order2, uneven, "
                         "adjoint")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding the "
              "slices over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2502_02704_amd import bgk
    from paper_2502_02704_amd import workloads as wl

    torch.cuda.set_device(0)
    wk = wl.c2_smooth_periodic(eps=args.eps)
    p = wk.problem
    B = wk.n_slices
    span = wk.T / wk.n_slices
    n_fine, _ = bgk.n_steps(p, span)
    V_np = slice_moments(wk, B)
    V = torch.from_numpy(V_np).cuda()
    updates_per_step = B * p.cells * n_fine

    for _ in range(args.warmup):
        bgk.fine_propagate_moments(p, V, span)
    bgk.check_status()
    torch.cuda.synchronize()

    bgk.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = bgk.fine_propagate_moments(p, V, span)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    which = "three"
    k_ms, k_launches, k_upd, k_bytes = bgk.prof_read(bgk.PROF_THREE_STEP)
    if k_launches == 0:
        which = "two"
        k_ms, k_launches, k_upd, k_bytes = bgk.prof_read(bgk.PROF_TWO_STEP)
    a_ms, a_launches, a_upd, a_bytes = bgk.prof_read(bgk.PROF_ALL)
    bgk.prof_enable(False)
    bgk.check_status()
    assert torch.isfinite(out).all().item()

    # the same batch with two steps per pass, for comparison
    two = None
    if which == "three":
        bgk.set_step_fusion(2)
        try:
            bgk.fine_propagate_moments(p, V, span)
            torch.cuda.synchronize()
            bgk.prof_enable(True)
            reps2 = max(1, min(args.steps, 3))
            t2 = time.perf_counter()
            for _ in range(reps2):
                bgk.fine_propagate_moments(p, V, span)
            torch.cuda.synchronize()
            el2 = (time.perf_counter() - t2) / reps2
            m2, l2, u2, b2 = bgk.prof_read(bgk.PROF_TWO_STEP)
            bgk.prof_enable(False)
            bgk.check_status()
        finally:
            bgk.set_step_fusion(3)
        ach2 = b2 / (m2 * 1e-3) / 1e9
        two = {"kernel": "k_step2x2 relax passes (two IMEX steps per pass over f)",
               "updates_per_s": updates_per_step / el2, "ms_per_step": round(el2 * 1e3, 3),
               "achieved": round(ach2, 1), "frac": round(ach2 / HBM_PEAK_GBS, 4),
               "avg_launch_us": round(m2 * 1e3 / max(l2, 1), 2), "launches": l2,
               "alg_bytes_per_update": round(b2 / max(u2, 1.0), 3),
               "traffic": traffic_from_profile("two")}

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    value = updates_per_step * args.steps / elapsed
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    per_launch_alg = k_bytes / max(k_launches, 1)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_from_profile(which),
                "kernel": ("k_step3x relax passes (three IMEX steps per pass over f)"
                           if which == "three" else
                           "k_step2x2 relax passes (two IMEX steps per pass over f)"),
                "launches": k_launches, "avg_launch_us": round(k_ms * 1e3 / max(k_launches, 1), 2),
                "alg_bytes_per_launch": per_launch_alg,
                "alg_bytes_per_update": round(k_bytes / max(k_upd, 1.0), 3),
                "all_step_kernels": {
                    "launches": a_launches, "avg_launch_us": round(a_ms * 1e3 / max(a_launches, 1), 2),
                    "achieved": round(a_bytes / (a_ms * 1e-3) / 1e9, 1),
                    "alg_bytes_per_update": round(a_bytes / max(a_upd, 1.0), 3)}}
    if which == "three":
        # the pass's own updates/s against the HBM ceiling of a two-steps-per-pass
        # design (8 B per update): what moving a third fewer bytes buys
        pass_ups = k_upd / (k_ms * 1e-3)
        roofline["pass_updates_per_s"] = pass_ups
        roofline["frac_of_8B_per_update_ceiling"] = round(pass_ups / (HBM_PEAK_GBS * 1e9 / 8.0), 4)
    if two is not None:
        roofline["two_step_pass"] = two
    line = {"metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"smooth_periodic_nx{p.nx}_nv{p.nv[0]}_slices{B}",
                       "nx": p.nx, "nv": list(p.nv), "slices_batched": B,
                       "fine_steps_per_slice": n_fine,
                       "last_steps_on_moments": (n_fine - 2) % 3 if n_fine >= 4 else 0,
                       "eps": p.eps, "bc": "periodic",
                       "updates_per_step": updates_per_step},
            "roofline": roofline}
    extras = set() if args.no_parareal else {x for x in args.extras.split(",") if x}
    if "parareal" in extras:
        line["parareal"] = parareal_speedup(torch, bgk, wl)
    if "force" in extras:
        line["exterior_force"] = force_throughput(torch, bgk, wl)
    if "order2" in extras:
        line["second_order_fine"] = second_order_throughput(torch, bgk, V, p, span)
    if "uneven" in extras:
        line["uneven_batch"] = uneven_throughput(torch, bgk, wl)
    if "adjoint" in extras:
        line["adjoint"] = adjoint_timing(torch, bgk, wl)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wk, V_np, span)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
