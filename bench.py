"""Throughput benchmark of the EM-PIC step on one MI355X.

One step = sort (every 4 steps, amortised) + fused gather/Boris/position/
Esirkepov tile kernel + Yee update + FP64 reductions, over a 256^3 periodic
uniform plasma with 8 particles per cell (134,217,728 particles), order-3
shapes, u_th = 0.05c, in split precision (int32 cell + FP32 offset, FP32
fields and momenta).  Companion measurements on the same GPU: the same
workload in FP64, and one adjoint step against one forward step.  Inputs are
seeded synthetic particles drawn on the device; nothing is read from disk.

Prints one JSON line.  Kernel times come from HIP events the library records
on the launch stream (pic_timing); the CPU baseline is the FP64 oracle timed
on a bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (gather+push+deposit+Yee), FP32 vs FP64, fwd vs adjoint"
HBM_PEAK_GBS = 8000.0
# vector FMA peak with packed FP32 disabled: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
VALU_PEAK_TFLOPS = 78.6
# algorithmic flops of one order-3 particle step that stays in its cell
# (weights 105, gather 6 x 84 FMA = 1008, Boris 68, position 28, Esirkepov
# shapes 123, Esirkepov products and sums 696); order 1: weights 9, gather
# 6 x 14 FMA = 168, Boris 68, position 28, Esirkepov shapes 12, products and
# sums 126
FLOPS_PER_PARTICLE = {3: 2028, 1: 411}
# calibrated HBM bytes per launch of the FP32 two-phase tile kernel at
# 256^3 / 8 ppc, from the FETCH_SIZE / WRITE_SIZE passes (scaled by a 1 GiB
# copy); only figures taken on the current kernel are listed
MEASURED_TRAFFIC = {"uniform256_o3_f32": 17.49e9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def particle_bytes(n, tsize, has_w):
    # state read + written once: 3 int32 cells, 3 offsets, 3 momenta (+ weight read)
    return n * (2 * (3 * 4 + 6 * tsize) + (tsize if has_w else 0))


def field_bytes(ncell, tsize):
    # E, B read once and J read+written once per cell
    return ncell * (6 * tsize + 6 * tsize)


def run_forward(w, steps, warmup, sort_every, label):
    import torch
    from paper_2101_12149_amd import _lib
    g = w.grid
    sp, f = w.species, w.fields
    dtype = w.dtype
    ws = _lib.workspace(g, dtype, sp.n)
    ts = torch.zeros(_lib.pic_tile_count(g, dtype) + 1, dtype=torch.int32, device="cuda")
    diag = torch.zeros((max(steps, warmup, 1), 5), dtype=torch.float64, device="cuda")
    src = w.source
    log(f"[{label}] warmup {warmup} steps, {sp.n} particles")
    if sort_every == 0:   # a workload that keeps one binning (the rollout's) is sorted once, untimed
        _lib.pic_sort_tiles(g, sp, ts, ws)
    _lib.pic_step(g, sp, f, src, 0, warmup, sort_every, ts, ws, diag[:max(warmup, 1)])
    torch.cuda.synchronize()
    _lib.pic_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    _lib.pic_step(g, sp, f, src, warmup, steps, sort_every, ts, ws, diag[:steps])
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = _lib.pic_timing(False)
    ev_ms = e0.elapsed_time(e1)
    log(f"[{label}] {steps} steps: {ev_ms:.2f} ms (events), {wall * 1e3:.2f} ms (wall)")
    return dict(ms=ev_ms, wall_ms=wall * 1e3, kernels=kt, diag=diag[:steps].cpu().numpy(), ws=ws, ts=ts)


def run_adjoint(w, nrep, tile_start):
    """Adjoint steps as the differentiable rollout runs them: its reverse
    sweep bins each replay segment afresh at the segment's checkpoint, so the
    state the forward run ended in is re-binned and advanced two steps (the
    middle of a 5-step segment), untimed, before the adjoint steps are timed."""
    import torch
    from paper_2101_12149_amd import _lib
    g = w.grid
    sp, f = w.species, w.fields
    ws = _lib.workspace(g, w.dtype, sp.n)
    src = w.source
    if tile_start is not None:
        _lib.pic_sort_tiles(g, sp, tile_start, ws)
        _lib.pic_step(g, sp, f, src, 0, 2, 0, tile_start, ws)
        torch.cuda.synchronize()

    class Lam:
        pass
    lam = Lam()
    tdt = sp.off.dtype
    lam.lx = torch.zeros_like(sp.off)
    lam.lu = torch.zeros_like(sp.u)
    lam.lE = f.E.clone()
    lam.lB = f.B.clone()
    dA = None
    if src is not None:   # the source map's gradient is accumulated in FP64, as the rollout does
        dA = torch.zeros(tuple(src.amp.shape), dtype=torch.float64, device=src.amp.device)
    _lib.pic_step_adjoint(g, sp, f, src, 0, lam, dA, ws, tile_start=tile_start)   # warm
    torch.cuda.synchronize()
    _lib.pic_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(nrep):
        _lib.pic_step_adjoint(g, sp, f, src, r, lam, dA, ws, tile_start=tile_start)
    e1.record()
    torch.cuda.synchronize()
    kt = _lib.pic_timing(False)
    del tdt
    return dict(ms=e0.elapsed_time(e1), kernels=kt)


def tile_kernel_name(npart, ncell, tsize, order):
    """The fused particle kernel the library runs: the two-phase one for
    FP32 order 3 at 6 or more particles per cell, else the one-pass one."""
    return "k_particles_cells" if tsize == 4 and order == 3 and npart >= 6 * ncell else "k_particles_tile"


def kernel_roofs(kernels, npart, ncell, tsize, has_w, order):
    """The fused tile kernel's mean launch time and its HBM and ALU
    fractions from the algorithmic bytes and flops per particle-step."""
    ms, n = kernels["particles"]
    avg = ms / max(n, 1)
    alg_bytes = particle_bytes(npart, tsize, has_w) + field_bytes(ncell, tsize)
    gbs = alg_bytes / (avg * 1e-3) / 1e9
    tfs = FLOPS_PER_PARTICLE[order] * npart / (avg * 1e-3) / 1e12
    return {"kernel": tile_kernel_name(npart, ncell, tsize, order), "avg_ms": round(avg, 4),
            "alg_bytes_per_particle": round(alg_bytes / npart, 2),
            "hbm_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "alu_TFLOPs": round(tfs, 2),
            "alu_frac": round(tfs / VALU_PEAK_TFLOPS, 4)}


def run_rollout(w, label):
    """The differentiable rollout as a user runs it: forward (checkpoints
    every w.checkpoint_every steps, one binning) for the loss, then the
    reverse sweep (re-binning and replay per segment, adjoint steps) for
    dL/du0 and dL/damp.  Wall time of each half, synchronised."""
    import torch
    from paper_2101_12149_amd import rollout
    pb = rollout.Problem(w.grid, w.species, w.fields, w.source, w.nsteps, w.checkpoint_every or 5, w.dtype)
    times = []
    for _ in range(2):   # the first run pays the first calls' set-up; the second is reported
        u0 = w.species.u.clone().requires_grad_(True)
        amp = w.source.amp.clone().requires_grad_(True) if w.source is not None else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = rollout.rollout_loss(u0, amp, pb)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append(((t1 - t0) * 1e3, (t2 - t1) * 1e3))
    (fwd0, bwd0), (fwd, bwd) = times
    log(f"[{label}] rollout {w.nsteps} steps: forward {fwd:.1f} ms, reverse sweep {bwd:.1f} ms "
        f"(first run {fwd0:.1f} / {bwd0:.1f} ms)")
    return {"steps": w.nsteps, "checkpoint_every": pb.k, "forward_ms": round(fwd, 3), "backward_ms": round(bwd, 3),
            "ratio_backward_over_forward": round(bwd / fwd, 4),
            "first_run_ms": [round(fwd0, 3), round(bwd0, 3)],
            "grad_u0_norm": float(u0.grad.double().norm()),
            "grad_amp_norm": float(amp.grad.double().norm()) if amp is not None else None}


# the other workloads, each with its own step count: (name, timed steps,
# warm-up steps, timed adjoint steps, rollout window in steps or 0)
CONFIGS = (("uniform32_o1_f64", 10, 2, 3, 0),
           ("laser128x128x1024_o3_f32", 40, 4, 5, 0),
           ("diff64_o3_f64", 20, 2, 5, 20),
           ("stress512_o3_f32", 40, 4, 3, 20))


def bench_config(name, steps, warmup, nadj, window):
    import torch
    from paper_2101_12149_amd import workloads as wl
    w = wl.named(name, device="cuda")
    g = w.grid
    npart, ncell = w.species.n, g.ncells
    tsize = 4 if w.dtype == "f32" else 8
    init = (w.species.clone(), w.fields.clone()) if window else None
    fw = run_forward(w, steps, warmup, w.sort_every, name)
    ms = fw["ms"] / steps
    row = {"cells": list(g.n), "particles": npart, "dtype": w.dtype, "order": g.order, "sort_every": w.sort_every,
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
           "particle_steps_per_s": npart * steps / (fw["ms"] * 1e-3),
           "kernels_ms_per_step": {k: round(v[0] / steps, 4) for k, v in fw["kernels"].items() if v[1]},
           "dominant": kernel_roofs(fw["kernels"], npart, ncell, tsize, w.species.w is not None, g.order)}
    adj = run_adjoint(w, nadj, fw["ts"])
    adj_ms = adj["ms"] / nadj
    row["adjoint"] = {"steps": nadj, "ms_per_step": round(adj_ms, 4), "ratio_adjoint_over_forward": adj_ms / ms,
                      "ratio_with_replay": (adj_ms + ms) / ms,
                      "kernels_ms_per_step": {k: round(v[0] / nadj, 4) for k, v in adj["kernels"].items() if v[1]}}
    del fw
    if window:
        w.species, w.fields = init
        w.nsteps = window
        w.checkpoint_every = w.checkpoint_every or 5
        del init
        torch.cuda.empty_cache()
        row["rollout"] = run_rollout(w, name)
    del w
    torch.cuda.empty_cache()
    return row


def cpu_configs():
    """The oracle on the two small workloads in full: the 32^3 order-1 plasma
    (10 steps) and the 64^3 differentiable plasma's 20 forward steps."""
    import oracle
    from paper_2101_12149_amd import workloads as wl
    rows = {}
    for name, warm, steps in (("uniform32_o1_f64", 0, 10), ("diff64_o3_f64", 0, 20)):
        w = wl.named(name)
        sp, f = w.species.numpy(), w.fields.numpy()
        src = w.source.numpy() if w.source is not None else None
        if warm:
            oracle.step(w.grid, sp, f, src, 0, warm)
        t0 = time.perf_counter()
        oracle.step(w.grid, sp, f, src, warm, steps)
        dt = time.perf_counter() - t0
        rows[name] = {"value": sp.cell.shape[1] * steps / dt, "unit": "particle-steps/s", "steps": steps,
                      "warmup": warm, "seconds": round(dt, 2), "cores": oracle.num_threads()}
        log(f"[cpu] {name}: {steps} steps in {dt:.2f} s")
    return rows


def cpu_baseline():
    """FP64 oracle on a bounded sample of the same workload shape."""
    import oracle
    from paper_2101_12149_amd import workloads as wl
    n = (96, 96, 96)
    ppc, nsteps = 8, 5
    w = wl.uniform_plasma(n, ppc, 0.05, 3, nsteps, "f64", 1002, 4)
    sp, f = w.species.numpy(), w.fields.numpy()
    oracle.step(w.grid, sp, f, None, 0, 1)   # warm (page-in, thread start)
    t0 = time.perf_counter()
    oracle.step(w.grid, sp, f, None, 1, nsteps)
    dt = time.perf_counter() - t0
    npart = sp.cell.shape[1]
    cores = oracle.num_threads()
    # the same oracle on one thread, on a smaller box of the same plasma
    n1, nsteps1 = (32, 32, 32), 3
    w1 = wl.uniform_plasma(n1, ppc, 0.05, 3, nsteps1, "f64", 1002, 4)
    sp1, f1 = w1.species.numpy(), w1.fields.numpy()
    oracle.set_num_threads(1)
    try:
        oracle.step(w1.grid, sp1, f1, None, 0, 1)
        t0 = time.perf_counter()
        oracle.step(w1.grid, sp1, f1, None, 1, nsteps1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    npart1 = sp1.cell.shape[1]
    return {"value": npart * nsteps / dt, "unit": "particle-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"uniform plasma {n[0]}^3, {ppc} ppc ({npart} particles), order 3, FP64, {nsteps} steps "
                      f"after 1 warm-up step ({dt:.1f} s)",
            "value_1thread": npart1 * nsteps1 / dt1,
            "sample_1thread": f"uniform plasma {n1[0]}^3, {ppc} ppc ({npart1} particles), order 3, FP64, "
                              f"{nsteps1} steps after 1 warm-up step, 1 thread ({dt1:.1f} s)"}


MICRO_MODES = ("lds_add_f32", "lds_add_f64", "lds_add_u32", "lds_add_u64", "lds_read_f32", "lds_read_f64",
               "lds_write_f32", "lds_write_f64", "global_add_f32", "global_add_f64")


def atomic_micro():
    """LDS and global atomic / access throughput (libpic355_micro.so), in
    lane-operations per clock per CU at the 2.4 GHz peak clock: 8 workgroups
    of 256 threads per CU, 64 x 32 operations per lane on in-bounds indices
    (stride 1: consecutive words per lane; 2 and 17 spread lanes over the
    banks).  LDS arrays hold 8192 elements; global ones 8192 per workgroup."""
    import ctypes as C
    lib = C.CDLL(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2101_12149_amd",
                              "libpic355_micro.so"))
    lib.picmb_run.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                              C.POINTER(C.c_double)]
    cus, clk = 256, 2.4e9
    res = []
    for mode, name in enumerate(MICRO_MODES):
        for stride in (1, 2, 17):
            ms, ops = C.c_double(), C.c_double()
            rc = lib.picmb_run(mode, cus * 8, 64, stride, 8192, C.byref(ms), C.byref(ops))
            if rc != 0:
                raise RuntimeError(f"picmb_run({name}, stride {stride}) failed with {rc}")
            rate = ops.value / (ms.value * 1e-3)
            res.append({"op": name, "stride": stride, "ms": round(ms.value, 4),
                        "lane_ops_per_clk_per_cu": round(rate / cus / clk, 3)})
            log(f"[micro] {name:15s} stride {stride:2d}: {ms.value:8.3f} ms, "
                f"{rate / cus / clk:7.3f} lane-ops/clk/CU")
    return {"probe": "atomic and LDS throughput", "cus": cus, "clock_GHz": 2.4, "results": res}


def stray_fraction(w, ts):
    """Fraction of the particles whose cell lies outside their tile's LDS
    region (tile + slack) under the binning ts: the particles the stray
    kernel takes."""
    import torch
    from paper_2101_12149_amd import _lib
    g = w.grid
    info = _lib.tile_geometry(g, w.dtype)
    t, nt, slack = info["tile"], info["ntiles_xyz"], info["slack"]
    n = w.species.n
    idx = torch.arange(n, device=ts.device, dtype=torch.int32)
    tile = torch.searchsorted(ts[1:].contiguous(), idx, right=True)
    origin = [(tile % nt[0]) * t[0], ((tile // nt[0]) % nt[1]) * t[1], (tile // (nt[0] * nt[1])) * t[2]]
    outside = torch.zeros(n, dtype=torch.bool, device=ts.device)
    for d in range(3):
        v = w.species.cell[d].long() - origin[d]
        v = torch.where(v < -slack, v + g.n[d], torch.where(v >= t[d] + slack, v - g.n[d], v))
        outside |= (v < -slack) | (v >= t[d] + slack)
    return float(outside.float().mean())


def sort_sweep(args):
    """Sort interval x tile size on one workload: throughput, the sort, tile
    and stray kernel times per step, and the fraction of stray particles in
    the last step of a sort cycle."""
    import torch
    from paper_2101_12149_amd import workloads as wl
    rows = []
    for tile in [tuple(int(x) for x in t.split(",")) for t in args.sweep_tiles.split(";")]:
        for se in [int(x) for x in args.sweep_intervals.split(",")]:
            w = wl.named(args.workload, device="cuda")
            w.grid.tile = tile
            fw = run_forward(w, args.steps, args.warmup, se, f"tile {tile} sort every {se}")
            k = fw["kernels"]
            per = {c: round(k[c][0] / args.steps, 3) for c in ("sort", "particles", "strays", "yee", "reduce")}
            # strays at the end of a sort cycle: sort, then se - 1 steps on that binning
            from paper_2101_12149_amd import _lib
            ts = fw["ts"]
            _lib.pic_sort_tiles(w.grid, w.species, ts, fw["ws"])
            if se > 1:
                _lib.pic_step(w.grid, w.species, w.fields, None, args.warmup + args.steps, se - 1, 0, ts, fw["ws"])
            torch.cuda.synchronize()
            rows.append({"tile": list(tile), "sort_every": se,
                         "particle_steps_per_s": w.species.n * args.steps / (fw["ms"] * 1e-3),
                         "ms_per_step": round(fw["ms"] / args.steps, 3), "kernels_ms_per_step": per,
                         "stray_fraction_cycle_end": round(stray_fraction(w, ts), 6)})
            log(json.dumps(rows[-1]))
            del w, fw
            torch.cuda.empty_cache()
    print(json.dumps({"sweep": "sort interval x tile", "workload": args.workload, "steps": args.steps,
                      "warmup": args.warmup, "rows": rows}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="uniform256_o3_f32")
    ap.add_argument("--sort-every", type=int, default=None)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="leave out the other workloads (32^3, laser, 64^3 differentiable, 512^3)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--slack", type=int, default=-1)
    ap.add_argument("--pusher", choices=("boris", "vay"), default="boris",
                    help="momentum update of the push (the workload's field and particle setup is unchanged)")
    ap.add_argument("--solver", choices=("yee", "ckc"), default="yee",
                    help="field solver (same time step as the workload's Yee setup)")
    ap.add_argument("--gather-filter", action="store_true",
                    help="filter E and B along z before the gather (binomial taps 1/4, 1/2, 1/4 on every component)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 1 GiB device-to-device first (HBM counter calibration)")
    ap.add_argument("--atomic-micro", action="store_true",
                    help="LDS / global atomic throughput probe instead of the step benchmark")
    ap.add_argument("--sort-sweep", action="store_true",
                    help="sweep the sort interval and the tile size instead of the benchmark line")
    ap.add_argument("--sweep-intervals", default="1,2,4,8,16")
    ap.add_argument("--sweep-tiles", default="8,8,8;8,8,4;4,4,4")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is a design, not built)"}))
        sys.exit(2)

    import torch
    from paper_2101_12149_amd import _lib
    from paper_2101_12149_amd import workloads as wl
    _lib.load()
    torch.cuda.set_device(0)

    if args.sort_sweep:
        sort_sweep(args)
        return
    if args.atomic_micro:
        print(json.dumps(atomic_micro()))
        return

    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    w = wl.named(args.workload, device="cuda")
    if args.tile:
        w.grid.tile = (args.tile,) * 3
    w.grid.slack = args.slack
    w.grid.pusher = 1 if args.pusher == "vay" else 0
    w.grid.solver = 1 if args.solver == "ckc" else 0
    if args.gather_filter:
        w.grid.gather_filter = [[0.5, 0.25, 0.0, 0.0]] * 6
    sort_every = w.sort_every if args.sort_every is None else args.sort_every
    g = w.grid
    npart, ncell = w.species.n, g.ncells
    tsize = 4 if w.dtype == "f32" else 8
    fw = run_forward(w, args.steps, args.warmup, sort_every, w.dtype)
    ms_step = fw["ms"] / args.steps
    value = npart * args.steps / (fw["ms"] * 1e-3)

    # dominant kernel: the fused tile kernel (gather + push + deposit); its
    # binding units are the VALU and the LDS pipe (not HBM), so the roofline
    # is the vector-ALU one, with the HBM figures alongside
    pk_ms, pk_n = fw["kernels"]["particles"]
    pk_avg = pk_ms / max(pk_n, 1)
    alg_bytes = particle_bytes(npart, tsize, w.species.w is not None) + field_bytes(ncell, tsize)
    alg_flops = FLOPS_PER_PARTICLE[g.order] * npart
    achieved_tf = alg_flops / (pk_avg * 1e-3) / 1e12
    hbm_gbs = alg_bytes / (pk_avg * 1e-3) / 1e9
    roofline = {"bound": "alu", "achieved": round(achieved_tf, 2), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tf / VALU_PEAK_TFLOPS, 4), "traffic": MEASURED_TRAFFIC.get(w.name),
                "kernel": tile_kernel_name(npart, ncell, tsize, g.order), "avg_ms": round(pk_avg, 4),
                "alg_flops_per_particle": FLOPS_PER_PARTICLE[g.order],
                "hbm_achieved_GBps": round(hbm_gbs, 1), "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
                "alg_bytes_per_launch": int(alg_bytes),
                "alg_bytes_per_particle": round(alg_bytes / npart, 2)}
    breakdown = {k: {"ms_per_step": round(v[0] / args.steps, 4), "launch_groups": v[1]}
                 for k, v in fw["kernels"].items() if v[1]}

    out = {"metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": w.dtype, "data": "synthetic",
           "config": {"workload": w.name, "cells": list(g.n), "particles": npart, "ppc": w.meta.get("ppc"),
                      "order": g.order, "u_th": w.meta.get("u_th"), "sort_every": sort_every,
                      "pusher": args.pusher, "solver": args.solver, "gather_filter": bool(args.gather_filter),
                      "precision": "int32 cell + FP32 offset, FP32 fields/momenta, FP64 reductions"
                      if w.dtype == "f32" else "FP64"},
           "kernels": breakdown, "roofline": roofline}
    fwd_diag_last = fw["diag"][-1].tolist()
    out["diag_last"] = fwd_diag_last

    if not args.no_adjoint:
        nrep = max(3, min(10, args.steps // 4))
        adj = run_adjoint(w, nrep, fw["ts"])
        adj_ms = adj["ms"] / nrep
        out["adjoint"] = {"ms_per_step": adj_ms, "particle_steps_per_s": npart / (adj_ms * 1e-3),
                          "ratio_adjoint_over_forward": adj_ms / ms_step,
                          "ratio_with_replay": (adj_ms + ms_step) / ms_step,
                          "kernels": {k: round(v[0] / nrep, 4) for k, v in adj["kernels"].items() if v[1]}}
    del w, fw
    torch.cuda.empty_cache()

    if not args.no_fp64 and args.workload.endswith("_f32"):
        w64 = wl.named(args.workload[:-4] + "_f64", device="cuda")
        w64.grid.slack = args.slack
        k64 = max(4, args.steps // 2)
        fw64 = run_forward(w64, k64, 2, sort_every, "f64")
        v64 = w64.species.n * k64 / (fw64["ms"] * 1e-3)
        pk64 = fw64["kernels"]["particles"]
        out["fp64"] = {"value": v64, "ms_per_step": fw64["ms"] / k64, "steps": k64,
                       "particles_kernel_ms": pk64[0] / max(pk64[1], 1),
                       "ratio_f32_over_f64": value / v64}
        del w64, fw64
        torch.cuda.empty_cache()

    if not args.no_configs and args.workload == "uniform256_o3_f32":
        out["configs"] = {}
        for name, k, wu, nadj, window in CONFIGS:
            out["configs"][name] = bench_config(name, k, wu, nadj, window)

    if not args.no_cpu_baseline:
        log("[cpu] timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline()
        if not args.no_configs:
            out["cpu_baseline"]["configs"] = cpu_configs()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
