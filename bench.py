#!/usr/bin/env python3
"""Throughput of the pore-MD hot path on one MI355X.

Workload: the single large system -- a 128^3 box with a slit pore (two
simple-cubic wall slabs 4 thick, gap 8), 262144 vapour atoms placed at random
clear of each other and of the walls, T* = 1.2, dt = 0.005, reduced LJ units.
The headline is the mixed-precision path (FP32 pair forces, FP64 sums,
integration and energies); the plain FP64 path is timed beside it on the
same input.  A "step" is one velocity-Verlet step of every atom (neighbour
list rebuilds included); throughput is vapour atom-steps per second with the
state resident in device memory when the timed region starts.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic bytes per vapour atom-step (mixed / FP64): FP64 x and v read and
# written once, plus the FP32 (FP64) neighbour copy written once and read once
ALG_BYTES = {"mixed": 120.0, "fp64": 144.0}
PEAK_HBM_GBS = 8000.0

# HBM bytes per k_step<float> launch from the FETCH_SIZE / WRITE_SIZE counter
# passes summarised in profiles/k_step_slit128_mixed.md (128^3 slit workload,
# skins 0.7 and 1.0), keyed by the hash of the device sources they were taken on, the
# vapour atom count, the skin and the workgroup shape (block, target atoms per
# brick).  The rebuild period is not part of the key: it changes how often
# the lists are rebuilt, not what one step launch reads and writes.  Any
# other source, workload or tuning reports null.
MEASURED_TRAFFIC = {
    ("2f5fb16131aad05e", 262144, 0.7, 256, 270): 87.00e6,
    ("2f5fb16131aad05e", 262144, 0.7, 512, 460): 83.62e6,
    ("2f5fb16131aad05e", 262144, 1.0, 256, 270): 89.08e6,
    ("2f5fb16131aad05e", 262144, 1.0, 256, 256): 91.06e6,
}


def kernel_source_hash():
    """sha256 prefix of the device code's sources (kernels and the layout
    header they include)."""
    import hashlib

    h = hashlib.sha256()
    for name in ("pmd_kernels.hip", "pmd_internal.h"):
        with open(os.path.join(ROOT, "paper_1812_07993_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def energy_drift(tot, burn):
    seg = np.asarray(tot[burn:], dtype=np.float64)
    if seg.shape[0] < 3:
        return None, None
    t = np.arange(seg.shape[0], dtype=np.float64)
    slope = np.polyfit(t, seg, 1)[0]
    return float(abs(slope) * (seg.shape[0] - 1) / abs(seg[0])), float(
        np.abs(seg - seg[0]).max() / abs(seg[0]))


def force_errors(F, F_ref):
    """Relative force error ||F - F_ref|| / ||F_ref|| and the per-atom error
    max_i |F_i - F_ref,i| / rms_i |F_ref,i| at identical positions."""
    d = np.asarray(F) - np.asarray(F_ref)
    rms = float(np.sqrt(np.mean(np.sum(F_ref * F_ref, axis=1))))
    return (float(np.linalg.norm(d) / np.linalg.norm(F_ref)),
            float(np.sqrt(np.sum(d * d, axis=1)).max() / rms))


DRIFT_BURN, DRIFT_WINDOW = 100, 1000


def accuracy_run(poremd, desc, prec, tuning_kw):
    """Untimed: a fresh system from the workload's initial state; its forces
    at creation (for the force error against the oracle's sample) and the
    energy drift over DRIFT_WINDOW steps after a DRIFT_BURN-step burn-in,
    energies recorded every step: the least-squares trend over the window and
    the largest deviation from its first value, both relative to |E|."""
    tun = poremd.make_tuning(**dict(tuning_kw, energy_every=1))
    t0 = time.perf_counter()
    s = poremd.System.from_desc(desc, precision=prec, tuning=tun)
    F0 = s.forces()
    s.step(DRIFT_BURN + DRIFT_WINDOW)
    E = s.energy_history()
    s.close()
    burn = int(np.searchsorted(E["step"], DRIFT_BURN))
    trend, maxdev = energy_drift(E["etotal"][: burn + DRIFT_WINDOW + 1], burn)
    log("[accuracy %s %s] drift trend %.3e, max deviation %.3e over steps %d..%d (%.1f s)"
        % (desc.name, prec, trend, maxdev, DRIFT_BURN, DRIFT_BURN + DRIFT_WINDOW,
           time.perf_counter() - t0))
    return dict(F0=F0, drift_trend=trend, drift_max=maxdev)


def autotune(poremd, desc, prec, trial_steps, tuning_kw):
    """Skin and rebuild period from the library's autotuner (untimed): every
    candidate of its built-in grid runs trial_steps steps of this workload."""
    params, pore = poremd.params_of(desc, prec)
    grid = poremd.pmd_autotune_grid(params, desc.n)
    for t in grid:
        if tuning_kw.get("block"):
            t.block = tuning_kw["block"]
        if tuning_kw.get("brick_atoms"):
            t.brick_atoms = tuning_kw["brick_atoms"]
        if tuning_kw.get("brick_order"):
            t.brick_order = tuning_kw["brick_order"]
    t0 = time.perf_counter()
    best, us = poremd.pmd_autotune(params, pore, desc.x, desc.v, grid, trial_steps)
    b = grid[best]
    log("[%s] autotune: %d candidates in %.1f s; best skin %.2f, rebuild every %d: %.2f us/step"
        % (prec, len(grid), time.perf_counter() - t0, b.skin, b.rebin_every, us[best]))
    order = np.argsort(us)[:5]
    log("[%s] autotune top 5: %s" % (prec, ", ".join(
        "(%.2f, %d) %.2f" % (grid[i].skin, grid[i].rebin_every, us[i]) for i in order)))
    out = dict(skin=float(b.skin), rebin_every=int(b.rebin_every))
    if tuning_kw.get("block") or tuning_kw.get("brick_atoms"):
        return out
    # second stage: workgroup size and atoms per brick, jointly with the three
    # fastest (skin, period) pairs of the first stage (which ran at the
    # default shape, so its ranking can change with the shape)
    shapes = [(256, 0), (256, 256), (256, 270), (256, 160), (512, 460), (128, 0)]
    pairs = []
    for i in order:
        sr = (float(grid[i].skin), int(grid[i].rebin_every))
        if sr not in pairs:
            pairs.append(sr)
        if len(pairs) == 3:
            break
    combos = [(sk, rb, bl, ba) for sk, rb in pairs for bl, ba in shapes]
    cands = [poremd.make_tuning(skin=sk, rebin_every=rb, block=bl, brick_atoms=ba)
             for sk, rb, bl, ba in combos]
    best2, us2 = poremd.pmd_autotune(params, pore, desc.x, desc.v, cands, trial_steps)
    log("[%s] autotune shapes: %s" % (prec, ", ".join(
        "(%.2f, %d, %d, %d) %.2f" % (c + (u,)) for c, u in zip(combos, us2))))
    # third stage: the three fastest combinations again, five times longer
    # each (short trials of close shapes can swap places)
    fin = [int(i) for i in np.argsort(us2)[:3]]
    best3, us3 = poremd.pmd_autotune(params, pore, desc.x, desc.v, [cands[i] for i in fin],
                                     5 * trial_steps)
    log("[%s] autotune finalists: %s" % (prec, ", ".join(
        "(%.2f, %d, %d, %d) %.2f" % (combos[i] + (u,)) for i, u in zip(fin, us3))))
    sk, rb, bl, ba = combos[fin[best3]]
    log("[%s] autotune choice: skin %.2f, rebuild every %d, block %d, atoms per brick %d: %.2f us/step"
        % (prec, sk, rb, bl, ba, us3[best3]))
    # candidates for tuning on the measured call length (see call_tune): the
    # finalists, and the three fastest skins at the chosen shape with their
    # period and with a period of 20 steps
    fins = []
    for c in [combos[i] for i in fin] + [(p[0], r, bl, ba) for p in pairs for r in (p[1], 20)]:
        d = dict(skin=c[0], rebin_every=c[1], block=c[2], brick_atoms=c[3])
        if d not in fins:
            fins.append(d)
    return dict(skin=sk, rebin_every=rb, block=bl, brick_atoms=ba, finalists=fins)


# Timed calls shorter than this are tuned on the call itself (call_tune).
CALL_TUNE_STEPS = 1000


def call_tune(poremd, desc, prec, cands, steps, warmup, energy_every, reps=5):
    """Among candidate tunings, the fastest for the measured call: every
    pmd_step call begins with a rebuild and may stop early for a displacement
    halt, so for a call of a few dozen steps the per-call costs outweigh the
    steady-state rate the autotuner ranks by.  Each candidate system runs the
    warm-up call and then `reps` timed calls of `steps` steps, synchronised
    like the timed region; the median decides.  Untimed for the benchmark."""
    import torch

    times = []
    for kw in cands:
        stream = torch.cuda.Stream()
        s = poremd.System.from_desc(desc, precision=prec,
                                    tuning=poremd.make_tuning(energy_every=energy_every, **kw),
                                    stream=stream.cuda_stream)
        if warmup:
            s.step(warmup)
            s.sync()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.step(steps)
            s.sync()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        s.close()
        times.append(float(np.median(ts)) * 1000.0 / steps)
    best = int(np.argmin(times))
    log("[%s] call tuning (%d-step calls): %s" % (prec, steps, ", ".join(
        "(%.2f, %d, %d, %d) %.2f" % (c["skin"], c["rebin_every"], c["block"], c["brick_atoms"], t)
        for c, t in zip(cands, times))))
    return dict(cands[best]), [dict(c, us_per_step=t) for c, t in zip(cands, times)]


def run_path(poremd, desc, prec, steps, warmup, energy_every, tuning_kw):
    import torch

    stream = torch.cuda.Stream()
    tun = poremd.make_tuning(energy_every=energy_every, **tuning_kw)
    t0 = time.perf_counter()
    s = poremd.System.from_desc(desc, precision=prec, tuning=tun, stream=stream.cuda_stream)
    log("[%s] created in %.2f s (walls %d)" % (prec, time.perf_counter() - t0, s.n_wall))
    if warmup:
        s.step(warmup)
        s.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    s.sync()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    hist = s.energy_history()
    rebuilds, maxlen = poremd.pmd_debug_lists(s.h)
    out = dict(ms=ms, wall_s=wall, hist=hist, rebuilds=rebuilds, max_list=maxlen, sys=s)
    log("[%s] %d steps: %.3f ms (%.2f us/step), wall %.3f s, rebuilds %d"
        % (prec, steps, ms, 1000 * ms / steps, wall, rebuilds))
    return out


def thermostat_leg(poremd, desc, steps, tuning_kw, tau=0.5, t0=1.2):
    """The 128^3 slit workload in mixed precision with the Berendsen
    thermostat on (rise time tau = 100 dt, target t0 = T* = 1.2), at the NVE
    path's tuning: the cost of the F4 step (two extra launches per step)."""
    import torch

    params, pore = poremd.params_of(desc, "mixed")
    params.thermostat_tau, params.thermostat_t0 = tau, t0
    stream = torch.cuda.Stream()
    tun = poremd.make_tuning(energy_every=10, **tuning_kw)
    s = poremd.System(params, pore, desc.x, desc.v, None, stream.cuda_stream, tun)
    s.step(max(steps // 10, 10))
    s.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps)
    s.sync()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    T_end = float(s.energies()["temperature"])
    s.close()
    out = {"value": desc.n * steps / (ms / 1000.0), "unit": "atom-steps/s",
           "ms_per_step": ms / steps, "steps": steps, "tau": tau, "t0": t0,
           "temperature_end": T_end}
    log("[thermostat] %d steps: %.2f us/step, T = %.4f" % (steps, 1000 * ms / steps, T_end))
    return out


def allpairs_leg(poremd, n_pores, calls=50):
    """The force function as the paper states it (every pair, no cutoff, no
    shift), at the paper's sizes: N_pore molecules in the pore plus an outer
    space 21 times the pore volume at a fifth of the pore density, N = 5.2
    N_pore atoms in all; placed uniformly (random sequential addition at
    density 0.05, minimum image in a periodic cube), which costs the same as
    the pore geometry for an all-pairs sum.  Times `calls` back-to-back force
    evaluations per precision with HIP events on the stream they run on."""
    import torch

    from paper_1812_07993_amd import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for npore in n_pores:
        n = int(round(5.2 * npore))
        L = (n / 0.05) ** (1.0 / 3.0)
        x = synth.rsa_place(np.random.default_rng(npore), (L, L, L), n, np.zeros((0, 3)), 0.9)
        xd = torch.as_tensor(x, dtype=torch.float64, device=dev)
        f = torch.empty((n, 3), dtype=torch.float64, device=dev)
        u = torch.empty((n,), dtype=torch.float64, device=dev)
        e = torch.empty((1,), dtype=torch.float64, device=dev)
        row = {"n_pore": npore, "n": n}
        for prec in ("mixed", "fp64"):
            def call():
                poremd.pmd_allpairs_forces(prec, n, xd.data_ptr(), (L, L, L), 1.0, 1.0, f.data_ptr(),
                                           u.data_ptr(), e.data_ptr(), stream.cuda_stream)
            for _ in range(3):
                call()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(calls):
                call()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / calls
            row[prec + "_ms"] = ms
            row[prec + "_pairs_per_s"] = n * (n - 1) / (ms / 1000.0)
        log("[allpairs] N_pore %d (N = %d): mixed %.3f ms (%.3g pairs/s), fp64 %.3f ms (%.3g pairs/s)"
            % (npore, n, row["mixed_ms"], row["mixed_pairs_per_s"], row["fp64_ms"],
               row["fp64_pairs_per_s"]))
        rows.append(row)
    return rows


# The paper's own per-step times (ms) of its full GPU step at N_pore = 100,
# 200, ..., 1500 molecules in the pore, 128-thread blocks, on its cluster's
# GPU (Tables 2 and 3, "total GPU time"): context, not a target.
PAPER_GPU_MS = {
    2: [1.577, 2.957, 4.371, 5.541, 7.040, 8.317, 9.660, 10.563, 12.675, 13.706, 15.175, 17.212,
        18.956, 19.767, 21.522],
    3: [1.042, 1.776, 2.504, 3.374, 4.115, 4.829, 5.571, 6.162, 7.276, 8.175, 9.035, 9.924, 10.501,
        11.587, 12.434],
}


def paper_model_leg(poremd, dims=(2, 3), n_pores=tuple(range(100, 1501, 100)), steps=2000,
                    precision="fp64"):
    """The paper's own workload (Secs. 4-5): its 2D pore (1 um, k = 3, 35 C)
    and 3D prism (500 x 50 x 50 nm, k = 1, 25 C) with N_pore molecules in the
    pore and a fifth of the pore density outside, all-pairs forces, reflecting
    pore walls, periodic outer space, the Berendsen thermostat on (rise time
    1 ps), dt = 0.016 ps: the full step (F2, F1, F3, F4) timed over `steps`
    steps with HIP events on the stream, as in Tables 2 and 3."""
    import torch

    from paper_1812_07993_amd import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    for dim in dims:
        rows = []
        for i, npore in enumerate(n_pores):
            x, v, geo = synth.paper_model_system(dim, npore)
            n = x.shape[0]
            m = poremd.make_pm_model(dim, geo["lx"], geo["ly"], geo["lz"], geo["k"], precision,
                                     dt=geo["dt"], thermostat_tau=1.0 / synth.PAPER_TAU_PS,
                                     thermostat_t0=geo["temperature"])
            xd = torch.as_tensor(x, dtype=torch.float64, device=dev)
            vd = torch.as_tensor(v, dtype=torch.float64, device=dev)
            rec = torch.zeros((2, poremd.PM_RECORD_DTYPE.itemsize // 8), dtype=torch.float64,
                              device=dev)
            poremd.pmd_pm_run(m, n, xd.data_ptr(), vd.data_ptr(), 0, 20, 0, rec.data_ptr(), 2,
                              stream.cuda_stream)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            poremd.pmd_pm_run(m, n, xd.data_ptr(), vd.data_ptr(), 0, steps, 0, rec.data_ptr(), 2,
                              stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            r = rec.cpu().numpy().view(poremd.PM_RECORD_DTYPE).reshape(2)
            row = {"n_pore": npore, "n": n, "ms_per_step": ms, "us_per_particle_step": 1000 * ms / n,
                   "pairs_per_s": n * (n - 1) / (ms / 1000.0), "n_outside": int(r["n_outside"][-1]),
                   "paper_gpu_ms": PAPER_GPU_MS[dim][i] if len(n_pores) == 15 else None}
            rows.append(row)
        log("[paper %dD] ms per step at N_pore %s: %s" % (dim, ",".join(str(r["n_pore"]) for r in rows),
                                                       ", ".join("%.4f" % r["ms_per_step"] for r in rows)))
        out["%dd" % dim] = rows
    return out


def kernel_time(poremd, s, steps):
    """Mean duration of one step-kernel launch, from HIP events around the R
    back-to-back launches of each replay that did R full steps."""
    poremd.pmd_timing_enable(s.h, True)
    s.step(steps)
    s.sync()
    n, mean_ms = poremd.pmd_kernel_time(s.h)
    poremd.pmd_timing_enable(s.h, False)
    return n, mean_ms


def cpu_baseline(desc, sample_atoms, extra=(), extra_atoms=512, seed=0):
    """The oracle timed on the host: its F1 sums (every partner, FP64, OpenMP
    over the host cores) for `sample_atoms` randomly chosen vapour atoms of
    the headline system, scaled to atom-steps per second (F1 is 99.9% of an
    oracle step).  The same leg computes the oracle's forces for
    `extra_atoms` atoms of each system in `extra` ((name, desc) pairs: the
    4M-atom pores); the sampled forces serve as references for the force
    error of the GPU paths at the same positions."""
    import oracle

    def walls_of(d):
        q = d.pore
        return oracle.wall_lattice(oracle.make_pore(q.kind, q.lattice_a, q.slab_center_z,
                                                    q.slab_thickness, q.r0, q.r1, q.slit_gap),
                                   d.params.box)

    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(desc.n, sample_atoms, replace=False))
    p = oracle.make_params(desc.params.box)
    walls = walls_of(desc)
    t0 = time.perf_counter()
    Fref, _ = oracle.forces_subset(desc.x, walls, p, sel)
    dt = time.perf_counter() - t0
    base = dict(value=sample_atoms / dt, unit="atom-steps/s", cores=oracle.num_threads(),
                kind="oracle",
                sample="F1 force sums (all %d partners each, 99.9%% of an oracle step) for %d "
                       "randomly chosen vapour atoms of the same system, %.1f s"
                       % (desc.n + walls.shape[0], sample_atoms, dt))
    refs = {"headline": (sel, Fref)}
    for name, d in extra:
        r = np.random.default_rng(seed + 1)
        zc, half = d.pore.slab_center_z, 0.5 * d.pore.slab_thickness
        near = np.flatnonzero(np.abs(d.x[:, 2] - zc) < half + 3.0)
        k = extra_atoms // 2
        es = np.unique(np.concatenate([r.choice(d.n, k, replace=False),
                                       r.choice(near, k, replace=False)]))
        t1 = time.perf_counter()
        Fe, _ = oracle.forces_subset(d.x, walls_of(d), oracle.make_params(d.params.box), es)
        log("oracle sample of %s: %d atoms in %.1f s" % (name, len(es), time.perf_counter() - t1))
        refs[name] = (es, Fe)
    return base, refs


def _request_payload(spec):
    from paper_1812_07993_amd import synth

    return synth.request_system(spec)


def serve_leg(n_requests, budget_gb, chunk, workers=2):
    """Served trace: Poisson arrivals at 200 requests/s, vapour N log-uniform in
    [2k, 500k], pore from {cylinder, slit, cone, ink-bottle}, 1k-20k steps,
    mixed or FP64 with probability 1/2; one batch per precision, each bounded
    by the device budget.  The requests' initial states (the clients' data)
    are generated before the trace starts, by host worker threads (the
    placement runs in C through ctypes, which releases the GIL); creating
    each system on the device (upload, first forces) is part of its latency
    and runs on `workers` threads beside the tick loop."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_1812_07993_amd import serve, synth

    t0 = time.perf_counter()
    specs = synth.request_trace(n_requests)
    nproc = max(1, min(16, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=nproc) as ex:
        payloads = list(ex.map(_request_payload, specs))
    reqs = [serve.Request(s["index"], s["arrival"], s["precision"], s["steps"], s["n"], p)
            for s, p in zip(specs, payloads)]
    log("serve: %d requests generated in %.1f s on %d threads (%.2e atom-steps offered)"
        % (len(reqs), time.perf_counter() - t0, nproc, sum(r.n * r.steps for r in reqs)))
    be = serve.PoremdBackend(hbm_budget=int(budget_gb * 2 ** 30), max_slots=256)
    res = serve.Server(be, chunk_steps=chunk, create_workers=workers).run(reqs)
    s = serve.summarize(res)
    span_arrivals = max(r.arrival for r in reqs) - min(r.arrival for r in reqs)
    s["offered_req_per_s"] = (len(reqs) - 1) / span_arrivals if span_arrivals > 0 else None
    s["offered_atom_steps"] = float(sum(r.n * r.steps for r in reqs))
    s["budget_gb_per_precision"] = budget_gb
    s["chunk_steps"] = chunk
    s["create_workers"] = workers
    by = {}
    for p in ("mixed", "fp64"):
        rs = [r for r in res if r.precision == p]
        if rs:
            lat = np.array([r.latency for r in rs])
            by[p] = {"requests": len(rs), "p50_s": float(np.percentile(lat, 50)),
                     "p99_s": float(np.percentile(lat, 99))}
    s["by_precision"] = by
    log("serve: p50 %.3f s, p99 %.3f s, %.3e atom-steps/s over %.2f s"
        % (s["p50_s"], s["p99_s"], s["atom_steps_per_s"], s["makespan_s"]))
    return s


def batch_autotune(poremd, descs, trial_steps, stream):
    """Tuning of the replica batch on the batch itself: the library's
    autotuner ranks (skin, rebuild period) on the median replica, then the
    three best pairs times three workgroup shapes are each timed on all the
    replicas resident in one batch (trial_steps steps, wall clock), and the
    fastest is kept.  The systems are created once per workgroup shape at the
    smallest skin (the largest cell grid) and retuned per (skin, period)."""
    import torch

    med = sorted(descs, key=lambda d: d.n)[len(descs) // 2]
    params, pore = poremd.params_of(med, "mixed")
    grid = poremd.pmd_autotune_grid(params, med.n)
    best, us = poremd.pmd_autotune(params, pore, med.x, med.v, grid, trial_steps)
    pairs = []
    for i in np.argsort(us):
        sr = (float(grid[i].skin), int(grid[i].rebin_every))
        if np.isfinite(us[i]) and sr not in pairs:
            pairs.append(sr)
        if len(pairs) == 3:
            break
    smin = min(sk for sk, _ in pairs)
    cands, times = [], []
    for bl, ba in ((256, 0), (256, 270), (512, 460)):
        # the replicas are created once per workgroup shape (a shape sizes the
        # cell tables), at the smallest skin, and retuned per (skin, period)
        hs = [poremd.System.from_desc(d, tuning=poremd.make_tuning(skin=smin, block=bl, brick_atoms=ba),
                                      stream=stream.cuda_stream) for d in descs]
        # ascending skin: a system released from a batch keeps cell tables
        # sized for its last grid, which fit every coarser one
        for sk, rb in sorted(pairs):
            c = dict(skin=sk, rebin_every=rb, block=bl, brick_atoms=ba)
            for h in hs:
                h.set_tuning(poremd.make_tuning(**c))
            b = poremd.pmd_batch_create(0, len(hs), stream.cuda_stream)
            slots = [poremd.pmd_batch_admit(b, h.h, trial_steps) for h in hs]
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            poremd.pmd_batch_advance(b, trial_steps)
            while len(poremd.pmd_batch_poll(b)) < len(hs):
                poremd.pmd_batch_advance(b, max(trial_steps // 10, 1))
            torch.cuda.synchronize()
            cands.append(c)
            times.append((time.perf_counter() - w0) / trial_steps * 1e6)
            for sl in slots:
                poremd.pmd_batch_release(b, sl)
            poremd.pmd_batch_destroy(b)
        for h in hs:
            h.close()
    k = int(np.argmin(times))
    log("batch autotune: %s" % ", ".join("(%.2f, %d, %d, %d) %.1f us/step" % (
        c["skin"], c["rebin_every"], c["block"], c["brick_atoms"], t) for c, t in zip(cands, times)))
    return cands[k], [dict(c, us_per_step=t) for c, t in zip(cands, times)]


def batch_leg(poremd, count, steps, autotune_steps):
    """Replica batch: `count` independent systems (vapour N log-uniform in
    [1k, 64k], pore from {cylinder, slit, cone}, box at density 0.1),
    mixed precision, tuned on the batch itself, resident in one batch and
    advanced together for `steps` steps each; against the same systems
    stepped one at a time (one after another on one stream, the same steps,
    one wait at the end).  Energies are recorded every 10 steps, and every
    system's drift (trend over steps 100..1100 and largest deviation) is
    reported."""
    import torch

    from paper_1812_07993_amd import synth

    t0 = time.perf_counter()
    descs = [synth.replica(sp, "mixed", steps) for sp in synth.replica_specs(count)]
    natoms = sum(d.n for d in descs)
    stream = torch.cuda.Stream()
    log("batch: %d systems, %d vapour atoms, generated in %.1f s" % (count, natoms, time.perf_counter() - t0))
    tkw, cand_times = batch_autotune(poremd, descs, autotune_steps, stream)
    tun = poremd.make_tuning(energy_every=10, **tkw)
    # all in one batch: every system runs exactly `steps` steps; the timed
    # region spans the first advance to the last system finishing (one graph
    # capture and the replays re-queued after early rebuilds included)
    handles = [poremd.System.from_desc(d, tuning=tun, stream=stream.cuda_stream) for d in descs]
    b = poremd.pmd_batch_create(0, count, stream.cuda_stream)
    slots = [poremd.pmd_batch_admit(b, h.h, steps) for h in handles]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    poremd.pmd_batch_advance(b, steps)
    while len(poremd.pmd_batch_poll(b)) < count:
        poremd.pmd_batch_advance(b, max(steps // 10, 1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    batched = natoms * steps / wall
    for sl in slots:
        poremd.pmd_batch_release(b, sl)
    poremd.pmd_batch_destroy(b)
    trends, maxes, bad = [], [], 0
    for h in handles:
        E = h.energy_history()
        burn = int(np.searchsorted(E["step"], DRIFT_BURN))
        end = int(np.searchsorted(E["step"], DRIFT_BURN + DRIFT_WINDOW, side="right"))
        tr, mx = energy_drift(E["etotal"][:end], burn)
        bad += not np.all(np.isfinite(E["etotal"]))
        trends.append(tr)
        maxes.append(mx)
        h.close()
    # one at a time: the same systems from the same start, each stepped alone
    # in turn on one stream, the host waiting once at the end
    alone_h = [poremd.System.from_desc(d, tuning=tun, stream=stream.cuda_stream) for d in descs]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for h in alone_h:
        h.step(steps)
    for h in alone_h:
        h.sync()
    torch.cuda.synchronize()
    alone = natoms * steps / (time.perf_counter() - w0)
    for h in alone_h:
        h.close()
    trends = np.array(trends)
    maxes = np.array(maxes)
    log("batch: %.3e atom-steps/s batched (%d steps, %.3f s), %.3e one at a time; drift trend "
        "median %.2e max %.2e" % (batched, steps, wall, alone, np.median(trends), trends.max()))
    return {"systems": count, "vapour_atoms": natoms, "steps": steps, "value": batched,
            "unit": "atom-steps/s", "tuning": tkw, "autotune": cand_times,
            "one_at_a_time": alone, "one_at_a_time_steps": steps, "speedup": batched / alone,
            "nonfinite_systems": bad,
            "drift_trend_median": float(np.median(trends)), "drift_trend_max": float(trends.max()),
            "drift_max_median": float(np.median(maxes)), "drift_max_max": float(maxes.max()),
            "drift_window": "steps %d..%d of the batched run, energies every 10 steps"
                            % (DRIFT_BURN, DRIFT_BURN + DRIFT_WINDOW)}


def pore_sweep_leg(poremd, kinds, steps, autotune_steps, tuning_kw, precisions=("mixed", "fp64"),
                   accuracy=True):
    """The dense workload: 256 x 256 x 128 box, one 8-thick wall slab with a
    pore (cylinder r = 6, cone 4 -> 12, ink-bottle 3 / 10), 4194304 vapour
    atoms (density 0.5); the mixed path and the plain FP64 path, each with
    its own tuning, timed over `steps` steps, plus the untimed accuracy run
    of each.  Returns the figures and the inputs (for the oracle's sample)."""
    import torch

    from paper_1812_07993_amd import synth

    out, keep = {}, {}
    for kind in kinds:
        t0 = time.perf_counter()
        desc = synth.pore_sweep(kind)
        log("[sweep %s] %d vapour atoms generated in %.1f s" % (kind, desc.n, time.perf_counter() - t0))
        row = {"n_vapour": desc.n, "steps": steps}
        keep[kind] = {"desc": desc}
        for prec in precisions:
            kw = dict(tuning_kw)
            if autotune_steps > 0:
                t = autotune(poremd, desc, prec, autotune_steps, tuning_kw)
                t.pop("finalists", None)  # the sweep times 500-step calls: steady state
                kw.update(t)
            r = run_path(poremd, desc, prec, steps, max(steps // 10, 10), 10, kw)
            n_launch, kms = kernel_time(poremd, r["sys"], min(steps, 100))
            n = desc.n
            fig = {"value": n * steps / (r["ms"] / 1000.0), "unit": "atom-steps/s",
                   "ms_per_step": r["ms"] / steps, "kernel_ms": kms,
                   "roofline_frac": ALG_BYTES[prec] * n / (kms / 1000.0) / 1e9 / PEAK_HBM_GBS,
                   "rebuilds": r["rebuilds"], "max_list": r["max_list"], "tuning": kw}
            row["n_wall"] = r["sys"].n_wall
            r["sys"].close()
            torch.cuda.synchronize()
            if accuracy:
                acc = accuracy_run(poremd, desc, prec, kw)
                fig["drift_trend"], fig["drift_max"] = acc["drift_trend"], acc["drift_max"]
                keep[kind][prec] = acc["F0"]
            log("[sweep %s %s] %.3e atom-steps/s, step kernel %.3f ms"
                % (kind, prec, fig["value"], kms))
            if prec == "mixed":
                row.update(fig)  # the mixed figures at the top level of the row
            else:
                row[prec] = fig
        if "value" in row and "fp64" in row:
            row["mixed_over_fp64"] = row["value"] / row["fp64"]["value"]
        out[kind] = row
    return out, keep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--box", type=float, default=128.0)
    ap.add_argument("--energy-every", type=int, default=10)
    ap.add_argument("--skin", type=float, default=0.0)
    ap.add_argument("--rebin-every", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--brick-atoms", type=int, default=0)
    ap.add_argument("--brick-order", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the served trace (0 = skip the serving leg)")
    ap.add_argument("--serve-budget-gb", type=float, default=2.0)
    ap.add_argument("--batch-systems", type=int, default=256,
                    help="replica systems of the batched leg (0 = skip it)")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--sweep", default="cylinder,cone,inkbottle",
                    help="pores of the 4M-atom leg, comma separated (cylinder,cone,inkbottle); "
                         "'none' skips it")
    ap.add_argument("--sweep-steps", type=int, default=500)
    ap.add_argument("--sweep-only", action="store_true",
                    help="run only the 4M-atom pore leg (for profiling it)")
    ap.add_argument("--thermostat-steps", type=int, default=2000,
                    help="steps of the 128^3 workload with the Berendsen thermostat on (0: skip)")
    ap.add_argument("--serve-chunk", type=int, default=250)
    ap.add_argument("--allpairs", default="100,500,1500",
                    help="pore molecule counts of the all-pairs force leg, or 'none'")
    ap.add_argument("--timing-steps", type=int, default=500)
    ap.add_argument("--paper-model", default="fp64",
                    help="precision of the paper-model table (fp64 or mixed), or 'none'")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before the timed run, two elementwise kernels of known traffic (this "
                         "many MiB read and written; this many read and half written) to scale "
                         "the hardware byte counters by")
    ap.add_argument("--autotune-steps", type=int, default=200,
                    help="timed steps per autotuner candidate (0 = library defaults); "
                         "skipped when --skin or --rebin-every is given")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent replicas shard trivially across GPUs, one process each).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1812_07993_amd import poremd, synth

    poremd.load()
    assert torch.cuda.is_available(), "needs a GPU"
    if args.sweep_only:
        tkw = dict(skin=args.skin, rebin_every=args.rebin_every, block=args.block,
                   brick_atoms=args.brick_atoms, brick_order=args.brick_order)
        sweep, _ = pore_sweep_leg(poremd, args.sweep.split(","), args.sweep_steps,
                                  0 if (args.skin or args.rebin_every)
                                  else min(args.autotune_steps, 50), tkw,
                                  precisions=("mixed",) if args.no_fp64 else ("mixed", "fp64"),
                                  accuracy=False)
        print(json.dumps({"pore_sweep": sweep}), flush=True)
        return
    if args.copy_mib > 0:
        # an elementwise kernel (not a DMA copy) that reads and writes exactly
        # copy_mib MiB each
        src = torch.ones(args.copy_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        # a second calibration kernel of another shape: two operands of
        # copy_mib / 2 MiB read, copy_mib / 2 MiB written
        half = src.shape[0] // 2
        torch.add(src[:half], src[half:], out=dst[:half])
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read + %d MiB written by one elementwise kernel, "
            "then %d MiB read + %d MiB written by a two-operand one"
            % (args.copy_mib, args.copy_mib, args.copy_mib, args.copy_mib // 2))
        del src, dst
    t0 = time.perf_counter()
    desc = synth.slit_large(n=args.n, box=args.box)
    log("inputs: %d vapour atoms, box %g, generated in %.1f s"
        % (desc.n, args.box, time.perf_counter() - t0))
    tkw = dict(skin=args.skin, rebin_every=args.rebin_every, block=args.block,
               brick_atoms=args.brick_atoms, brick_order=args.brick_order)

    res = {}
    tuned = {}
    call_tables = {}
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        kw = dict(tkw)
        if args.autotune_steps > 0 and not (args.skin or args.rebin_every):
            t = autotune(poremd, desc, prec, args.autotune_steps, tkw)
            fins = t.pop("finalists", None)
            kw.update(t)
            if fins and args.steps < CALL_TUNE_STEPS:
                best, table = call_tune(poremd, desc, prec, [dict(t)] + [f for f in fins if f != t],
                                        args.steps, args.warmup, args.energy_every)
                kw.update(best)
                call_tables[prec] = table
        tuned[prec] = kw
        r = run_path(poremd, desc, prec, args.steps, args.warmup, args.energy_every, kw)
        n_launch, kms = kernel_time(poremd, r["sys"], args.timing_steps)
        r["kernel_ms"] = kms
        r["kernel_launches"] = n_launch
        log("[%s] step kernel mean %.4f ms over %d launches" % (prec, kms, n_launch))
        # accuracy: untimed, from the initial state, independent of --steps
        acc = accuracy_run(poremd, desc, prec, kw)
        r["drift_trend"], r["drift_max"], r["F0"] = acc["drift_trend"], acc["drift_max"], acc["F0"]
        res[prec] = r

    # force error of the mixed path against the FP64 path at identical positions
    eps_f = None
    if "fp64" in res:
        X = res["mixed"]["sys"].positions()
        V = res["mixed"]["sys"].velocities()
        params_m, pore = poremd.params_of(desc, "mixed")
        params_d, _ = poremd.params_of(desc, "fp64")
        a = poremd.System(params_m, pore, X, V)
        b = poremd.System(params_d, pore, X, V)
        Fm, Fd = a.forces(), b.forces()
        eps_f = float(np.linalg.norm(Fm - Fd) / np.linalg.norm(Fd))
        a.close()
        b.close()
        log("force error mixed vs fp64 at identical positions: %.3e" % eps_f)

    m = res["mixed"]
    n = desc.n
    value = n * args.steps / (m["ms"] / 1000.0)
    alg = ALG_BYTES["mixed"] * n
    achieved = alg / (m["kernel_ms"] / 1000.0) / 1e9
    out = {
        "metric": "atom-steps/s mixed vs plain FP64 at <=1e-4 energy drift; served p50/p99 latency",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-pair/f64-accumulate",
        "data": "synthetic",
        "config": {"workload": "slit pore, 128^3 box, %d vapour + %d wall atoms, T*=1.2, "
                               "dt=0.005, mixed precision" % (n, m["sys"].n_wall),
                   "n_vapour": n, "n_wall": m["sys"].n_wall, "box": args.box,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": MEASURED_TRAFFIC.get((kernel_source_hash(), n,
                                                      round(tuned["mixed"].get("skin", 0.0), 3),
                                                      tuned["mixed"].get("block") or 256,
                                                      tuned["mixed"].get("brick_atoms") or 0)),
                     "traffic_unit": "bytes per launch",
                     "kernel": "k_step<float>", "kernel_ms": m["kernel_ms"],
                     "alg_bytes_per_atom_step": ALG_BYTES["mixed"]},
        "accuracy": {"mixed_drift_trend": m["drift_trend"], "mixed_drift_max": m["drift_max"],
                     "drift_window": "steps %d..%d of an untimed run from the initial state, "
                                     "energies every step" % (DRIFT_BURN, DRIFT_BURN + DRIFT_WINDOW),
                     "force_err_mixed_vs_fp64": eps_f,
                     "force_err_mixed_vs_oracle": None, "force_err_fp64_vs_oracle": None},
        "detail": {"mixed_rebuilds": m["rebuilds"], "mixed_max_list": m["max_list"],
                   "tuning": tuned, "call_tuning": call_tables or None},
    }
    if "fp64" in res:
        d = res["fp64"]
        out["fp64"] = {"value": n * args.steps / (d["ms"] / 1000.0),
                       "ms_per_step": d["ms"] / args.steps, "kernel_ms": d["kernel_ms"],
                       "drift_trend": d["drift_trend"], "drift_max": d["drift_max"],
                       "roofline_frac": ALG_BYTES["fp64"] * n / (d["kernel_ms"] / 1000.0) / 1e9
                       / PEAK_HBM_GBS}
        out["mixed_over_fp64"] = out["value"] / out["fp64"]["value"]
    for r in res.values():
        r["sys"].close()
        r["sys"] = None
    if args.thermostat_steps > 0:
        out["thermostat"] = thermostat_leg(poremd, desc, args.thermostat_steps, tuned["mixed"])
        out["thermostat"]["over_nve"] = out["thermostat"]["value"] / out["value"]
    if args.allpairs != "none":
        out["allpairs"] = allpairs_leg(poremd, [int(v) for v in args.allpairs.split(",")])
    sweep_keep = {}
    if args.paper_model != "none":
        out["paper_model"] = paper_model_leg(poremd, precision=args.paper_model)
    if args.sweep != "none":
        out["pore_sweep"], sweep_keep = pore_sweep_leg(
            poremd, args.sweep.split(","), args.sweep_steps,
            0 if (args.skin or args.rebin_every) else min(args.autotune_steps, 50), tkw,
            precisions=("mixed",) if args.no_fp64 else ("mixed", "fp64"))
    if args.batch_systems > 0:
        out["batched"] = batch_leg(poremd, args.batch_systems, args.batch_steps,
                                   min(args.autotune_steps, 200) if args.autotune_steps > 0 else 200)
        if "fp64" in out:
            out["batched"]["over_single_system_fp64"] = out["batched"]["value"] / out["fp64"]["value"]
    if args.serve_requests > 0:
        out["serve"] = serve_leg(args.serve_requests, args.serve_budget_gb, args.serve_chunk)
        out["served_p50_s"] = out["serve"]["p50_s"]
        out["served_p99_s"] = out["serve"]["p99_s"]
    if not args.no_cpu:
        log("timing the oracle on the host ...")
        out["cpu_baseline"], refs = cpu_baseline(
            desc, args.cpu_sample, extra=[(k, v["desc"]) for k, v in sweep_keep.items()])
        # force errors at the initial positions against the oracle's sample
        sel, Fref = refs["headline"]
        for prec, r in res.items():
            e, a = force_errors(r["F0"][sel], Fref)
            out["accuracy"]["force_err_%s_vs_oracle" % prec] = e
            out["accuracy"]["force_err_%s_vs_oracle_per_atom" % prec] = a
            log("[%s] force error vs the oracle's %d-atom sample: %.3e (per atom %.3e)"
                % (prec, len(sel), e, a))
        out["accuracy"]["oracle_sample_atoms"] = int(len(sel))
        for kind, kv in sweep_keep.items():
            es, Fe = refs[kind]
            row = out["pore_sweep"][kind]
            for prec in ("mixed", "fp64"):
                if prec not in kv:
                    continue
                e, a = force_errors(kv[prec][es], Fe)
                tgt = row if prec == "mixed" else row[prec]
                tgt["force_err_vs_oracle"], tgt["force_err_vs_oracle_per_atom"] = e, a
                log("[sweep %s %s] force error vs the oracle's %d-atom sample: %.3e (per atom %.3e)"
                    % (kind, prec, len(es), e, a))
            row["oracle_sample_atoms"] = int(len(es))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
