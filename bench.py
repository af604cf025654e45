"""Benchmark of the MI355X CBS operator.

Workload (one GPU): the ragged batch of 64 synthetic Helmholtz instances with
square grids drawn from {128, 192, 256, 384, 512}, 6-12 points per wavelength,
random-field media of contrast 1.5-4, 32-cell sponge layers and seeded point
sources (about 6.9 M cells).  A step is one batched CBS sweep over all
instances (prologue V u + s, forward 2D FFT, Green symbol, inverse 2D FFT,
epilogue u += gamma r with FP64 partial norms), issued as one set of launches
covering the whole ragged batch; the timed steps form one chain of fused
sweeps issued with direct launches (--graph: replayed from a captured HIP
graph).

Printed: one JSON line with Gcell*CBS-apply/s (value), the HBM roofline of
the sweep (32 algorithmic bytes per cell: read u, V, s, write u), the FP64
oracle timed on the host cores on a bounded sample, and the time to a 1e-6
Born residual for the batch run from a captured hipGraph versus a plain
per-instance loop on the same GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = 32  # complex64: read u, V (from k^2), s; write u


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_18527_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per sweep from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_sweep")


def traffic_record(fetch_csv: str, write_csv: str, workload: str, out_path: str):
    """Turn two rocprofv3 --pmc runs of `bench.py --steps 60 --chain 60
    --warmup 2 --no-layered --no-graph --calib-copy` (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) into the per-sweep traffic record.  These counters count the
    L2's requests to the data fabric, Infinity-Cache hits included: the bytes
    a sweep moves between the L2s and memory, not DRAM-only bytes.

    Each counter is scaled by what it reads for the 1 GiB calibration copy
    (the largest __amd_rocclr_copyBuffer dispatch, issued after the
    autotuner).  Only dispatches from the first k_row_fwd after that copy to
    the last k_row_inv before the NPBS steps count (the autotuner's races
    before and the NPBS steps after launch the sweep kernels on the lanes'
    grids too; the lanes join before the NPBS steps start; the cbs_apply calls
    in the window launch on the whole batch's grids, which the count below
    leaves out).  In between
    the run makes, per lane
    (two lanes, or one when the batch is not split), 62 column-pass (k_col or
    k_col_wide, whichever the autotuner picked) and 60 k_row_sweep dispatches
    of the lane's grid (warm-up call of 2 sweeps, one chain of 60).  Per-sweep bytes: the bytes of every dispatch of a grid
    launched at least that often, divided by the number of sweeps."""
    import csv
    import collections
    sweeps = {"k_row_sweep": 60, "k_col": 62}

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        scale = (1 << 30) / (max(copies) * 1024.0)
        tc = max(int(r["Start_Timestamp"]) for r in rows
                 if "copyBuffer" in r["Kernel_Name"] and float(r["Counter_Value"]) == max(copies))
        t0 = min(int(r["Start_Timestamp"]) for r in rows
                 if "k_row_fwd<float>" in r["Kernel_Name"] and int(r["Start_Timestamp"]) > tc)
        tn = min([int(r["Start_Timestamp"]) for r in rows if "k_row_npbs" in r["Kernel_Name"]] + [1 << 62])
        t1 = max(int(r["Start_Timestamp"]) for r in rows
                 if "k_row_inv<float>" in r["Kernel_Name"] and int(r["Start_Timestamp"]) < tn)
        rows = [r for r in rows if t0 <= int(r["Start_Timestamp"]) <= t1]
        out, grids = {}, {}
        for kern, tags in (("k_row_sweep", ("k_row_sweep<float>",)),
                           ("k_col", ("k_col<float>", "k_col_wide<float>"))):
            by_grid = collections.defaultdict(list)
            for r in rows:
                if any(t in r["Kernel_Name"] for t in tags):
                    by_grid[int(r["Grid_Size"])].append(float(r["Counter_Value"]))
            lanes = sorted(g for g, v in by_grid.items() if len(v) >= sweeps[kern])
            for g in lanes:
                if len(by_grid[g]) % sweeps[kern]:
                    raise ValueError(f"{kern} grid {g}: {len(by_grid[g])} dispatches, not a whole "
                                     f"number of lanes x {sweeps[kern]} sweeps")
            out[kern] = 1024.0 * scale * sum(sum(by_grid[g]) for g in lanes) / sweeps[kern]
            grids[kern] = lanes
        return scale, out, grids

    fs, fetch, grids = load(fetch_csv, "FETCH_SIZE")
    ws, write, _ = load(write_csv, "WRITE_SIZE")
    cmd = ("python -u bench.py --steps 60 --chain 60 --warmup 2 --no-cpu --no-solve --no-layered --no-graph "
           "--calib-copy" + ("" if workload == "ragged64" else f" --workload {workload}"))
    rec = {
        "workload": workload,
        "kernel_source_hash": kernel_source_hash(),
        "fetch_scale": fs,
        "write_scale": ws,
        "lane_grids": grids,
        "bytes_read": fetch,
        "bytes_written": write,
        "bytes_per_sweep": sum(fetch.values()) + sum(write.values()),
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pmc_fetch -o fetch -- " + cmd,
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/pmc_write -o write -- " + cmd,
        ],
    }
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def build_workload(name: str):
    import synthetic as S
    if name == "ragged64":
        probs = S.ragged_batch()
        desc = ("ragged64: 64 instances, N uniform in {128,192,256,384,512}, 6-12 ppw, "
                "contrast 1.5-4, 32-cell sponge, point sources")
    elif name == "layered1024":
        probs = S.layered_batch()
        desc = "layered1024: 8 instances of 1024^2, 5 layers + 10% random field, 8 ppw, 64-cell sponge"
    elif name == "grf256":
        probs = S.workload("grf256")
        desc = "grf256: one 256^2 random-field instance, 10 ppw, 32-cell sponge"
    else:
        raise SystemExit(f"unknown workload {name}")
    return probs, desc


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sweeps(probs, budget_s: float, max_rounds: int):
    """Oracle (FP64, naive DFT) CBS sweeps of every instance in workload
    order, repeated until the time budget is used; the first round's times
    are discarded as warm-up.  Returns (cell-sweeps, seconds, sweeps)."""
    import oracle as O
    state = []
    for p in probs:
        eps = O.choose_eps(p.k2, p.k0sq)
        state.append([p, eps, torch.zeros(p.n, p.n, dtype=torch.complex128)])
    cells = 0
    t_total = 0.0
    sweeps = 0
    for rnd in range(max_rounds + 1):
        for st in state:
            p, eps, u = st
            t0 = time.perf_counter()
            st[2] = O.cbs_sweep(p.k2, p.k0sq, eps, u, p.source)
            dt = time.perf_counter() - t0
            if rnd > 0:
                t_total += dt
                cells += p.n * p.n
                sweeps += 1
        if rnd > 0 and t_total >= budget_s:
            break
    return cells, t_total, sweeps


def cpu_baseline(probs, budget_s: float = 12.0, budget_1t_s: float = 4.0, max_rounds: int = 200):
    """The oracle timed on the host cores over a bounded sample of the
    workload (all torch CPU threads), and the same with one thread on the
    instances of one size (N = 256, or the smallest present)."""
    threads = torch.get_num_threads()
    cells, t_total, sweeps = _oracle_sweeps(probs, budget_s, max_rounds)
    n1 = 256 if any(p.n == 256 for p in probs) else min(p.n for p in probs)
    sub = [p for p in probs if p.n == n1][:2]
    torch.set_num_threads(1)
    try:
        c1, t1, s1 = _oracle_sweeps(sub, budget_1t_s, max_rounds)
    finally:
        torch.set_num_threads(threads)
    return {
        "value": cells / t_total / 1e9,
        "unit": "Gcell*CBS-apply/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "host_logical_cpus": os.cpu_count(),
        "sample": f"{sweeps} FP64 oracle sweeps ({sweeps // len(probs)} per instance over all "
                  f"{len(probs)} instances, {cells} cell-sweeps, {t_total:.1f} s after one warm-up "
                  f"round; torch CPU threads={threads}, host={os.cpu_count()} logical CPUs, {cpu_model()})",
        "one_thread": {"value": c1 / t1 / 1e9, "unit": "Gcell*CBS-apply/s", "cores": 1,
                       "sample": f"{s1} oracle sweeps of {len(sub)} instance(s) of {n1}^2, {t1:.1f} s"},
    }


def lone_sweep_us(k2_i, s_i, n, k0sq_i, use_graph=True, sweeps=2000, chunk=50, dtype=None):
    """Microseconds per sweep of one instance run alone by cbs_iterate (chunks
    of `chunk` sweeps, replayed from a graph or launched directly), with a
    tolerance no run reaches so that every sweep is run."""
    from paper_2603_18527_amd import cbs
    dtype = cbs.CBS_C64 if dtype is None else dtype
    plan = cbs.Plan(k2_i, [n], k0sq=[k0sq_i], dtype=dtype)
    try:
        u = plan.zeros()
        plan.iterate(u, s_i, max_sweeps=chunk, rtol=1e-30, check_every=chunk, use_graph=use_graph)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, _, _ = plan.iterate(u, s_i, max_sweeps=sweeps, rtol=1e-30, check_every=chunk,
                                 use_graph=use_graph)
        dt = time.perf_counter() - t0
    finally:
        plan.close()
    return dt * 1e6 / max(1, its[0])


def tail_probe(probs):
    """Per-sweep cost of a lone instance of each grid size of the batch (the
    convergence tail of a batched solve runs one or two such instances)."""
    import synthetic as S
    from paper_2603_18527_amd import cbs
    out = {}
    seen = set()
    for p in probs:
        if p.n in seen:
            continue
        seen.add(p.n)
        k2 = cbs.pack([p.k2], torch.complex64)
        s = cbs.pack([p.source], torch.complex64)
        out[str(p.n)] = {"graph_us_per_sweep": lone_sweep_us(k2, s, p.n, p.k0sq, True),
                         "direct_us_per_sweep": lone_sweep_us(k2, s, p.n, p.k0sq, False)}
        print(f"# lone {p.n}^2: {out[str(p.n)]}", flush=True)
    # the shape of the paper's own CBS timing (one 288^2 instance, 256^2
    # interior and a 16-cell layer, random-field medium), in FP64 and FP32
    q = S.grf_problem(n=288, layer=16)
    row = {}
    for name, dt, tdt in (("fp64", cbs.CBS_C128, torch.complex128), ("fp32", cbs.CBS_C64, torch.complex64)):
        k2 = cbs.pack([q.k2], tdt)
        s = cbs.pack([q.source], tdt)
        row[name + "_graph_us_per_sweep"] = lone_sweep_us(k2, s, 288, q.k0sq, True, dtype=dt)
    out["288_grf"] = row
    print(f"# lone 288^2 random field: {row}", flush=True)
    return out


def time_to_solution(probs, plan_k2, sizes, k0sq, s_packed, rtol=1e-6, chunk=50, max_sweeps=20000):
    from paper_2603_18527_amd import cbs
    out = {}
    # batched: one plan, every chunk replayed from a captured hipGraph
    plan = cbs.Plan(plan_k2, sizes, k0sq=k0sq)
    u = plan.zeros()
    plan.iterate(u, s_packed, max_sweeps=60, rtol=rtol, check_every=chunk, use_graph=True)  # capture
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, rel, stat = plan.iterate(u, s_packed, max_sweeps=max_sweeps, rtol=rtol, check_every=chunk,
                                  use_graph=True)
    t_batch = time.perf_counter() - t0
    out["batched_graph_s"] = t_batch
    out["batched_sweeps_max"] = int(max(its))
    by = {}
    for n, k in zip(sizes, its):
        lo, hi = by.get(str(n), (k, k))
        by[str(n)] = (min(lo, k), max(hi, k))
    out["sweeps_min_max_by_size"] = by
    out["sweeps_sorted_top8"] = sorted((int(k) for k in its), reverse=True)[:8]
    out["batched_all_converged"] = all(s == cbs.INST_CONVERGED for s in stat)
    out["batched_max_relres"] = float(max(rel))
    # the slowest instance run alone: its sweep count times its lone per-sweep
    # cost is the tail the batched time cannot go below
    offs = cbs.offsets(sizes)
    i_slow = int(np.argmax(its))
    n_slow = sizes[i_slow]
    sl = slice(offs[i_slow], offs[i_slow] + n_slow * n_slow)
    us = lone_sweep_us(plan_k2[sl].contiguous(), s_packed[sl].contiguous(), n_slow, k0sq[i_slow])
    out["slowest_instance"] = {"n": n_slow, "sweeps": int(its[i_slow]), "lone_us_per_sweep": us,
                               "lone_sweeps_s": us * 1e-6 * int(its[i_slow])}
    # plain: a per-instance loop of plans with ordinary launches
    t_plain = 0.0
    t_512 = []
    for i, n in enumerate(sizes):
        sl = slice(offs[i], offs[i] + n * n)
        pi = cbs.Plan(plan_k2[sl].contiguous(), [n], k0sq=[k0sq[i]])
        ui = pi.zeros()
        si = s_packed[sl].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pi.iterate(ui, si, max_sweeps=max_sweeps, rtol=rtol, check_every=chunk, use_graph=False)
        dt = time.perf_counter() - t0
        t_plain += dt
        if n == 512:
            t_512.append(dt)
        pi.close()
    out["plain_loop_s"] = t_plain
    out["speedup_batched_vs_plain"] = t_plain / t_batch
    if t_512:
        # the 512^2 instances alone: one batched plan (graph replay) against
        # the per-instance loop over the same instances timed above
        idx = [i for i, n in enumerate(sizes) if n == 512]
        k2_512 = torch.cat([plan_k2[offs[i]:offs[i] + n * n] for i, n in enumerate(sizes) if n == 512])
        s_512 = torch.cat([s_packed[offs[i]:offs[i] + n * n] for i, n in enumerate(sizes) if n == 512])
        pb = cbs.Plan(k2_512.contiguous(), [512] * len(idx), k0sq=[k0sq[i] for i in idx])
        ub = pb.zeros()
        pb.iterate(ub, s_512, max_sweeps=60, rtol=rtol, check_every=chunk, use_graph=True)
        ub.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its5, rel5, st5 = pb.iterate(ub, s_512, max_sweeps=max_sweeps, rtol=rtol, check_every=chunk,
                                     use_graph=True)
        t_b512 = time.perf_counter() - t0
        pb.close()
        out["n_512_instances"] = len(t_512)
        out["batched_512_s"] = t_b512
        out["batched_512_sweeps_max"] = int(max(its5))
        out["batched_512_all_converged"] = all(x == cbs.INST_CONVERGED for x in st5)
        out["plain_512_loop_s"] = float(np.sum(t_512))
        out["plain_512_each_s_mean"] = float(np.mean(t_512))
        out["speedup_512_batched_vs_plain"] = float(np.sum(t_512)) / t_b512
    out["chunk"] = chunk
    out["rtol"] = rtol
    return out


def apply_throughput(plan, sizes, s, calls=20):
    """cbs_apply y = G(V u + s) on the batch, `calls` independent calls back
    to back (three launches each; the two lanes of a large batch overlap one
    lane's column pass with the other's row passes): Gcell * apply / s and the
    fraction of the HBM roofline at 32 algorithmic bytes per cell."""
    cells = sum(n * n for n in sizes)
    g = torch.Generator(device="cpu").manual_seed(2027)
    u = torch.complex(torch.randn(cells, generator=g), torch.randn(cells, generator=g)).to(torch.complex64).cuda()
    y = plan.empty()
    for _ in range(3):
        plan.apply(u, s, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(calls):
        plan.apply(u, s, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    achieved = BYTES_PER_CELL * cells / (ms * 1e-3) / 1e9
    return {"unit": "Gcell*apply/s", "value": cells / (ms * 1e-3) / 1e9, "ms_per_apply": ms, "calls": calls,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS}}


def npbs_throughput(plan, sizes, s, steps=20):
    """NPBS steps with a linear Fourier layer of seeded random weights (the
    learned preconditioner's residual branch; two transform pairs per step)
    over the same batch: Gcell * NPBS-step / s."""
    g = torch.Generator(device="cpu").manual_seed(2026)
    cells = sum(n * n for n in sizes)

    def field(scale):
        x = torch.complex(torch.randn(cells, generator=g), torch.randn(cells, generator=g))
        return (scale * x).to(torch.complex64).cuda()
    wf, wl = field(0.3), field(0.3)
    u = plan.zeros()
    plan.npbs_step(u, s, wf, wl, count=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.npbs_step(u, s, wf, wl, count=steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"unit": "Gcell*NPBS-step/s", "value": cells / dt / 1e9, "ms_per_step": dt * 1e3,
            "steps": steps, "transform_pairs_per_step": 2,
            "weights": "seeded random spectral and local weights, 0.3 * CN(0, 1)"}


def _gcell(cells, applies, seconds):
    return cells * applies / seconds / 1e9


def fp64_born_relres(p, plan, u, s):
    """||G(V u + s) - u|| / ||G s|| of an FP32 plan's solution, evaluated by an
    FP64 plan of the same problem (same k0^2 and eta) on the GPU."""
    from paper_2603_18527_amd import cbs
    c128 = torch.complex128
    p64 = cbs.Plan(cbs.pack([p.k2], c128), [p.n], k0sq=plan.k0sq, eps=plan.eps, dtype=cbs.CBS_C128,
                   guard=False)
    _, rn = p64.residual(u.to(c128), s.to(c128), store=False)
    _, bn = p64.residual(None, s.to(c128), store=False)
    return float(torch.sqrt(rn[0] / bn[0]))


def fp64_physical_relres(p, plan, u, s):
    """||s - A u|| / ||s|| evaluated by an FP64 plan on the GPU."""
    from paper_2603_18527_amd import cbs
    c128 = torch.complex128
    p64 = cbs.Plan(cbs.pack([p.k2], c128), [p.n], k0sq=plan.k0sq, eps=plan.eps, dtype=cbs.CBS_C128,
                   guard=False)
    _, hn = p64.helmholtz_residual(u.to(c128), s.to(c128), store=False)
    return float(torch.sqrt(hn[0]) / torch.linalg.vector_norm(s.to(c128)))


def time_sweeps(plan, s, steps: int, warmup: int, chain_len: int, graph: bool = True, repeats: int = 10):
    """`steps` CBS sweeps in place on a zero field, as chains of `chain_len`
    fused sweeps (one cbs_sweep call each), after `warmup` untimed sweeps.
    With graph=True the chain is captured once into a HIP graph during the
    warm-up (the lanes' fork and join included) and replayed.  Wall time over
    the whole timed region (synchronised before and after) and HIP events on
    the launch stream (the lanes join back into it) around every chain."""
    u = plan.zeros()
    stream = torch.cuda.current_stream()
    chain = max(1, min(chain_len, steps))
    plan.sweep(u, s, count=max(1, warmup))
    torch.cuda.synchronize()
    run = lambda: plan.sweep(u, s, count=chain)
    if graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            plan.sweep(u, s, count=chain)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            plan.sweep(u, s, count=chain)
        torch.cuda.synchronize()
        run = g.replay
    nchains = max(1, steps // chain)
    steps = nchains * chain
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nchains + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(nchains):
        run()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    chain_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(nchains)]
    # the same timed region repeated (outside the region the line reports):
    # median, min and max over 10 runs of `steps` sweeps by events
    reps = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _k in range(nchains):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) / steps)
    return {"steps": steps, "chain": chain, "graph": graph, "wall_ms_per_sweep": wall * 1e3 / steps,
            "event_ms_per_sweep": float(np.mean(chain_ms)) / chain,
            "repeats_ms_per_sweep": None if not reps else
            {"runs": len(reps), "median": float(np.median(reps)), "min": float(np.min(reps)),
             "max": float(np.max(reps))}}


def layered_leg(fgmres: bool = True, graph: bool = False):
    """8 x 1024^2 layered media (the high-wavenumber stress batch): the sweep
    on a working set larger than the 256 MB Infinity Cache (u, k^2, s and the
    spectral buffer: 268 MB), with its own roofline, and FGMRES(50) + 4 CBS
    sweeps to 1e-6 in FP32 (FP64 Arnoldi) against an all-FP64 GPU run of the
    same problems, error per instance."""
    import synthetic as S
    from paper_2603_18527_amd import cbs
    probs = S.layered_batch()
    sizes = [q.n for q in probs]
    cells = sum(n * n for n in sizes)
    k2 = cbs.pack([q.k2 for q in probs], torch.complex64)
    s = cbs.pack([q.source for q in probs], torch.complex64)
    plan = cbs.Plan(k2, sizes, k0sq=[q.k0sq for q in probs], max_restart=50 if fgmres else 0)
    tiles = plan.autotune()
    st = time_sweeps(plan, s, 100, 10, 50, graph=graph)
    traffic = measured_traffic("layered1024")
    achieved = BYTES_PER_CELL * cells / (st["event_ms_per_sweep"] * 1e-3) / 1e9
    out = {
        "workload": "layered1024: 8 instances of 1024^2, 5 layers + 10% random field, 8 ppw, 64-cell sponge",
        "cells": cells, "working_set_bytes": 4 * 8 * cells, "column_tile": tiles[0],
        "sweep": {"value": cells / (st["wall_ms_per_sweep"] * 1e-3) / 1e9, "unit": "Gcell*CBS-apply/s",
                  "steps": st["steps"], "ms_per_step": st["wall_ms_per_sweep"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "event_ms_per_sweep": st["event_ms_per_sweep"],
                     "algorithmic_bytes_per_sweep": BYTES_PER_CELL * cells, "traffic": traffic,
                     # L2-to-fabric bytes; the working set exceeds the Infinity
                     # Cache, so nearly all of them reach DRAM
                     "l2_fabric_bytes_per_cell": None if traffic is None else traffic / cells,
                     "l2_fabric_gbs": None if traffic is None else
                     traffic / (st["event_ms_per_sweep"] * 1e-3) / 1e9},
    }
    if fgmres:
        sol = {}
        for name, dtype, tdt in (("fp32", cbs.CBS_C64, torch.complex64), ("fp64", cbs.CBS_C128, torch.complex128)):
            if name == "fp64":
                del plan
                plan = cbs.Plan(cbs.pack([q.k2 for q in probs], tdt), sizes, k0sq=[q.k0sq for q in probs],
                                dtype=dtype, max_restart=50)
                plan.autotune()
            sv = cbs.pack([q.source for q in probs], tdt)
            u = plan.zeros()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its, rel, stt = plan.fgmres(u, sv, restart=50, sweeps=4, max_iters=3000, rtol=1e-6)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            out[f"fgmres50_k4_{name}"] = {"seconds": dt, "iterations": its, "relres": rel,
                                          "all_converged": all(x == cbs.INST_CONVERGED for x in stt)}
            sol[name] = u.to(torch.complex128)
        out["fgmres_rel_err_fp32_vs_fp64_gpu"] = [
            float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
            for a, b in zip(cbs.unpack(sol["fp32"], sizes), cbs.unpack(sol["fp64"], sizes))]
    return out


def cdr_throughput():
    """Convection-diffusion-reaction plans (App. B.1) on a ragged batch of 64
    instances (sizes as ragged64): G_cdr (V_cdr u + s) and R^H e, timed with
    HIP events on the launch stream; the FP32 apply is compared with an FP64
    plan of the same batch on the GPU."""
    import synthetic as S
    from paper_2603_18527_amd import cbs
    probs = S.cdr_batch()
    sizes = [q.n for q in probs]
    cells = sum(n * n for n in sizes)
    ks = cbs.pack([q.kappa + 1j * q.sigma for q in probs], torch.complex64)
    vel = cbs.pack([q.vx + 1j * q.vy for q in probs], torch.complex64)
    plan = cbs.CdrPlan(ks, vel, sizes, [q.background for q in probs])
    tiles = plan.autotune()
    s = cbs.pack([q.source for q in probs], torch.complex64)
    g = torch.Generator(device="cpu").manual_seed(5)
    x = torch.complex(torch.randn(cells, generator=g), torch.randn(cells, generator=g)).to(torch.complex64).cuda()
    y = plan.empty()

    def ev_time(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b) / reps)
        return best * 1e-3

    dta = ev_time(lambda: plan.apply(x, s, out=y))
    dtg = ev_time(lambda: plan.born_adjoint(x, out=y))
    yi = plan.apply(x, s)
    c128 = torch.complex128
    plan64 = cbs.CdrPlan(cbs.pack([q.kappa + 1j * q.sigma for q in probs], c128),
                         cbs.pack([q.vx + 1j * q.vy for q in probs], c128), sizes,
                         [q.background for q in probs], dtype=cbs.CBS_C128)
    y64 = plan64.apply(x.to(c128), s.to(c128))
    errs = [float(torch.linalg.vector_norm(a.to(c128) - b) / torch.linalg.vector_norm(b))
            for a, b in zip(cbs.unpack(yi, sizes), cbs.unpack(y64, sizes))]
    return dict(
        instances=len(sizes), cells=cells, column_tiles={str(n): t for n, t in sorted(set(zip(sizes, tiles)))},
        apply_ms=dta * 1e3, apply_gcell_s=_gcell(cells, 1, dta),
        apply_algorithmic_gbs=40.0 * cells / dta / 1e9,
        born_adjoint_ms=dtg * 1e3, born_adjoint_gcell_s=_gcell(cells, 1, dtg),
        note="40 algorithmic B/cell per apply: read u, (kappa, sigma), (vx, vy), s; write y",
        max_rel_err_fp32_vs_fp64_gpu=max(errs))


def run_suite(args):
    """Solver runs on the five synthetic workloads (configs of the metric):
    blob64 CBS, grf256 FGMRES(30)+CBS(4) and CBS, ragged64 FGMRES batched,
    diff16 adjoint, layered1024 FGMRES(50)+CBS(4) in FP32 vs an FP64 GPU run;
    the Dirichlet (DST-I) Newton-system batch newton64 (damped reference with
    FGMRES + CBS sweeps, and the undamped reference with GMRES); the DST-I
    path at its largest size (9 x 511^2) beside a periodic 9 x 512^2 batch;
    and the convection-diffusion-reaction batch cdr64 (apply and R^H e
    throughput).
    Accuracy figures come from FP64 plans of the same problems on the GPU
    (parity with the FP64 CPU oracle is the test suite's job)."""
    import synthetic as S
    from paper_2603_18527_amd import cbs

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    res = {}
    # 1. blob64: stationary CBS to 1e-6, FP32 operator with FP64 refinement
    p = S.blob_problem()
    k2 = cbs.pack([p.k2], torch.complex64)
    plan = cbs.Plan(k2, [p.n], k0sq=[p.k0sq])
    s = cbs.pack([p.source], torch.complex64)
    u = plan.zeros()
    plan.iterate(u, s, max_sweeps=50, check_every=25)
    u.zero_()
    (its, rel, st), dt = timed(lambda: plan.iterate(u, s, max_sweeps=5000, rtol=1e-6, check_every=25))
    ev64 = fp64_born_relres(p, plan, u, s)
    res["blob64_cbs"] = dict(sweeps=its[0], seconds=dt, relres_reported=rel[0],
                             relres_fp64_gpu_eval=ev64,
                             gcell_apply_s=_gcell(p.n * p.n, its[0], dt), converged=st[0] == 1)
    # the same solve under the paper's unified rule rTol = ||s - A u|| / ||s||
    u.zero_()
    (its, rel, st), dt = timed(lambda: plan.iterate(u, s, max_sweeps=5000, rtol=1e-6, check_every=25,
                                                    stop="physical"))
    res["blob64_cbs_rtol_physical"] = dict(
        sweeps=its[0], check_every=25, seconds=dt, rtol_reported=rel[0],
        rtol_fp64_gpu_eval=fp64_physical_relres(p, plan, u, s), converged=st[0] == 1)
    print("# suite blob64 done", flush=True)
    # 2. grf256: FGMRES(30) with 4 CBS sweeps, and stationary CBS
    p = S.grf_problem()
    k2 = cbs.pack([p.k2], torch.complex64)
    plan = cbs.Plan(k2, [p.n], k0sq=[p.k0sq], max_restart=30)
    s = cbs.pack([p.source], torch.complex64)
    u = plan.zeros()
    plan.fgmres(u, s, restart=30, sweeps=4, max_iters=5)
    u.zero_()
    (its, rel, st), dt = timed(lambda: plan.fgmres(u, s, restart=30, sweeps=4, max_iters=2500, rtol=1e-6))
    res["grf256_fgmres30_k4"] = dict(iterations=its[0], seconds=dt, relres_reported=rel[0],
                                     relres_fp64_gpu_eval=fp64_born_relres(p, plan, u, s),
                                     applies_per_iteration=5,   # K = 4 sweeps of P_K and B z
                                     gcell_apply_s=_gcell(p.n * p.n, 5 * its[0], dt), converged=st[0] == 1)
    u2 = plan.zeros()
    plan.iterate(u2, s, max_sweeps=50)
    u2.zero_()
    (its, rel, st), dt = timed(lambda: plan.iterate(u2, s, max_sweeps=20000, rtol=1e-6, check_every=50))
    res["grf256_cbs"] = dict(sweeps=its[0], seconds=dt, relres_reported=rel[0],
                             relres_fp64_gpu_eval=fp64_born_relres(p, plan, u2, s),
                             gcell_apply_s=_gcell(p.n * p.n, its[0], dt), converged=st[0] == 1)
    print("# suite grf256 done", flush=True)
    # 3. ragged64: batched FGMRES(30)+CBS(4) (the CBS runs are in the main line)
    probs = S.ragged_batch()
    sizes = [q.n for q in probs]
    k2 = cbs.pack([q.k2 for q in probs], torch.complex64)
    s = cbs.pack([q.source for q in probs], torch.complex64)
    plan = cbs.Plan(k2, sizes, k0sq=[q.k0sq for q in probs], max_restart=30)
    plan.autotune()
    u = plan.zeros()
    (its, rel, st), dt = timed(lambda: plan.fgmres(u, s, restart=30, sweeps=4, max_iters=2500, rtol=1e-6))
    res["ragged64_fgmres30_k4_batched"] = dict(max_iterations=max(its), seconds=dt,
                                               max_relres=max(rel), all_converged=all(x == 1 for x in st))
    del plan
    print("# suite ragged64 fgmres done", flush=True)
    # 4. diff16: K = 8 unrolled steps, loss with W = gamma, hand adjoint
    probs, u0s, ss = S.diff_batch()
    sizes = [q.n for q in probs]
    cells = sum(n * n for n in sizes)
    k2 = cbs.pack([q.k2 for q in probs], torch.complex64)
    u0 = cbs.pack(u0s, torch.complex64)
    s = cbs.pack(ss, torch.complex64)
    plan = cbs.Plan(k2, sizes, k0sq=[q.k0sq for q in probs])

    def fwd_bwd():
        us = plan.sweep_checkpoints(u0, s, 8)   # u_0..u_8, one fused chain
        loss, lam, grad = plan.loss_seed(us[-1], s, True)
        for m in range(7, -1, -1):
            plan.adjoint_step(us[m], s, lam, lam, grad)
        return loss

    fwd_bwd()
    _, dt = timed(fwd_bwd)
    # applications: 8 sweeps + seed (2) + 8 adjoint steps (2 each)
    res["diff16_k8_forward_backward"] = dict(seconds=dt, applies=26,
                                             gcell_apply_s=_gcell(cells, 26, dt))
    print("# suite diff16 done", flush=True)
    # 5. layered1024: FGMRES(50) + CBS(4), FP32 operator vs an all-FP64 GPU run
    probs = S.layered_batch()
    sizes = [q.n for q in probs]
    cells = sum(n * n for n in sizes)
    out = {}
    sol = {}
    for name, dtype, tdt in (("fp32", cbs.CBS_C64, torch.complex64), ("fp64", cbs.CBS_C128, torch.complex128)):
        k2 = cbs.pack([q.k2 for q in probs], tdt)
        s = cbs.pack([q.source for q in probs], tdt)
        plan = cbs.Plan(k2, sizes, k0sq=[q.k0sq for q in probs], dtype=dtype, max_restart=50)
        plan.autotune()
        u = plan.zeros()
        (its, rel, st), dt = timed(lambda: plan.fgmres(u, s, restart=50, sweeps=4, max_iters=3000,
                                                       rtol=1e-6))
        out[name] = dict(iterations=its, seconds=dt, relres=rel, converged=[x == 1 for x in st],
                         gcell_apply_s=_gcell(cells, 5 * max(its), dt))   # K + 1 applies per step
        sol[name] = u.to(torch.complex128)
        # sweep throughput on this > Infinity-Cache working set
        if name == "fp32":
            x = plan.zeros()
            plan.sweep(x, s, count=10)
            dts = min(timed(lambda: plan.sweep(x, s, count=50))[1] for _ in range(3))
            out["fp32_sweep_gcell_apply_s"] = _gcell(cells, 50, dts)
            out["fp32_sweep_ms"] = dts * 1e3 / 50
        del plan
        print(f"# suite layered1024 {name} done", flush=True)
    errs = []
    for a, b in zip(cbs.unpack(sol["fp32"], sizes), cbs.unpack(sol["fp64"], sizes)):
        errs.append(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)))
    out["rel_err_fp32_vs_fp64_per_instance"] = errs
    res["layered1024_fgmres50_k4"] = out
    # 6. newton64: Dirichlet (DST-I reference) Newton Jacobians J = L_D - 2 diag(u_m),
    #    100 instances of 64^2 interior points; FGMRES(20) + 3 CBS sweeps to 1e-6 with
    #    the damped reference, GMRES(20) with the undamped J_0 = L_D - 2 mean(u_m)
    probs = S.newton_batch()
    sizes = [q.n for q in probs]
    cells = sum(n * n for n in sizes)
    k2 = cbs.pack([q.k2 for q in probs], torch.complex64)
    s = cbs.pack([q.source for q in probs], torch.complex64)
    plan = cbs.Plan(k2, sizes, dirichlet=True, max_restart=20)
    x = plan.zeros()
    plan.apply(x, s)
    dta = min(timed(lambda: [plan.apply(x, s) for _ in range(20)])[1] for _ in range(3)) / 20
    plan.sweep(x, s, count=10)
    dts = min(timed(lambda: plan.sweep(x, s, count=50))[1] for _ in range(3)) / 50
    u = plan.zeros()
    (its, rel, st), dt = timed(lambda: plan.fgmres(u, s, restart=20, sweeps=3, max_iters=2000, rtol=1e-6))
    c128 = torch.complex128
    p64 = cbs.Plan(k2.to(c128), sizes, k0sq=plan.k0sq, eps=plan.eps, dtype=cbs.CBS_C128,
                   dirichlet=True, guard=False)
    _, rn = p64.residual(u.to(c128), s.to(c128), store=False)
    _, bn = p64.residual(None, s.to(c128), store=False)
    ev = float(torch.max(torch.sqrt(rn / bn)))
    k0u = [float(np.mean(np.real(q.k2))) for q in probs]   # k0^2 = 2 mean(u_m) = mean(k^2), alpha = 0
    pu = cbs.Plan(k2, sizes, k0sq=k0u, dirichlet=True, undamped=True, max_restart=20)
    uu = pu.zeros()
    (itu, relu, stu), dtu = timed(lambda: pu.fgmres(uu, s, restart=20, sweeps=0, max_iters=2000, rtol=1e-6))
    res["newton64_dirichlet"] = dict(
        instances=len(sizes), cells=cells, apply_ms=dta * 1e3, apply_gcell_s=_gcell(cells, 1, dta),
        sweep_ms=dts * 1e3, sweep_gcell_s=_gcell(cells, 1, dts),
        fgmres20_k3=dict(seconds=dt, max_iterations=max(its), max_relres=max(rel),
                         all_converged=all(x == 1 for x in st), max_relres_fp64_gpu_eval=ev),
        undamped_gmres20=dict(seconds=dtu, max_iterations=max(itu), max_relres=max(relu),
                              all_converged=all(x == 1 for x in stu)))
    print("# suite newton64 done", flush=True)
    # 7. dirichlet511: the DST-I path at its largest size, 9 x 511^2 interior
    #    points (transforms of length 1024 on the odd extension), FP32 apply and
    #    fused-sweep throughput against the 32 algorithmic B/cell of a sweep,
    #    beside a periodic 9 x 512^2 batch of the same media recipe
    #    (k^2 = 100 + 60 zeta, zeta a random field of correlation n/8); nine
    #    instances put both batches above the two-lane threshold of 2^21 cells
    big = {}
    for name, n, dirichlet in (("dirichlet_511", 511, True), ("periodic_512", 512, False)):
        k2l, srcl = [], []
        for i in range(9):
            rng = S.rng_for(7, i)
            k2l.append(100.0 + 60.0 * S.gaussian_random_field(n, n / 8, rng))
            srcl.append(S.random_field_c(n, rng))
        sizes = [n] * 9
        cells = 9 * n * n
        plan = cbs.Plan(cbs.pack(k2l, torch.complex64), sizes, dirichlet=dirichlet)
        s = cbs.pack(srcl, torch.complex64)
        x = plan.zeros()
        plan.apply(x, s)
        dta = min(timed(lambda: [plan.apply(x, s) for _ in range(20)])[1] for _ in range(3)) / 20
        plan.sweep(x, s, count=10)
        dts = min(timed(lambda: plan.sweep(x, s, count=50))[1] for _ in range(3)) / 50
        big[name] = dict(cells=cells, lanes=plan.layout()[0], apply_us=dta * 1e6, apply_gcell_s=_gcell(cells, 1, dta),
                         sweep_us=dts * 1e6, sweep_gcell_s=_gcell(cells, 1, dts),
                         sweep_frac_of_8tbs_by_32b=cells * 32 / dts / 8e12)
        del plan
    res["dirichlet511_vs_periodic512"] = big
    print("# suite dirichlet511 done", flush=True)
    res["cdr64_apply"] = cdr_throughput()
    print("# suite cdr64 done", flush=True)
    return res


def main():

    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ragged64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1e-6 and FGMRES runs")
    ap.add_argument("--no-layered", action="store_true", help="skip the 8 x 1024^2 layered leg")
    ap.add_argument("--graph", action="store_true",
                    help="replay the timed sweep chains from a captured graph (default: direct launches, "
                         "about 2 us per sweep faster at 20 sweeps per chain on MI355X)")
    ap.add_argument("--no-graph", action="store_true", help="direct launches (the default)")
    ap.add_argument("--chain", type=int, default=50, help="sweeps fused per cbs_sweep call")
    ap.add_argument("--cdr", action="store_true",
                    help="only time the convection-diffusion-reaction apply / adjoint (cdr64 batch)")
    ap.add_argument("--tail", action="store_true",
                    help="only time one sweep of a lone instance of each grid size (graph and direct)")
    ap.add_argument("--suite", action="store_true",
                    help="also run the solver suite over all five synthetic workloads")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from rocprofv3 counter CSVs and exit")
    args = ap.parse_args()
    if args.traffic_from:
        rec = traffic_record(args.traffic_from[0], args.traffic_from[1], args.workload,
                             os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json"))
        print(json.dumps(rec))
        return
    if args.cdr:
        if not torch.cuda.is_available():
            raise SystemExit("no GPU visible")
        print(json.dumps({"cdr64_apply": cdr_throughput()}), flush=True)
        return
    if args.tail:
        if not torch.cuda.is_available():
            raise SystemExit("no GPU visible")
        probs, _ = build_workload(args.workload)
        print(json.dumps({"lone_instance_sweep": tail_probe(probs)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the instances of a batch "
              "are independent, so several GPUs would each run their own share.", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")

    from paper_2603_18527_amd import cbs
    probs, desc = build_workload(args.workload)
    sizes = [p.n for p in probs]
    cells = sum(n * n for n in sizes)
    k0sq = [p.k0sq for p in probs]
    k2 = cbs.pack([p.k2 for p in probs], torch.complex64)
    s = cbs.pack([p.source for p in probs], torch.complex64)
    plan = cbs.Plan(k2, sizes, k0sq=k0sq)
    tiles = plan.autotune()
    tile_by_size = {str(n): t for n, t in sorted(set(zip(sizes, tiles)))}
    if args.calib_copy:
        # after the autotuner, so that the copy also marks where its races end
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("# calibration copy: 1073741824 bytes read, 1073741824 bytes written", flush=True)
        del a, b
    print(f"# workload {args.workload}: {len(sizes)} instances, {cells} cells, column tiles "
          f"{tile_by_size}", flush=True)

    use_graph = args.graph and not args.no_graph
    # the counter runs (--calib-copy) count the dispatches of one timed chain
    # per lane, so they skip the repeated runs
    st = time_sweeps(plan, s, args.steps, args.warmup, args.chain, graph=use_graph,
                     repeats=0 if args.calib_copy else 10)
    ms_step = st["wall_ms_per_sweep"]
    ev_ms = st["event_ms_per_sweep"]
    value = cells / (ms_step * 1e-3) / 1e9
    achieved = BYTES_PER_CELL * cells / (ev_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    line = {
        "metric": "Gcell*CBS-apply/s (batched CBS sweep); time to 1e-6 residual batched vs plain",
        "value": value,
        "unit": "Gcell*CBS-apply/s",
        "n_gpus": 1,
        "steps": st["steps"],
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 complex), fp64 norms",
        "data": "synthetic",
        "config": {"workload": desc, "instances": len(sizes), "cells": cells,
                   "sizes": {str(n): sizes.count(n) for n in sorted(set(sizes))},
                   "column_tiles": tile_by_size},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "CBS sweep: k_col + k_row_sweep (fused inverse/forward rows) over the ragged batch",
            "sweeps_per_chain": st["chain"],
            "chain_from_graph": st["graph"],
            "algorithmic_bytes_per_sweep": BYTES_PER_CELL * cells,
            "event_ms_per_sweep": ev_ms,
            # 10 further runs of the same region (median, min, max), and the
            # fraction at their median
            "repeats_ms_per_sweep": st["repeats_ms_per_sweep"],
            "frac_at_repeat_median": None if st["repeats_ms_per_sweep"] is None else
            BYTES_PER_CELL * cells / (st["repeats_ms_per_sweep"]["median"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            # FETCH_SIZE / WRITE_SIZE count L2-to-fabric requests: Infinity-Cache
            # hits included, so these are not DRAM-only bytes
            "l2_fabric_bytes_per_cell": None if traffic is None else traffic / cells,
            "l2_fabric_gbs": None if traffic is None else traffic / (ev_ms * 1e-3) / 1e9,
            "working_set_bytes": 4 * 8 * cells,
        },
    }
    line["apply"] = apply_throughput(plan, sizes, s)
    line["npbs_step"] = npbs_throughput(plan, sizes, s)
    if not args.no_layered:
        del plan
        torch.cuda.empty_cache()
        line["layered1024"] = layered_leg(fgmres=not args.no_solve, graph=use_graph)
        plan = None
    if not args.no_solve:
        line["time_to_1e-6"] = time_to_solution(probs, k2, sizes, k0sq, s)
    if args.suite:
        line["suite"] = run_suite(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(probs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
