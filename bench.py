"""Benchmark of the MI355X CBS operator.

Workload (one GPU): the ragged batch of 64 synthetic Helmholtz instances with
square grids drawn from {128, 192, 256, 384, 512}, 6-12 points per wavelength,
random-field media of contrast 1.5-4, 32-cell sponge layers and seeded point
sources (about 6.9 M cells).  A step is one batched CBS sweep over all
instances (prologue V u + s, forward 2D FFT, Green symbol, inverse 2D FFT,
epilogue u += gamma r with FP64 partial norms), issued as one set of launches
covering the whole ragged batch.

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


def cpu_baseline(probs, budget_s: float = 12.0, max_rounds: int = 200):
    """Oracle (FP64, naive DFT) CBS sweeps on the host over a bounded sample:
    one sweep of every instance in workload order, repeated until the time
    budget is used (the first round's times are discarded as warm-up)."""
    import oracle as O
    threads = torch.get_num_threads()
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
    return {
        "value": cells / t_total / 1e9,
        "unit": "Gcell*CBS-apply/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{sweeps} FP64 oracle sweeps ({sweeps // len(probs)} per instance over all "
                  f"{len(probs)} instances, {cells} cell-sweeps, {t_total:.1f} s after one warm-up "
                  f"round; torch CPU threads={threads}, host={os.cpu_count()} logical CPUs)",
    }


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
    out["batched_all_converged"] = all(s == cbs.INST_CONVERGED for s in stat)
    out["batched_max_relres"] = float(max(rel))
    # plain: a per-instance loop of plans with ordinary launches
    offs = cbs.offsets(sizes)
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
        out["plain_512_each_s_mean"] = float(np.mean(t_512))
        out["n_512_instances"] = len(t_512)
    out["chunk"] = chunk
    out["rtol"] = rtol
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ragged64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1e-6 runs")
    ap.add_argument("--tile", type=int, default=0, help="force the column tile (0: autotune)")
    ap.add_argument("--chain", type=int, default=50, help="sweeps fused per cbs_sweep call")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the instances of a batch "
              "are independent, so several GPUs would each run their own share.", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")

    from paper_2603_18527_amd import cbs
    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("# calibration copy: 1073741824 bytes read, 1073741824 bytes written", flush=True)
        del a, b
    probs, desc = build_workload(args.workload)
    sizes = [p.n for p in probs]
    cells = sum(n * n for n in sizes)
    k0sq = [p.k0sq for p in probs]
    k2 = cbs.pack([p.k2 for p in probs], torch.complex64)
    s = cbs.pack([p.source for p in probs], torch.complex64)
    plan = cbs.Plan(k2, sizes, k0sq=k0sq)
    tile = plan.set_tile(args.tile) if args.tile else plan.autotune()
    print(f"# workload {args.workload}: {len(sizes)} instances, {cells} cells, column tile "
          f"{args.tile or tile}", flush=True)

    u = plan.zeros()
    stream = torch.cuda.current_stream()
    # Steps run as chains of `chain` fused sweeps (one cbs_sweep call each);
    # HIP events on the launch stream bracket every chain.
    chain = max(1, min(args.chain, args.steps))
    plan.sweep(u, s, count=max(1, args.warmup))
    torch.cuda.synchronize()
    nchains = max(1, args.steps // chain)
    steps = nchains * chain
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nchains + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(nchains):
        plan.sweep(u, s, count=chain)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    chain_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(nchains)]
    ms_step = wall * 1e3 / steps
    ev_ms = float(np.mean(chain_ms)) / chain
    value = cells / (ms_step * 1e-3) / 1e9
    achieved = BYTES_PER_CELL * cells / (ev_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    line = {
        "metric": "Gcell*CBS-apply/s (batched CBS sweep); time to 1e-6 residual batched vs plain",
        "value": value,
        "unit": "Gcell*CBS-apply/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 complex), fp64 norms",
        "data": "synthetic",
        "config": {"workload": desc, "instances": len(sizes), "cells": cells,
                   "sizes": {str(n): sizes.count(n) for n in sorted(set(sizes))}},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "CBS sweep: k_col + k_row_sweep (fused inverse/forward rows) over the ragged batch",
            "sweeps_per_chain": chain,
            "algorithmic_bytes_per_sweep": BYTES_PER_CELL * cells,
            "event_ms_per_sweep": ev_ms,
        },
    }
    if not args.no_solve:
        line["time_to_1e-6"] = time_to_solution(probs, k2, sizes, k0sq, s)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(probs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
