"""Benchmark of the FS2D HLF hot path on one MI355X.

Headline (the timed region): the N=5 grid workload -- n = 25 qubits, every
nearest-neighbour edge, diagonal Bernoulli(0.5), seeds 0..7.  One step runs,
for each of the 8 instances, pack -> factor -> materialise all 2^r solutions as
uint32 words in HBM (2^23 .. 2^25 per instance).  Inputs are resident in HBM
before timing starts; outputs are preallocated.  `value` is solutions written
per second over the whole step.

Secondary measurements (outside the headline timed region, reported under
"modes"): reduce mode on the N=6, p=0.5 instances (seeds 0..3, every solution
hashed, 2^29 .. 2^32 each) and sampling at n = 1024.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Full-rate 32-bit VALU lane operations per second: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU instructions per solution in the full-tile loop of the reduce kernel
# (read from its gfx950 assembly): 2 XOR for z, 17 for mix13, 1 add.
REDUCE_VALU_OPS_PER_SOLUTION = 20
METRIC = "solutions enumerated/s (G/s) + % HBM/VALU roofline; batched instances/s, p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-modes", action="store_true", help="skip the secondary measurements")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   "the multi-GPU sharding is described in DESIGN.md"}))
        sys.exit(2)

    import numpy as np
    import torch

    from hlf_inputs import CONFIG2_SEEDS, CONFIG3_SEEDS, grid_instance
    from paper_2103_00693_amd import hlf

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    dev = torch.device("cuda", 0)

    # ---------------- headline workload: N=5 grid, 8 seeds ----------------
    n = 25
    insts = []
    with torch.cuda.stream(stream):
        for s in CONFIG2_SEEDS:
            A = torch.from_numpy(grid_instance(5, seed=s)).to(dev)
            rows = torch.empty((n, 1), dtype=torch.int64, device=dev)
            st = torch.empty(1, dtype=torch.int32, device=dev)
            F = hlf.Factors(n, device=dev, kernel=True)
            hlf.pack_dense(A, rows, st, stream=stream)
            hlf.factor(rows, n, F, stream=stream)
            insts.append({"seed": s, "A": A, "rows": rows, "st": st, "F": F})
    stream.synchronize()
    for it in insts:
        it["F"].check()
        it["r"] = int(it["F"].rank.item())
        it["count"] = 1 << it["r"]
        it["out"] = torch.empty(it["count"], dtype=torch.int32, device=dev)
    solutions_per_step = sum(it["count"] for it in insts)
    bytes_per_step = 4 * solutions_per_step

    def step(events=None):
        for k, it in enumerate(insts):
            hlf.pack_dense(it["A"], it["rows"], it["st"], stream=stream)
            hlf.factor(it["rows"], n, it["F"], stream=stream)
            if events is not None:
                events[k][0].record(stream)
            hlf.enumerate_solutions(it["F"], 0, it["count"], 32, out=it["out"], stream=stream)
            if events is not None:
                events[k][1].record(stream)

    for _ in range(args.warmup):
        step()
    stream.synchronize()

    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
           for _ in insts] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    stream.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for it in insts:
        it["F"].check()

    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = solutions_per_step * args.steps / elapsed / 1e9
    enum_ms = [ev[k][j][0].elapsed_time(ev[k][j][1]) for k in range(args.steps) for j in range(len(insts))]
    enum_bytes = [4 * it["count"] for _ in range(args.steps) for it in insts]
    achieved_gbs = sum(enum_bytes) / (sum(enum_ms) * 1e-3) / 1e9

    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G solutions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "N=5 grid (n=25), all edges, diagonal Bernoulli(0.5), seeds 0-7: "
                        "pack + factor + materialise all 2^r solutions as uint32 per seed",
            "instances": len(insts),
            "ranks": [it["r"] for it in insts],
            "solutions_per_step": solutions_per_step,
            "bytes_written_per_step": bytes_per_step,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "enum_tile_kernel<uint32_t>",
            "achieved": round(achieved_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
            "avg_launch_us": round(1e3 * sum(enum_ms) / len(enum_ms), 3),
            "algorithmic_bytes_per_launch": sum(enum_bytes) // len(enum_bytes),
        },
        "context": {"fpga_solutions_per_s": 1.0e8,
                    "fpga": "Kintex-7 XC7K410T at 100 MHz, one solution per clock (paper, Section 4)"},
    }

    # ---------------- secondary measurements ----------------
    if not args.no_modes:
        modes = {}
        # reduce mode, N=6 p=0.5 seeds 0..3, every solution hashed
        red = []
        with torch.cuda.stream(stream):
            for s in CONFIG3_SEEDS:
                A = torch.from_numpy(grid_instance(6, p=0.5, seed=s)).to(dev)
                rows, st = hlf.pack_dense(A, stream=stream)
                F = hlf.factor(rows, 36, stream=stream)
                red.append(F)
        stream.synchronize()
        ranks = []
        outs = []
        for F in red:
            F.check()
            ranks.append(int(F.rank.item()))
            outs.append((torch.zeros(36, dtype=torch.int64, device=dev),
                         torch.zeros(1, dtype=torch.int64, device=dev),
                         torch.zeros(1, dtype=torch.int64, device=dev)))
        for F, r, o in zip(red, ranks, outs):  # warm-up
            hlf.enumerate_reduce(F, 0, 1 << r, counts=o[0], hash_out=o[1], xorfold=o[2], stream=stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for F, r, o in zip(red, ranks, outs):
            hlf.enumerate_reduce(F, 0, 1 << r, counts=o[0], hash_out=o[1], xorfold=o[2], stream=stream)
        e1.record(stream)
        stream.synchronize()
        red_s = e0.elapsed_time(e1) * 1e-3
        red_sol = sum(1 << r for r in ranks)
        rate = red_sol / red_s
        ops = rate * REDUCE_VALU_OPS_PER_SOLUTION / 1e12
        modes["reduce"] = {
            "workload": "N=6 grid (n=36), edges p=0.5, seeds 0-3: counts + hash + xorfold over all 2^r",
            "ranks": ranks,
            "value": round(rate / 1e9, 2),
            "unit": "G solutions/s",
            "roofline": {"bound": "alu", "kernel": "reduce_tile_kernel<8>",
                         "achieved": round(ops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                         "unit": "T VALU instr-lane-ops/s", "frac": round(ops / VALU_PEAK_TOPS, 4),
                         "valu_ops_per_solution": REDUCE_VALU_OPS_PER_SOLUTION},
        }
        # sampling at n = 1024
        A = torch.from_numpy(grid_instance(32, p=0.5, seed=17)).to(dev)
        rows, st = hlf.pack_dense(A, stream=stream)
        F = hlf.factor(rows, 1024, stream=stream)
        out = torch.empty((65536, 16), dtype=torch.int64, device=dev)
        hlf.sample(F, 1, 65536, out=out, stream=stream)
        stream.synchronize()
        F.check()
        e0.record(stream)
        reps = 5
        for k in range(reps):
            hlf.sample(F, k, 65536, out=out, stream=stream)
        e1.record(stream)
        stream.synchronize()
        smp_s = e0.elapsed_time(e1) * 1e-3 / reps
        e0.record(stream)
        for k in range(reps):
            hlf.factor(rows, 1024, F, stream=stream)
        e1.record(stream)
        stream.synchronize()
        fac_s = e0.elapsed_time(e1) * 1e-3 / reps
        modes["sample"] = {"workload": "N=32 grid (n=1024), p=0.5: 65536 uniform samples",
                           "rank": int(F.rank.item()), "samples_per_s": round(65536 / smp_s, 1),
                           "ms_per_65536": round(smp_s * 1e3, 4),
                           "factor_ms_n1024": round(fac_s * 1e3, 4)}
        result["modes"] = modes

    # ---------------- CPU baseline: the oracle, on this host ----------------
    if not args.no_cpu_baseline:
        from oracle import c_oracle, hlf_oracle

        oracle_F = [hlf_oracle.factor(grid_instance(5, seed=s)) for s in CONFIG2_SEEDS]
        chunk = 1 << 24
        done = 0
        t_start = time.perf_counter()
        passes = 0
        while True:
            for Fo in oracle_F:
                total = 1 << Fo["rank"]
                for b in range(0, total, chunk):
                    c_oracle.enumerate_range(Fo, b, min(chunk, total - b))
                done += total
            passes += 1
            if time.perf_counter() - t_start >= args.cpu_seconds:
                break
        cpu_s = time.perf_counter() - t_start
        result["cpu_baseline"] = {
            "value": round(done / cpu_s / 1e9, 4),
            "unit": "G solutions/s",
            "cores": c_oracle.threads(),
            "kind": "oracle",
            "sample": f"{passes} full pass(es) of the headline workload (all 2^r solutions of the 8 N=5 "
                      f"seeds) through the plain C per-index oracle, {done} solutions in {cpu_s:.1f} s",
        }

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
