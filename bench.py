"""Benchmark of the FS2D HLF hot path on one MI355X.

Headline (the timed region): the N=5 grid workload -- n = 25 qubits, every
nearest-neighbour edge, diagonal Bernoulli(0.5), seeds 0..7.  One step runs,
for each of the 8 instances, pack -> factor -> materialise all 2^r solutions as
uint32 words in HBM (2^23 .. 2^25 per instance): one launch per step that
materialises this step's instances and runs stage 1 for the next step.  Inputs are resident in HBM
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
FP4_MFMA_PEAK_TFLOPS = 10100.0  # dense fp4 (E2M1) matrix-core peak
# Full-rate 32-bit VALU lane operations per second: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU instructions per solution in the full-tile loop of the reduce kernel
# (read from its gfx950 assembly): 2 XOR to form the input of the mix13 tail
# (its GF(2)-linear first step is applied per lane and per tile), 14 for the
# rest of mix13 (2 x [3 multiplies + add3], 2 x [64-bit shift + 2 XOR]), 1 add.
REDUCE_VALU_OPS_PER_SOLUTION = 17
# Measured: rocprofv3 --pmc SQ_INSTS_VALU over the four timed reduce launches
# (ranks 30, 29, 32, 32): 3,032,022,924 wave instructions x 64 lanes /
# 10,200,547,328 solutions = 19.02 lane operations per solution (the full-tile
# loop plus per-tile and per-wave work).  The roofline uses it while the
# kernel's sources are the measured ones, else the loop count above.
REDUCE_VALU_MEASURED = {"src_sha256_16": "322899540ce79507", "ops_per_solution": 19.02}
REDUCE_VALU_SOURCES = ("paper_2103_00693_amd/csrc/stage2.h", "paper_2103_00693_amd/csrc/enumerate.hip",
                       "paper_2103_00693_amd/csrc/hlf_device.h")
# Measured: rocprofv3 --pmc SQ_INSTS_VALU (a pass of four counters) over the
# sample launches of the sample mode (65536 samples of the N=32 grid, p=0.5,
# seed 17; the basis has at most 5 set bits per row and column, so every
# workgroup takes the sparse path): 3,302,592 wave instructions x 64 lanes /
# 65536 samples = 3225.2 lane operations per sample.  Used while the sampler's
# sources are the measured ones.
SAMPLE_VALU_MEASURED = {"src_sha256_16": "4c261b6ea9be0de1", "ops_per_sample": 3225.2}
SAMPLE_VALU_SOURCES = ("paper_2103_00693_amd/csrc/sample.hip", "paper_2103_00693_amd/csrc/hlf_device.h")
# HBM traffic of one batch_enum_kernel<uint32_t, overlap> launch of the headline step,
# from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch), each scaled by what the same counter reads for a plain 256 MiB
# device copy (WRITE_SIZE 262144 KiB -> x1.0, FETCH_SIZE 131085 KiB -> x2.0).
# Valid only for the kernel sources it was taken on (sha256 prefix below).
ENUM_TRAFFIC = {"src_sha256_16": "22ef894c3eb80077", "fetch_kib_raw": 69.2, "fetch_scale": 2.0,
                "write_kib_raw": 688822.9, "write_scale": 1.0}
ENUM_TRAFFIC_SOURCES = ("paper_2103_00693_amd/csrc/stage2.h", "paper_2103_00693_amd/csrc/batch.hip",
                        "paper_2103_00693_amd/csrc/factor_wave.h",
                        "paper_2103_00693_amd/csrc/hlf_device.h")
# Streams that take the headline steps in turn (launches in flight).
HEADLINE_STREAMS = 2
METRIC = "solutions enumerated/s (G/s) + % HBM/VALU roofline; batched instances/s, p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-modes", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--only", default="",
                    help="comma-separated secondary modes to run (reduce, sample, tiny, steady, batch, "
                         "general, circuit, verify, serve); default all")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (for HBM counter scaling)")
    return ap.parse_args()


def _sources_sha256_16(paths):
    import hashlib

    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def reduce_valu_ops_per_solution():
    """(VALU lane operations per solution, how it was obtained) for the reduce
    roofline: the counter measurement while the sources match, else the
    count of the full-tile loop."""
    if _sources_sha256_16(REDUCE_VALU_SOURCES) == REDUCE_VALU_MEASURED["src_sha256_16"]:
        return REDUCE_VALU_MEASURED["ops_per_solution"], "SQ_INSTS_VALU x 64 / solutions (rocprofv3)"
    return REDUCE_VALU_OPS_PER_SOLUTION, "full-tile loop instruction count (assembly)"


def sample_valu_ops_per_sample():
    """VALU lane operations per sample of the sample mode's workload (sparse
    path), or None if the sampler's sources changed since the counters were
    taken."""
    if _sources_sha256_16(SAMPLE_VALU_SOURCES) == SAMPLE_VALU_MEASURED["src_sha256_16"]:
        return SAMPLE_VALU_MEASURED["ops_per_sample"]
    return None


def enum_traffic_bytes():
    """Measured HBM bytes per launch of the headline kernel, or None if its
    sources changed since the counters were taken."""
    if _sources_sha256_16(ENUM_TRAFFIC_SOURCES) != ENUM_TRAFFIC["src_sha256_16"]:
        return None
    t = ENUM_TRAFFIC
    return int(1024 * (t["fetch_kib_raw"] * t["fetch_scale"] + t["write_kib_raw"] * t["write_scale"]))


def copy_calibration():
    """A plain device-to-device copy of 256 MiB, three times: the reference
    kernel whose FETCH_SIZE / WRITE_SIZE counters scale the ones of the
    enumerate kernel."""
    import torch

    src = torch.ones(1 << 25, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {src.numel() * 8} bytes x3", flush=True)



class _Pipeline:
    pass


def headline_pipeline(hlf, torch, dev, stream, n_streams=HEADLINE_STREAMS):
    """The headline step and its buffers.

    Step k is ONE launch (hlf_batch_enumerate_overlap): it materialises all
    2^r solutions of the 8 N=5 instances from record set k % 2S and, in extra
    workgroups of the same launch, runs stage 1 (pack + validate + factor) of
    the 8 instances into record set (k+S) % 2S for step k+S, S = n_streams.
    Steps go to the S streams in turn, each with its own output set, so S
    launches are in flight and each one's start-up and drain overlap the
    others'; a launch depends only on the launch S steps back, on its own
    stream.  Record sets 0..S-1 are factored here, before the first step.
    """
    from hlf_inputs import CONFIG2_SEEDS, grid_instance

    P = _Pipeline()
    n = 25
    P.n_streams = n_streams
    P.mats = [grid_instance(5, seed=s) for s in CONFIG2_SEEDS]
    P.Bs = [hlf.Batch([n] * len(P.mats)) for _ in range(2 * n_streams)]
    P.A = P.Bs[0].dense_input(P.mats, device=dev)
    P.streams = [stream] + [torch.cuda.Stream() for _ in range(n_streams - 1)]
    for Bk in P.Bs[:n_streams]:
        Bk.factor_dense(P.A, stream=stream)
    stream.synchronize()
    if not all(st == hlf.HLF_OK for Bk in P.Bs[:n_streams] for st in Bk.statuses()):
        raise RuntimeError("factor failed")
    P.ranks = [int(r) for r in P.Bs[0].ranks()]
    P.counts = [1 << r for r in P.ranks]
    P.out_sets = [[torch.empty(c, dtype=torch.int32, device=dev) for c in P.counts] for _ in P.streams]
    inst = list(range(len(P.mats)))
    zeros = [0] * len(P.mats)

    def step(k):
        P.Bs[k % (2 * n_streams)].enumerate_overlap(inst, zeros, P.counts, P.out_sets[k % n_streams], 32,
                                                    P.Bs[(k + n_streams) % (2 * n_streams)], P.A,
                                                    stream=P.streams[k % n_streams])

    P.step = step
    return P


def tiny_mode(hlf, torch, stream, dev):
    """N=4 grid (n = 16), all edges, seed 0: pack + factor + materialise all
    2^r solutions as uint16 -- a latency measurement (a single launch chain)."""
    from hlf_inputs import grid_instance

    A = torch.from_numpy(grid_instance(4, seed=0)).to(dev)
    rows = torch.empty((16, 1), dtype=torch.int64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    F = hlf.Factors(16, device=dev)
    hlf.pack_dense(A, rows, st, stream=stream)
    hlf.factor(rows, 16, F, stream=stream)
    stream.synchronize()
    r = int(F.rank.item())
    out = torch.empty(1 << r, dtype=torch.int16, device=dev)
    reps = 50
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ms = []
    for k in range(reps + 5):
        e0.record(stream)
        hlf.pack_dense(A, rows, st, stream=stream)
        hlf.factor(rows, 16, F, stream=stream)
        hlf.enumerate_solutions(F, 0, 1 << r, 16, out=out, stream=stream)
        e1.record(stream)
        stream.synchronize()
        if k >= 5:
            ms.append(e0.elapsed_time(e1))
    F.check()
    med = sorted(ms)[len(ms) // 2]
    # The same work as ONE launch: hlf_solve_dense (every workgroup packs and
    # factors the instance, then materialises its own tiles).
    F1 = hlf.Factors(16, device=dev)
    out1 = torch.empty(1 << r, dtype=torch.int16, device=dev)
    fused = []
    for k in range(reps + 5):
        e0.record(stream)
        hlf.solve_dense(A, F1, 0, 1 << r, 16, out=out1, stream=stream)
        e1.record(stream)
        stream.synchronize()
        if k >= 5:
            fused.append(e0.elapsed_time(e1))
    if not torch.equal(out1, out) or int(F1.status.item()) != hlf.HLF_OK:
        raise RuntimeError("one-launch solve differs from the launch chain")
    fmed = sorted(fused)[len(fused) // 2]
    return {"workload": "N=4 grid (n=16), all edges, seed 0: pack + factor + materialise 2^r uint16",
            "rank": r, "median_us": round(med * 1e3, 2),
            "solutions_per_s_G": round((1 << r) / (med * 1e-3) / 1e9, 3),
            "launches": "pack, factor, enumerate",
            "one_launch_median_us": round(fmed * 1e3, 2),
            "one_launch": "hlf_solve_dense"}


def steady_mode(hlf, torch, stream, dev):
    """Steady-state window of the materialise kernel: the full-rank n = 36
    instance (N=6, all edges, b = 1^36, r = 36), indices [0, 2^30) as uint64
    words (8 GiB written by one launch)."""
    from hlf_inputs import grid_instance

    A = torch.from_numpy(grid_instance(6, b="1" * 36)).to(dev)
    rows, st = hlf.pack_dense(A, stream=stream)
    F = hlf.factor(rows, 36, stream=stream)
    count = 1 << 30
    out = torch.empty(count, dtype=torch.int64, device=dev)
    hlf.enumerate_solutions(F, 0, count, 64, out=out, stream=stream)
    stream.synchronize()
    F.check()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record(stream)
    for _ in range(reps):
        hlf.enumerate_solutions(F, 0, count, 64, out=out, stream=stream)
    e1.record(stream)
    stream.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    del out
    return {"workload": "N=6 grid (n=36), all edges, b=1^36 (r=36): solutions [0, 2^30) as uint64",
            "kernel": "enum_tile_kernel<uint64_t>", "bytes": 8 * count,
            "achieved_GBs": round(8 * count / s / 1e9, 1), "frac_of_8TBs": round(8 * count / s / 8e12, 4),
            "solutions_per_s_G": round(count / s / 1e9, 1)}


def _queue_behind_spin(torch, stream, reps):
    """Keep the stream busy (torch's spin kernel, about 60 us per call plus
    0.5 ms) while the host enqueues the timed calls, so that they run back
    to back and host launch overhead stays out of the device interval."""
    with torch.cuda.stream(stream):
        torch.cuda._sleep(int(2.4e9 * (60e-6 * reps + 0.5e-3)))


def _timed(torch, stream, fn, reps):
    """Device seconds per call of fn, the calls queued back to back."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    stream.synchronize()
    _queue_behind_spin(torch, stream, reps)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def general_mode(hlf, torch, stream, dev):
    """Arbitrary symmetric A (Section 5): (a) a dense random graph with
    self-loops at n = 1024 (density 0.5): stage 1 and 65536 uniform samples;
    (b) a low-rank graph at n = 1024 (A = M^T M, M 24 x 1024): all 2^r
    solutions as 16-word vectors, in counter order (the paper's circuit order)
    and in Gray order."""
    from hlf_inputs import low_rank_symmetric, random_symmetric

    out = {}
    A = torch.from_numpy(random_symmetric(1024, seed=1, density=0.5)).to(dev)
    rows = torch.empty((1024, 16), dtype=torch.int64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    F = hlf.Factors(1024, device=dev)
    hlf.pack_dense(A, rows, st, stream=stream)
    hlf.factor(rows, 1024, F, stream=stream)
    stream.synchronize()
    F.check()
    smp = torch.empty((65536, 16), dtype=torch.int64, device=dev)
    out["dense"] = {
        "workload": "random symmetric 0/1 matrix, n=1024, density 0.5 (self-loops included)",
        "rank": int(F.rank.item()),
        "pack_ms": round(_timed(torch, stream, lambda: hlf.pack_dense(A, rows, st, stream=stream), 5) * 1e3, 4),
        "factor_ms": round(_timed(torch, stream, lambda: hlf.factor(rows, 1024, F, stream=stream), 5) * 1e3, 4),
        "ms_per_65536_samples": round(_timed(torch, stream, lambda: hlf.sample(F, 3, 65536, out=smp, stream=stream), 5) * 1e3, 4),
    }
    # dense basis (up to hundreds of set bits per row): the matrix-core path
    rk = out["dense"]["rank"]
    fl = 2.0 * 65536 * rk * 1024 / (out["dense"]["ms_per_65536_samples"] * 1e-3) / 1e12
    out["dense"]["sample_roofline"] = {"bound": "mfma", "kernel": "sample_mfma_kernel (fp4 E2M1 32x32x64, fp32 sums)",
                                       "achieved": round(fl, 1), "peak": FP4_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                       "frac": round(fl / FP4_MFMA_PEAK_TFLOPS, 4)}
    del smp
    A = torch.from_numpy(low_rank_symmetric(1024, 24, seed=2)).to(dev)
    hlf.pack_dense(A, rows, st, stream=stream)
    hlf.factor(rows, 1024, F, stream=stream)
    stream.synchronize()
    F.check()
    r = int(F.rank.item())
    count = 1 << r
    buf = torch.empty((count, 16), dtype=torch.int64, device=dev)
    bytes_ = count * 128
    res = {"workload": "low-rank symmetric A = M^T M mod 2, M uniform 24 x 1024: all 2^r solutions as 16 uint64 words",
           "rank": r, "bytes": bytes_, "kernel": "enum_wide_tile_kernel<16>"}
    for order in ("counter", "gray"):
        sec = _timed(torch, stream,
                     lambda: hlf.enumerate_solutions(F, 0, count, 1024, out=buf, stream=stream, order=order), 3)
        res[order] = {"ms": round(sec * 1e3, 3), "achieved_GBs": round(bytes_ / sec / 1e9, 1),
                      "frac_of_8TBs": round(bytes_ / sec / 8e12, 4),
                      "solutions_per_s_G": round(count / sec / 1e9, 3)}
    F.check()
    out["low_rank"] = res
    del buf
    return out


def circuit_mode(hlf, torch, stream, dev):
    """The paper's circuit evaluated literally (Section 2, Eqs. (1)-(2),
    Fig. 1(c)) in the FPGA's counter order (Section 4): (a) the N=5 workload,
    all 2^r solutions of each of the 8 seeds as uint32, one launch per seed,
    beside the Gray-order materialise of the same instances with the same
    launches, on one stream and on two streams in turn; (b) a 32 x 32 grid subgraph with 10 edges and 4 coloured
    vertices (n = 1024, r = 24): all 2^24 solutions as 16-word vectors."""
    from hlf_inputs import CONFIG2_SEEDS, grid_instance, sparse_grid_instance

    out = {}
    Fs, rows = [], []
    for s in CONFIG2_SEEDS:
        A = torch.from_numpy(grid_instance(5, seed=s)).to(dev)
        r_, _ = hlf.pack_dense(A, stream=stream)
        Fs.append(hlf.factor(r_, 25, stream=stream))
        rows.append(r_)
    stream.synchronize()
    ranks = [int(F.rank.item()) for F in Fs]
    outs = [torch.empty(1 << r, dtype=torch.int32, device=dev) for r in ranks]

    def circ():
        for F, r_, o, rk in zip(Fs, rows, outs, ranks):
            hlf.enumerate_circuit(F, r_, 5, 0, 1 << rk, 32, out=o, stream=stream)

    def gray():
        for F, o, rk in zip(Fs, outs, ranks):
            hlf.enumerate_solutions(F, 0, 1 << rk, 32, out=o, stream=stream)

    # The same launches with the seeds dealt to two streams in turn, so that
    # one launch's start-up and drain overlap the other's (the headline's
    # pattern).
    s2 = torch.cuda.Stream(device=dev)

    def circ2():
        for k, (F, r_, o, rk) in enumerate(zip(Fs, rows, outs, ranks)):
            hlf.enumerate_circuit(F, r_, 5, 0, 1 << rk, 32, out=o, stream=stream if k % 2 == 0 else s2)

    def gray2():
        for k, (F, o, rk) in enumerate(zip(Fs, outs, ranks)):
            hlf.enumerate_solutions(F, 0, 1 << rk, 32, out=o, stream=stream if k % 2 == 0 else s2)

    def timed_two(fn, reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        joined = torch.cuda.Event()
        fn()
        torch.cuda.synchronize()
        _queue_behind_spin(torch, stream, reps * 8)
        e0.record(stream)
        s2.wait_event(e0)
        for _ in range(reps):
            fn()
        joined.record(s2)
        stream.wait_event(joined)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    nbytes = 4 * sum(1 << r for r in ranks)
    res = {"workload": "N=5 grid (n=25), all edges, seeds 0-7: all 2^r solutions as uint32, one launch per seed",
           "ranks": ranks, "bytes": nbytes, "kernel": "circuit_tile_kernel<uint32_t>"}
    for name, fn, timer in (("circuit", circ, lambda f: _timed(torch, stream, f, 10)),
                            ("gray_tile_algebra", gray, lambda f: _timed(torch, stream, f, 10)),
                            ("circuit_two_streams", circ2, lambda f: timed_two(f, 10)),
                            ("gray_tile_algebra_two_streams", gray2, lambda f: timed_two(f, 10))):
        sec = timer(fn)
        res[name] = {"us": round(sec * 1e6, 2), "achieved_GBs": round(nbytes / sec / 1e9, 1),
                     "frac_of_8TBs": round(nbytes / sec / 8e12, 4),
                     "solutions_per_s_G": round(nbytes / 4 / sec / 1e9, 2)}
    for F in Fs:
        F.check()
    out["n25"] = res
    del outs
    A = sparse_grid_instance(32, 10, 0, 4)
    Ad = torch.from_numpy(A).to(dev)
    r_, _ = hlf.pack_dense(Ad, stream=stream)
    F = hlf.factor(r_, 1024, stream=stream)
    stream.synchronize()
    F.check()
    r = int(F.rank.item())
    count = 1 << r
    buf = torch.empty((count, 16), dtype=torch.int64, device=dev)
    nbytes = count * 128
    res = {"workload": "32x32 grid subgraph, 10 edges, 4 coloured vertices (n=1024): all 2^r solutions "
                       "as 16 uint64 words", "rank": r, "bytes": nbytes, "kernel": "circuit_wide_kernel<16>"}
    for name, fn in (("circuit", lambda: hlf.enumerate_circuit(F, r_, 32, 0, count, 1024, out=buf, stream=stream)),
                     ("counter_tile_algebra", lambda: hlf.enumerate_solutions(F, 0, count, 1024, out=buf,
                                                                              stream=stream, order="counter"))):
        sec = _timed(torch, stream, fn, 3)
        res[name] = {"ms": round(sec * 1e3, 3), "achieved_GBs": round(nbytes / sec / 1e9, 1),
                     "frac_of_8TBs": round(nbytes / sec / 8e12, 4),
                     "solutions_per_s_G": round(count / sec / 1e9, 3)}
    F.check()
    out["n1024"] = res
    del buf
    return out


def verify_mode(hlf, torch, stream, dev):
    """Verification data at n = 1024 (N=32 grid, p=0.5): membership of 2^20
    strings (ideal probabilities for a cross-entropy benchmark), the linear
    XEB of exact samples and of uniform strings, and the pair statistics."""
    from hlf_inputs import grid_instance

    A = torch.from_numpy(grid_instance(32, p=0.5, seed=17)).to(dev)
    rows, st = hlf.pack_dense(A, stream=stream)
    F = hlf.factor(rows, 1024, stream=stream)
    stream.synchronize()
    F.check()
    n, r = 1024, int(F.rank.item())
    num = 1 << 20
    z = hlf.sample(F, 11, num, stream=stream)
    mem = torch.empty(num, dtype=torch.uint8, device=dev)
    t_mem = _timed(torch, stream, lambda: hlf.membership(F, z, out=mem, stream=stream), 5)
    # linear XEB estimate 2^(n-r) * (fraction of members) - 1 (report arithmetic only)
    xeb_exact = (2.0 ** (n - r)) * (int(mem.sum().item()) / num) - 1.0
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    u = torch.randint(-(1 << 62), 1 << 62, (num, 16), dtype=torch.int64, device=dev, generator=g)
    hlf.membership(F, u, out=mem, stream=stream)
    stream.synchronize()
    uniform_members = int(mem.sum().item())
    q = torch.empty((n, n), dtype=torch.uint8, device=dev)
    t_pair = _timed(torch, stream, lambda: hlf.pair_stats(F, rows, out=q, stream=stream), 5)
    hist = torch.bincount(q.flatten().to(torch.int64), minlength=3).cpu().tolist()
    return {"workload": "N=32 grid (n=1024), p=0.5: membership of 2^20 strings, pair statistics",
            "rank": r, "membership_strings_per_s": round(num / t_mem, 1),
            "membership_ms_per_2^20": round(t_mem * 1e3, 4),
            "kernel_vectors": n - r,
            "xeb_exact_samples": xeb_exact, "xeb_exact_expected": 2.0 ** (n - r) - 1.0,
            "uniform_strings_that_are_solutions": uniform_members,
            "pair_stats_ms": round(t_pair * 1e3, 4),
            "pair_quarters_histogram_0_1_2": hist[:3]}


def batch_mode(hlf, torch, stream, dev):
    """4096 instances (N ~ U{3..12}, p ~ U{0.3, 0.5, 1.0}): factor every
    instance and reduce every instance with r <= 28.  Batched: the tuned
    persistent kernel replayed from a HIP graph.  Plain: one pack + factor
    launch per instance, then one reduce per small-rank instance."""
    from hlf_inputs import batch_instances

    max_rank = 28
    insts = batch_instances(4096, master_seed=0)
    mats = [a for (_, _, _, a) in insts]
    B = hlf.Batch([m.shape[0] for m in mats])
    A = B.dense_input(mats, device=dev)
    params, tune_ms = B.tune(A, max_rank, stream=stream)
    B.graph_capture(A, max_rank, params)
    B.graph_launch(stream=stream)
    stream.synchronize()
    reps = 5
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        B.graph_launch(stream=stream)
    e1.record(stream)
    stream.synchronize()
    batched_s = e0.elapsed_time(e1) * 1e-3 / reps
    ranks = [int(r) for r in B.ranks()]
    counts_b, hashes_b = B.reduce_results()
    sols = sum(1 << r for r in ranks if r <= max_rank)

    # Plain per-instance launches, same outputs.  Inputs are uploaded and the
    # records allocated before timing; the timed parts are the per-instance
    # pack + factor launches and the per-instance reduce launches (HIP events
    # on the stream, as for the batched run); between them one copy brings
    # every rank to the host (host time, reported separately).
    Ads = [torch.from_numpy(m).to(dev) for m in mats]
    rows_l = [torch.empty((m.shape[0], hlf.words_for(m.shape[0])), dtype=torch.int64, device=dev)
              for m in mats]
    pst = torch.empty(1, dtype=torch.int32, device=dev)
    Fs = [hlf.Factors(m.shape[0], device=dev, kernel=False) for m in mats]
    outs = {}
    for i, m in enumerate(mats):
        n = m.shape[0]
        outs[i] = (torch.empty(n, dtype=torch.int64, device=dev), torch.empty(1, dtype=torch.int64, device=dev))
    e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    with torch.cuda.stream(stream):
        rank_view = torch.empty(len(mats), dtype=torch.int32, device=dev)
        stream.synchronize()
        e0.record(stream)
        for i, m in enumerate(mats):
            hlf.pack_dense(Ads[i], rows_l[i], pst, stream=stream)
            hlf.factor(rows_l[i], m.shape[0], Fs[i], stream=stream)
        e1.record(stream)
        t0 = time.perf_counter()
        torch.stack([F.rank.view(()) for F in Fs], out=rank_view)
        rp = [int(r) for r in rank_view.cpu().numpy()]
        t_ranks = time.perf_counter() - t0
        e2.record(stream)
        for i, F in enumerate(Fs):
            if rp[i] <= max_rank:
                c, h = outs[i]
                hlf.enumerate_reduce(F, 0, 1 << rp[i], counts=c, hash_out=h, want_xorfold=False,
                                     stream=stream)
        e3.record(stream)
        stream.synchronize()
    plain_s = (e0.elapsed_time(e1) + e2.elapsed_time(e3)) * 1e-3
    reduced = [i for i in range(len(mats)) if rp[i] <= max_rank]
    same = rp == ranks and all(
        int(hlf.as_uint64(outs[i][1])[0]) == hashes_b[i] and
        (hlf.as_uint64(outs[i][0]) == counts_b[i]).all() for i in reduced)
    B.close()
    return {
        "workload": "4096 grid instances, N ~ U{3..12}, p ~ U{0.3,0.5,1.0}, diagonal Bernoulli(0.5): "
                    "factor all, reduce (counts + hash) every instance with r <= 28",
        "reduced_instances": len(reduced),
        "solutions": sols,
        "batched": {"instances_per_s": round(4096 / batched_s, 1), "ms": round(batched_s * 1e3, 3),
                    "solutions_per_s_G": round(sols / batched_s / 1e9, 2),
                    "params": {"chunk_log2": params.chunk_log2, "waves_per_cu": params.waves_per_cu},
                    "launch": "hipGraph replay of queue reset + one persistent kernel"},
        "plain": {"instances_per_s": round(4096 / plain_s, 1), "ms": round(plain_s * 1e3, 3),
                  "rank_readback_ms": round(t_ranks * 1e3, 3),
                  "launch": "pack + factor per instance, then reduce per small-rank instance; inputs resident "
                            "and records preallocated; HIP events around the launches (the rank readback "
                            "between them is not included)"},
        "speedup": round(plain_s / batched_s, 2),
        "identical_outputs": bool(same),
    }


def serve_mode(torch):
    """Poisson arrivals of requests with N ~ U{4..32} (n = 16..1024), p = 0.5:
    stage 1 + 65536 uniform samples, or the full enumeration when r <= 24,
    through the native server (8 slots).  Saturated throughput first (every
    request present at t = 0), then arrival rates of 0.5, 0.8 and 0.95 of it,
    2000 requests per point; latency = arrival -> result in pinned host
    memory.  Results are released as they arrive."""
    from hlf_inputs import serve_requests
    from paper_2103_00693_amd.serve import Request, Server, percentile

    count = 2000

    def reqs(rate, seed, k=count):
        return [Request(rid=i, A=q["A"], seed=q["seed"], arrival=q["t"])
                for i, q in enumerate(serve_requests(k, rate, master_seed=seed))]

    srv = Server(slots=8, hbm_budget=1 << 30, host_budget=1 << 30)
    srv.run(reqs(1000.0, 99, 300), realtime=False, keep_data=False)  # warm-up
    sat_reqs = reqs(1000.0, 1)
    t0 = time.perf_counter()
    res = srv.run(sat_reqs, realtime=False, keep_data=False)
    sat = count / (time.perf_counter() - t0)
    out = {"workload": "requests with N ~ U{4..32} (n = 16..1024), p = 0.5, diagonal Bernoulli(0.5): "
                       "stage 1 + 65536 uniform samples, or all 2^r solutions when r <= 24",
           "server": "native (C++ worker thread, 8 HIP streams, 1 GiB device arena, pinned result arena)",
           "slots": 8, "requests_per_run": count,
           "saturated_requests_per_s": round(sat, 1),
           "kinds": {k: sum(1 for r in res if r.kind == k) for k in ("sample", "enumerate", "error")},
           "loads": []}
    # Result bytes handed to the host (pinned memory) in the saturated run:
    # every solution of an enumeration in 2-, 4- or 8-byte words (n <= 16, 32,
    # 64), 65536 samples of ceil(n/64) words otherwise.
    def result_bytes(r):
        if r.kind == "enumerate":
            return (1 << r.rank) * (2 if r.n <= 16 else 4 if r.n <= 32 else 8)
        return 65536 * 8 * ((r.n + 63) // 64) if r.kind == "sample" else 0
    rb = sum(result_bytes(r) for r in res)
    out["saturated_result_bytes"] = rb
    out["saturated_result_GB_per_s"] = round(rb * sat / count / 1e9, 2)
    for frac in (0.5, 0.8, 0.95):
        rq = reqs(frac * sat, 2)
        res = srv.run(rq, realtime=True, keep_data=False)
        lat = [r.latency * 1e3 for r in res]
        span = max(r.finished for r in res) - min(q.arrival for q in rq)
        out["loads"].append({"offered_fraction": frac, "offered_per_s": round(frac * sat, 1),
                             "served_per_s": round(count / span, 1),
                             "p50_ms": round(percentile(lat, 50), 3),
                             "p99_ms": round(percentile(lat, 99), 3)})
    # The host link's rate for such copies: 256 MiB device -> pinned host.
    src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    dst = torch.empty(1 << 28, dtype=torch.uint8, pin_memory=True)
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    out["d2h_pinned_GB_per_s"] = round(4 * (1 << 28) / (time.perf_counter() - t0) / 1e9, 2)
    del src, dst
    st = srv.stats()
    out["hbm_arena_bytes"] = st["hbm_bytes"]
    out["hbm_peak_bytes"] = st["hbm_peak_bytes"]
    out["cache_hits"] = st["cache_hits"]
    srv.close()
    return out


def mode_cpu_baselines(modes, seconds):
    """The oracle (plain C per-index definitions, Python stage 1) on this
    host's cores for the secondary workloads, each on a bounded sample."""
    import numpy as np

    from hlf_inputs import CONFIG3_SEEDS, batch_instances, grid_instance
    from oracle import c_oracle, hlf_oracle

    cores = c_oracle.threads()
    if "reduce" in modes:
        # the 16 random 2^20-index chunks per N=6 seed that the parity tests check
        done, t_all = 0, 0.0
        for s in CONFIG3_SEEDS:
            Fo = hlf_oracle.factor(grid_instance(6, p=0.5, seed=s))
            rng = np.random.default_rng(1000 + s)
            for _ in range(16):
                b = int(rng.integers(0, (1 << Fo["rank"]) - (1 << 20)))
                t0 = time.perf_counter()
                c_oracle.reduce_range(Fo, b, 1 << 20)
                t_all += time.perf_counter() - t0
                done += 1 << 20
        modes["reduce"]["cpu_baseline"] = {
            "value": round(done / t_all / 1e9, 4), "unit": "G solutions/s", "cores": cores, "kind": "oracle",
            "sample": f"16 chunks of 2^20 solutions per N=6 seed (64 chunks, {done} solutions) through the "
                      f"plain C per-index oracle (counts + hash + xorfold), {t_all:.2f} s"}
    if "sample" in modes:
        Fo = hlf_oracle.factor(grid_instance(32, p=0.5, seed=17))
        t0 = time.perf_counter()
        num = 0
        while time.perf_counter() - t0 < min(seconds, 3.0) or num == 0:
            c_oracle.sample(Fo, num, 65536)
            num += 65536
        t = time.perf_counter() - t0
        modes["sample"]["cpu_baseline"] = {
            "value": round(num / t, 1), "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{num} samples at n=1024 (r={Fo['rank']}) through the plain C per-sample oracle, {t:.2f} s"}
    if "batch" in modes:
        insts = batch_instances(4096, master_seed=0)
        t0 = time.perf_counter()
        k, sols = 0, 0
        while k < len(insts) and (time.perf_counter() - t0 < seconds or k == 0):
            Fo = hlf_oracle.factor(insts[k][3])
            if Fo["rank"] <= 28:
                c_oracle.reduce_range(Fo, 0, 1 << Fo["rank"])
                sols += 1 << Fo["rank"]
            k += 1
        t = time.perf_counter() - t0
        modes["batch"]["cpu_baseline"] = {
            "value": round(k / t, 2), "unit": "instances/s", "cores": cores, "kind": "oracle",
            "sample": f"the first {k} of the 4096 instances (stage 1 in the Python oracle, one thread; "
                      f"counts + hash of every solution of the r <= 28 ones, {sols} solutions, in the C "
                      f"oracle), {t:.1f} s"}


def _progress(msg):
    """One progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; across GPUs the "
                                   "index range [0, 2^r) would split into contiguous slices, "
                                   "materialised with no communication and reduced with one "
                                   "all-reduce"}))
        sys.exit(2)

    import numpy as np
    import torch

    from hlf_inputs import CONFIG2_SEEDS, CONFIG3_SEEDS, grid_instance
    from paper_2103_00693_amd import hlf

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    dev = torch.device("cuda", 0)

    # ---------------- headline workload: N=5 grid, 8 seeds ----------------
    P = headline_pipeline(hlf, torch, dev, stream)
    mats, Bs, A, streams, out_sets, step = P.mats, P.Bs, P.A, P.streams, P.out_sets, P.step
    n_streams, ranks, counts = P.n_streams, P.ranks, P.counts
    outs = out_sets[0]
    inst = list(range(len(mats)))
    zeros = [0] * len(mats)
    solutions_per_step = sum(counts)
    bytes_per_step = 4 * solutions_per_step

    warmup = max(n_streams, args.warmup)
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()

    # HIP events: ev0 on stream 0 before the first timed launch (the other
    # streams wait for it), ev1 on stream 0 after the other streams' last
    # launches have been joined, so ev0..ev1 covers every timed launch.
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    joins = [torch.cuda.Event() for _ in streams[1:]]
    t0 = time.perf_counter()
    ev0.record(streams[0])
    for st in streams[1:]:
        st.wait_event(ev0)
    for k in range(args.steps):
        step(warmup + k)
    for st, j in zip(streams[1:], joins):
        j.record(st)
        streams[0].wait_event(j)
    ev1.record(streams[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for Bk in Bs:
        if not all(st == hlf.HLF_OK for st in Bk.statuses()):
            raise RuntimeError("enumerate failed")
    for other in out_sets[1:]:
        for a, b in zip(out_sets[0], other):
            if not torch.equal(a, b):
                raise RuntimeError("the streams' outputs differ")

    # the same step as ONE launch (hlf_batch_solve), for comparison
    Bs[0].solve(A, inst, zeros, counts, outs, 32, stream=stream)
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        Bs[0].solve(A, inst, zeros, counts, outs, 32, stream=stream)
    e1.record(stream)
    stream.synchronize()
    fused_us = e0.elapsed_time(e1) * 1e3 / 5

    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = solutions_per_step * args.steps / elapsed / 1e9
    # average time per launch with n_streams in flight: the events' span / launches
    launch_ms = ev0.elapsed_time(ev1) / args.steps
    achieved_gbs = bytes_per_step / (launch_ms * 1e-3) / 1e9

    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G solutions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "N=5 grid (n=25), all edges, diagonal Bernoulli(0.5), seeds 0-7: "
                        "pack + factor + materialise all 2^r solutions as uint32 per seed",
            "instances": len(mats),
            "ranks": ranks,
            "solutions_per_step": solutions_per_step,
            "bytes_written_per_step": bytes_per_step,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "batch_enum_kernel<uint32_t, overlap> (materialise of the 8 instances + stage 1 of the next step, one launch)",
            "achieved": round(achieved_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
            "traffic": enum_traffic_bytes(),
            "launches_in_flight": n_streams,
            "launch_interval_us": round(1e3 * launch_ms, 3),
            "algorithmic_bytes_per_launch": bytes_per_step,
            "fused_one_launch_step_us": round(fused_us, 2),
        },
        "context": {"fpga_solutions_per_s": 1.0e8,
                    "fpga": "Kintex-7 XC7K410T at 100 MHz, one solution per clock (paper, Section 4)"},
    }

    # ---------------- secondary measurements ----------------
    _progress("headline done")
    if not args.no_modes:
        modes = {}
        def reduce_block():
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
            per_sol, how = reduce_valu_ops_per_solution()
            ops = rate * per_sol / 1e12
            return {
                "workload": "N=6 grid (n=36), edges p=0.5, seeds 0-3: counts + hash + xorfold over all 2^r",
                "ranks": ranks,
                "value": round(rate / 1e9, 2),
                "unit": "G solutions/s",
                "roofline": {"bound": "alu", "kernel": "reduce_wave_kernel<1>",
                             "achieved": round(ops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                             "unit": "T VALU instr-lane-ops/s", "frac": round(ops / VALU_PEAK_TOPS, 4),
                             "valu_ops_per_solution": per_sol, "valu_ops_source": how},
            }

        def sample_block():
            # sampling at n = 1024
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            A = torch.from_numpy(grid_instance(32, p=0.5, seed=17)).to(dev)
            rows, st = hlf.pack_dense(A, stream=stream)
            F = hlf.factor(rows, 1024, stream=stream)
            out = torch.empty((65536, 16), dtype=torch.int64, device=dev)
            hlf.sample(F, 1, 65536, out=out, stream=stream)
            stream.synchronize()
            F.check()
            reps = 20
            _queue_behind_spin(torch, stream, reps)
            e0.record(stream)
            for k in range(reps):
                hlf.sample(F, k, 65536, out=out, stream=stream)
            e1.record(stream)
            stream.synchronize()
            smp_s = e0.elapsed_time(e1) * 1e-3 / reps
            reps = 5
            _queue_behind_spin(torch, stream, reps)
            e0.record(stream)
            for k in range(reps):
                hlf.factor(rows, 1024, F, stream=stream)
            e1.record(stream)
            stream.synchronize()
            fac_s = e0.elapsed_time(e1) * 1e-3 / reps
            rk = int(F.rank.item())
            # Basis weights per 256-column group (the sampler's unit for
            # choosing between its sparse path and the matrix cores).
            bw = np.ascontiguousarray(F.basis.cpu().numpy()[:rk]).view(np.uint64)  # [r, 16]
            bits = np.unpackbits(bw.view(np.uint8), axis=1, bitorder="little")  # [r, 1024]
            grp = [bits[:, 256 * g:256 * (g + 1)] for g in range(4)]
            max_row = max(int(b.sum(axis=1).max(initial=0)) for b in grp)
            max_col = max(int(b.sum(axis=0).max(initial=0)) for b in grp)
            sparse = max_row <= 16 and max_col <= 16
            dense_ops = 2.0 * 65536 * rk * 1024 / smp_s / 1e12  # the dense GF(2) product's multiply-adds, x2
            per = sample_valu_ops_per_sample()
            if sparse:
                roof = {"bound": "alu", "kernel": "sample_mfma_kernel, sparse path (bit slices, row lists gathered in LDS)",
                        "achieved": round(per * 65536 / smp_s / 1e12, 2) if per else None,
                        "peak": round(VALU_PEAK_TOPS, 2), "unit": "T VALU instr-lane-ops/s",
                        "frac": round(per * 65536 / smp_s / 1e12 / VALU_PEAK_TOPS, 4) if per else None,
                        "valu_ops_per_sample": per,
                        "valu_ops_source": "SQ_INSTS_VALU x 64 / samples (rocprofv3)" if per else "sources changed since the counters were taken"}
            else:
                roof = {"bound": "mfma", "kernel": "sample_mfma_kernel (fp4 E2M1 32x32x64, fp32 sums)",
                        "achieved": round(dense_ops, 1), "peak": FP4_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(dense_ops / FP4_MFMA_PEAK_TFLOPS, 4), "ops_per_sample": 2 * rk * 1024}
            return {"workload": "N=32 grid (n=1024), p=0.5: 65536 uniform samples",
                    "rank": rk, "samples_per_s": round(65536 / smp_s, 1),
                    "ms_per_65536": round(smp_s * 1e3, 4),
                    "path": "sparse" if sparse else "matrix cores",
                    "basis_max_row_weight": max_row, "basis_max_col_weight": max_col,
                    "roofline": roof,
                    "dense_product_equivalent": {"TFLOP_s": round(dense_ops, 1),
                                                 "frac_of_fp4_peak": round(dense_ops / FP4_MFMA_PEAK_TFLOPS, 4),
                                                 "note": "rate of the dense fp4 product that gives the same samples"},
                    "factor_ms_n1024": round(fac_s * 1e3, 4)}

        only = set(x for x in args.only.split(",") if x)
        for name, fn in (("reduce", reduce_block),
                         ("sample", sample_block),
                         ("tiny", lambda: tiny_mode(hlf, torch, stream, dev)),
                         ("steady", lambda: steady_mode(hlf, torch, stream, dev)),
                         ("batch", lambda: batch_mode(hlf, torch, stream, dev)),
                         ("general", lambda: general_mode(hlf, torch, stream, dev)),
                         ("circuit", lambda: circuit_mode(hlf, torch, stream, dev)),
                         ("verify", lambda: verify_mode(hlf, torch, stream, dev)),
                         ("serve", lambda: serve_mode(torch))):
            if only and name not in only:
                continue
            modes[name] = fn()
            _progress(f"{name} mode done")
        result["modes"] = modes

    # ---------------- CPU baseline: the oracle, on this host ----------------
    if not args.no_cpu_baseline:
        if not args.no_modes:
            _progress("mode cpu baselines (oracle) starting")
            mode_cpu_baselines(result["modes"], args.cpu_seconds)
        _progress("cpu baseline (oracle) starting")
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
