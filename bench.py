"""Benchmark of the checksum-protected GEMM hot path on one MI355X.

One step = one pass of the whole path on resident synthetic inputs:
encode (checksum rows/columns + threshold statistics), protected product,
one injected bit flip and (block encodings) one erased block, verify with the
erasure known, host classification, correction, block rebuild and re-verify.

Default workload: binary64, n = 8192 with an 8 x 8 grid of 1024 x 1024 blocks
(one checksum block row and column).  value = useful TFLOP/s of the whole step
(2 n^3 flops per step / step time).  The protected product kernel is also timed
per launch with events on the launch stream (the roofline object), the plain
product of the same kernel gives the ABFT overhead, and the CPU oracle is
timed on a bounded sample of the same product (rank 0, N = 1 only).

With --workload c2panel the product runs as a loop of panel updates
(outer-product form) and the erasure and flip are repaired mid-loop.

    python bench.py [--steps K] [--warmup W]
                    [--workload c2|c2b1|c2panel|c2w|c2chain|c2bc|c2v|c1|c1b64|c3|c4|c4fp8|c5]
                    [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "protected-GEMM TFLOP/s and % MFMA peak; ABFT overhead vs plain GEMM"
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6, "fp8": 5033.2}  # TFLOP/s, MI355X dense matrix-core peaks
WORKLOADS = {
    # name: (dtype, m, n, k, b, erase)
    "c2": ("f64", 8192, 8192, 8192, 1024, True),
    "c2b1": ("f64", 8192, 8192, 8192, 1, False),
    "c1": ("f64", 256, 256, 256, 1, False),
    "c1b64": ("f64", 256, 256, 256, 64, True),
    "c3": ("f32", 16384, 8192, 32768, 1, False),
    "c4": ("bf16", 16384, 16384, 16384, 1, False),
    "c4fp8": ("fp8", 16384, 16384, 16384, 1, False),
    # the same product as c2 computed as 8 rank-1024 panel updates; the block is lost, and the flip
    # lands, half-way through the k loop and both are repaired there before the loop goes on
    "c2panel": ("f64", 8192, 8192, 8192, 1024, True),
    "c2w": ("f64", 8192, 8192, 8192, 512, True),
    "c2chain": ("f64", 8192, 8192, 8192, 1024, True),
    "c2bc": ("f64", 8192, 8192, 8192, 1024, True),
    "c2v": ("f64", 16384, 1, 16384, 512, True),
    # batched: 512 bfloat16 problems, m, n, k uniform on multiples of 32 in [64, 2048]
    "c5": ("bf16", 0, 0, 0, 32, True),
}
PANELS = {"c2panel": 8}
# chained products (Sec. 3.2): the verified C_f of one n = 8192, b = 1024 product is the A_f of the next
CHAINED = {"c2chain": {"m": 8192, "n": 8192, "k": 8192, "b": 1024}}
# 2-D block-cyclic (Sec. 4.1): an 8 x 8 process grid with blocks of 64 over n = 8192; the local arrays are
# stacked on the GPU, the checksum process row/column is the block checksum of height n/8
BLOCK_CYCLIC = {"c2bc": {"n": 8192, "nb": 64, "P": 8, "Q": 8}}
# protected matrix-vector product (weighted checksums, n = 1): A_f streamed once per product
GEMV = {"c2v": {"m": 16384, "k": 16384, "b": 512, "f": 2}}
# weighted f-checksums (Sec. 2.1): n = 8192, 512 x 512 blocks (16 x 16 grid), two weighted checksum block rows
# and columns; per step two blocks of one block column are lost and two flips land in other column groups
WEIGHTED = {"c2w": {"dtype": "f64", "m": 8192, "n": 8192, "k": 8192, "b": 512, "f": 2, "flips": 2}}
BATCH = {"count": 512, "lo": 64, "hi": 2048, "step": 32, "br": 32, "bc": 1, "lam": 20.0,
         "flips": 5, "erasures": 3}
# flip bits per C type: binary64 40..62; binary32 24..29 (exponent bits and the
# top fraction bit: always above the statistical threshold, so every step's
# flip is located)
FLIP_BITS = {"f64": (40, 62), "f32": (24, 29), "bf16": (24, 29), "fp8": (24, 29)}
# HBM bytes per protected-product call (read + write, all its launches), from rocprofv3 FETCH_SIZE and
# WRITE_SIZE on this benchmark, FETCH_SIZE scaled by 2 (a 1 GiB copy reads 0.5 GiB of FETCH_SIZE);
# summarized in profiles/hbm_traffic_counters_c2_c2b1_c2panel_c2w_c4_c5.txt.  Re-measure when those kernels change.
TRAFFIC = {
    "c2": 41.728e9 + 0.679e9,                       # k_gemm_mfma2 (checksum blocks tiled with the data)
    "c2b1": 40.120e9 + 0.562e9 + 2 * 0.538e9,       # k_gemm_mfma2 + two k_sliver launches
    "c2panel": 3.832e9 + 0.679e9,                   # one accumulating panel launch of k_gemm_mfma2
    "c2w": 41.595e9 + 0.680e9,                      # k_gemm_mfma2 over the weighted-checksum C_f
    "c4": 14.040e9 + 1.120e9 + 2 * 0.538e9,         # k_gemm_lowp2 + two k_sliver1 launches
    "c5": 4.361e9 + 2.650e9 + 0.225e9 + 0.087e9,    # kb_gemm (the chosen 256 x 256 launch) + kb_combine
}
SEED = 20080523
# bound on max|C - C_oracle| / max|C_oracle| for the reported oracle check: binary64 as the parity tests;
# binary32 accumulation of k products of magnitude <= 1 (rounding of the sum, stored binary32)
TOL_VS_ORACLE = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5, "fp8": 1e-5}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_single_core(Bf, A, target_s=3.0):
    """The oracle's product rate on one thread: leading rows of A against the
    encoded B_f, about target_s seconds.  Returns (TFLOP/s, rows, seconds)."""
    from oracle import oracle as orc

    threads = orc.num_threads()
    orc.set_num_threads(1)
    try:
        rows = 4
        t0 = time.perf_counter()
        orc.gemm(A[:rows], Bf)
        t = time.perf_counter() - t0
        rows = int(min(A.shape[0], max(rows, rows * target_s / max(t, 1e-3))))
        t0 = time.perf_counter()
        orc.gemm(A[:rows], Bf)
        t = time.perf_counter() - t0
    finally:
        orc.set_num_threads(threads)
    return 2.0 * rows * Bf.shape[1] * Bf.shape[0] / t / 1e12, rows, t


def cpu_baseline(dt_name, m, n, k, b, target_s=12.0):
    """Oracle (FP64 i-l-j loops, all host threads) on leading rows of the same
    encoded product, sized to about target_s seconds; returns (TFLOP/s,
    threads, seconds, rows, the oracle's rows of C_f, the unquantized rows, the
    single-thread (TFLOP/s, rows, seconds))."""
    import numpy as np

    from oracle import oracle as orc
    from paper_0806_3121_amd import synth

    ndt = np.float64 if dt_name == "f64" else np.float32

    def quant(X):
        # the oracle's own quantizer (FP8: per-tensor scale of this sample)
        if dt_name == "bf16":
            return orc.bf16_bits_to_f64(orc.to_bf16_bits(X))
        if dt_name == "fp8":
            e = orc.e4m3_scale_exp(X)
            return orc.e4m3_values(orc.to_e4m3_codes(X * np.float32(2.0 ** e))) * 2.0 ** -e
        return X.astype(np.float64)

    B32 = synth.uniform(SEED, synth.STREAM_B, k, n, ndt)
    probe = 32
    A32 = synth.uniform_rows(SEED, synth.STREAM_A, np.arange(probe), k, ndt).astype(ndt)
    # low precision: the first rows of the product of the unquantized binary32 inputs (numpy, binary64),
    # against which the quantization error of the result is reported
    Cu = A32.astype(np.float64) @ B32.astype(np.float64) if dt_name in ("bf16", "fp8") else None
    B = quant(B32)
    del B32
    A0 = quant(A32)
    Bf = np.zeros((k, n + b))
    Bf[:, :n] = B
    del B
    orc.lib().orc_encode_cols(k, n, b, orc._p(Bf), n + b, int(dt_name != "f64"))
    t0 = time.perf_counter()
    orc.gemm(A0, Bf)
    t_probe = time.perf_counter() - t0
    rows = int(min(m, max(probe, probe * target_s / max(t_probe, 1e-3))))
    A = synth.uniform_rows(SEED, synth.STREAM_A, np.arange(rows), k, ndt).astype(ndt)
    t0 = time.perf_counter()
    A = quant(A)
    Cref = orc.gemm(A, Bf)
    dt = time.perf_counter() - t0
    flops = 2.0 * rows * (n + b) * k
    single = cpu_single_core(Bf, A, target_s=max(1.0, target_s / 4))
    return flops / dt / 1e12, orc.num_threads(), dt, rows, Cref, Cu, single


def residual_rho(A_dev, Bt_dev, C_dev, m, n, k, u):
    """The paper's residual check (Sec. 4.3) on the device's final product, in
    the infinity norm: rho = ||C x - A (B x)|| / (k u ||C|| ||x||), x seeded
    uniform[-1, 1]; computed on the host from the device's operands (as
    stored, quantized ones included) and C."""
    import numpy as np

    from paper_0806_3121_amd import synth

    A = A_dev[:m].double().cpu().numpy()
    Bt = Bt_dev[:n].double().cpu().numpy()
    C = C_dev[:m, :n].double().cpu().numpy()
    x = synth.uniform(SEED, synth.STREAM_X, n, 1)[:, 0]
    r = np.abs(C @ x - A @ (Bt.T @ x)).max()
    return float(r / (k * u * np.abs(C).sum(axis=1).max() * np.abs(x).max()))


def oracle_check(C_dev, Cref, cols):
    """Largest |C_gpu - C_oracle| / max|C_oracle| over the oracle's rows and
    the first cols columns of the device's final C_f."""
    import numpy as np

    rows = Cref.shape[0]
    Cg = C_dev[:rows, :cols].double().cpu().numpy()
    Co = Cref[:, :cols]
    return float(np.abs(Cg - Co).max() / max(np.abs(Co).max(), 1e-300))


def measure_product(torch, abft, synth, name, reps=5):
    """Protected and plain (ABFT_PLAIN, same kernel) product of one workload,
    each timed with events on the launch stream over `reps` calls after two
    warm-up calls; operands seeded as in the workload's own benchmark (binary32
    inputs quantized on the device for bfloat16 / FP8)."""
    dt_name, m, n, k, b, _ = WORKLOADS[name]
    adt = {"f64": abft.ABFT_F64, "f32": abft.ABFT_F32, "bf16": abft.ABFT_BF16, "fp8": abft.ABFT_FP8_E4M3}[dt_name]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    P = abft.Protected(adt, m, n, k, b, b, device=dev)
    if dt_name in ("bf16", "fp8"):
        A32 = torch.empty(m, k, dtype=torch.float32, device=dev)
        Bt32 = torch.empty(n, k, dtype=torch.float32, device=dev)
        abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED, synth.STREAM_A, A32)
        abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED, synth.STREAM_B, Bt32)
        abft.quantize_encode(P.p, A32, Bt32, P.A, P.Bt, P.ws)
        del A32, Bt32
    else:
        abft.fill_uniform(adt, m, k, k, 0, SEED, synth.STREAM_A, P.A)
        abft.fill_uniform(adt, k, n, k, 1, SEED, synth.STREAM_B, P.Bt)
        P.encode()
    Cplain = torch.empty(m, n, dtype=torch.float64 if dt_name == "f64" else torch.float32, device=dev)
    pplain = abft.problem(adt, m, n, k, b, b, ldc=n)

    def timed_calls(fn):
        for _ in range(2):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return sorted(e0.elapsed_time(e1) for e0, e1 in ev)

    prot = timed_calls(P.gemm)
    plain = timed_calls(lambda: abft.gemm(pplain, P.A, P.Bt, Cplain, P.ws, flags=abft.ABFT_PLAIN))
    rep = P.verify()
    if rep.n_flag_c or rep.n_flag_r:
        raise RuntimeError(f"{name}: the timed product does not verify clean")
    peak = PEAK[dt_name]
    useful, executed = 2.0 * m * n * k, 2.0 * (m + b) * (n + b) * k
    pm, qm = sum(prot) / reps, sum(plain) / reps
    out = {"workload": f"{dt_name} m={m} n={n} k={k} b={b}", "kernel": abft.describe_gemm(P.p),
           "protected_ms": round(pm, 4), "protected_ms_min": round(prot[0], 4),
           "protected_ms_median": round(prot[reps // 2], 4), "plain_ms": round(qm, 4),
           "frac": round(executed / (pm * 1e-3) / 1e12 / peak, 4),
           "frac_useful": round(useful / (pm * 1e-3) / 1e12 / peak, 4),
           "frac_plain": round(useful / (qm * 1e-3) / 1e12 / peak, 4),
           "overhead_pct": round(100 * (pm / qm - 1), 2), "floor_pct": round(100 * (executed / useful - 1), 3),
           "peak": peak}
    del P, Cplain
    torch.cuda.empty_cache()
    return out


def run_probes(torch, abft):
    """Measured peaks: the matrix-core loop probes (FP64, FP32, bfloat16) and the
    HBM read probe, each the median of five timed launches on the current stream."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sink = torch.zeros(4096, dtype=torch.float64, device=dev)

    def med(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[reps // 2]

    out = {}
    # iterations sized for tens of milliseconds per launch at the datasheet rates
    for name, dt, iters in (("f64", abft.ABFT_F64, 96000), ("f32", abft.ABFT_F32, 96000),
                            ("bf16", abft.ABFT_BF16, 384000)):
        flops = abft.probe_mfma(dt, iters, sink)
        ms = med(lambda: abft.probe_mfma(dt, iters, sink))
        out[f"mfma_{name}_tflops"] = round(flops / (ms * 1e-3) / 1e12, 2)
    buf = torch.empty(4 << 30, dtype=torch.uint8, device=dev)
    buf.fill_(1)
    ms = med(lambda: abft.probe_stream(buf, sink), reps=9)
    out["hbm_read_gbs"] = round(buf.numel() / (ms * 1e-3) / 1e9, 1)
    del buf
    torch.cuda.empty_cache()
    return out


def cpu_baseline_batched(shapes, br, bc, target_s=12.0):
    """Oracle on whole problems of the batch, in order, until about target_s
    seconds: quantize (its own RNE), encode, binary64 product of the encoded
    operands.  Returns (TFLOP/s, threads, seconds, problems)."""
    import numpy as np

    from oracle import oracle as orc
    from paper_0806_3121_amd import synth

    flops = 0.0
    t0 = time.perf_counter()
    q = 0
    while q < len(shapes) and time.perf_counter() - t0 < target_s:
        m, n, k = shapes[q]
        A = orc.bf16_bits_to_f64(orc.to_bf16_bits(synth.uniform(SEED + q, synth.STREAM_A, m, k, np.float32)))
        B = orc.bf16_bits_to_f64(orc.to_bf16_bits(synth.uniform(SEED + q, synth.STREAM_B, k, n, np.float32)))
        Af, Bf = orc.encode(A, B, br, bc, store_f32=True)
        orc.gemm(Af, Bf)
        flops += 2.0 * (m + br) * (n + bc) * k
        q += 1
    dt = time.perf_counter() - t0
    return flops / dt / 1e12, orc.num_threads(), dt, q


def run_batched(args):
    """The batched workload: per step one graph replay of quantize + encode,
    one of the persistent product (timed with events), seeded flips and
    erasures on distinct problems, block rebuilds, one graph replay of the
    verification, host classification and correction of every flagged
    problem, and a verification replay that must come back clean."""
    import torch

    from paper_0806_3121_amd import abft, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    cfg = BATCH
    br, bc = cfg["br"], cfg["bc"]
    shapes = synth.batched_shapes(SEED, cfg["count"], cfg["lo"], cfg["hi"], cfg["step"])
    log(f"workload c5: {len(shapes)} bf16 problems, br={br} bc={bc}")
    Bt = abft.Batch([(m, n, k, br, bc) for (m, n, k) in shapes], device=dev, tau_mode=abft.ABFT_TAU_STAT,
                    lam=cfg["lam"])
    for q, (m, n, k) in enumerate(shapes):
        abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED + q, synth.STREAM_A, Bt.A32[q])
        abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED + q, synth.STREAM_B, Bt.Bt32[q])
    abft.batch_quantize(Bt.plan)
    # product tile shape per problem: from the tuning cache when every problem's
    # bucket is there, else measured now (every problem under every shape) and stored
    found, tiles = abft.batch_cache_lookup(args.tile_cache, Bt.probs)
    tile_source = "cache"
    if found < len(shapes):
        costs, _ = abft.batch_tune(Bt.plan)
        abft.batch_cache_store(args.tile_cache, Bt.probs, costs)
        found, tiles = abft.batch_cache_lookup(args.tile_cache, Bt.probs)
        tile_source = "tuned"
        single = [sum(row[t] for row in costs) for t in range(abft.ABFT_BATCH_TILES)]
        mixed = sum(row[t] for row, t in zip(costs, tiles))
        # costs are in ticks of the 100 MHz device clock, summed over every tile (all CUs)
        log(f"tuned: summed tile time per single shape {[round(x * 1e-5, 2) for x in single]} ms, per-problem "
            f"shapes {mixed * 1e-5:.2f} ms")
    Bt.set_tiles(tiles)
    plan = Bt.plan
    tile_counts = [tiles.count(t) for t in range(abft.ABFT_BATCH_TILES)]
    log(f"tile shapes ({tile_source}, {args.tile_cache}): problems per shape {tile_counts}")
    # launch-level choice: each uniform shape and the per-problem shapes, timed whole
    abft.batch_quantize_encode(plan)
    choice_ms, tile = abft.batch_choose(plan, reps=5)
    choice_names = [f"{abft.BATCH_TILE_SHAPES[t][0]}x{abft.BATCH_TILE_SHAPES[t][1]}"
                    for t in range(abft.ABFT_BATCH_TILES)] + ["per-problem"]
    log(f"product by launch choice (ms): {dict(zip(choice_names, [round(x, 3) for x in choice_ms]))} -> "
        f"{choice_names[tile]}")
    torch.cuda.synchronize()

    side = torch.cuda.Stream()
    side.wait_stream(stream)
    graphs = {}
    with torch.cuda.stream(side):
        for name, fn in (("pre", lambda: abft.batch_quantize_encode(plan)),
                         ("gemm", lambda: abft.batch_gemm(plan, tile)),
                         ("verify", lambda: abft.batch_verify(plan))):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                fn()
            graphs[name] = g
    stream.wait_stream(side)
    torch.cuda.synchronize()

    ev = {"pre": [], "gemm": [], "verify": []}

    def timed(name):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        graphs[name].replay()
        e1.record(stream)
        ev[name].append((e0, e1))

    nf, ne = cfg["flips"], cfg["erasures"]

    def step(s):
        timed("pre")
        timed("gemm")
        picks = synth.pick_distinct(SEED + 7 + s, nf + ne, len(shapes))
        flips = {}
        for e, q in enumerate(picks[:nf]):
            m, n, k = shapes[q]
            i, j, bit = synth.flip_site(SEED, s * 16 + e, m + br, n + bc, 24, 29)
            abft.inject_flip(Bt.probs[q], Bt.C[q], i, j, bit)
            flips[q] = (i, j)
        for e, q in enumerate(picks[nf:]):
            m, n, k = shapes[q]
            I, J = synth.erase_block(SEED, s * 16 + e, m // br + 1, n // 32)
            rect = (I * br, J * 32, br, 32)
            abft.inject_erase(Bt.probs[q], Bt.C[q], rect)
            abft.recover_block(Bt.probs[q], Bt.C[q], rect, use_rows=False)
        timed("verify")
        flagged = Bt.fetch_reports()   # synchronises
        if sorted(flagged) != sorted(flips):
            raise RuntimeError(f"step {s}: flagged {flagged}, flipped {sorted(flips)}")
        for q in flagged:
            loc = abft.classify(Bt.probs[q], Bt.report(q))
            if (loc.cls, loc.i, loc.j) != ((abft.ABFT_CLS_DATA if flips[q][0] < shapes[q][0] and flips[q][1] <
                                            shapes[q][1] else abft.ABFT_CLS_CHECKSUM),) + flips[q]:
                raise RuntimeError(f"step {s}: problem {q} flip {flips[q]} classified {loc.cls} ({loc.i},{loc.j})")
            abft.correct(Bt.probs[q], Bt.C[q], loc)
        timed("verify")
        if Bt.fetch_reports():
            raise RuntimeError(f"step {s}: not clean after repair")

    for s in range(args.warmup):
        step(1000 + s)
    for v in ev.values():
        v.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {dt:.3f} s")
    ms = {name: sum(a.elapsed_time(c) for a, c in v) / len(v) for name, v in ev.items()}

    pe = []
    for s in range(0 if args.no_plain else max(3, min(args.steps, 10))):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        abft.batch_gemm(plan, tile, abft.ABFT_PLAIN)
        e1.record(stream)
        pe.append((e0, e1))
    torch.cuda.synchronize()
    plain_ms = sum(a.elapsed_time(c) for a, c in pe[1:]) / len(pe[1:]) if pe else None

    useful = sum(2.0 * m * n * k for (m, n, k) in shapes)
    executed = sum(2.0 * (m + br) * (n + bc) * k for (m, n, k) in shapes)
    ms_step = dt / args.steps * 1e3
    value = useful / (ms_step * 1e-3) / 1e12
    achieved = executed / (ms["gemm"] * 1e-3) / 1e12
    peak = PEAK["bf16"]
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"batched BF16->FP32 protected GEMMs c5: {len(shapes)} problems, m, n, k uniform "
                               f"on multiples of {cfg['step']} in [{cfg['lo']}, {cfg['hi']}], checksum blocks "
                               f"{br}x{bc}; per step {nf} flips and {ne} erased {br}x32 blocks on distinct "
                               f"problems; graph-captured passes",
                   "problems": len(shapes), "br": br, "bc": bc, "tile": choice_names[tile],
                   "tile_source": tile_source, "problems_per_tile_shape": tile_counts,
                   "product_ms_by_choice": dict(zip(choice_names, [round(x, 4) for x in choice_ms])),
                   "global_batch": len(shapes),
                   "seq_len": 0, "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": TRAFFIC["c5"],
                     "kernel": "kb_gemm (persistent, all problems) + kb_combine (carried checksums)",
                     "flops_per_launch": executed, "avg_launch_ms": round(ms["gemm"], 4)},
        "pct_mfma_peak_useful": round(100 * value / peak, 2),
        "phase_ms": {"quantize_encode": round(ms["pre"], 4), "gemm_protected": round(ms["gemm"], 4),
                     "verify": round(ms["verify"], 4)},
        "gemm_protected_ms": round(ms["gemm"], 4),
        "gemm_plain_ms": round(plain_ms, 4) if plain_ms else None,
        "abft_overhead_pct": round(100 * (ms["gemm"] / plain_ms - 1), 2) if plain_ms else None,
        "abft_floor_pct": round(100 * (executed / useful - 1), 2),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        tf, thr, sec, nprob = cpu_baseline_batched(shapes, br, bc, args.cpu_seconds)
        out["cpu_baseline"] = {"value": round(tf, 6), "unit": "TFLOP/s", "cores": thr, "kind": "oracle",
                               "sample": f"problems 0..{nprob - 1} of the batch, whole (quantize, encode, FP64 "
                                         f"i-l-j product of the encoded operands), {sec:.1f} s"}
    print(json.dumps(out), flush=True)


def run_weighted(args):
    """Weighted f-checksum step: encode (f weighted checksum block rows and
    columns), product, f lost blocks of one block column and flips in other
    column groups, verify with the loss known, locate the flips from the
    weight ratios, correct, rebuild the f blocks (f x f solve), re-verify."""
    import torch

    from paper_0806_3121_amd import abft, synth

    cfg = WEIGHTED[args.workload]
    m, n, k, b, f = cfg["m"], cfg["n"], cfg["k"], cfg["b"], cfg["f"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    Gr, Gc = m // b, n // b
    Wr = 0.5 + (synth.uniform(SEED, synth.STREAM_X, f, Gr) + 1) / 2
    Wc = 0.5 + (synth.uniform(SEED, synth.STREAM_PICK, f, Gc) + 1) / 2
    log(f"workload {args.workload}: f64 m={m} n={n} k={k} b={b} f={f}")
    P = abft.WProtected(m, n, k, b, b, Wr, Wc, device=dev)
    abft.fill_uniform(abft.ABFT_F64, m, k, k, 0, SEED, synth.STREAM_A, P.A)
    abft.fill_uniform(abft.ABFT_F64, k, n, k, 1, SEED, synth.STREAM_B, P.Bt)
    Cplain = torch.empty(m, n, dtype=torch.float64, device=dev)
    pplain = abft.problem(abft.ABFT_F64, m, n, k, b, b, ldc=n)
    torch.cuda.synchronize()
    bit_lo, bit_hi = FLIP_BITS["f64"]
    g_events = []

    def step(s):
        P.encode()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.gemm()
        e1.record(stream)
        g_events.append((e0, e1))
        # f lost blocks of one block column (f failed processes of a process column)
        I = synth.pick_distinct(SEED + s, f, Gr, stream=synth.STREAM_ERASE)
        J = synth.randint(SEED, synth.STREAM_ERASE, 1000 + s, Gc)
        rects = [(i * b, J * b, b, b) for i in I]
        sites, groups, t = [], set(), 0
        while len(sites) < cfg["flips"]:
            x, y, bit = synth.flip_site(SEED, 4 * s + t, m, n, bit_lo, bit_hi, avoid=(0, J * b, m, b))
            t += 1
            if (x % b, y) not in groups:
                groups.add((x % b, y))
                sites.append((x, y, bit))
        for (x, y, bit) in sites:
            v = P.C[x, y].view(torch.int64) ^ (1 << bit)
            P.C[x, y] = v.view(torch.float64)
        for (i0, j0, h, w) in rects:
            P.C[i0:i0 + h, j0:j0 + w] = float("nan")
        rep = P.verify(known=rects)
        st, locs = abft.wlocate(P.p, rep)
        got = sorted((l.cls, l.i, l.j) for l in locs)
        want = sorted((abft.ABFT_CLS_DATA, x, y) for (x, y, _) in sites)
        if st != abft.ABFT_OK or got != want:
            raise RuntimeError(f"step {s}: flips {sites} located as {got}")
        abft.wcorrect(P.p, P.C, locs, P.ws)
        abft.wrecover(P.p, P.C, abft.ABFT_DIR_COL, I, J * b, b, P.ws)
        rep = P.verify()
        if rep.n_fail_c or rep.n_fail_r:
            raise RuntimeError(f"step {s}: not clean after repair")

    for s in range(args.warmup):
        step(1000 + s)
    g_events.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {dt:.3f} s")
    gemm_ms = sum(a.elapsed_time(c) for a, c in g_events) / len(g_events)
    pe = []
    for s in range(0 if args.no_plain else max(3, min(args.steps, 10))):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        abft.gemm(pplain, P.A, P.Bt, Cplain, None, flags=abft.ABFT_PLAIN)
        e1.record(stream)
        pe.append((e0, e1))
    torch.cuda.synchronize()
    plain_ms = sum(a.elapsed_time(c) for a, c in pe[1:]) / len(pe[1:]) if pe else None
    peak = PEAK["f64"]
    useful = 2.0 * m * n * k
    executed = 2.0 * (m + f * b) * (n + f * b) * k
    ms_step = dt / args.steps * 1e3
    value = useful / (ms_step * 1e-3) / 1e12
    achieved = executed / (gemm_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"F64 weighted-checksum GEMM {args.workload}: m={m} n={n} k={k}, {b}x{b} blocks "
                               f"({Gr}x{Gc} grid), {f} weighted checksum block rows and columns (weights uniform "
                               f"in [0.5, 1.5)); per step {f} lost blocks of one block column rebuilt by an "
                               f"{f}x{f} solve and {cfg['flips']} flips located by weight ratios",
                   "m": m, "n": n, "k": k, "br": b, "bc": b, "f": f, "global_batch": 1, "seq_len": 0,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": TRAFFIC.get(args.workload),
                     "kernel": "k_gemm_mfma2 (weighted-checksum product, all M x N entries)",
                     "flops_per_launch": executed, "avg_launch_ms": round(gemm_ms, 4)},
        "pct_mfma_peak_useful": round(100 * value / peak, 2),
        "gemm_protected_ms": round(gemm_ms, 4),
        "gemm_plain_ms": round(plain_ms, 4) if plain_ms else None,
        "abft_overhead_pct": round(100 * (gemm_ms / plain_ms - 1), 2) if plain_ms else None,
        "abft_floor_pct": round(100 * (executed / useful - 1), 2),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        tf, thr, sec, rows, Cref, _, _ = cpu_baseline("f64", m, n, k, f * b, args.cpu_seconds)
        # data columns only: the oracle's sample encodes unit-weight checksum columns
        out["oracle_check"] = {"rows": rows, "cols": n, "max_rel_err": oracle_check(P.C, Cref, n),
                               "bound": 1e-12}
        out["cpu_baseline"] = {"value": round(tf, 6), "unit": "TFLOP/s", "cores": thr, "kind": "oracle",
                               "sample": f"rows 0..{rows - 1} of an encoded product ({rows} x {n + f * b} x {k}, "
                                         f"FP64 i-l-j loops), {sec:.1f} s"}
    print(json.dumps(out), flush=True)


def _timed(torch, stream, fn):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    return (e0, e1)


def _steps(torch, args, step):
    for s in range(args.warmup):
        step(1000 + s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(s)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_chained(args):
    """Two chained products per step: C_f = A_f B_f (encoded, verified), then
    D_f = C_f[:, :n] B2_f with C_f's carried rows reused as checksum rows
    (abft_encode_chained); D_f gets one flip and one erased block, is verified
    with the erasure known, corrected, rebuilt and verified again."""
    import torch

    from paper_0806_3121_amd import abft, synth

    cfg = CHAINED[args.workload]
    m, n, k, b = cfg["m"], cfg["n"], cfg["k"], cfg["b"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    log(f"workload {args.workload}: f64 chained m={m} n={n} k={k} b={b}")
    P1 = abft.Protected(abft.ABFT_F64, m, n, k, b, b, device=dev)
    abft.fill_uniform(abft.ABFT_F64, m, k, k, 0, SEED, synth.STREAM_A, P1.A)
    abft.fill_uniform(abft.ABFT_F64, k, n, k, 1, SEED, synth.STREAM_B, P1.Bt)
    N = n + b
    p2 = abft.problem(abft.ABFT_F64, m, n, n, b, b, lda=P1.ldc, ldb=n, ldc=P1.ldc)
    Bt2 = torch.zeros(N, n, dtype=torch.float64, device=dev)
    abft.fill_uniform(abft.ABFT_F64, n, n, n, 1, SEED + 1, synth.STREAM_B, Bt2)
    ws2 = torch.zeros(abft.workspace_size(p2), dtype=torch.uint8, device=dev)
    D = torch.zeros(m + b, P1.ldc, dtype=torch.float64, device=dev)
    host = abft.new_report_buffer()
    torch.cuda.synchronize()
    ev = []

    def step(s):
        P1.encode()
        e1 = _timed(torch, stream, P1.gemm)
        if P1.verify().n_flag_c:
            raise RuntimeError("first product not clean")
        abft.encode_chained(p2, P1.Cbuf, Bt2, ws2, P1.p, P1.ws)
        e2 = _timed(torch, stream, lambda: abft.gemm(p2, P1.Cbuf, Bt2, D, ws2))
        ev.append((e1, e2))
        I, J = synth.erase_block(SEED, s, m // b, n // b)
        rect = (I * b, J * b, b, b)
        i, j, bit = synth.flip_site(SEED, s, m, n, 40, 62, avoid=rect)
        abft.inject_flip(p2, D, i, j, bit)
        abft.inject_erase(p2, D, rect)
        abft.verify(p2, D, ws2, known=[rect], host_out=host)
        stream.synchronize()
        loc = abft.classify(p2, abft.read_report(host), known=[rect])
        if (loc.cls, loc.i, loc.j) != (abft.ABFT_CLS_DATA, i, j):
            raise RuntimeError(f"step {s}: flip ({i},{j}) located as {loc.cls} ({loc.i},{loc.j})")
        abft.correct(p2, D, loc)
        abft.recover_block(p2, D, rect)
        abft.verify(p2, D, ws2, host_out=host)
        stream.synchronize()
        rep = abft.read_report(host)
        if rep.n_flag_c or rep.n_flag_r:
            raise RuntimeError(f"step {s}: chained result not clean after repair")

    dt = _steps(torch, args, step)
    ev = ev[-args.steps:]
    g1 = sum(a.elapsed_time(c) for (a, c), _ in ev) / len(ev)
    g2 = sum(a.elapsed_time(c) for _, (a, c) in ev) / len(ev)
    useful = 2 * 2.0 * m * n * k
    executed = 2 * 2.0 * (m + b) * (n + b) * k
    ms_step = dt / args.steps * 1e3
    value = useful / (ms_step * 1e-3) / 1e12
    achieved = executed / ((g1 + g2) * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"F64 chained protected GEMMs {args.workload}: two products m=n=k={n}, {b}x{b} blocks; "
                               "the verified C_f of the first is the A_f of the second (carried checksum rows "
                               "reused); the second gets one erased block and one flip per step",
                   "m": m, "n": n, "k": k, "br": b, "bc": b, "global_batch": 1, "seq_len": 0,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f64"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK["f64"], 4), "traffic": None,
                     "kernel": "k_gemm_mfma2 (both products)", "flops_per_launch": executed / 2,
                     "avg_launch_ms": round((g1 + g2) / 2, 4)},
        "gemm_first_ms": round(g1, 4), "gemm_chained_ms": round(g2, 4),
    }
    print(json.dumps(out), flush=True)


def run_block_cyclic(args):
    """Step: the global A and B are stacked into the grid's local arrays (A's
    rows over the process rows, B's columns over the process columns), encoded
    (checksum process row and column), multiplied; one process's local array
    of C_f is lost and one element elsewhere flipped; verify with the loss
    known, locate, correct, rebuild the process, verify; C unstacked back to
    the global layout."""
    import torch

    from paper_0806_3121_amd import abft, synth

    cfg = BLOCK_CYCLIC[args.workload]
    n, nb, P, Q = cfg["n"], cfg["nb"], cfg["P"], cfg["Q"]
    m = k = n
    br, bc = m // P, n // Q
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    log(f"workload {args.workload}: f64 n={n} nb={nb} grid {P}x{Q}")
    Ag = torch.empty(m, k, dtype=torch.float64, device=dev)
    Btg = torch.empty(n, k, dtype=torch.float64, device=dev)
    abft.fill_uniform(abft.ABFT_F64, m, k, k, 0, SEED, synth.STREAM_A, Ag)
    abft.fill_uniform(abft.ABFT_F64, k, n, k, 1, SEED, synth.STREAM_B, Btg)
    Pr = abft.Protected(abft.ABFT_F64, m, n, k, br, bc, device=dev)
    Cg = torch.empty(m, n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ev = []

    def step(s):
        e_st = _timed(torch, stream, lambda: (abft.block_cyclic_stack(Ag, m, k, nb, P, 1, Pr.A[:m]),
                                              abft.block_cyclic_stack(Btg, n, k, nb, Q, 1, Pr.Bt[:n])))
        Pr.encode()
        e_g = _timed(torch, stream, Pr.gemm)
        pq = synth.erase_block(SEED, s, P, Q)
        rect = (pq[0] * br, pq[1] * bc, br, bc)
        i, j, bit = synth.flip_site(SEED, s, m, n, 40, 62, avoid=rect)
        abft.inject_flip(Pr.p, Pr.C, i, j, bit)
        abft.inject_erase(Pr.p, Pr.C, rect)
        rep = Pr.verify(known=[rect])
        loc = abft.classify(Pr.p, rep, known=[rect])
        if (loc.cls, loc.i, loc.j) != (abft.ABFT_CLS_DATA, i, j):
            raise RuntimeError(f"step {s}: flip ({i},{j}) located as {loc.cls} ({loc.i},{loc.j})")
        abft.correct(Pr.p, Pr.C, loc)
        abft.recover_block(Pr.p, Pr.C, rect)
        rep = Pr.verify()
        if rep.n_flag_c or rep.n_flag_r:
            raise RuntimeError(f"step {s}: not clean after repair")
        e_un = _timed(torch, stream, lambda: abft.block_cyclic_unstack(Pr.C[:m, :n], m, n, nb, P, Q, Cg))
        ev.append((e_st, e_g, e_un))

    dt = _steps(torch, args, step)
    ev = ev[-args.steps:]
    st_ms = sum(a.elapsed_time(c) for (a, c), _, _ in ev) / len(ev)
    g_ms = sum(a.elapsed_time(c) for _, (a, c), _ in ev) / len(ev)
    un_ms = sum(a.elapsed_time(c) for _, _, (a, c) in ev) / len(ev)
    useful = 2.0 * m * n * k
    executed = 2.0 * (m + br) * (n + bc) * k
    ms_step = dt / args.steps * 1e3
    out = {
        "metric": METRIC, "value": round(useful / (ms_step * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"F64 protected GEMM on a 2-D block-cyclic {P}x{Q} grid {args.workload}: n={n}, "
                               f"blocks of {nb}; local arrays stacked, checksum process row and column; per step "
                               "one process's local array of C lost and one flip elsewhere",
                   "m": m, "n": n, "k": k, "br": br, "bc": bc, "nb": nb, "grid": [P, Q], "global_batch": 1,
                   "seq_len": 0, "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": round(executed / (g_ms * 1e-3) / 1e12, 3), "peak": PEAK["f64"],
                     "unit": "TFLOP/s", "frac": round(executed / (g_ms * 1e-3) / 1e12 / PEAK["f64"], 4),
                     "traffic": None, "kernel": "k_gemm_mfma2", "flops_per_launch": executed,
                     "avg_launch_ms": round(g_ms, 4)},
        "stack_ms": round(st_ms, 4), "stack_GBps": round(2 * 2 * 8.0 * n * k / (st_ms * 1e-3) / 1e9, 1),
        "unstack_ms": round(un_ms, 4), "unstack_GBps": round(2 * 8.0 * m * n / (un_ms * 1e-3) / 1e9, 1),
    }
    print(json.dumps(out), flush=True)


def run_gemv(args):
    """Protected matrix-vector product y = A x with f weighted checksum block
    rows (a weighted problem with n = 1): encode, product (the streaming
    kernel reads A_f once), two flips of y located by the weight ratios and
    corrected, then f lost blocks of y rebuilt, verify."""
    import torch

    from paper_0806_3121_amd import abft, synth

    cfg = GEMV[args.workload]
    m, k, b, f = cfg["m"], cfg["k"], cfg["b"], cfg["f"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    Gr = m // b
    Wr = 0.5 + (synth.uniform(SEED, synth.STREAM_X, f, Gr) + 1) / 2
    log(f"workload {args.workload}: f64 matrix-vector m={m} k={k} b={b} f={f}")
    P = abft.WProtected(m, 1, k, b, 1, Wr, [[1.0]], device=dev)
    abft.fill_uniform(abft.ABFT_F64, m, k, k, 0, SEED, synth.STREAM_A, P.A)
    abft.fill_uniform(abft.ABFT_F64, k, 1, k, 1, SEED, synth.STREAM_B, P.Bt)
    torch.cuda.synchronize()
    ev = []

    def step(s):
        P.encode()
        ev.append(_timed(torch, stream, P.gemm))
        # two flips of y in distinct residues (distinct column groups): located by the weight ratios
        r0 = synth.randint(SEED, synth.STREAM_FLIP, 4 * s, b)
        r1 = (r0 + 1 + synth.randint(SEED, synth.STREAM_FLIP, 4 * s + 1, b - 1)) % b
        sites = [(r0 + b * synth.randint(SEED, synth.STREAM_FLIP, 4 * s + 2, Gr), 52),
                 (r1 + b * synth.randint(SEED, synth.STREAM_FLIP, 4 * s + 3, Gr), 57)]
        for x, bit in sites:
            v = P.C[x, 0].view(torch.int64) ^ (1 << bit)
            P.C[x, 0] = v.view(torch.float64)
        rep = P.verify()
        st, locs = abft.wlocate(P.p, rep)
        if st != abft.ABFT_OK or sorted((l.i, l.j) for l in locs) != sorted((x, 0) for x, _ in sites):
            raise RuntimeError(f"step {s}: flips {sites} located as {[(l.cls, l.i, l.j) for l in locs]}")
        abft.wcorrect(P.p, P.C, locs, P.ws)
        # then f lost blocks of y (f failed processes), rebuilt by an f x f solve
        lost = synth.pick_distinct(SEED + s, f, Gr, stream=synth.STREAM_ERASE)
        for g in lost:
            P.C[g * b:(g + 1) * b, :] = float("nan")
        abft.wrecover(P.p, P.C, abft.ABFT_DIR_COL, lost, 0, 2, P.ws)
        rep = P.verify()
        if rep.n_fail_c or rep.n_fail_r:
            raise RuntimeError(f"step {s}: not clean after repair")

    dt = _steps(torch, args, step)
    ev = ev[-args.steps:]
    g = sum(a.elapsed_time(c) for a, c in ev) / len(ev)
    M = m + f * b
    bytes_read = M * k * 8.0
    ms_step = dt / args.steps * 1e3
    out = {
        "metric": METRIC, "value": round(2.0 * m * k / (ms_step * 1e-3) / 1e12, 4), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"F64 protected matrix-vector product {args.workload}: m=k={m}, {f} weighted "
                               f"checksum block rows of {b}; per step two flips of y located by weight ratios and "
                               f"{f} lost blocks of y rebuilt", "m": m, "n": 1, "k": k, "br": b, "bc": 1, "f": f,
                   "global_batch": 1, "seq_len": 0, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(bytes_read / (g * 1e-3) / 1e9, 1), "peak": 8000.0,
                     "unit": "GB/s", "frac": round(bytes_read / (g * 1e-3) / 8e12, 4), "traffic": None,
                     "kernel": "k_sliver (A_f streamed once)", "bytes_per_launch": bytes_read,
                     "avg_launch_ms": round(g, 4)},
    }
    print(json.dumps(out), flush=True)


class OracleFlips:
    """The oracle's decision on single flips of one product (the reliability
    campaigns, counted against the FP64 oracle as Sec. 4.3's stress test is
    read here).  It holds the encoded operands in binary64 (bfloat16 / FP8:
    the oracle's own quantization of the same binary32 inputs, FP8 in the
    scaled domain with the result scaled back), and the thresholds of the
    library's model computed by the oracle.  For a flip of bit `bit` of
    element (i, j) it computes, with the oracle's product (ascending-k sums),
    every member of the two relations through (i, j), rounds them as C is
    stored, flips the bit of its own element and takes each relation's
    residual with the oracle's verification and classification.  Only the
    inputs are shared with the GPU run; no value comes from the GPU."""

    def __init__(self, dt_name, A, B, br, bc, lam=10.0, carried_steps=0.0):
        """carried_steps: accumulation steps of the stored totals when the product computes them in
        binary32 (the batched path's matrix-core checksum rows, k / 4); 0 when they are binary64 sums."""
        import numpy as np

        from oracle import oracle as orc

        self.orc, self.np = orc, np
        self.dt, self.br, self.bc = dt_name, br, bc
        self.acc_exp = 0          # FP8: the product's accumulators are C scaled by 2^acc_exp
        self.m, self.k = A.shape
        self.n = B.shape[1]
        sc = 1.0
        if dt_name == "bf16":
            A = orc.bf16_bits_to_f64(orc.to_bf16_bits(A))
            B = orc.bf16_bits_to_f64(orc.to_bf16_bits(B))
        elif dt_name == "fp8":
            eA, eB = orc.e4m3_scale_exp(A), orc.e4m3_scale_exp(B)
            A = orc.e4m3_values(orc.to_e4m3_codes(np.ldexp(A.astype(np.float64), eA).astype(np.float32)))
            B = orc.e4m3_values(orc.to_e4m3_codes(np.ldexp(B.astype(np.float64), eB).astype(np.float32)))
            sc = 2.0 ** -(eA + eB)
            self.acc_exp = eA + eB
        self.sc = sc
        self.Af, self.Bf = orc.encode(np.asarray(A, dtype=np.float64), np.asarray(B, dtype=np.float64), br, bc,
                                      store_f32=(dt_name != "f64"))
        m, n, k = self.m, self.n, self.k
        # the oracle's C_f once, in row chunks (progress on stderr), as C stores it
        M, N = m + br, n + bc
        self.C = np.empty((M, N))
        step = max(1, -(-M // 16))
        for r0 in range(0, M, step):
            r1 = min(M, r0 + step)
            self.C[r0:r1] = self._stored(orc.gemm(self.Af[r0:r1], self.Bf) * sc)
            if M * N * k > 1e10:
                log(f"oracle C_f rows {r1} / {M}")
        self.stat = dt_name != "f64"
        if not self.stat:
            self.tc, self.tr = orc.tau_det(self.Af, self.Bf, m, n, br, bc)
        else:
            T = k if dt_name == "f32" else k / 4.0
            s_store = 2.0 + (2.0 ** 18 if dt_name == "fp8" else 0.0)

            def tau(Cf):
                tc, tr = orc.tau_stat(self.Af, self.Bf, m, n, br, bc, u_acc=2.0 ** -24, T=T, s_store=s_store,
                                      lam=lam, Cf=Cf / sc if sc != 1.0 else Cf, T_c=carried_steps)
                return tc * sc, tr * sc
            self._tau = tau
            self.tc, self.tr = tau(self.C)

    def _stored(self, v):
        """Values of C as stored: binary64, or rounded once to binary32."""
        np = self.np
        return v if self.dt == "f64" else v.astype(np.float32).astype(np.float64)

    def _flip(self, v, bit):
        np = self.np
        if self.dt == "f64":
            x = np.array([v], dtype=np.float64).view(np.uint64) ^ np.uint64(1 << bit)
            return float(x.view(np.float64)[0])
        x = np.array([v], dtype=np.float32).view(np.uint32) ^ np.uint32(1 << bit)
        return float(x.view(np.float32)[0])

    def _residual(self, members):
        """The oracle's residual of one relation: its data members summed in
        order, minus its stored total (the last member)."""
        np, orc = self.np, self.orc
        G = len(members) - 1
        Cr = np.zeros((G + 1, 2))
        Cr[:, 0] = members
        Dc, _, _ = orc.verify(Cr, G, 1, 1, 1, np.zeros((1, 2)), np.zeros((G + 1, 1)))
        return Dc[0, 0]

    def decide(self, i, j, bit, accumulator=False):
        """-> dict: delta, the two residual / threshold ratios, the class
        ('above': both relations beyond 2 tau or non-finite; 'below': both
        within tau / 2; 'gray' otherwise) and the oracle's classification.
        accumulator: the bit is flipped in the product's accumulator, before
        the FP8 result is scaled back (an exponent bit then changes the value
        differently than in the stored C)."""
        np, orc = self.np, self.orc
        m, n, br, bc = self.m, self.n, self.br, self.bc
        r, c = (i % br if i < m else i - m), (j % bc if j < n else j - n)
        rows = [g * br + r for g in range(m // br)] + [m + r]
        cols = [h * bc + c for h in range(n // bc)] + [n + c]
        col = self.C[rows, j].copy()
        row = self.C[i, cols].copy()
        ic, jr = rows.index(i), cols.index(j)
        old = col[ic]
        if accumulator and self.acc_exp:
            with np.errstate(over="ignore", invalid="ignore"):
                acc = float(np.float32(np.ldexp(old, self.acc_exp)))       # exact: C = acc 2^-acc_exp
                new = float(np.float32(np.ldexp(self._flip(acc, bit), -self.acc_exp)))
        else:
            new = self._flip(old, bit)
        col[ic] = new
        row[jr] = new
        with np.errstate(invalid="ignore", over="ignore"):
            dc, dr = self._residual(col), self._residual(row)
        tc, tr = self.tc[r, j], self.tr[i, c]
        if self.stat and (i >= m or j >= n):
            # a flip on a stored total also moves that relation's rounding term
            self.C[i, j] = new
            try:
                tcs, trs = self._tau(self.C)
            finally:
                self.C[i, j] = old
            tc, tr = tcs[r, j], trs[i, c]
        rep = orc.Report()
        for side, (a, bb, d, t) in (("c", (r, j, dc, tc)), ("r", (i, c, dr, tr))):
            if not abs(d) <= t:
                if side == "c":
                    rep.n_flag_c = 1
                    rep.fc_r[0], rep.fc_j[0], rep.fc_d[0], rep.fc_t[0] = a, bb, d, t
                else:
                    rep.n_flag_r = 1
                    rep.fr_i[0], rep.fr_c[0], rep.fr_d[0], rep.fr_t[0] = a, bb, d, t
        cls, oi, oj, _ = orc.classify(rep, m, n, br, bc)
        finite = np.isfinite(dc) and np.isfinite(dr)
        with np.errstate(over="ignore"):
            rc = abs(dc) / tc if finite and tc > 0 else float("inf")
            rr = abs(dr) / tr if finite and tr > 0 else float("inf")
        if not finite or (rc > 2 and rr > 2):
            klass = "above"
        elif rc <= 0.5 and rr <= 0.5:
            klass = "below"
        else:
            klass = "gray"
        return {"delta": float(new - old), "ratio_c": float(rc), "ratio_r": float(rr), "class": klass,
                "tau": float(min(tc, tr)), "oracle_located": bool(cls in (orc.DATA, orc.CHECKSUM) and (oi, oj) == (i, j))}


def flip_tally(nbits):
    """Counters of a flip campaign: totals per oracle class and per bit."""
    return {"flips": 0, "gpu_detected": 0, "gpu_false_alarm_below": 0,
            "above": 0, "above_oracle_located": 0, "above_gpu_located": 0, "above_gpu_corrected": 0,
            "gray": 0, "gray_gpu_located": 0, "below": 0, "below_gpu_detected": 0,
            "per_bit": {str(bit): {"flips": 0, "above": 0, "above_located": 0, "gray": 0, "gray_located": 0,
                                   "below": 0} for bit in range(nbits)}}


def flip_count(st, bit, dec, detected, located, corrected):
    detected, located, corrected = bool(detected), bool(located), bool(corrected)
    st["flips"] += 1
    st["gpu_detected"] += detected
    pb = st["per_bit"][str(bit)]
    pb["flips"] += 1
    k = dec["class"]
    st[k] += 1
    pb[k] += 1
    if k == "above":
        st["above_oracle_located"] += bool(dec["oracle_located"])
        st["above_gpu_located"] += located
        st["above_gpu_corrected"] += corrected
        pb["above_located"] += located
    elif k == "gray":
        st["gray_gpu_located"] += located
        pb["gray_located"] += located
    else:
        st["below_gpu_detected"] += detected
        st["gpu_false_alarm_below"] += bool(detected and dec["ratio_c"] < 0.5 and dec["ratio_r"] < 0.5)


def run_campaign(args):
    """Reliability campaign on one workload, counted against the FP64 oracle.

    Clean runs: args.campaign products on fresh seeded inputs (uniform, or
    with --inputs heavy N(0,1) with 1 % of the entries x 1e3, generated on the
    device); every relation must pass (false positives counted; the largest
    |D|/tau reported).

    Flip runs: args.campaign single flips of one product (seeded sites, every
    bit position of C's type) on inputs generated on the host, which the
    oracle (OracleFlips) also reads.  For each flip the oracle decides the
    class (above: both relations beyond 2 tau or non-finite; gray; below:
    both within tau / 2) and whether it locates the element; the GPU's
    verify, classification and correction run on the flipped C.  The target:
    every flip above the oracle's thresholds located and corrected.  Counts
    per class and per bit position."""
    import numpy as np
    import torch

    from paper_0806_3121_amd import abft, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dt_name, m, n, k, b, _ = WORKLOADS[args.workload]
    adt = {"f64": abft.ABFT_F64, "f32": abft.ABFT_F32, "bf16": abft.ABFT_BF16, "fp8": abft.ABFT_FP8_E4M3}[dt_name]
    lowp = dt_name in ("bf16", "fp8")
    heavy = args.inputs == "heavy"
    if heavy and dt_name == "f64":
        print(json.dumps({"error": "--inputs heavy is a binary32-input set"}))
        sys.exit(2)
    nbits = 64 if dt_name == "f64" else 32
    P = abft.Protected(adt, m, n, k, b, b, device=dev)
    if lowp:
        A32 = torch.empty(m, k, dtype=torch.float32, device=dev)
        Bt32 = torch.empty(n, k, dtype=torch.float32, device=dev)
    site_k = args.site == "k"
    if site_k and b != 1:
        print(json.dumps({"error": "--site k needs a b = 1 workload"}))
        sys.exit(2)

    def fill_device(seed):
        dstA, dstB = (A32, Bt32) if lowp else (P.A, P.Bt)
        if heavy:
            abft.fill_normal(m, k, k, 0, seed, dstA)
            abft.fill_normal(k, n, k, 1, seed + 1, dstB)
        else:
            fdt = abft.ABFT_F64 if dt_name == "f64" else abft.ABFT_F32
            abft.fill_uniform(fdt, m, k, k, 0, seed, synth.STREAM_A, dstA)
            abft.fill_uniform(fdt, k, n, k, 1, seed, synth.STREAM_B, dstB)

    def encode_and_multiply():
        if lowp:
            abft.quantize_encode(P.p, A32, Bt32, P.A, P.Bt, P.ws)
        else:
            P.encode()
        P.gemm(abft.ABFT_FUSED if site_k else 0)

    def first_verify():
        return P.verify_fused() if site_k else P.verify()

    t0 = time.perf_counter()
    fp, worst = 0, 0.0
    for r in range(args.campaign):
        fill_device(SEED + 1000 + 2 * r)
        encode_and_multiply()
        rep = first_verify()
        if rep.n_flag_c or rep.n_flag_r:
            fp += 1
        worst = max(worst, rep.max_ratio_c, rep.max_ratio_r)
        if r % 100 == 0:
            log(f"clean run {r}: false positives so far {fp}, max |D|/tau {worst:.3f}")
    t_clean = time.perf_counter() - t0

    # the flip product: host-generated inputs, uploaded; the oracle reads the same arrays
    log("flip product: inputs on the host, the oracle's operands and thresholds ...")
    ndt = np.float64 if dt_name == "f64" else np.float32
    if heavy:
        A = synth.normal_with_outliers(SEED + 101, m, k)
        B = synth.normal_with_outliers(SEED + 102, k, n)
    else:
        A = synth.uniform(SEED, synth.STREAM_A, m, k, ndt)
        B = synth.uniform(SEED, synth.STREAM_B, k, n, ndt)
    t_or = time.perf_counter()
    orf = OracleFlips(dt_name, A, B, b, b)
    t_or = time.perf_counter() - t_or
    if lowp:
        A32.copy_(torch.from_numpy(A))
        Bt32.copy_(torch.from_numpy(np.ascontiguousarray(B.T)))
    else:
        P.A[:m].copy_(torch.from_numpy(A))
        P.Bt[:n].copy_(torch.from_numpy(np.ascontiguousarray(B.T)))
    del A, B
    encode_and_multiply()
    torch.cuda.synchronize()
    clean = P.C.clone()
    M, N = m + b, n + b
    st = flip_tally(nbits)
    t0 = time.perf_counter()
    t_oracle_flips = 0.0
    for r in range(args.campaign):
        if site_k:
            # inside the product kernel: an accumulator of the data part, flipped before the epilogue
            i, j, bit = synth.flip_site(SEED + 17, r, m, n, 0, nbits - 1)
            P.gemm_fault(i, j, bit, abft.ABFT_FUSED)
        else:
            i, j, bit = synth.flip_site(SEED + 17, r, M, N, 0, nbits - 1)
            P.C.copy_(clean)
            abft.inject_flip(P.p, P.C, i, j, bit)
        rep = first_verify()
        detected = bool(rep.n_flag_c or rep.n_flag_r)
        loc = abft.classify(P.p, rep)
        located = (loc.i, loc.j) == (i, j) and loc.cls in (abft.ABFT_CLS_DATA, abft.ABFT_CLS_CHECKSUM)
        ta = time.perf_counter()
        dec = orf.decide(i, j, bit, accumulator=site_k)
        t_oracle_flips += time.perf_counter() - ta
        corrected = False
        if located:
            abft.correct(P.p, P.C, loc)
            rep2 = P.verify()
            corrected = not (rep2.n_flag_c or rep2.n_flag_r) and abs(P.C[i, j].item() - clean[i, j].item()) <= dec["tau"]
        flip_count(st, bit, dec, detected, located, corrected)
        if dec["class"] == "above" and not (located and corrected):
            log(f"flip run {r}: ({i},{j}) bit {bit} above the oracle's thresholds but not repaired: gpu cls "
                f"{loc.cls} ({loc.i},{loc.j}), ratios {dec['ratio_c']:.3g} / {dec['ratio_r']:.3g}")
        if r % 100 == 0:
            log(f"flip run {r}: above {st['above']} (gpu located {st['above_gpu_located']}), gray {st['gray']}, "
                f"below {st['below']}")
    t_flip = time.perf_counter() - t0
    out = {"campaign": args.workload, "inputs": args.inputs, "site": args.site, "dtype": dt_name, "m": m, "n": n,
           "k": k, "b": b, "clean_runs": args.campaign, "false_positives": fp,
           "max_ratio_clean": float(f"{worst:.3g}"), "flip_runs": args.campaign, "flip_bits": f"0..{nbits - 1}",
           **st, "seconds": {"clean": round(t_clean, 1), "flips": round(t_flip, 1),
                             "oracle_setup": round(t_or, 1), "oracle_per_flip": round(t_oracle_flips, 1)}}
    print(json.dumps(out), flush=True)


def run_weighted_campaign(args):
    """Reliability campaign on the weighted-checksum workload: args.campaign
    clean products on fresh seeded inputs (false positives counted), then
    args.campaign runs with two flips (every bit position, anywhere in C_f, in
    distinct column groups) located by the weight ratios and corrected, and
    f lost blocks of one block column rebuilt."""
    import torch

    from paper_0806_3121_amd import abft, synth

    cfg = WEIGHTED[args.workload]
    m, n, k, b, f = cfg["m"], cfg["n"], cfg["k"], cfg["b"], cfg["f"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Gr, Gc = m // b, n // b
    Wr = 0.5 + (synth.uniform(SEED, synth.STREAM_X, f, Gr) + 1) / 2
    Wc = 0.5 + (synth.uniform(SEED, synth.STREAM_PICK, f, Gc) + 1) / 2
    P = abft.WProtected(m, n, k, b, b, Wr, Wc, device=dev)

    def product(seed):
        abft.fill_uniform(abft.ABFT_F64, m, k, k, 0, seed, synth.STREAM_A, P.A)
        abft.fill_uniform(abft.ABFT_F64, k, n, k, 1, seed, synth.STREAM_B, P.Bt)
        P.encode()
        P.gemm()

    t0 = time.perf_counter()
    fp, worst = 0, 0.0
    for r in range(args.campaign):
        product(SEED + 3000 + r)
        rep = P.verify()
        fp += bool(rep.n_fail_c or rep.n_fail_r)
        worst = max(worst, rep.max_ratio_c, rep.max_ratio_r)
        if r % 100 == 0:
            log(f"clean run {r}: false positives so far {fp}, max |D|/tau {worst:.3g}")
    t_clean = time.perf_counter() - t0
    product(SEED)
    clean = P.C.clone()
    M, N = P.M, P.N
    # flips whose group failed, by size: non-finite, |delta| >= 1000 tau (clear), below that (near the
    # threshold: one relation may fail alone, or several weight columns may fit the residuals)
    st = {"flips": 0, "flips_group_failed": 0, "flips_located": 0, "clear": 0, "clear_located": 0, "near": 0,
          "near_located": 0, "nonfinite": 0, "runs_all_located_and_corrected": 0, "runs_multi": 0,
          "erasures_rebuilt": 0}
    t0 = time.perf_counter()
    for r in range(args.campaign):
        P.C.copy_(clean)
        sites = []
        t = 0
        while len(sites) < 2:
            x, y, bit = synth.flip_site(SEED + 29, 4 * r + t, M, N, 0, 63)
            t += 1
            if all((x % b, y) != (u % b, v) for u, v, _ in sites):
                sites.append((x, y, bit))
        for (x, y, bit) in sites:
            v = P.C[x, y].view(torch.int64) ^ (1 << bit)
            P.C[x, y] = v.view(torch.float64)
        rep = P.verify()
        groups = {(g[0], g[1]): g[3] for g in rep.groups_c(f)}
        status, locs = abft.wlocate(P.p, rep)
        got = {(l.i, l.j) for l in locs if l.cls in (abft.ABFT_CLS_DATA, abft.ABFT_CLS_CHECKSUM)}
        st["flips"] += 2
        for (x, y, _) in sites:
            if (x % b, y) in groups:
                hit = (x, y) in got
                st["flips_group_failed"] += 1
                st["flips_located"] += hit
                delta = P.C[x, y].item() - clean[x, y].item()
                cls = ("nonfinite" if not math.isfinite(delta)
                       else "clear" if abs(delta) >= 1000 * max(groups[(x % b, y)]) else "near")
                st[cls] += 1
                if cls != "nonfinite":
                    st[cls + "_located"] += hit
        st["runs_multi"] += status != abft.ABFT_OK
        if status == abft.ABFT_OK:
            abft.wcorrect(P.p, P.C, locs, P.ws)
            rep = P.verify()
            if not (rep.n_fail_c or rep.n_fail_r) and got == {(x, y) for x, y, _ in sites if (x % b, y) in groups}:
                st["runs_all_located_and_corrected"] += 1
        # then f lost blocks of one block column
        P.C.copy_(clean)
        lost = synth.pick_distinct(SEED + 5000 + r, f, Gr + f, stream=synth.STREAM_ERASE)
        J = synth.randint(SEED, synth.STREAM_ERASE, 7000 + r, Gc + f)
        for g in lost:
            P.C[g * b:(g + 1) * b, J * b:(J + 1) * b] = float("nan")
        try:
            abft.wrecover(P.p, P.C, abft.ABFT_DIR_COL, lost, J * b, b, P.ws)
            rep = P.verify()
            err = (P.C - clean).abs().max().item() / clean.abs().max().item()
            st["erasures_rebuilt"] += bool(not (rep.n_fail_c or rep.n_fail_r) and err < 1e-10)
        except abft.AbftError:
            pass
        if r % 100 == 0:
            log(f"flip/erasure run {r}: {st}")
    out = {"campaign": args.workload, "dtype": "f64", "m": m, "n": n, "k": k, "b": b, "f": f,
           "clean_runs": args.campaign, "false_positives": fp, "max_ratio_clean": float(f"{worst:.3g}"),
           "runs": args.campaign, "flip_bits": "0..63", **st,
           "seconds": {"clean": round(t_clean, 1), "faults": round(time.perf_counter() - t0, 1)}}
    print(json.dumps(out), flush=True)


def run_chained_campaign(args):
    """Clean-run campaign of chained products: args.campaign pairs of chained
    products on fresh seeded inputs; every relation of both results must pass
    (the second's threshold carries the first's residual)."""
    import torch

    from paper_0806_3121_amd import abft, synth

    cfg = CHAINED[args.workload]
    m, n, k, b = cfg["m"], cfg["n"], cfg["k"], cfg["b"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P1 = abft.Protected(abft.ABFT_F64, m, n, k, b, b, device=dev)
    p2 = abft.problem(abft.ABFT_F64, m, n, n, b, b, lda=P1.ldc, ldb=n, ldc=P1.ldc)
    Bt2 = torch.zeros(n + b, n, dtype=torch.float64, device=dev)
    ws2 = torch.zeros(abft.workspace_size(p2), dtype=torch.uint8, device=dev)
    D = torch.zeros(m + b, P1.ldc, dtype=torch.float64, device=dev)
    host = abft.new_report_buffer()
    t0 = time.perf_counter()
    fp1 = fp2 = 0
    w1 = w2 = 0.0
    for r in range(args.campaign):
        seed = SEED + 9000 + r
        abft.fill_uniform(abft.ABFT_F64, m, k, k, 0, seed, synth.STREAM_A, P1.A)
        abft.fill_uniform(abft.ABFT_F64, k, n, k, 1, seed, synth.STREAM_B, P1.Bt)
        abft.fill_uniform(abft.ABFT_F64, n, n, n, 1, seed + 1, synth.STREAM_B, Bt2)
        P1.encode()
        P1.gemm()
        rep = P1.verify()
        fp1 += bool(rep.n_flag_c or rep.n_flag_r)
        w1 = max(w1, rep.max_ratio_c, rep.max_ratio_r)
        abft.encode_chained(p2, P1.Cbuf, Bt2, ws2, P1.p, P1.ws)
        abft.gemm(p2, P1.Cbuf, Bt2, D, ws2)
        abft.verify(p2, D, ws2, host_out=host)
        torch.cuda.current_stream().synchronize()
        rep = abft.read_report(host)
        fp2 += bool(rep.n_flag_c or rep.n_flag_r)
        w2 = max(w2, rep.max_ratio_c, rep.max_ratio_r)
        if r % 100 == 0:
            log(f"chained run {r}: false positives {fp1} / {fp2}, max |D|/tau {w1:.3g} / {w2:.3g}")
    out = {"campaign": args.workload, "dtype": "f64", "m": m, "n": n, "k": k, "b": b, "runs": args.campaign,
           "false_positives_first": fp1, "false_positives_chained": fp2, "max_ratio_first": float(f"{w1:.3g}"),
           "max_ratio_chained": float(f"{w2:.3g}"), "seconds": round(time.perf_counter() - t0, 1)}
    print(json.dumps(out), flush=True)


def run_batched_campaign(args):
    """Reliability campaign on the batched workload: clean passes over fresh
    seeded inputs until args.campaign problems have been verified (false
    positives counted per problem), then args.campaign single flips, one per
    problem of a pass (every bit position, seeded sites anywhere in C_f), each
    classified by the oracle (OracleFlips on the problem's own inputs) and
    counted per class and bit as in the single-problem campaign."""
    import torch

    from paper_0806_3121_amd import abft, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = BATCH
    br, bc = cfg["br"], cfg["bc"]
    shapes = synth.batched_shapes(SEED, cfg["count"], cfg["lo"], cfg["hi"], cfg["step"])
    Bt = abft.Batch([(m, n, k, br, bc) for (m, n, k) in shapes], device=dev, tau_mode=abft.ABFT_TAU_STAT,
                    lam=cfg["lam"])
    plan = Bt.plan

    def fill(seed):
        for q, (m, n, k) in enumerate(shapes):
            abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, seed + q, synth.STREAM_A, Bt.A32[q])
            abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, seed + q, synth.STREAM_B, Bt.Bt32[q])

    t0 = time.perf_counter()
    verified = fp = passes = 0
    worst = 0.0
    while verified < args.campaign:
        fill(SEED + 100000 + passes * len(shapes))
        abft.batch_quantize_encode(plan)
        abft.batch_gemm(plan, 0)
        abft.batch_verify(plan)
        flagged = Bt.fetch_reports()
        fp += len(flagged)
        for q in range(len(shapes)):
            r = Bt.report(q)
            worst = max(worst, r.max_ratio_c, r.max_ratio_r)
        verified += len(shapes)
        passes += 1
        log(f"clean pass {passes}: problems verified {verified}, false positives {fp}")
    t_clean = time.perf_counter() - t0

    fill(SEED)
    abft.batch_quantize_encode(plan)
    abft.batch_gemm(plan, 0)
    torch.cuda.synchronize()
    clean = [c.clone() for c in Bt.C]
    # the oracle's view of each problem that receives a flip, from the same host-generated inputs
    import numpy as np
    oracles = {}

    def oracle_of(q):
        if q not in oracles:
            m, n, k = shapes[q]
            A = synth.uniform(SEED + q, synth.STREAM_A, m, k, np.float32)
            B = synth.uniform(SEED + q, synth.STREAM_B, k, n, np.float32)
            oracles[q] = OracleFlips("bf16", A, B, br, bc, lam=cfg["lam"], carried_steps=k / 4.0)
        return oracles[q]

    st = flip_tally(32)
    t0 = time.perf_counter()
    for r in range(args.campaign):
        q = r % len(shapes)
        m, n, k = shapes[q]
        i, j, bit = synth.flip_site(SEED + 23, r, m + br, n + bc, 0, 31)
        Bt.C[q].copy_(clean[q])
        abft.inject_flip(Bt.probs[q], Bt.C[q], i, j, bit)
        abft.batch_verify(plan)
        flagged = Bt.fetch_reports()
        rep = Bt.report(q)
        loc = abft.classify(Bt.probs[q], rep)
        located = (loc.i, loc.j) == (i, j) and loc.cls in (abft.ABFT_CLS_DATA, abft.ABFT_CLS_CHECKSUM)
        dec = oracle_of(q).decide(i, j, bit)
        corrected = False
        if located:
            abft.correct(Bt.probs[q], Bt.C[q], loc)
            abft.batch_verify(plan)
            corrected = not Bt.fetch_reports() and abs(Bt.C[q][i, j].item() - clean[q][i, j].item()) <= dec["tau"]
        flip_count(st, bit, dec, q in flagged, located, corrected)
        if dec["class"] == "above" and not (located and corrected):
            log(f"flip run {r}: problem {q} ({i},{j}) bit {bit} above the oracle's thresholds but not repaired")
        Bt.C[q].copy_(clean[q])
        if r % 100 == 0:
            log(f"flip run {r}: above {st['above']} (gpu located {st['above_gpu_located']}), gray {st['gray']}, "
                f"below {st['below']}")
    t_flip = time.perf_counter() - t0
    out = {"campaign": "c5", "dtype": "bf16", "problems": len(shapes), "br": br, "bc": bc,
           "clean_problem_runs": verified, "clean_passes": passes, "false_positives": fp,
           "max_ratio_clean": round(worst, 4), "flip_runs": args.campaign, "flip_bits": "0..31", **st,
           "seconds": {"clean": round(t_clean, 1), "flips": round(t_flip, 1)}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the unprotected-kernel timing (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tile-cache", default=os.path.join(ROOT, "paper_0806_3121_amd", "batch_tiles.txt"),
                    help="batched workload: tile-shape tuning cache (read, and written after a tuning run)")
    ap.add_argument("--no-targets", action="store_true",
                    help="default workload only: skip the target-shape products (binary64 b = 1, bfloat16 and FP8 "
                         "n = 16384) and the peak probes")
    ap.add_argument("--site", choices=["m", "k"], default="m",
                    help="where the step's flip lands: m = C in memory after the product (re-reading verify), "
                         "k = an accumulator inside the product kernel (b = 1 workloads: fused partial sums, "
                         "fused verify)")
    ap.add_argument("--inputs", choices=["uniform", "heavy"], default="uniform",
                    help="campaign inputs: uniform [-1, 1), or heavy (binary32 workloads): N(0,1) with 1%% of the "
                         "entries scaled by 1e3")
    ap.add_argument("--campaign", type=int, default=0,
                    help="run N clean products and N single flips instead of the benchmark, print the tallies")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the path is built and measured on one "
                                   "MI355X; sharding across GPUs is not built", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.campaign:
        if args.workload in WEIGHTED:
            return run_weighted_campaign(args)
        if args.workload in CHAINED:
            return run_chained_campaign(args)
        if args.workload in PANELS or args.workload in GEMV or args.workload in BLOCK_CYCLIC:
            print(json.dumps({"error": f"--campaign is not defined for workload {args.workload}"}))
            sys.exit(2)
        return run_batched_campaign(args) if args.workload == "c5" else run_campaign(args)
    if args.workload == "c5":
        return run_batched(args)
    if args.workload in WEIGHTED:
        return run_weighted(args)
    if args.workload in CHAINED:
        return run_chained(args)
    if args.workload in GEMV:
        return run_gemv(args)
    if args.workload in BLOCK_CYCLIC:
        return run_block_cyclic(args)

    import torch

    from paper_0806_3121_amd import abft, synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    dt_name, m, n, k, b, erase = WORKLOADS[args.workload]
    adt = {"f64": abft.ABFT_F64, "f32": abft.ABFT_F32, "bf16": abft.ABFT_BF16, "fp8": abft.ABFT_FP8_E4M3}[dt_name]
    tdt = torch.float64 if dt_name == "f64" else torch.float32
    lowp = dt_name in ("bf16", "fp8")
    bit_lo, bit_hi = FLIP_BITS[dt_name]

    log(f"workload {args.workload}: {dt_name} m={m} n={n} k={k} b={b}")
    P = abft.Protected(adt, m, n, k, b, b, device=dev)
    if lowp:
        # binary32 inputs resident in HBM; each step quantizes them
        A32 = torch.empty(m, k, dtype=torch.float32, device=dev)
        Bt32 = torch.empty(n, k, dtype=torch.float32, device=dev)
        abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED, synth.STREAM_A, A32)
        abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED, synth.STREAM_B, Bt32)
    else:
        abft.fill_uniform(adt, m, k, k, 0, SEED, synth.STREAM_A, P.A)
        # B (k x n) stored column-major: the Bt tensor holds B^T row-major
        abft.fill_uniform(adt, k, n, k, 1, SEED, synth.STREAM_B, P.Bt)
    Cplain = torch.empty(m, n, dtype=tdt, device=dev)
    pplain = abft.problem(adt, m, n, k, b, b, ldc=n)
    torch.cuda.synchronize()

    g_events = []

    n_panels = PANELS.get(args.workload, 0)
    site_k = args.site == "k"
    if site_k and (b != 1 or n_panels):
        print(json.dumps({"error": "--site k needs a b = 1 workload (c1, c2b1, c3, c4, c4fp8)"}))
        sys.exit(2)
    v_events = []

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        return (e0, e1)

    def panel(q):
        k0, k1 = q * k // n_panels, (q + 1) * k // n_panels
        return timed(lambda: abft.gemm_panel(P.p, P.A, P.Bt, P.C, k0, k1, abft.ABFT_ACCUMULATE if q else 0))

    def repair(s):
        rect = None
        if erase:
            I, J = synth.erase_block(SEED, s, m // b, n // b)
            rect = (I * b, J * b, b, b)
        i, j, bit = synth.flip_site(SEED, s, m, n, bit_lo, bit_hi, avoid=rect)
        if not site_k:
            abft.inject_flip(P.p, P.C, i, j, bit)
        known = [rect] if rect else None
        if rect:
            abft.inject_erase(P.p, P.C, rect)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if site_k:
            abft.verify_fused(P.p, P.C, P.ws, host_out=P.rep_host)
        else:
            abft.verify(P.p, P.C, P.ws, known=known, host_out=P.rep_host)
        e1.record(stream)
        v_events.append((e0, e1))
        stream.synchronize()              # the host classifies the report
        rep = abft.read_report(P.rep_host)
        loc = abft.classify(P.p, rep, known=known)
        if (loc.cls, loc.i, loc.j) != (abft.ABFT_CLS_DATA, i, j):
            raise RuntimeError(f"step {s}: flip at ({i},{j}) bit {bit} classified as {loc.cls} ({loc.i},{loc.j})")
        abft.correct(P.p, P.C, loc)
        if rect:
            abft.recover_block(P.p, P.C, rect)

    def step(s):
        if lowp:
            # quantize both binary32 operands and encode them in one pass
            abft.quantize_encode(P.p, A32, Bt32, P.A, P.Bt, P.ws)
        else:
            P.encode()
        if n_panels:
            # rank-(k/n_panels) updates; repair half-way through the loop
            ev = [panel(q) for q in range(n_panels // 2)]
            repair(s)
            ev += [panel(q) for q in range(n_panels // 2, n_panels)]
            g_events.append(ev)
        elif site_k:
            # the step's flip happens inside the product kernel (one accumulator bit before the epilogue)
            i, j, bit = synth.flip_site(SEED, s, m, n, bit_lo, bit_hi)
            g_events.append([timed(lambda: P.gemm_fault(i, j, bit, abft.ABFT_FUSED))])
            repair(s)
        else:
            g_events.append([timed(P.gemm)])
            repair(s)
        rep = P.verify()
        if rep.n_flag_c or rep.n_flag_r:
            raise RuntimeError(f"step {s}: not clean after repair")

    for s in range(args.warmup):
        step(1000 + s)
    g_events.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {dt:.3f} s")
    # per step: the product's launches (all panels of the loop)
    gemm_ms = sum(sum(a.elapsed_time(c) for a, c in ev) for ev in g_events) / len(g_events)
    verify_ms = sum(a.elapsed_time(c) for a, c in v_events[-args.steps:]) / max(1, min(len(v_events), args.steps))

    # plain product of the same kernel (no checksum rows/columns)
    pe = []
    for s in range(0 if args.no_plain else max(3, min(args.steps, 10))):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        abft.gemm(pplain, P.A, P.Bt, Cplain, P.ws, flags=abft.ABFT_PLAIN)
        e1.record(stream)
        pe.append((e0, e1))
    torch.cuda.synchronize()
    plain_ms = sum(a.elapsed_time(c) for a, c in pe[1:]) / len(pe[1:]) if pe else None
    peak = PEAK[dt_name]

    useful = 2.0 * m * n * k
    executed = 2.0 * (m + b) * (n + b) * k
    ms_step = dt / args.steps * 1e3
    value = useful / (ms_step * 1e-3) / 1e12
    achieved = executed / (gemm_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt_name,
        "data": "synthetic",
        "config": {"workload": f"{dt_name.upper()} protected GEMM {args.workload}: m={m} n={n} k={k}, checksum blocks "
                               f"{b}x{b} ({f'{m // b}x{n // b} grid, one erased block + one flip per step' if erase else 'one flip per step'})"
                               + (f"; product as {n_panels} rank-{k // n_panels} panel updates, repaired after panel "
                                  f"{n_panels // 2}" if n_panels else "")
                               + ("; the flip is an accumulator bit inside the product kernel, detected from the "
                                  "fused epilogue partial sums" if site_k else ""),
                   "site": args.site,
                   "m": m, "n": n, "k": k, "br": b, "bc": b, "global_batch": 1, "seq_len": 0,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4),
                     # the counters were taken on the site-M product (the fused epilogue is another kernel)
                     "traffic": None if site_k else TRAFFIC.get(args.workload),
                     "kernel": abft.describe_gemm(P.p, abft.ABFT_FUSED if site_k else 0)
                               + (f", {n_panels} accumulating panel launches per product" if n_panels else ""),
                     "flops_per_launch": executed / max(1, n_panels),
                     "avg_launch_ms": round(gemm_ms / max(1, n_panels), 4)},
        "pct_mfma_peak_useful": round(100 * value / peak, 2),
        "gemm_protected_ms": round(gemm_ms, 4),
        "gemm_plain_ms": round(plain_ms, 4) if plain_ms else None,
        "abft_overhead_pct": round(100 * (gemm_ms / plain_ms - 1), 2) if plain_ms else None,
        "abft_floor_pct": round(100 * (executed / useful - 1), 2),
        "first_verify_ms": round(verify_ms, 4),
    }
    if args.workload == "c2" and not args.no_targets:
        # the products the targets are stated for (>= 70 % of the dtype's peak, <= 10 % overhead), timed in
        # this same run, and the measured peaks the fractions can also be read against
        log("target-shape products ...")
        out["targets"] = {name: measure_product(torch, abft, synth, name) for name in ("c2b1", "c4", "c4fp8")}
        log("peak probes ...")
        probes = run_probes(torch, abft)
        out["probes"] = probes
        out["roofline"]["probe_peak"] = probes["mfma_f64_tflops"]
        out["roofline"]["frac_of_probe"] = round(achieved / probes["mfma_f64_tflops"], 4)
        for name, key in (("c2b1", "mfma_f64_tflops"), ("c4", "mfma_bf16_tflops")):
            t = out["targets"][name]
            t["frac_of_probe"] = round(t["frac"] * t["peak"] / probes[key], 4)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        tf, thr, sec, rows, Cref, Cu, single = cpu_baseline(dt_name, m, n, k, b, args.cpu_seconds)
        out["cpu_baseline"] = {"value": round(tf, 6), "unit": "TFLOP/s", "cores": thr, "kind": "oracle",
                               "sample": f"rows 0..{rows - 1} of the encoded product C_f = A_f B_f "
                                         f"({rows} x {n + b} x {k}, FP64 i-l-j loops), {sec:.1f} s",
                               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                               "single_core": {"value": round(single[0], 6), "unit": "TFLOP/s", "cores": 1,
                                               "sample": f"rows 0..{single[1] - 1} of the same product, "
                                                         f"{single[2]:.1f} s"}}
        # the last step's repaired C_f against the oracle's rows (the same seeded inputs, quantized by the
        # oracle's own rounding for bfloat16 / FP8)
        out["oracle_check"] = {"rows": rows, "cols": n + b, "max_rel_err": oracle_check(P.C, Cref, n + b),
                               "bound": TOL_VS_ORACLE[dt_name]}
        if Cu is not None:
            # what the quantization of the inputs costs: the result against the unquantized product
            out["oracle_check"]["max_rel_err_vs_unquantized"] = oracle_check(P.C, Cu, n)
            out["oracle_check"]["unquantized_rows"] = int(Cu.shape[0])
    if not args.no_cpu_baseline and dt_name != "fp8":
        # FP8 results carry the operands' scale factors, which stay on the device
        log("residual check ...")
        out["residual_check"] = {"rho": residual_rho(P.A, P.Bt, P.C, m, n, k, 2.0 ** -53 if dt_name == "f64"
                                                     else 2.0 ** -24), "bound": 10.0}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
