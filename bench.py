"""Benchmark: 3D R2C + C2R round trip of a 1024^3 FP64 grid on one MI355X.

One step = the whole hot path once through the public calls: gfft_exec_r2c
(z pass, y pass, x pass) and gfft_exec_c2r (x, y, z passes with the 1/N^3
normalization fused), on a synthetic seeded uniform[-1,1) field already
resident in HBM.  `value` is the wall-clock rate of those K steps; HIP events
around each step give its median and minimum.  An instrumented repeat of the
same K steps through the single-pass entry points, with HIP events between
the passes on the launch stream, gives each kernel's live duration (the
roofline figure).  Two yardsticks sit beside it: the library's streaming
copy (contiguous traffic) and the y and x passes' loads and stores without
their transform (the ceiling of their access pattern).

Prints ONE JSON line (rank 0).  Run ``python bench.py --help`` for options.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import torch

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, published

METRIC = ("3D R2C+C2R GFLOP/s and % HBM roofline per GPU at 1024^3 FP64 "
          "(vs FP32/adjoint)")


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32 and adjoint lines")
    ap.add_argument("--cpu-planes", type=int, default=512,
                    help="x-planes (and pencil columns) in the oracle sample")
    ap.add_argument("--traffic", default=None,
                    help="PMC traffic summary (default: the committed 1024^3 FP64 one)")
    ap.add_argument("--only", choices=sorted(ONLY), default=None,
                    help="time one other workload group alone and print its JSON "
                         "(for profiling it); no 1024^3 line")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "full_1024_f64_pmc_traffic.md")


def kernel_source_hash() -> str:
    """Hash of the HIP sources, to tell whether recorded counters still apply."""
    import glob
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "paper_2202_12756_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(path: str, pass_name: str):
    """Calibrated HBM bytes per launch of `pass_name` from the PMC summary,
    or None when the summary is missing or the kernels changed since."""
    if not os.path.exists(path):
        return None
    sha, rows, col = None, {}, None
    with open(path) as fh:
        for line in fh:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if line.startswith("kernel_source_sha256_16:"):
                sha = line.split(":", 1)[1].strip()
            elif line.startswith("| pass"):
                col = cells.index("HBM bytes (scaled)") if "HBM bytes (scaled)" in cells else None
            elif line.startswith("| ") and col is not None and len(cells) > col \
                    and cells[col].isdigit():
                rows[cells[0]] = int(cells[col])
    if sha != kernel_source_hash():
        return None
    return rows.get(pass_name)


def gflop_pair(n: int) -> float:
    """5 (N^3/2) log2 N^3 per R2C, twice per forward+inverse pair."""
    return 2 * 5.0 * (n ** 3 / 2) * math.log2(n ** 3) / 1e9


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(n: int, planes: int, seed: int, min_seconds: float, max_reps: int):
    """Repeat the oracle sample until `min_seconds` have passed; return
    (repetitions, seconds, GFLOP per repetition)."""
    import oracle
    import synth

    k = n // 2 + 1
    f = synth.uniform((planes, n, n), seed, torch.float64).numpy()
    pen = (synth.uniform((n, planes, k), seed + 1, torch.float64).numpy()
           + 1j * synth.uniform((n, planes, k), seed + 2, torch.float64).numpy())
    reps = 0
    t0 = time.perf_counter()
    while True:
        g = oracle.r2c2d_planes(f)
        oracle.c2r2d_planes(g, n, 1.0 / n ** 3)
        h = oracle.x_c2c(pen, -1)
        oracle.x_c2c(h, +1)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or reps >= max_reps:
            break
    # nominal flops: one third of 5 (N^3/2) log2 N^3 per axis and direction,
    # pro rata for `planes` of N planes (y and z lines) and `planes` of N
    # pencil columns (x lines)
    per_rep = gflop_pair(n) / 3.0 * (2 * planes / n + planes / n)
    return reps, dt, per_rep


def cpu_baseline(n: int, planes: int, seed: int, min_seconds: float = 10.0) -> dict:
    """Time the FP64 oracle on a bounded sample of the same workload.

    Sample: the forward 2D R2C (z and y lines) and its inverse on `planes`
    x-planes of the N^3 grid, plus the forward and inverse x lines of a
    [N][planes][K] pencil, on all the oracle's OpenMP threads; then a
    sixteenth of that sample on one thread.  The nominal flop count of those
    lines (one third of 5 (N^3/2) log2 N^3 per axis, pro rata) over the wall
    time gives a rate in the metric's unit.
    """
    import oracle

    k = n // 2 + 1
    threads = oracle.num_threads()
    reps, dt, per_rep = _oracle_sample(n, planes, seed, min_seconds, 20)
    one_planes = max(1, planes // 16)
    oracle.set_num_threads(1)
    try:
        reps1, dt1, per_rep1 = _oracle_sample(n, one_planes, seed, min_seconds / 2, 20)
    finally:
        oracle.set_num_threads(threads)
    slab = _oracle_slab_4096_sample(seed)
    return {"value": round(reps * per_rep / dt, 3), "unit": "GFLOP/s",
            "cores": threads, "kind": "oracle",
            "sample": (f"radix-2 FP64 oracle: 2D R2C+C2R on {planes} of {n} "
                       f"x-planes and x-line C2C fwd+inv on a [{n}][{planes}][{k}] "
                       f"pencil, repeated {reps}x; {dt:.2f} s wall, rate = nominal flops of those "
                       f"lines / time"),
            "seconds": round(dt, 3),
            "cpu_model": cpu_model(),
            "one_core": {"value": round(reps1 * per_rep1 / dt1, 3), "unit": "GFLOP/s",
                         "sample": (f"the same sample on {one_planes} planes and a "
                                    f"[{n}][{one_planes}][{k}] pencil, one thread, "
                                    f"repeated {reps1}x"),
                         "seconds": round(dt1, 3)},
            "slab_4096_p64_f64": slab}


def _oracle_slab_4096_sample(seed: int) -> dict:
    """The 4096^3 / 64-rank slab share's forward work on the oracle, scaled:
    the 2D R2C of one of the 64 x-planes and the x lines of one of the 64
    y_l slices of the received pencil, each timed once on all threads and
    multiplied by 64 (labelled as scaled)."""
    import oracle
    import synth

    n, planes = 4096, 64
    k = n // 2 + 1
    f = synth.uniform((1, n, n), seed + 10, torch.float64).numpy()
    pen = (synth.uniform((n, 1, k), seed + 11, torch.float64).numpy()
           + 1j * synth.uniform((n, 1, k), seed + 12, torch.float64).numpy())
    t0 = time.perf_counter()
    oracle.r2c2d_planes(f)
    t1 = time.perf_counter()
    oracle.x_c2c(pen, -1)
    t2 = time.perf_counter()
    fwd = planes * ((t1 - t0) + (t2 - t1))
    gflop = 5.0 * (n ** 3 / 2) * math.log2(n ** 3) / planes / 1e9
    return {"scaled_forward_ms": round(fwd * 1e3, 1), "GFLOPs": round(gflop / fwd, 3),
            "sample": (f"2D R2C of one 4096x4096 plane ({(t1 - t0) * 1e3:.1f} ms) and the x lines "
                       f"of one [4096][1][2049] pencil slice ({(t2 - t1) * 1e3:.1f} ms), each x64 "
                       f"(scaled, not run on the whole share)")}


def time_pairs(fn, steps: int, warmup: int) -> float:
    """Average ms of fn() over `steps` calls (after `warmup`), HIP events."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def pattern_copies(plan, ydata, xdata, nbytes: int, steps: int = 5) -> dict:
    """GB/s of the y and x passes' loads and stores without their transform
    (gfft_exec_pass_copy; the data end up conjugated an odd number of times),
    nbytes read and written per launch."""
    out = {}
    for ax, key, data in ((0, "y", ydata), (1, "x", xdata)):
        ms = time_pairs(lambda: plan.pass_copy(data, ax), steps, 1)
        out[key] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    return out


def time_stats(fn, steps: int, warmup: int) -> dict:
    """Per-call HIP-event times of fn() over `steps` calls (after `warmup`):
    mean, median and min in ms, events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return {"mean_ms": round(sum(ts) / len(ts), 4), "median_ms": round(ts[len(ts) // 2], 4),
            "min_ms": round(ts[0], 4)}


def variants(n: int, steps: int, x64: torch.Tensor, dev) -> dict:
    """The FP32 forms and the adjoint pair beside the FP64 line.

    fp32, fp32_mfma_bf16x2, fp32_mfma_bf16x3: the same round trip on the FP32
    values of the FP64 input, with every stage on the vector ALUs or with the
    first radix-16 stage of the y and x passes on the matrix cores (2 or 3
    BF16 terms per operand); each forward spectrum is compared with the FP64
    path's on the same GPU.
    slab_pack_p8_f64: the slab transpose (the paper's steps 2-4) for rank 0
    of 8: the standalone pack into 8 send chunks, and the local 2D R2C with
    and without the pack fused into the z pass's stores.
    adjoint_f64: the gradient pair of a loss through both transforms,
    C2R^T (scale w R2C) then R2C^T (C2R(G/w)), on the FP64 input.
    """
    from paper_2202_12756_amd import Plan

    out = {}
    gflop = gflop_pair(n)
    k = n // 2 + 1
    p64 = Plan(n, torch.float64, device=dev)
    F64 = p64.r2c(x64)
    f64_norm = torch.linalg.vector_norm(F64).item()
    x32 = x64.float()
    R, C = n ** 3 * 4, n * n * k * 8
    for name, terms in (("fp32", 0), ("fp32_mfma_bf16x2", 2), ("fp32_mfma_bf16x3", 3)):
        p32 = Plan(n, torch.float32, device=dev, mfma_terms=terms)
        F32 = p32.r2c(x32)
        fwd_err = (torch.linalg.vector_norm(F32.to(torch.complex128) - F64).item()
                   / f64_norm)
        y32 = p32.empty_real()
        ms = time_pairs(lambda: (p32.r2c(x32, F32), p32.c2r(F32, y32, 1.0 / n ** 3)),
                        steps, 2)
        rt = (torch.linalg.vector_norm(y32.double() - x64)
              / torch.linalg.vector_norm(x64)).item()
        out[name] = {"ms_per_pair": round(ms, 4), "GFLOPs": round(gflop / (ms * 1e-3), 2),
                     "pair_hbm_roofline_frac": round(2 * (R + 5 * C) / (ms * 1e-3) / 1e9
                                                     / PEAK_HBM_GBS, 4),
                     "forward_rel_l2_vs_fp64_path": fwd_err,
                     "roundtrip_rel_l2_vs_fp64_input": rt}
        if terms == 0:
            out[name]["pattern_copy_GBps"] = pattern_copies(p32, F32, F32, 2 * C)
        del F32, y32, p32
        torch.cuda.empty_cache()
    del x32, F64
    torch.cuda.empty_cache()
    out.update(slab_pack_p8(steps, dev, x64 if n == 1024 else None))
    # adjoint pair in FP64
    G = p64.empty_spectrum()
    h = p64.empty_real()
    ms = time_pairs(lambda: (p64.c2r_adjoint(x64, G, 1.0 / n ** 3),
                             p64.r2c_adjoint(G, h, 1.0)), steps, 2)
    R, C = n ** 3 * 8, n * n * k * 16
    out["adjoint_f64"] = {"ms_per_pair": round(ms, 4),
                          "GFLOPs": round(gflop / (ms * 1e-3), 2),
                          "pair_hbm_roofline_frac": round(2 * (R + 5 * C) / (ms * 1e-3)
                                                          / 1e9 / PEAK_HBM_GBS, 4)}
    del G, h, p64
    torch.cuda.empty_cache()
    out.update(kolmogorov_512(steps, dev))
    out.update(losses_8x256(steps, dev))
    out.update(slab_share_4096(steps, dev))
    out.update(pencil_variants(steps, dev))
    out.update(graph_variants(steps, dev))
    out.update(full_grid_2048(steps, dev))
    return out


def slab_pack_p8(steps: int, dev, x64: torch.Tensor | None = None) -> dict:
    """The slab transpose of the paper's steps 2-4 at p = 8 on the 1024^3 FP64
    grid (rank 0: X = 128 planes, chunks of 128 x 128 x 513): the standalone
    pack into the 8 send chunks, and the local 2D R2C (step 1) with and
    without the pack fused into the z pass's stores (send buffers compared
    bit for bit)."""
    import synth
    from paper_2202_12756_amd import Plan

    n, ranks = 1024, 8
    k = n // 2 + 1
    ps = Plan(n, torch.float64, slab_x=n // ranks, device=dev)
    pf = Plan(n, torch.float64, slab_x=n // ranks, fuse_pack=True, device=dev)
    if x64 is not None:
        xs = x64[0, : n // ranks].contiguous()
    else:
        xs = synth.uniform(ps.real_shape, 3, torch.float64, dev)
    S = ps.r2c(xs)
    send = torch.empty(ps.send_shape, dtype=torch.complex128, device=dev)
    pack = time_stats(lambda: ps.pack(S, send), steps, 2)
    unfused = time_stats(lambda: (ps.r2c(xs, S), ps.pack(S, send)), steps, 2)
    send2 = torch.empty_like(send)
    fused = time_stats(lambda: pf.r2c(xs, send2), steps, 2)
    cs = S.numel() * 16
    out = {"slab_pack_p8_f64": {
        "chunk": f"{n // ranks}x{n // ranks}x{k}",
        "pack_ms": pack["mean_ms"], "pack": pack,
        "pack_GBps": round(2 * cs / (pack["median_ms"] * 1e-3) / 1e9, 1),
        "r2c2d_then_pack_ms": unfused["mean_ms"], "r2c2d_then_pack": unfused,
        "r2c2d_fused_pack_ms": fused["mean_ms"], "r2c2d_fused_pack": fused,
        "fused_equals_standalone": bool(torch.equal(send, send2)),
    }}
    del ps, pf, xs, S, send, send2
    torch.cuda.empty_cache()
    return out


def full_grid_2048(steps: int, dev) -> dict:
    """The paper's 2048^3 grid held whole on one GPU (FP64: 137 GB for the
    field and its half spectrum), round trip in FP64 and FP32.  The inverse
    writes back into the input buffer, so two buffers suffice; the round-trip
    error is checked on the first 64 planes of the first pair."""
    import synth
    from paper_2202_12756_amd import Plan

    n, out = 2048, {}
    k = n // 2 + 1
    gflop = gflop_pair(n)
    for dtype, b, name in ((torch.float64, 8, "full_2048_f64"), (torch.float32, 4, "full_2048_f32")):
        p = Plan(n, dtype, device=dev)
        x = torch.empty(p.real_shape, dtype=dtype, device=dev)
        for s0 in range(0, n, 256):
            x[0, s0:s0 + 256] = synth.uniform((256, n, n), 6, dtype, dev, offset=s0 * n * n)
        head = x[0, :64].clone()
        F = p.empty_spectrum()
        pair = lambda: (p.r2c(x, F), p.c2r(F, x, 1.0 / n ** 3))
        pair()
        rel = (torch.linalg.vector_norm(x[0, :64] - head) / torch.linalg.vector_norm(head)).item()
        ms = time_pairs(pair, min(steps, 5), 1)
        R, C = n ** 3 * b, n * n * k * 2 * b
        out[name] = {"ms_per_pair": round(ms, 3), "GFLOPs": round(gflop / (ms * 1e-3), 2),
                     "pair_hbm_roofline_frac": round(2 * (R + 5 * C) / (ms * 1e-3) / 1e9
                                                     / PEAK_HBM_GBS, 4),
                     "roundtrip_rel_l2_first_64_planes": rel}
        del p, x, F, head
        torch.cuda.empty_cache()
    return out


def graph_variants(steps: int, dev) -> dict:
    """Small transforms whose kernels last tens of microseconds, eager and as
    one replayed HIP graph (the exec calls only enqueue kernels, so a
    forward + inverse pair captures as is): 8 x 256^3 FP32 round trip, and
    the local forward chain of a 64 x 128 pencil share of 4096^3 FP64."""
    import synth
    from paper_2202_12756_amd import PencilPlan, Plan

    def capture(fn):
        s = torch.cuda.Stream(dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream(dev).wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        return g

    out = {}
    n = 256
    p = Plan(n, torch.float32, batch=8, device=dev)
    x = synth.uniform(p.real_shape, 5, torch.float32, dev)
    F, y = p.empty_spectrum(), p.empty_real()
    pair = lambda: (p.r2c(x, F), p.c2r(F, y, 1.0 / n ** 3))
    eager = time_pairs(pair, steps, 2)
    g = capture(pair)
    graph = time_pairs(g.replay, steps, 2)
    out["graph_8x256_f32_pair"] = {"eager_ms": round(eager, 4), "graph_ms": round(graph, 4)}
    del p, x, F, y, g
    pp = PencilPlan(4096, torch.float64, (64, 128), 0, device=dev)
    xr = synth.uniform(pp.real_shape, 11, torch.float64, dev)
    send = torch.empty(pp.send_shape, dtype=torch.complex128, device=dev)
    yp = torch.view_as_complex(synth.uniform(pp.ypencil_shape + (2,), 12, torch.float64, dev))
    xp = torch.view_as_complex(synth.uniform(pp.xpencil_shape + (2,), 13, torch.float64, dev))
    chain = lambda: (pp.z_r2c(xr, send), pp.y_c2c(yp, -1), pp.x_c2c(xp, -1))
    eager = time_pairs(chain, steps, 2)
    g = capture(chain)
    graph = time_pairs(g.replay, steps, 2)
    out["graph_pencil_4096_64x128_f64_chain"] = {"eager_ms": round(eager, 4),
                                                 "graph_ms": round(graph, 4)}
    del pp, xr, send, yp, xp, g
    torch.cuda.empty_cache()
    return out


def slab_share_4096(steps: int, dev) -> dict:
    """Rank 0's slab share of a 4096^3 FP64 grid over 64 ranks: the local
    2D R2C of the 64 x 4096 x 4096 real slab with the z pass storing the 64
    all-to-all send blocks of 64 x 64 x 2049 (pack fused), the y pass on the
    send blocks, and the x pass on a synthetic received pencil [4096][64][2049]
    (the exchange is the caller's).  Bytes per pass: z reads the slab and
    writes the send buffer, y and x read and write their array in place."""
    import synth
    from paper_2202_12756_amd import Plan

    n, ranks = 4096, 64
    X = n // ranks
    p = Plan(n, torch.float64, slab_x=X, fuse_pack=True, device=dev)
    xr = synth.uniform(p.real_shape, 4, torch.float64, dev)
    send = p.empty_spectrum()
    pen = torch.view_as_complex(synth.uniform(p.pencil_shape + (2,), 40, torch.float64, dev))
    ms = {"z_r2c_send": time_pairs(lambda: p.z_r2c(xr, send), steps, 2),
          "y_fwd": time_pairs(lambda: p.y_c2c(send, -1), steps, 2),
          "x_fwd": time_pairs(lambda: p.x_c2c(pen, -1), steps, 2)}
    bts = {"z_r2c_send": xr.numel() * 8 + send.numel() * 16,
           "y_fwd": 2 * send.numel() * 16, "x_fwd": 2 * pen.numel() * 16}
    chain = time_pairs(lambda: (p.r2c(xr, send), p.x_c2c(pen, -1)), steps, 2)
    out = {"slab_4096_p64_f64": {
        "real_slab": f"{X}x{n}x{n}", "send_blocks": f"{ranks}x{X}x{X}x{n // 2 + 1}",
        "pass_ms": {k: round(v, 4) for k, v in ms.items()},
        "pass_GBps": {k: round(bts[k] / (ms[k] * 1e-3) / 1e9, 1) for k in ms},
        "pattern_copy_GBps": pattern_copies(p, send, pen, bts["y_fwd"]),
        "chain_ms": round(chain, 4),
        "chain_hbm_roofline_frac": round(sum(bts.values()) / (chain * 1e-3) / 1e9
                                         / PEAK_HBM_GBS, 4),
    }}
    del p, xr, send, pen
    torch.cuda.empty_cache()
    return out


def pencil_variants(steps: int, dev) -> dict:
    """One rank's local forward chain of a pencil-decomposed 4096^3 FP64 grid
    (z R2C into the first-exchange order, y pass on the received y-pencil,
    for pr > pc the second exchange's pack, x pass on the received x-pencil;
    the exchanges are the caller's), for rank (0, 0) of a 16 x 32 grid (512
    ranks, the paper's largest count), of a 64 x 128 grid (8192 ranks > N)
    and of a 64 x 32 grid (pr > pc).  Bytes per pass: z reads the real
    pencil and writes the first-exchange buffer, y and x read and write their
    pencil in place."""
    import synth
    from paper_2202_12756_amd import PencilPlan

    n, out = 4096, {}
    for pr, pc in ((16, 32), (64, 128), (64, 32)):
        p = PencilPlan(n, torch.float64, (pr, pc), 0, device=dev)
        xr = synth.uniform(p.real_shape, 11, torch.float64, dev)
        send = torch.empty(p.send_shape, dtype=torch.complex128, device=dev)
        yp = torch.view_as_complex(synth.uniform(p.ypencil_shape + (2,), 12, torch.float64, dev))
        xp = torch.view_as_complex(synth.uniform(p.xpencil_shape + (2,), 13, torch.float64, dev))
        ms = {"z_r2c": time_pairs(lambda: p.z_r2c(xr, send), steps, 2),
              "y_fwd": time_pairs(lambda: p.y_c2c(yp, -1), steps, 2)}
        bts = {"z_r2c": xr.numel() * 8 + send.numel() * 16, "y_fwd": 2 * yp.numel() * 16}
        if p.h > 1:        # pr > pc: the second exchange's pack
            send2 = torch.empty(p.send2_shape, dtype=torch.complex128, device=dev)
            ms["pack2"] = time_pairs(lambda: p.pack2(yp, send2), steps, 2)
            bts["pack2"] = 2 * yp.numel() * 16
            del send2
        ms["x_fwd"] = time_pairs(lambda: p.x_c2c(xp, -1), steps, 2)
        bts["x_fwd"] = 2 * xp.numel() * 16
        total_ms = sum(ms.values())
        out[f"pencil_4096_{pr}x{pc}_f64"] = {
            "ranks": pr * pc, "real_pencil": f"{p.x}x{p.y}x{n}", "kz_width": p.w,
            "pass_ms": {k: round(v, 4) for k, v in ms.items()},
            "pass_GBps": {k: round(bts[k] / (ms[k] * 1e-3) / 1e9, 1) for k in ms},
            "chain_ms": round(total_ms, 4),
            "chain_hbm_roofline_frac": round(sum(bts.values()) / (total_ms * 1e-3) / 1e9
                                             / PEAK_HBM_GBS, 4),
        }
        del p, xr, send, yp, xp
        torch.cuda.empty_cache()
    return out


def _hermitian_part(G: torch.Tensor) -> torch.Tensor:
    """The half spectrum a real field actually has when C2R is applied to G:
    on the kz = 0 and kz = N/2 planes, (G(k) + conj G(-k)) / 2; elsewhere G."""
    H = G.clone()
    n = G.shape[-2]
    for kz in (0, G.shape[-1] - 1):
        pl = G[..., kz]
        mirror = torch.roll(torch.flip(pl, dims=(-2, -1)), shifts=(1, 1), dims=(-2, -1))
        H[..., kz] = 0.5 * (pl + mirror.conj())
    assert H.shape[-2] == n
    return H


def _kolmogorov_fields(n: int, seeds, dev):
    """Unit-rms real fields [len(seeds), N, N, N] (FP64, on the GPU) from the
    seeded half spectra of synth.kolmogorov_half_spectrum, turned into real
    space by this library's FP64 C2R; returns (fields, exact half spectra of
    the fields).  For f = C2R(G) / s the forward transform is exactly
    N^3 H(G) / s, H the Hermitian part of G (R2C o C2R = N^3 H), so the
    second value is the exact spectrum of the generated input."""
    import synth
    from paper_2202_12756_amd import Plan

    p = Plan(n, torch.float64, batch=len(seeds), device=dev)
    G = torch.stack([torch.from_numpy(synth.kolmogorov_half_spectrum(n, s)) for s in seeds])
    G = G.view(p.spectrum_shape).to(dev)
    f = p.c2r(G.clone(), scale=1.0)
    rms = f.pow(2).mean(dim=(1, 2, 3), keepdim=True).sqrt()
    f /= rms
    exact = _hermitian_part(G) * (float(n) ** 3 / rms)
    del G, p
    return f, exact


def kolmogorov_512(steps: int, dev) -> dict:
    """The 512^3 k^-5/3 Gaussian field (seed 2), forward + inverse pair in
    FP64 and in FP32 (the FP32 values of the same field).  Errors: each
    forward spectrum against the exact spectrum of its generator, and the
    FP32 spectrum against the FP64 path on the FP32 values themselves."""
    from paper_2202_12756_amd import Plan

    n = 512
    k = n // 2 + 1
    f64, exact = _kolmogorov_fields(n, [2], dev)
    out, ref32 = {}, None
    for dtype, b, name in ((torch.float64, 8, "kolmogorov_512_f64"),
                           (torch.float32, 4, "kolmogorov_512_f32")):
        p = Plan(n, dtype, device=dev)
        x = f64.to(dtype)
        F = p.r2c(x)
        cF = F.to(torch.complex128)
        entry = {"rel_l2_vs_exact_spectrum": (torch.linalg.vector_norm(cF - exact)
                                              / torch.linalg.vector_norm(exact)).item()}
        if dtype == torch.float32:
            ref32 = Plan(n, torch.float64, device=dev).r2c(x.double())
            entry["rel_l2_vs_fp64_path_same_input"] = (
                torch.linalg.vector_norm(cF - ref32) / torch.linalg.vector_norm(ref32)).item()
            del ref32
        y = p.empty_real()
        st = time_stats(lambda: (p.r2c(x, F), p.c2r(F, y, 1.0 / n ** 3)), steps, 2)
        entry["roundtrip_rel_l2"] = (torch.linalg.vector_norm(y.double() - x.double())
                                     / torch.linalg.vector_norm(x.double())).item()
        R, C = n ** 3 * b, n * n * k * 2 * b
        entry.update({"pair": st,
                      "GFLOPs": round(gflop_pair(n) / (st["median_ms"] * 1e-3), 2),
                      "pair_hbm_roofline_frac": round(2 * (R + 5 * C) / (st["median_ms"] * 1e-3)
                                                      / 1e9 / PEAK_HBM_GBS, 4)})
        out[name] = entry
        del p, x, F, y, cF
        torch.cuda.empty_cache()
    del f64, exact
    torch.cuda.empty_cache()
    return out


def losses_8x256(steps: int, dev) -> dict:
    """The differentiable workload: 8 k^-5/3 fields of 256^3 in FP32 (seeds
    5..12; Poisson sources uniform[-1,1), seeds 105..112).  L1 = sum_k |k|^2 |u_hat|^2 through
    rfft3; L2 = sum_j u_j^2 with u = N^-3 C2R(-R2C(f)/|k|^2) through rfft3
    and irfft3; one step = the loss and its backward pass (hand-written
    adjoints).  Vector FP32 stages, and the split-BF16 matrix-core stage with
    2 or 3 terms.  Gradients are compared with their closed forms evaluated
    through the FP64 path: grad L1 = 2 C2R(|k|^2 u_hat), grad L2 =
    2 N^-3 C2R(m R2C(u))."""
    from paper_2202_12756_amd import Plan, irfft3, rfft3

    n, B = 256, 8
    k = n // 2 + 1
    import synth

    u64, _ = _kolmogorov_fields(n, [5 + b for b in range(B)], dev)
    s32 = torch.stack([synth.uniform((n, n, n), 105 + b, torch.float32, dev) for b in range(B)])
    s64 = s32.double()
    sig = torch.arange(n, device=dev, dtype=torch.float64)
    sig = torch.where(sig <= n // 2, sig, sig - n)
    kz = torch.arange(k, device=dev, dtype=torch.float64)
    ksq = sig[:, None, None] ** 2 + sig[None, :, None] ** 2 + kz[None, None, :] ** 2
    w = torch.full((k,), 2.0, device=dev, dtype=torch.float64)
    w[0] = w[-1] = 1.0
    m = torch.where(ksq > 0, -1.0 / torch.where(ksq > 0, ksq, 1.0), 0.0)
    # closed-form gradients in FP64
    p64 = Plan(n, torch.float64, batch=B, device=dev)
    U = p64.r2c(u64)
    g1 = 2.0 * p64.c2r((ksq * U).contiguous(), scale=1.0)
    P = p64.c2r((m * p64.r2c(s64)).contiguous(), scale=1.0 / n ** 3)
    g2 = 2.0 * p64.c2r((m * p64.r2c(P)).contiguous(), scale=1.0 / n ** 3)
    del U, P, p64
    ksq32, w32, m32 = ksq.float(), w.float(), m.float()
    u32 = u64.float()
    out = {}
    for name, terms in (("vector", 0), ("mfma_bf16x2", 2), ("mfma_bf16x3", 3)):
        p = Plan(n, torch.float32, batch=B, device=dev, mfma_terms=terms)
        state = {}

        def l1_step():
            u = u32.detach().requires_grad_(True)
            F = rfft3(u, p)
            L = (w32 * ksq32 * torch.view_as_real(F).pow(2).sum(-1)).sum()
            L.backward()
            state["g1"] = u.grad

        def l2_step():
            f = s32.detach().requires_grad_(True)
            uu = irfft3(m32 * rfft3(f, p), p, 1.0 / n ** 3)
            L = uu.pow(2).sum()
            L.backward()
            state["g2"] = f.grad

        t1 = time_stats(l1_step, steps, 2)
        t2 = time_stats(l2_step, steps, 2)
        e1 = (torch.linalg.vector_norm(state["g1"].double() - g1)
              / torch.linalg.vector_norm(g1)).item()
        e2 = (torch.linalg.vector_norm(state["g2"].double() - g2)
              / torch.linalg.vector_norm(g2)).item()
        out[name] = {"energy_loss_fwd_bwd": t1, "poisson_loss_fwd_bwd": t2,
                     "energy_grad_rel_l2_vs_fp64_closed_form": e1,
                     "poisson_grad_rel_l2_vs_fp64_closed_form": e2}
        del p, state
        torch.cuda.empty_cache()
    del u64, s64, g1, g2, u32, s32
    torch.cuda.empty_cache()
    return {"losses_8x256_f32": out}


def eq5_1024(plan, F, y, n: int, dev) -> dict:
    """The paper's test field (section 4) on the benchmark grid: the forward
    spectrum against its eight nonzero bins (tests/golden/eq5_spectrum.txt,
    derived from the field's closed form) and the max-abs error of the
    normalized round trip, next to the paper's 1e-14."""
    import synth

    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                          "eq5_spectrum.txt")
    bins = []
    with open(golden) as fh:
        for line in fh:
            parts = line.split()
            if not parts or parts[0].startswith("#") or len(parts) != 5:
                continue
            idx = [n - int(v[2:]) if v.startswith("N-") else int(v) for v in parts[:3]]
            bins.append((idx, complex(float(parts[3]), float(parts[4]))))
    f = synth.paper_test_field_torch(n, plan.dtype, dev)
    plan.r2c(f, F)
    D = F / float(n) ** 3
    for (i, j, kk), v in bins:
        D[0, i, j, kk] -= v
    spec_dev = D.abs().max().item()
    del D
    plan.c2r(F, y, 1.0 / n ** 3)
    err = 0.0
    for s0 in range(0, n, 64):
        err = max(err, (y[0, s0:s0 + 64] - f[0, s0:s0 + 64]).abs().max().item())
    fmax = f.abs().max().item()
    del f
    return {"spectrum_maxabs_dev_over_N3": spec_dev, "roundtrip_maxabs": err,
            "roundtrip_maxabs_over_maxf": err / fmax, "paper_claim": 1e-14}


# workload groups that --only runs by themselves
ONLY = {"slab_4096": slab_share_4096, "pencil_4096": pencil_variants,
        "full_2048": full_grid_2048, "graphs": graph_variants,
        "kolmogorov_512": kolmogorov_512, "losses_8x256": losses_8x256,
        "slab_pack_p8": slab_pack_p8}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU's share of the transform; --gpus "
              f"{args.gpus} is not supported (the library drives one GPU; the "
              f"exchange between GPUs belongs to the caller).", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    import synth
    from paper_2202_12756_amd import Plan, device_copy

    n = args.n
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    b = 8 if dtype == torch.float64 else 4
    k = n // 2 + 1
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.only:
        print(json.dumps({"only": args.only, "steps": args.steps,
                          "variants": ONLY[args.only](args.steps, dev)}), flush=True)
        return
    plan = Plan(n, dtype, device=dev)
    x = synth.uniform(plan.real_shape, args.seed, dtype, dev)
    F = plan.empty_spectrum()
    y = plan.empty_real()
    scale = 1.0 / n ** 3
    stream = torch.cuda.current_stream(dev)
    print(f"[bench] n={n} dtype={args.dtype} input ready; warmup {args.warmup}",
          file=sys.stderr, flush=True)

    # One step = the public calls: gfft_exec_r2c (z, y, x passes) and
    # gfft_exec_c2r (x, y, z passes, 1/N^3 fused).
    for _ in range(args.warmup):
        plan.r2c(x, F)
        plan.c2r(F, y, scale)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
           for _ in range(args.steps)]
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ev in evs:
        ev[0].record(stream)
        plan.r2c(x, F)
        ev[1].record(stream)
        plan.c2r(F, y, scale)
        ev[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()
    step_ms = sorted(ev[0].elapsed_time(ev[2]) for ev in evs)
    r2c_ms = sum(ev[0].elapsed_time(ev[1]) for ev in evs) / args.steps
    c2r_ms = sum(ev[1].elapsed_time(ev[2]) for ev in evs) / args.steps
    ms_step = wall * 1e3 / args.steps

    # correctness of the measured work (outside the timed region), in slabs
    # of planes so the temporaries stay small
    err, num, den = 0.0, 0.0, 0.0
    for s0 in range(0, n, 64):
        dlt = y[0, s0:s0 + 64] - x[0, s0:s0 + 64]
        err = max(err, dlt.abs().max().item())
        num += torch.linalg.vector_norm(dlt).item() ** 2
        den += torch.linalg.vector_norm(x[0, s0:s0 + 64]).item() ** 2
        del dlt
    rel = math.sqrt(num / den)

    # Instrumented repeat: the same K steps through the single-pass entry
    # points (the same kernels in the same order), with HIP events between
    # the passes on the launch stream: each kernel's live average duration.
    passes = ["z_r2c", "y_fwd", "x_fwd", "x_inv", "y_inv", "z_c2r"]

    def step(ev):
        ev[0].record(stream)
        plan.z_r2c(x, F)
        ev[1].record(stream)
        plan.y_c2c(F, -1)
        ev[2].record(stream)
        plan.x_c2c(F, -1)
        ev[3].record(stream)
        plan.x_c2c(F, +1)
        ev[4].record(stream)
        plan.y_c2c(F, +1)
        ev[5].record(stream)
        plan.z_c2r(F, y, scale)
        ev[6].record(stream)

    pevs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)]
            for _ in range(args.steps)]
    torch.cuda.synchronize()
    for ev in pevs:
        step(ev)
    torch.cuda.synchronize()
    per_pass = {p: 0.0 for p in passes}
    for ev in pevs:
        for i, p in enumerate(passes):
            per_pass[p] += ev[i].elapsed_time(ev[i + 1])
    per_pass = {p: v / args.steps for p, v in per_pass.items()}
    ms_instrumented = sum(per_pass.values())

    R = n ** 3 * b
    C = n * n * k * 2 * b
    bytes_pass = {"z_r2c": R + C, "y_fwd": 2 * C, "x_fwd": 2 * C,
                  "x_inv": 2 * C, "y_inv": 2 * C, "z_c2r": C + R}
    kernel_name = {"z_r2c": "k_z_r2c", "y_fwd": "k_strided", "x_fwd": "k_strided",
                   "x_inv": "k_strided", "y_inv": "k_strided", "z_c2r": "k_z_c2r"}
    gbs = {p: bytes_pass[p] / (per_pass[p] * 1e-3) / 1e9 for p in passes}
    dom = max(passes, key=lambda p: per_pass[p])
    traffic = None
    if n == 1024 and dtype == torch.float64:
        traffic = recorded_traffic(args.traffic or TRAFFIC_FILE, dom)

    gflop = gflop_pair(n)
    model_bytes = 2 * (R + 5 * C)
    line = {
        "metric": METRIC,
        "value": round(gflop / (ms_step * 1e-3), 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": (f"{n}^3 real {args.dtype.upper()} grid held whole on one "
                                f"GPU, seeded uniform[-1,1) (SplitMix64 seed "
                                f"{args.seed}); forward R2C + inverse C2R with 1/N^3 "
                                f"through gfft_exec_r2c / gfft_exec_c2r"),
                   "n": n, "slab_x": n, "batch": 1},
        "roofline": {"bound": "hbm",
                     "kernel": f"{kernel_name[dom]} ({dom})",
                     "achieved": round(gbs[dom], 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs[dom] / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_pass[dom],
                     "avg_launch_ms": round(per_pass[dom], 4),
                     "source": ("HIP events between the passes of an instrumented repeat "
                                "of the K steps through the single-pass entry points")},
        "step_ms": {"mean_wall": round(ms_step, 4),
                    "mean_events": round(sum(step_ms) / len(step_ms), 4),
                    "median": round(step_ms[len(step_ms) // 2], 4),
                    "min": round(step_ms[0], 4), "max": round(step_ms[-1], 4)},
        "exec_ms": {"r2c": round(r2c_ms, 4), "c2r": round(c2r_ms, 4)},
        "per_pass_ms": {p: round(v, 4) for p, v in per_pass.items()},
        "per_pass_GBps": {p: round(v, 1) for p, v in gbs.items()},
        "instrumented_ms_per_step": round(ms_instrumented, 4),
        "pair_hbm_roofline_frac": round(model_bytes / (ms_step * 1e-3) / 1e9
                                        / PEAK_HBM_GBS, 4),
        "model_bytes_per_pair": model_bytes,
        "paper_convention_GFLOPs": round(2 * gflop / (ms_step * 1e-3), 2),
        "roundtrip_maxabs": err,
        "roundtrip_rel_l2": rel,
    }
    # the paper's test field on the same grid (section 4); it needs two more
    # grid-sized buffers, so only up to 1024^3
    if dtype == torch.float64 and n <= 1024:
        line["eq5_test_field"] = eq5_1024(plan, F, y, n, dev)
    # achievable bandwidth: the library's streaming copy of the real field
    # (one 16-byte element per work-item), and torch's copy beside it
    ms_copy = time_pairs(lambda: device_copy(y, x), 5, 1)
    ms_tcopy = time_pairs(lambda: y.copy_(x), 5, 1)
    line["copy_GBps"] = round(2 * R / (ms_copy * 1e-3) / 1e9, 1)
    line["torch_copy_GBps"] = round(2 * R / (ms_tcopy * 1e-3) / 1e9, 1)
    line["roofline"]["frac_of_copy"] = round(gbs[dom] / line["copy_GBps"], 4)
    line["pair_frac_of_copy"] = round(model_bytes / (ms_step * 1e-3) / 1e9
                                      / line["copy_GBps"], 4)
    # the strided passes' own access-pattern ceilings: their loads and stores
    # without the transform (gfft_exec_pass_copy), on the same spectrum
    line["pattern_copy_GBps"] = pattern_copies(plan, F, F, 2 * C)
    if dom[0] in "yx":
        ceil = line["pattern_copy_GBps"][dom[0]]
        line["roofline"]["pattern_copy_GBps"] = ceil
        line["roofline"]["frac_of_pattern_copy"] = round(gbs[dom] / ceil, 4)
    if not args.no_variants:
        del F, y
        torch.cuda.empty_cache()
        line["variants"] = variants(n, args.steps, x if dtype == torch.float64
                                    else x.double(), dev)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_planes, args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
