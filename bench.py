"""Benchmark: 3D R2C + C2R round trip of a 1024^3 FP64 grid on one MI355X.

One step = the whole hot path once: forward R2C (z pass, y pass, x pass)
and inverse C2R (x, y, z passes with the 1/N^3 normalization fused), on a
synthetic seeded uniform[-1,1) field already resident in HBM.  Each pass is
bracketed by HIP events on the stream it is launched on, inside the timed
region, so the per-kernel durations below are live measurements.

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
    sha, rows = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("kernel_source_sha256_16:"):
                sha = line.split(":", 1)[1].strip()
            elif line.startswith("| ") and not line.startswith("| pass"):
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                if len(cells) >= 5 and cells[4].isdigit():
                    rows[cells[0]] = int(cells[4])
    if sha != kernel_source_hash():
        return None
    return rows.get(pass_name)


def gflop_pair(n: int) -> float:
    """5 (N^3/2) log2 N^3 per R2C, twice per forward+inverse pair."""
    return 2 * 5.0 * (n ** 3 / 2) * math.log2(n ** 3) / 1e9


def cpu_baseline(n: int, planes: int, seed: int, min_seconds: float = 10.0) -> dict:
    """Time the FP64 oracle on a bounded sample of the same workload.

    Sample: the forward 2D R2C (z and y lines) and its inverse on `planes`
    x-planes of the N^3 grid, plus the forward and inverse x lines of a
    [N][planes][K] pencil.  The nominal flop count of those lines (one third
    of 5 (N^3/2) log2 N^3 per axis, pro rata) over the wall time gives a
    rate in the metric's unit.
    """
    import numpy as np

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
        if dt >= min_seconds or reps >= 20:
            break
    per_axis_pair = gflop_pair(n) / 3.0
    work = reps * per_axis_pair * (2 * planes / n + planes / n)
    return {"value": round(work / dt, 3), "unit": "GFLOP/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"radix-2 FP64 oracle: 2D R2C+C2R on {planes} of {n} "
                       f"x-planes and x-line C2C fwd+inv on a [{n}][{planes}][{k}] "
                       f"pencil, repeated {reps}x; {dt:.2f} s wall, rate = nominal flops of those "
                       f"lines / time"),
            "seconds": round(dt, 3)}


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
        del F32, y32, p32
        torch.cuda.empty_cache()
    del x32, F64
    torch.cuda.empty_cache()
    # the slab transpose of steps 2-4 at p = 8 (X = N/8 planes): the standalone
    # pack, and step 1 with and without the pack fused into its stores
    ranks = 8
    ps = Plan(n, torch.float64, slab_x=n // ranks, device=dev)
    pf = Plan(n, torch.float64, slab_x=n // ranks, fuse_pack=True, device=dev)
    xs = x64[0, : n // ranks].contiguous()
    S = ps.r2c(xs)
    send = torch.empty(ps.send_shape, dtype=torch.complex128, device=dev)
    ms_pack = time_pairs(lambda: ps.pack(S, send), steps, 2)
    ms_unfused = time_pairs(lambda: (ps.r2c(xs, S), ps.pack(S, send)), steps, 2)
    send2 = torch.empty_like(send)
    ms_fused = time_pairs(lambda: pf.r2c(xs, send2), steps, 2)
    cs = S.numel() * 16
    out["slab_pack_p8_f64"] = {
        "chunk": f"{n // ranks}x{n // ranks}x{k}",
        "pack_ms": round(ms_pack, 4),
        "pack_GBps": round(2 * cs / (ms_pack * 1e-3) / 1e9, 1),
        "r2c2d_then_pack_ms": round(ms_unfused, 4),
        "r2c2d_fused_pack_ms": round(ms_fused, 4),
        "fused_equals_standalone": bool(torch.equal(send, send2)),
    }
    del ps, pf, xs, S, send, send2
    torch.cuda.empty_cache()
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
    out.update(slab_share_4096(steps, dev))
    out.update(pencil_variants(steps, dev))
    out.update(graph_variants(steps, dev))
    out.update(full_grid_2048(steps, dev))
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


# workload groups that --only runs by themselves
ONLY = {"slab_4096": slab_share_4096, "pencil_4096": pencil_variants,
        "full_2048": full_grid_2048, "graphs": graph_variants}


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
    from paper_2202_12756_amd import Plan

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

    passes = ["z_r2c", "y_fwd", "x_fwd", "x_inv", "y_inv", "z_c2r"]

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.z_r2c(x, F)
        if ev is not None:
            ev[1].record(stream)
        plan.y_c2c(F, -1)
        if ev is not None:
            ev[2].record(stream)
        plan.x_c2c(F, -1)
        if ev is not None:
            ev[3].record(stream)
        plan.x_c2c(F, +1)
        if ev is not None:
            ev[4].record(stream)
        plan.y_c2c(F, +1)
        if ev is not None:
            ev[5].record(stream)
        plan.z_c2r(F, y, scale)
        if ev is not None:
            ev[6].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)]
           for _ in range(args.steps)]
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()

    per_pass = {p: 0.0 for p in passes}
    for ev in evs:
        for i, p in enumerate(passes):
            per_pass[p] += ev[i].elapsed_time(ev[i + 1])
    per_pass = {p: v / args.steps for p, v in per_pass.items()}
    ms_step = wall * 1e3 / args.steps
    ms_events = sum(per_pass.values())

    # correctness of the measured work (outside the timed region)
    # (in slabs of planes, so the temporaries stay small at 2048^3)
    err, num, den = 0.0, 0.0, 0.0
    for s0 in range(0, n, 64):
        dlt = y[0, s0:s0 + 64] - x[0, s0:s0 + 64]
        err = max(err, dlt.abs().max().item())
        num += torch.linalg.vector_norm(dlt).item() ** 2
        den += torch.linalg.vector_norm(x[0, s0:s0 + 64]).item() ** 2
        del dlt
    rel = math.sqrt(num / den)

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
                                f"{args.seed}); forward R2C + inverse C2R with 1/N^3"),
                   "n": n, "slab_x": n, "batch": 1},
        "roofline": {"bound": "hbm",
                     "kernel": f"{kernel_name[dom]} ({dom})",
                     "achieved": round(gbs[dom], 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs[dom] / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_pass[dom],
                     "avg_launch_ms": round(per_pass[dom], 4)},
        "per_pass_ms": {p: round(v, 4) for p, v in per_pass.items()},
        "per_pass_GBps": {p: round(v, 1) for p, v in gbs.items()},
        "pair_hbm_roofline_frac": round(model_bytes / (ms_step * 1e-3) / 1e9
                                        / PEAK_HBM_GBS, 4),
        "model_bytes_per_pair": model_bytes,
        "event_ms_per_step": round(ms_events, 4),
        "paper_convention_GFLOPs": round(2 * gflop / (ms_step * 1e-3), 2),
        "roundtrip_maxabs": err,
        "roundtrip_rel_l2": rel,
    }
    # achievable bandwidth: an 8.6 GB device-to-device copy
    ms_copy = time_pairs(lambda: y.copy_(x), 5, 1)
    line["copy_GBps"] = round(2 * R / (ms_copy * 1e-3) / 1e9, 1)
    line["roofline"]["frac_of_copy"] = round(gbs[dom] / line["copy_GBps"], 4)
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
