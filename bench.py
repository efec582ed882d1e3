#!/usr/bin/env python3
"""Benchmark of the strided-swap stencil path on one MI355X.

Workload (default): Box-2D49P (7x7 box, radius 3) on a 10240 x 10240 grid, 50
Jacobi time steps per pass, fp16 carry, fp16 operands with fp32 accumulation
on the structured-sparse matrix instruction; coefficients N(0,1) rescaled to sum
1 (first stable seed), grid = mean of 8 random plane sinusoids + 1% uniform
noise.  One benchmark step = one spider_apply of the whole 50-step time loop on
inputs already resident in HBM.

Prints one JSON line with the throughput (GStencil/s = grid points x time steps
per second) over the K timed passes and over a sustained region of at least one
second, the roofline position of the dominant kernel against the roof that binds
it (the larger of its HBM time and its matrix-instruction time over its measured
launch duration), the fp64 oracle timed on the host's cores on a bounded sample,
normwise errors against the oracle over every grid point of every workload, the
plain fp32 GPU path on the same workloads, per-pass latency percentiles, an
engine ablation and a short serving sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
MFMA_PEAK_TFLOPS = 2500.0    # MI355X dense fp16 / bf16 matrix peak, 2.5 PFLOP/s
# multiply-adds per matrix instruction over the operands it holds: a dense
# 16x16x32 product, or a 2:4 16x16x64 smfmac (16 x 16 outputs x 32 stored A values)
MACS_PER_INSTRUCTION = 16 * 16 * 32
METRIC = "GStencil/s at stated error vs FP64 oracle (vs plain GPU path); p50/p99 latency"
TOL = {"f16": (2e-3, 1e-2), "bf16": (3e-2, 6e-2), "f32": (1e-5, 1e-5), "f32s3": (5e-5, 5e-5),
       "f64": (1e-13, 1e-13)}
KERNEL_SOURCES = ["paper_2506_22035_amd/csrc/kernels_band_pair.hip", "paper_2506_22035_amd/csrc/band_pair.h",
                  "paper_2506_22035_amd/csrc/band_common.h"]
# measured HBM bytes of the headline's dominant kernel (four fused time steps per launch)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "band2d_pair_tbt_box49p_f16_10240_traffic.json")
SUSTAIN_S = 1.0              # length of the sustained timed region


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(steps_per_launch, tile_h2, grid):
    """HBM bytes per launch from committed rocprofv3 counters, if they were taken on this
    kernel source, fused depth, segment height and grid."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    if (t.get("time_steps_per_launch") != steps_per_launch or t.get("tile_h2") != tile_h2
            or t.get("grid") != list(grid)):
        return None
    return t.get("hbm_bytes_per_launch")


def timed_applies(torch, plan, xd, y, steps_per_pass, k, stream):
    """Run k passes; return (total ms over the region, per-pass ms list), HIP events on `stream`."""
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(k):
        plan.apply(xd, y, steps_per_pass, stream=stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(k)]
    return evs[0].elapsed_time(evs[k]), per


def gstencil(npts, steps, ms):
    return npts * steps / (ms * 1e-3) / 1e9


def to_host64(torch, t):
    return t.to(torch.float64).cpu().numpy()


def full_grid_error(oracle, w, x64, steps, got, tol_key, ref=None):
    """Normwise errors of `got` against the oracle run on the whole grid (or against
    `ref`, that oracle result computed before):
    rel-RMS = ||got - ref||_2 / ||ref||_2 and rel-max = ||got - ref||_inf / ||ref||_inf."""
    if ref is None:
        ref = oracle.apply(w, x64, steps)
    d = got - ref
    rms = float(np.sqrt(np.sum(d * d) / np.sum(ref * ref)))
    mx = float(np.max(np.abs(d)) / np.max(np.abs(ref)))
    tr, tm = TOL[tol_key]
    if tol_key == "f16":
        # one round-to-nearest fp16 rounding per step (at most 2^-12 relative), coherent
        # over the steps, bounds the largest error by steps * 2^-12 of the largest value
        tm = max(tm, steps * 2.0 ** -12)
    return {"rel_rms": rms, "rel_max": mx, "tol_rel_rms": tr, "tol_rel_max": tm, "points": int(ref.size),
            "method": "every grid point against the fp64 oracle", "pass": bool(rms <= tr and mx <= tm)}


def load_oracle():
    import oracle
    oracle.ensure_built()
    return oracle


def roofline(torch, sp, plan, xd, elem, npts, grid, operand, stream, headline_traffic, steps, pass_ms):
    """Sustained throughput and the roofline position of the plan's dominant kernel.

    Sustained: passes of the workload (`steps` time steps from the same input, as in
    the timed region) for at least SUSTAIN_S seconds.  Roofline: passes of only the
    fused launches (the largest multiple of the fused depth not above `steps`), again
    from the same input -- a long loop of one time loop would smooth the field, and
    smoother data draws less power and runs at higher clocks -- for at least
    SUSTAIN_S / 2 seconds; the launch time is their average (HIP events on `stream`).
    Two roofs bound a launch from below: HBM (bytes moved / 8 TB/s) and the matrix
    pipe (matrix instructions x 8192 multiply-adds x 2 / 2.5 PFLOP/s); the larger
    fraction is the binding one."""
    info = plan.info()
    tb = max(1, info["time_block"])
    yl = torch.empty_like(xd)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_s = max(20, int(math.ceil(SUSTAIN_S * 1e3 / max(pass_ms, 1e-3))))
    plan.apply(xd, yl, steps, stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n_s):
        plan.apply(xd, yl, steps, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1)
    sustained = {"value": round(gstencil(npts, steps * n_s, ms_s), 2), "seconds": round(ms_s * 1e-3, 3),
                 "passes": n_s, "ms_per_step": round(ms_s / n_s, 4),
                 "method": "passes of the workload from the same input, back to back"}
    nl = max(1, steps // tb)              # fused launches per roofline pass
    n_r = max(20, int(math.ceil(0.5 * SUSTAIN_S * 1e3 / max(pass_ms * nl * tb / steps, 1e-3))))
    plan.apply(xd, yl, nl * tb, stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n_r):
        plan.apply(xd, yl, nl * tb, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del yl
    avg_s = ms * 1e-3 / (n_r * nl)
    compulsory = npts * 2 * elem          # one read and one write of the state per launch
    charged = compulsory * tb             # the same per time step, all steps of the launch
    traffic = headline_traffic(tb, info["tile_h2"], grid)
    hbm_bytes = traffic if traffic is not None else compulsory
    hbm_frac = hbm_bytes / avg_s / 1e9 / HBM_PEAK_GBS
    _, n_mi = plan.work(tb)
    roof = {}
    if n_mi is not None and n_mi > 0:
        flop = n_mi * MACS_PER_INSTRUCTION * 2
        mfma_tflops = flop / avg_s / 1e12
        mfma_frac = mfma_tflops / MFMA_PEAK_TFLOPS
    else:
        mfma_frac = None
    if mfma_frac is not None and mfma_frac > hbm_frac:
        roof.update({"bound": "mfma", "achieved": round(mfma_tflops, 1), "peak": MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(mfma_frac, 4)})
    else:
        roof.update({"bound": "hbm", "achieved": round(hbm_bytes / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(hbm_frac, 4)})
    roof["traffic"] = traffic
    roof["hbm"] = {"bytes_per_launch": hbm_bytes,
                   "bytes_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated" if traffic is not None
                   else "compulsory: one read and one write of the grid",
                   "GBs": round(hbm_bytes / avg_s / 1e9, 1), "frac": round(hbm_frac, 4),
                   "compulsory_bytes_per_launch": compulsory}
    if mfma_frac is not None:
        roof["mfma"] = {"instructions_per_launch": n_mi, "operand": operand,
                        "macs_per_instruction": MACS_PER_INSTRUCTION, "TFLOPs": round(mfma_tflops, 1),
                        "frac": round(mfma_frac, 4)}
    roof.update({"avg_launch_us": round(avg_s * 1e6, 2), "time_steps_per_launch": tb,
                 "launch_timing": "%d passes of %d fused launches from the workload's input (%.0f ms), after the "
                                  "timed passes" % (n_r, nl, ms),
                 "alg_GBs_charged": round(charged / avg_s / 1e9, 1),
                 "alg_bytes_charged_per_launch": charged})
    return roof, sustained


def matrix_ceiling(sp, engine, stream, waves=(2, 4), iterations=200000):
    """Sustained fp16 matrix-instruction rates of this GPU (spider_measure_matrix_rate):
    the sparse and the dense instruction at each residency in `waves` (waves per SIMD),
    with the clock the chip holds.  The fused kernels hold two waves per SIMD."""
    out = {}
    for kind in ("sparse", "dense"):
        for w in waves:
            m = sp.measure_matrix_rate(kind == "sparse", w, iterations, stream=stream)
            out["%s_w%d" % (kind, w)] = {"TFLOPs": round(m["TFLOPs"], 1), "clock_GHz": round(m["clock_GHz"], 3),
                                         "cycles_per_instruction": round(m["cycles_per_instruction"], 2)}
    out["sparse_over_dense"] = {"w%d" % w: round(out["sparse_w%d" % w]["TFLOPs"] / out["dense_w%d" % w]["TFLOPs"], 3)
                                for w in waves}
    out["method"] = ("register-resident fp16 operands, 8 independent accumulators per wave, %d x 8 instructions "
                     "per wave after a warm-up launch; TFLOP/s counts 2 x 16 x 16 x 32 flop per instruction"
                     % iterations)
    return out


def kernel_name(info, shape, carry, engine, r, row_swap):
    tb = info["time_block"]
    if engine == "direct":
        kname = "direct2d_fused_kernel" if (len(shape) == 2 and tb > 1) else "direct%dd_kernel" % len(shape)
    elif carry == "f32":
        kname = ("band2d_pair_f32_kernel" if info["band_height"] == 8 else "band2d_f32_kernel")
    elif len(shape) == 1:
        kname = "band1d_tbt_kernel" if tb > 1 else "band1d_kernel"
    elif len(shape) == 3:
        kname = "band3d_kernel"
    elif info["band_height"] == 8:
        kname = {1: "band2d_pair_kernel", 2: "band2d_pair_tb2_kernel"}.get(tb, "band2d_pair_tbt_kernel")
    else:
        kname = "band2d_tb2_kernel" if tb == 2 else "band2d_kernel"
    return kname + "<r=%d,%s,%s%s%s>" % (r, carry, engine, ",T=%d" % tb if tb > 1 else "",
                                         ",explicit row swap" if row_swap == "explicit" else "")


def serving_run(torch, sp, si, reqs, rate, plans, bases, budget, slots):
    """Submit `reqs` (arrival times scaled to `rate` req/s) to a fresh server; return stats."""
    srv = sp.Server(hbm_budget_bytes=budget, max_slots=slots, max_queue=len(reqs) + 1)
    outs = {}
    pending = []
    t0 = time.perf_counter()
    try:
        for r in reqs:
            t_arr = r["t"] / rate
            while time.perf_counter() - t0 < t_arr:
                # poll while waiting so finished outputs are released
                for tk in list(outs):
                    if srv.poll(tk)[0]:
                        del outs[tk]
            shape = tuple(r["shape"])
            key = (r["stencil"], shape)
            if key not in plans:
                plans[key] = sp.Plan(si.serving_coeffs(r["stencil"]), shape, carry="f16")
            n = int(np.prod(shape))
            xin = bases[len(shape)][:n].view(shape)
            o = torch.empty(shape, dtype=torch.float16, device="cuda")
            tk = srv.submit(plans[key], xin, o, r["steps"])
            outs[tk] = o
            pending.append(tk)
        for tk in pending:
            while not srv.poll(tk)[0]:
                time.sleep(0.0002)
        t1 = time.perf_counter()
        st = srv.stats()
    finally:
        srv.close()
    return {"rate_req_s": round(rate, 2), "requests": len(reqs), "p50_ms": round(st["p50_us"] / 1e3, 3),
            "p99_ms": round(st["p99_us"] / 1e3, 3), "GStencil/s": round(st["stencil_updates"] / (t1 - t0) / 1e9, 2),
            "wall_s": round(t1 - t0, 3)}


def serving(torch, sp, si, n, fractions, seed=11):
    """Serving mix: saturation throughput first (all requests at once), then Poisson rates."""
    torch.manual_seed(seed)
    bases = {2: (torch.rand(8192 * 8192, device="cuda")).to(torch.float16),
             3: (torch.rand(384 ** 3, device="cuda")).to(torch.float16)}
    plans = {}
    reqs = si.serving_requests(n, 1.0, seed)   # times for rate 1 req/s, rescaled per run
    budget, slots = 32 << 30, 64
    # plans are built before any timed run (the offline transformation is not served work)
    for r in reqs:
        key = (r["stencil"], tuple(r["shape"]))
        if key not in plans:
            plans[key] = sp.Plan(si.serving_coeffs(r["stencil"]), key[1], carry="f16")
    sat = serving_run(torch, sp, si, [dict(r, t=0.0) for r in reqs], 1.0, plans, bases, budget, slots)
    sat_rate = n / sat["wall_s"]
    out = {"saturation": dict(sat, rate_req_s=round(sat_rate, 2)), "sweep": []}
    for f in fractions:
        out["sweep"].append(dict(serving_run(torch, sp, si, reqs, f * sat_rate, plans, bases, budget, slots),
                                 load=f))
    for p in plans.values():
        p.close()
    return out


def batch3d_run(torch, sp, si, passes, warmup, with_errors, oracle=None):
    """Box-3D27P 512^3 and Heat-3D 256^3, 20 steps each, advanced together by batched
    launches (one launch per time step covering both grids), fp16 carry; compared with
    the two grids run one after the other on their own plans, and with the plain fp32
    path.  With errors: every point of both results against the fp64 oracle."""
    wls = [si.workload("box3d27p_512"), si.workload("heat3d_256")]
    xh = [torch.from_numpy(wl["make_grid"](np.float32)).to(torch.float16) for wl in wls]
    xs = [x.to("cuda:0") for x in xh]
    ys = [torch.empty_like(x) for x in xs]
    plans = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16", autotune=True) for wl in wls]
    steps = [wl["steps"] for wl in wls]
    npts = sum(int(np.prod(wl["shape"])) * wl["steps"] for wl in wls)
    stream = torch.cuda.current_stream()
    # the same batch launched step by step (plans without graph replay): the
    # descriptors are staged and the launches enqueued on every call
    direct = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16", autotune=True, use_graph=False) for wl in wls]
    ysd = [torch.empty_like(x) for x in xs]
    for _ in range(warmup):
        sp.apply_batch(plans, xs, ys, steps)
        sp.apply_batch(direct, xs, ysd, steps)
    torch.cuda.synchronize()
    # graph replay and direct launches timed in alternating blocks, so that neither
    # mode is measured alone while the clocks are still settling
    per, total, direct_total = [], 0.0, 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for block in (passes // 2, passes - passes // 2):  # the passes, in two blocks
        if block == 0:
            continue
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(block + 1)]
        evs[0].record(stream)
        for k in range(block):
            sp.apply_batch(plans, xs, ys, steps)
            evs[k + 1].record(stream)
        torch.cuda.synchronize()
        per += [evs[k].elapsed_time(evs[k + 1]) for k in range(block)]
        total += evs[0].elapsed_time(evs[-1])
        e0.record(stream)
        for _ in range(block):
            sp.apply_batch(direct, xs, ysd, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        direct_total += e0.elapsed_time(e1)
    direct_ms = direct_total / passes
    same = all(bool(torch.equal(a, b)) for a, b in zip(ys, ysd))
    del ysd
    # the same work, each grid alone on its own plan (one step per launch, as batched)
    solo = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16", autotune=True, time_block=1) for wl in wls]
    ys2 = [torch.empty_like(x) for x in xs]
    for p, x, y, st in zip(solo, xs, ys2, steps):
        p.apply(x, y, st)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(passes):
        for p, x, y, st in zip(solo, xs, ys2, steps):
            p.apply(x, y, st)
    e1.record(stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1) / passes
    del ys2
    value = npts * passes / (total * 1e-3) / 1e9
    # the plain fp32 GPU path (direct engine) on the same grids and steps
    x32 = [x.to(torch.float32) for x in xs]
    y32 = [torch.empty_like(x) for x in x32]
    p32 = [sp.Plan(wl["coeffs"], wl["shape"], carry="f32") for wl in wls]
    for p, x, y, st in zip(p32, x32, y32, steps):
        p.apply(x, y, st)
    torch.cuda.synchronize()
    e0.record(stream)
    for p, x, y, st in zip(p32, x32, y32, steps):
        p.apply(x, y, st)
    e1.record(stream)
    torch.cuda.synchronize()
    fp32_value = npts / (e0.elapsed_time(e1) * 1e-3) / 1e9
    # the fp32 carry on the sparse engine (every input value split into 16-bit hi + lo
    # operands, split 3) for the same pair in one batched call
    pc = [sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, autotune=True) for wl in wls]
    yc = [torch.empty_like(x) for x in x32]
    sp.apply_batch(pc, x32, yc, steps)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(passes):
        sp.apply_batch(pc, x32, yc, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    f32c_ms = e0.elapsed_time(e1) / passes
    f32c_value = npts / (f32c_ms * 1e-3) / 1e9
    res = {"value": round(value, 2), "unit": "GStencil/s", "ms_per_pass": round(total / passes, 4),
           "hbm_compulsory": compulsory_hbm(1, npts, 2, total / passes),
           "latency_ms": {"p50": round(float(np.percentile(per, 50)), 4),
                          "p99": round(float(np.percentile(per, 99)), 4)},
           "graph_replay": True,
           "direct_launches": {"ms_per_pass": round(direct_ms, 4),
                               "GStencil/s": round(npts / (direct_ms * 1e-3) / 1e9, 2),
                               "identical_to_graph_replay": same},
           "separate_plans": {"ms_per_pass": round(seq_ms, 4),
                              "GStencil/s": round(npts / (seq_ms * 1e-3) / 1e9, 2),
                              "tile_h": [p.info()["tile_h"] for p in solo],
                              "hbm_compulsory": compulsory_hbm(1, npts, 2, seq_ms),
                              "mfma": run_mfma({"ms_per_pass": seq_ms, "matrix_instructions_per_pass": sum(
                                  p.work(st)[1] or 0 for p, st in zip(solo, steps))})},
           "plain_gpu_fp32": {"value": round(fp32_value, 2), "unit": "GStencil/s", "engine": "direct (VALU fp32)",
                              "speedup_batched_lowp_over_fp32": round(value / fp32_value, 3)},
           "f32_carry_sparse_split3": {"value": round(f32c_value, 2), "unit": "GStencil/s",
                                       "speedup_over_plain_fp32": round(f32c_value / fp32_value, 3),
                                       "hbm_compulsory": compulsory_hbm(1, npts, 4, f32c_ms)}}
    if with_errors:
        got = [to_host64(torch, y) for y in ys]
        got32 = [to_host64(torch, y) for y in y32]
        gotc = [to_host64(torch, y) for y in yc]
        del xs, ys, x32, y32, yc
        res["error_vs_fp64_oracle"] = {}
        res["plain_gpu_fp32"]["error_vs_fp64_oracle"] = {}
        res["f32_carry_sparse_split3"]["error_vs_fp64_oracle"] = {}
        for wl, x, g, g32, gc in zip(wls, xh, got, got32, gotc):
            x64 = x.to(torch.float64).numpy()
            # the fp32 paths ran on the same (fp16-rounded) values: one oracle run serves all three
            ref = oracle.apply(wl["coeffs"], x64, wl["steps"])
            res["error_vs_fp64_oracle"][wl["name"]] = full_grid_error(oracle, wl["coeffs"], x64, wl["steps"], g,
                                                                      "f16", ref)
            res["plain_gpu_fp32"]["error_vs_fp64_oracle"][wl["name"]] = full_grid_error(
                oracle, wl["coeffs"], x64, wl["steps"], g32, "f32", ref)
            res["f32_carry_sparse_split3"]["error_vs_fp64_oracle"][wl["name"]] = full_grid_error(
                oracle, wl["coeffs"], x64, wl["steps"], gc, "f32s3", ref)
    for p in plans + direct + solo + p32 + pc:
        p.close()
    return res


def batch3d(torch, sp, si, args):
    oracle = None if args.no_extras else load_oracle()
    r = batch3d_run(torch, sp, si, args.steps, args.warmup, not args.no_extras, oracle)
    return {"metric": METRIC, "value": r["value"], "unit": "GStencil/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": r["ms_per_pass"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
            "config": {"workload": "batch3d: box3d27p 512^3 x 20 steps + heat3d 256^3 x 20 steps, one batched "
                                   "launch per time step", "carry": "f16", "engine": "sparse"},
            **{k: v for k, v in r.items() if k not in ("value", "unit", "ms_per_pass")}}


def size_trend(torch, sp, si, args):
    """Throughput versus grid size for the Box-2D49P stencil (the paper's size trend, Fig. 11):
    square grids of the headline recipe's stencil and field, 50 steps per pass, fp16 carry."""
    wl = si.workload("box2d49p_10240")
    res = []
    for n in (512, 1024, 2048, 4096, 6144, 8192, 10240, 12288, 14336):
        x = torch.from_numpy(si.grid_sinusoids((n, n), wl["seeds"]["grid"])).to(torch.float16).to("cuda:0")
        y = torch.empty_like(x)
        row = {"n": n, "grid_MB": round(2 * n * n / 1e6, 1)}
        for band in (8, 16):
            p = sp.Plan(wl["coeffs"], (n, n), carry="f16", autotune=True, band_height=band)
            p.apply(x, y, 50)
            ms1, _ = timed_applies(torch, p, x, y, 50, 2, torch.cuda.current_stream())
            k = max(5, int(math.ceil(250.0 / max(ms1 / 2, 1e-3))))   # about a quarter second of passes
            ms, _ = timed_applies(torch, p, x, y, 50, k, torch.cuda.current_stream())
            row["band%d_GStencil_s" % band] = round(n * n * 50 * k / (ms * 1e-3) / 1e9, 1)
            row["band%d_time_steps_per_launch" % band] = p.info()["time_block"]
            p.close()
        res.append(row)
        del x, y
    return {"metric": "GStencil/s versus grid size (Box-2D49P, 50 steps, fp16 carry, sparse engine)",
            "config": {"workload": "box2d49p_size_trend", "steps_per_pass": 50}, "trend": res}


_GRIDS = {}


def workload_grid(si, name, dtype):
    """The workload's host grid (drawn once per process and dtype)."""
    key = (name, np.dtype(dtype).str)
    if key not in _GRIDS:
        _GRIDS[key] = si.workload(name)["make_grid"](dtype)
    return _GRIDS[key]


def compulsory_hbm(launches, npts, elem, ms_per_pass):
    """HBM position of a time loop from its compulsory traffic: every launch reads and
    writes the whole state once (a fused launch keeps its inner steps on chip)."""
    b = launches * 2 * npts * elem
    gbs = b / (ms_per_pass * 1e-3) / 1e9
    return {"bytes_per_pass": int(b), "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_source": "compulsory: one read and one write of the state per launch"}


def run_hbm(info, wl, carry):
    return compulsory_hbm(info["launches_per_pass"], int(np.prod(wl["shape"])),
                          {"f16": 2, "bf16": 2, "f32": 4, "f64": 8}[carry], info["ms_per_pass"])


def run_mfma(info):
    """Matrix-pipe position of a time loop: its matrix instructions (spider_plan_work)
    x 16 x 16 x 32 multiply-adds x 2 over the pass time, against the published peak;
    None where the library keeps no count for the plan."""
    n = info.get("matrix_instructions_per_pass")
    if not n:
        return None
    tf = n * MACS_PER_INSTRUCTION * 2 / (info["ms_per_pass"] * 1e-3) / 1e12
    return {"instructions_per_pass": int(n), "TFLOPs": round(tf, 1), "frac": round(tf / MFMA_PEAK_TFLOPS, 4)}


def workload_run(torch, sp, si, name, carry, engine, split, passes, stream, keep_result=True):
    """Plan (autotuned) and time `passes` passes of workload `name`; return (GStencil/s,
    plan info, result on the host in fp64 or None, input on the host in fp64)."""
    wl = si.workload(name)
    x32 = workload_grid(si, name, np.float64 if carry == "f64" else np.float32)
    xh = torch.from_numpy(x32).to(sp.torch_dtype(carry))
    xd = xh.to("cuda:0")
    y = torch.empty_like(xd)
    p = sp.Plan(wl["coeffs"], wl["shape"], carry=carry, engine=engine, split=split, autotune=True)
    p.apply(xd, y, wl["steps"], stream=stream)
    ms, _ = timed_applies(torch, p, xd, y, wl["steps"], passes, stream)
    info = p.info()
    info["launches_per_pass"], info["matrix_instructions_per_pass"] = p.work(wl["steps"])
    info["ms_per_pass"] = ms / passes
    p.close()
    got = to_host64(torch, y) if keep_result else None
    del xd, y
    return gstencil(int(np.prod(wl["shape"])), wl["steps"] * passes, ms), info, got, xh.to(torch.float64).numpy()


def other_configs(torch, sp, si, stream, oracle):
    """The other workloads: throughput and full-grid errors of each, with the plain fp32
    GPU path where it is the metric's comparison."""
    out = {}
    # Star-2D13P 8192^2, 100 steps: fp16 sparse vs the plain fp32 GPU path, and the fp32 carry
    name = "star2d13p_8192"
    wl = si.workload(name)
    v16, i16, g16, x16 = workload_run(torch, sp, si, name, "f16", "sparse", 2, 3, stream)
    e16 = full_grid_error(oracle, wl["coeffs"], x16, wl["steps"], g16, "f16")
    del g16, x16
    v32, i32, g32, x32 = workload_run(torch, sp, si, name, "f32", "direct", 2, 3, stream)
    vs3, is3, gs3, _ = workload_run(torch, sp, si, name, "f32", "sparse", 3, 3, stream)
    ref32 = oracle.apply(wl["coeffs"], x32, wl["steps"])
    e32 = full_grid_error(oracle, wl["coeffs"], x32, wl["steps"], g32, "f32", ref32)
    es3 = full_grid_error(oracle, wl["coeffs"], x32, wl["steps"], gs3, "f32s3", ref32)
    del ref32
    del g32, gs3, x32
    out[name] = {"f16_sparse": {"value": round(v16, 2), "time_steps_per_launch": i16["time_block"],
                                "error_vs_fp64_oracle": e16, "hbm_compulsory": run_hbm(i16, wl, "f16"),
                                "mfma": run_mfma(i16)},
                 "plain_gpu_fp32": {"value": round(v32, 2), "engine": "direct (VALU fp32)",
                                    "error_vs_fp64_oracle": e32, "hbm_compulsory": run_hbm(i32, wl, "f32")},
                 "f32_carry_sparse_split3": {"value": round(vs3, 2), "time_steps_per_launch": is3["time_block"],
                                             "error_vs_fp64_oracle": es3, "hbm_compulsory": run_hbm(is3, wl, "f32"),
                                             "mfma": run_mfma(is3)},
                 "speedup_f16_over_plain_fp32": round(v16 / v32, 3),
                 "speedup_f32_carry_over_plain_fp32": round(vs3 / v32, 3)}
    # Box-3D27P 512^3 + Heat-3D 256^3 in one batched launch per step
    out["batch3d"] = batch3d_run(torch, sp, si, 10, 2, True, oracle)
    # Box-2D9P 256^2, fp64 on the direct engine (latency-bound at this size)
    name = "box2d9p_256_f64"
    wl = si.workload(name)
    v64, _, g64, x64 = workload_run(torch, sp, si, name, "f64", "direct", 2, 20, stream)
    out[name] = {"value": round(v64, 2), "us_per_time_step": round(65536 / (v64 * 1e9) * 1e6, 3),
                 "error_vs_fp64_oracle": full_grid_error(oracle, wl["coeffs"], x64, wl["steps"], g64, "f64")}
    # the paper's 1-D workloads, 100 steps: fp16 carry, and the fp32 carry on the sparse
    # engine (16-bit operands split from the fp32 values)
    for name in ("1d3p_10240000", "1d5p_10240000"):
        wl = si.workload(name)
        v1, i1, g1, x1 = workload_run(torch, sp, si, name, "f16", "sparse", 2, 5, stream)
        e1 = full_grid_error(oracle, wl["coeffs"], x1, wl["steps"], g1, "f16")
        del g1, x1
        vf, iff, gf, xf = workload_run(torch, sp, si, name, "f32", "sparse", 3, 5, stream)
        ef = full_grid_error(oracle, wl["coeffs"], xf, wl["steps"], gf, "f32s3")
        del gf, xf
        # 16-bit grid, split 3: the levels inside a fused launch kept as hi/lo pairs,
        # the grid rounded to fp16 once per launch instead of once per step
        vh, ih, gh, xh = workload_run(torch, sp, si, name, "f16", "sparse", 3, 5, stream)
        eh = full_grid_error(oracle, wl["coeffs"], xh, wl["steps"], gh, "f16")
        del gh, xh
        # (the 1-D lines, 20 and 41 MB, stay in the last-level cache between launches)
        modes = {"f16_sparse": {"value": round(v1, 2), "time_steps_per_launch": i1["time_block"],
                                "tile_h2": i1["tile_h2"], "error_vs_fp64_oracle": e1,
                                "hbm_compulsory": run_hbm(i1, wl, "f16"), "mfma": run_mfma(i1)},
                 "f32_carry_sparse_split3": {"value": round(vf, 2), "time_steps_per_launch": iff["time_block"],
                                             "tile_h2": iff["tile_h2"], "error_vs_fp64_oracle": ef,
                                             "hbm_compulsory": run_hbm(iff, wl, "f32"), "mfma": run_mfma(iff)},
                 "f16_carry_sparse_split3": {"value": round(vh, 2), "time_steps_per_launch": ih["time_block"],
                                             "tile_h2": ih["tile_h2"], "error_vs_fp64_oracle": eh,
                                             "hbm_compulsory": run_hbm(ih, wl, "f16"), "mfma": run_mfma(ih)}}
        # the config's value: the fastest mode whose error meets its stated bound
        ok = [(m["value"], k) for k, m in modes.items() if m["error_vs_fp64_oracle"]["pass"]]
        best = max(ok)[1] if ok else None
        out[name] = dict(value=modes[best]["value"] if best else None, mode=best, **modes)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed passes (each = 50 time steps)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="box2d49p_10240",
                    choices=["box2d49p_10240", "star2d13p_8192", "box2d9p_256_f64", "box3d27p_512", "heat3d_256",
                             "1d3p_10240000", "1d5p_10240000", "box2d7r_10240", "batch3d"],
                    help="workload recipe (default: the headline Box-2D49P)")
    ap.add_argument("--carry", default=None, choices=["f16", "bf16", "f32", "f64"],
                    help="grid dtype (default f16; f64 for box2d9p_256_f64)")
    ap.add_argument("--engine", default=None, choices=["sparse", "dense", "direct"],
                    help="default: sparse for 16-bit carries, direct otherwise")
    ap.add_argument("--split", type=int, default=0,
                    help="products per kernel row (default 2; 3 for an fp32 carry on a matrix engine)")
    ap.add_argument("--tile-h", type=int, default=0)
    ap.add_argument("--band-height", type=int, default=0, choices=[0, 8, 16],
                    help="output points per band row (0: the library's choice)")
    ap.add_argument("--time-block", type=int, default=0, choices=list(range(17)),
                    help="time steps fused per launch (0: the library's choice)")
    ap.add_argument("--row-swap", default="implicit", choices=["implicit", "explicit"],
                    help="row swap in the gather offsets (implicit) or by an LDS copy (explicit; the comparison "
                         "of the paper's Table 3: sparse engine, band height 16, one step per launch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip errors, the other workloads, the fp32 path, the ablation and the serving sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of the grid size (for HBM counter scaling)")
    ap.add_argument("--serving", action="store_true",
                    help="run only the serving-mix sweep (1000 requests per rate) and print its JSON line")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--trend", action="store_true",
                    help="run only the 2-D size trend (Box-2D49P recipe, square grids 512^2 .. 14336^2) and print "
                         "its JSON line")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (a slab decomposition over several GPUs is not built); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2506_22035_amd as sp
    import stencil_inputs as si

    if args.trend:
        print(json.dumps(size_trend(torch, sp, si, args)))
        return

    if args.workload == "batch3d":
        print(json.dumps(batch3d(torch, sp, si, args)))
        return

    if args.serving:
        res = serving(torch, sp, si, args.serving_requests, [0.25, 0.5, 1.0, 1.5])
        print(json.dumps({"metric": "serving mix: p50/p99 latency (ms) and GStencil/s per Poisson rate",
                          "config": {"workload": "serving_mix", "stencils": list(si.SERVING_STENCILS),
                                     "grids_2d": "512^2..8192^2", "grids_3d": "64^3..384^3", "steps": "1..100",
                                     "carry": "f16"}, "serving": res}))
        return

    wl = si.workload(args.workload)
    if args.carry is None:
        args.carry = "f64" if args.workload == "box2d9p_256_f64" else "f16"
    if args.engine is None:
        args.engine = "sparse" if args.carry in ("f16", "bf16") else "direct"
    if args.split == 0:
        args.split = 3 if (args.carry == "f32" and args.engine != "direct") else 2
    headline = args.workload == "box2d49p_10240" and args.carry in ("f16", "bf16")
    T = wl["steps"]
    shape = tuple(wl["shape"])
    ny, nx = (shape[-2] if len(shape) > 1 else 1), shape[-1]
    npts = int(np.prod(shape))
    x32 = workload_grid(si, args.workload, np.float64 if args.carry == "f64" else np.float32)
    tdt = sp.torch_dtype(args.carry)
    xh = torch.from_numpy(x32).to(tdt)
    xd = xh.to("cuda:0")
    y = torch.empty_like(xd)
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry=args.carry, engine=args.engine, split=args.split,
                   tile_h=args.tile_h, autotune=True, band_height=args.band_height, time_block=args.time_block,
                   row_swap=args.row_swap)
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()

    for _ in range(args.warmup):
        plan.apply(xd, y, T, stream=stream)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    total_ms, per = timed_applies(torch, plan, xd, y, T, args.steps, stream)
    wall_ms = (time.perf_counter() - wall0) * 1e3
    ms_per_step = total_ms / args.steps
    value = gstencil(npts, T * args.steps, total_ms)
    launches, mi_pass = plan.work(T)

    elem = {"f16": 2, "bf16": 2, "f32": 4, "f64": 8}[args.carry]
    operand = args.carry if args.carry in ("f16", "bf16") else "f16"
    rr = (wl["coeffs"].shape[0] - 1) // 2

    def traffic_lookup(tb, tile_h2, grid):
        if headline and args.carry == "f16" and args.engine == "sparse":
            return measured_traffic(tb, tile_h2, grid)
        return None

    roof, sustained = roofline(torch, sp, plan, xd, elem, npts, shape, operand, stream, traffic_lookup, T,
                               ms_per_step)
    roof["kernel"] = kernel_name(info, shape, args.carry, args.engine, rr, args.row_swap)
    ceiling = None
    if "mfma" in roof and not args.no_extras:
        # the matrix pipe's attainable rate at the fused kernel's residency (two waves per
        # SIMD), beside the published peak: power holds the clock below its 2.4 GHz boost
        ceiling = matrix_ceiling(sp, info["engine"], stream)
        att = ceiling["%s_w2" % ("dense" if info["engine"] == "dense" else "sparse")]
        roof["mfma"]["attainable_TFLOPs"] = att["TFLOPs"]
        roof["mfma"]["attainable_source"] = ("spider_measure_matrix_rate, %s fp16, 2 waves per SIMD "
                                             "(the fused kernel's residency)" % info["engine"])
        roof["mfma"]["frac_of_attainable"] = round(roof["mfma"]["TFLOPs"] / att["TFLOPs"], 4)

    # a plain device copy of the same grid: read + write of the same bytes, for reference
    z = torch.empty_like(xd)
    z.copy_(xd)
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ncopy = 10 if not args.copy_calibration else 3
    ce0.record(stream)
    for _ in range(ncopy):
        z.copy_(xd)
    ce1.record(stream)
    torch.cuda.synchronize()
    roof["copy_kernel_GBs"] = round(npts * 2 * elem / (ce0.elapsed_time(ce1) * 1e-3 / ncopy) / 1e9, 1)
    del z

    out = {"metric": METRIC, "value": round(value, 2), "unit": "GStencil/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.carry, "data": "synthetic",
           "config": {"workload": args.workload, "grid": list(shape),
                      "time_steps_per_step": T, "carry": args.carry,
                      "operand": operand if args.engine != "direct" else args.carry,
                      "accumulate": "f32" if args.carry in ("f16", "bf16") else args.carry,
                      "engine": info["engine"], "split": args.split if args.engine != "direct" else None,
                      "tile_h": info["tile_h"],
                      "time_steps_per_launch": info["time_block"], "tile_h2": info["tile_h2"],
                      "band_height": info["band_height"], "row_swap": args.row_swap,
                      "coeff_seed": wl["seeds"]["coeffs"], "grid_seed": wl["seeds"]["grid"]},
           "wall_ms_timed_region": round(wall_ms, 3), "plan_ms": round(plan_ms, 3),
           "latency_ms": {"p50": round(float(np.percentile(per, 50)), 4),
                          "p99": round(float(np.percentile(per, 99)), 4)},
           "sustained": sustained,
           "launches_per_step": launches,
           "matrix_instructions_per_step": mi_pass,
           "roofline": roof}
    if ceiling is not None:
        out["matrix_rate"] = ceiling

    if not args.no_extras:
        oracle = load_oracle()
        got = to_host64(torch, y)
        x64 = xh.to(torch.float64).numpy()
        del y
        tol_key = "f32s3" if (args.carry == "f32" and args.engine != "direct") else args.carry
        out["error_vs_fp64_oracle"] = full_grid_error(oracle, wl["coeffs"], x64, T, got, tol_key)
        del got
        if len(shape) == 2 and args.carry in ("f16", "bf16"):
            # the plain fp32 GPU path and the fp32 carry on the sparse engine (every input
            # value split into 16-bit hi + lo operands, split 3), same workload
            v32, i32, g32, x32h = workload_run(torch, sp, si, args.workload, "f32", "direct", 2, 3, stream)
            out["plain_gpu_fp32"] = {"value": round(v32, 2), "unit": "GStencil/s", "engine": "direct (VALU fp32)",
                                     "speedup_lowp_over_fp32": round(value / v32, 3),
                                     "hbm_compulsory": run_hbm(i32, wl, "f32")}
            del g32
            vm, im, gm, _ = workload_run(torch, sp, si, args.workload, "f32", "sparse", 3, 3, stream)
            out["f32_carry_sparse_split3"] = {
                "value": round(vm, 2), "unit": "GStencil/s", "time_steps_per_launch": im["time_block"],
                "tile_h": im["tile_h2"] or im["tile_h"], "hbm_compulsory": run_hbm(im, wl, "f32"),
                "mfma": run_mfma(im), "error_vs_fp64_oracle": full_grid_error(oracle, wl["coeffs"], x32h, T, gm, "f32s3"),
                "speedup_over_plain_fp32": round(vm / v32, 3)}
            del gm, x32h
            # ablation: the other engine / operand type on the same pass; bf16 with its error
            abl = {}
            for carry, engine in [("f16", "dense"), ("f16", "sparse"), ("bf16", "sparse"), ("bf16", "dense")]:
                if carry == args.carry and engine == args.engine:
                    continue
                keep = carry == "bf16" and engine == "sparse"
                va, ia, ga, xa = workload_run(torch, sp, si, args.workload, carry, engine, 2, 3, stream, keep)
                abl["%s_%s" % (engine, carry)] = round(va, 2)
                if keep:
                    abl["%s_%s_error_vs_fp64_oracle" % (engine, carry)] = full_grid_error(
                        oracle, wl["coeffs"], xa, T, ga, carry)
                del ga, xa
            out["ablation_gstencil_s"] = abl
        if headline:
            out["configs"] = other_configs(torch, sp, si, stream, oracle)
            # serving: saturation and two Poisson loads over 1000 requests of the mix
            # (the four-rate sweep is `bench.py --serving`)
            out["serving_sample"] = serving(torch, sp, si, 1000, [0.5, 1.0])

    if headline and not args.no_cpu_baseline:
        oracle = load_oracle()
        rows, st = ny, 12
        sample = xh[:rows].to(torch.float64).numpy()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.apply(wl["coeffs"], sample, st)
            times.append(time.perf_counter() - t0)
        dt = min(times)
        out["cpu_baseline"] = {"value": round(rows * nx * st / dt / 1e9, 5), "unit": "GStencil/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": "fp64 oracle, all %d rows of the %dx%d grid, %d time steps, best of 3 "
                                         "runs (%.1f s each at best)" % (rows, ny, nx, st, dt)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
