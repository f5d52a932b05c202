#!/usr/bin/env python3
"""Benchmark of the fused hdiff + vadv time step on one MI355X.

Workload: the fused time step at 512 x 512 x 80 (halo 2), FP64, seeded
synthetic fields (u ~ U[0,1), w ~ U[-1,1] on 81 levels, data ~ U[-0.1,0.1],
coeff 0.025, dt/dz 0.5), K steps captured in one hipGraph (ping-pong state,
frozen halo) and timed with HIP events on the capture/launch stream.

Prints ONE JSON line: grid points/s of the step (value), HBM GB/s and the
fraction of the 8 TB/s peak (roofline), the adjoint/forward time ratio,
FP32 and plain-kernel comparisons, and the CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "grid points/s and HBM GB/s (% of peak) for fused hdiff+vadv step; adjoint/fwd ratio"
KERNEL_SOURCES = ["common.hpp", "k_step.hpp", "k_split.hpp", "k_step.hip", "k_step_inst.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_fused_512x512x80_f64.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_08322_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def step_bytes(ni, nj, nk, es, mask=False) -> int:
    """Algorithmic HBM bytes of one fused step: u with its halo, data, the
    interior levels 1..nk-1 of w (w_0 and w_nk never enter the matrix), the
    new interior; plus 2 bits per point when the limiter mask is saved."""
    b = es * (nk * (ni + 4) * (nj + 4) + nk * ni * nj + (nk - 1) * ni * nj + nk * ni * nj)
    if mask:
        b += nk * nj * ((ni + 63) // 64) * 8 * 2 + nk * (ni + nj)
    return b


def adjoint_bytes(ni, nj, nk, es) -> int:
    """Algorithmic bytes of the step adjoint with data_bar: read x_bar, w
    (levels 1..nk-1) and the mask, write u_bar (padded) and data_bar."""
    return es * (nk * ni * nj + (nk - 1) * ni * nj + nk * (ni + 4) * (nj + 4) + nk * ni * nj) + \
        nk * nj * ((ni + 63) // 64) * 16 + nk * (ni + nj)


def adjoint_kernel_bytes(ni, nj, nk, es) -> int:
    """Algorithmic bytes of the two kernels the step adjoint runs: the
    column adjoint (read x_bar and w, write lambda = data_bar) and the
    gather (read lambda and the mask, write u_bar): the step adjoint's
    bytes plus lambda read back once."""
    return adjoint_bytes(ni, nj, nk, es) + es * nk * ni * nj


def stream_mix_bandwidth(mib: int, reps: int) -> dict:
    """One elementwise pass that reads three arrays and writes a fourth
    (torch.addcmul over `mib` MiB each): plain streaming with the fused
    step's 3:1 read/write mix, the practical ceiling for its traffic."""
    import torch

    n = mib * 1024 * 1024 // 8
    a, b, c = (torch.full((n,), 0.5, dtype=torch.float64, device="cuda") for _ in range(3))
    d = torch.empty_like(a)
    torch.addcmul(a, b, c, out=d)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.addcmul(a, b, c, out=d)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    return {"gbs": round(4 * n * 8 / t / 1e9, 1),
            "what": f"torch.addcmul over {mib} MiB FP64 arrays: 3 streams read, 1 written"}


def split_class(nkh: int) -> int:
    """Half-column register class of the two-ended FP64 step kernel."""
    for c in (16, 24, 40):
        if nkh <= c:
            return c
    return 72


def copy_bandwidth(mib: int, reps: int) -> dict:
    """A plain device-to-device copy of `mib` MiB (reads and writes that many
    bytes): the achievable-bandwidth reference and the known-size kernel
    the HBM byte counters are scaled by."""
    import torch

    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    return {"copy_mib": mib, "bytes_per_copy": 2 * n * 8, "s_per_copy": t, "gbs": round(2 * n * 8 / t / 1e9, 1)}


def bench_batched(api, fields, inputs, time_eager, dtype) -> dict:
    """The 32-field uneven workload: the forward step as one persistent
    launch against 32 separate fused launches (and, in FP64, 32 plain
    per-stage chains), and the step adjoint of the batch (with data_bar)
    against 32 separate adjoint calls."""
    import torch

    dev = "cuda:0"
    es = 8 if dtype == torch.float64 else 4
    items, adj, pts, byts, abyts = [], [], 0, 0, 0
    for ni, nj, nk, f in inputs.batch_fields():
        dims = (ni, nj, nk)
        it = dict(u=fields.from_padded(f.u, dtype, dev), data=fields.from_interior(f.data, dtype, dev),
                  w=fields.from_interior(f.w, dtype, dev), out=fields.alloc(ni, nj, nk, dtype, dev, fill=0.0),
                  domain=dims, coeff=inputs.COEFF, dt_dz=inputs.DT_DZ, mask=None)
        items.append(it)
        adj.append(dict(x_bar=fields.from_interior(inputs.cotangent(ni, nj, nk), dtype, dev), w=it["w"],
                        u_bar=fields.alloc(ni, nj, nk, dtype, dev, fill=0.0),
                        data_bar=fields.alloc(ni, nj, nk, dtype, dev, halo=0, fill=0.0), domain=dims,
                        coeff=inputs.COEFF, dt_dz=inputs.DT_DZ, mask=fields.mask_tensor(dims, dev)))
        pts += ni * nj * nk
        byts += step_bytes(ni, nj, nk, es)
        abyts += adjoint_bytes(ni, nj, nk, es)
    ws = torch.empty(api.stencil_batch_workspace_bytes(dtype, items), dtype=torch.uint8, device=dev)
    t_batch = time_eager(lambda: api.stencil_step_batched(dtype, items, ws), reps=10)

    def separate():
        for it in items:
            api.stencil_step(it["u"], it["data"], it["w"], it["out"], it["domain"], inputs.COEFF, inputs.DT_DZ)

    t_sep = time_eager(separate, reps=10)
    res = {"fields": len(items), "points": pts, "dtype": "f64" if es == 8 else "f32",
           "persistent_ms": round(t_batch * 1e3, 4), "separate_ms": round(t_sep * 1e3, 4),
           "points_per_s": round(pts / t_batch, 1), "gbs": round(byts / t_batch / 1e9, 1),
           "frac": round(byts / t_batch / 1e9 / PEAK_GBS, 4)}
    if es == 8:
        po = api.Options(impl=api.IMPL_PLAIN)
        po.workspace = torch.empty(max(api.stencil_workspace_bytes(api.OP_STEP, api.F64, it["domain"], po)
                                       for it in items), dtype=torch.uint8, device=dev)

        def plain():
            for it in items:
                api.stencil_step(it["u"], it["data"], it["w"], it["out"], it["domain"], inputs.COEFF,
                                 inputs.DT_DZ, opts=po)

        res["plain_ms"] = round(time_eager(plain, reps=3) * 1e3, 4)
    # the forward saving its masks, then the adjoint of the batch on them
    for it, a in zip(items, adj):
        it["mask"] = a["mask"]
    t_mask = time_eager(lambda: api.stencil_step_batched(dtype, items, ws), reps=10)
    res["persistent_mask_ms"] = round(t_mask * 1e3, 4)
    torch.cuda.synchronize()
    aws = torch.empty(api.stencil_batch_adjoint_workspace_bytes(dtype, adj), dtype=torch.uint8, device=dev)
    t_adj = time_eager(lambda: api.stencil_step_adjoint_batched(dtype, adj, aws), reps=10)

    def separate_adj():
        for a in adj:
            api.stencil_step_adjoint(a["x_bar"], a["w"], a["mask"], a["u_bar"], a["data_bar"], a["domain"],
                                     inputs.COEFF, inputs.DT_DZ)

    t_adj_sep = time_eager(separate_adj, reps=10)
    res["adjoint"] = {"persistent_ms": round(t_adj * 1e3, 4), "separate_ms": round(t_adj_sep * 1e3, 4),
                      "gbs": round(abyts / t_adj / 1e9, 1), "frac": round(abyts / t_adj / 1e9 / PEAK_GBS, 4),
                      "ratio_adj_over_fwd_mask": round(t_adj / t_mask, 3)}
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inputs, f512, adj32) -> dict:
    """The CPU oracle (plain FP64 C loops) timed on the host: one step of
    the 256x256x80 and 512x512x80 workloads and one step adjoint of the
    256x256x80 workload, each single-threaded and with OpenMP on every
    thread the process may use, median of 3 runs.  `value` is the all-cores
    512x512x80 step rate.  With adj32 (the GPU's FP32 adjoint of the
    256x256x80 workload and its forward mask), the oracle's adjoint on the
    same binary32-rounded inputs and mask also gives that result's error."""
    import numpy as np

    from oracle import oracle as orc
    from tests.helpers import rel_err, round_f32, unpack_mask

    print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
    f256 = inputs.fields_for(inputs.STEP_256)
    w4 = inputs.ADJ_256
    f4 = inputs.fields_for(w4)
    ob4 = inputs.cotangent(w4.ni, w4.nj, w4.nk)
    mx4, my4 = orc.hdiff_masks(f4.u)
    C, R = inputs.COEFF, inputs.DT_DZ
    work = [("step 256x256x80", 256 * 256 * 80, lambda: orc.step(f256.u, f256.data, f256.w, C, R)),
            ("step 512x512x80", 512 * 512 * 80, lambda: orc.step(f512.u, f512.data, f512.w, C, R)),
            ("step adjoint 256x256x80", 256 * 256 * 80, lambda: orc.step_adjoint(ob4, f4.w, mx4, my4, C, R))]

    def med3(fn):
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[1]

    legs, t_total = [], time.perf_counter()
    threads = 1
    for mode in ("single", "openmp"):
        for name, pts, fn in work:
            if mode == "openmp":
                with orc.threaded():
                    threads = orc.threads()
                    t = med3(fn)
            else:
                t = med3(fn)
            legs.append({"workload": name, "threads": 1 if mode == "single" else threads,
                         "ms": round(t * 1e3, 2), "points_per_s": round(pts / t, 1)})
    # the whole-array NumPy step: the analogue of the paper's numpy backend
    # (the same results bit for bit), single-threaded as NumPy's elementwise
    # operations are
    from oracle import numpy_step

    t = med3(lambda: numpy_step.step(f512.u, f512.data, f512.w, C, R))
    legs.append({"workload": "step 512x512x80", "threads": 1, "kind": "numpy (whole-array operations)",
                 "ms": round(t * 1e3, 2), "points_per_s": round(512 * 512 * 80 / t, 1)})
    head = [g for g in legs if g["workload"] == "step 512x512x80" and g["threads"] == threads
            and "kind" not in g][-1]
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    res = {"value": head["points_per_s"], "unit": "grid points/s", "cores": threads, "kind": "oracle",
           "sample": "median of 3 runs of one FP64 step of the 512x512x80 workload on every host thread "
                     "(OpenMP over independent levels and columns); the legs below time the 256x256x80 "
                     "step and step adjoint and the single-threaded runs too",
           "nproc": os.cpu_count(), "affinity": affinity, "cpu_model": cpu_model(), "legs": legs,
           "wall_s": round(time.perf_counter() - t_total, 1)}
    if adj32 is not None:
        d4 = (w4.ni, w4.nj, w4.nk)
        gx, gy = unpack_mask(adj32["mask"], *d4)
        with orc.threaded():
            ubr, dbr = orc.step_adjoint(round_f32(ob4), round_f32(f4.w), gx, gy, float(np.float32(C)), R)
        res["fp32_adjoint_256_rel_err"] = {"u_bar": rel_err(adj32["ub"], ubr), "data_bar": rel_err(adj32["db"], dbr),
                                           "what": "GPU FP32 step adjoint at 256x256x80 vs the FP64 oracle on "
                                                   "the binary32-rounded cotangent and w with the GPU's FP32 mask "
                                                   "(relative inf-norm error per output)"}
    return res


def paper_context(cb: dict, t_step: float, call_us) -> dict:
    """The paper's own comparisons (Sec. 3.1, Fig. 3; ratios only, no
    absolute numbers are printed) beside the same ratios measured here.
    Context, not targets: other hardware, other domain sizes."""
    def leg(threads, kind=None):
        for g in cb["legs"]:
            if g["workload"] == "step 512x512x80" and g["threads"] == threads and g.get("kind") == kind:
                return g["ms"] / 1e3
        return None

    t_np, t_omp = leg(1, "numpy (whole-array operations)"), leg(cb["cores"])
    return {
        "compiled_cpu_vs_numpy": {
            "paper": ">= 10x (generated C++ CPU backends vs the numpy backend; 12-core Xeon E5-2690)",
            "here": round(t_np / t_omp, 1) if t_np and t_omp else None,
            "what": "oracle C loops on every host thread vs the whole-array NumPy step, 512x512x80 FP64"},
        "gpu_vs_cpu": {
            "paper": "5-10x (generated CUDA on a P100 vs the CPU backends on that Xeon)",
            "here": round(t_omp / t_step, 1) if t_omp else None,
            "what": "fused HIP step on one MI355X vs the oracle on every host thread, 512x512x80 FP64"},
        "python_call_overhead": {
            "paper": "about 1 ms per call on small domains (run-time checks of layout and dtype)",
            "here_us": call_us,
            "what": "Python call of the step on an 8x8x8 domain, field descriptors kept between calls"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only-step", action="store_true", help="time the fused forward step only")
    ap.add_argument("--with-frontend", action="store_true",
                    help="with --only-step: also time the step written in the stencil language")
    ap.add_argument("--with-adjoint", action="store_true",
                    help="with --only-step: also run the step adjoint a few times (counter collection)")
    ap.add_argument("--with-f32", action="store_true",
                    help="with --only-step: also run the FP32 step of every tile (counter collection)")
    ap.add_argument("--reps", type=int, default=10, help="graph replays for the median")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only time a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); multi-GPU runs are not "
              "part of it", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2311_08322_amd import api, fields, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.copy_mib:
        print(json.dumps(copy_bandwidth(args.copy_mib, args.reps)), flush=True)
        return
    wl = inputs.STEP_512
    ni, nj, nk = wl.ni, wl.nj, wl.nk
    dims = (ni, nj, nk)
    npts = ni * nj * nk
    f = inputs.fields_for(wl)
    K, W = args.steps, args.warmup
    out = {}
    adj32 = None

    def mkfields(dtype):
        u_a = fields.from_padded(f.u, dtype, dev)
        u_b = fields.from_padded(f.u, dtype, dev)
        data = fields.from_interior(f.data, dtype, dev)
        w = fields.from_interior(f.w, dtype, dev)
        return u_a, u_b, data, w

    tuned = {}

    def time_graph(dtype, nsteps, reps):
        u_a, u_b, data, w = mkfields(dtype)
        s = torch.cuda.Stream()
        # the library's autotuner picks tile, column store and tile order for
        # this size class on the very buffers the graph will step (where the
        # fields sit in memory matters as well as their shape)
        print(f"bench: autotuning the fused step ({dtype}) on its fields", file=sys.stderr, flush=True)
        api.stencil_autotune_fields(u_a, data, w, u_b, dims, reps=10, stream=s)
        tuned["f64" if dtype == torch.float64 else "f32"] = api.stencil_tuning_lookup(dtype, api.OP_STEP, dims)
        for n in range(W):  # eager warm-up steps
            src, dst = (u_a, u_b) if n % 2 == 0 else (u_b, u_a)
            api.stencil_step(src, data, w, dst, dims, inputs.COEFF, inputs.DT_DZ, stream=s)
        g = api.stencil_graph_capture_steps(nsteps, u_a, u_b, data, w, dims, inputs.COEFF, inputs.DT_DZ,
                                            stream=s)
        try:
            api.stencil_graph_launch(g, stream=s)  # warm replay
            s.synchronize()
            times = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                e0.record(s)
                api.stencil_graph_launch(g, stream=s)
                e1.record(s)
                s.synchronize()
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                times.append((e0.elapsed_time(e1) / 1e3, wall))
        finally:
            api.stencil_graph_destroy(g)
        times.sort()
        return times[len(times) // 2]

    def time_eager(fn, reps=20, warm_s=0.03, windows=3):
        """Per-call time of back-to-back eager calls: the median of `windows`
        windows of `reps` calls, after calling fn for at least warm_s seconds
        of device time (the first milliseconds after a change of workload
        run measurably slower)."""
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        warm, calls = 0.0, 0
        while warm < warm_s and calls < 2000:
            e0.record(s)
            for _ in range(4):
                fn()
            e1.record(s)
            torch.cuda.synchronize()
            warm += e0.elapsed_time(e1) / 1e3
            calls += 4
        ts = []
        for _ in range(windows):
            e0.record(s)
            for _ in range(reps):
                fn()
            e1.record(s)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3 / reps)
        return sorted(ts)[len(ts) // 2]

    # ---------------------------------------------------------------- FP64 step
    print(f"bench: fused step {dims} fp64, {K} steps per graph, {args.reps} replays", file=sys.stderr,
          flush=True)
    t_ev, t_wall = time_graph(torch.float64, K, args.reps)
    t_step = t_ev / K
    b64 = step_bytes(ni, nj, nk, 8)
    gbs = b64 / t_step / 1e9
    ti, tj, col, _ = tuned["f64"]
    nkh = nk - nk // 2
    kname = (f"k_step_split<double, {ti}, {tj}, {split_class(nkh)}, 2, false, {1 if nk <= 80 else 2}, false>"
             if col == api.COLUMN_SPLIT else f"k_step_fused<double, {ti}, {tj}, 80, 2, {col}>")
    # measured HBM bytes of this kernel (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    # copy-calibrated), valid only while the kernel sources are unchanged
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        key = f"{kname} order={tuned['f64'][3]}"
        if tr.get("kernel_hash") == kernel_hash() and key in tr.get("kernels", {}):
            traffic = round(tr["kernels"][key]["bytes_per_launch"])
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": b64, "kernel": kname, "tile_order": tuned["f64"][3],
            "avg_launch_us": round(t_step * 1e6, 2)}
    out.update({
        "metric": METRIC, "value": round(npts * K / t_ev, 1), "unit": "grid points/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded U[0,1) u, U[-1,1] w, U[-0.1,0.1] data)",
        "config": {"workload": "fused hdiff+vadv step 512x512x80, halo 2, hipGraph of K steps",
                   "ni": ni, "nj": nj, "nk": nk, "graph_steps": K, "wall_s_per_graph": round(t_wall, 6),
                   "tuned_tile_f64": f"{tuned['f64'][0]}x{tuned['f64'][1]}", "column_store_f64": tuned["f64"][2],
                   "tile_order_f64": tuned["f64"][3]},
        "roofline": roof,
    })

    if args.only_step:
        # a few eager launches of the step kernel of every tile (the tuned
        # one among them): counter collection sees dispatches outside graph
        # replays, and every tile the tuner may pick gets measured
        def every_tile(dtype):
            u_a, u_b, data, w = mkfields(dtype)
            for tile in (64, 32, 16):
                for nt in (256, 128):  # both workgroup sizes
                    for order in (api.ORDER_XCD, api.ORDER_DISPATCH):
                        o = api.Options(tile_i=tile, tile_j=nt // tile, column_store=api.COLUMN_SPLIT,
                                        tile_order=order)
                        for n in range(3):
                            api.stencil_step(u_a, data, w, u_b, dims, inputs.COEFF, inputs.DT_DZ, opts=o)
            return u_a, u_b, data, w

        if args.with_f32:
            every_tile(torch.float32)
            torch.cuda.synchronize()
        u_a, u_b, data, w = every_tile(torch.float64)
        if args.with_adjoint:
            # the step adjoint (column adjoint + gather) on the forward's mask
            mask = fields.mask_tensor(dims, dev)
            api.stencil_step(u_a, data, w, u_b, dims, inputs.COEFF, inputs.DT_DZ, mask=mask)
            xb = fields.from_interior(inputs.cotangent(ni, nj, nk), torch.float64, dev)
            ub = fields.alloc(ni, nj, nk, torch.float64, dev, fill=0.0)
            db = fields.alloc(ni, nj, nk, torch.float64, dev, halo=0, fill=0.0)
            for n in range(3):
                api.stencil_step_adjoint(xb, w, mask, ub, db, dims, inputs.COEFF, inputs.DT_DZ)
            del mask, xb, ub, db
        torch.cuda.synchronize()
        del u_a, u_b, data, w
    if not args.only_step:
        # ------------------------------------------------------------ FP32 step
        print("bench: fused step fp32", file=sys.stderr, flush=True)
        t32, _ = time_graph(torch.float32, K, args.reps)
        out["config"].update({"tuned_tile_f32": f"{tuned['f32'][0]}x{tuned['f32'][1]}",
                              "column_store_f32": tuned["f32"][2], "tile_order_f32": tuned["f32"][3]})
        b32 = step_bytes(ni, nj, nk, 4)
        out["fp32"] = {"value": round(npts * K / t32, 1), "unit": "grid points/s",
                       "ms_per_step": round(t32 / K * 1e3, 4), "gbs": round(b32 / (t32 / K) / 1e9, 1),
                       "frac": round(b32 / (t32 / K) / 1e9 / PEAK_GBS, 4)}
        # ------------------------------------------------ adjoint / forward ratio
        print("bench: adjoint vs forward (eager, mask saved)", file=sys.stderr, flush=True)
        u_a, u_b, data, w = mkfields(torch.float64)
        mask = fields.mask_tensor(dims, dev)
        xb = fields.from_interior(inputs.cotangent(ni, nj, nk), torch.float64, dev)
        ub = fields.alloc(ni, nj, nk, torch.float64, dev, fill=0.0)
        db = fields.alloc(ni, nj, nk, torch.float64, dev, halo=0, fill=0.0)
        t_fwd = time_eager(lambda: api.stencil_step(u_a, data, w, u_b, dims, inputs.COEFF, inputs.DT_DZ,
                                                    mask=mask))
        t_adj = time_eager(lambda: api.stencil_step_adjoint(xb, w, mask, ub, db, dims, inputs.COEFF,
                                                            inputs.DT_DZ))
        ab = adjoint_bytes(ni, nj, nk, 8)
        out["adjoint"] = {"ratio_adj_over_fwd": round(t_adj / t_fwd, 3), "fwd_mask_ms": round(t_fwd * 1e3, 4),
                          "adj_ms": round(t_adj * 1e3, 4), "adj_gbs": round(ab / t_adj / 1e9, 1),
                          "adj_frac": round(ab / t_adj / 1e9 / PEAK_GBS, 4),
                          "adj_kernels_gbs": round(adjoint_kernel_bytes(ni, nj, nk, 8) / t_adj / 1e9, 1),
                          "fwd_mask_gbs": round(step_bytes(ni, nj, nk, 8, True) / t_fwd / 1e9, 1)}
        # ---------------------------- the adjoint workload 256x256x80, rotating sets
        # one set (about 170 MB in FP64) fits the 256 MB last-level cache, so
        # R sets (> 512 MB together in FP64) are cycled and each call touches
        # a cold set
        w4 = inputs.ADJ_256
        d4 = (w4.ni, w4.nj, w4.nk)
        f4 = inputs.fields_for(w4)
        ob4 = inputs.cotangent(*d4)
        for dtype, key, nsets in ((torch.float64, "adjoint_256", 4), (torch.float32, "adjoint_256_f32", 8)):
            print(f"bench: adjoint vs forward at 256x256x80 {key} (rotating buffer sets)", file=sys.stderr,
                  flush=True)
            sets = []
            for _ in range(nsets):
                sets.append(dict(u=fields.from_padded(f4.u, dtype, dev),
                                 data=fields.from_interior(f4.data, dtype, dev),
                                 w=fields.from_interior(f4.w, dtype, dev),
                                 out=fields.alloc(*d4, dtype, dev, halo=0, fill=0.0),
                                 mask=fields.mask_tensor(d4, dev),
                                 xb=fields.from_interior(ob4, dtype, dev),
                                 ub=fields.alloc(*d4, dtype, dev, fill=0.0),
                                 db=fields.alloc(*d4, dtype, dev, halo=0, fill=0.0)))
            rot = {"n": 0}

            def fwd4():
                z = sets[rot["n"] % len(sets)]
                rot["n"] += 1
                api.stencil_step(z["u"], z["data"], z["w"], z["out"], d4, inputs.COEFF, inputs.DT_DZ,
                                 mask=z["mask"])

            def adj4():
                z = sets[rot["n"] % len(sets)]
                rot["n"] += 1
                api.stencil_step_adjoint(z["xb"], z["w"], z["mask"], z["ub"], z["db"], d4, inputs.COEFF,
                                         inputs.DT_DZ)

            t_f4 = time_eager(fwd4, reps=40)
            t_a4 = time_eager(adj4, reps=40)
            es = 8 if dtype == torch.float64 else 4
            ab4 = adjoint_bytes(*d4, es)
            out[key] = {"ratio_adj_over_fwd": round(t_a4 / t_f4, 3), "fwd_mask_ms": round(t_f4 * 1e3, 4),
                        "adj_ms": round(t_a4 * 1e3, 4), "adj_gbs": round(ab4 / t_a4 / 1e9, 1),
                        "adj_frac": round(ab4 / t_a4 / 1e9 / PEAK_GBS, 4),
                        "what": f"step adjoint (with data_bar) vs forward step saving the mask, 256x256x80 "
                                f"{'FP64' if es == 8 else 'FP32'}, {nsets} rotating buffer sets of "
                                f"~{round(ab4 / 1e6)} MB"}
            if dtype == torch.float32:
                # the outputs of set 0 (forward mask, u_bar, data_bar) for the
                # error statement the CPU leg makes from its own adjoint run
                z = sets[0]
                torch.cuda.synchronize()
                adj32 = dict(mask=z["mask"].cpu(), ub=fields.padded(z["ub"], *d4).cpu().numpy(),
                             db=fields.interior(z["db"], *d4).cpu().numpy())
            del sets
        # ------------------------------------------------ plain per-stage chain
        print("bench: plain per-stage kernels", file=sys.stderr, flush=True)
        po = api.Options(impl=api.IMPL_PLAIN)
        po.workspace = fields.workspace(api.OP_STEP, torch.float64, dims, po)
        t_plain = time_eager(lambda: api.stencil_step(u_a, data, w, u_b, dims, inputs.COEFF, inputs.DT_DZ,
                                                      opts=po), reps=10)
        del po
        out["plain"] = {"ms_per_step": round(t_plain * 1e3, 4), "fused_speedup": round(t_plain / t_step, 3)}
        # ------------------------------------------------ call vs kernel time
        s = torch.cuda.current_stream()
        torch.cuda.synchronize()
        n = 50
        t0 = time.perf_counter()
        for _ in range(n):
            api.stencil_step(u_a, data, w, u_b, (8, 8, 8), inputs.COEFF, inputs.DT_DZ)
        host_call = (time.perf_counter() - t0) / n
        torch.cuda.synchronize()
        out["python_call_us"] = round(host_call * 1e6, 2)
        del u_a, u_b, data, w, mask, xb, ub, db

    # ------------------------------------------------ the frontend's generated step
    if not args.only_step or args.with_frontend:
        print("bench: the step written in the stencil language (generated HIP)", file=sys.stderr, flush=True)
        from paper_2311_08322_amd.frontend import stencils as fs

        u_a, u_b, data, w = mkfields(torch.float64)
        xo = fields.alloc(ni, nj, nk, torch.float64, dev, halo=0, fill=0.0)
        fs.step.build("float64")
        t_gen = time_eager(lambda: fs.step(u_a, data, w, xo, coeff=inputs.COEFF, dt_dz=inputs.DT_DZ,
                                           domain=dims), reps=20)
        bg = step_bytes(ni, nj, nk, 8)
        out["frontend"] = {"ms_per_step": round(t_gen * 1e3, 4), "alg_gbs": round(bg / t_gen / 1e9, 1),
                           "frac": round(bg / t_gen / 1e9 / PEAK_GBS, 4),
                           "handwritten_speedup": round(t_gen / t_step, 3),
                           "what": "the step written in the stencil language: one generated kernel "
                                   "(the run of parallel computations fused into the forward sweep, the "
                                   "backward sweep appended; c' and d' through a workspace), timed "
                                   "eagerly; the same algorithmic bytes as the fused step"}
        del u_a, u_b, data, w, xo

    # ------------------------------------------------ batched uneven fields
    if not args.only_step:
        print("bench: 32 uneven fields, persistent launch vs separate launches", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(api, fields, inputs, time_eager, torch.float64)
        out["batched_f32"] = bench_batched(api, fields, inputs, time_eager, torch.float32)

    # ------------------------------------------------------ achievable bandwidth
    if not args.only_step:
        cb = copy_bandwidth(1024, 10)
        out["copy_reference"] = {"gbs": cb["gbs"], "what": "torch device copy of 1 GiB (read + write)",
                                 "step_frac_of_copy": round(gbs / cb["gbs"], 4)}
        sm = stream_mix_bandwidth(512, 10)
        out["stream_reference"] = {"gbs": sm["gbs"], "what": sm["what"],
                                   "step_frac_of_stream": round(gbs / sm["gbs"], 4)}

    # -------------------------------------------------------------- CPU baseline
    if not args.no_cpu:
        cb = out["cpu_baseline"] = cpu_baseline(inputs, f, adj32 if not args.only_step else None)
        if not args.only_step:
            out["paper_context"] = paper_context(cb, t_step, out.get("python_call_us"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
