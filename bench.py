#!/usr/bin/env python
"""Benchmark of the restarted narrow-band fast marching solver on one MI355X.

Default workload: the 1024^3 full-domain march with an FP32 random speed field
(F = clip(exp(0.5 g), 0.25, 4), g a Gaussian field with correlation length
0.05) and four point sources, FP64 arithmetic, 8^3 tiles, the restart stride
swept by the library's autotuner (3h, 4h and 5h by default).
Prints one JSON line: accepted grid points per second of the whole solve with
inputs resident in HBM, the roofline of the restart driver (the dominant
kernel) and a CPU baseline from the oracle on a bounded sample.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid pts accepted/s @1024^3 FP64; batch vs serial; adjoint/forward time"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per accepted point of a whole solve: read F once, write T
# once (FP64, 8 B) and the status byte once: 13 B with FP32 speeds, 17 B with
# FP64 speeds.  The restart driver itself moves the first two (12 B / 16 B);
# the finalize kernel writes the outputs.
SOLVE_BYTES_PER_POINT = {torch.float32: 13, torch.float64: 17}
DRIVER_BYTES_PER_POINT = {torch.float32: 12, torch.float64: 16}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "driver_traffic_random_speed_1024.txt")
# the paper's restart strides (Sec. 5.1) plus the tuned range, in units of h
PAPER_STRIDE_TABLE = "8:0.5,1.5,2,2.5,3.5,4,inf"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def read_traffic(kernel_tag, stride_h):
    """HBM bytes per driver launch from the committed rocprofv3 counter summary,
    if it was taken with the current kernel build (tag match) at the same
    restart stride (lines "hbm_bytes_per_launch_stride_<s>h: <bytes>"); else
    None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_tag") != kernel_tag:
        return None
    try:
        return float(vals[f"hbm_bytes_per_launch_stride_{float(stride_h):g}h"])
    except (KeyError, ValueError):
        return None


def _code_only(text):
    """C++ source without comments, string literals kept, and without blank
    lines or trailing spaces: the tag follows the code, not its comments."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = [l.rstrip() for l in "".join(out).split("\n")]
    return "\n".join(l for l in lines if l)


def kernel_tag():
    """Hash of the driver's sources (code only), tying the committed HBM
    counter summary to the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("fmm_kernels.hip", "fmm_internal.h", "fmm_device.h", "fmm_tile.h", "fmm_api.cpp"):
        with open(os.path.join(ROOT, "paper_1502_07303_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def host_info():
    """CPU model, logical CPUs, the CPUs this process may use, and host RAM."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    mem = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "mem_total_GiB": mem}


class pinned_to_one_core:
    """Run the calling thread on a single core (the first it may use), then
    restore its affinity: the oracle is single-threaded and timed pinned."""

    def __enter__(self):
        self.saved = os.sched_getaffinity(0)
        self.core = min(self.saved)
        os.sched_setaffinity(0, {self.core})
        return self

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.saved)


def time_oracle(F, h, idx, val, width=math.inf, runs=5):
    """The oracle as it stands (one thread, pinned to one core), ``runs``
    times on the same inputs; init + heap + march timed, inputs prepared
    outside.  Returns the median, mean and minimum seconds and the count of
    accepted points."""
    import oracle
    oracle._load()
    secs, acc = [], None
    with pinned_to_one_core() as pin:
        for _ in range(runs):
            t0 = time.perf_counter()
            T, st, stats, _ = oracle.solve(F, h, idx, val, width=width)
            secs.append(time.perf_counter() - t0)
            acc = int(stats.n_accepted)
            del T, st
    return {"runs": runs, "median_s": round(float(np.median(secs)), 4), "mean_s": round(float(np.mean(secs)), 4),
            "min_s": round(float(np.min(secs)), 4), "accepted": acc,
            "points_per_s": acc / float(np.median(secs)), "core": pin.core}


def cpu_baseline(w, crop, small=None):
    """The oracle on a bounded sample of the benchmark workload: the crop^3
    block of the same FP32 speed field around source 0, one run, pinned to
    one core.  ``small``: oracle 5-run medians of the point-source and
    sphere workloads (see gpu_small_configs)."""
    F = w.F
    n = F.shape[0]
    src = [tuple(p) for p in w.meta["sources"]]
    c0 = [min(max(s - crop // 2, 0), n - crop) for s in src[0]]
    sub = F[c0[0]:c0[0] + crop, c0[1]:c0[1] + crop, c0[2]:c0[2] + crop].contiguous().cpu().numpy()
    inside = [tuple(s[k] - c0[k] for k in range(3)) for s in src
              if all(c0[k] <= s[k] < c0[k] + crop for k in range(3))]
    idx = np.array([(a * crop + b) * crop + c for a, b, c in inside], dtype=np.int64)
    val = np.zeros(len(idx))
    r = time_oracle(sub, w.h, idx, val, runs=1)
    return {"value": r["points_per_s"], "unit": "grid points/s", "cores": 1, "kind": "oracle",
            "seconds": r["median_s"], "accepted": r["accepted"],
            "sample": (f"oracle full-domain march on the {crop}^3 crop of the {n}^3 FP32 speed field "
                       f"at corner {tuple(c0)} with the {len(idx)} source(s) inside it, h = 1/{n - 1}, "
                       f"one thread pinned to core {r['core']}, init + heap + march timed, one run"),
            "build": "gcc -O3 -ffp-contract=off -fno-fast-math (oracle/build.py)",
            "host": host_info(), "configs": small}


def gpu_small_configs(fmm, inputs, dev, steps, with_oracle=True):
    """The point-source (64^3, F = 1 FP64, one source at the centre, full
    march) and sphere-reinitialisation (256^3, 8 spheres, band 0.1, both
    sides, FP64) workloads: GPU solve time (1 warm-up, then ``steps`` timed
    solves; HIP events on the stream) at the paper's stride 2h and at 4h /
    infinity, and the oracle's 5-run median on one pinned core."""
    out = {}
    for name, w, strides in (("point_source_64", inputs.point_source(64), (2.0, math.inf)),
                             ("spheres_256", inputs.spheres(n=256), (2.0, 4.0))):
        wd = w.to(dev)
        T = torch.empty(w.shape, dtype=torch.float64, device=dev)
        st = torch.empty(w.shape, dtype=torch.uint8, device=dev)
        res = {"points": int(w.F.numel()), "seeds": int(w.seed_idx.numel()), "band_width": w.width}
        stream = torch.cuda.current_stream()
        for sh in strides:
            sv = fmm.Solver(w.shape, w.seed_idx.numel(), w.h, band_width=w.width, stride=sh * w.h, timing=True,
                            device=dev, speed_dtype=w.F.dtype)
            sv.solve_into(wd.F, wd.seed_idx, wd.seed_val, T, st)
            sv.stats()
            ms, drv = [], []
            for _ in range(max(steps, 5)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                sv.solve_into(wd.F, wd.seed_idx, wd.seed_val, T, st)
                e1.record(stream)
                s2 = sv.stats()
                ms.append(e0.elapsed_time(e1))
                drv.append(s2.ms_driver)
            acc = int(s2.n_accepted)
            res[f"gpu_{sh:g}h"] = {"ms_median": round(float(np.median(ms)), 4),
                                   "ms_mean": round(float(np.mean(ms)), 4), "ms_min": round(float(np.min(ms)), 4),
                                   "driver_ms_median": round(float(np.median(drv)), 4), "reps": len(ms),
                                   "accepted": acc, "restarts": int(s2.n_restarts),
                                   "points_per_s": acc / (float(np.median(ms)) / 1e3)}
            log(f"  {name} stride {sh:g}h: median {np.median(ms):.3f} ms, {acc} accepted, "
                f"{s2.n_restarts} restarts")
            del sv
        if with_oracle:
            F, idx, val = w.numpy()
            res["oracle"] = time_oracle(F, w.h, idx, val, width=w.width, runs=5)
            log(f"  {name} oracle: median {res['oracle']['median_s']} s")
        out[name] = res
        del T, st, wd
    return out


def batch_vs_serial(fmm, inputs, dev, steps, tune=True):
    """The 64-problem batch (cube edges 32-192, smooth FP64 speeds in (0.5, 2),
    1-4 point sources each): one persistent batched launch (autotuned tile edge
    and stride) against 64 sequential plain solves of the same problems."""
    ws = inputs.batch_problems(64, seed=0, device=dev)
    probs = [{"F": w.F, "h": w.h, "seed_idx": w.seed_idx, "seed_val": w.seed_val} for w in ws]
    n_pts = sum(w.F.numel() for w in ws)
    n_seeds = sum(w.seed_idx.numel() for w in ws)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        return best

    # serial: one plain solve per problem, library defaults (8^3 tiles, stride 2h)
    solvers = [fmm.Solver(w.shape, w.seed_idx.numel(), w.h, device=dev) for w in ws]
    outs = [(torch.empty(w.shape, dtype=torch.float64, device=dev), torch.empty(w.shape, dtype=torch.uint8,
                                                                                 device=dev)) for w in ws]

    def serial():
        for sv, w, (T, st) in zip(solvers, ws, outs):
            sv.solve_into(w.F, w.seed_idx, w.seed_val, T, st)

    ms_serial = timed(serial, steps)
    acc_serial = sum(sv.stats().n_accepted for sv in solvers)
    del solvers

    b = fmm.BatchSolver(probs, workspace_edges=[4, 8, 16])
    ms_default = timed(b.solve, steps)
    tune_ms, t0 = None, time.perf_counter()
    if tune:
        tune_ms = b.tune(edges=(4, 8, 16), strides_h=(1.0, 2.0, 4.0, 8.0), reps=1)
    tune_s = time.perf_counter() - t0
    ms_batch = timed(b.solve, steps)
    st = b.stats()
    acc_batch = sum(x.n_accepted for x in st)
    # the same launch sequence captured in a HIP graph and replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            b.solve(stream=side)
    stream.wait_stream(side)
    ms_graph = timed(g.replay, steps)
    b.stats()
    return {"config": "64 problems, cube edges U{32..192} (seeded), FP64 speed 2^tanh(g) in (0.5, 2) with "
                      "correlation length 0.1, 1-4 point sources each, full march",
            "problems": 64, "points": n_pts, "seeds": n_seeds, "accepted": acc_batch,
            "accepted_serial": acc_serial,
            "serial_ms": round(ms_serial, 3), "batched_default_ms": round(ms_default, 3),
            "batched_ms": round(ms_batch, 3), "graph_replay_ms": round(ms_graph, 3),
            "speedup": round(ms_serial / ms_batch, 3), "speedup_graph": round(ms_serial / ms_graph, 3),
            "batched_points_per_s": acc_batch / (ms_batch / 1e3),
            "tuned": {"tile_edge": int(b.opts.tile_edge), "stride_h": float(b.opts.stride_h)},
            "tune_seconds": round(tune_s, 2),
            "tune_ms": {f"{e}x{sh:g}h": round(v, 3) for (e, sh), v in (tune_ms or {}).items()},
            "timing": "min over steps of HIP events on the stream; serial = 64 plain fmm_solve calls "
                      "(8^3 tiles, stride 2h) back to back"}


def adjoint_vs_forward(fmm, inputs, dev, steps):
    """The 256^3 tomography problem: 16 shots on the z = 0 face over one FP64
    speed model 1 + 0.3 g, 1024 receivers on z = 1, squared misfit against a
    perturbed model.  Forward = the 16-shot batched solve; adjoint = dL/dF of
    all 16 shots summed into one gradient."""
    tp = inputs.tomography(n=256, n_shots=16, n_receivers=1024, seed=0, device=dev)
    S, n, h, rec = len(tp["shots"]), tp["n"], tp["h"], tp["receivers"]
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        return best

    def batch(F):
        T = torch.empty((S, n, n, n), dtype=torch.float64, device=dev)
        st = torch.empty((S, n, n, n), dtype=torch.uint8, device=dev)
        b = fmm.BatchSolver([{"F": F, "h": h, "seed_idx": i, "seed_val": v} for i, v in tp["shots"]],
                            T_out=[T[k] for k in range(S)], status_out=[st[k] for k in range(S)])
        return b, T, st

    bo, To, _ = batch(tp["F_obs"])
    bo.solve()
    bo.stats()
    dobs = To.reshape(S, -1)[:, rec].clone()
    del bo, To
    b, T, st = batch(tp["F"])
    ms_fwd = timed(b.solve, steps)
    b.stats()
    gT = torch.zeros((S, n ** 3), dtype=torch.float64, device=dev)
    gT[:, rec] = 2.0 * (T.reshape(S, -1)[:, rec] - dobs)
    gT = gT.reshape(S, n, n, n)
    gF = torch.empty((n, n, n), dtype=torch.float64, device=dev)
    a = fmm.AdjointSolver([{"F": tp["F"], "h": h, "T": T[k], "status": st[k], "dL_dT": gT[k], "dL_dF": gF}
                           for k in range(S)])
    ms_adj = timed(a.run, steps)
    ast = a.stats()
    loss = float(((T.reshape(S, -1)[:, rec] - dobs) ** 2).sum().item())
    return {"config": "256^3 FP64 speed max(1 + 0.3 g, 0.1), 16 shots on the z=0 face (one batch), 1024 receivers "
                      "on z=1, squared misfit against a perturbed model",
            "forward_ms": round(ms_fwd, 3), "adjoint_ms": round(ms_adj, 3),
            "adjoint_over_forward": round(ms_adj / ms_fwd, 4),
            "equations": int(ast.n_points), "levels": int(ast.n_levels), "loss": loss,
            "timing": "min over steps of HIP events; forward = fmm_solve_batch of the 16 shots (8^3 tiles, "
                      "stride 2h), adjoint = fmm_adjoint_batch of the 16 shots into one dL/dF"}


def stride_table(fmm, w, spec, T, status, inner_h=None, reps=2):
    """Driver time of the same solve for each (tile edge, restart stride) of
    ``spec`` ("edge:s1,s2,...;edge:..." with strides in units of h, 'inf'
    allowed): ``reps`` solves each, the minimum, with the solve statistics
    (local solves and reopened values per accepted point).  ``inner_h``: the
    in-tile level step in units of h (None: the library default)."""
    out = {}
    for part in spec.split(";"):
        e_s, strides = part.split(":")
        e = int(e_s)
        sv = fmm.Solver(w.shape, w.seed_idx.numel(), w.h, band_width=w.width, tile_edge=e, timing=True,
                        time_limit_s=60, device=w.F.device, speed_dtype=w.F.dtype,
                        inner_stride=None if inner_h is None else inner_h * w.h)
        for sh in (float(x) for x in strides.split(",")):
            sv.opts.stride = sh * w.h
            best, st = None, None
            key = f"E{e} {sh:g}h" + ("" if inner_h is None else f" inner {inner_h:g}h")
            try:
                for _ in range(reps):
                    sv.solve_into(w.F, w.seed_idx, w.seed_val, T, status)
                    st = sv.stats()
                    best = st.ms_driver if best is None else min(best, st.ms_driver)
            except fmm.FmmError as ex:  # e.g. the 60 s time limit
                out[key] = {"error": str(ex)}
                log(f"  table {key}: {ex}")
                continue
            acc = max(1, st.n_accepted)
            out[key] = {"driver_ms": round(best, 2), "restarts": int(st.n_restarts),
                        "tile_marches": int(st.n_tile_marches),
                        "solves_per_point": round(st.n_solves / acc, 2),
                        "reopened_per_point": round(st.n_reopened / acc, 2)}
            log(f"  table {key}: driver {best:.2f} ms, restarts {st.n_restarts}, "
                f"marches {st.n_tile_marches}, solves/pt {st.n_solves / acc:.2f}, "
                f"reopened/pt {st.n_reopened / acc:.2f}")
        del sv
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--stride-h", type=float, default=None,
                    help="restart stride in units of h (inf allowed); default: swept by the library's autotuner")
    ap.add_argument("--sweep", default="3,3.5,4,4.5", help="strides (units of h) the autotuner tries")
    ap.add_argument("--tile", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-crop", type=int, default=352)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-serial measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-vs-forward measurement")
    ap.add_argument("--table", default=PAPER_STRIDE_TABLE,
                    help="tile-edge x stride table on the same workload, e.g. '8:0.5,2,4,inf;4:2,4' (edge: "
                         "strides in units of h); two solves each, minimum; default: the paper's strides "
                         "(Sec. 5.1) with 8^3 tiles; 'none' to skip")
    ap.add_argument("--inner-table", default=None,
                    help="in-tile level steps (units of h, comma separated, 'inf' allowed) to time at the "
                         "chosen stride with the chosen tile edge, e.g. '0.25,0.5,1,inf'")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 64^3 point-source and 256^3 sphere timings (GPU and oracle)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="GiB for a plain device copy, timed as achievable-HBM context and used to "
                         "calibrate HBM byte counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    from paper_1502_07303_amd import fmm, inputs

    dev = torch.device("cuda:0")
    copy_probe = None
    if args.copy_probe > 0:
        nbytes = int(args.copy_probe * 2 ** 30) // 8 * 8
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms_copy = e0.elapsed_time(e1)
        copy_probe = {"bytes_read": nbytes, "bytes_written": nbytes, "ms": round(ms_copy, 4),
                      "GBs": round(2 * nbytes / (ms_copy / 1e3) / 1e9, 1)}
        log(f"copy probe: {2 * nbytes / 2**30:.1f} GiB moved in {ms_copy:.3f} ms = {copy_probe['GBs']} GB/s")
        del a, b
        torch.cuda.empty_cache()
    log(f"generating random-speed workload n={args.n} on {torch.cuda.get_device_name(0)}")
    t0 = time.perf_counter()
    w = inputs.random_speed(n=args.n, seed=args.seed, device=dev)
    torch.cuda.synchronize()
    log(f"  generated in {time.perf_counter() - t0:.1f}s; sources {w.meta['sources']}")
    f_print = inputs.fingerprint(w.F)
    log(f"  F {f_print}")
    N = w.F.numel()
    sweep = None
    stride_h = args.stride_h
    if stride_h is None:
        # the restart stride is swept (Alg. 16's delta-s) by the library's autotuner
        cand = [float(x) for x in args.sweep.split(",")]
        t0 = time.perf_counter()
        tb = fmm.BatchSolver([{"F": w.F, "h": w.h, "seed_idx": w.seed_idx, "seed_val": w.seed_val}],
                             tile_edge=args.tile, with_status=False)
        ms = tb.tune(edges=(args.tile,), strides_h=cand, reps=2)
        stride_h = float(tb.opts.stride_h)
        sweep = {f"{sh:g}h": round(v, 3) for (_, sh), v in ms.items()}
        del tb
        torch.cuda.empty_cache()
        log(f"  stride sweep {sweep} -> {stride_h:g}h ({time.perf_counter() - t0:.1f}s)")
    stride = stride_h * w.h
    solver = fmm.Solver(w.shape, w.seed_idx.numel(), w.h, band_width=w.width, stride=stride,
                        tile_edge=args.tile, timing=True, device=dev, speed_dtype=w.F.dtype)
    T = torch.empty(w.shape, dtype=torch.float64, device=dev)
    status = torch.empty(w.shape, dtype=torch.uint8, device=dev)

    for i in range(args.warmup):
        solver.solve_into(w.F, w.seed_idx, w.seed_val, T, status)
        st = solver.stats()
        log(f"  warmup {i}: {st.ms_prepare + st.ms_driver + st.ms_finalize:.2f} ms, restarts {st.n_restarts}")

    stream = torch.cuda.current_stream()
    times, drv, stats = [], [], None
    torch.cuda.synchronize()
    for i in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.solve_into(w.F, w.seed_idx, w.seed_val, T, status)
        e1.record(stream)
        stats = solver.stats()
        times.append(e0.elapsed_time(e1))
        drv.append(stats.ms_driver)
        log(f"  step {i}: {times[-1]:.2f} ms (driver {stats.ms_driver:.2f} ms, prepare {stats.ms_prepare:.2f}, "
            f"finalize {stats.ms_finalize:.2f}), restarts {stats.n_restarts}, marches {stats.n_tile_marches}")
    torch.cuda.synchronize()

    ms = float(np.mean(times))
    n_acc = int(stats.n_accepted)
    value = n_acc / (ms / 1e3)
    ms_drv = float(np.mean(drv))
    # the solve's algorithmic bytes (read F, write T and status once per
    # accepted point), over the dominant kernel's duration and over the solve
    bytes_per_pt = SOLVE_BYTES_PER_POINT[w.F.dtype]
    alg_bytes = bytes_per_pt * n_acc
    achieved = alg_bytes / (ms_drv / 1e3) / 1e9
    drv_bytes = DRIVER_BYTES_PER_POINT[w.F.dtype] * n_acc
    tag = kernel_tag()
    traffic = read_traffic(tag, stride_h)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "k_driver (restart loop: tile marches + exchange)",
                "algorithmic_bytes_per_launch": alg_bytes, "bytes_per_accepted_point": bytes_per_pt,
                "ms_per_launch": round(ms_drv, 4), "kernel_tag": tag,
                "whole_solve": {"achieved": round(alg_bytes / (ms / 1e3) / 1e9, 2), "ms": round(ms, 4),
                                "frac": round(alg_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 5)},
                "driver_own_bytes": {"bytes_per_accepted_point": DRIVER_BYTES_PER_POINT[w.F.dtype],
                                     "achieved": round(drv_bytes / (ms_drv / 1e3) / 1e9, 2),
                                     "frac": round(drv_bytes / (ms_drv / 1e3) / 1e9 / HBM_PEAK_GBS, 5)}}
    if traffic is not None:
        roofline["traffic_GBs"] = round(traffic / (ms_drv / 1e3) / 1e9, 2)
        roofline["traffic_bytes_per_accepted_point"] = round(traffic / n_acc, 2)

    del solver
    table = None
    if args.table and args.table != "none":
        log("stride table ...")
        table = stride_table(fmm, w, args.table, T, status)
    inner_table = None
    if args.inner_table:
        log("in-tile level-step table ...")
        inner_table = {}
        for ih in (float(x) for x in args.inner_table.split(",")):
            inner_table.update(stride_table(fmm, w, f"{args.tile}:{stride_h:g}", T, status, inner_h=ih))
    del T, status
    torch.cuda.empty_cache()
    batch = None
    if not args.no_batch:
        log("batched vs serial (64 problems) ...")
        batch = batch_vs_serial(fmm, inputs, dev, max(args.steps, 3))
        log(f"  serial {batch['serial_ms']} ms, batched {batch['batched_ms']} ms "
            f"(default {batch['batched_default_ms']}, graph {batch['graph_replay_ms']}), "
            f"speedup {batch['speedup']}x, tuned {batch['tuned']}")

    adj = None
    if not args.no_adjoint:
        log("adjoint vs forward (256^3, 16 shots) ...")
        adj = adjoint_vs_forward(fmm, inputs, dev, max(args.steps, 3))
        log(f"  forward {adj['forward_ms']} ms, adjoint {adj['adjoint_ms']} ms "
            f"({adj['adjoint_over_forward']}x), {adj['levels']} levels")

    small = None
    if not args.no_small:
        log("64^3 point source and 256^3 spheres ...")
        small = gpu_small_configs(fmm, inputs, dev, max(args.steps, 5), with_oracle=not args.no_cpu_baseline)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the oracle on a {args.cpu_crop}^3 crop ...")
        cpu = cpu_baseline(w, min(args.cpu_crop, args.n),
                           {k: v.get("oracle") for k, v in small.items()} if small else None)
        log(f"  oracle {cpu['value']:.3e} points/s in {cpu['seconds']} s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"random_speed_{args.n}: full-domain march, {args.n}^3 grid on [0,1]^3, "
                               "FP32 speed clip(exp(0.5 g), 0.25, 4), Gaussian g with correlation length 0.05, "
                               "4 point sources",
                   "n": args.n, "h": w.h, "speed_dtype": "f32", "sources": len(w.meta["sources"]),
                   "band_width": "inf", "stride_h": stride_h, "stride_sweep_ms": sweep, "tile_edge": args.tile,
                   "seed": args.seed, "F_fingerprint": f_print,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_copy_probe": copy_probe,
        "batch_vs_serial": batch,
        "stride_table": table,
        "inner_step_table": inner_table,
        "small_configs": small,
        "adjoint_vs_forward": adj,
        "solve": {"accepted": n_acc, "points": N, "restarts": int(stats.n_restarts),
                  "tile_marches": int(stats.n_tile_marches), "solves": int(stats.n_solves),
                  "rounds": int(stats.n_rounds), "reopened": int(stats.n_reopened),
                  "workgroups": int(stats.n_workgroups), "max_abs_T": stats.max_abs_T,
                  "ms_prepare": round(stats.ms_prepare, 4), "ms_finalize": round(stats.ms_finalize, 4),
                  "ms_solve": {"mean": round(ms, 4), "median": round(float(np.median(times)), 4),
                               "min": round(float(np.min(times)), 4), "max": round(float(np.max(times)), 4)},
                  "ms_driver": {"mean": round(ms_drv, 4), "median": round(float(np.median(drv)), 4),
                                "min": round(float(np.min(drv)), 4), "max": round(float(np.max(drv)), 4)}},
        "context": "paper: CPU cluster only (Cray XE6, Fortran+MPI); its sequential-time fit implies "
                   "~1.3e5-1.6e5 accepted points/s on one 2014 Opteron core at 1024^3 (not a target)",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
