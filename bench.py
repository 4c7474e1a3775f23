#!/usr/bin/env python3
"""Benchmark: contour-particle Sobolev updates per second on one MI355X.

A step is one Region Competition iteration with Sobolev gradients -- the whole
hot path: L2 gradient, cell-list Sobolev update, acceptance, statistics and
particle-set update -- on the 3D 256^3 uint16 workload (25 ellipsoids, PC
model, E = 6).  W warm-up iterations run first; the context is then
re-initialised from the seeded labels (outside the timed region) and exactly K
iterations are timed, so the timed region is the workload's first K
iterations.  value = sum over timed iterations of the particle count N_t,
divided by the wall time.

The timed region replays the iterations as captured HIP graphs.  Per-kernel
durations come from a second pass over the same K iterations (same seeded
start, same particle counts, checked) in which the library brackets every
kernel with HIP events on its launch stream; the dominant kernel's algorithmic
bytes per launch (per particle, times N_t) over its average duration give the
roofline figure.  Its measured HBM bytes per launch come from the committed
counter summary while the kernel sources are unchanged since it was taken.
The CPU baseline times the FP64 oracle on a bounded sample of the same
workload on the host's cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Algorithmic bytes per particle that each kernel itself moves (each input
# read once, each output written once; neighbour data reused on chip is not
# counted).
#   k_l2diff : record 8 + intensity 2 (u16) + face-label stencil 3.4 + gradient write 4
#              + the same value written to its pixel for the brick kernel 4
#   k_sobolev: L2 gradient read by pixel 4 + Sobolev gradient write 4 (plus the
#              tile rows' particle bits, 256 B per non-empty tile: about 2 B
#              per particle on the 3D workload, not counted here)
#   k_flip   : record 8 + gradient read 4
#   k_write  : record write 8 (the particle set of the next iteration)
KERNEL_OWN_BYTES = {"k_l2diff": 21.4, "k_sobolev": 8.0, "k_flip": 12.0, "k_write": 8.0}



def grad_eval_bytes(w):
    """Algorithmic bytes per particle-update of one gradient evaluation:
    record 8 + intensity (2 for uint16, 4 for fp32) + face-label stencil 3.4 +
    cell-sorted record write 8 + Sobolev gradient write 4, plus about 41 for
    the piecewise-smooth local-mean ball (6.9 unique pixels per particle x
    intensity and label)."""
    b = 8 + (2 if w.image.dtype == np.uint16 else 4) + 3.4 + 8 + 4
    return b + (41.0 if w.model != 0 else 0.0)

PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1403_0240_amd", "csrc", f)
                  for f in ("sobrc_kernels.hip", "sobrc_dev.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary.

    The summary holds FETCH_SIZE and WRITE_SIZE per dispatch (two separate
    counter runs), each already scaled by what the counter reads for a plain
    device copy of known size, and the hash of the kernel sources at the time.
    Returns None when there is no summary or the kernels have changed since.
    """
    path = os.path.join(PROFILES, f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        blob = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(blob)
    except (IndexError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def copy_probe():
    """A plain device-to-device copy of 256 MiB, three times: the calibration
    run for the HBM byte counters (known traffic: 256 MiB read, 256 MiB
    written per copy)."""
    import torch
    n = 64 << 20
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 4 * n, "copies": 3}), flush=True)


def copy_bandwidth():
    """Measured HBM bandwidth of a plain 1 GiB device copy (read + write
    bytes over the median of five copies timed with events on the current
    stream): the practical ceiling beside the 8 TB/s peak."""
    import torch
    n = 256 << 20
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    t = float(np.median(times))
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2 * 4 * n, "seconds": t, "gbs": 2 * 4 * n / t / 1e9}


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def batch_bench(a):
    """The batched workload: every image advanced together by one set of
    launches per iteration, against the same images run one after another
    through the stand-alone path.  Both start from the seeded labels and run
    the same iterations; the label fields must come out identical."""
    import torch
    from paper_1403_0240_amd import sobrc as S
    from paper_1403_0240_amd import workloads as W

    ws = W.batch2d()
    iters = a.steps
    caps = []
    for w in ws:
        # capacity: three times the initial contour (at least 4096 particles)
        p0 = S.from_workload(w)
        S.init_labels(*p0)
        caps.append(max(4096, 3 * S.particle_count(p0[0])))
        del p0

    def contexts(tile):
        out = []
        for w, cap in zip(ws, caps):
            ctx, img, lab = S.from_workload(w, max_particles=cap, tile=tile)
            S.init_labels(ctx, img, lab)
            out.append((ctx, img, lab))
        return out

    tune = None
    if a.tile is None:
        # cell shape for the whole batch (one shape per batch): each shape's
        # batch timed over a few iterations from the seeded start
        ms = {}
        for tile in (S.TILE_DEFAULT, S.TILE_WIDE, S.TILE_TALL):
            cs = contexts(tile)
            Bt = S.Batch(len(cs))
            for k, c in enumerate(cs):
                Bt.set(k, c[0])
            Bt.autotune(S.MODE_SOBOLEV, iters_per_trial=1)
            for rep in range(2):  # the first pass warms up (graphs, first launches)
                for k, c in enumerate(cs):
                    Bt.set(k, None)
                    S.init_labels(*c)
                    Bt.set(k, c[0])
                if rep == 0:
                    Bt.run(TUNE_ITERS, 0.0, S.MODE_SOBOLEV)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Bt.run(TUNE_ITERS, 0.0, S.MODE_SOBOLEV)
            torch.cuda.synchronize()
            ms[tile] = (time.perf_counter() - t0) * 1e3 / TUNE_ITERS
            Bt.close()
            del cs
        # as the library's autotuner: the fastest other shape if it beats the
        # default by 1.5 %, else the default
        alt = min((S.TILE_WIDE, S.TILE_TALL), key=ms.get)
        tile = alt if ms[alt] < 0.985 * ms[S.TILE_DEFAULT] else S.TILE_DEFAULT
        tune = {"chosen": tile_name(2, tile), "iters": TUNE_ITERS,
                "ms_per_iter": {tile_name(2, k): v for k, v in ms.items()}}
    else:
        tile = a.tile
    for w in ws:
        w.tile = tile
    ctxs = contexts(tile)
    n0 = sum(S.particle_count(c[0]) for c in ctxs)
    # stand-alone: each image's run (graph replays), one after another
    for c in ctxs[:2]:
        S.run(c[0], a.warmup, 0.0, S.MODE_SOBOLEV)
    solo_ms, solo_upd, solo_labels = 0.0, 0, []
    for ctx, img, lab in ctxs:
        S.init_labels(ctx, img, lab)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.run(ctx, iters, 0.0, S.MODE_SOBOLEV)
        torch.cuda.synchronize()
        solo_ms += (time.perf_counter() - t0) * 1e3
        hn, _ = S.get_history(ctx, cap=iters)
        solo_upd += int(hn.astype(np.int64).sum())
        solo_labels.append(S.get_labels(ctx).cpu())
    # batched: one batch of all images
    B = S.Batch(len(ctxs))
    for k, (ctx, img, lab) in enumerate(ctxs):
        S.init_labels(ctx, img, lab)
        B.set(k, ctx)
    shape, _ = B.autotune(S.MODE_SOBOLEV, iters_per_trial=2)  # warm-up: launch shape
    B.run(a.warmup, 0.0, S.MODE_SOBOLEV)
    for k, (ctx, img, lab) in enumerate(ctxs):
        B.set(k, None)
        S.init_labels(ctx, img, lab)
        B.set(k, ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = B.run(iters, 0.0, S.MODE_SOBOLEV)
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) * 1e3
    assert (done == iters).all()
    upd = 0
    same = True
    for k, (ctx, _, _) in enumerate(ctxs):
        hn, _ = S.get_history(ctx, cap=iters)
        upd += int(hn.astype(np.int64).sum())
        same = same and torch.equal(S.get_labels(ctx).cpu(), solo_labels[k])
    B.close()
    n = len(ws)
    rec = {
        "metric": "batched images/s (one set of launches per iteration for all images)",
        "value": n / (batch_ms * 1e-3),
        "unit": "images/s",
        "n_gpus": 1, "steps": iters, "warmup": a.warmup,
        "ms_per_step": batch_ms / iters,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch2d_64", "images": n,
                   "sides": [int(min(min(w.image.shape) for w in ws)),
                             int(max(max(w.image.shape) for w in ws))],
                   "E": ws[0].E, "lambda": ws[0].lam, "particles_init": n0,
                   "tile": tile_name(2, ws[0].tile)},
        "updates_per_s": upd / (batch_ms * 1e-3),
        "standalone": {"images_per_s": n / (solo_ms * 1e-3), "ms_total": solo_ms,
                       "updates_per_s": solo_upd / (solo_ms * 1e-3)},
        "speedup_vs_standalone": solo_ms / batch_ms,
        "launch_shape": {"part_chunk": shape[0], "lg_range": shape[1], "sob_tiles": shape[2]},
        "tile_autotune": tune,
        "labels_identical_to_standalone": bool(same and upd == solo_upd),
    }
    print(json.dumps(rec), flush=True)


def serve_bench(a):
    """The serving workload: a seeded Poisson stream of 2D and 3D requests
    (mean 50 requests/s) through the continuous-batching server, each run to
    convergence; p50/p99 arrival-to-result latency and images/s."""
    import torch
    from paper_1403_0240_amd import serve as SV
    from paper_1403_0240_amd import workloads as W

    reqs = W.serve_stream(a.requests, rate=50.0)
    # warm-up: the whole request list once, all at once (library load, graph
    # captures, the allocator's and the page-locked staging pools' first
    # allocations): the timed runs see a server that has been running
    srv = SV.Server(hbm_budget=a.hbm_gb << 30, slots=64, tol=1e-3, max_iters=500, tick=4)
    srv.serve(reqs, realtime=False)
    srv.close()
    torch.cuda.synchronize()
    srv = SV.Server(hbm_budget=a.hbm_gb << 30, slots=64, tol=1e-3, max_iters=500, tick=4)
    done = srv.serve(reqs, realtime=True)
    srv.close()
    st = SV.latency_stats(done)
    # capacity: the same requests all arriving at once
    srv = SV.Server(hbm_budget=a.hbm_gb << 30, slots=64, tol=1e-3, max_iters=500, tick=4)
    sat = SV.latency_stats(srv.serve(reqs, realtime=False))
    srv.close()
    it = np.array([r.iterations for r in done])
    conv = sum(r.iterations < 500 for r in done)
    rec = {
        "metric": "served images/s + p99 (continuous batching, Poisson arrivals)",
        "value": st["images_per_s"], "unit": "images/s", "n_gpus": 1,
        "steps": len(done), "warmup": len(reqs), "ms_per_step": 1e3 * st["span_s"] / max(len(done), 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serve_mix", "requests": len(done), "rate_per_s": 50.0,
                   "mix": "80% 2D fp32 256^2-2048^2, 20% 3D uint16 64^3-192^3",
                   "tol": 1e-3, "max_iters": 500, "hbm_budget_gb": a.hbm_gb, "slots": 64},
        "latency": {"p50_s": st["p50_s"], "p99_s": st["p99_s"], "mean_s": st["mean_s"]},
        "saturated": {"images_per_s": sat["images_per_s"], "p50_s": sat["p50_s"],
                      "p99_s": sat["p99_s"], "span_s": sat["span_s"]},
        "iterations": {"p50": float(np.percentile(it, 50)), "max": int(it.max()),
                       "converged": conv},
    }
    print(json.dumps(rec), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=150)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ellipsoids3d_256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-events", action="store_true",
                    help="time without per-kernel events (roofline omitted)")
    ap.add_argument("--requests", type=int, default=120, help="serving workload: request count")
    ap.add_argument("--hbm-gb", type=int, default=16, help="serving workload: HBM budget (GiB)")
    ap.add_argument("--topo", action="store_true",
                    help="ranked acceptance with topological control (simple points)")
    ap.add_argument("--tile", type=int, default=None,
                    help="cell shape: 0 default (8^3 / 16^2), 1 wide (16x8x8 / 16x32), 2 tall (2D: 16x64); "
                         "default: the faster on this workload (autotuner, before the timed region)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the 256 MiB copy used to calibrate byte counters")
    return ap.parse_args()


def _oracle_rate(w, threads, budget_s, max_iters):
    from oracle import oracle as O
    P = O.params_of(w, threads=threads)
    L = w.labels.copy()
    I = w.image.astype(np.float64)
    done, upd = 0, 0
    t0 = time.perf_counter()
    while done < min(max_iters, w.iterations) and (done == 0 or time.perf_counter() - t0 < budget_s):
        L, info = O.step(P, I, L, O.MODE_SOBOLEV, want_arrays=False)
        upd += info["n"]
        done += 1
    return upd, done, time.perf_counter() - t0


TUNE_ITERS = 20  # fewest iterations per cell shape in the autotuner's trials


def tile_name(ndim, tile):
    """Cell shape of a context as voxels (x by y (by z))."""
    if ndim == 3:
        return "16x8x8" if tile else "8x8x8"
    return f"16x{16 << tile}"


def cpu_baseline(w, budget_s):
    """The FP64 oracle on the host: iterations from the seeded start on all
    host cores (at most 16 threads) until the budget is spent, and the first
    iteration on one thread."""
    threads = min(os.cpu_count() or 1, 16)
    upd, done, dt = _oracle_rate(w, threads, budget_s, 1 << 30)
    upd1, done1, dt1 = _oracle_rate(w, 1, 0.0, 1)
    return {"value": upd / dt, "unit": "particle-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done} iterations of {w.name} from the seeded start "
                      f"({upd} particle updates in {dt:.1f} s, FP64, OpenMP over particles, "
                      f"{threads} threads)",
            "one_thread": {"value": upd1 / dt1, "unit": "particle-updates/s", "cores": 1,
                           "sample": f"first {done1} iteration(s) of {w.name} ({upd1} particle "
                                     f"updates in {dt1:.1f} s)"},
            "host": host_info()}


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
        return
    if a.workload == "serve_mix":
        if a.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        serve_bench(a)
        return
    if a.workload == "batch2d_64":
        if a.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        batch_bench(a)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              f"(images are independent jobs: run one process per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1403_0240_amd import sobrc as S
    from paper_1403_0240_amd import workloads as W

    w = W.make(a.workload)
    if a.topo:
        w.topo = S.TOPO_SIMPLE
    tune = None
    if a.tile is not None:
        w.tile = a.tile
    else:
        # cell shape: each admitted shape timed over the iterations this run
        # takes from the workload's seeded start, warm-up and timed (at least
        # TUNE_ITERS), by the library's autotuner.  The first iterations flip
        # the most pixels, so shorter trials can favour a shape that is slower
        # over the whole run.
        tune_iters = min(1000, max(TUNE_ITERS, a.warmup + a.steps))
        img0, lab0 = S.workload_tensors(w)
        tile, ms = S.tile_autotune(S.workload_params(w), img0, lab0, iters=tune_iters)
        del img0, lab0
        w.tile = tile
        tune = {"chosen": tile_name(w.ndim, tile), "iters": tune_iters,
                "ms_per_iter": {tile_name(w.ndim, k): ms[k] for k in range(3) if ms[k] >= 0}}
    ctx, img, lab = S.from_workload(w)
    S.init_labels(ctx, img, lab)
    n0 = S.particle_count(ctx)
    if a.warmup:
        S.run(ctx, a.warmup, 0.0, S.MODE_SOBOLEV)
    # timed region: the workload's first K iterations from the seeded labels,
    # replayed as captured HIP graphs with no per-kernel events
    S.init_labels(ctx, img, lab)
    S.profile_enable(ctx, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = S.run(ctx, a.steps, 0.0, S.MODE_SOBOLEV)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hn, hf = S.get_history(ctx, cap=max(a.steps, 1))
    assert done == a.steps == len(hn)
    updates = int(hn.astype(np.int64).sum())
    # per-kernel durations: the same K iterations again, each kernel bracketed
    # by HIP events recorded on its launch stream
    prof = None
    if not a.no_events:
        S.init_labels(ctx, img, lab)
        S.profile_enable(ctx, True)
        S.profile_read(ctx, reset=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        done2 = S.run(ctx, a.steps, 0.0, S.MODE_SOBOLEV)
        torch.cuda.synchronize()
        dt_ev = time.perf_counter() - t1
        prof = S.profile_read(ctx, reset=True)
        S.profile_enable(ctx, False)
        hn2, _ = S.get_history(ctx, cap=max(a.steps, 1))
        assert done2 == a.steps and int(hn2.astype(np.int64).sum()) == updates

    rec = {
        "metric": "contour-particle Sobolev updates/s (frac. HBM roofline)",
        "value": updates / dt,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "tile_autotune": tune,
        "config": {"workload": w.name, "shape": list(w.image.shape),
                   "image_dtype": str(w.image.dtype), "image_model": "piecewise-constant"
                   if w.model == W.PC else "piecewise-smooth", "E": w.E, "lambda": w.lam,
                   "acceptance": "ranked, topology-controlled" if a.topo else "simultaneous",
                   "psf_sigma": w.psf_sigma, "tile": tile_name(w.ndim, w.tile),
                   "particles_init": n0, "particles_mean": updates / a.steps,
                   "flips_last": int(hf[-1]) if len(hf) else 0},
    }
    if prof:
        kt = {k: {"ms_total": v[0], "launches": v[1],
                  "us_avg": 1e3 * v[0] / v[1] if v[1] else 0.0} for k, v in prof.items()}
        rec["kernels"] = kt
        rec["ms_per_step_with_events"] = dt_ev * 1e3 / a.steps
        dom = max(kt, key=lambda k: kt[k]["ms_total"])
        gb = grad_eval_bytes(w)
        copy = copy_bandwidth()
        rec["hbm_copy"] = copy
        own = KERNEL_OWN_BYTES.get(dom)
        if own is not None and kt[dom]["ms_total"] > 0:
            # priced at the algorithmic bytes of one particle-update of the
            # gradient evaluation (record, intensity, face labels, sorted
            # record write, Sobolev gradient write); the kernel's own bytes
            # beside it
            launches = kt[dom]["launches"]
            alg_per_launch = gb * updates / launches
            sec = kt[dom]["us_avg"] * 1e-6
            achieved = alg_per_launch / sec / 1e9
            own_gbs = own * updates / launches / sec / 1e9
            rec["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": achieved,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": achieved / HBM_PEAK_GBS,
                               "traffic": measured_traffic(w.name, dom),
                               "alg_bytes_per_launch": alg_per_launch,
                               "bytes_per_particle": gb,
                               "alg_bytes_source": "gradient evaluation per particle-update: record 8 + "
                                                   "intensity + face labels 3.4 + sorted record write 8 "
                                                   "+ Sobolev gradient write 4",
                               "frac_of_copy": achieved / copy["gbs"],
                               "kernel_own_bytes_per_particle": own,
                               "kernel_own_achieved": own_gbs,
                               "kernel_own_frac": own_gbs / HBM_PEAK_GBS,
                               "us_per_launch": kt[dom]["us_avg"]}
        else:
            rec["roofline"] = {"kernel": dom, "bound": "alu", "achieved": None, "peak": None,
                               "unit": None, "frac": None, "traffic": None}
        g_ms = kt["k_l2diff"]["ms_total"] + kt["k_sobolev"]["ms_total"]
        g_rate = updates / (g_ms * 1e-3)
        rec["gradient_eval"] = {"us_per_iter": 1e3 * g_ms / a.steps,
                                "updates_per_s": g_rate, "bytes_per_update": gb,
                                "hbm_frac": gb * g_rate / 1e9 / HBM_PEAK_GBS,
                                "frac_of_copy": gb * g_rate / 1e9 / copy["gbs"]}
    if not a.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
