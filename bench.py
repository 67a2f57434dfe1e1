#!/usr/bin/env python3
"""Throughput of the map/reduce BLAS hot path on one MI355X.

A step is one pass of scal, asum and dot (binary32, per-call kernels) over
vectors of n = 2^24 elements (64 MiB each), alpha = 2.5, x and y uniform in
[-1, 1) from seed 1 -- the paper's "small" 16M-element vector size.  `value`
is the step's algorithmic HBM bytes (scal reads and writes n floats, asum
reads n, dot reads 2n: 20n bytes) divided by the measured time per step, in
GB/s (1e9 B/s).  Inputs are resident in HBM before timing starts; steps
rotate over enough copies of the buffers (> 1 GiB in total) that no step
finds its operands in the 256 MB Infinity Cache.

Also reported on the same JSON line:
  roofline     : the dominant kernel's algorithmic bytes per launch over its
                 average duration, from HIP events recorded with its dispatch
                 (lift_time_next_launch) in every 20th step of the timed
                 region (the kernel before it in those steps carries a pair
                 too, so the timed kernel's start is stamped after that
                 kernel has finished); peak 8 TB/s; HBM traffic per launch
                 from rocprofv3 counters when they were taken on the current
                 kernel source (else null)
  cpu_baseline : the binary64 oracle on the same workload and data, in its
                 split-join form on the host cores (value) and sequentially on
                 one thread; each timed for a bounded number of seconds
  kernels      : per-kernel average durations from back-to-back launches, and
                 median / p10 / p90 of 200 single launches timed inside their
                 dispatch, cold (rotating buffer sets) and warm (one set)
  forms        : asum fp32 at n = 2^20 (50 launches replayed from one HIP
                 graph), gemv fp32 (4096^2, 8192^2, 16384^2), 16-bit storage
                 (n = 2^26 asum/dot, bf16 gemv 16384^2) in each accumulation
                 variant, the batch of 4096 reductions + 256 gemv (fp32 and
                 bf16, against the same problems per call), BlackScholes over
                 2^22 prices, MD (12288 and 2^20 particles), as GB/s and
                 binary32-equivalent GB/s

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-forms] [--forms LIST]
       [--no-cpu-baseline] [--cpu-seconds S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0
METRIC = "HBM GB/s and % of 8 TB/s peak: asum/dot/gemv FP32 vs BF16 and batched forms"
COLD_BYTES = 1 << 30          # rotate buffer sets until at least this much is touched
ROOFLINE_LAUNCHES = 50        # the roofline kernel is timed on at least this many launches
FORMS = ("large", "small", "gemv", "gemvrect", "half", "batch", "blackscholes", "md", "gemv16")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash(kernel: str) -> str:
    """Hash of the sources a kernel is built from (device helpers + its unit)."""
    csrc = os.path.join(ROOT, "paper_1502_02389_amd", "csrc")
    files = {"scal": ["lift_device.hpp", "lift_internal.hpp", "lift_scal.hip"],
             "asum": ["lift_device.hpp", "lift_internal.hpp", "lift_reduce.hpp", "lift_reduce_f32.hip"],
             "dot": ["lift_device.hpp", "lift_internal.hpp", "lift_reduce.hpp", "lift_reduce_f32.hip"],
             "gemv": ["lift_device.hpp", "lift_internal.hpp", "lift_gemv.hpp", "lift_gemv_f32.hip"]}[kernel]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current source of that kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--forms", default=",".join(FORMS),
                    help="forms to run: " + ", ".join(FORMS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--event-every", type=int, default=20,
                    help="time the dominant kernel in every k-th step of the timed region")
    ap.add_argument("--stamps", default=None, metavar="OPS",
                    help="diagnostic only: per-work-group clock stamps of the step's asum / dot launches, "
                         "per-tile stamps of the batched workload's two launches (e.g. asum,dot,batch); "
                         "prints a JSON summary and exits")
    ap.add_argument("--stamp-n", type=int, default=24, help="log2 n for --stamps")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1502_02389_amd as L
    import workloads as W

    lib = L.library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    props = torch.cuda.get_device_properties(dev)
    log("device", props.name, "CUs", props.multi_processor_count, "lib", L.lift_version())

    if args.stamps:
        ops = args.stamps.split(",")
        out = {}
        if "batch" in ops:
            out["batch"] = batch_stamp_report(L, W, dev)
            ops = [o for o in ops if o != "batch"]
        if ops:
            out.update(stamp_report(L, W, dev, stream, ops, 1 << args.stamp_n))
        print(json.dumps(out), flush=True)
        return

    # ------------------------------------------------------------ main step
    n = W.STREAM_N
    x_cpu, y_cpu, alpha = W.stream_vectors(n)
    x0, y0 = x_cpu.to(dev), y_cpu.to(dev)
    set_bytes = 5 * 4 * n
    nsets = max(2, -(-COLD_BYTES // set_bytes))
    sets = []
    for _ in range(nsets):
        sets.append(dict(xs=x0.clone(), out=torch.empty_like(x0), xa=x0.clone(), xd=x0.clone(), yd=y0.clone(),
                         ra=torch.zeros((), device=dev), rd=torch.zeros((), device=dev)))
    del x0, y0
    ws = L.workspace(dev)
    wsp, wsb = ws.data_ptr(), ws.numel()
    ptr = [{k: v.data_ptr() for k, v in s.items()} for s in sets]
    bytes_kernel = {"scal": 8 * n, "asum": 4 * n, "dot": 8 * n}
    step_bytes = sum(bytes_kernel.values())

    def launch(kernel, p):
        if kernel == "scal":
            st = lib.lift_scal(n, alpha, p["xs"], p["out"], sh)
        elif kernel == "asum":
            st = lib.lift_asum(n, p["xa"], p["ra"], wsp, wsb, sh)
        else:
            st = lib.lift_dot(n, p["xd"], p["yd"], p["rd"], wsp, wsb, sh)
        if st != 0:
            raise L.LiftError(st, f"lift_{kernel}")

    order = ("scal", "asum", "dot")

    def step(i, ev_kernel=None, ev=None, slot=None, ev_prev=None):
        p = ptr[i % nsets]
        for j, k in enumerate(order):
            if slot is not None and (k == ev_kernel or (ev_prev is not None and j + 1 < len(order)
                                                        and order[j + 1] == ev_kernel)):
                # events recorded with the kernel's own dispatch; the kernel
                # before the timed one carries a pair too, so the timed
                # kernel's start is recorded after that kernel has finished
                # (otherwise the start can be stamped while it still drains)
                evs = ev if k == ev_kernel else ev_prev
                st = lib.lift_time_next_launch(evs.events[2 * slot], evs.events[2 * slot + 1])
                if st != 0:
                    raise L.LiftError(st, "lift_time_next_launch")
            launch(k, p)

    log("warmup", args.warmup, "sets", nsets)
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    # per-kernel durations from back-to-back launches (outside the timed region)
    kernels = {}
    reps = 200
    for k in order:
        for i in range(5):
            launch(k, ptr[i % nsets])
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for i in range(reps):
            launch(k, ptr[i % nsets])
        t1.record(stream)
        torch.cuda.synchronize()
        us = t0.elapsed_time(t1) * 1e3 / reps
        gbs = bytes_kernel[k] / (us * 1e-6) / 1e9
        kernels[k] = {"avg_us": round(us, 3), "bytes": bytes_kernel[k], "GB_s": round(gbs, 1),
                      "frac_of_peak": round(gbs / PEAK_GBS, 4)}
        # per-launch durations (events inside each dispatch): cold (rotating
        # sets) and warm (one set, 64-128 MiB that the 256 MB cache can hold)
        for label, pick in (("cold", lambda i: ptr[i % nsets]), ("warm", lambda i: ptr[0])):
            d = _per_launch_us(L, lambda i, pick=pick, k=k: launch(k, pick(i)), 200)
            kernels[k][label] = {"median_us": round(d[len(d) // 2], 3), "p10_us": round(d[len(d) // 10], 3),
                                 "p90_us": round(d[(9 * len(d)) // 10], 3),
                                 "median_GB_s": round(bytes_kernel[k] / (d[len(d) // 2] * 1e-6) / 1e9, 1)}
        log("kernel", k, kernels[k])
    # the roofline kernel: dot -- with scal the largest share of the step
    # (the two move the same bytes and time within noise of each other)
    dominant = "dot"

    # timed region: K steps.  In every `event_every`-th step the dominant
    # kernel is launched with HIP events recorded with its own dispatch (on
    # the stream it runs on), and so is the kernel before it (without that,
    # the timed kernel's start can be stamped while the previous kernel
    # still drains, which reads ~1 us long); timing every step would add
    # ~5 us of idle GPU per step, so a sample is timed.
    sampled = [i for i in range(args.steps) if i % args.event_every == 0]
    # at least ROOFLINE_LAUNCHES timed launches: when the timed region holds
    # fewer sampled steps, the same steps continue right after it (events on
    # every one of them) until there are enough
    extra = max(0, ROOFLINE_LAUNCHES - len(sampled))
    ev = L.HipEvents(2 * (len(sampled) + extra))
    ev_prev = L.HipEvents(2 * (len(sampled) + extra))
    slot_of = {i: j for j, i in enumerate(sampled)}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(i, dominant, ev, slot_of.get(i), ev_prev)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    for j in range(extra):
        step(args.steps + j, dominant, ev, len(sampled) + j, ev_prev)
    torch.cuda.synchronize()
    durs = [ev.elapsed_ms(2 * j, 2 * j + 1) * 1e3 for j in range(len(sampled) + extra)]
    ev.close()
    ev_prev.close()
    dom_us = sum(durs) / len(durs)
    achieved = bytes_kernel[dominant] / (dom_us * 1e-6) / 1e9
    log("timed", args.steps, "steps", f"{ms_per_step:.4f} ms/step", f"{value:.1f} GB/s",
        "dominant", dominant, f"{dom_us:.2f} us over {len(durs)} launches")

    roofline = {"bound": "hbm", "kernel": f"lift {dominant} (fp32, n=2^24)", "achieved": round(achieved, 1),
                "peak": PEAK_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_GBS, 4),
                "traffic": measured_traffic(dominant), "algorithmic_bytes": bytes_kernel[dominant],
                "avg_us": round(dom_us, 3), "median_us": round(statistics.median(durs), 3),
                "p10_us": round(sorted(durs)[len(durs) // 10], 3),
                "p90_us": round(sorted(durs)[(9 * len(durs)) // 10], 3),
                "timed_launches": len(durs), "in_timed_region": len(sampled)}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "scal+asum+dot fp32 per-call kernels, n=2^24 (64 MiB per vector), alpha=2.5, "
                               "x,y ~ U[-1,1) seed 1, cold Infinity Cache (rotating buffer sets)",
                   "n": n, "bytes_per_step": step_bytes, "buffer_sets": nsets,
                   "frac_of_peak": round(value / PEAK_GBS, 4)},
        "roofline": roofline,
        "kernels": kernels,
    }

    gpu_results = (float(sets[0]["ra"].item()), float(sets[0]["rd"].item()))
    del sets, ptr
    torch.cuda.empty_cache()
    # measured ceiling: the library's flat read and copy kernels at the sizes
    # of the step's kernels (and of the 2^27 form), best launch shape of a sweep
    ceil = ceilings(L, dev, stream)
    result["ceiling"] = ceil
    # what each step kernel reaches of the ceiling of its own bytes
    own = {"scal": "copy_2^24", "asum": "read_2^24", "dot": "read_2^25"}
    for k in order:
        c = ceil[own[k]]
        kernels[k]["ceiling"] = own[k]
        kernels[k]["frac_of_ceiling"] = round(c["avg_us"] / kernels[k]["avg_us"], 4)
        kernels[k]["cold"]["frac_of_ceiling"] = round(c["cold_median_us"] / kernels[k]["cold"]["median_us"], 4)
    roofline["ceiling_GB_s"] = ceil["read_2^25"]["GB_s"]
    roofline["frac_of_ceiling"] = round(achieved / ceil["read_2^25"]["GB_s"], 4)

    # ------------------------------------------------------------ CPU oracle
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(x_cpu, y_cpu, alpha, args.cpu_seconds, gpu_results, step_bytes)

    # ------------------------------------------------------------ other forms
    if not args.no_forms:
        precision = {}
        result["forms"] = forms(L, W, dev, stream, tuple(args.forms.split(",")), precision)
        if not args.no_cpu_baseline and precision:
            result["cpu_baseline"]["precision_forms_vs_oracle"] = precision_errors(precision)

    print(json.dumps(result), flush=True)


def stamp_report(L, W, dev, stream, ops, n, launches=40):
    """Where the time of a plain asum / dot launch goes, from per-work-group
    wall-clock stamps (lift_stamp_next_launch) of `launches` launches on
    rotating buffer sets (cold Infinity Cache), each also timed by HIP events
    in its dispatch.  Per launch, relative to the first work-group's entry:
    entry spread (dispatch ramp), first and last end of a streaming loop,
    stream time per work-group, work-group tree, partial store, arrival, and
    the combine tail from the last streaming loop's end to the result; the
    medians over launches are reported."""
    import torch

    lib = L.library()
    sh = stream.cuda_stream
    x_cpu, y_cpu, _ = W.stream_vectors(n)
    per_set = 8 * n
    ns = max(2, -(-COLD_BYTES // per_set))
    xs = [x_cpu.to(dev) for _ in range(ns)]
    ys = [y_cpu.to(dev) for _ in range(ns)]
    ws = L.workspace(dev)
    res = torch.zeros((), device=dev)
    cap = L.lift_max_workgroups()
    buf = torch.zeros((cap, 8), dtype=torch.int64, device=dev)
    out = {"n": n, "launches": launches}
    for op in ops:
        def call(i, op=op):
            if op == "asum":
                st = lib.lift_asum(n, xs[i].data_ptr(), res.data_ptr(), ws.data_ptr(), ws.numel(), sh)
            else:
                st = lib.lift_dot(n, xs[i].data_ptr(), ys[i].data_ptr(), res.data_ptr(), ws.data_ptr(), ws.numel(), sh)
            if st != 0:
                raise L.LiftError(st, f"lift_{op}")
        for i in range(5):
            call(i % ns)
        rows = []
        ev = L.HipEvents(2)
        for i in range(launches):
            buf.zero_()
            torch.cuda.synchronize()
            st, khz = L.lift_stamp_next_launch(buf.data_ptr(), cap)
            assert st == 0 and khz > 0
            assert L.lift_time_next_launch(ev.events[0], ev.events[1]) == 0
            call(i % ns)
            torch.cuda.synchronize()
            ev_us = ev.elapsed_ms(0, 1) * 1e3
            b = buf.cpu().numpy()
            g = int((b[:, 0] != 0).sum())
            b = b[:g].astype("float64")
            us = 1e3 / khz                         # microseconds per tick
            t0 = b[:, 0].min()
            last = int(((b[:, 6].astype("int64") >> 32) & 1).argmax())
            rows.append({
                "event_us": ev_us,
                "span_us": (b[:, 5].max() - t0) * us,
                "entry_spread_us": (b[:, 0].max() - t0) * us,
                "first_stream_end_us": (b[:, 1].min() - t0) * us,
                "last_stream_end_us": (b[:, 1].max() - t0) * us,
                "stream_median_us": float(statistics.median((b[:, 1] - b[:, 0]) * us)),
                "tree_median_us": float(statistics.median((b[:, 2] - b[:, 1]) * us)),
                "store_median_us": float(statistics.median((b[:, 3] - b[:, 2]) * us)),
                "arrive_median_us": float(statistics.median((b[:, 4] - b[:, 3]) * us)),
                "last_tree_done_us": (b[:, 2].max() - t0) * us,
                "last_arrival_us": (b[:, 4].max() - t0) * us,
                "tail_after_last_stream_us": (b[last, 5] - b[:, 1].max()) * us,
                "combine_us": (b[last, 5] - b[last, 4]) * us,
                "grid": g,
                "xccs": len(set(((b[:, 6].astype("int64") >> 16) & 0xF).tolist())),
            })
        ev.close()
        summary = {k: round(statistics.median(r[k] for r in rows), 3) for k in rows[0]}
        summary["knobs"] = L.lift_default_knobs(op, L.LIFT_F32, 0, n)[1]
        out[op] = summary
        log("stamps", op, summary)
    return out


def batch_stamp_report(L, W, dev, runs=4):
    """Where the batched workload's time goes, from per-tile wall-clock
    stamps (lift_stamp_next_launch on lift_batch_run) of `runs` runs per
    storage.  Per launch (reduction tiles, gemv tiles) of the last run: its
    span from the first tile's start, the work-groups, busy time per
    work-group (median), the gaps between a work-group's tiles (mean sum per
    work-group), the spread of the work-groups' last tile ends, and the
    algorithmic GB/s over the span; for the gemv launch, the rate per
    work-group by row class (rows starting on a vector boundary, rows with
    heads against shifted copies of x, element loads) and row length."""
    import torch
    import numpy as np

    spec = W.batch_shapes()
    nred = len(spec.red_kind)
    out = {}
    for storage, eb in (("bf16", 2), ("f32", 4)):
        reds, gemvs = W.batch_values(spec, storage)
        probs = []
        for kind, x, y in reds:
            probs.append(("dot", x.to(dev), y.to(dev)) if kind == "dot" else ("asum", x.to(dev)))
        for A, x, y in gemvs:
            probs.append(("gemv", W.GEMV_ALPHA, A.to(dev), x.to(dev), W.GEMV_BETA, y.to(dev)))
        del reds, gemvs
        b = L.Batch(probs)
        _, kn = L.lift_default_knobs("batch", {"f32": L.LIFT_F32, "bf16": L.LIFT_BF16}[storage], L.LIFT_ACC_F32, 0)
        vb = kn["vec_bytes"] or 16          # the library default when no tuned entry applies
        buf = torch.zeros((b.tiles, 4), dtype=torch.int64, device=dev)
        ev = L.HipEvents(2)
        for _ in range(2):
            b.run()
        torch.cuda.synchronize()
        run_us = []
        for _ in range(runs):
            buf.zero_()
            torch.cuda.synchronize()
            st, khz = L.lift_stamp_next_launch(buf.data_ptr(), b.tiles)
            assert st == 0 and khz > 0
            assert L.lift_time_next_launch(ev.events[0], ev.events[1]) == 0
            b.run()
            torch.cuda.synchronize()
            run_us.append(ev.elapsed_ms(0, 1) * 1e3)
        ev.close()
        t = buf.cpu().numpy().astype(np.int64)
        us = 1e3 / khz
        prob = t[:, 2] >> 32
        length = t[:, 2] & 0xFFFFFFFF
        rep = {"run_us": [round(v, 1) for v in run_us], "knobs": kn}
        ntiles = np.bincount(prob[prob < nred], minlength=nred)
        for name, mask in (("reductions", prob < nred), ("gemv", prob >= nred)):
            a, p, ln = t[mask], prob[mask], length[mask]
            t0 = a[:, 0].min()
            s, e = (a[:, 0] - t0) * us, (a[:, 1] - t0) * us
            wg = a[:, 3] & 0xFFFFFFFF
            if name == "reductions":
                n = np.array([spec.red_len[i] for i in p])
                opnd = np.array([2 if spec.red_kind[i] == "dot" else 1 for i in p])
                tb = n / ntiles[p] * eb * opnd                     # a problem's bytes over its tiles
            else:
                mn = np.array([spec.gemv_mn[i - nred] for i in p])
                n = mn[:, 1]
                tb = ln * n * eb
            groups = np.unique(wg)
            busy, gaps, last = [], [], []
            for g in groups:
                m = wg == g
                o = np.argsort(s[m])
                gs, ge = s[m][o], e[m][o]
                busy.append(float((ge - gs).sum()))
                gaps.append(float((gs[1:] - ge[:-1]).sum()))
                last.append(float(ge.max()))
            span = float(e.max())
            r = {"tiles": int(mask.sum()), "work_groups": int(len(groups)), "span_us": round(span, 1),
                 "GB_s_over_span": round(float(tb.sum()) / span / 1e3, 1),
                 "busy_us_per_wg_median": round(float(np.median(busy)), 1),
                 "gaps_us_per_wg_mean": round(float(np.mean(gaps)), 1),
                 "last_end_us_min_median_max": [round(min(last), 1), round(float(np.median(last)), 1),
                                                round(max(last), 1)],
                 "tile_us_p10_p50_p90": [round(float(np.percentile(e - s, q)), 1) for q in (10, 50, 90)]}
            if name == "gemv":
                aptr = np.array([probs[i][2].data_ptr() for i in p], dtype=np.int64)
                E = vb // eb
                aligned = ((n * eb) % vb == 0) & (aptr % vb == 0)
                heads = ~aligned & (E > 1) & (vb <= 8) & (n >= 64 * E) & (E * ((n + 3) // 4 * 4) <= 16320)
                classes = {}
                dur = e - s
                for cname, cm in (("aligned", aligned), ("heads", heads), ("elements", ~aligned & ~heads)):
                    for lo, hi in ((0, 1024), (1024, 2048), (2048, 4097)):
                        mm = cm & (n >= lo) & (n < hi)
                        if mm.sum():
                            classes[f"{cname} n in [{lo},{hi})"] = {
                                "tiles": int(mm.sum()), "GB": round(float(tb[mm].sum()) / 1e9, 3),
                                "GB_s_per_wg": round(float(tb[mm].sum()) / float(dur[mm].sum()) / 1e3, 2)}
                r["rows"] = classes
            rep[name] = r
        out[storage] = rep
        log("batch stamps", storage, rep)
        b.close()
        del probs
        torch.cuda.empty_cache()
    return out


def precision_errors(precision):
    """Part of the CPU-baseline leg: the binary64 oracle on the stored 16-bit
    inputs of the precision forms, and each GPU result's error against it
    (asum relative; dot over sum |x y|; gemv worst row over
    |alpha| sum |A x| + |beta y|)."""
    import numpy as np

    import oracle

    def bits(t):
        return t.view(torch_int16()).numpy().view(np.uint16) if str(t.dtype) == "torch.bfloat16" else t.numpy()

    out = {}
    for storage, (x, y, got) in precision.get("half", {}).items():
        tag = "bf16" if storage == "bf16" else None
        xs, ys = bits(x), bits(y)
        ra = oracle.asum(xs, dtype=tag)
        rd = oracle.dot(xs, ys, dtype=tag)
        mass = oracle.dot_absmass(xs, ys, dtype=tag)
        for (op, acc), v in got.items():
            err = abs(v - ra) / ra if op == "asum" else abs(v - rd) / mass
            out[f"{op}_{storage}_{acc}_2^26"] = float(f"{err:.3e}")
    if "gemv16" in precision:
        A, x, y, alpha, beta, got = precision["gemv16"]
        a16 = bits(A)
        r = oracle.gemv(alpha, a16, x.numpy(), beta, y.numpy(), adtype="bf16")
        mass = oracle.gemv_absmass(alpha, a16, x.numpy(), beta, y.numpy(), adtype="bf16")
        for acc, g in got.items():
            out[f"gemv_bf16_{acc}_16384"] = float(f"{float(np.max(np.abs(g - r) / mass)):.3e}")
    log("precision forms vs oracle", out)
    return out


def torch_int16():
    import torch

    return torch.int16


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_cpu, y_cpu, alpha, seconds, gpu_set, step_bytes):
    """The binary64 oracle timed on whole steps of the same workload (scal,
    asum, dot over the same host arrays): first the sequential composition on
    one thread, then its split-join form (rule 3d) on every host core this
    process may use, each for `seconds` (at least 5 steps); the median step
    time gives the rate.  Timing includes the exact widening to binary64.
    gpu_set: the GPU's (asum, dot) results on the same data, for the error
    report."""
    import oracle

    xs, ys = x_cpu.numpy(), y_cpu.numpy()
    oracle.asum(xs[:1024])  # load
    threads = oracle.host_threads()

    def timed(step):
        times, t_end, res = [], time.perf_counter() + seconds, None
        while len(times) < 5 or time.perf_counter() < t_end:
            t0 = time.perf_counter()
            res = step()
            times.append(time.perf_counter() - t0)
        return sorted(times), res

    def seq():
        oracle.scal(alpha, xs)
        return oracle.asum(xs), oracle.dot(xs, ys)

    def par():
        oracle.scal_par(alpha, xs, threads)
        return oracle.asum_par(xs, threads), oracle.dot_par(xs, ys, threads)

    t1, (ra, rd) = timed(seq)
    tp, _ = timed(par)
    m1, mp = t1[len(t1) // 2], tp[len(tp) // 2]
    g1, gp = step_bytes / m1 / 1e9, step_bytes / mp / 1e9
    ga, gd = gpu_set
    mass = oracle.dot_absmass(xs, ys)
    log("cpu oracle 1 thread:", len(t1), "steps, median", f"{m1 * 1e3:.1f} ms", f"{g1:.3f} GB/s;",
        threads, "threads:", len(tp), "steps, median", f"{mp * 1e3:.1f} ms", f"{gp:.3f} GB/s")
    return {"value": round(gp, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"median of {len(tp)} full steps (scal+asum+dot, n=2^24, same arrays, binary64 widening "
                      f"included) of the C oracle in its split-join form on {threads} threads, "
                      f"{sum(tp):.1f} s in all",
            "cpu_model": _cpu_model(),
            "single_thread": {"value": round(g1, 4), "unit": "GB/s", "cores": 1,
                              "sample": f"median of {len(t1)} full steps of the sequential composition, "
                                        f"{sum(t1):.1f} s in all"},
            "gpu_vs_oracle": {"asum_rel_err": abs(ga - ra) / ra, "dot_err_over_absmass": abs(gd - rd) / mass}}


def _per_launch_us(L, launch, reps):
    """Sorted durations of `reps` launches, each timed by HIP events recorded
    with its own dispatch (launch(i) must make exactly one library launch)."""
    import torch

    ev = L.HipEvents(2 * reps)
    try:
        for i in range(reps):
            st = L.lift_time_next_launch(ev.events[2 * i], ev.events[2 * i + 1])
            if st != 0:
                raise L.LiftError(st, "lift_time_next_launch")
            launch(i)
        torch.cuda.synchronize()
        return sorted(ev.elapsed_ms(2 * i, 2 * i + 1) * 1e3 for i in range(reps))
    finally:
        ev.close()


def _time_calls(fn, nsets, stream, reps=50, warm=5):
    """Average device time per call of fn(i) over reps back-to-back calls."""
    import torch

    for i in range(warm):
        fn(i % nsets)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(reps):
        fn(i % nsets)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def _time_graph(fn, nsets, stream, reps=50, warm=5):
    """Average device time per call of fn(i, stream_handle) over reps calls
    captured in one HIP graph and replayed: for launch-bound kernels, whose
    back-to-back host launches would leave the device idle between them."""
    import torch

    for i in range(warm):
        fn(i % nsets, stream.cuda_stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for i in range(reps):
                fn(i % nsets, side.cuda_stream)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
    torch.cuda.synchronize()
    del g
    return e0.elapsed_time(e1) * 1e3 / reps


CEILING_SIZES = (("read", 24), ("read", 25), ("read", 27), ("read", 28), ("copy", 24), ("copy", 27))


def ceilings(L, dev, stream, sizes=CEILING_SIZES):
    """Achievable rate of one launch of a flat read / copy of 2^e floats: the
    library's stream kernels over a sweep of launch shapes (work-group size,
    loads in flight, work-groups per CU, chunked or interleaved steps), the
    best back-to-back average on rotating buffers (cold Infinity Cache), and
    the median of 200 single launches of that shape timed in their dispatch."""
    import itertools

    import torch

    lib = L.library()
    sh = stream.cuda_stream
    out = {}
    sink = torch.zeros(4, dtype=torch.float32, device=dev)
    for kind, e in sizes:
        n = 1 << e
        moved = 4 * n * (2 if kind == "copy" else 1)
        ns = max(2, -(-COLD_BYTES // moved))
        xs = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(ns)]
        outs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(ns)] if kind == "copy" else None
        best = None
        for b, u, w, il in itertools.product((256, 512, 1024), (4, 8), (1, 2, 4, 8),
                                             (L.LIFT_INTERLEAVE_CHUNK, L.LIFT_INTERLEAVE_STRIDE)):
            kn = L.knobs(block=b, unroll=u, wg_per_cu=w, interleave=il)

            def call(i, kn=kn):
                if kind == "copy":
                    st = lib.lift_stream_copy(n, xs[i].data_ptr(), outs[i].data_ptr(), ctypes_ref(kn), sh)
                else:
                    st = lib.lift_stream_read(n, xs[i].data_ptr(), sink.data_ptr(), ctypes_ref(kn), sh)
                if st != 0:
                    raise L.LiftError(st, f"lift_stream_{kind}")
            us = _time_calls(call, ns, stream, reps=max(50, ns))
            if best is None or us < best[0]:
                best = (us, dict(block=b, unroll=u, wg_per_cu=w,
                                 interleave="chunk" if il == L.LIFT_INTERLEAVE_CHUNK else "stride"), call)
        us, knobs, call = best
        d = _per_launch_us(L, lambda i, call=call: call(i % ns), 200)
        med = d[len(d) // 2]
        out[f"{kind}_2^{e}"] = {"bytes": moved, "avg_us": round(us, 3), "GB_s": round(moved / (us * 1e-6) / 1e9, 1),
                                "frac_of_peak": round(moved / (us * 1e-6) / 1e9 / PEAK_GBS, 4),
                                "cold_median_us": round(med, 3),
                                "cold_median_GB_s": round(moved / (med * 1e-6) / 1e9, 1), "knobs": knobs}
        log("ceiling", f"{kind}_2^{e}", out[f"{kind}_2^{e}"])
        del xs, outs
        torch.cuda.empty_cache()
    return out


def ctypes_ref(k):
    import ctypes

    return ctypes.byref(k)


def forms(L, W, dev, stream, which=FORMS, precision=None):
    import torch

    lib = L.library()
    sh = stream.cuda_stream
    ws = L.workspace(dev)
    wsp, wsb = ws.data_ptr(), ws.numel()
    out = {}

    def rec(name, us, nbytes, fp32_bytes):
        gbs = nbytes / (us * 1e-6) / 1e9
        out[name] = {"avg_us": round(us, 3), "GB_s": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_GBS, 4),
                     "fp32_equiv_GB_s": round(fp32_bytes / (us * 1e-6) / 1e9, 1)}
        log("form", name, out[name])

    if "gemv" in which:
        # gemv fp32, square 4096 and 8192, and 16384 (A 1 GiB) for the large-size roofline
        for size in W.GEMV_SIZES + (16384,):
            A, x, y, alpha, beta = W.gemv_square(size)
            nb = 4 * size * size + 4 * size + 8 * size
            ns = max(2, -(-COLD_BYTES // nb))
            As = [A.to(dev) for _ in range(ns)]
            xd, yd = x.to(dev), y.to(dev)

            def call(i, As=As, xd=xd, yd=yd, size=size, alpha=alpha, beta=beta):
                st = lib.lift_gemv(size, size, alpha, As[i].data_ptr(), size, xd.data_ptr(), beta, yd.data_ptr(), sh)
                assert st == 0
            rec(f"gemv_f32_{size}", _time_calls(call, ns, stream), nb, nb)
            del As
            torch.cuda.empty_cache()

    if "large" in which:
        # scal, asum and dot fp32 at n = 2^27 (512 MiB per vector: the paper's
        # large vector size), plain entry points, two rotating buffer sets
        n = W.LARGE_N
        x, y, alpha = W.stream_vectors(n)
        ns = 2
        xs = [x.to(dev) for _ in range(ns)]
        ys = [y.to(dev) for _ in range(ns)]
        del x, y
        res = torch.zeros((), dtype=torch.float32, device=dev)
        outs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(ns)]

        def cs(i):
            assert lib.lift_scal(n, alpha, xs[i].data_ptr(), outs[i].data_ptr(), sh) == 0

        def ca(i):
            assert lib.lift_asum(n, xs[i].data_ptr(), res.data_ptr(), wsp, wsb, sh) == 0

        def cd(i):
            assert lib.lift_dot(n, xs[i].data_ptr(), ys[i].data_ptr(), res.data_ptr(), wsp, wsb, sh) == 0
        for name, fn, nb in (("scal", cs, 8 * n), ("asum", ca, 4 * n), ("dot", cd, 8 * n)):
            rec(f"{name}_f32_2^27", _time_calls(fn, ns, stream, reps=40), nb, nb)
            d = _per_launch_us(L, lambda i, fn=fn: fn(i % ns), 100)
            out[f"{name}_f32_2^27"]["cold_median_us"] = round(d[len(d) // 2], 3)
            out[f"{name}_f32_2^27"]["cold_median_GB_s"] = round(nb / (d[len(d) // 2] * 1e-6) / 1e9, 1)
        del xs, ys, outs
        torch.cuda.empty_cache()

    if "gemvrect" in which:
        # the paper's large gemv, 8192 x 16384, in both readings of its
        # "vector size 8192": 8192 rows of 16384 columns (x of 16384) and
        # 16384 rows of 8192 columns (x of 8192); A 512 MiB, two rotating copies
        for m, k in ((8192, 16384), (16384, 8192)):
            A, x, y, alpha, beta = W.gemv_rect(m, k)
            nb = 4 * m * k + 4 * k + 8 * m
            As = [A.to(dev) for _ in range(2)]
            xd, yd = x.to(dev), y.to(dev)
            del A

            def cr(i, As=As, xd=xd, yd=yd, m=m, k=k, alpha=alpha, beta=beta):
                assert lib.lift_gemv(m, k, alpha, As[i].data_ptr(), k, xd.data_ptr(), beta, yd.data_ptr(), sh) == 0
            rec(f"gemv_f32_{m}x{k}", _time_calls(cr, 2, stream, reps=40), nb, nb)
            del As
            torch.cuda.empty_cache()

    if "small" in which:
        # asum fp32 n = 2^20 (4 MiB): uniform and integer inputs.  The kernel
        # runs ~5 us, less than a host launch through Python takes, so the
        # launches are captured in a HIP graph and timed as one replay.
        for kind in ("uniform", "integer"):
            x = W.asum_small_vector(integer=kind == "integer")
            n = x.numel()
            ns = max(2, -(-COLD_BYTES // (4 * n)))
            xs = [x.to(dev) for _ in range(ns)]
            res = torch.zeros((), dtype=torch.float32, device=dev)

            def ca(i, h, xs=xs, res=res, n=n):
                assert lib.lift_asum(n, xs[i].data_ptr(), res.data_ptr(), wsp, wsb, h) == 0
            rec(f"asum_f32_{kind}_2^20", _time_graph(ca, ns, stream), 4 * n, 4 * n)
            del xs

    if "half" in which:
        # 16-bit storage asum / dot, n = 2^26
        n = W.HALF_N
        for storage, code in (("bf16", L.LIFT_BF16), ("f16", L.LIFT_F16)):
            x, y = W.half_vectors(storage)
            ns = max(2, -(-COLD_BYTES // (4 * n)))
            xs = [x.to(dev) for _ in range(ns)]
            ys = [y.to(dev) for _ in range(ns)]
            res = torch.zeros((), dtype=torch.float64, device=dev)
            for acc_name, acc in (("f32", 0), ("comp", 1), ("f64combine", 2)):
                def ca(i, acc=acc):
                    assert lib.lift_asum_ex(n, code, xs[i].data_ptr(), acc, L.LIFT_F64, res.data_ptr(), wsp, wsb,
                                            None, sh) == 0

                def cd(i, acc=acc):
                    assert lib.lift_dot_ex(n, code, xs[i].data_ptr(), ys[i].data_ptr(), acc, L.LIFT_F64,
                                           res.data_ptr(), wsp, wsb, None, sh) == 0
                rec(f"asum_{storage}_{acc_name}_2^26", _time_calls(ca, ns, stream), 2 * n, 4 * n)
                if precision is not None:
                    got = precision.setdefault("half", {}).setdefault(storage, (x, y, {}))[2]
                    got[("asum", acc_name)] = res.item()
                rec(f"dot_{storage}_{acc_name}_2^26", _time_calls(cd, ns, stream), 4 * n, 8 * n)
                if precision is not None:
                    got[("dot", acc_name)] = res.item()
            del xs, ys
            torch.cuda.empty_cache()

    if "batch" in which:
        # batched form (4096 reductions + 256 gemv) vs the same problems per call
        for storage in ("f32", "bf16"):
            out.update(batch_form(L, W, dev, stream, storage))
            torch.cuda.empty_cache()

    if "blackscholes" in which:
        # BlackScholes over 2^22 stock prices: 4 B in, 8 B ({call, put}) out per price
        s_cpu, params = W.blackscholes_prices()
        n = s_cpu.numel()
        ns = max(2, -(-COLD_BYTES // (12 * n)))
        ss = [s_cpu.to(dev) for _ in range(ns)]
        outs = [torch.empty((n, 2), device=dev) for _ in range(ns)]

        def cb(i):
            assert lib.lift_blackscholes(n, ss[i].data_ptr(), *params, outs[i].data_ptr(), sh) == 0
        rec("blackscholes_f32_2^22", _time_calls(cb, ns, stream), 12 * n, 12 * n)
        out["blackscholes_f32_2^22"]["options_per_s"] = round(n / (out["blackscholes_f32_2^22"]["avg_us"] * 1e-6), 1)
        del ss, outs
        torch.cuda.empty_cache()

    if "md" in which:
        # MD: 12288 particles (the paper's size) and 2^20, 128 neighbour slots
        # each, particles in random order (irregular gathers); 2^20 also in
        # lattice order, as after a spatial sort of the particles
        for box, tag, shuffle in ((W.MD_BOX, "12288", True), (W.MD_BOX_LARGE, "2^20", True),
                                  (W.MD_BOX_LARGE, "2^20_sorted", False)):
            pos, nbr, params = W.md_system(box, shuffle=shuffle)
            n, k = nbr.shape
            nb = n * k * 4 + 2 * 16 * n
            pairs = out_pairs(pos, nbr, params[0], dev)
            ns = max(2, -(-COLD_BYTES // nb))
            ps = [pos.to(dev) for _ in range(ns)]
            nbs = [nbr.to(dev) for _ in range(ns)]
            fs = [torch.empty((n, 4), device=dev) for _ in range(ns)]

            def cm(i, s, ps=ps, nbs=nbs, fs=fs, n=n, k=k, params=params):
                assert lib.lift_md(n, ps[i].data_ptr(), k, nbs[i].data_ptr(), *params, fs[i].data_ptr(), s) == 0
            name = f"md_f32_{tag}_particles"
            # replayed from a HIP graph: at 12288 particles a launch takes
            # less device time than its host-side call
            rec(name, _time_graph(cm, ns, stream), nb, nb)
            out[name]["interactions_per_s"] = round(pairs / (out[name]["avg_us"] * 1e-6), 1)
            out[name]["slots_per_particle"] = k
            del ps, nbs, fs
            torch.cuda.empty_cache()

    if "gemv16" in which:
        # bf16 gemv 16384^2 (A 512 MiB: larger than the Infinity Cache by itself)
        A, x, y, alpha, beta = W.half_gemv()
        size = A.shape[0]
        Ad, xd, yd = A.to(dev), x.to(dev), y.to(dev)
        nb = 2 * size * size + 4 * size + 8 * size
        fb = 4 * size * size + 4 * size + 8 * size
        got = {}
        for acc_name, acc in (("f32", 0), ("comp", 1), ("f64combine", 2)):
            def cg(i, acc=acc, yv=yd):
                assert lib.lift_gemv_ex(size, size, alpha, L.LIFT_BF16, Ad.data_ptr(), size, xd.data_ptr(), beta,
                                        yv.data_ptr(), acc, None, sh) == 0
            rec(f"gemv_bf16_{acc_name}_{size}", _time_calls(cg, 1, stream, reps=20), nb, fb)
            y1 = y.to(dev)                  # one call on the original y, for the error report
            cg(0, yv=y1)
            got[acc_name] = y1.cpu().numpy().astype("float64")
        if precision is not None:
            precision["gemv16"] = (A, x, y, alpha, beta, got)
    return out


def out_pairs(pos, nbr, cutoff, dev):
    """Interacting (particle, neighbour) pairs: listed, valid, within the cutoff
    (binary32 squared distance against binary32(cutoff^2)), for the
    interactions-per-second figure; counted with torch on the device."""
    import numpy as np
    import torch

    p = pos.to(dev)
    n = p.shape[0]
    t2 = float(np.float32(float(cutoff) * float(cutoff)))
    total = 0
    for lo in range(0, n, 1 << 16):
        idx = nbr[lo:lo + (1 << 16)].to(dev).long()
        ok = (idx >= 0) & (idx < n)
        q = p[idx.clamp(0, n - 1)]
        d = p[lo:lo + (1 << 16), None, :3] - q[..., :3]
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        total += int((ok & (r2 < t2)).sum().item())
    return total


def batch_form(L, W, dev, stream, storage):
    """The batch of 4096 reductions + 256 gemv: one batched run (two persistent
    launches) vs per-call kernels (eager and captured in a graph) over the same
    problems.  Values are drawn on the CPU with the workload's recipe (seed 5)
    and copied to the device once."""
    import torch

    lib = L.library()
    spec = W.batch_shapes()
    reds, gemvs = W.batch_values(spec, storage)
    probs = []
    for kind, x, y in reds:
        probs.append(("dot", x.to(dev), y.to(dev)) if kind == "dot" else ("asum", x.to(dev)))
    for A, x, y in gemvs:
        probs.append(("gemv", W.GEMV_ALPHA, A.to(dev), x.to(dev), W.GEMV_BETA, y.to(dev)))
    del reds, gemvs
    # no knobs: the library's own choice (its autotuned entry for the batch on this device)
    source, _ = L.lift_default_knobs("batch", {"f32": L.LIFT_F32, "bf16": L.LIFT_BF16}[storage], L.LIFT_ACC_F32, 0)
    b = L.Batch(probs)
    fp32_bytes = sum(4 * n * (2 if k == "dot" else 1) + 4 for k, n in zip(spec.red_kind, spec.red_len)) + \
        sum(4 * m * n + 4 * n + 8 * m for m, n in spec.gemv_mn)
    ev = L.HipEvents(2)
    times = []
    for i in range(7):
        if i >= 2:
            lib.lift_time_next_launch(ev.events[0], ev.events[1])
        b.run()
        torch.cuda.synchronize()
        if i >= 2:
            times.append(ev.elapsed_ms(0, 1) * 1e3)
    ev.close()
    batch_us = statistics.median(times)

    # the same problems as per-call plain kernels, back to back on one stream
    ws = L.workspace(dev)
    code = {"f32": L.LIFT_F32, "bf16": L.LIFT_BF16}[storage]
    res = torch.zeros(len(probs), dtype=torch.float32, device=dev)
    calls = []
    for i, pr in enumerate(probs):
        if pr[0] == "asum":
            calls.append(("a", pr[1].numel(), pr[1].data_ptr(), 0, res.data_ptr() + 4 * i))
        elif pr[0] == "dot":
            calls.append(("d", pr[1].numel(), pr[1].data_ptr(), pr[2].data_ptr(), res.data_ptr() + 4 * i))
        else:
            A, x, y = pr[2], pr[3], pr[5]
            calls.append(("g", A.shape[0], A.shape[1], A.data_ptr(), x.data_ptr(), y.data_ptr()))

    def per_call(sh):
        for c in calls:
            if c[0] == "a":
                st = lib.lift_asum_ex(c[1], code, c[2], 0, L.LIFT_F32, c[4], ws.data_ptr(), ws.numel(), None, sh)
            elif c[0] == "d":
                st = lib.lift_dot_ex(c[1], code, c[2], c[3], 0, L.LIFT_F32, c[4], ws.data_ptr(), ws.numel(), None, sh)
            else:
                st = lib.lift_gemv_ex(c[1], c[2], 1.0, code, c[3], c[2], c[4], 0.5, c[5], 0, None, sh)
            if st != 0:
                raise L.LiftError(st, "per-call baseline")

    per_call(stream.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    per_call(stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    eager_us = e0.elapsed_time(e1) * 1e3

    graph_us = None
    try:
        cg = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            with torch.cuda.graph(cg, stream=side):
                per_call(torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        e0.record(stream)
        cg.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        graph_us = e0.elapsed_time(e1) * 1e3
        del cg
    except Exception as exc:  # report, do not fail the bench
        log("per-call graph capture failed:", exc)

    bb = b.bytes
    rec = {"problems": len(probs), "tiles": b.tiles, "grid": b.grid, "bytes": bb, "fp32_bytes": fp32_bytes,
           "batch_us": round(batch_us, 1), "GB_s": round(bb / (batch_us * 1e-6) / 1e9, 1),
           "frac_of_peak": round(bb / (batch_us * 1e-6) / 1e9 / PEAK_GBS, 4),
           "fp32_equiv_GB_s": round(fp32_bytes / (batch_us * 1e-6) / 1e9, 1),
           "per_call_eager_us": round(eager_us, 1),
           "per_call_eager_GB_s": round(bb / (eager_us * 1e-6) / 1e9, 1),
           "per_call_graph_us": round(graph_us, 1) if graph_us else None,
           "per_call_graph_GB_s": round(bb / (graph_us * 1e-6) / 1e9, 1) if graph_us else None,
           "knobs": {0: "default", 1: "tuned", 2: "forced"}[source]}
    log("form batch", storage, rec)
    b.close()
    return {f"batch_{storage}_4096red_256gemv": rec}


if __name__ == "__main__":
    main()
