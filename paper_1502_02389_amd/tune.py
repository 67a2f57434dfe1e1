"""Autotuner for the launch knobs.

The paper picks its split factors and vector widths by trying values
(Section 6.2) and sketches an automatic search (Section 6.3).  This module
does that search on the device: for one (op, storage, accumulation, size)
it times every point of a knob grid -- work-group size, bytes per load
(asVector width), loads in flight per lane, split factor (elements per
work-group), rows per wavefront for gemv -- and keeps the fastest.

Timing: back-to-back launches bracketed by one HIP event pair on the stream
the kernels run on, operands rotated over enough copies (>= 1 GiB) that no
launch finds them in the 256 MB Infinity Cache; best of `trials` repeats.

Results persist in a JSON cache of entries keyed by ``op/storage/acc/bucket``
(bucket = floor(log2(elements))), recorded for one device: its architecture
(e.g. gfx950) and compute-unit count.  ``lookup`` answers only for that
device (None elsewhere), and the library build compiles the same entries
into a table that C callers get when they pass no knobs on such a device
(``lift_default_knobs`` reports it).  ``LIFT_TUNE_CACHE`` overrides the
cache path read by ``lookup`` and written by ``--write``; the library's
table is built from the package's ``tuning.json``.

CLI:  python -m paper_1502_02389_amd.tune --ops asum,dot --sizes 24 [--write]
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import threading

from . import lift as B

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
COLD_BYTES = 1 << 30

STORAGE_BYTES = {"f32": 4, "bf16": 2, "f16": 2}
STORAGE_CODE = {"f32": B.LIFT_F32, "bf16": B.LIFT_BF16, "f16": B.LIFT_F16}


def cache_path() -> str:
    return os.environ.get("LIFT_TUNE_CACHE", DEFAULT_CACHE)


def bucket(elements: int) -> int:
    return int(math.floor(math.log2(elements))) if elements > 0 else 0


def key(op: str, storage: str, acc: str, elements: int, row_length: int = 0) -> str:
    """Cache key: op/storage/acc/bucket; gemv adds the bucket of its row
    length (the lowering that wins depends on it: whether x fits in a
    work-group's registers, how many rows share a wavefront)."""
    k = f"{op}/{storage}/{acc}/{bucket(elements)}"
    if op == "gemv":
        k += f"/{bucket(row_length)}"
    return k


_CACHE = None
_LOCK = threading.Lock()


def load_cache(path: str | None = None) -> dict:
    global _CACHE
    path = path or cache_path()
    with _LOCK:
        if _CACHE is None or _CACHE.get("_path") != path:
            try:
                with open(path) as f:
                    data = json.load(f)
            except (OSError, ValueError):
                data = {"entries": {}}
            data["_path"] = path
            _CACHE = data
    return _CACHE


def current_device():
    """(architecture, compute units) of cuda:0, e.g. ("gfx950", 256)."""
    import torch

    props = torch.cuda.get_device_properties(0)
    return props.gcnArchName.split(":")[0], props.multi_processor_count


def lookup(op: str, storage: str, acc: str, elements: int, device=None, row_length: int = 0):
    """Tuned knobs for this call shape on `device` ((arch, cus); None = the
    current GPU), or None: no entry, or the cache was tuned on another
    device (then the library's defaults apply).  gemv: elements = m n and
    row_length = n."""
    data = load_cache()
    meta = data.get("device") or {}
    if device is None:
        device = current_device()
    if (meta.get("arch"), meta.get("cus")) != tuple(device):
        return None
    ent = data["entries"].get(key(op, storage, acc, elements, row_length))
    if not ent:
        return None
    return B.knobs(**ent["knobs"])


def save_cache(entries: dict, meta: dict, path: str | None = None):
    path = path or cache_path()
    data = load_cache(path)
    data.setdefault("entries", {}).update(entries)
    data["device"] = meta
    out = {k: v for k, v in data.items() if k != "_path"}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


# ---------------------------------------------------------------- search space


def grid(op: str, storage: str, quick: bool = False):
    eb = STORAGE_BYTES[storage]
    if op == "batch":
        blocks = (256, 512) if quick else (128, 256, 512)
        vecs = (16,) if quick else tuple(v for v in (8, 16) if v >= eb)
        splits = (1 << 16, 1 << 17, 1 << 18) if quick else tuple(1 << s for s in range(15, 21))
        for b, v, u, s, w in itertools.product(blocks, vecs, (2, 4, 8), splits, (1, 2, 4, 8)):
            yield dict(block=b, vec_bytes=v, unroll=u, split=s, wg_per_cu=w)
        return
    if op == "gemv":
        blocks = (64, 256, 1024) if quick else (64, 128, 256, 512, 1024)
        vecs = (16,) if quick else tuple(v for v in (4, 8, 16) if v >= eb)
        for b, v, u, r in itertools.product(blocks, vecs, (1, 2, 4, 8), (1, 2, 4)):
            yield dict(block=b, vec_bytes=v, unroll=u, rows_per_wave=r, row_split=1)
        # a work-group per row (16-byte loads); wg_per_cu 0 = library grid
        for b, u, r, w in itertools.product((128, 256, 512, 1024), (2, 4, 8), (1, 2), (0, 2, 8)):
            yield dict(block=b, vec_bytes=16, unroll=u, rows_per_wave=r, row_split=2, wg_per_cu=w)
        return
    if op == "md":
        blocks = (256,) if quick else (64, 256, 1024)
        for b, v, u, l in itertools.product(blocks, (4, 8, 16), (1, 2, 4), (1, 2, 4, 8, 16)):
            yield dict(block=b, vec_bytes=v, unroll=u, lanes_per_item=l)
        return
    if op == "blackscholes":
        blocks = (256, 512) if quick else (128, 256, 512, 1024)
        for b, v, u, w in itertools.product(blocks, (4, 8, 16), (1, 2, 4), (2, 4, 8, 16, 32)):
            yield dict(block=b, vec_bytes=v, unroll=u, wg_per_cu=w)
        return
    # 64 lanes: one wavefront per work-group, whose tree is the wave's
    # butterfly alone (no LDS stage)
    blocks = (256, 512) if quick else (64, 128, 256, 512, 1024)
    vecs = (16,) if quick else tuple(v for v in (4, 8, 16) if v >= eb)
    splits = (0, 1 << 15, 1 << 16, 1 << 17, 1 << 18) if quick else \
        (0, 1 << 13, 1 << 14, 1 << 15, 1 << 16, 1 << 17, 1 << 18)
    for b, v, u, s in itertools.product(blocks, vecs, (1, 2, 4, 8), splits):
        if op in ("asum", "dot"):
            yield dict(block=b, vec_bytes=v, unroll=u, split=s, interleave=B.LIFT_INTERLEAVE_CHUNK)
            yield dict(block=b, vec_bytes=v, unroll=u, split=s, interleave=B.LIFT_INTERLEAVE_STRIDE)
        else:
            yield dict(block=b, vec_bytes=v, unroll=u, split=s)


# ---------------------------------------------------------------- timing


class BatchOperands:
    """The batched workload (reductions + gemv problems), drawn on the CPU with
    the workload's recipe and copied to the device once; each knob point plans
    its own batch over the same tensors."""

    def __init__(self, storage, seed=5):
        import torch

        import workloads as W

        self.op, self.storage = "batch", storage
        dev = torch.device("cuda:0")
        spec = W.batch_shapes()
        reds, gemvs = W.batch_values(spec, storage, seed=seed)
        self.problems = []
        for kind, x, y in reds:
            self.problems.append(("dot", x.to(dev), y.to(dev)) if kind == "dot" else ("asum", x.to(dev)))
        for A, x, y in gemvs:
            self.problems.append(("gemv", W.GEMV_ALPHA, A.to(dev), x.to(dev), W.GEMV_BETA, y.to(dev)))
        self.bytes = None
        self.sets = 1

    def time_us(self, acc, k, reps=5, trials=1, median=False):
        import statistics

        import torch

        b = B.Batch(self.problems, acc=acc, knobs=k)
        self.bytes = b.bytes
        ev = B.HipEvents(2)
        ts = []
        try:
            for i in range(reps + 2):
                if i >= 2:
                    B.lift_time_next_launch(ev.events[0], ev.events[1])
                b.run()
                torch.cuda.synchronize()
                if i >= 2:
                    ts.append(ev.elapsed_ms(0, 1) * 1e3)
        finally:
            ev.close()
            b.close()
        return statistics.median(ts) if median else min(ts)


class Operands:
    """Rotating copies of the operands of one call shape, resident on the GPU."""

    def __init__(self, op, storage, elements, m=None, n=None, seed=11):
        import torch

        self.op, self.storage = op, storage
        dev = torch.device("cuda:0")
        g = torch.Generator("cpu").manual_seed(seed)
        dt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[storage]
        eb = STORAGE_BYTES[storage]
        if op == "gemv":
            self.m, self.n = m, n
            per = m * n * eb
            self.sets = max(2, -(-COLD_BYTES // per))
            A = (torch.rand((m, n), generator=g) * 2 - 1).to(dt).to(dev)
            self.A = [A.clone() for _ in range(self.sets)]
            self.x = (torch.rand(n, generator=g) * 2 - 1).to(dev)
            self.y = torch.zeros(m, device=dev)
            self.bytes = per + 4 * n + 8 * m
        elif op == "md":
            import workloads as W

            box = W.MD_BOX if elements <= W.MD_SLOTS * 16 * 16 * 48 else W.MD_BOX_LARGE
            pos, nbr, self.params = W.md_system(box)
            self.n, self.k = pos.shape[0], nbr.shape[1]
            self.bytes = self.n * self.k * 4 + 2 * 16 * self.n   # lists, positions once, forces
            self.sets = max(2, -(-COLD_BYTES // self.bytes))
            self.x = [pos.to(dev) for _ in range(self.sets)]
            self.nb = [nbr.to(dev) for _ in range(self.sets)]
            self.y = [torch.empty((self.n, 4), device=dev) for _ in range(self.sets)]
        elif op == "blackscholes":
            self.n = elements
            self.bytes = 12 * elements                  # a price in, a {call, put} pair out
            self.sets = max(2, -(-COLD_BYTES // self.bytes))
            s = (torch.rand(elements, generator=g) * 25 + 5).to(dev)
            self.x = [s.clone() for _ in range(self.sets)]
            self.y = [torch.empty((elements, 2), device=dev) for _ in range(self.sets)]
        else:
            self.n = elements
            streams = {"scal": 2, "asum": 1, "dot": 2}[op]
            per = streams * elements * eb
            self.sets = max(2, -(-COLD_BYTES // per))
            x = (torch.rand(elements, generator=g) * 2 - 1).to(dt).to(dev)
            self.x = [x.clone() for _ in range(self.sets)]
            self.y = [x.clone() for _ in range(self.sets)] if op in ("dot", "scal") else None
            self.bytes = per
            self.res = torch.zeros((), dtype=torch.float64, device=dev)
        self.ws = B.workspace(dev)
        self.stream = torch.cuda.current_stream(dev).cuda_stream

    def call(self, i, acc, k):
        s = self.stream
        if self.op == "scal":
            st = B.lift_scal_ex(self.n, 1.5, self.x[i].data_ptr(), self.y[i].data_ptr(), k, s)
        elif self.op == "md":
            st = B.lift_md_ex(self.n, self.x[i].data_ptr(), self.k, self.nb[i].data_ptr(), *self.params,
                              self.y[i].data_ptr(), k, s)
        elif self.op == "blackscholes":
            st = B.lift_blackscholes_ex(self.n, self.x[i].data_ptr(), 20.0, 0.02, 0.3, 1.0, self.y[i].data_ptr(),
                                        k, s)
        elif self.op == "asum":
            st = B.lift_asum_ex(self.n, STORAGE_CODE[self.storage], self.x[i].data_ptr(), acc, B.LIFT_F64,
                                self.res.data_ptr(), self.ws.data_ptr(), self.ws.numel(), k, s)
        elif self.op == "dot":
            st = B.lift_dot_ex(self.n, STORAGE_CODE[self.storage], self.x[i].data_ptr(), self.y[i].data_ptr(), acc,
                               B.LIFT_F64, self.res.data_ptr(), self.ws.data_ptr(), self.ws.numel(), k, s)
        else:
            st = B.lift_gemv_ex(self.m, self.n, 1.0, STORAGE_CODE[self.storage], self.A[i].data_ptr(), self.n,
                                self.x.data_ptr(), 0.5, self.y.data_ptr(), acc, k, s)
        if st != B.LIFT_OK:
            raise B.LiftError(st, f"tune {self.op}")

    def time_us(self, acc, k, reps=40, trials=5):
        """Median over `trials` of the average time of `reps` back-to-back
        calls that rotate over the operand sets (cold Infinity Cache)."""
        import torch

        for i in range(4):
            self.call(i % self.sets, acc, k)
        times = []
        for _ in range(trials):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(reps):
                self.call(i % self.sets, acc, k)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e3 / reps)
        return sorted(times)[len(times) // 2]


def derived(op: str, storage: str, elements: int = None, n: int = None):
    """Knob points of the derivations (rewrite.py) of asum / dot / scal, or of
    gemv rows of n elements: each is the launch of the kernel that executes
    one derived low-level expression."""
    from . import rewrite

    eb = STORAGE_BYTES[storage]
    if op in ("asum", "dot"):
        return rewrite.derived_knob_points(op, elements, elem_bytes=eb)
    if op == "scal":
        return rewrite.scal_knob_points(elements)
    if op == "gemv":
        return rewrite.gemv_knob_points(n, elem_bytes=eb)
    raise ValueError(f"no derived search for {op}")


def tune_one(op, storage, acc, elements=None, m=None, n=None, quick=False, log=None, space="grid"):
    """Search one call shape over the fixed grid or, for asum / dot with
    space="derived", over the kernels of the derived expressions; returns
    (best entry, all results)."""
    ops = BatchOperands(storage) if op == "batch" else Operands(op, storage, elements, m, n)
    accc = acc if op == "batch" else B.ACC[acc]
    if space == "derived":
        points = derived(op, storage, elements, n)
    else:
        points = [(kn, None) for kn in grid(op, storage, quick)]
    results = []
    for kn, d in points:
        k = B.knobs(**kn)
        us = ops.time_us(accc, k)
        gbs = ops.bytes / (us * 1e-6) / 1e9
        results.append((us, kn, gbs, d))
        if log:
            log(f"{op} {storage} {acc} {kn} {us:.2f} us {gbs:.0f} GB/s")
    results.sort(key=lambda r: r[0])
    if op == "batch":
        # runs of a batch differ by about 1 % from one to the next, as much as
        # the leading points do: the best 8 are timed again, interleaved over
        # three rounds, and ranked by their median
        top = results[:8]
        again = {i: [] for i in range(len(top))}
        for _ in range(3):
            for i, (_, kn, _, _) in enumerate(top):
                again[i].append(ops.time_us(accc, B.knobs(**kn), reps=5, median=True))
        import statistics

        results[:8] = sorted(((statistics.median(again[i]), kn, ops.bytes / (statistics.median(again[i]) * 1e-6) / 1e9, d)
                              for i, (_, kn, _, d) in enumerate(top)), key=lambda r: r[0])
        if log:
            for us, kn, gbs, _ in results[:8]:
                log(f"{op} {storage} {acc} re-timed {kn} {us:.2f} us {gbs:.0f} GB/s")
    us, kn, gbs, d = results[0]
    best = {"knobs": kn, "us": round(us, 3), "GB_s": round(gbs, 1), "bytes": ops.bytes}
    if d is not None:
        best["expression"] = str(d.expr)
    return best, [r[:3] for r in results]


def main(argv=None):
    ap = argparse.ArgumentParser(description="tune lift launch knobs on the current GPU")
    ap.add_argument("--ops", default="scal,asum,dot,gemv")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--acc", default="f32")
    ap.add_argument("--sizes", default="20,24", help="log2 element counts (reductions / scal)")
    ap.add_argument("--gemv", default="4096x4096,8192x8192", help="MxN shapes for gemv")
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--write", action="store_true", help="merge winners into the cache")
    ap.add_argument("--top", type=int, default=5)
    ap.add_argument("--verbose", action="store_true", help="print every knob point")
    ap.add_argument("--space", default="grid", choices=("grid", "derived"),
                    help="grid: fixed knob grid; derived: the kernels of the rewrite derivations (asum, dot, scal, gemv)")
    args = ap.parse_args(argv)

    import torch

    props = torch.cuda.get_device_properties(0)
    arch, cus = current_device()
    meta = {"name": props.name, "arch": arch, "cus": cus, "lib": B.lift_version()}
    cached = load_cache().get("device")
    if args.write and cached and cached.get("arch") and (cached.get("arch"), cached.get("cus")) != (arch, cus):
        raise SystemExit(f"the cache holds entries tuned on {cached['arch']} / {cached['cus']} CUs; "
                         f"this device is {arch} / {cus} CUs: set LIFT_TUNE_CACHE to a new file")
    entries = {}

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    for op in args.ops.split(","):
        for storage in args.storage.split(","):
            for acc in args.acc.split(","):
                if op in ("scal", "blackscholes", "md") and (storage != "f32" or acc != "f32"):
                    continue
                shapes = ([tuple(int(v) for v in s.split("x")) for s in args.gemv.split(",")] if op == "gemv"
                          else [(0,)] if op == "batch" else [(1 << int(s),) for s in args.sizes.split(",")])
                for shp in shapes:
                    if op == "gemv":
                        best, res = tune_one(op, storage, acc, m=shp[0], n=shp[1], quick=args.quick,
                                             log=log if args.verbose else None, space=args.space)
                        elements, row_length = shp[0] * shp[1], shp[1]
                    else:
                        best, res = tune_one(op, storage, acc, elements=shp[0], quick=args.quick,
                                             log=log if args.verbose else None, space=args.space)
                        elements, row_length = shp[0], 0
                    k = key(op, storage, acc, elements, row_length)
                    entries[k] = best
                    log(f"== {k}: best {best}")
                    for us, kn, gbs in res[: args.top]:
                        log(f"   {us:8.2f} us {gbs:7.0f} GB/s {kn}")
                    log(f"   ({len(res)} points; slowest {res[-1][0]:.2f} us)")
    print(json.dumps({"device": meta, "entries": entries}), flush=True)
    if args.write:
        save_cache(entries, meta)


if __name__ == "__main__":
    main()
