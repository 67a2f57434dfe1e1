"""C ABI contract on the CPU: the library loads, exports every entry point
declared in include/lift.h, and rejects invalid arguments before any HIP
call.

The rejection cases pass made-up device addresses that the library must turn
down during argument checking, so this module is skipped wherever a GPU is
visible (a broken check would otherwise hand those addresses to a kernel).
"""
import ctypes
import os
import re

import pytest

import paper_1502_02389_amd as L
from paper_1502_02389_amd import lift as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = open(os.path.join(ROOT, "include", "lift.h")).read()


def _gpu_visible():
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def declared_functions():
    body = re.sub(r"/\*.*?\*/", "", HEADER, flags=re.S)
    return sorted(set(re.findall(r"\b(lift_[a-z0-9_]+)\s*\(", body)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("lift_scal", "lift_asum", "lift_dot", "lift_gemv", "lift_workspace_bytes",
                 "lift_asum_ex", "lift_dot_ex", "lift_gemv_ex", "lift_scal_ex"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(B.SIGNATURES)
    for n in declared_functions():
        assert hasattr(B, n), n


def test_enum_values_match_header():
    for name, value in [("LIFT_OK", 0), ("LIFT_EINVAL", -1), ("LIFT_EWORKSPACE", -2), ("LIFT_EHIP", -3),
                        ("LIFT_EUNSUPPORTED", -4), ("LIFT_F32", 0), ("LIFT_BF16", 1), ("LIFT_F16", 2),
                        ("LIFT_F64", 3), ("LIFT_ACC_F32", 0), ("LIFT_ACC_F32_COMP", 1),
                        ("LIFT_ACC_F32_F64COMBINE", 2), ("LIFT_LANES_TREE", 0), ("LIFT_LANES_SEQ", 1),
                        ("LIFT_LANES_RUNS_TREE", 2), ("LIFT_LANES_RUNS_SEQ", 3)]:
        assert re.search(rf"\b{name}\s*=\s*{value}\b", HEADER), name
        assert getattr(B, name) == value


def test_struct_layouts():
    # lift_knobs: int32 x4, int64 split, int32 wg_per_cu, row_split, lanes_per_item, interleave,
    # lane_form (padded to 48)
    assert ctypes.sizeof(B.lift_knobs) == 48
    assert B.lift_knobs.split.offset == 16 and B.lift_knobs.wg_per_cu.offset == 24
    assert B.lift_knobs.lanes_per_item.offset == 32 and B.lift_knobs.lane_form.offset == 40
    # lift_problem: int32 kind, int32 reserved, int64 m, n, lda, 3 pointers, 2 floats
    assert ctypes.sizeof(B.lift_problem) == 64
    assert B.lift_problem.a.offset == 32 and B.lift_problem.alpha.offset == 56


def test_workspace_size_and_version():
    assert L.lift_workspace_bytes() >= 256 + 16 * L.lift_max_workgroups()
    assert (L.lift_workspace_bytes() - 16 * L.lift_max_workgroups()) % 256 == 0
    assert L.lift_max_workgroups() >= 1024
    assert "gfx950" in L.lift_version()
    assert L.lift_status_string(L.LIFT_EINVAL) == "invalid argument"


# ------------------------------------------------------------------ rejections

cpu_only = pytest.mark.skipif(_gpu_visible(), reason="passes fake device addresses; CPU only")

X = 0x7F0000000000          # made-up, 256-byte aligned "device" addresses
Y = 0x7F0001000000
R = 0x7F0002000000
WS = 0x7F0003000000
WSB = None


def wsb():
    return L.lift_workspace_bytes()


@cpu_only
@pytest.mark.parametrize("case,expect", [
    (lambda: L.lift_asum(-1, X, R, WS, wsb()), L.LIFT_EINVAL),                 # negative n
    (lambda: L.lift_asum(10, 0, R, WS, wsb()), L.LIFT_EINVAL),                 # null x
    (lambda: L.lift_asum(10, X, 0, WS, wsb()), L.LIFT_EINVAL),                 # null result
    (lambda: L.lift_asum(10, X + 2, R, WS, wsb()), L.LIFT_EINVAL),             # x not 4-aligned
    (lambda: L.lift_asum(10, X, R + 1, WS, wsb()), L.LIFT_EINVAL),             # result misaligned
    (lambda: L.lift_asum(10, X, R, 0, wsb()), L.LIFT_EWORKSPACE),              # no workspace
    (lambda: L.lift_asum(10, X, R, WS, wsb() - 1), L.LIFT_EWORKSPACE),         # too small
    (lambda: L.lift_asum(10, X, R, WS + 4, wsb()), L.LIFT_EINVAL),             # ws not 16-aligned
    (lambda: L.lift_asum(10, X, X + 8, WS, wsb()), L.LIFT_EINVAL),             # result inside x
    (lambda: L.lift_asum(10, X, WS + 64, WS, wsb()), L.LIFT_EINVAL),           # result inside ws
    (lambda: L.lift_dot(10, X, 0, R, WS, wsb()), L.LIFT_EINVAL),               # null y
    (lambda: L.lift_dot(10, X, Y + 2, R, WS, wsb()), L.LIFT_EINVAL),           # y misaligned
    (lambda: L.lift_dot(10, X, Y, Y + 4, WS, wsb()), L.LIFT_EINVAL),           # result inside y
    (lambda: L.lift_scal(-5, 2.0, X, Y), L.LIFT_EINVAL),
    (lambda: L.lift_scal(10, 2.0, 0, Y), L.LIFT_EINVAL),
    (lambda: L.lift_scal(10, 2.0, X, 0), L.LIFT_EINVAL),
    (lambda: L.lift_scal(10, 2.0, X, X + 4), L.LIFT_EINVAL),                   # partial overlap
    (lambda: L.lift_scal(10, 2.0, X + 36, X), L.LIFT_EINVAL),                  # partial overlap
    (lambda: L.lift_gemv(-1, 4, 1.0, X, 4, Y, 0.5, R), L.LIFT_EINVAL),
    (lambda: L.lift_gemv(4, -1, 1.0, X, 4, Y, 0.5, R), L.LIFT_EINVAL),
    (lambda: L.lift_gemv(4, 8, 1.0, X, 7, Y, 0.5, R), L.LIFT_EINVAL),          # lda < n
    (lambda: L.lift_gemv(4, 0, 1.0, X, 0, Y, 0.5, R), L.LIFT_EINVAL),          # lda < 1
    (lambda: L.lift_gemv(4, 8, 1.0, 0, 8, Y, 0.5, R), L.LIFT_EINVAL),          # null A
    (lambda: L.lift_gemv(4, 8, 1.0, X, 8, 0, 0.5, R), L.LIFT_EINVAL),          # null x
    (lambda: L.lift_gemv(4, 8, 1.0, X, 8, Y, 0.5, 0), L.LIFT_EINVAL),          # null y
    (lambda: L.lift_gemv(4, 8, 1.0, X, 8, Y, 0.5, X + 16), L.LIFT_EINVAL),     # y inside A
    (lambda: L.lift_gemv(4, 8, 1.0, X, 8, Y, 0.5, Y + 4), L.LIFT_EINVAL),      # y inside x
    (lambda: L.lift_gemv(4, 8, 1.0, X, 8, Y + 2, 0.5, R), L.LIFT_EINVAL),      # x misaligned
    (lambda: L.lift_blackscholes(-1, X, 20.0, 0.02, 0.3, 1.0, Y), L.LIFT_EINVAL),
    (lambda: L.lift_blackscholes(8, 0, 20.0, 0.02, 0.3, 1.0, Y), L.LIFT_EINVAL),       # null prices
    (lambda: L.lift_blackscholes(8, X, 20.0, 0.02, 0.3, 1.0, 0), L.LIFT_EINVAL),       # null output
    (lambda: L.lift_blackscholes(8, X + 2, 20.0, 0.02, 0.3, 1.0, Y), L.LIFT_EINVAL),   # prices misaligned
    (lambda: L.lift_blackscholes(8, X, 20.0, 0.02, 0.3, 1.0, Y + 4), L.LIFT_EINVAL),   # pairs not 8-aligned
    (lambda: L.lift_blackscholes(8, X, 20.0, 0.02, 0.3, 1.0, X + 16), L.LIFT_EINVAL),  # overlap
    (lambda: L.lift_blackscholes(8, X, 0.0, 0.02, 0.3, 1.0, Y), L.LIFT_EINVAL),        # strike
    (lambda: L.lift_blackscholes(8, X, 20.0, 0.02, -0.3, 1.0, Y), L.LIFT_EINVAL),      # volatility
    (lambda: L.lift_blackscholes(8, X, 20.0, 0.02, 0.3, 0.0, Y), L.LIFT_EINVAL),       # expiry
    (lambda: L.lift_blackscholes(8, X, 20.0, float("nan"), 0.3, 1.0, Y), L.LIFT_EINVAL),  # rate
    (lambda: L.lift_blackscholes(8, X, float("inf"), 0.02, 0.3, 1.0, Y), L.LIFT_EINVAL),
    (lambda: L.lift_blackscholes(0, X, 20.0, 0.02, 0.3, 1.0, Y), L.LIFT_OK),           # empty: no-op
    (lambda: L.lift_md(-1, X, 4, Y, 2.5, 1.0, 1.0, R), L.LIFT_EINVAL),
    (lambda: L.lift_md(8, X, -1, Y, 2.5, 1.0, 1.0, R), L.LIFT_EINVAL),
    (lambda: L.lift_md(8, 0, 4, Y, 2.5, 1.0, 1.0, R), L.LIFT_EINVAL),                # null positions
    (lambda: L.lift_md(8, X, 4, 0, 2.5, 1.0, 1.0, R), L.LIFT_EINVAL),                # null lists
    (lambda: L.lift_md(8, X, 4, Y, 2.5, 1.0, 1.0, 0), L.LIFT_EINVAL),                # null forces
    (lambda: L.lift_md(8, X + 4, 4, Y, 2.5, 1.0, 1.0, R), L.LIFT_EINVAL),            # pos not 16-aligned
    (lambda: L.lift_md(8, X, 4, Y + 2, 2.5, 1.0, 1.0, R), L.LIFT_EINVAL),            # lists misaligned
    (lambda: L.lift_md(8, X, 4, Y, 2.5, 1.0, 1.0, R + 8), L.LIFT_EINVAL),            # forces misaligned
    (lambda: L.lift_md(8, X, 4, Y, 2.5, 1.0, 1.0, X + 64), L.LIFT_EINVAL),           # forces overlap pos
    (lambda: L.lift_md(8, X, 4, Y, 2.5, 1.0, 1.0, Y + 64), L.LIFT_EINVAL),           # forces overlap lists
    (lambda: L.lift_md(8, X, 4, Y, -1.0, 1.0, 1.0, R), L.LIFT_EINVAL),               # cutoff
    (lambda: L.lift_md(8, X, 4, Y, 2.5, 1.0, 0.0, R), L.LIFT_EINVAL),                # sigma
    (lambda: L.lift_md(8, X, 4, Y, 2.5, float("inf"), 1.0, R), L.LIFT_EINVAL),       # epsilon
    (lambda: L.lift_md(1 << 31, X, 4, Y, 2.5, 1.0, 1.0, R), L.LIFT_EINVAL),          # n too large
    (lambda: L.lift_md(0, X, 4, Y, 2.5, 1.0, 1.0, R), L.LIFT_OK),                    # empty: no-op
    (lambda: L.lift_stream_read(-4, X, R), L.LIFT_EINVAL),
    (lambda: L.lift_stream_read(6, X, R), L.LIFT_EINVAL),                            # not a multiple of 4
    (lambda: L.lift_stream_read(8, X + 4, R), L.LIFT_EINVAL),                        # x not 16-aligned
    (lambda: L.lift_stream_read(8, 0, R), L.LIFT_EINVAL),                            # null x
    (lambda: L.lift_stream_read(8, X, 0), L.LIFT_EINVAL),                            # null sink
    (lambda: L.lift_stream_read(8, X, X + 8), L.LIFT_EINVAL),                        # sink inside x
    (lambda: L.lift_stream_read(8, X, R, B.knobs(vec_bytes=8)), L.LIFT_EUNSUPPORTED),
    (lambda: L.lift_stream_read(8, X, R, B.knobs(unroll=3)), L.LIFT_EINVAL),
    (lambda: L.lift_stream_copy(8, X, Y + 4), L.LIFT_EINVAL),                        # out not 16-aligned
    (lambda: L.lift_stream_copy(8, X, X + 16), L.LIFT_EINVAL),                       # overlap
    (lambda: L.lift_stream_copy(0, X, Y), L.LIFT_OK),                                # empty: no-op
    (lambda: L.lift_dot_ex_noalloc(-1, 0, X, Y, 0, 0, R), L.LIFT_EINVAL),            # the no-workspace dot:
    (lambda: L.lift_dot_ex_noalloc(8, 0, X, 0, 0, 0, R), L.LIFT_EINVAL),             # same checks, before
    (lambda: L.lift_dot_ex_noalloc(8, 0, X, Y, 0, 0, X + 4), L.LIFT_EINVAL),         # any HIP call
    (lambda: L.lift_dot_ex_noalloc(8, 7, X, Y, 0, 0, R), L.LIFT_EINVAL),
    (lambda: L.lift_dot_ex_noalloc(8, 0, X, Y, 0, 0, R, B.knobs(unroll=3)), L.LIFT_EINVAL),
])
def test_rejects_before_any_hip_call(case, expect):
    assert case() == expect


@cpu_only
def test_ex_rejects_bad_enums_and_knobs():
    w = wsb()
    assert L.lift_asum_ex(8, 7, X, 0, 0, R, WS, w) == L.LIFT_EINVAL                # dtype
    assert L.lift_asum_ex(8, L.LIFT_F64, X, 0, 0, R, WS, w) == L.LIFT_EINVAL       # f64 storage
    assert L.lift_asum_ex(8, 0, X, 9, 0, R, WS, w) == L.LIFT_EINVAL                # acc
    assert L.lift_asum_ex(8, 0, X, 0, L.LIFT_BF16, R, WS, w) == L.LIFT_EINVAL      # result type
    assert L.lift_asum_ex(8, 0, X, 0, L.LIFT_F64, R + 4, WS, w) == L.LIFT_EINVAL   # f64 result misaligned
    assert L.lift_asum_ex(8, L.LIFT_BF16, X + 1, 0, 0, R, WS, w) == L.LIFT_EINVAL  # bf16 misaligned
    for bad in (B.knobs(block=96), B.knobs(block=2048), B.knobs(block=32), B.knobs(vec_bytes=3),
                B.knobs(vec_bytes=2), B.knobs(vec_bytes=32), B.knobs(unroll=3), B.knobs(unroll=16),
                B.knobs(rows_per_wave=8), B.knobs(split=-1), B.knobs(row_split=3), B.knobs(row_split=-1)):
        assert L.lift_asum_ex(8, 0, X, 0, 0, R, WS, w, bad) == L.LIFT_EINVAL
    assert L.lift_gemv_ex(4, 8, 1.0, 5, X, 8, Y, 0.5, R, 0) == L.LIFT_EINVAL
    assert L.lift_gemv_ex(4, 8, 1.0, 0, X, 8, Y, 0.5, R, 4) == L.LIFT_EINVAL
    assert L.lift_gemv_ex(4, 8, 1.0, 0, X, 8, Y, 0.5, R, 0, B.knobs(row_split=5)) == L.LIFT_EINVAL
    assert L.lift_scal_ex(8, 1.0, X, Y, B.knobs(unroll=5)) == L.LIFT_EINVAL
    assert L.lift_blackscholes_ex(8, X, 20.0, 0.02, 0.3, 1.0, Y, B.knobs(vec_bytes=2)) == L.LIFT_EINVAL
    assert L.lift_blackscholes_ex(8, X, 20.0, 0.02, 0.3, 1.0, Y, B.knobs(block=100)) == L.LIFT_EINVAL
    for bad in (B.knobs(lanes_per_item=3), B.knobs(lanes_per_item=32), B.knobs(unroll=8), B.knobs(vec_bytes=2)):
        assert L.lift_md_ex(8, X, 4, Y, 2.5, 1.0, 1.0, R, bad) == L.LIFT_EINVAL
    for bad in (B.knobs(interleave=3), B.knobs(interleave=-1)):
        assert L.lift_asum_ex(8, 0, X, 0, 0, R, WS, w, bad) == L.LIFT_EINVAL
    # lane forms: a value outside the enum (any op), a tree form with fewer
    # than 64 lanes, a sequential form with a block that is no power of two,
    # the stride partition; other accumulations and storages are unsupported
    for bad in (B.knobs(lane_form=4), B.knobs(lane_form=-1), B.knobs(lane_form=2, block=32),
                B.knobs(lane_form=3, block=24), B.knobs(lane_form=1, interleave=L.LIFT_INTERLEAVE_STRIDE)):
        assert L.lift_asum_ex(8, 0, X, 0, 0, R, WS, w, bad) == L.LIFT_EINVAL
    assert L.lift_scal_ex(8, 1.0, X, Y, B.knobs(lane_form=5)) == L.LIFT_EINVAL
    assert L.lift_scal_ex(8, 1.0, X, Y, B.knobs(lane_form=1, block=8)) == L.LIFT_EINVAL   # no small blocks
    assert L.lift_asum_ex(8, 0, X, L.LIFT_ACC_F32_COMP, 0, R, WS, w, B.knobs(lane_form=1)) == L.LIFT_EUNSUPPORTED
    assert L.lift_asum_ex(8, L.LIFT_F16, X, 0, 0, R, WS, w, B.knobs(lane_form=3)) == L.LIFT_EUNSUPPORTED


@cpu_only
def test_valid_call_without_gpu_reports_hip_error():
    # all checks pass; the first HIP call fails because no device exists
    st = L.lift_asum(16, X, R, WS, wsb())
    assert st == L.LIFT_EHIP
    assert L.lift_last_hip_error() != 0


def test_tensor_layer_refuses_cpu_tensors():
    import torch

    with pytest.raises(ValueError, match="GPU"):
        L.asum(torch.ones(4))
    with pytest.raises(ValueError, match="GPU"):
        L.scal(2.0, torch.ones(4))


@cpu_only
def test_time_next_launch_argument_rules():
    assert L.lift_time_next_launch(0x1000, 0) == L.LIFT_EINVAL
    assert L.lift_time_next_launch(0, 0x1000) == L.LIFT_EINVAL
    assert L.lift_time_next_launch(0, 0) == L.LIFT_OK


def _batch_status(probs, storage=0, acc=0, rt=0, knobs=None, count=None):
    arr = (B.lift_problem * max(1, len(probs)))()
    for i, p in enumerate(probs):
        for k, v in p.items():
            setattr(arr[i], k, v)
    h = ctypes.c_void_p()
    st = L.lift_batch_create(arr, len(probs) if count is None else count, storage, acc, rt, knobs, h)
    assert not h.value  # nothing is created on error (and no GPU here)
    return st


@cpu_only
def test_batch_rejects_bad_problems():
    ok_red = dict(kind=0, n=16, a=X, out=R)
    assert _batch_status([dict(kind=7, n=4, a=X, out=R)]) == L.LIFT_EINVAL            # kind
    assert _batch_status([dict(ok_red, reserved=1)]) == L.LIFT_EINVAL                  # reserved
    assert _batch_status([dict(ok_red, n=-1)]) == L.LIFT_EINVAL                        # n < 0
    assert _batch_status([dict(ok_red, a=0)]) == L.LIFT_EINVAL                         # null x
    assert _batch_status([dict(ok_red, out=0)]) == L.LIFT_EINVAL                       # null result
    assert _batch_status([dict(ok_red, a=X + 2)]) == L.LIFT_EINVAL                     # misaligned
    assert _batch_status([dict(kind=1, n=16, a=X, out=R)]) == L.LIFT_EINVAL            # dot without y
    assert _batch_status([ok_red, dict(ok_red, a=Y)]) == L.LIFT_EINVAL                 # two results alias
    assert _batch_status([ok_red, dict(kind=0, n=16, a=Y, out=X + 8)]) == L.LIFT_EINVAL  # result in an input
    gemv = dict(kind=2, m=8, n=16, lda=16, a=X, b=Y, out=R, alpha=1.0, beta=0.5)
    assert _batch_status([dict(gemv, lda=15)]) == L.LIFT_EINVAL                        # lda < n
    assert _batch_status([dict(gemv, m=-1)]) == L.LIFT_EINVAL
    assert _batch_status([dict(gemv, b=0)]) == L.LIFT_EINVAL                           # null x
    assert _batch_status([dict(gemv, out=X + 64)]) == L.LIFT_EINVAL                    # y inside A
    assert _batch_status([ok_red], storage=L.LIFT_F64) == L.LIFT_EINVAL
    assert _batch_status([ok_red], acc=5) == L.LIFT_EINVAL
    assert _batch_status([ok_red], rt=L.LIFT_F16) == L.LIFT_EINVAL
    assert _batch_status([ok_red], knobs=B.knobs(wg_per_cu=-1)) == L.LIFT_EINVAL
    assert _batch_status([ok_red], knobs=B.knobs(vec_bytes=2), storage=L.LIFT_BF16) == L.LIFT_EUNSUPPORTED
    assert _batch_status([ok_red], count=-1) == L.LIFT_EINVAL
    assert _batch_status([ok_red], knobs=B.knobs(block=1024)) == L.LIFT_EUNSUPPORTED
    assert _batch_status([ok_red], knobs=B.knobs(row_split=3)) == L.LIFT_EINVAL
    assert _batch_status([ok_red], knobs=B.knobs(row_split=2)) == L.LIFT_EUNSUPPORTED


@cpu_only
def test_batch_null_handles():
    assert L.lift_batch_run(None) == L.LIFT_EINVAL
    st, *_ = L.lift_batch_info(None)
    assert st == L.LIFT_EINVAL
    L.lift_batch_destroy(None)   # no-op
    h = ctypes.c_void_p()
    assert B._lib().lift_batch_create(None, 0, 0, 0, 0, None, None) == L.LIFT_EINVAL


@cpu_only
def test_batch_valid_plan_without_gpu_reports_hip_error():
    assert _batch_status([dict(kind=0, n=16, a=X, out=R),
                          dict(kind=2, m=8, n=16, lda=16, a=Y, b=WS, out=R + 256, alpha=1.0, beta=0.5)]) == L.LIFT_EHIP


def test_names_used_by_gpu_tests_and_bench_exist():
    # the GPU tests only run on a GPU; a name they take from the package
    # that does not exist would surface there first, so check it here
    import glob

    import paper_1502_02389_amd as pkg

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    files = glob.glob(os.path.join(root, "tests", "*.py")) + [os.path.join(root, "bench.py"),
                                                                os.path.join(root, "__graft_entry__.py")]
    missing = []
    for f in files:
        src = open(f).read()
        if "import paper_1502_02389_amd as L" not in src:
            continue
        missing += [(os.path.basename(f), n) for n in set(re.findall(r"\bL\.([A-Za-z_]\w*)", src))
                    if not hasattr(pkg, n)]
    assert not missing, missing


# far-apart (never dereferenced) device-like addresses, so that only the size rule can reject
_P, _N, _F = 1 << 44, 2 << 44, 3 << 44


def test_md_rejects_more_than_2p32_work_items():
    # one thread per lane of each particle: n x 16 (default lanes) must stay below 2^32
    assert L.lift_md((1 << 28) + 1, _P, 4, _N, 2.5, 1.0, 1.0, _F) == L.LIFT_EINVAL
    assert L.lift_md_ex((1 << 29) + 1, _P, 4, _N, 2.5, 1.0, 1.0, _F, B.knobs(lanes_per_item=8)) == L.LIFT_EINVAL


@cpu_only
def test_md_just_below_2p32_work_items_reaches_hip():
    assert L.lift_md((1 << 28) - 64, _P, 4, _N, 2.5, 1.0, 1.0, _F) == L.LIFT_EHIP
