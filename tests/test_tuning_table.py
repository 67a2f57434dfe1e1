"""The autotuned knobs as the C library and the Python cache see them (CPU).

The build compiles tuning.json into a table inside liblift.so; a call
without knobs uses an entry only on the device the cache was tuned on.
These tests query the table through lift_default_knobs with an explicit
architecture and CU count (no GPU needed) and check it against tune.lookup
for every cache entry, the device keying, the size buckets, and the
LIFT_FORCE_CONFIG override (read once per process, so those cases run in a
child process).
"""
import json
import os
import subprocess
import sys

import pytest

import paper_1502_02389_amd as L
from paper_1502_02389_amd import lift as B
from paper_1502_02389_amd import tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STORAGE = {"f32": L.LIFT_F32, "bf16": L.LIFT_BF16, "f16": L.LIFT_F16}
ACC = {"f32": 0, "comp": 1, "f64combine": 2}
FIELDS = [f for f, _ in B.lift_knobs._fields_]


def _cache():
    with open(tune.DEFAULT_CACHE) as f:
        return json.load(f)


def _device():
    d = _cache()["device"]
    return d["arch"], d["cus"]


def _entries():
    return sorted(_cache()["entries"].items())


def _as_dict(k):
    return {f: getattr(k, f) for f in FIELDS}


def test_cache_records_its_device():
    arch, cus = _device()
    assert arch.startswith("gfx") and cus > 0


@pytest.mark.parametrize("key,ent", _entries(), ids=[k for k, _ in _entries()])
def test_c_table_and_python_cache_agree(key, ent, monkeypatch):
    monkeypatch.delenv("LIFT_TUNE_CACHE", raising=False)
    op, storage, acc, bucket = key.split("/")[:4]
    rows = [1 << int(key.split("/")[4]), (2 << int(key.split("/")[4])) - 1] if op == "gemv" else [0]
    arch, cus = _device()
    want = {f: int(ent["knobs"].get(f, 0)) for f in FIELDS}
    for elements in ([0] if op == "batch" else [1 << int(bucket), (1 << int(bucket)) + 12345,
                                                (2 << int(bucket)) - 1]):
        for n in rows:
            src, got = L.lift_default_knobs(op, STORAGE[storage], ACC[acc], elements, arch, cus, row_length=n)
            assert src == 1 and got == want, (elements, n, got, want)
            py = tune.lookup(op, storage, acc, elements, device=(arch, cus), row_length=n)
            assert py is not None and _as_dict(py) == want


def test_gemv_entries_are_keyed_by_row_length():
    # the two shapes of the paper's 8192 x 16384 gemv share m n = 2^27 but
    # not the row length: each gets its own entry, and a row length with no
    # entry gets the defaults
    arch, cus = _device()
    keys = {k for k, _ in _entries()}
    assert {"gemv/f32/f32/27/13", "gemv/f32/f32/27/14"} <= keys
    a = L.lift_default_knobs("gemv", L.LIFT_F32, 0, 1 << 27, arch, cus, row_length=8192)
    b = L.lift_default_knobs("gemv", L.LIFT_F32, 0, 1 << 27, arch, cus, row_length=16384)
    assert a[0] == b[0] == 1 and a[1] != b[1]
    assert L.lift_default_knobs("gemv", L.LIFT_F32, 0, 1 << 27, arch, cus, row_length=64)[0] == 0


def test_other_device_gets_defaults():
    key, ent = _entries()[0]
    op, storage, acc, bucket = key.split("/")[:4]
    arch, cus = _device()
    elements = 0 if op == "batch" else 1 << int(bucket)
    for other in (("gfx942", cus), (arch, cus - 1), ("gfx9500", cus)):
        src, got = L.lift_default_knobs(op, STORAGE[storage], ACC[acc], elements, *other)
        assert src == 0 and not any(got.values()), other
        assert tune.lookup(op, storage, acc, elements, device=other) is None


def test_untuned_shapes_get_defaults():
    arch, cus = _device()
    tuned = {k for k, _ in _entries()}
    for op, e in (("asum", 10), ("dot", 40), ("scal", 3), ("gemv", 13)):
        assert f"{op}/f32/f32/{e}" not in tuned
        src, got = L.lift_default_knobs(op, L.LIFT_F32, 0, 1 << e, arch, cus)
        assert src == 0 and not any(got.values())


def test_query_rejects_bad_arguments():
    arch, cus = _device()
    with pytest.raises(L.LiftError):
        L.lift_default_knobs("gemm", L.LIFT_F32, 0, 16, arch, cus)
    with pytest.raises(L.LiftError):
        L.lift_default_knobs("asum", L.LIFT_F64, 0, 16, arch, cus)
    with pytest.raises(L.LiftError):
        L.lift_default_knobs("asum", L.LIFT_F32, 3, 16, arch, cus)
    with pytest.raises(L.LiftError):
        L.lift_default_knobs("asum", L.LIFT_F32, 0, -1, arch, cus)
    with pytest.raises(L.LiftError):
        L.lift_default_knobs("gemv", L.LIFT_F32, 0, 16, arch, cus, row_length=-4)


def _child(code, env_value):
    env = dict(os.environ)
    env["LIFT_FORCE_CONFIG"] = env_value
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return json.loads(r.stdout.strip().splitlines()[-1])


QUERY = """
import json
import paper_1502_02389_amd as L
try:
    print(json.dumps(list(L.lift_default_knobs("asum", L.LIFT_F32, 0, 1 << 24, "gfx950", 256))))
except L.LiftError as e:
    print(json.dumps([e.status, None]))
"""


def test_force_config_overrides_tuned_and_defaults():
    src, k = _child(QUERY, "block=512,unroll=2,split=65536,interleave=stride,wgcu=4,vec=8")
    assert src == 2
    assert (k["block"], k["unroll"], k["split"], k["interleave"], k["wg_per_cu"], k["vec_bytes"]) == \
        (512, 2, 65536, L.LIFT_INTERLEAVE_STRIDE, 4, 8)
    src, k = _child(QUERY, "wg=128,rpw=2,rowsplit=1,lanes=8,interleave=2,laneform=3")
    assert src == 2 and (k["block"], k["rows_per_wave"], k["row_split"], k["lanes_per_item"], k["interleave"],
                         k["lane_form"]) == (128, 2, 1, 8, L.LIFT_INTERLEAVE_CHUNK, L.LIFT_LANES_RUNS_SEQ)


@pytest.mark.parametrize("bad", ["block", "block=", "block=abc", "blocks=256", "block=-64", "block=256;unroll=2",
                                 "split=99999999999999"])
def test_malformed_force_config_is_rejected(bad):
    src, _ = _child(QUERY, bad)
    assert src == L.LIFT_EINVAL


def _gpu_visible():
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_gpu_visible(), reason="passes fake device addresses; CPU only")
def test_malformed_force_config_fails_calls_without_knobs():
    # a valid asum call without knobs: EINVAL (the override is malformed)
    # before any HIP call; with explicit knobs the override does not apply
    code = """
import json
import paper_1502_02389_amd as L
X, R, WS = 0x7F0000000000, 0x7F0002000000, 0x7F0003000000
a = L.lift_asum(16, X, R, WS, L.lift_workspace_bytes())
b = L.lift_asum_ex(16, 0, X, 0, 0, R, WS, L.lift_workspace_bytes(), L.knobs(block=256))
print(json.dumps([a, b]))
"""
    a, b = _child(code, "block=abc")
    assert a == L.LIFT_EINVAL
    assert b == L.LIFT_EHIP          # checks pass; the first HIP call fails (no device here)
