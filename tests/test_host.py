"""Host-side logic of the library: exported symbols, layout arithmetic, the
tiling of the moment contraction, argument validation.  No GPU needed."""
import ctypes
import itertools
import math
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pc():
    import paper_1701_05420_amd as pc

    return pc


def test_exports_every_declared_symbol(pc):
    header = open(os.path.join(ROOT, "include", "cumulants.h")).read()
    declared = set(re.findall(r"^\s*(?:cum_status|const char \*)\s*(cum_\w+)\s*\(", header, re.M))
    assert len(declared) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", pc.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\bT (cum_\w+)$", out.stdout, re.M))
    assert declared <= exported, declared - exported
    assert set(pc.EXPORTS) == declared
    for name in declared:
        assert getattr(pc._lib, name)


@pytest.mark.parametrize("n,b", [(1, 1), (5, 2), (7, 3), (16, 2), (48, 4), (24, 3), (64, 4), (255, 16)])
def test_layout_matches_oracle_counts(pc, orc, n, b):
    for d in range(1, 7):
        L = pc.layout(n, d, b)
        nbar = -(-n // b)
        assert L["nbar"] == nbar and L["b_last"] == n - b * (nbar - 1)
        assert L["nblocks"] == math.comb(nbar + d - 1, d)
        assert L["block_elems"] == b ** d
        if L["elems"] <= 2_000_000:
            assert L["elems"] == orc.block_elems(n, d, b)


def test_layout_rejects_bad_arguments(pc):
    for args in [(0, 2, 1), (4, 2, 0), (4, 2, 5), (4, 0, 1), (4, 11, 1)]:
        with pytest.raises(pc.CumulantError):
            pc.layout(*args)


@pytest.mark.parametrize("n,d,b", [(5, 3, 2), (7, 4, 3), (6, 2, 2), (4, 5, 1), (9, 6, 3)])
def test_stored_offset_against_oracle_positions(pc, orc, n, d, b):
    elems = pc.layout(n, d, b)["elems"]
    offs = np.arange(elems)
    idx = orc.block_indices(n, d, b, offs)
    for o, ix in zip(offs, idx):
        if ix[0] < 0:
            continue
        o2 = pc.stored_offset(n, d, b, ix)
        ix2 = orc.block_indices(n, d, b, [o2])[0]
        assert sorted(ix2) == sorted(ix)
        assert list(ix2) == sorted(ix2)  # the canonical copy holds the sorted index
        if list(ix) == sorted(ix):
            assert o2 == o


@pytest.mark.parametrize("n,b", [(1, 1), (3, 1), (5, 2), (7, 3), (16, 2), (13, 4), (33, 5)])
def test_plan_covers_every_stored_entry_once(pc, n, b):
    for d in range(2, 11):
        if pc.layout(n, d, b)["elems"] > 3_000_000:
            continue
        pc.plan_check(n, d, b)


@pytest.mark.parametrize("n,b,d", [(48, 4, 4), (24, 3, 6), (32, 4, 4), (64, 4, 4)])
def test_plan_workload_shapes(pc, n, b, d):
    pc.plan_check(n, d, b)


@pytest.mark.parametrize("n,b,d", [(9, 8, 6), (34, 34, 4), (6, 2, 10), (6, 2, 8), (5, 1, 9)])
def test_recursion_tables(pc, n, b, d):
    """The finalisation's tables: partitions into >= 2 parts of >= 2
    positions, each once and as many as there are set partitions without
    singletons (less the one-part partition); staged sub-block slots.  The
    first three shapes hold too many lower-order entries per block (72640,
    6936, 52884) to stage them in LDS, the last two stage them (5264, 492)."""
    pc.plan_check(n, d, b)


def test_workspace_size_is_host_only_and_monotone(pc):
    a = pc.workspace_size(100_000, 48, 4, 4, "f32")
    b = pc.workspace_size(100_000, 48, 4, 4, "f64")
    c = pc.workspace_size(200_000, 48, 4, 4, "f32")
    assert a > 100_000 * 48 * 4 and b > a - 100_000 * 48 * 4 and c >= a
    with pytest.raises(pc.CumulantError):
        pc.workspace_size(0, 48, 4, 4, "f32")
    with pytest.raises(pc.CumulantError):
        pc.workspace_size(10, 48, 11, 4, "f32")


def _raw(pc, fn, *args):
    return getattr(pc._lib, fn)(*args)


def test_entry_points_validate_before_touching_the_device(pc):
    # bogus non-null device pointers are never dereferenced: validation fails first
    P = ctypes.c_void_p(0x1000)
    N = None
    kap = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    kap_null = (ctypes.c_void_p * 3)(0x1000, None, 0x1000)
    assert _raw(pc, "cum_cumulants", P, 0, 4, 4, 4, 2, 0, N, kap, P, 1 << 30, N) == -1      # t = 0
    assert _raw(pc, "cum_cumulants", P, 10, 4, 3, 4, 2, 0, N, kap, P, 1 << 30, N) == -1     # ldx < n
    assert _raw(pc, "cum_cumulants", P, 10, 4, 4, 4, 5, 0, N, kap, P, 1 << 30, N) == -1     # b > n
    assert _raw(pc, "cum_cumulants", P, 10, 4, 4, 11, 2, 0, N, kap, P, 1 << 30, N) == -1    # d_max > 10
    assert _raw(pc, "cum_cumulants", P, 10, 4, 4, 4, 2, 7, N, kap, P, 1 << 30, N) == -4     # prec
    assert _raw(pc, "cum_cumulants", P, 10, 4, 4, 4, 2, 0, N, kap_null, P, 1 << 30, N) == -1
    assert _raw(pc, "cum_cumulants", N, 10, 4, 4, 4, 2, 0, N, kap, P, 1 << 30, N) == -1
    assert _raw(pc, "cum_cumulants", P, 10, 4, 4, 4, 2, 0, N, kap, P, 16, N) == -2          # workspace
    assert b"workspace" in pc._lib.cum_last_error()
    assert _raw(pc, "cum_moment_blocks", P, 0, 10, 4, 1, 2, P, P, 1 << 30, N) == -1         # d = 1
    assert _raw(pc, "cum_moment_blocks", P, 0, 10, 4, 4, 2, P, P, 8, N) == -2
    assert _raw(pc, "cum_center", P, 10, 4, 2, 0, P, P, P, 1 << 20, N) == -1                # ldx < n
    assert _raw(pc, "cum_unfold", P, 4, 11, 2, P, N) == -1
    # streams: arguments are checked before any device memory is allocated
    h = ctypes.c_void_p()
    assert _raw(pc, "cum_stream_create", 0, 4, 1, 0, N, ctypes.byref(h)) == -1              # n = 0
    assert _raw(pc, "cum_stream_create", 5, 11, 2, 0, N, ctypes.byref(h)) == -1             # d_max > 10
    assert _raw(pc, "cum_stream_create", 5, 4, 6, 0, N, ctypes.byref(h)) == -1              # b > n
    assert _raw(pc, "cum_stream_create", 5, 4, 2, 9, N, ctypes.byref(h)) == -4              # prec
    assert _raw(pc, "cum_stream_create", 5, 4, 2, 0, N, N) == -1
    assert _raw(pc, "cum_stream_update", N, P, 10, 5, 1, N) == -1
    assert _raw(pc, "cum_stream_cumulants", N, P, kap, N) == -1
    assert _raw(pc, "cum_stream_count", N, ctypes.byref(ctypes.c_int64())) == -1


def test_tuning_round_trip_and_validation(pc):
    shape = (1000, 12, 4, 3, "f32")
    pc.set_tuning(*shape, None)
    assert pc.get_tuning(*shape) == {"shape": 0, "target_items": 4096, "inner_b": 1}
    pc.set_tuning(*shape, "32x64", 2048, inner_b=3)
    assert pc.get_tuning(*shape) == {"shape": 2, "target_items": 2048, "inner_b": 3}
    for bad in [dict(inner_b=0), dict(inner_b=4), dict(target_items=0)]:
        with pytest.raises(pc.CumulantError):
            pc.set_tuning(*shape, "32x32", **{"target_items": 512, **bad})
    with pytest.raises(pc.CumulantError):
        pc.set_tuning(*shape, 1, 512)  # no such tile shape
    assert pc.get_tuning(*shape)["target_items"] == 2048  # refused settings change nothing
    pc.set_tuning(*shape, None)
    # the workspace follows the chosen chunking: more work items, more
    # sample chunks, a larger partial-sum buffer
    pc.set_tuning(100_000, 48, 4, 4, "f32", "32x32", 16384, inner_b=1)
    big = pc.workspace_size(100_000, 48, 4, 4, "f32")
    pc.set_tuning(100_000, 48, 4, 4, "f32", "32x32", 1024, inner_b=1)
    small = pc.workspace_size(100_000, 48, 4, 4, "f32")
    pc.set_tuning(100_000, 48, 4, 4, "f32", None)
    assert small < big


def test_tune_file_is_read_and_bad_lines_skipped(tmp_path):
    """The cache file: one "n b dlo dhi prec t shape target inner_b" line per
    shape; lines that do not parse or name an invalid choice are skipped."""
    f = tmp_path / "tune.txt"
    f.write_text("12 3 2 4 1 1000 2 4096 2\n"     # valid
                 "12 3 2 5 1 1000 2 4096\n"       # too few fields
                 "12 3 2 6 1 1000 2 4096 7\n"     # inner_b > b
                 "12 3 2 3 1 1000 5 4096 1\n")    # unknown shape
    code = ("import paper_1701_05420_amd as pc\n"
            "print(pc.get_tuning(1000, 12, 4, 3, 'f32'))\n"
            "print(pc.get_tuning(1000, 12, 5, 3, 'f32'))\n"
            "print(pc.get_tuning(1000, 12, 6, 3, 'f32'))\n"
            "print(pc.get_tuning(1000, 12, 3, 3, 'f32'))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CUM_TUNE_FILE=str(f), PYTHONPATH=root)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True,
                         timeout=120).stdout.splitlines()
    assert out[0] == "{'shape': 2, 'target_items': 4096, 'inner_b': 2}"
    for line in out[1:]:
        assert line == "{'shape': 0, 'target_items': 4096, 'inner_b': 1}"


def test_plan_info_counts(pc):
    """The split of a call: partial sums in the inner layout (each sorted
    variable tuple once at inner block size 1), outputs in block storage, and
    one work item per (tile, chunk) at most."""
    shape = (100_000, 48, 4, 4, "f32")
    pc.set_tuning(*shape, None)
    info = pc.plan_info(*shape)
    assert info["partial_entries"] == sum(math.comb(48 + d - 1, d) for d in range(2, 5))
    assert info["stored_entries"] == sum(pc.layout(48, d, 4)["elems"] for d in range(2, 5))
    assert 1 <= info["nchunks"] <= 100_000 // 64 // 4
    assert info["work_items"] <= info["tiles"] * info["nchunks"]
    pc.set_tuning(*shape, "32x32", 1024, inner_b=4)
    info4 = pc.plan_info(*shape)
    assert info4["partial_entries"] == info4["stored_entries"]
    pc.set_tuning(*shape, None)


def test_missing_library_fails_loudly(tmp_path):
    """A copy of the package without its built library refuses to import:
    there is no fallback implementation to take over."""
    import shutil

    pkg = tmp_path / "paper_1701_05420_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1701_05420_amd", "__init__.py"), pkg / "__init__.py")
    out = subprocess.run([sys.executable, "-c", "import paper_1701_05420_amd"], cwd=tmp_path,
                         env=dict({k: v for k, v in os.environ.items() if k != "CUM_LIBRARY"},
                                  PYTHONPATH=str(tmp_path)), capture_output=True, text=True, timeout=120)
    assert out.returncode != 0
    assert "ImportError" in out.stderr and "no fallback" in out.stderr


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: --gpus 2 ends with a message, before
    any device work."""
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU only" in out.stderr and not out.stdout


def test_workspace_holds_lower_moments_from_order_7(pc):
    """From d_max = 7 on, the workspace also holds the central moments of
    orders 2..d_max-2 in block storage (the first-position finalisation):
    going from d_max = 6 to 7 adds at least those bytes."""
    t, n, b = 20_000, 8, 2
    lower = sum(pc.layout(n, m, b)["elems"] * 8 for m in range(2, 6))
    assert pc.workspace_size(t, n, 7, b, "f32") >= pc.workspace_size(t, n, 6, b, "f32") + lower


def test_blocks_beyond_32_bit_entries_are_refused(pc):
    """b^d is checked without wrapping: 97^10 and 112^10 exceed 64 bits and
    wrapped to negative values in a plain product."""
    P = ctypes.c_void_p(0x1000)
    for n, b in [(100, 97), (112, 112), (112, 84)]:
        L = pc.Layout()
        assert _raw(pc, "cum_layout_query", n, 10, b, ctypes.byref(L)) == -4
        sz = ctypes.c_size_t()
        assert _raw(pc, "cum_workspace_size", 1000, n, 10, b, 1, ctypes.byref(sz)) == -4
        assert _raw(pc, "cum_moment_blocks", P, 1, 1000, n, 10, b, P, P, 1 << 40, None) == -4
        h = ctypes.c_void_p()
        assert _raw(pc, "cum_stream_create", n, 10, b, 1, None, ctypes.byref(h)) == -4
        ts = (ctypes.c_int64 * 2)(100, 200)
        assert _raw(pc, "cum_batch_create", 2, ts, n, 10, b, 1, ctypes.byref(h)) == -4
    # within 32 bits the layout is reported exactly
    assert pc.layout(100, 4, 97)["block_elems"] == 97 ** 4


def test_orders_7_and_above_stage_in_fp64(pc):
    """A call that centres its own data with d_max >= 7 stages and contracts
    in FP64 in every precision: its workspace and its plan are those of the
    FP64 call, while d_max = 6 keeps the precision asked for."""
    t, n, b = 20_000, 8, 2
    for prec in ("f32", "bf16x2", "bf16x3", "f16x2"):
        for dmax in (7, 10):
            assert pc.workspace_size(t, n, dmax, b, prec) == pc.workspace_size(t, n, dmax, b, "f64")
            assert pc.plan_info(t, n, dmax, b, prec) == pc.plan_info(t, n, dmax, b, "f64")
        assert pc.workspace_size(t, n, 6, b, prec) < pc.workspace_size(t, n, 6, b, "f64")


def test_noalloc_entry_point_refuses_before_any_device_work(pc):
    """The allocation-free entry point checks on the host, before anything is
    enqueued: a call whose workspace exceeds the fixed scratch is refused
    (CUM_ENOMEM), and so is one whose device tables do not exist yet
    (CUM_EUNSUPPORTED); argument errors are those of cum_cumulants."""
    P = ctypes.c_void_p(0x1000)
    kap = (ctypes.c_void_p * 9)(*([0x1000] * 9))
    # n = 64, d <= 5, t = 5e6: hundreds of MB of staged data alone
    assert pc.workspace_size(5_000_000, 64, 5, 4, "f32") > pc.NOALLOC_SCRATCH_BYTES
    assert _raw(pc, "cum_cumulants_noalloc", P, 5_000_000, 64, 64, 5, 4, 1, P, kap, None) == -2
    assert b"scratch" in pc._lib.cum_last_error()
    # a configuration never run: no device tables
    assert _raw(pc, "cum_cumulants_noalloc", P, 1000, 11, 11, 4, 3, 1, P, kap, None) == -4
    assert b"cum_cumulants once" in pc._lib.cum_last_error()
    assert _raw(pc, "cum_cumulants_noalloc", P, 0, 11, 11, 4, 3, 1, P, kap, None) == -1     # t = 0
    assert _raw(pc, "cum_cumulants_noalloc", P, 10, 4, 4, 4, 2, 7, P, kap, None) == -4      # prec
