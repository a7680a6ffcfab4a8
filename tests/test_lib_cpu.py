"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2603_16623_amd import wake

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wake.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wake_[a-z_]+)\s*\(", src)))


def test_header_declares_the_core_calls():
    names = _declared()
    for n in ("wake_create", "wake_add_beam", "wake_solve", "wake_fields"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(wake.LIB_PATH):
        pytest.fail("libwake.so is not built (python -m paper_2603_16623_amd.build)")
    lib = ctypes.CDLL(wake.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(_declared()) <= set(wake._SIGS)


def test_strerror_and_footprint_need_no_device():
    lib = wake.load()
    assert wake.strerror(wake.WAKE_EBREAKDOWN).startswith("quasistatic breakdown")
    small = wake.wake_footprint(1000, 1200, 10_000, 0)
    big = wake.wake_footprint(20_000, 4000, 70_000, 0)
    assert 0 < small < big
    assert wake.wake_footprint(-1, 10, 0, 0) < 0
    assert wake.wake_tiling_count() == 2
    assert lib.wake_set_tiling(1024, 0) == wake.WAKE_EINVAL   # 1024-thread marcher not offered


def test_malformed_tunings_are_refused_without_a_device():
    import ctypes
    from paper_2603_16623_amd import wake
    lib = wake.load()
    t = wake._Tuning()
    t.n_buckets = 2
    t.lo[0], t.lo[1] = 5, 100          # first bucket must start at 0
    t.threads[0] = t.threads[1] = 512
    assert lib.wake_set_tuning(ctypes.byref(t)) == wake.WAKE_EINVAL
    t.lo[0], t.lo[1] = 0, 0            # not increasing
    assert lib.wake_set_tuning(ctypes.byref(t)) == wake.WAKE_EINVAL
    t.lo[1] = 100
    t.threads[1] = 300                 # no such workgroup size
    assert lib.wake_set_tuning(ctypes.byref(t)) == wake.WAKE_EINVAL
    t.n_buckets = 9                    # more buckets than the table holds
    assert lib.wake_set_tuning(ctypes.byref(t)) == wake.WAKE_EINVAL
    assert lib.wake_get_tuning(ctypes.byref(t)) == wake.WAKE_ESTATE
