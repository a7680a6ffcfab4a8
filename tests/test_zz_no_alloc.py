"""GPU test of wake_prepare_noalloc (the entry point for callers that cannot
allocate device memory): through the C ABI, a context prepared into a
caller-owned table with the build staged in the library's static device
array marches bitwise as one prepared by wake_prepare, on two calls in a row
(the second smaller, so the staging array holds the first call's contents
when it starts); sizes beyond the limits and short tables are refused."""
import ctypes

import numpy as np
import pytest

from paper_2603_16623_amd import workloads as W
from parity import FIELDS

pytestmark = pytest.mark.gpu

WAKE_EINVAL = -1


def _hip_runtime():
    """The HIP runtime the library itself loaded."""
    with open("/proc/self/maps") as fh:
        paths = {ln.split()[-1] for ln in fh if "libamdhip64" in ln}
    assert paths, "libamdhip64 not loaded"
    hip = ctypes.CDLL(sorted(paths)[0])
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    return hip


@pytest.fixture(scope="module")
def wk():
    from paper_2603_16623_amd import wake
    wake.load()
    wake.wake_set_tiling(512, 0)
    wake.wake_set_cluster(0, 0)
    yield wake


def _table_bytes(inst):
    n_part = sum(len(s.x) for s in inst.sources if getattr(s, "kind", "") == "particles")
    return 4 * (inst.n_xi + 1) + 32 * n_part + 1024


def _run(wk, inst, hip=None):
    """March the whole window; with hip, prepared by wake_prepare_noalloc
    into a table this function allocates (as the caller would)."""
    s = wk.WakeSolver.from_instance(inst, record_stride=25)
    table = None
    if hip is not None:
        table = ctypes.c_void_p()
        nbytes = _table_bytes(inst)
        assert hip.hipMalloc(ctypes.byref(table), nbytes) == 0
        assert wk.load().wake_prepare_noalloc(s.h, table, nbytes - 1024 - 1) == WAKE_EINVAL  # short
        s.wake_prepare_noalloc(table.value, nbytes)
        s.wake_prepare_noalloc(table.value, nbytes)          # prepared already: nothing done
    s.wake_solve(0, inst.n_xi)
    out = dict(status=s.wake_status(), lineout=s.wake_lineout(),
               snaps=[s.wake_fields(n) for n in range(0, inst.n_xi, 25)],
               last=s.wake_fields(-1), state=s.wake_get_state())
    s.close()
    if table is not None:
        assert hip.hipFree(table) == 0
    return out


def _same(a, b):
    assert a["status"] == b["status"]
    for x, y in zip(a["lineout"], b["lineout"]):
        assert np.array_equal(x, y)
    for fa, fb in zip(a["snaps"] + [a["last"]], b["snaps"] + [b["last"]]):
        for q in FIELDS + ("rho", "ur"):
            assert np.array_equal(fa[q], fb[q]), q
    for q in ("rho", "ur", "f_rho", "f_u"):
        assert np.array_equal(a["state"][q], b["state"][q]), q


def test_noalloc_prepare_matches_wake_prepare_twice(wk):
    hip = _hip_runtime()
    rng = np.random.default_rng(71)
    big = W.batched_instance(rng, 2600, 160, n_drv=9000, n_wit=3000, r_max=4.0)
    small = W.batched_instance(rng, 700, 90, n_drv=2000, n_wit=600, r_max=4.0)
    for inst in (big, small):
        print(f"no-alloc prepare: {inst.n_rings} rings x {inst.n_xi} slices", flush=True)
        _same(_run(wk, inst, hip), _run(wk, inst))


def test_noalloc_prepare_refuses_sizes_beyond_its_limits(wk):
    hip = _hip_runtime()
    rng = np.random.default_rng(72)
    r0, dr = W.uniform_rings(50, 2.0)
    p = W.gaussian_particles(rng, 131073, 1.0, 0.2, 0.3, 1.0)
    s = wk.WakeSolver(r0, dr, 0.05, 40, [p])
    lib = wk.load()
    nbytes = 4 * 41 + 32 * 131073 + 1024
    table = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(table), nbytes) == 0
    assert lib.wake_prepare_noalloc(s.h, None, nbytes) == WAKE_EINVAL
    assert lib.wake_prepare_noalloc(s.h, table, nbytes) == WAKE_EINVAL     # 131073 particles
    s.wake_prepare()                                                        # the allocating path still works
    s.close()
    assert hip.hipFree(table) == 0
