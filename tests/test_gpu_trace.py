"""WAKE_TRACE: per-slice timings of a solve, results unchanged."""
import os

import numpy as np
import pytest

from paper_2603_16623_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wk():
    from paper_2603_16623_amd import wake
    wake.load()
    return wake


@pytest.mark.parametrize("ion_mass", [None, 1836.0])
def test_traced_solve_writes_one_line_per_slice_and_is_bitwise(wk, tmp_path, ion_mass):
    inst = W.small_instance(7, n_rings=300, n_xi=60, n_peak=4.0, sigma_r=0.1, dxi=0.02)
    print(f"trace ion_mass={ion_mass}", flush=True)

    def make():
        return wk.WakeSolver(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, record_stride=10,
                             ion_mass=ion_mass)

    plain = make()
    plain.wake_solve(0, inst.n_xi)
    ref = [plain.wake_fields(n) for n in range(0, inst.n_xi, 10)], plain.wake_lineout()
    plain.close()
    path = tmp_path / "trace.txt"
    traced = make()
    os.environ["WAKE_TRACE"] = str(path)
    try:
        traced.wake_solve(0, 25)
        traced.wake_solve(25, inst.n_xi - 25)
    finally:
        del os.environ["WAKE_TRACE"]
    lines = path.read_text().splitlines()
    assert len(lines) == inst.n_xi
    fields = [dict(kv.split("=") for kv in ln.split()[1:]) for ln in lines]
    assert [int(f["slice"]) for f in fields] == list(range(inst.n_xi))
    assert all(float(f["us"]) > 0 and int(f["breakdown"]) == -1 for f in fields)
    assert all(int(f["rings"]) == inst.n_rings for f in fields)
    got = [traced.wake_fields(n) for n in range(0, inst.n_xi, 10)], traced.wake_lineout()
    for a, b in zip(ref[0], got[0]):
        for q in a:
            assert np.array_equal(a[q], b[q])
    assert np.array_equal(ref[1][0], got[1][0]) and np.array_equal(ref[1][1], got[1][1])
    assert traced.wake_counters()["slices"] == inst.n_xi
    traced.close()
