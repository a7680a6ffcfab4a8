"""GPU tests of the autotuner: the layout it measures and installs is the one
new contexts take, the same tuning gives bitwise the same results, and a
tuned layout keeps per-slice parity with the oracle."""
import numpy as np
import pytest

from oracle.wake_oracle import RingOracle
from paper_2603_16623_amd import workloads as W
from parity import FIELDS, check_fields, field_scales

pytestmark = pytest.mark.gpu

LO = [0, 2048, 4096, 8192, 16384, 32768, 65536, 131072]


@pytest.fixture(scope="module")
def wk():
    from paper_2603_16623_amd import wake
    wake.load()
    wake.wake_set_tiling(512, 0)
    wake.wake_set_cluster(0, 0)
    yield wake
    wake.wake_set_tuning(None)


def _insts():
    rng = np.random.default_rng(91)
    sizes = [1500, 1800, 3000, 3500, 5000, 9500]
    return [W.batched_instance(rng, n, 60, n_drv=2000, n_wit=600, r_max=4.0) for n in sizes]


def _bucket(N):
    return max(b for b, lo in enumerate(LO) if N >= lo)


def _batch_results(wk, insts):
    solvers = [wk.WakeSolver.from_instance(i, record_stride=20) for i in insts]
    b = wk.WakeBatch(solvers)
    b.wake_batch_solve(-1)
    b.wake_batch_sync()
    out = [([s.wake_fields(n) for n in (20, 40)], s.wake_lineout(), s.threads(), s.layout())
           for s in solvers]
    b.close()
    for s in solvers:
        s.close()
    return out


def test_tuning_is_measured_applied_and_reproducible(wk):
    insts = _insts()
    print("autotune on 6 instances, 40 slices", flush=True)
    t = wk.wake_autotune(insts, 40)
    print(f"tuning: {t}", flush=True)
    assert wk.wake_get_tuning() == t
    for inst in insts:
        b = _bucket(inst.n_rings)
        assert t["rate"][b] > 0
        assert t["threads"][b] in (256, 512)
    first = _batch_results(wk, insts)
    for inst, (_, _, nt, (g, c)) in zip(insts, first):
        b = _bucket(inst.n_rings)
        assert nt == t["threads"][b]
        rpt = t["rings_per_thread"][b]
        if rpt == 0:
            assert g == 1
        elif g > 1:
            assert c >= rpt
    # the same tuning installed again: bitwise the same results
    wk.wake_set_tuning(None)
    wk.wake_set_tuning(t)
    again = _batch_results(wk, insts)
    for (f1, l1, _, _), (f2, l2, _, _) in zip(first, again):
        for a, b in zip(f1, f2):
            for q in FIELDS:
                assert np.array_equal(a[q], b[q]), q
        assert np.array_equal(l1[0], l2[0]) and np.array_equal(l1[1], l2[1])


def test_tuned_layouts_keep_slice_parity(wk):
    """Every layout a tuning can give, forced on one instance each: the fields
    at a slice inside the driver match the oracle on identical state."""
    rng = np.random.default_rng(92)
    inst = W.batched_instance(rng, 5200, 60, n_drv=2000, n_wit=600, r_max=4.0)
    o = RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens)
    state = o.initial_state()
    for m in range(30):
        _, state = o.slice(m, state)
    ref, _ = o.slice(30, state, keep=True)
    sc = field_scales(ref)
    for nt, rpt in ((512, 0), (512, 1), (512, 2), (512, 4), (512, 8), (256, 0)):
        tun = dict(lo=LO, threads=[nt] * 8, rings_per_thread=[rpt] * 8)
        wk.wake_set_tuning(tun)
        s = wk.WakeSolver.from_instance(inst, record_stride=1)
        label = f"tuned layout threads={nt} rings/thread={rpt} -> {s.layout()}"
        print(label, flush=True)
        assert s.threads() == nt
        s.wake_set_state(30, state["rho"], state["u"], state["fr"], state["fu"])
        s.wake_solve(30, 1)
        check_fields(s.wake_fields(30), ref, sc, label)
        s.close()
    wk.wake_set_tuning(None)
