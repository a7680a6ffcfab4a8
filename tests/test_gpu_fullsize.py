"""Parity at the configurations' full sizes, in the launch configuration the
benchmark times (512-thread workgroups).

Per-slice parity on identical state: a seeded perturbed state (radii jittered
across their neighbours, random momenta and Adams-Bashforth history), not the
product of either march, is given to both sides at a slice inside the driver,
witness or laser; the fields at that slice and the pushed state must agree to
the per-slice, per-field tolerance (tests/parity.py).  The jitter
crosses hundreds of rings, so the device's first order fix-up runs its long-run
sort at these sizes.
"""
import numpy as np
import pytest

from oracle.wake_oracle import RingOracle, grid_radii
from paper_2603_16623_amd import workloads as W
from parity import FIELDS, check_axis, check_fields, check_state, field_scales

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wk():
    from paper_2603_16623_amd import wake
    wake.load()
    wake.wake_set_tiling(512, 0)
    yield wake
    wake.wake_set_tiling(512, 0)


def _say(*a):
    print(*a, flush=True)


def _perturbed(inst, seed, jitter):
    rng = np.random.default_rng(seed)
    N = inst.n_rings
    return dict(rho=inst.r0 * (1.0 + jitter * rng.standard_normal(N)).clip(0.5, 1.5),
                u=0.02 * rng.standard_normal(N), fr=0.02 * rng.standard_normal(N),
                fu=0.02 * rng.standard_normal(N))


def _check_slice(wk, inst, n, state, label, grid=None, layout=None):
    """grid = (n_r, r_max): also the radial field grid of that slice;
    layout = (members, rings per thread) the context must have."""
    o = RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens)
    ref, new = o.slice(n, state, push=True, keep=True)
    assert ref["status"] == 0, label
    sc = field_scales(ref)
    s = wk.WakeSolver.from_instance(inst, record_stride=n)
    lay = s.layout()
    _say(f"full-size slice parity {label}: N={inst.n_rings} slice={n} layout={lay} grid={grid}")
    if layout is not None:
        assert lay == layout, (label, lay, layout)
    if grid is not None:
        s.wake_set_grid(*grid)
    s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
    s.wake_solve(n, 1)
    got = s.wake_fields(n)
    check_fields(got, ref, sc, label)
    st = s.wake_get_state()
    assert st["slice"] == n + 1
    check_state(st, new, label)
    lp, le = s.wake_lineout()
    check_axis(lp, le, n, ref, sc, label)
    if grid is not None:
        want = o.fields_at(n, ref, grid_radii(*grid))
        got = s.wake_grid_fields(n)
        check_fields(got, ref, field_scales(ref, want), label + " grid", want=want)
    s.close()


def test_blowout_20000_rings_full_size(wk):
    inst = W.config2()                     # 20000 rings, 4000 slices, driver + witness
    for n, seed in ((int(2.8 / inst.dxi), 1), (int(7.3 / inst.dxi), 2)):   # driver, witness centres
        _check_slice(wk, inst, n, _perturbed(inst, seed, 0.01), "blowout-20000x4000", grid=(400, 2.0))


def test_laser_200000_rings_full_size(wk):
    inst = W.config5()                     # 2e5 rings, 8000 slices, laser + witness
    n = int(2.0 / inst.dxi)                # laser centre
    _check_slice(wk, inst, n, _perturbed(inst, 3, 0.002), "laser-200000x8000", grid=(600, 18.0))


def test_batched_instances_full_size(wk):
    insts = W.config3(n_inst=512, n_xi=2000)
    picks = sorted(range(len(insts)), key=lambda i: insts[i].n_rings)
    for i in (picks[0], picks[len(picks) // 2], picks[-1]):   # smallest, median, largest
        inst = insts[i]
        _check_slice(wk, inst, 800, _perturbed(inst, 10 + i, 0.01), f"batched[{i}]", grid=(64, 1.0))


def test_laser_witness_region_matches_split_launches(wk):
    """The 200000-ring laser case through the start of its witness region
    (slices 4000-4100 of 8000), where pushed rings cross hundreds of
    neighbours and the march's order fix-up goes past its block rounds to the
    sort by segments: one launch is bitwise the march split into launches of
    ten slices, whose prologues order each launch's start from scratch."""
    inst = W.config5()
    _say("laser 200000 rings: one launch vs launches of 10 slices through slice 4100")
    a = wk.WakeSolver.from_instance(inst)
    a.wake_solve(0, 4100)
    b = wk.WakeSolver.from_instance(inst)
    b.wake_solve(0, 4000)
    for n in range(4000, 4100, 10):
        b.wake_solve(n, 10)
    assert a.wake_status()[0] == -1 and b.wake_status()[0] == -1
    la, lb = a.wake_lineout(), b.wake_lineout()
    assert np.array_equal(la[0][:4100], lb[0][:4100]) and np.array_equal(la[1][:4100], lb[1][:4100])
    fa, fb = a.wake_fields(-1), b.wake_fields(-1)
    for q in FIELDS + ("rho",):
        assert np.array_equal(fa[q], fb[q]), q
    sa, sb = a.wake_get_state(), b.wake_get_state()
    for q in ("rho", "ur", "f_rho", "f_u"):
        assert np.array_equal(sa[q], sb[q]), q
    a.close()
    b.close()


# The cooperative layouts the autotuner chooses from for instances beyond
# 2048 rings (512-thread members with 1, 2, 4 or 8 rings per thread): the
# benchmark times the large solves in the one it measured fastest.
TUNED_RINGS_PER_THREAD = (1, 2, 4, 8)


def _tuned_layout(wk, rpt):
    return dict(lo=[0, 2048, 4096, 8192, 16384, 32768, 65536, 131072], threads=[512] * 8,
                rings_per_thread=[0, 0, 0] + [rpt] * 5)


def _expect(inst, rpt, nt=512):
    """(members, rings per thread) of a context under that layout."""
    c = max(rpt, -(-inst.n_rings // (256 * nt)))
    return -(-inst.n_rings // (c * nt)), c


def test_large_solves_at_every_tuned_layout(wk):
    """The 20000-ring and 200000-ring solves in every layout the autotuner
    can give them: per-slice parity with a field grid."""
    try:
        for rpt in TUNED_RINGS_PER_THREAD:
            wk.wake_set_tuning(_tuned_layout(wk, rpt))
            inst = W.config2()
            n = int(7.3 / inst.dxi)
            _check_slice(wk, inst, n, _perturbed(inst, 4 + rpt, 0.01),
                         f"blowout-20000x4000 {rpt} rings/thread", grid=(400, 2.0), layout=_expect(inst, rpt))
            inst = W.config5()
            _check_slice(wk, inst, int(2.0 / inst.dxi), _perturbed(inst, 6 + rpt, 0.002),
                         f"laser-200000x8000 {rpt} rings/thread", grid=(600, 18.0), layout=_expect(inst, rpt))
    finally:
        wk.wake_set_tuning(None)


def test_tuned_layouts_split_launches_bitwise(wk):
    """In every such layout, the 20000-ring blowout through its driver
    (slices 0-1200) and the 200000-ring laser case through the start of its
    witness region: one launch is bitwise the march split into launches."""
    try:
        for rpt in TUNED_RINGS_PER_THREAD:
            wk.wake_set_tuning(_tuned_layout(wk, rpt))
            for mk, stop, start, step in ((W.config2, 1200, 0, 100), (W.config5, 4100, 4000, 10)):
                inst = mk()
                _say(f"{rpt} rings/thread: split launches N={inst.n_rings} through slice {stop}")
                a = wk.WakeSolver.from_instance(inst)
                assert a.layout() == _expect(inst, rpt)
                a.wake_solve(0, stop)
                b = wk.WakeSolver.from_instance(inst)
                if start:
                    b.wake_solve(0, start)
                for n in range(start, stop, step):
                    b.wake_solve(n, step)
                assert a.wake_status()[0] == -1 and b.wake_status()[0] == -1
                la, lb = a.wake_lineout(), b.wake_lineout()
                assert np.array_equal(la[0][:stop], lb[0][:stop]) and np.array_equal(la[1][:stop], lb[1][:stop])
                fa, fb = a.wake_fields(-1), b.wake_fields(-1)
                for q in FIELDS + ("rho",):
                    assert np.array_equal(fa[q], fb[q]), q
                a.close()
                b.close()
    finally:
        wk.wake_set_tuning(None)
