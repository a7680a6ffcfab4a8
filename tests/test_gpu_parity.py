"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Per-slice cases feed both sides the identical ring state at slice n and
compare the fields at n and the state pushed to n+1.  End-to-end cases
compare whole marches (linear regime) to 1e-8.

Tolerance reading (tests/parity.py).  Fields: per slice and per field,
max_i |gpu - oracle| <= 1e-12 * scale of that field at that slice (B_theta's
scale also takes the beam field B^(b) and the jumps C_i it is assembled
from); every margin is printed.  Ring state: elementwise, 1e-12 of the
largest magnitude of each quantity.  End to end: 1e-8 of each quantity's
largest magnitude.
"""
import numpy as np
import pytest

from oracle.wake_oracle import RingOracle
from paper_2603_16623_amd import workloads as W
from parity import (FIELDS, TOL_E2E, TOL_SLICE, check_axis, check_fields, check_state, field_scales,
                    pushed_by_device, rel as _rel, say as _say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wk():
    from paper_2603_16623_amd import wake
    wake.load()
    yield wake
    wake.wake_set_tiling(512, 0)


def _oracle(inst):
    return RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens)


def _advance(o, state, n0, n1):
    for n in range(n0, n1):
        _, state = o.slice(n, state)
        assert state is not None
    return state


def _case(name):
    if name == "blowout-geometric":
        return W.small_instance(7, n_rings=300, n_xi=200, n_peak=4.0, sigma_r=0.1, dxi=0.01)
    if name == "laser-beam":
        return W.small_instance(8, n_rings=257, n_xi=200, n_peak=1.0, laser=True, dxi=0.01)
    if name == "uniform-linear":
        return W.config1(analytic=False, n_part=4000)
    if name == "laser-channel":   # parabolic channel, three times the axis density at the edge
        return W.small_instance(10, n_rings=700, n_xi=200, n_peak=1.0, laser=True, dxi=0.01,
                                channel_w0=2.0)
    if name == "multitile-1200":
        return W.small_instance(9, n_rings=1200, n_xi=150, n_peak=3.0, sigma_r=0.2, dxi=0.01)
    raise KeyError(name)


# tiling = (threads per workgroup, workgroups per compute unit); each thread
# owns ceil(N / threads) consecutive rings
SLICE_CASES = [
    ("blowout-geometric", (256, 0), (0, 1, 60, 130, 199)),   # 300 rings: 2 per thread, ragged
    ("blowout-geometric", (512, 0), (0, 90, 150)),           # 1 ring per thread, idle threads
    ("laser-beam", (512, 0), (0, 40, 100, 170)),
    ("uniform-linear", (512, 0), (0, 250, 700)),
    ("laser-channel", (256, 0), (0, 50, 120, 190)),          # 3 rings per thread, ragged
    ("multitile-1200", (256, 0), (0, 70, 120)),              # 5 rings per thread
    ("multitile-1200", (512, 0), (100,)),
]

@pytest.mark.parametrize("case,tiling,slices", SLICE_CASES)
def test_slice_parity_on_identical_state(wk, case, tiling, slices):
    inst = _case(case)
    o = _oracle(inst)
    wk.wake_set_tiling(*tiling)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    state = o.initial_state()
    at = 0
    for n in slices:
        state = _advance(o, state, at, n)
        at = n
        ref, new = o.slice(n, state, push=n < inst.n_xi - 1, keep=True)
        assert ref["status"] == 0
        sc = field_scales(ref)
        label = f"{case} tiling={tiling} slice={n} N={inst.n_rings}"
        _say(f"slice parity {label}")
        s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
        s.wake_solve(n, 1)
        got = s.wake_fields(n)
        check_fields(got, ref, sc, label)
        assert np.array_equal(got["rho"], state["rho"])
        if new is not None:
            st = s.wake_get_state()
            assert st["slice"] == n + 1
            check_state(st, new, label)
        lp, le = s.wake_lineout()
        check_axis(lp, le, n, ref, sc, label)
    s.close()


def test_linear_end_to_end(wk):
    """Linear-regime driver (1000 rings x 1200 slices, 10^4 particles)."""
    wk.wake_set_tiling(512, 0)
    inst = W.config1()
    _say("e2e linear 1000x1200")
    ref = _oracle(inst).run(record_stride=100)
    s = wk.WakeSolver.from_instance(inst, record_stride=100)
    s.wake_solve(0, inst.n_xi)
    assert s.wake_status() == (-1, inst.n_xi)
    lp, le = s.wake_lineout()
    assert _rel(lp, ref["axis"][:, 0]) <= TOL_E2E
    assert _rel(le, ref["axis"][:, 1]) <= TOL_E2E
    for n in range(0, inst.n_xi, 100):
        got = s.wake_fields(n)
        for q in FIELDS:
            assert _rel(got[q], ref["snap"][n][q]) <= TOL_E2E, (n, q)
        assert _rel(got["rho"], ref["snap"][n]["rho"]) <= TOL_E2E
        assert _rel(got["ur"], ref["snap"][n]["u"]) <= TOL_E2E
    last = s.wake_fields(-1)
    for q in FIELDS:
        assert _rel(last[q], ref["snap"][inst.n_xi - 1][q]) <= TOL_E2E
    s.close()


def test_linear_channel_end_to_end(wk):
    """Linear driver in a parabolic channel (n = 1 + 4 r^2/w0^4, k_p w0 = 3.4,
    the laser benchmark's profile): density-scaled weights and ion tables."""
    wk.wake_set_tiling(512, 0)
    inst = W.config1(channel_w0=3.4)
    _say("e2e linear channel 1000x1200")
    ref = _oracle(inst).run(record_stride=300)
    s = wk.WakeSolver.from_instance(inst, record_stride=300)
    s.wake_solve(0, inst.n_xi)
    assert s.wake_status() == (-1, inst.n_xi)
    lp, le = s.wake_lineout()
    assert _rel(lp, ref["axis"][:, 0]) <= TOL_E2E
    assert _rel(le, ref["axis"][:, 1]) <= TOL_E2E
    for n in range(0, inst.n_xi, 300):
        got = s.wake_fields(n)
        for q in FIELDS:
            assert _rel(got[q], ref["snap"][n][q]) <= TOL_E2E, (n, q)
        assert _rel(got["ur"], ref["snap"][n]["u"]) <= TOL_E2E
    s.close()


def test_analytic_linear_end_to_end_and_closed_form_sign(wk):
    inst = W.config1(analytic=True, n_peak=1e-3)
    _say("e2e analytic linear")
    ref = _oracle(inst).run(record_stride=0)
    s = wk.WakeSolver.from_instance(inst)
    s.wake_solve(0, inst.n_xi)
    lp, le = s.wake_lineout()
    assert _rel(le, ref["axis"][:, 1]) <= TOL_E2E
    assert _rel(lp, ref["axis"][:, 0]) <= TOL_E2E
    assert le[200] > 0   # the head of an electron driver decelerates it
    s.close()


def test_unperturbed_plasma_stays_at_rest(wk):
    r0, dr = W.geometric_rings(700, 1e-3, 5.0)
    _say("unperturbed 700 rings")
    s = wk.WakeSolver(r0, dr, 0.01, 40, [], record_stride=1)
    s.wake_solve(0, 40)
    for n in (0, 17, 39):
        f = s.wake_fields(n)
        for q in FIELDS:
            assert np.max(np.abs(f[q])) <= 1e-15, (n, q)
    st = s.wake_get_state()
    assert np.max(np.abs(st["rho"] - r0)) <= 1e-15 * r0.max()
    assert np.max(np.abs(st["ur"])) <= 1e-15
    s.close()


def test_unsorted_injected_state_is_sorted_first(wk):
    """Heavily crossed rings (a random state) give the same slice."""
    rng = np.random.default_rng(21)
    inst = W.small_instance(3, n_rings=500, n_xi=50, n_peak=2.0)
    o = _oracle(inst)
    state = o.initial_state()
    state["rho"] = inst.r0 * np.exp(rng.normal(0, 0.2, inst.n_rings))
    state["u"] = rng.normal(0, 0.1, inst.n_rings)
    state["fr"] = rng.normal(0, 0.1, inst.n_rings)
    state["fu"] = rng.normal(0, 0.1, inst.n_rings)
    for tiling in ((512, 0), (256, 0)):
        wk.wake_set_tiling(*tiling)
        _say(f"unsorted state tiling={tiling}")
        ref, new = o.slice(20, state, keep=True)
        s = wk.WakeSolver.from_instance(inst, record_stride=1)
        s.wake_set_state(20, state["rho"], state["u"], state["fr"], state["fu"])
        s.wake_solve(20, 1)
        got = s.wake_fields(20)
        check_fields(got, ref, field_scales(ref), f"unsorted tiling={tiling}")
        st = s.wake_get_state()
        assert _rel(st["rho"], new["rho"]) <= TOL_SLICE
        assert _rel(st["ur"], new["u"]) <= TOL_SLICE
        s.close()


@pytest.mark.parametrize("u_amp", [0.05, 2.0, 40.0])
def test_reorder_after_push(wk, u_amp):
    """Rings pushed past many neighbours in one step (from a few positions up
    to thousands) come out in the same order as the oracle's sort: the slice
    after the push, marched in the same launch, matches the oracle's slice
    on the device's pushed state (itself within 1e-12 of the oracle's)."""
    rng = np.random.default_rng(31)
    inst = W.small_instance(5, n_rings=3000, n_xi=40, n_peak=2.0, geometric=False)
    o = _oracle(inst)
    state = o.initial_state()
    state["u"] = rng.normal(0, u_amp, inst.n_rings)
    n = 10
    _, mid = o.slice(n, state, keep=True)
    order = np.lexsort((np.arange(inst.n_rings), mid["rho"]))
    disp = int(np.abs(np.argsort(order) - np.arange(inst.n_rings)).max())
    for tiling in ((512, 0), (256, 0)):
        wk.wake_set_tiling(*tiling)
        label = f"reorder after push u_amp={u_amp} tiling={tiling}"
        _say(f"{label} max displacement {disp}")
        st, mid_dev = pushed_by_device(wk, inst, n, state)
        check_state(st, mid, label)
        ref, _ = o.slice(n + 1, mid_dev, keep=True)
        s = wk.WakeSolver.from_instance(inst, record_stride=1)
        s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
        s.wake_solve(n, 2)
        got = s.wake_fields(n + 1)
        check_fields(got, ref, field_scales(ref), label)
        assert np.array_equal(got["rho"], mid_dev["rho"])
        s.close()


def test_breakdown_is_reported_at_the_same_slice(wk):
    inst = W.small_instance(4, n_rings=200, n_xi=30, n_peak=1.0)
    o = _oracle(inst)
    state = o.initial_state()
    state["rho"] = 0.5 * inst.r0          # compressed column: psibar < 0
    ref, _ = o.slice(5, state)
    assert ref["status"] == O_BREAKDOWN
    _say("breakdown case")
    wk.wake_set_tiling(512, 0)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    s.wake_set_state(5, state["rho"], state["u"], state["fr"], state["fu"])
    s.wake_solve(5, 3)
    assert s.wake_status()[0] == 5
    with pytest.raises(wk.WakeError) as e:
        s.wake_fields(5)
    assert e.value.code == wk.WAKE_EBREAKDOWN
    st = s.wake_get_state()
    assert st["slice"] == 5
    s.close()


O_BREAKDOWN = -5


def test_edge_sizes(wk):
    """One ring; one slice; ragged first tile; no particles in the window."""
    wk.wake_set_tiling(512, 0)
    cases = []
    r0, dr = W.uniform_rings(1, 2.0)
    cases.append(("one ring", r0, dr, 0.05, 20, [W.GaussianBeam(-1.0, 0.5, 0.5, 0.3, 0.6)]))
    r0, dr = W.uniform_rings(37, 3.0)
    cases.append(("one slice", r0, dr, 0.05, 1, [W.GaussianBeam(-1.0, 0.5, 0.5, 0.3, 0.0)]))
    rng = np.random.default_rng(2)
    far = W.gaussian_particles(rng, 500, 1.0, 0.2, 0.1, 100.0)   # all beyond the window
    r0, dr = W.geometric_rings(1025, 1e-3, 4.0)
    cases.append(("ragged 1025", r0, dr, 0.02, 30, [far, W.GaussianBeam(-1.0, 2.0, 0.2, 0.2, 0.3)]))
    for name, r0, dr, dxi, n_xi, src in cases:
        _say(f"edge case {name}")
        o = RingOracle(r0, dr, dxi, n_xi, src)
        ref = o.run(record_stride=1)
        s = wk.WakeSolver(r0, dr, dxi, n_xi, src, record_stride=1)
        s.wake_solve(0, n_xi)
        for n in range(0, n_xi, max(1, n_xi // 4)):
            got = s.wake_fields(n)
            for q in FIELDS:
                assert _rel(got[q], ref["snap"][n][q]) <= 1e-10, (name, n, q)
        s.close()


def test_particle_radius_rounding_matches_numpy(wk):
    """The beam table's radii are computed exactly like the oracle's
    (sqrt(x*x + y*y), no contraction, correctly rounded sqrt): fields
    agree on a slice where many particles sit near ring radii."""
    rng = np.random.default_rng(5)
    r0, dr = W.uniform_rings(400, 2.0)
    p = W.gaussian_particles(rng, 20000, 1.0, 0.4, 0.05, 0.5)
    o = RingOracle(r0, dr, 0.01, 60, [p])
    ref = o.run(record_stride=1)
    s = wk.WakeSolver(r0, dr, 0.01, 60, [p], record_stride=1)
    s.wake_solve(0, 60)
    for n in (45, 50, 55):
        got = s.wake_fields(n)
        assert _rel(got["bt"], ref["snap"][n]["bt"]) <= 1e-10
    s.close()


def test_batched_equals_alone_bitwise(wk):
    wk.wake_set_tiling(512, 0)
    rng = np.random.default_rng(44)
    insts = [W.batched_instance(rng, n, 120, n_drv=3000, n_wit=1000, r_max=4.0)
             for n in (300, 1500, 777, 64, 2100)]
    _say("batched vs alone")
    alone = []
    for inst in insts:
        s = wk.WakeSolver.from_instance(inst, record_stride=40)
        s.wake_solve(0, inst.n_xi)
        alone.append((s.wake_fields(40), s.wake_lineout(), s.wake_get_state()))
        s.close()
    solvers = [wk.WakeSolver.from_instance(inst, record_stride=40) for inst in insts]
    b = wk.WakeBatch(solvers)
    b.wake_batch_solve(60)     # two chunks: continuous-batching style resume
    b.wake_batch_solve(-1)
    b.wake_batch_sync()
    for s, (f, (lp, le), st) in zip(solvers, alone):
        g = s.wake_fields(40)
        for q in FIELDS:
            assert np.array_equal(g[q], f[q]), q
        glp, gle = s.wake_lineout()
        assert np.array_equal(glp, lp) and np.array_equal(gle, le)
        gst = s.wake_get_state()
        assert np.array_equal(gst["rho"], st["rho"])
    b.close()
    for s in solvers:
        s.close()


def test_graph_replays_match_eager(wk):
    wk.wake_set_tiling(512, 0)
    rng = np.random.default_rng(45)
    insts = [W.batched_instance(rng, n, 80, n_drv=2000, n_wit=500, r_max=4.0) for n in (200, 900, 450)]
    _say("graph replay")
    eager = []
    for inst in insts:
        s = wk.WakeSolver.from_instance(inst)
        s.wake_solve(0, inst.n_xi)
        eager.append((s.wake_lineout(), s.wake_get_state()["rho"]))
        s.close()
    solvers = [wk.WakeSolver.from_instance(inst) for inst in insts]
    b = wk.WakeBatch(solvers)
    b.wake_batch_capture()
    for rep in range(3):
        b.wake_batch_replay()
        b.wake_batch_sync()
        for s, ((lp, le), rho) in zip(solvers, eager):
            glp, gle = s.wake_lineout()
            assert np.array_equal(gle, le), rep
            assert np.array_equal(s.wake_get_state()["rho"], rho), rep
        # eager work of the program between replays
        x = wk.WakeSolver.from_instance(insts[0])
        x.wake_solve(0, 10)
        x.wake_sync()
        x.close()
    b.close()
    for s in solvers:
        s.close()


def test_graph_replay_after_an_eager_solve_of_the_batch(wk):
    """Capture, then an eager partial solve of the same batch, then a replay:
    the replay marches every instance through its whole window from slice 0
    (the graph keeps descriptors of its own), bitwise as the eager solve."""
    wk.wake_set_tiling(512, 0)
    rng = np.random.default_rng(46)
    insts = [W.batched_instance(rng, n, 70, n_drv=2000, n_wit=500, r_max=4.0) for n in (900, 200, 450)]
    _say("capture, eager solve(25), replay")
    eager = []
    for inst in insts:
        s = wk.WakeSolver.from_instance(inst)
        s.wake_solve(0, inst.n_xi)
        eager.append((s.wake_lineout(), s.wake_get_state()["rho"], s.wake_fields(-1)))
        s.close()
    solvers = [wk.WakeSolver.from_instance(inst) for inst in insts]
    b = wk.WakeBatch(solvers)
    b.wake_batch_capture()
    b.wake_batch_solve(25)
    b.wake_batch_sync()
    for s in solvers:
        assert s.wake_status() == (-1, 25)
    b.wake_batch_replay()
    b.wake_batch_sync()
    for s, inst, ((lp, le), rho, last) in zip(solvers, insts, eager):
        assert s.wake_status() == (-1, inst.n_xi)
        glp, gle = s.wake_lineout()
        assert np.array_equal(glp, lp) and np.array_equal(gle, le)
        assert np.array_equal(s.wake_get_state()["rho"], rho)
        g = s.wake_fields(-1)
        for q in FIELDS:
            assert np.array_equal(g[q], last[q]), q
    b.close()
    for s in solvers:
        s.close()


def test_snapshots_before_an_injected_state_are_refused(wk):
    """After wake_set_state(n), recorded slices before n belong to no march of
    this state: wake_fields refuses them (WAKE_ESTATE); slices marched from n
    on are served."""
    wk.wake_set_tiling(512, 0)
    inst = W.small_instance(3, n_rings=300, n_xi=40, n_peak=1.0)
    o = _oracle(inst)
    state = o.initial_state()
    for m in range(10):
        _, state = o.slice(m, state)
    s = wk.WakeSolver.from_instance(inst, record_stride=5)
    s.wake_set_state(10, state["rho"], state["u"], state["fr"], state["fu"])
    s.wake_solve(10, 10)
    for n in (0, 5):
        with pytest.raises(wk.WakeError) as e:
            s.wake_fields(n)
        assert e.value.code == wk.WAKE_ESTATE
    ref, _ = o.slice(10, state, keep=True)
    check_fields(s.wake_fields(10), ref, field_scales(ref), "after injected state")
    s.close()
