"""GPU parity of cooperative instances: several workgroups march one instance
(the large-ring-count path), here forced onto small instances so the oracle
stays fast.  Same tolerances as the single-workgroup parity tests; the
cooperative march must also be bitwise reproducible across launch splits and
inside a batch."""
import numpy as np
import pytest

from oracle.wake_oracle import RingOracle
from paper_2603_16623_amd import workloads as W

pytestmark = pytest.mark.gpu

from parity import (FIELDS, TOL_SLICE, check_axis, check_fields, check_state, field_scales,
                    pushed_by_device, rel as _rel)


@pytest.fixture(scope="module")
def wk():
    from paper_2603_16623_amd import wake
    wake.load()
    yield wake
    wake.wake_set_cluster(0, 0)
    wake.wake_set_tiling(512, 0)


def _say(*a):
    print(*a, flush=True)


def _oracle(inst):
    return RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens)


def _inst(n=3000, n_xi=60, channel_w0=None):
    return W.small_instance(5, n_rings=n, n_xi=n_xi, n_peak=3.0, sigma_r=0.2, geometric=False, dxi=0.02,
                            channel_w0=channel_w0)


# (threads, rings per thread): members = ceil(3000 / (threads * rings)); the
# last case in a parabolic channel (n = 1 + 4 r^2/w0^4, w0 = 2)
LAYOUTS = [((256, 0), 2, 6, None), ((512, 0), 1, 6, None), ((512, 0), 4, 2, None),
           ((256, 0), 2, 6, 2.0)]


@pytest.mark.parametrize("tiling,rings,members,channel_w0", LAYOUTS,
                         ids=["256x2", "512x1", "512x4", "256x2-channel"])
def test_cluster_slice_parity(wk, tiling, rings, members, channel_w0):
    inst = _inst(channel_w0=channel_w0)
    o = _oracle(inst)
    wk.wake_set_tiling(*tiling)
    wk.wake_set_cluster(rings, 500)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    assert s.layout() == (members, rings)
    state = o.initial_state()
    at = 0
    for n in (0, 25, 50):
        for m in range(at, n):
            _, state = o.slice(m, state)
        at = n
        ref, new = o.slice(n, state, keep=True)
        sc = field_scales(ref)
        label = (f"cluster tiling={tiling} rings={rings} members={members} channel={channel_w0} "
                 f"slice={n}")
        _say(f"cluster slice parity {label}")
        s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
        s.wake_solve(n, 1)
        got = s.wake_fields(n)
        check_fields(got, ref, sc, label)
        st = s.wake_get_state()
        assert st["slice"] == n + 1
        check_state(st, new, label)
        lp, le = s.wake_lineout()
        check_axis(lp, le, n, ref, sc, label)
    s.close()


@pytest.mark.parametrize("n_rings,members", [(16300, 64), (16500, 65)], ids=["64-members", "65-members"])
def test_cluster_member_count_edges(wk, n_rings, members):
    """At 64 members the member scans still take one member per lane while the
    stamps already sit side by side; at 65 the scans take four members per
    lane.  Slice parity against the oracle at both edges."""
    inst = _inst(n=n_rings, n_xi=40)
    o = _oracle(inst)
    wk.wake_set_tiling(256, 0)
    wk.wake_set_cluster(1, 500)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    assert s.layout() == (members, 1)
    state = o.initial_state()
    at = 0
    for n in (0, 30):
        for m in range(at, n):
            _, state = o.slice(m, state)
        at = n
        ref, new = o.slice(n, state, keep=True)
        sc = field_scales(ref)
        label = f"cluster {members} members slice={n}"
        _say(f"cluster member-count edge {label}")
        s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
        s.wake_solve(n, 1)
        got = s.wake_fields(n)
        check_fields(got, ref, sc, label)
        check_state(s.wake_get_state(), new, label)
    s.close()


@pytest.mark.parametrize("u_amp", [0.05, 2.0, 40.0])
def test_cluster_reorder_after_push(wk, u_amp):
    """Pushed rings crossing a few to thousands of neighbours, across member
    boundaries: block rounds over all members, and the sort by segments for
    the far moves.
    The slice after the push (same launch) against the oracle's slice on
    the device's pushed state."""
    rng = np.random.default_rng(31)
    inst = _inst(n_xi=40)
    o = _oracle(inst)
    state = o.initial_state()
    state["u"] = rng.normal(0, u_amp, inst.n_rings)
    n = 10
    _, mid = o.slice(n, state, keep=True)
    wk.wake_set_tiling(256, 0)
    wk.wake_set_cluster(2, 500)
    label = f"cluster reorder u_amp={u_amp}"
    _say(label)
    st, mid_dev = pushed_by_device(wk, inst, n, state)
    check_state(st, mid, label)
    ref, _ = o.slice(n + 1, mid_dev, keep=True)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    assert s.layout()[0] == 6
    s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
    s.wake_solve(n, 2)
    got = s.wake_fields(n + 1)
    check_fields(got, ref, field_scales(ref), label)
    assert np.array_equal(got["rho"], mid_dev["rho"])
    c = s.wake_counters()
    print(label, {k: c[k] for k in ("fixups", "member_local_rounds", "all_member_rounds", "segment_sorts", "bitonic_fallbacks")}, flush=True)
    # the crossings reach over member boundaries: rounds over all members
    # (each with one fenced meeting; both members of a straddling block sort
    # it) ran, and at the largest velocities the sort by segments after them
    assert c["all_member_rounds"] >= 1
    if u_amp >= 40.0:
        assert c["segment_sorts"] + c["bitonic_fallbacks"] >= 1
    s.close()


def test_cluster_unsorted_injected_state(wk):
    """A random (heavily crossed) injected state is ordered before the first
    slice (the bitonic fallback over all members)."""
    rng = np.random.default_rng(21)
    inst = _inst(n_xi=40)
    o = _oracle(inst)
    state = o.initial_state()
    state["rho"] = inst.r0 * np.exp(rng.normal(0, 0.2, inst.n_rings))
    state["u"] = rng.normal(0, 0.1, inst.n_rings)
    ref, new = o.slice(20, state, keep=True)
    wk.wake_set_tiling(256, 0)
    wk.wake_set_cluster(2, 500)
    _say("cluster unsorted injected state")
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    s.wake_set_state(20, state["rho"], state["u"], state["fr"], state["fu"])
    s.wake_solve(20, 1)
    got = s.wake_fields(20)
    check_fields(got, ref, field_scales(ref), "cluster unsorted")
    st = s.wake_get_state()
    assert _rel(st["rho"], new["rho"]) <= TOL_SLICE
    s.close()


def test_cluster_split_and_batch_bitwise(wk):
    """A cooperative march split over launches, and inside a batch with
    single-workgroup instances, is bitwise the one-launch march."""
    wk.wake_set_tiling(256, 0)
    wk.wake_set_cluster(2, 2000)
    big = _inst(n_xi=60)
    rng = np.random.default_rng(44)
    small = [W.batched_instance(rng, n, 60, n_drv=2000, n_wit=500, r_max=4.0) for n in (300, 1500)]
    _say("cluster split / batch")
    ref = wk.WakeSolver.from_instance(big, record_stride=20)
    assert ref.layout()[0] > 1
    ref.wake_solve(0, 60)
    f_ref = ref.wake_fields(40)
    st_ref = ref.wake_get_state()
    lp_ref, le_ref = ref.wake_lineout()
    ref.close()
    s = wk.WakeSolver.from_instance(big, record_stride=20)
    for a, b in ((0, 7), (7, 30), (37, 23)):
        s.wake_solve(a, b)
    g = s.wake_fields(40)
    for q in FIELDS:
        assert np.array_equal(g[q], f_ref[q]), q
    assert np.array_equal(s.wake_get_state()["rho"], st_ref["rho"])
    s.close()
    solvers = [wk.WakeSolver.from_instance(i, record_stride=20) for i in [big] + small]
    assert solvers[1].layout()[0] == 1
    b = wk.WakeBatch(solvers)
    b.wake_batch_solve(25)
    b.wake_batch_solve(-1)
    b.wake_batch_sync()
    g = solvers[0].wake_fields(40)
    for q in FIELDS:
        assert np.array_equal(g[q], f_ref[q]), q
    lp, le = solvers[0].wake_lineout()
    assert np.array_equal(lp, lp_ref) and np.array_equal(le, le_ref)
    b.close()
    for x in solvers:
        x.close()


def test_cluster_multi_round_fixups_match_split_launches(wk):
    """A 9000-ring instance whose order fix-ups at some slices take more than
    one block round (rings that return to their own chunk after a later
    round must get their own sums back): the one-launch march is bitwise the
    march split into launches of four slices, whose prologues order from
    scratch."""
    wk.wake_set_tiling(512, 0)
    wk.wake_set_cluster(0, 0)
    rng = np.random.default_rng(61)
    sizes = [(300, 90), (1500, 60), (777, 130), (64, 40), (2100, 75), (9000, 30)]
    inst = [W.batched_instance(rng, n, n_xi, n_drv=2500, n_wit=800, r_max=4.0) for n, n_xi in sizes][-1]
    _say("cooperative multi-round fix-ups, 9000 rings")
    a = wk.WakeSolver.from_instance(inst, record_stride=1)
    assert a.layout()[0] == 3
    a.wake_solve(0, inst.n_xi)
    b = wk.WakeSolver.from_instance(inst, record_stride=1)
    for n in range(0, inst.n_xi, 4):
        b.wake_solve(n, min(4, inst.n_xi - n))
    for n in range(inst.n_xi):
        fa, fb = a.wake_fields(n), b.wake_fields(n)
        for q in FIELDS + ("rho",):
            assert np.array_equal(fa[q], fb[q]), (n, q)
    a.close()
    b.close()


def test_cluster_members_wait_for_busy_workgroups(wk):
    """A batch launched on fewer workgroups than it has tasks: an instance's
    first member starts while the rest of its members still wait for
    workgroups busy with an earlier instance, and waits for them (the wait
    bound counts from the last task taken).  Every instance ends bitwise as
    when solved alone."""
    wk.wake_set_tiling(256, 0)
    wk.wake_set_cluster(2, 500)
    insts = [W.small_instance(seed, n_rings=3000, n_xi=30, n_peak=3.0, sigma_r=0.2, geometric=False,
                              dxi=0.02) for seed in (5, 6, 7)]
    rng = np.random.default_rng(48)
    insts += [W.batched_instance(rng, n, 30, n_drv=2000, n_wit=500, r_max=4.0) for n in (300, 450)]
    _say("cluster batch on a 7-workgroup grid")
    alone = []
    for inst in insts:
        s = wk.WakeSolver.from_instance(inst, record_stride=10)
        s.wake_solve(0, inst.n_xi)
        alone.append(([s.wake_fields(n) for n in (10, 20)], s.wake_lineout(), s.wake_get_state()["rho"]))
        s.close()
    solvers = [wk.WakeSolver.from_instance(inst, record_stride=10) for inst in insts]
    assert [s.layout()[0] for s in solvers] == [6, 6, 6, 1, 1]
    b = wk.WakeBatch(solvers)
    b.wake_batch_capture(7)
    b.wake_batch_replay()
    b.wake_batch_sync()
    for s, (fields, (lp, le), rho) in zip(solvers, alone):
        assert s.wake_status()[0] == -1
        for n, f in zip((10, 20), fields):
            g = s.wake_fields(n)
            for q in FIELDS:
                assert np.array_equal(g[q], f[q]), (n, q)
        glp, gle = s.wake_lineout()
        assert np.array_equal(glp, lp) and np.array_equal(gle, le)
        assert np.array_equal(s.wake_get_state()["rho"], rho)
    b.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("u_amp", [0.5, 40.0])
def test_cluster_fixups_in_device_memory(wk, u_amp):
    """Members whose keys exceed the LDS area (512-thread workgroups, sixteen
    rings per thread: 8192 positions per member) fix their order in device
    memory: member-local rounds, rounds over all members and the bitonic
    network, after pushes that move rings a few to thousands of places.  The
    slice after the push against the oracle's on the device's pushed state."""
    rng = np.random.default_rng(37)
    inst = W.small_instance(8, n_rings=17000, n_xi=20, n_peak=3.0, sigma_r=0.2, geometric=False, dxi=0.02)
    o = _oracle(inst)
    state = o.initial_state()
    state["u"] = rng.normal(0, u_amp, inst.n_rings)
    n = 8
    _, mid = o.slice(n, state, keep=True)
    wk.wake_set_tiling(512, 0)
    wk.wake_set_cluster(16, 500)
    label = f"cluster fix-ups in device memory u_amp={u_amp}"
    _say(label)
    st, mid_dev = pushed_by_device(wk, inst, n, state)
    check_state(st, mid, label)
    ref, _ = o.slice(n + 1, mid_dev, keep=True)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    assert s.layout() == (3, 16)
    s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
    s.wake_solve(n, 2)
    got = s.wake_fields(n + 1)
    check_fields(got, ref, field_scales(ref), label)
    assert np.array_equal(got["rho"], mid_dev["rho"])
    s.close()
