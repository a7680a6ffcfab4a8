"""GPU parity of the radial field grid (the ring solve's sums at the nodes
of a uniform cell-centred grid, every slice) against the oracle's
fields_at, through the C ABI.

Tolerances as for the ring fields (tests/parity.py): per slice and per
field, 1e-12 of that field's scale at the slice over the rings and the grid
nodes (B_theta's also takes B^(b) and the jumps C_i); end to end 1e-8 of each
quantity's largest magnitude.
"""
import numpy as np
import pytest

from oracle.wake_oracle import RingOracle, grid_radii
from paper_2603_16623_amd import workloads as W

pytestmark = pytest.mark.gpu

from parity import FIELDS, TOL_E2E, check_fields, field_scales, rel as _rel
WAKE_ESTATE = -4
WAKE_EINVAL = -1


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


def _check_slices(wk, inst, tiling, cluster, n_r, r_max, slices, layout=None):
    """Inject the oracle's state at each slice, march one slice, compare the
    grid fields with the oracle's fields at the same nodes."""
    o = _oracle(inst)
    wk.wake_set_tiling(*tiling)
    wk.wake_set_cluster(*cluster)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    if layout is not None:
        assert s.layout() == layout
    s.wake_set_grid(n_r, r_max)
    gr = grid_radii(n_r, r_max)
    assert np.array_equal(s.grid_radii(), gr)
    state = o.initial_state()
    at = 0
    for n in slices:
        for m in range(at, n):
            _, state = o.slice(m, state)
        at = n
        ref, _ = o.slice(n, state, keep=True)
        assert ref["status"] == 0
        want = o.fields_at(n, ref, gr)
        rho = np.sort(state["rho"])
        label = f"grid {inst.name} tiling={tiling} cluster={cluster} n_r={n_r} slice={n}"
        _say(f"grid slice {label} nodes inside first ring={int(np.sum(gr <= rho[0]))} "
             f"beyond last={int(np.sum(gr > rho[-1]))}")
        s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
        s.wake_solve(n, 1)
        got = s.wake_grid_fields(n)
        check_fields(got, ref, field_scales(ref, want), label, want=want)
        last = s.wake_grid_fields(-1)
        for q in FIELDS:
            assert np.array_equal(last[q], got[q])
    s.close()


def test_grid_slice_parity_small_tilings(wk):
    """300 geometric rings, 2 per thread (256) and one per thread with idle
    threads (512); nodes inside the first ring, between rings, beyond the
    last ring and beyond the plasma edge (r_max = 1.5 R_p)."""
    inst = W.small_instance(7, n_rings=300, n_xi=200, n_peak=4.0, sigma_r=0.1, dxi=0.01)
    for tiling in ((256, 0), (512, 0)):
        _check_slices(wk, inst, tiling, (0, 0), 97, 4.5, (0, 60, 130, 199))


def test_grid_slice_parity_laser_channel_fine_grid(wk):
    """700 rings in a parabolic channel with a laser; a grid finer than the
    rings near the axis (many nodes per interval) and coarser outside."""
    inst = W.small_instance(10, n_rings=700, n_xi=200, n_peak=1.0, laser=True, dxi=0.01,
                            channel_w0=2.0)
    _check_slices(wk, inst, (512, 0), (0, 0), 3000, 3.3, (0, 50, 120, 190))


def test_grid_slice_parity_blowout_cavity(wk):
    """A driver that clears the axis (150 uniform rings, peak density 60):
    up to ~120 nodes inside the first ring, all in interval 0 of one
    thread, no ring below them."""
    inst = W.small_instance(11, n_rings=150, n_xi=300, n_peak=60.0, sigma_r=0.1, geometric=False,
                            dxi=0.01)
    _check_slices(wk, inst, (256, 0), (0, 0), 400, 3.3, (150, 225, 290))


def test_grid_rings_exactly_at_nodes(wk):
    """An injected state whose radii are node radii (every third node, so
    the nodes between rings and on rings alternate): a ring exactly at a
    node counts as outside it on both sides."""
    wk.wake_set_tiling(256, 0)
    wk.wake_set_cluster(0, 0)
    inst = W.small_instance(13, n_rings=200, n_xi=40, n_peak=2.0, sigma_r=0.3, geometric=False,
                            dxi=0.02)
    o = _oracle(inst)
    n_r, r_max = 600, 3.0
    gr = grid_radii(n_r, r_max)
    rng = np.random.default_rng(8)
    state = o.initial_state()
    state["rho"] = gr[1::3][: inst.n_rings].copy()
    state["u"] = rng.normal(0.0, 0.05, inst.n_rings)
    n = 20
    ref, _ = o.slice(n, state, keep=True)
    want = o.fields_at(n, ref, gr)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    s.wake_set_grid(n_r, r_max)
    s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
    s.wake_solve(n, 1)
    got = s.wake_grid_fields(n)
    _say("grid rings at nodes")
    check_fields(got, ref, field_scales(ref, want), "grid rings at nodes", want=want)
    s.close()


def test_grid_slice_parity_unstaged_beam_table(wk):
    """A slice table longer than the LDS stage (20000 particles over a short
    beam): node charges searched in device memory."""
    rng = np.random.default_rng(5)
    r0, dr = W.uniform_rings(400, 2.0)
    p = W.gaussian_particles(rng, 20000, 1.0, 0.4, 0.05, 0.5)
    inst = W.Instance("dense-beam-400x60", r0, dr, 0.01, 60, [p])
    _check_slices(wk, inst, (512, 0), (0, 0), 160, 2.4, (45, 50, 55))


def test_grid_slice_parity_cooperative(wk):
    """A 3000-ring instance over six cooperative members (256 threads, two
    rings per thread): member boundaries inside the grid."""
    inst = W.small_instance(5, n_rings=3000, n_xi=60, n_peak=3.0, sigma_r=0.2, geometric=False,
                            dxi=0.02)
    _check_slices(wk, inst, (256, 0), (2, 500), 1201, 3.6, (0, 25, 50), layout=(6, 2))


def test_grid_linear_end_to_end(wk):
    """Linear driver, 1000 rings x 1200 slices, 64 nodes to r = 6 (beyond
    the plasma at r = 5): every slice's grid fields within 1e-8."""
    wk.wake_set_tiling(512, 0)
    inst = W.config1()
    _say("grid e2e linear 1000x1200")
    ref = _oracle(inst).run(record_stride=0, grid=(64, 6.0))
    s = wk.WakeSolver.from_instance(inst)
    s.wake_set_grid(64, 6.0)
    s.wake_solve(0, inst.n_xi)
    assert s.wake_status() == (-1, inst.n_xi)
    got = np.stack([[s.wake_grid_fields(n)[q] for q in FIELDS] for n in range(inst.n_xi)])
    for qi, q in enumerate(FIELDS):
        assert _rel(got[:, qi], ref["grid"][:, qi]) <= TOL_E2E, q
    s.close()


def test_grid_batched_equals_alone(wk):
    """Instances with and without grids in one persistent launch: the grid
    fields and the ring fields equal those of each instance marched alone."""
    wk.wake_set_tiling(512, 0)
    wk.wake_set_cluster(0, 0)
    rng = np.random.default_rng(45)
    insts = [W.batched_instance(rng, n, 90, n_drv=3000, n_wit=1000, r_max=4.0)
             for n in (300, 1500, 777)]
    grids = [(50, 4.5), None, (500, 2.0)]
    _say("grid batched vs alone")
    alone = []
    for inst, g in zip(insts, grids):
        s = wk.WakeSolver.from_instance(inst, record_stride=30)
        if g:
            s.wake_set_grid(*g)
        s.wake_solve(0, inst.n_xi)
        alone.append((s.wake_fields(60), [s.wake_grid_fields(n) for n in (0, 45, 89)] if g else None))
        s.close()
    solvers = []
    for inst, g in zip(insts, grids):
        s = wk.WakeSolver.from_instance(inst, record_stride=30)
        if g:
            s.wake_set_grid(*g)
        solvers.append(s)
    b = wk.WakeBatch(solvers)
    b.wake_batch_solve(40)
    b.wake_batch_solve(-1)
    b.wake_batch_sync()
    for s, g, (f, gf) in zip(solvers, grids, alone):
        got = s.wake_fields(60)
        for q in FIELDS:
            if g:
                assert np.array_equal(got[q], f[q]), q
            else:     # marched by the grid variant of the kernel here
                assert _rel(got[q], f[q]) <= 1e-13, q
        if g:
            for n, want in zip((0, 45, 89), gf):
                have = s.wake_grid_fields(n)
                for q in FIELDS:
                    assert np.array_equal(have[q], want[q]), (n, q)
    b.close()
    for s in solvers:
        s.close()


def test_grid_call_order_and_arguments(wk):
    wk.wake_set_tiling(512, 0)
    inst = W.small_instance(3, n_rings=100, n_xi=20)
    s = wk.WakeSolver.from_instance(inst)
    lib = wk.load()
    assert lib.wake_grid_fields(s.h, 0, None, None, None, None, 0) == WAKE_ESTATE   # no grid
    assert lib.wake_set_grid(s.h, -1, 1.0) == WAKE_EINVAL
    assert lib.wake_set_grid(s.h, 10, 0.0) == WAKE_EINVAL
    assert lib.wake_set_grid(s.h, 10, float("nan")) == WAKE_EINVAL
    assert lib.wake_set_grid(s.h, (1 << 20) + 1, 1.0) == WAKE_EINVAL
    s.wake_set_grid(10, 1.0)
    assert lib.wake_grid_fields(s.h, 0, None, None, None, None, 0) == WAKE_ESTATE   # not solved
    st = s.wake_get_state()
    s.wake_set_state(3, st["rho"], st["ur"])
    s.wake_solve(3, 2)
    assert lib.wake_grid_fields(s.h, 1, None, None, None, None, 0) == WAKE_ESTATE   # before the state
    assert np.all(np.isfinite(s.wake_grid_fields(4)["psi"]))
    s.close()
    s = wk.WakeSolver.from_instance(inst)
    s.wake_set_grid(10, 1.0)
    s.wake_solve(0, 5)
    s.wake_grid_fields(4)
    assert lib.wake_grid_fields(s.h, 5, None, None, None, None, 0) == WAKE_ESTATE
    assert lib.wake_grid_fields(s.h, 20, None, None, None, None, 0) == WAKE_EINVAL
    assert lib.wake_set_grid(s.h, 12, 1.0) == WAKE_ESTATE                         # after a solve
    s.close()
    s = wk.WakeSolver.from_instance(inst)
    b = wk.WakeBatch([s])
    assert lib.wake_set_grid(s.h, 12, 1.0) == WAKE_ESTATE                         # held by a batch
    b.close()
    s.wake_set_grid(12, 1.0)                                                      # released
    s.close()


def test_grid_graph_replays_match_eager(wk):
    """A captured batch with field grids: every replay (with eager work of
    the program in between) gives the eager solve's grid fields bitwise."""
    wk.wake_set_tiling(512, 0)
    wk.wake_set_cluster(0, 0)
    rng = np.random.default_rng(46)
    insts = [W.batched_instance(rng, n, 70, n_drv=2000, n_wit=500, r_max=4.0) for n in (250, 800)]
    grids = [(40, 2.0), (120, 4.5)]
    _say("grid graph replay")
    eager = []
    for inst, g in zip(insts, grids):
        s = wk.WakeSolver.from_instance(inst)
        s.wake_set_grid(*g)
        s.wake_solve(0, inst.n_xi)
        eager.append([s.wake_grid_fields(n) for n in (0, 35, 69)])
        s.close()
    solvers = []
    for inst, g in zip(insts, grids):
        s = wk.WakeSolver.from_instance(inst)
        s.wake_set_grid(*g)
        solvers.append(s)
    b = wk.WakeBatch(solvers)
    b.wake_batch_capture()
    for rep in range(3):
        b.wake_batch_replay()
        b.wake_batch_sync()
        for s, want in zip(solvers, eager):
            for n, w in zip((0, 35, 69), want):
                have = s.wake_grid_fields(n)
                for q in FIELDS:
                    assert np.array_equal(have[q], w[q]), (rep, n, q)
        x = wk.WakeSolver.from_instance(insts[0])
        x.wake_set_grid(16, 1.0)
        x.wake_solve(0, 10)
        x.wake_sync()
        x.close()
    b.close()
    for s in solvers:
        s.close()


def _hip_runtime():
    """The HIP runtime the library itself loaded (the same process-wide one)."""
    import ctypes
    with open("/proc/self/maps") as fh:
        paths = {ln.split()[-1] for ln in fh if "libamdhip64" in ln}
    assert paths, "HIP runtime not loaded"
    hip = ctypes.CDLL(sorted(paths)[0])
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    return hip


def test_device_destinations_match_host(wk):
    """Device destinations (wake_fields, wake_grid_fields, wake_lineout,
    wake_get_state with dst_is_device = 1, buffers from hipMalloc) receive
    what host destinations do, and a state injected from device sources
    marches like the same state from host arrays."""
    import ctypes
    wk.wake_set_tiling(512, 0)
    wk.wake_set_cluster(0, 0)
    inst = W.small_instance(14, n_rings=333, n_xi=50, n_peak=2.0)
    s = wk.WakeSolver.from_instance(inst, record_stride=10)
    s.wake_set_grid(77, 3.0)
    s.wake_solve(0, inst.n_xi)
    lib, hip = wk.load(), _hip_runtime()

    def through_device(call, count, n_out):
        bufs = []
        for _ in range(n_out):
            p = ctypes.c_void_p()
            assert hip.hipMalloc(ctypes.byref(p), 8 * count) == 0
            bufs.append(p)
        try:
            assert call(*[b.value for b in bufs]) == 0
            out = []
            for b in bufs:
                a = np.empty(count)
                assert hip.hipMemcpy(a.ctypes.data, b.value, 8 * count, 2) == 0   # device to host
                out.append(a)
            return out
        finally:
            for b in bufs:
                hip.hipFree(b.value)

    for n in (20, -1):
        host = s.wake_fields(n)
        dev = through_device(lambda *p: lib.wake_fields(s.h, n, *p, 1), inst.n_rings, 6)
        for k, a in zip(("psi", "er_bt", "ez", "bt", "rho", "ur"), dev):
            assert np.array_equal(a, host[k]), (n, k)
        ghost = s.wake_grid_fields(n)
        gdev = through_device(lambda *p: lib.wake_grid_fields(s.h, n, *p, 1), 77, 4)
        for k, a in zip(FIELDS, gdev):
            assert np.array_equal(a, ghost[k]), (n, k)
    lp, le = s.wake_lineout()
    dl = through_device(lambda *p: lib.wake_lineout(s.h, *p, 1), inst.n_xi, 2)
    assert np.array_equal(dl[0], lp) and np.array_equal(dl[1], le)
    st = s.wake_get_state()
    sl = wk._I()
    ds = through_device(lambda *p: lib.wake_get_state(s.h, ctypes.byref(sl), *p, 1), inst.n_rings, 4)
    assert sl.value == st["slice"]
    for k, a in zip(("rho", "ur", "f_rho", "f_u"), ds):
        assert np.array_equal(a, st[k]), k
    # an injected state from device sources marches like the same host state
    rng = np.random.default_rng(3)
    new = [st["rho"] * (1.0 + 0.01 * rng.standard_normal(inst.n_rings)).clip(0.9, 1.1),
           st["ur"], st["f_rho"], st["f_u"]]
    s.wake_set_state(30, *new)
    s.wake_solve(30, 5)
    want = s.wake_fields(-1)
    bufs = []
    for a in new:
        p = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(p), 8 * inst.n_rings) == 0
        assert hip.hipMemcpy(p.value, np.ascontiguousarray(a).ctypes.data, 8 * inst.n_rings, 1) == 0
        bufs.append(p)
    try:
        assert lib.wake_set_state(s.h, 30, *[b.value for b in bufs], 1) == 0
    finally:
        for b in bufs:
            hip.hipFree(b.value)
    s.wake_solve(30, 5)
    have = s.wake_fields(-1)
    for k in want:
        assert np.array_equal(have[k], want[k]), k
    s.close()
