"""GPU parity of the field grid at caller-given radii and at the beam
particles' own radii (wake_set_grid_radii, wake_set_grid_beam) against the
oracle's fields_at, through the C ABI.

Tolerances as for the ring fields (tests/parity.py): per slice and per
field, 1e-12 of that field's scale at the slice over the rings and the
nodes (B_theta's also takes B^(b) and the jumps C_i).
"""
import numpy as np
import pytest

from oracle.wake_oracle import RingOracle
from paper_2603_16623_amd import workloads as W
from parity import FIELDS, check_fields, field_scales

pytestmark = pytest.mark.gpu


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


def _radii(rng, n, inst, r_hi):
    """Log-uniform radii from inside the first ring to beyond the plasma edge,
    plus a few initial ring radii exactly, sorted and distinct."""
    r = np.exp(rng.uniform(np.log(inst.r0[0] * 0.1), np.log(r_hi), n))
    r = np.concatenate([r, inst.r0[rng.integers(0, inst.n_rings, 5)]])
    return np.unique(r)


def _march_and_check(wk, s, o, inst, slices, radii_of, label):
    state = o.initial_state()
    at = 0
    for n in slices:
        for m in range(at, n):
            _, state = o.slice(m, state)
        at = n
        ref, _ = o.slice(n, state, keep=True)
        assert ref["status"] == 0
        r = radii_of(n)
        assert np.array_equal(s.grid_nodes(n), r)
        s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
        s.wake_solve(n, 1)
        got = s.wake_grid_fields(n)
        if r.size == 0:
            assert all(got[q].size == 0 for q in FIELDS)
            continue
        want = o.fields_at(n, ref, r)
        check_fields(got, ref, field_scales(ref, want), f"{label} slice={n} nodes={r.size}", want=want)


@pytest.mark.parametrize("tiling,cluster,layout", [((256, 0), (0, 0), None), ((512, 0), (0, 0), None),
                                                   ((256, 0), (2, 500), (6, 2))])
def test_fixed_radii_slice_parity(wk, tiling, cluster, layout):
    """The same 300-odd radii every slice (inside the first ring, between
    rings, exactly at initial ring radii, beyond the plasma edge), one
    workgroup at two tilings and a six-member cooperative instance."""
    rng = np.random.default_rng(41)
    if layout is None:
        inst = W.small_instance(7, n_rings=300, n_xi=200, n_peak=4.0, sigma_r=0.1, dxi=0.01)
        slices = (0, 60, 130, 199)
    else:
        inst = W.small_instance(5, n_rings=3000, n_xi=60, n_peak=3.0, sigma_r=0.2, geometric=False,
                                dxi=0.02)
        slices = (0, 25, 50)
    wk.wake_set_tiling(*tiling)
    wk.wake_set_cluster(*cluster)
    radii = _radii(rng, 300, inst, 1.4 * (inst.r0[-1] + inst.dr[-1] / 2))
    o = _oracle(inst)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    if layout is not None:
        assert s.layout() == layout
    s.wake_set_grid_radii(radii)
    _say(f"fixed radii tiling={tiling} cluster={cluster} nodes={radii.size}")
    _march_and_check(wk, s, o, inst, slices, lambda n: radii, f"fixed radii {tiling}")
    s.close()
    wk.wake_set_cluster(0, 0)


def test_per_slice_radii_slice_parity(wk):
    """Every slice its own node set (0 to 400 radii, some repeated), the
    slices' fields at their own nodes."""
    wk.wake_set_tiling(512, 0)
    rng = np.random.default_rng(42)
    inst = W.small_instance(8, n_rings=257, n_xi=200, n_peak=1.0, laser=True, dxi=0.01)
    sets = []
    for n in range(inst.n_xi):
        k = int(rng.integers(0, 400)) if n % 7 else 0
        r = np.sort(np.exp(rng.uniform(np.log(1e-3), np.log(4.0), k)))
        if k > 3:
            r[1] = r[2]                                  # equal radii in one slice
        sets.append(r)
    off = np.concatenate([[0], np.cumsum([len(r) for r in sets])]).astype(np.int64)
    o = _oracle(inst)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    s.wake_set_grid_radii(np.concatenate(sets), off)
    _say(f"per-slice radii, {off[-1]} nodes")
    _march_and_check(wk, s, o, inst, (0, 14, 40, 99, 170), lambda n: sets[n], "per-slice radii")
    s.close()


def test_beam_particle_radii_slice_parity(wk):
    """Nodes at the beam particles' own radii: slice n's nodes are its
    beam-table entries (the particles depositing on that slice node, their
    radii from x, y), the same radii the oracle's beam table holds."""
    wk.wake_set_tiling(512, 0)
    inst = W.small_instance(9, n_rings=1200, n_xi=150, n_peak=3.0, sigma_r=0.2, dxi=0.01)
    o = _oracle(inst)
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    s.wake_set_grid_beam()
    t = o.table
    counts = [int(t.off[n + 1] - t.off[n]) for n in range(inst.n_xi)]
    _say(f"beam radii: {sum(counts)} entries, up to {max(counts)} per slice")
    for n in (0, 50, 70, 120):
        got = s.grid_nodes(n)
        want = np.asarray(t.r[t.off[n]:t.off[n + 1]], np.float64)
        assert got.size == want.size
        assert np.max(np.abs(got - want), initial=0.0) <= 1e-15 * max(1.0, float(np.max(want, initial=0.0)))
    _march_and_check(wk, s, o, inst, (50, 70, 120), lambda n: s.grid_nodes(n), "beam radii")
    s.close()


def test_probe_grids_batched_equal_alone_and_refusals(wk):
    """Fixed, per-slice and beam-radius grids marched in one batch are
    bitwise as alone; malformed node sets are refused."""
    wk.wake_set_tiling(512, 0)
    rng = np.random.default_rng(43)
    insts = [W.small_instance(7, n_rings=300, n_xi=80, n_peak=4.0, sigma_r=0.1, dxi=0.02),
             W.small_instance(8, n_rings=257, n_xi=90, n_peak=1.0, laser=True, dxi=0.02),
             W.small_instance(9, n_rings=700, n_xi=70, n_peak=3.0, sigma_r=0.2, dxi=0.02)]
    fixed = _radii(rng, 100, insts[0], 4.0)
    sets = [np.sort(rng.uniform(0.01, 3.0, int(rng.integers(0, 50)))) for _ in range(insts[1].n_xi)]
    off = np.concatenate([[0], np.cumsum([len(r) for r in sets])]).astype(np.int64)

    def make():
        ss = [wk.WakeSolver.from_instance(i, record_stride=0) for i in insts]
        ss[0].wake_set_grid_radii(fixed)
        ss[1].wake_set_grid_radii(np.concatenate(sets), off)
        ss[2].wake_set_grid_beam()
        return ss

    alone = make()
    for s, i in zip(alone, insts):
        s.wake_solve(0, i.n_xi)
    together = make()
    b = wk.WakeBatch(together)
    b.wake_batch_solve(-1)
    b.wake_batch_sync()
    _say("probe grids batched")
    for a, t, i in zip(alone, together, insts):
        for n in range(0, i.n_xi, 9):
            fa, ft = a.wake_grid_fields(n), t.wake_grid_fields(n)
            for q in FIELDS:
                assert np.array_equal(fa[q], ft[q]), (i.name, n, q)
    b.close()
    for s in alone + together:
        s.close()
    s = wk.WakeSolver.from_instance(insts[0])
    bad = [(np.array([0.5, 0.4]), None), (np.array([0.0, 0.4]), None), (np.array([np.nan]), None),
           (np.array([0.5, 0.4]), np.array([0] + [0] * (insts[0].n_xi - 1) + [2], np.int64)),
           (np.array([0.5, 0.6]), np.array([0] + [1] * insts[0].n_xi, np.int64))]
    for r, o in bad:
        with pytest.raises(wk.WakeError) as e:
            s.wake_set_grid_radii(r, o)
        assert e.value.code == wk.WAKE_EINVAL
    s.wake_solve(0, 5)
    with pytest.raises(wk.WakeError) as e:
        s.wake_set_grid_radii(fixed)
    assert e.value.code == wk.WAKE_ESTATE
    s.close()
    r0, dr = W.uniform_rings(100, 2.0)
    nob = wk.WakeSolver(r0, dr, 0.02, 20, [W.GaussianBeam(-1.0, 1.0, 0.2, 0.3, 0.5)])
    with pytest.raises(wk.WakeError) as e:
        nob.wake_set_grid_beam()                          # no particles, no table entries
    assert e.value.code == wk.WAKE_EINVAL
    nob.close()
