"""GPU parity of the two-species (mobile ion) path against the two-species
oracle (oracle/mobile_ions.py), through the C ABI.

Per-slice cases set the identical state of both species at slice n on both
sides and compare the fields of both species at n (per field, 1e-12 of the
field's scale at that slice, tests/parity.py; psi, E_r - B_theta and E_z are
one field sampled at the rings of either species, so their scale is taken
over both species' rings and the axis; B_theta's also takes the terms the
electrons' B^(p) is assembled from, which the ions receive interpolated),
psi(0) and E_z(0), and both species' state pushed to n+1.  End-to-end cases
compare whole linear-regime marches to 1e-8 of each quantity's largest
magnitude.
"""
import numpy as np
import pytest

from oracle.mobile_ions import TwoSpeciesOracle
from oracle.wake_oracle import RingOracle
from paper_2603_16623_amd import workloads as W
from parity import FIELDS, TOL_E2E, TOL_SLICE, check_fields, field_scales, rel, say, tol_of

pytestmark = pytest.mark.gpu

ION = "ion_"


@pytest.fixture(scope="module")
def wk():
    from paper_2603_16623_amd import wake
    wake.load()
    return wake


def _oracle(inst, m_i):
    return TwoSpeciesOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, m_i, inst.sources, inst.dens)


def _solver(wk, inst, m_i, stride=1):
    return wk.WakeSolver(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens,
                         record_stride=stride, ion_mass=m_i)


def _advance(o, state, n0, n1):
    for n in range(n0, n1):
        _, state = o.slice(n, state)
        assert state is not None
    return state


def scales2(ref):
    """Per-field scales of one two-species oracle slice (keep=True)."""
    def m(x):
        x = np.asarray(x)
        return float(np.max(np.abs(x))) if x.size else 0.0
    s = field_scales(ref)
    for q in FIELDS:
        s[q] = max(s[q], m(ref[ION + q]))
    return s


def _ion_view(d):
    return {q: d[ION + q] for q in FIELDS}


def _set_both(s, n, state):
    for sp, key in ((0, "e"), (1, "i")):
        st = state[key]
        s.wake_set_species_state(sp, n, st["rho"], st["u"], st["fr"], st["fu"])


def _check_slice(s, n, ref, new, label):
    sc = scales2(ref)
    ge = s.wake_species_fields(0, n)
    gi = s.wake_species_fields(1, n)
    check_fields(ge, ref, sc, label + " electrons")
    check_fields(gi, None, sc, label + " ions", want=_ion_view(ref))
    assert np.array_equal(ge["rho"], ref["rho"]) and np.array_equal(gi["rho"], ref[ION + "rho"])
    lp, le = s.wake_lineout()
    ep = abs(lp[n] - ref["psi_axis"]) / tol_of(sc["psi"])
    ee = abs(le[n] - ref["ez_axis"]) / tol_of(sc["ez"])
    assert ep <= 1.0 and ee <= 1.0, (label, "axis", ep, ee)
    if new is not None:
        for sp, key in ((0, "e"), (1, "i")):
            st = s.wake_get_species_state(sp)
            assert st["slice"] == n + 1
            for a, b in (("rho", "rho"), ("ur", "u"), ("f_rho", "fr"), ("f_u", "fu")):
                r = rel(st[a], new[key][b])
                assert r <= TOL_SLICE, (label, key, a, r)


def _case(name):
    if name == "blowout-300":
        return W.small_instance(7, n_rings=300, n_xi=200, n_peak=4.0, sigma_r=0.1, dxi=0.01)
    if name == "strong-300":
        return W.small_instance(12, n_rings=300, n_xi=300, n_peak=20.0, sigma_r=0.3, dxi=0.01)
    if name == "laser-257":
        return W.small_instance(8, n_rings=257, n_xi=200, n_peak=1.0, laser=True, dxi=0.01)
    if name == "channel-700":
        return W.small_instance(10, n_rings=700, n_xi=200, n_peak=1.0, laser=True, dxi=0.01,
                                channel_w0=2.0)
    if name == "multitile-2500":
        return W.small_instance(9, n_rings=2500, n_xi=150, n_peak=3.0, sigma_r=0.2, dxi=0.01,
                                geometric=False)
    if name == "max-8192":
        return W.small_instance(11, n_rings=8192, n_xi=60, n_peak=2.0, sigma_r=0.2, dxi=0.02,
                                geometric=False)
    raise KeyError(name)


# (case, ion mass in electron masses, slices): hydrogen, light ions, equal
# masses (the ions move as far as the electrons), a ragged multi-ring tile
# (3 rings per thread) and the largest size (8 rings per thread)
SLICE_CASES = [
    ("blowout-300", 1836.0, (0, 1, 60, 130, 199)),
    ("blowout-300", 1.0, (0, 60, 130, 199)),
    ("strong-300", 1.0, (80, 160, 290)),
    ("strong-300", 4.0, (100, 250)),
    ("laser-257", 25.0, (0, 40, 100, 170)),
    ("channel-700", 100.0, (0, 120, 190)),
    ("multitile-2500", 100.0, (0, 70, 140)),
    ("max-8192", 1836.0, (0, 30)),
]


@pytest.mark.parametrize("case,m_i,slices", SLICE_CASES)
def test_two_species_slice_parity_on_identical_state(wk, case, m_i, slices):
    inst = _case(case)
    o = _oracle(inst, m_i)
    s = _solver(wk, inst, m_i)
    state = o.initial_state()
    at = 0
    for n in slices:
        state = _advance(o, state, at, n)
        at = n
        ref, new = o.slice(n, state, push=n < inst.n_xi - 1, keep=True)
        assert ref["status"] == 0
        label = f"{case} m_i={m_i} slice={n} N={inst.n_rings}"
        say(f"two-species slice parity {label}")
        _set_both(s, n, state)
        s.wake_solve(n, 1)
        _check_slice(s, n, ref, new, label)
    s.close()


def test_two_species_crossed_states_are_sorted_first(wk):
    """Randomly crossed rings of both species (the bitonic order path)."""
    rng = np.random.default_rng(31)
    inst = W.small_instance(3, n_rings=1500, n_xi=50, n_peak=2.0, geometric=False)
    o = _oracle(inst, 9.0)
    state = o.initial_state()
    for key in ("e", "i"):
        state[key]["rho"] = inst.r0 * np.exp(rng.normal(0, 0.2, inst.n_rings))
        state[key]["u"] = rng.normal(0, 0.1, inst.n_rings)
        state[key]["fr"] = rng.normal(0, 0.1, inst.n_rings)
        state[key]["fu"] = rng.normal(0, 0.1, inst.n_rings)
    ref, new = o.slice(20, state, keep=True)
    assert ref["status"] == 0
    say("two-species crossed state")
    s = _solver(wk, inst, 9.0)
    _set_both(s, 20, state)
    s.wake_solve(20, 1)
    _check_slice(s, 20, ref, new, "crossed")
    assert s.wake_counters()["fixups"] >= 2          # both species were re-sorted
    s.close()


@pytest.mark.parametrize("m_i", [1836.0, 1.0])
def test_two_species_linear_end_to_end(wk, m_i):
    """Linear-regime driver (1000 rings x 1200 slices, 10^4 particles),
    hydrogen ions and equal masses: lineout, snapshots of both species every
    100 slices and the last slice to 1e-8."""
    inst = W.config1()
    say(f"two-species e2e linear m_i={m_i}")
    ref = _oracle(inst, m_i).run(record_stride=100)
    assert ref["breakdown"] == -1
    s = _solver(wk, inst, m_i, stride=100)
    s.wake_solve(0, inst.n_xi)
    assert s.wake_status() == (-1, inst.n_xi)
    lp, le = s.wake_lineout()
    assert rel(lp, ref["axis"][:, 0]) <= TOL_E2E
    assert rel(le, ref["axis"][:, 1]) <= TOL_E2E
    worst = {}
    for n in list(range(0, inst.n_xi, 100)) + [inst.n_xi - 1]:
        for sp, pre in ((0, ""), (1, ION)):
            got = s.wake_species_fields(sp, n if n % 100 == 0 else -1)
            want = ref["snap"][n]
            for q, wq in [(q, pre + q) for q in FIELDS + ("rho",)] + [("ur", pre + "u")]:
                r = rel(got[q], want[wq])
                worst[wq] = max(worst.get(wq, 0.0), r)
                assert r <= TOL_E2E, (n, sp, q, r)
    say("  worst e2e rel: " + " ".join(f"{k}={v:.2g}" for k, v in sorted(worst.items())))
    s.close()


def test_heavy_ions_match_the_immobile_ion_path(wk):
    """m_i = 1e30: the ions never move, and the electrons' fields agree with
    the one-species (immobile ion) kernels on the same state, slice by slice
    (two independent GPU paths), per field to 1e-12 of the scale."""
    inst = W.small_instance(7, n_rings=300, n_xi=200, n_peak=4.0, sigma_r=0.1, dxi=0.01)
    say("heavy ions vs the one-species path")
    o = RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources)
    two = _solver(wk, inst, 1e30)
    one = wk.WakeSolver.from_instance(inst, record_stride=1)
    state = o.initial_state()
    at = 0
    for n in (0, 50, 120, 190):
        state = _advance(o, state, at, n)
        at = n
        ref, _ = o.slice(n, state, keep=True)
        sc = field_scales(ref)
        one.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
        one.wake_solve(n, 1)
        two.wake_set_species_state(0, n, state["rho"], state["u"], state["fr"], state["fu"])
        two.wake_set_species_state(1, n, inst.r0, np.zeros(inst.n_rings))
        two.wake_solve(n, 1)
        a, b = one.wake_fields(n), two.wake_species_fields(0, n)
        check_fields(b, ref, sc, f"heavy ions slice={n} (vs oracle)")
        check_fields(b, ref, sc, f"heavy ions slice={n} (vs one-species path)", want=a)
        ions = two.wake_get_species_state(1)
        assert np.array_equal(ions["rho"], inst.r0)
    # a whole march: the ions stay exactly at rest
    two.wake_reset()
    two.wake_solve(0, inst.n_xi)
    ions = two.wake_get_species_state(1)
    assert np.array_equal(ions["rho"], inst.r0)
    assert float(np.max(np.abs(ions["ur"]))) < 1e-25
    one.close()
    two.close()


@pytest.mark.parametrize("which,m_i", [("e", 1836.0), ("i", 1.0)])
def test_two_species_breakdown_at_the_same_slice(wk, which, m_i):
    """A compressed electron column (psibar_e <= 0) or compressed light ions
    (psibar_i = 1 - psi/m_i <= 0) break down at the slice the oracle does;
    the state of that slice stays."""
    inst = W.small_instance(4, n_rings=200, n_xi=30, n_peak=1.0)
    o = _oracle(inst, m_i)
    state = o.initial_state()
    state[which]["rho"] = 0.5 * inst.r0
    ref, _ = o.slice(5, state)
    assert ref["status"] == -5
    say(f"two-species breakdown {which}")
    s = _solver(wk, inst, m_i)
    _set_both(s, 5, state)
    s.wake_solve(5, 3)
    assert s.wake_status()[0] == 5
    with pytest.raises(wk.WakeError) as e:
        s.wake_species_fields(1, 5)
    assert e.value.code == wk.WAKE_EBREAKDOWN
    st = s.wake_get_species_state(0 if which == "e" else 1)
    assert st["slice"] == 5
    assert np.array_equal(st["rho"], state[which]["rho"])
    s.close()


def test_two_species_split_solves_and_reset_are_bitwise(wk):
    """Solving in pieces, and again after wake_reset, gives bitwise the
    fields and states of one whole solve; the counters count the slices."""
    inst = W.small_instance(7, n_rings=300, n_xi=200, n_peak=4.0, sigma_r=0.1, dxi=0.01)
    say("two-species split solves")
    a = _solver(wk, inst, 25.0, stride=50)
    a.wake_solve(0, inst.n_xi)
    b = _solver(wk, inst, 25.0, stride=50)
    for first, cnt in ((0, 1), (1, 49), (50, 77), (127, 73)):
        b.wake_solve(first, cnt)
    for sp in (0, 1):
        for n in (0, 50, 100, 150, -1):
            fa, fb = a.wake_species_fields(sp, n), b.wake_species_fields(sp, n)
            for k in fa:
                assert np.array_equal(fa[k], fb[k]), (sp, n, k)
        sa, sb = a.wake_get_species_state(sp), b.wake_get_species_state(sp)
        for k in ("rho", "ur", "f_rho", "f_u"):
            assert np.array_equal(sa[k], sb[k])
    assert a.wake_counters()["slices"] == inst.n_xi and b.wake_counters()["slices"] == inst.n_xi
    la = a.wake_lineout()
    a.wake_reset()
    a.wake_solve(0, inst.n_xi)
    lb = a.wake_lineout()
    assert np.array_equal(la[0], lb[0]) and np.array_equal(la[1], lb[1])
    a.close()
    b.close()


def test_two_species_refusals(wk):
    inst = W.small_instance(7, n_rings=300, n_xi=20, n_peak=4.0)
    say("two-species refusals")
    s = _solver(wk, inst, 1836.0)
    with pytest.raises(wk.WakeError) as e:
        s.wake_set_grid(64, 3.0)
    assert e.value.code == wk.WAKE_EINVAL
    with pytest.raises(wk.WakeError) as e:
        s.wake_species_fields(2, 0)
    assert e.value.code == wk.WAKE_EINVAL
    assert s.threads() == 1024 and s.layout() == (1, 1)
    one = wk.WakeSolver.from_instance(inst)
    with pytest.raises(wk.WakeError) as e:
        one.wake_species_fields(1, -1)
    assert e.value.code == wk.WAKE_EINVAL
    with pytest.raises(wk.WakeError) as e:
        one.wake_get_species_state(1)
    assert e.value.code == wk.WAKE_EINVAL
    one.close()
    for m in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(wk.WakeError) as e:
            _solver(wk, inst, m)
        assert e.value.code == wk.WAKE_EINVAL
    r0, dr = W.uniform_rings(8193, 5.0)
    with pytest.raises(wk.WakeError) as e:
        wk.WakeSolver(r0, dr, 0.01, 10, [], ion_mass=1836.0)
    assert e.value.code == wk.WAKE_EINVAL
    s.close()


def test_two_species_in_a_mixed_batch_and_graph_are_bitwise_alone(wk):
    """A batch of two-species contexts (several ion masses and sizes) and
    one-species contexts: every context's lineout, fields of both species
    and final state are bitwise those of solving it alone, from an eager
    batch solve in two pieces and from replays of the captured graph (with
    eager work between replays)."""
    say("two-species mixed batch")
    insts = [(W.small_instance(7, n_rings=300, n_xi=120, n_peak=4.0, sigma_r=0.1, dxi=0.01), 1836.0),
             (W.small_instance(12, n_rings=700, n_xi=90, n_peak=20.0, sigma_r=0.3, dxi=0.01), 1.0),
             (W.small_instance(8, n_rings=257, n_xi=100, n_peak=1.0, laser=True, dxi=0.01), 25.0),
             (W.small_instance(9, n_rings=2500, n_xi=60, n_peak=3.0, sigma_r=0.2, dxi=0.01,
                               geometric=False), 100.0),
             (W.small_instance(5, n_rings=400, n_xi=80, n_peak=2.0), None)]

    def make(inst, m):
        if m is None:
            return wk.WakeSolver.from_instance(inst, record_stride=20)
        return _solver(wk, inst, m, stride=20)

    def result(s, inst, m):
        out = {"lineout": s.wake_lineout()}
        for sp in ((0, 1) if m is not None else (0,)):
            for n in range(0, inst.n_xi, 20):
                out[(sp, n)] = s.wake_species_fields(sp, n)
            out[(sp, "state")] = s.wake_get_species_state(sp)
        return out

    def same(a, b):
        for k in a:
            if k == "lineout":
                assert all(np.array_equal(x, y) for x, y in zip(a[k], b[k]))
            else:
                for q in a[k]:
                    assert np.array_equal(np.asarray(a[k][q]), np.asarray(b[k][q])), (k, q)

    alone = []
    for inst, m in insts:
        s = make(inst, m)
        s.wake_solve(0, inst.n_xi)
        alone.append(result(s, inst, m))
        s.close()
    solvers = [make(inst, m) for inst, m in insts]
    b = wk.WakeBatch(solvers)
    b.wake_batch_solve(50)
    b.wake_batch_solve(-1)
    b.wake_batch_sync()
    for s, (inst, m), ref in zip(solvers, insts, alone):
        assert s.wake_status() == (-1, inst.n_xi)
        same(result(s, inst, m), ref)
    b.wake_batch_capture()
    for rep in range(3):
        b.wake_batch_replay()
        b.wake_batch_sync()
        for s, (inst, m), ref in zip(solvers, insts, alone):
            same(result(s, inst, m), ref)
        solvers[0].wake_reset()                      # eager work between replays
        solvers[0].wake_solve(0, 10)
        solvers[0].wake_sync()
    b.close()
    for s in solvers:
        s.close()
