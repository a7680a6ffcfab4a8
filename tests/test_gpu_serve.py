"""Served form and chunked marching: results do not depend on the mix.

A solve split over several launches must be bitwise the one-launch solve
(the march restarts from the stored state and rebuilds its sums in the same
order), so a request served in a mix of others, stepped a few slices at a
time, returns exactly what solving it alone returns.
"""
import numpy as np
import pytest

from paper_2603_16623_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("psi", "er_bt", "ez", "bt", "rho", "ur")


@pytest.fixture(scope="module")
def wk():
    from paper_2603_16623_amd import wake
    wake.load()
    wake.wake_set_tiling(512, 0)
    yield wake
    wake.wake_set_tiling(512, 0)


def _say(*a):
    print(*a, flush=True)


def _alone(wk, inst):
    s = wk.WakeSolver.from_instance(inst)
    s.wake_solve(0, inst.n_xi)
    out = dict(s.wake_fields(-1))
    out["psi_axis"], out["ez_axis"] = s.wake_lineout()
    s.close()
    return out


def _mix(seed, sizes):
    rng = np.random.default_rng(seed)
    return [W.batched_instance(rng, n, n_xi, n_drv=2500, n_wit=800, r_max=4.0) for n, n_xi in sizes]


def test_chunked_solve_is_bitwise_one_solve(wk):
    # 9000 rings: keys beyond LDS (global order fix-up); 700: LDS permutation path
    for n, n_xi in ((700, 140), (9000, 60)):
        inst = _mix(51 + n, [(n, n_xi)])[0]
        _say("chunked", n)
        ref = _alone(wk, inst)
        s = wk.WakeSolver.from_instance(inst)
        cuts = sorted({0, 7, 8, 31, n_xi // 2, n_xi})
        for a, b in zip(cuts[:-1], cuts[1:]):
            s.wake_solve(a, b - a)
        got = s.wake_fields(-1)
        lp, le = s.wake_lineout()
        for q in FIELDS:
            assert np.array_equal(got[q], ref[q]), (n, q)
        assert np.array_equal(lp, ref["psi_axis"]) and np.array_equal(le, ref["ez_axis"]), n
        s.close()


@pytest.mark.parametrize("budget,step_us", [(0, 0), (40_000, 0), (0, 300)])
def test_served_results_equal_alone(wk, budget, step_us):
    """Fixed slices per step, a work budget per step, and time-sliced steps
    (chunk lengths then depend on timing) all give the alone results."""
    sizes = [(300, 90), (1500, 60), (777, 130), (64, 40), (2100, 75), (9000, 30), (1200, 110)]
    insts = _mix(61, sizes)
    _say("served mix, work budget per step", budget, "step us", step_us)
    ref = [_alone(wk, inst) for inst in insts]
    srv = wk.WakeServer(device_bytes=8 << 30, slices_per_step=17 if step_us == 0 else 100000,
                        ring_slices_per_step=budget, step_us=step_us)
    tickets = {}
    # requests arrive while others are resident
    for i in range(3):
        tickets[srv.submit_instance(insts[i])] = i
    results = {}
    pending = list(range(3, len(insts)))
    steps = 0
    while len(results) < len(insts):
        if pending and steps % 2 == 1:
            i = pending.pop(0)
            tickets[srv.submit_instance(insts[i])] = i
        srv.step()
        steps += 1
        assert steps < 5000
        for t, i in list(tickets.items()):
            r = srv.result(t)
            if r is not None:
                results[i] = r
                del tickets[t]
    for i, r in results.items():
        assert r["status"] == 0, i
        for q in FIELDS:
            assert np.array_equal(r[q], ref[i][q]), (i, q)
        assert np.array_equal(r["psi_axis"], ref[i]["psi_axis"]), i
        assert np.array_equal(r["ez_axis"], ref[i]["ez_axis"]), i
    st = srv.stats()
    assert st["active"] == 0 and st["queued"] == 0 and st["bytes_in_use"] == 0
    assert st["ring_slices"] == sum(i.ring_slices for i in insts)
    assert srv.ready() == []
    srv.close()


def test_served_admission_respects_the_footprint_budget(wk):
    sizes = [(1000, 50), (1400, 40), (900, 60), (1100, 30), (1300, 45)]
    insts = _mix(71, sizes)
    fps = [wk.wake_footprint(i.n_rings, i.n_xi, sum(len(s.x) for s in i.sources)) for i in insts]
    budget = max(fps) + min(fps)          # never more than two resident at once
    _say("admission budget", budget)
    srv = wk.WakeServer(device_bytes=budget, slices_per_step=20)
    tickets = [srv.submit_instance(i) for i in insts]
    done = 0
    steps = 0
    while done < len(insts):
        srv.step()
        steps += 1
        st = srv.stats()
        assert st["bytes_in_use"] <= budget
        assert st["active"] <= 2
        for t in tickets:
            if t in srv.meta:
                r = srv.result(t)
                if r is not None:
                    assert r["status"] == 0
                    done += 1
        assert steps < 200
    srv.close()


def test_breakdown_in_a_served_mix(wk):
    """One request whose beam drives psibar below zero (a wide, dense
    positively charged driver pulling the electrons in) is served among
    others: it comes back WAKE_EBREAKDOWN at the oracle's breakdown slice
    with its lineout up to there as alone, and every other result is
    bitwise its result alone."""
    from oracle.wake_oracle import RingOracle
    r0, dr = W.geometric_rings(400, 2e-3, 4.0)
    bad = W.Instance("breakdown-400x150", r0, dr, 0.02, 150, [W.GaussianBeam(+1.0, 20.0, 1.5, 0.5, 1.5)])
    want = RingOracle(bad.r0, bad.dr, bad.dxi, bad.n_xi, bad.sources).run(record_stride=0)["breakdown"]
    assert want == 91
    insts = _mix(62, [(300, 90), (1500, 60), (777, 130), (2100, 75)])
    insts.insert(2, bad)
    _say("served mix with a breakdown")
    ref = [_alone(wk, inst) if inst is not bad else None for inst in insts]
    alone = wk.WakeSolver.from_instance(bad)
    alone.wake_solve(0, bad.n_xi)
    assert alone.wake_status()[0] == want
    bad_psi, bad_ez = alone.wake_lineout()
    alone.close()
    srv = wk.WakeServer(device_bytes=8 << 30, slices_per_step=23)
    tickets = {srv.submit_instance(inst): i for i, inst in enumerate(insts)}
    results = {}
    steps = 0
    while len(results) < len(insts):
        srv.step()
        steps += 1
        assert steps < 5000
        for t, i in list(tickets.items()):
            r = srv.result(t)
            if r is not None:
                results[i] = r
                del tickets[t]
    for i, r in results.items():
        if insts[i] is bad:
            assert r["status"] == wk.WAKE_EBREAKDOWN and r["breakdown"] == want, (r["status"], r["breakdown"])
            assert np.array_equal(r["psi_axis"][:want], bad_psi[:want])
            assert np.array_equal(r["ez_axis"][:want], bad_ez[:want])
            continue
        assert r["status"] == 0, i
        for q in FIELDS:
            assert np.array_equal(r[q], ref[i][q]), (i, q)
        assert np.array_equal(r["psi_axis"], ref[i]["psi_axis"]), i
    st = srv.stats()
    assert st["active"] == 0 and st["queued"] == 0 and st["bytes_in_use"] == 0
    srv.close()
