"""Pins of two oracle steps that the paper leaves to the implementation.

Axis reflection (reading R9; the paper is silent on rings that reach the
axis).  A ring of negligible weight (density 1e-30 of the others) starts at
its own radius with an inward momentum while every other ring is at rest and
there are no sources.  Inside its initial radius no other ring and no ion
node of weight is below it, so it feels no field: it streams freely,
rho(xi) = |rho0 + u0 xi| and u_r changes sign at the axis, and second-order
Adams-Bashforth reproduces the straight line exactly when the step after the
crossing takes the reflected history.  A planted mistake (history not
negated, momentum not negated) fails it.

B^(p) solve (reading R15).  At the laser workload's 2e5 rings (geometric
spacing 1e-5 to 15, a seeded perturbed state), two steps of iterative
refinement reach the unknowns (a_i, b_i) that eight steps give to within an
ulp of their largest magnitude, the residual of the recursion computed in
80-bit arithmetic drops to the binary64 rounding of its terms, and the plain
binary64 LU does not reach the unknowns (a wrong-signed correction is
caught).  (B^(p) = a rho + b/rho cancels: there |a rho|
and |b/rho| are about 10^3 times |B^(p)|, so an ulp of a or b is a few 1e-13
of B^(p); both sides of a parity test carry binary64 unknowns.)
"""
import numpy as np
import pytest

from oracle import wake_oracle as O
from paper_2603_16623_amd import workloads as W


def _streaming_case():
    n, R = 50, 2.5
    r0, dr = W.uniform_rings(n, R)
    dens = np.ones(n)
    dens[0] = 1e-30                      # the test ring carries no charge to speak of
    dxi, n_xi = 0.004, 24
    o = O.RingOracle(r0, dr, dxi, n_xi, (), dens)
    st = o.initial_state()
    u0 = -0.5
    st["u"][0] = u0
    return o, st, r0[0], u0, dxi


def _march(o, st, n_slices):
    traj = []
    for n in range(n_slices):
        out, st = o.slice(n, st)
        assert out["status"] == 0
        traj.append((st["rho"][0], st["u"][0], st["fr"][0], st["fu"][0], st))
    return traj


def test_ring_streams_through_the_axis():
    o, st, rho0, u0, dxi = _streaming_case()
    traj = _march(o, st, 22)             # crossing at xi = 0.05; back at rho0 only at 0.1
    crossed = 0
    for k, (rho, u, fr, fu, s) in enumerate(traj):
        xi = (k + 1) * dxi
        line = rho0 + u0 * xi
        assert rho == pytest.approx(abs(line), abs=1e-15), (k, rho, line)
        want_u = u0 if line > 0 else -u0
        assert u == want_u, (k, u)
        assert fr == want_u, (k, fr)     # history d rho/d xi = u / psibar with psibar = 1
        assert abs(fu) < 1e-20
        crossed += line < 0
        # every other ring stays at rest at its initial radius
        assert np.array_equal(s["rho"][1:], o.r0[1:])
        assert np.max(np.abs(s["u"][1:])) < 1e-25
    assert crossed >= 8


def _no_history_flip(rho, u, fr, fu, fr_p, fu_p, dxi):
    rho_n = rho + dxi * (1.5 * fr - 0.5 * fr_p)
    u_n = u + dxi * (1.5 * fu - 0.5 * fu_p)
    neg = rho_n < 0
    rho_n[neg] = -rho_n[neg]
    u_n[neg] = -u_n[neg]
    return rho_n, u_n, np.array(fr), np.array(fu)


def _no_momentum_flip(rho, u, fr, fu, fr_p, fu_p, dxi):
    rho_n = rho + dxi * (1.5 * fr - 0.5 * fr_p)
    u_n = u + dxi * (1.5 * fu - 0.5 * fu_p)
    frs, fus = np.array(fr), np.array(fu)
    neg = rho_n < 0
    rho_n[neg] = -rho_n[neg]
    frs[neg] = -frs[neg]
    fus[neg] = -fus[neg]
    return rho_n, u_n, frs, fus


@pytest.mark.parametrize("mutant", [_no_history_flip, _no_momentum_flip],
                         ids=["history-not-negated", "momentum-not-negated"])
def test_planted_reflection_mistakes_break_free_streaming(monkeypatch, mutant):
    monkeypatch.setattr(O, "push_ab2", mutant)
    o, st, rho0, u0, dxi = _streaming_case()
    traj = _march(o, st, 22)
    err = max(abs(r - abs(rho0 + u0 * (k + 1) * dxi)) for k, (r, *_rest) in enumerate(traj))
    assert err > 1e-4


@pytest.fixture(scope="module")
def laser_system():
    inst = W.config5()
    rng = np.random.default_rng(3)
    N = inst.n_rings
    state = dict(rho=inst.r0 * (1.0 + 0.002 * rng.standard_normal(N)).clip(0.5, 1.5),
                 u=0.02 * rng.standard_normal(N), fr=0.02 * rng.standard_normal(N),
                 fu=0.02 * rng.standard_normal(N))
    o = O.RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens)
    ref, _ = o.slice(int(2.0 / inst.dxi), state, push=False, keep=True)
    assert ref["status"] == 0
    return ref


def _residual_scale(M, s, a, b):
    """max |residual| of the recursion (80-bit) over max |its terms|."""
    r = O._recursion_residual(M, s, a, b)
    terms = max(float(np.max(np.abs(s))), float(np.max(np.abs(a))), float(np.max(np.abs(b))))
    return float(np.max(np.abs(r))) / terms


def test_refined_recursion_solve_converges_at_200000_rings(laser_system):
    ref = laser_system
    M, s = ref["M"], ref["s"]
    sols = {k: O.solve_recursion(M, s, refine=k) for k in (0, 2, 8)}
    top = max(float(np.max(np.abs(sols[8][0]))), float(np.max(np.abs(sols[8][1]))))
    ulp = float(np.spacing(top))

    def dist(k):
        return max(float(np.max(np.abs(sols[k][0] - sols[8][0]))),
                   float(np.max(np.abs(sols[k][1] - sols[8][1])))) / ulp
    res = {k: _residual_scale(M, s, *sols[k]) for k in sols}
    print(f"(a, b) against eight refinements, in ulps of max|a, b| = {top:.3g}: refine=2 "
          f"{dist(2):.3g}, refine=0 {dist(0):.3g}; residuals {res[0]:.3e} {res[2]:.3e} {res[8]:.3e}")
    assert dist(2) <= 1.0
    assert dist(0) > 8.0
    assert res[2] <= 2.3e-16 and res[8] <= 2.3e-16


def _refine_wrong_sign(M, s, refine=2):
    ab, rhs = O._recursion_banded(M, s)
    z = O.solve_banded((2, 1), ab, rhs)
    a, b = z[0::2].copy(), z[1::2].copy()
    for _ in range(refine):
        r = O._recursion_residual(M, s, a, b)
        d = O.solve_banded((2, 1), ab, r.astype(np.float64))
        a, b = a - d[0::2], b - d[1::2]
    return a, b


def test_planted_refinement_mistake_breaks_the_pin(laser_system):
    ref = laser_system
    a8, b8 = O.solve_recursion(ref["M"], ref["s"], refine=8)
    a, b = _refine_wrong_sign(ref["M"], ref["s"])
    ulp = float(np.spacing(max(np.abs(a8).max(), np.abs(b8).max())))
    assert max(np.abs(a - a8).max(), np.abs(b - b8).max()) / ulp > 8.0
