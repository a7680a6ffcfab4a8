"""Pins of the oracle's accurate prefix sums and of the psi family at the
laser workload's 2e5 rings.

prefix_sum against exact rational sums of the same extended-precision terms
(heavy cancellation: terms of both signs about 1e3 times their running sum);
psi and d_rho psi at sampled rings of a perturbed 2e5-ring column against
sums in 40-digit arithmetic of the definitions (eqs. psi, dpsi_dr, with the
ions of reading R11 interpolated between their nodes).  A plain 80-bit
running sum (the planted mistake) misses the psi pin.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import wake_oracle as O
from paper_2603_16623_amd import workloads as W

LD = np.longdouble
mpmath.mp.dps = 40


def _exact_prefix(x):
    acc, out = Fraction(0), []
    for t in x:
        acc += Fraction(*t.as_integer_ratio())
        out.append(acc)
    return out


def test_prefix_sum_is_the_exact_sum_rounded():
    rng = np.random.default_rng(3)
    n = 5000
    x = (rng.normal(0.0, 1.0, n) * 1e3).astype(LD) * (LD(1) + LD(rng.random(n)) * LD(2.0) ** -60)
    x -= np.mean(x)                     # running sums far below the terms
    got = O.prefix_sum(x).ld()
    ex = _exact_prefix(x)
    ulp = float(np.finfo(LD).eps)
    worst = max(abs(Fraction(*g.as_integer_ratio()) - e) / max(abs(e), Fraction(1, 10 ** 6))
                for g, e in zip(got, ex))
    assert worst <= 2 * ulp
    suf = O.suffix_sum(x).ld()
    exs = _exact_prefix(x[::-1])[::-1]
    assert max(abs(Fraction(*g.as_integer_ratio()) - e) for g, e in zip(suf, exs)) <= 1e-14
    # a plain 80-bit running sum is further off than the pin allows
    plain = np.cumsum(x)
    worst_plain = max(abs(Fraction(*g.as_integer_ratio()) - e) / max(abs(e), Fraction(1, 10 ** 6))
                      for g, e in zip(plain, ex))
    assert worst_plain > 10 * worst


@pytest.fixture(scope="module")
def laser_slice():
    inst = W.config5()
    rng = np.random.default_rng(3)
    N = inst.n_rings
    state = dict(rho=inst.r0 * (1.0 + 0.002 * rng.standard_normal(N)).clip(0.5, 1.5),
                 u=0.02 * rng.standard_normal(N), fr=0.02 * rng.standard_normal(N),
                 fu=0.02 * rng.standard_normal(N))
    o = O.RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens)
    return o, state


def _mp_psi(o, state, i, lnr, lnr0, Q):
    """psi and d_rho psi at ring i by the definitions, 40 digits: electrons
    -q sum_k w_k ln max(rho_i, rho_k) (ring i itself by w^ in the Gauss sum),
    ions interpolated linearly between their nodes (reading R11).  lnr,
    lnr0: 40-digit logs of the radii and initial radii."""
    mp = mpmath.mpf
    rho, w, wh, r0 = state["rho"], o.w, o.wh, o.r0
    ri = mp(rho[i])
    lri = lnr[i]
    psi_e = mpmath.fsum(mp(w[k]) * (lri if rho[k] < rho[i] or k == i else lnr[k])
                        for k in range(len(rho)))
    below = mpmath.fsum(mp(w[k]) for k in range(len(rho)) if rho[k] < rho[i])
    dpsi_e = (below + mp(wh[i])) / ri
    j = int(np.searchsorted(r0, rho[i], side="left"))     # ion nodes r0[:j] below rho_i

    def node(k):            # ion node k = ion ring k-1 (k >= 1)
        rk, lk = mp(r0[k - 1]), lnr0[k - 1]
        ps = -mpmath.fsum(mp(w[m]) * (lk if m <= k - 1 else lnr0[m]) for m in range(len(r0)))
        bl = mpmath.fsum(mp(w[m]) for m in range(k - 1))
        return rk, ps, -(bl + mp(wh[k - 1])) / rk
    assert 0 < j < len(r0)
    (ra, pa, da), (rb, pb, db) = node(j), node(j + 1)
    t = (ri - ra) / (rb - ra)
    return psi_e + (1 - t) * pa + t * pb, dpsi_e + (1 - t) * da + t * db


PICKS = [10, 60000, 199990]


def _psi_errors(o, state, mp_ref):
    ref, _ = o.slice(int(2.0 / o.dxi), state, push=False, keep=True)
    scale = max(float(np.max(np.abs(ref["psi"]))), abs(float(ref["psi_axis"])))
    out = []
    for i, (ps, dp) in zip(PICKS, mp_ref):
        out.append((abs(float(ps - mpmath.mpf(ref["psi"][i]))) / scale,
                    abs(float(dp + mpmath.mpf(ref["er_bt"][i]))) / abs(float(dp))))
    return out


@pytest.fixture(scope="module")
def mp_psi(laser_slice):
    o, state = laser_slice
    lnr = [mpmath.log(mpmath.mpf(x)) for x in state["rho"]]
    lnr0 = [mpmath.log(mpmath.mpf(x)) for x in o.r0]
    return [_mp_psi(o, state, i, lnr, lnr0, None) for i in PICKS]


def test_psi_at_200000_rings_matches_40_digit_sums(laser_slice, mp_psi):
    """psi within 1e-13 of its slice scale (a tenth of the parity norm),
    d_rho psi within 1e-14 relative."""
    for i, (ep, ed) in zip(PICKS, _psi_errors(*laser_slice, mp_psi)):
        assert ep <= 1e-13, (i, ep)
        assert ed <= 1e-14, (i, ed)


def test_planted_plain_running_sums_miss_the_psi_pin(laser_slice, mp_psi, monkeypatch):
    monkeypatch.setattr(O, "prefix_sum", lambda x: O.DD.of(np.cumsum(O.DD.of(x).ld())))
    errs = _psi_errors(*laser_slice, mp_psi)
    assert max(ep for ep, _ in errs) > 1e-12
