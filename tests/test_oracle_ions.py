"""Pins of the two-species (mobile ion) oracle against facts from outside it.

* Heavy-ion limit: with m_i = 1e30 the ions stay at their initial radii and
  the electrons' fields are those of the one-species oracle over an
  immobile ion background (reading R11), slice by slice.
* Rest: without sources both species stay at rest and every field vanishes.
* Gather: psi, d_rho psi and d_zeta psi at the rings of each species are its
  own pairwise sums (40 digits, w^ for the ring itself) plus the other
  species' node values, themselves pairwise sums, interpolated linearly
  between its rings (Sec. "Key algorithmic adjustments"; reading R18).
* Mass and charge: in the linear regime the ions' displacement scales as
  1/m_i, and an electron driver pulls the ions toward the axis while it
  pushes the electrons out.  Planted mistakes (force without 1/m_i, ion
  charge sign flipped) fail these.
"""
import mpmath
import numpy as np
import pytest

from oracle import mobile_ions as MI
from oracle import wake_oracle as O
from paper_2603_16623_amd import workloads as W

mpmath.mp.dps = 40


def _blowout():
    return W.small_instance(7, n_rings=160, n_xi=160, n_peak=4.0, sigma_r=0.1, dxi=0.01)


def test_heavy_ions_reproduce_the_immobile_oracle():
    inst = _blowout()
    one = O.RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources)
    two = MI.TwoSpeciesOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, 1e30, inst.sources)
    s1, s2 = one.initial_state(), two.initial_state()
    worst = 0.0
    for n in range(150):
        a, s1 = one.slice(n, s1)
        b, s2 = two.slice(n, s2)
        assert a["status"] == 0 and b["status"] == 0
        if n % 10 == 0:
            for q in ("psi", "er_bt", "ez", "bt"):
                scale = max(float(np.max(np.abs(a[q]))), 1e-15)
                worst = max(worst, float(np.max(np.abs(a[q] - b[q]))) / scale)
            assert abs(a["psi_axis"] - b["psi_axis"]) <= 1e-14 * max(abs(a["psi_axis"]), 1e-15)
    assert worst <= 1e-13, worst
    assert np.array_equal(s2["i"]["rho"], inst.r0)          # ions never left their radii
    assert float(np.max(np.abs(s2["i"]["u"]))) < 1e-25
    assert float(np.max(np.abs(s1["rho"] - s2["e"]["rho"]))) <= 1e-13 * float(np.max(inst.r0))


def test_rest_state_without_sources():
    r0, dr = W.geometric_rings(120, 1e-3, 3.0)
    two = MI.TwoSpeciesOracle(r0, dr, 0.02, 20, 1836.0, [])
    st = two.initial_state()
    for n in range(20):
        out, st = two.slice(n, st)
        for q in ("psi", "er_bt", "ez", "bt", "ion_psi", "ion_er_bt", "ion_ez", "ion_bt"):
            assert float(np.max(np.abs(out[q]))) <= 1e-15, (n, q)
    for k in ("e", "i"):
        assert np.array_equal(st[k]["rho"], r0)
        assert float(np.max(np.abs(st[k]["u"]))) == 0.0


def _mp_own(rho, u, psibar, w, wh, q, i):
    """Own fields of a species at its ring i by the definitions (40 digits)."""
    mp = mpmath.mpf
    ri = mp(rho[i])
    n = len(rho)
    lnr = [mpmath.log(mp(x)) for x in rho]
    psi = -q * mpmath.fsum(mp(w[k]) * (mpmath.log(ri) if (rho[k], k) < (rho[i], i) or k == i else lnr[k])
                           for k in range(n))
    below = mpmath.fsum(mp(w[k]) for k in range(n) if (rho[k], k) < (rho[i], i))
    dpsi = -q * (below + mp(wh[i])) / ri
    c = [q * mp(u[k]) / (mp(rho[k]) * mp(psibar[k])) for k in range(n)]
    dz = mpmath.fsum(mp(w[k]) * c[k] for k in range(n) if (rho[k], k) > (rho[i], i)) + (mp(w[i]) - mp(wh[i])) * c[i]
    return psi, dpsi, dz


def _mp_nodes(rho, u, psibar, w, wh, dr, q):
    """Node radii and values of a species (reading R18), 40 digits."""
    mp = mpmath.mpf
    order = sorted(range(len(rho)), key=lambda k: (rho[k], k))
    rs, ps, ds, zs = [mp(0)], [], [mp(0)], []
    lnr = [mpmath.log(mp(x)) for x in rho]
    Q = mpmath.fsum(mp(x) for x in w)
    ps.append(-q * mpmath.fsum(mp(w[k]) * lnr[k] for k in range(len(rho))))
    zs.append(mpmath.fsum(mp(w[k]) * q * mp(u[k]) / (mp(rho[k]) * mp(psibar[k])) for k in range(len(rho))))
    for k in order:
        p, d, z = _mp_own(rho, u, psibar, w, wh, q, k)
        rs.append(mp(rho[k])); ps.append(p); ds.append(d); zs.append(z)
    last = order[-1]
    edge = mp(rho[last]) + mp(dr[last]) / 2
    rs.append(edge); ps.append(-q * Q * mpmath.log(edge)); ds.append(-q * Q / edge); zs.append(mp(0))
    return rs, ps, ds, zs


def _interp(rs, vals, x):
    j = max(k for k in range(len(rs)) if rs[k] < x)
    t = (x - rs[j]) / (rs[j + 1] - rs[j])
    return vals[j] + t * (vals[j + 1] - vals[j])


def test_fields_at_both_species_match_pairwise_sums_and_linear_gather():
    rng = np.random.default_rng(17)
    r0, dr = W.geometric_rings(36, 0.02, 2.0)
    two = MI.TwoSpeciesOracle(r0, dr, 0.01, 10, 50.0, [])
    st = two.initial_state()
    st["e"]["rho"] = r0 * np.exp(rng.normal(0, 0.15, len(r0)))
    st["e"]["u"] = rng.normal(0, 0.2, len(r0))
    st["i"]["rho"] = r0 * np.exp(rng.normal(0, 0.05, len(r0)))
    st["i"]["u"] = rng.normal(0, 0.02, len(r0))
    out, _ = two.slice(3, st, push=False, keep=True)
    assert out["status"] == 0
    w, wh = two.w, two.wh
    pb_e = np.empty(len(r0)); pb_e[out["order"]] = out["psibar"]
    pb_i = np.empty(len(r0)); pb_i[out["ion_order"]] = out["ion_psibar"]
    ne = _mp_nodes(st["e"]["rho"], st["e"]["u"], pb_e, w, wh, dr, -1.0)
    ni = _mp_nodes(st["i"]["rho"], st["i"]["u"], pb_i, w, wh, dr, +1.0)
    for key, own_st, pb, q, other, pre in (("e", st["e"], pb_e, -1.0, ni, ""), ("i", st["i"], pb_i, 1.0, ne, "ion_")):
        for k in (0, 5, 17, 35):
            p, d, z = _mp_own(own_st["rho"], own_st["u"], pb, w, wh, q, k)
            x = mpmath.mpf(own_st["rho"][k])
            p += _interp(other[0], other[1], x) if x < other[0][-1] else 0
            d += _interp(other[0], other[2], x)
            z += _interp(other[0], other[3], x)
            scale = max(float(np.max(np.abs(out[pre + "psi"]))), 1e-12)
            assert abs(float(p) - out[pre + "psi"][k]) <= 1e-13 * scale, (key, k)
            assert abs(float(-d) - out[pre + "er_bt"][k]) <= 1e-13 * float(np.max(np.abs(out[pre + "er_bt"]))), (key, k)
            assert abs(float(-z) - out[pre + "ez"][k]) <= 1e-12 * float(np.max(np.abs(out[pre + "ez"]))), (key, k)


def _linear(m_i):
    inst = W.config1(analytic=True, n_peak=1e-3)
    two = MI.TwoSpeciesOracle(inst.r0, inst.dr, inst.dxi, 400, m_i, inst.sources)
    st = two.initial_state()
    for n in range(300):
        out, st = two.slice(n, st)
    return inst, st


def test_ion_response_scales_with_inverse_mass_and_is_attractive():
    inst, a = _linear(100.0)
    _, b = _linear(400.0)
    da = a["i"]["rho"] - inst.r0
    db = b["i"]["rho"] - inst.r0
    k = int(np.argmax(np.abs(da)))
    assert abs(da[k] / db[k] - 4.0) < 0.05, da[k] / db[k]
    near = inst.r0 < 0.15
    assert np.all(a["i"]["rho"][near] <= inst.r0[near])      # ions drawn in
    assert np.max(a["e"]["rho"][near] - inst.r0[near]) > 0   # electrons pushed out


def test_planted_ion_mistakes_break_the_pins(monkeypatch):
    orig = MI.forces
    monkeypatch.setattr(MI, "forces", lambda u, pb, gm, dp, bt, da2, q, m: orig(u, pb, gm, dp, bt, da2, q, 1.0))
    inst, a = _linear(100.0)
    _, b = _linear(400.0)
    k = int(np.argmax(np.abs(a["i"]["rho"] - inst.r0)))
    assert abs((a["i"]["rho"][k] - inst.r0[k]) / (b["i"]["rho"][k] - inst.r0[k]) - 4.0) > 0.5
    monkeypatch.setattr(MI, "forces", lambda u, pb, gm, dp, bt, da2, q, m: orig(u, pb, gm, dp, bt, da2, -q if q > 0 else q, m))
    inst, a = _linear(100.0)
    near = inst.r0 < 0.15
    assert not np.all(a["i"]["rho"][near] <= inst.r0[near])
