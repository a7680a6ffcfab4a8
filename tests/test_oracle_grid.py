"""Pins of the oracle's fields at radii off the rings (the external field
grid of Fig. 2): brute-force pairwise sums, the jumps at a ring, the vacuum
field outside the plasma and the integrated Ampere law.  CPU only."""
import math

import mpmath
import numpy as np

from oracle import wake_oracle as O
from paper_2603_16623_amd import workloads as W

mp = mpmath.mpf


def _instance(channel_w0=None, laser=True, n_rings=60, dxi=0.004, n_xi=800, particles=True):
    r0, dr = W.geometric_rings(n_rings, 0.01, 3.0)
    src = [W.GaussianBeam(-1.0, 1.5, 0.3, 0.4, 1.2)]
    rng = np.random.default_rng(5)
    if particles:
        src.append(W.gaussian_particles(rng, 2000, 2.0, 0.2, 0.3, 1.0))
    if laser:
        src.append(W.GaussianLaser(1.2, 1.0, 0.5, 0.8))
    dens = None if channel_w0 is None else W.channel_density(r0, channel_w0)
    return O.RingOracle(r0, dr, dxi, n_xi, src, dens)


def _slice(o, n):
    state = o.initial_state()
    for m in range(n):
        _, state = o.slice(m, state)
    return o.slice(n, state, keep=True)[0]


def _radii(out, rng, o):
    """Radii in every kind of place: inside the first ring, between rings,
    beyond the last ring and beyond the plasma edge."""
    rho = np.sort(out["rho"])
    mids = 0.5 * (rho[:-1] + rho[1:])
    inner = rho[0] * rng.uniform(0.05, 0.95, 3)
    outer = rho[-1] + rng.uniform(0.01, 2.0, 4)
    return np.concatenate([inner, mids[::3], rng.uniform(rho[0], rho[-1], 20), outer, [o.Rp * 1.5]])


def test_fields_at_match_pairwise_sums():
    """psi = -q sum_k w_k ln max(r, rho_k) plus the ion nodes' interpolant,
    d_rho psi = -(q/r) sum_{rho_k<r} w_k plus the ions, d_zeta psi = sum of
    q w u/(rho psibar) over rings outside r (eqs. psi, dpsi_dr, dpsi_dzeta;
    R2, R11), summed pairwise in 50-digit arithmetic."""
    mpmath.mp.dps = 50
    rng = np.random.default_rng(3)
    for o in (_instance(), _instance(channel_w0=2.0)):
        out = _slice(o, 350)
        r = _radii(out, rng, o)
        got = o.fields_at(350, out, r)
        ids = out["order"]
        pb = np.empty(o.N)
        pb[ids] = out["psibar"]
        # ion nodes: 0, r0, R_p with the ion species' own Gauss/log sums
        nodes = [mp(0)] + [mp(x) for x in o.r0] + [mp(o.Rp)]
        Q = mpmath.fsum(mp(x) for x in o.w)
        ion_psi = [-mpmath.fsum(mp(o.w[j]) * mpmath.log(mp(o.r0[j])) for j in range(o.N))]
        ion_dpsi = [mp(0)]
        for k in range(o.N):
            ion_psi.append(-mpmath.fsum(mp(o.w[j]) * mpmath.log(max(mp(o.r0[k]), mp(o.r0[j])))
                                        for j in range(o.N)))
            ion_dpsi.append(-(mpmath.fsum(mp(o.w[j]) for j in range(k)) + mp(o.wh[k])) / mp(o.r0[k]))
        ion_psi.append(-Q * mpmath.log(mp(o.Rp)))
        ion_dpsi.append(-Q / mp(o.Rp))
        scale = max(np.abs(got["psi"]).max(), np.abs(got["er_bt"]).max(), np.abs(got["ez"]).max())
        assert scale > 1e-2
        for i, x in enumerate(r):
            xr = mp(x)
            e_psi = mpmath.fsum(mp(o.w[j]) * mpmath.log(max(xr, mp(out["rho"][j]))) for j in range(o.N))
            e_dpsi = mpmath.fsum(mp(o.w[j]) for j in range(o.N) if out["rho"][j] < x) / xr
            dz = -mpmath.fsum(mp(o.w[j]) * mp(out["u"][j]) / (mp(out["rho"][j]) * mp(pb[j]))
                              for j in range(o.N) if out["rho"][j] >= x)
            if xr >= nodes[-1]:
                i_psi, i_dpsi = -Q * mpmath.log(xr), -Q / xr
            else:
                j = max(m for m in range(len(nodes)) if nodes[m] < xr)
                t = (xr - nodes[j]) / (nodes[j + 1] - nodes[j])
                i_psi = (1 - t) * ion_psi[j] + t * ion_psi[j + 1]
                i_dpsi = (1 - t) * ion_dpsi[j] + t * ion_dpsi[j + 1]
            assert abs(got["psi"][i] - float(e_psi + i_psi)) <= 1e-14 * scale, (i, x)
            assert abs(got["er_bt"][i] + float(e_dpsi + i_dpsi)) <= 1e-14 * scale, (i, x)
            assert abs(got["ez"][i] + float(dz)) <= 1e-14 * scale, (i, x)


def test_fields_at_a_ring_take_its_inner_side_and_jump_across_it():
    """At r = rho_p the ring counts as outside: psi equals the ring's value,
    d_rho psi lacks the ring's w^ share, d_zeta psi carries the whole ring
    instead of w - w^, and B^(p) lacks (w^/w) C_p (R6).  Just outside the
    ring d_rho psi has gained w_p/rho_p, E_z lost the ring and B^(p) jumped
    by C_p (eq. ai_bi's jump)."""
    o = _instance(channel_w0=2.0)
    out = _slice(o, 400)
    ids = out["order"]
    rho = out["rho"][ids]
    w, wh = o.w[ids], o.wh[ids]
    c = O.Q_E * out["u"][ids] / (rho * out["psibar"])
    at = o.fields_at(400, out, rho)
    above = o.fields_at(400, out, np.nextafter(rho, np.inf))
    F = max(np.abs(out["psi"]).max(), np.abs(out["er_bt"]).max(), np.abs(out["bt"]).max())
    tol = 1e-12 * F
    ring = {q: out[q][ids] for q in ("psi", "er_bt", "ez", "bt")}
    assert np.max(np.abs(at["psi"] - ring["psi"])) <= tol
    assert np.max(np.abs(at["er_bt"] - (ring["er_bt"] - O.Q_E * wh / rho))) <= tol
    assert np.max(np.abs(at["ez"] - (ring["ez"] - c * wh))) <= tol
    assert np.max(np.abs(at["bt"] - (ring["bt"] - (wh / w) * out["C"]))) <= tol
    assert np.max(np.abs(above["er_bt"] - at["er_bt"] - O.Q_E * w / rho)) <= 1e-9 * F
    assert np.max(np.abs(above["ez"] - at["ez"] - c * w)) <= 1e-9 * F
    # B^(b) counts beam particles strictly inside: compare the plasma part only
    bb_at, _, _ = o.sources_at(400, rho)
    bb_up, _, _ = o.sources_at(400, np.nextafter(rho, np.inf))
    jump = (above["bt"] - bb_up) - (at["bt"] - bb_at)
    assert np.max(np.abs(jump - out["C"])) <= 1e-9 * F


def test_vacuum_outside_the_plasma():
    """Beyond every ring and the plasma edge the column is neutral: psi,
    d_rho psi and E_z vanish and r B_theta is the enclosed net current."""
    o = _instance()
    out = _slice(o, 300)
    r = o.Rp * np.array([1.01, 1.3, 2.0, 5.0])
    r = np.maximum(r, out["rho"].max() * np.array([1.01, 1.3, 2.0, 5.0]))
    got = o.fields_at(300, out, r)
    F = np.abs(out["psi"]).max()
    assert np.max(np.abs(got["psi"])) <= 1e-13 * F
    assert np.max(np.abs(got["er_bt"])) <= 1e-13 * F
    assert np.max(np.abs(got["ez"])) == 0.0
    rb = r * got["bt"]
    assert np.max(np.abs(rb - rb[0])) <= 1e-13 * abs(rb[0])
    assert abs(rb[0]) > 1e-3


def test_grid_bp_matches_integrated_ampere_law():
    """r B^(p)(r) = sum_{rho_k<r} q w_k u_z,k/psibar_k + d/dxi sum_k v_k
    min(r, rho_k)^2/2 (eq. maxwell_qsa_4 integrated from the axis) at grid
    nodes whose enclosed rings stay the same over three slices.  Analytic
    sources only: a particle beam's deposit is piecewise linear in xi, which
    spoils the centred difference."""
    o = _instance(laser=True, n_rings=40, dxi=0.002, n_xi=710, particles=False)
    gr = O.grid_radii(64, 3.2)
    state = o.initial_state()
    outs = []
    for n in range(702):
        out, state = o.slice(n, state, keep=True)
        outs.append(out)
    worst = scale = 0.0
    checked = 0
    for n in (300, 500, 700):
        prv, cur, nxt = outs[n - 1], outs[n], outs[n + 1]
        f = o.fields_at(n, cur, gr)
        bb, _, _ = o.sources_at(n, gr)
        ids = cur["order"]
        g = np.empty(o.N); g[ids] = cur["gamma"]
        pb = np.empty(o.N); pb[ids] = cur["psibar"]
        for i, x in enumerate(gr):
            inside = set(np.nonzero(cur["rho"] < x)[0])
            if any(set(np.nonzero(out["rho"] < x)[0]) != inside for out in (prv, nxt)):
                continue

            def F(out):
                pbk = np.empty(o.N); pbk[out["order"]] = out["psibar"]
                v = o.w * out["u"] / (out["rho"] * pbk)
                return math.fsum(v * np.minimum(x, out["rho"]) ** 2 / 2)

            below = sorted(inside)
            jz = O.Q_E * math.fsum(o.w[below] * (g[below] / pb[below] - 1.0)) if below else 0.0
            rhs = jz + (F(nxt) - F(prv)) / (2 * o.dxi)
            lhs = x * (f["bt"][i] - bb[i])
            worst = max(worst, abs(lhs - rhs))
            scale = max(scale, abs(rhs))
            checked += 1
    assert checked > 60
    assert worst < 1.5e-3 * scale, (worst, scale)


def test_grid_recorded_by_run_matches_fields_at():
    o = _instance()
    o.n_xi = 40
    res = o.run(record_stride=0, grid=(32, 4.0))
    assert res["grid"].shape == (40, 4, 32)
    out = _slice(o, 39)
    f = o.fields_at(39, out, O.grid_radii(32, 4.0))
    for q, name in enumerate(("psi", "er_bt", "ez", "bt")):
        assert np.array_equal(res["grid"][39, q], f[name])
