"""Plain CPU oracle of the gridless model with mobile ions (two species).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this file; only the tests do.  It shares no code with the HIP path.

What it computes (paper: Sec. "Gridless quasistatic model", "Key
algorithmic adjustments"; the beam-driven benchmark of Sec. "Validation
benchmarks" marches plasma ions): two plasma species, electrons (q = -1,
m = 1) and singly charged ions (q = +1, mass m_i in electron masses), each
discretised into rings at the same initial radii with the same weights.  Per
slice each species is sorted and its own Gauss/log and d_zeta psi sums are
formed at its own rings (eqs. dpsi_dr, psi, dpsi_dzeta, with the modified
weight w^ for the ring itself, reading R6); the fields of one species are
gathered at the rings of the other by linear interpolation between its rings
(the rule of "Key algorithmic adjustments": j = last ring of the other
species with rho_j below the radius); B_theta^(p) comes from the electrons
alone (the ion currents are neglected, as the paper does), from the same
two-point recursion as the one-species oracle, and reaches the ions by the
same linear interpolation.  Both species are pushed with Adams-Bashforth-2
(eqs. plasma_particle_motion_1-4 with their q and m; readings R3, R8, R9).

Readings beyond the one-species oracle's (numbered as in the design notes):
  R18 the interpolation nodes of a species are its rings at their current
      radii, plus a virtual node at the axis (psi(0) of the species, d_rho
      psi = 0, d_zeta psi(0), B^(p) = 0) and one at the species' outer edge,
      the outermost ring's radius plus half its initial radial extent
      (exterior values -q Q ln r, -q Q / r, d_zeta psi = 0, B^(p) = b_N / r);
      beyond the edge the exterior field itself.  Rings at rest give the
      immobile-ion nodes of reading R11 exactly.
  R19 mobile ions start at the electrons' initial radii with the same
      weights and momenta zero; psibar of an ion is 1 - psi / m_i (eq.
      plasma_particle_motion with q = +1).

With m_i -> infinity the ions stay at rest and the electrons' fields are
those of the one-species oracle (pinned).
"""
from __future__ import annotations

import numpy as np

from oracle.wake_oracle import (BREAKDOWN, DD, LD, M_E, Q_E, Q_ION, BeamTable, analytic_lambda,
                                b_plasma_at_rings, coefficients, dd_cat, dd_log, forces,
                                laser_terms, prefix_sum, push_ab2, ring_log, ring_weights,
                                solve_recursion, suffix_sum, transfer, _gauss_log_sums)


def local_quantities_q(psi, u, a2, q, m):
    """psibar = 1 - (q/m) psi and gamma (eq. plasma_particle_motion_4) of a
    species of charge q and mass m."""
    psibar = 1.0 - (q / m) * psi
    gamma = (1.0 + u * u + psibar * psibar + (q * q) / (2.0 * m * m) * a2) / (2.0 * psibar)
    return psibar, gamma


def dzeta_psi_q(rho, u, w, wh, psibar, q):
    """d_zeta psi of one species at its sorted rings (eq. dpsi_dzeta, R2,
    R6): the rings outside with q w u / (rho psibar), the ring itself with
    weight w - w^.  Returns (at the rings, at the axis) in 80-bit."""
    c = (q * u / (rho * psibar)).astype(LD)
    rsum = suffix_sum(w.astype(LD) * c).ld()
    above = np.concatenate([rsum[1:], np.zeros(1, LD)])
    return above + (w - wh).astype(LD) * c, rsum[0] if len(rsum) else LD(0)


class Nodes:
    """Interpolation nodes of one species at one slice (reading R18)."""

    def __init__(self, rho_sorted, edge, lnedge, q, Q):
        self.r = np.concatenate([[LD(0)], rho_sorted.astype(LD), [LD(edge)]])
        self.edge = LD(edge)
        self.lnedge = DD.of(lnedge)
        self.q, self.Q = q, Q                      # Q: total weight (DD)

    def set_psi(self, psi, dpsi, psi_axis):
        ext_psi = self.Q * self.lnedge * (-self.q)
        self.psi = dd_cat([psi_axis, psi, ext_psi])
        self.dpsi = np.concatenate([[LD(0)], dpsi, [-self.q * self.Q.ld()[0] / self.edge]])

    def set_dz(self, dz, dz_axis):
        self.dz = np.concatenate([[LD(dz_axis)], dz, [LD(0)]])

    def set_bp(self, bp, b_last):
        self.b_last = float(b_last)
        self.bp = np.concatenate([[0.0], bp, [self.b_last / float(self.edge)]])

    def _where(self, rho):
        rho_l = np.asarray(rho).astype(LD)
        j = np.searchsorted(self.r, rho_l, side="left") - 1
        outside = j >= len(self.r) - 1
        jj = np.clip(j, 0, len(self.r) - 2)
        t = (rho_l - self.r[jj]) / (self.r[jj + 1] - self.r[jj])
        return rho_l, jj, t, outside

    def gather_psi(self, rho, lnrho):
        """psi (DD) and d_rho psi (80-bit) of this species at radii rho."""
        rho_l, jj, t, out = self._where(rho)
        psi = self.psi[jj] + (self.psi[jj + 1] - self.psi[jj]) * DD.of(t)
        dpsi = (1 - t) * self.dpsi[jj] + t * self.dpsi[jj + 1]
        if np.any(out):
            ext = DD.of(lnrho)[out] * self.Q * (-self.q)
            psi.hi[out] = ext.hi
            psi.lo[out] = ext.lo
            dpsi[out] = -self.q * self.Q.ld()[0] / rho_l[out]
        return psi, dpsi

    def gather_dz(self, rho):
        rho_l, jj, t, out = self._where(rho)
        dz = (1 - t) * self.dz[jj] + t * self.dz[jj + 1]
        dz[out] = 0
        return dz

    def gather_bp(self, rho):
        rho_l, jj, t, out = self._where(rho)
        tt = t.astype(np.float64)
        bp = (1.0 - tt) * self.bp[jj] + tt * self.bp[jj + 1]
        r = np.asarray(rho, np.float64)
        bp[out] = self.b_last / r[out]
        return bp


class TwoSpeciesOracle:
    """One instance with electrons and mobile ions of mass m_i."""

    def __init__(self, r0, dr, dxi, n_xi, ion_mass, sources=(), dens=None):
        self.r0 = np.asarray(r0, np.float64)
        self.dr = np.asarray(dr, np.float64)
        self.N = len(self.r0)
        self.dxi = float(dxi)
        self.n_xi = int(n_xi)
        self.m_i = float(ion_mass)
        self.w, self.wh = ring_weights(self.r0, self.dr, dens)
        self.lnr0 = dd_log(self.r0)
        self.Q = prefix_sum(self.w)[self.N - 1:]   # total weight of each species (DD)
        beams = [s for s in sources if getattr(s, "kind", "") == "particles"]
        self.analytic = [s for s in sources if getattr(s, "kind", "") == "gaussian"]
        self.lasers = [s for s in sources if getattr(s, "kind", "") == "laser"]
        self.table = BeamTable(beams, self.dxi, self.n_xi)

    def initial_state(self):
        z = np.zeros(self.N)
        one = dict(rho=self.r0.copy(), u=z.copy(), fr=z.copy(), fu=z.copy())
        return dict(e=one, i={k: v.copy() for k, v in one.items()})

    def sources_at(self, n, rho):
        xi = n * self.dxi
        lam = self.table.lam(n, rho)
        for s in self.analytic:
            lam = lam + analytic_lambda(s, xi, rho)
        a2 = np.zeros_like(rho)
        da2 = np.zeros_like(rho)
        for s in self.lasers:
            x, dx = laser_terms(s, xi, rho)
            a2 = a2 + x
            da2 = da2 + dx
        return lam / rho, a2, da2

    def _species(self, st, q):
        """Sorted view and own sums of one species."""
        ids = np.lexsort((np.arange(self.N), st["rho"]))                # R7
        rho, u = st["rho"][ids], st["u"][ids]
        w, wh = self.w[ids], self.wh[ids]
        lnr = ring_log(rho, self.r0[ids], self.lnr0[ids])               # R14
        psi, dpsi, axis = _gauss_log_sums(rho.astype(LD), w, wh, q, lnr)
        edge = rho[-1] + self.dr[ids[-1]] / 2.0                          # R18
        nodes = Nodes(rho, edge, dd_log([edge]), q, self.Q)
        nodes.set_psi(psi, dpsi, axis)
        return dict(ids=ids, rho=rho, u=u, w=w, wh=wh, lnr=lnr, psi=psi, dpsi=dpsi, axis=axis,
                    nodes=nodes)

    def slice(self, n, state, push=True, keep=False):
        """Fields of both species at slice n and the state pushed to n+1
        (state = {'e': ..., 'i': ...}, arrays by ring id).  Returns (out,
        new_state); out['status'] = 0 or BREAKDOWN."""
        E = self._species(state["e"], Q_E)
        I = self._species(state["i"], Q_ION)
        bb_e, a2_e, da2_e = self.sources_at(n, E["rho"])
        bb_i, a2_i, da2_i = self.sources_at(n, I["rho"])
        # psi and d_rho psi: own sums plus the other species gathered
        gp, gd = I["nodes"].gather_psi(E["rho"], E["lnr"])
        psi_e, dpsi_e = (E["psi"] + gp).f64(), (E["dpsi"] + gd).astype(np.float64)
        gp, gd = E["nodes"].gather_psi(I["rho"], I["lnr"])
        psi_i, dpsi_i = (I["psi"] + gp).f64(), (I["dpsi"] + gd).astype(np.float64)
        psi_axis = float((E["axis"] + I["axis"]).f64()[0])
        pb_e, gm_e = local_quantities_q(psi_e, E["u"], a2_e, Q_E, M_E)
        pb_i, gm_i = local_quantities_q(psi_i, I["u"], a2_i, Q_ION, self.m_i)
        out = dict(status=0)
        for pb in (pb_e, pb_i):
            if not np.all(pb > 0) or not np.all(np.isfinite(pb)):        # R10
                out["status"] = BREAKDOWN
                return out, None
        # d_zeta psi: own sums plus the other species gathered
        dz_e_own, dza_e = dzeta_psi_q(E["rho"], E["u"], E["w"], E["wh"], pb_e, Q_E)
        dz_i_own, dza_i = dzeta_psi_q(I["rho"], I["u"], I["w"], I["wh"], pb_i, Q_ION)
        E["nodes"].set_dz(dz_e_own, dza_e)
        I["nodes"].set_dz(dz_i_own, dza_i)
        dz_e = (dz_e_own + I["nodes"].gather_dz(E["rho"])).astype(np.float64)
        dz_i = (dz_i_own + E["nodes"].gather_dz(I["rho"])).astype(np.float64)
        dz_axis = float(dza_e + dza_i)
        # B^(p) from the electrons alone (eqs. b_coeffs_1-3, ai_bi)
        A, B, C = coefficients(E["rho"], E["u"], E["w"], pb_e, gm_e, dpsi_e, dz_e, bb_e, da2_e)
        M, s = transfer(A, B, C, E["rho"])
        a, b = solve_recursion(M, s)
        bp_e = b_plasma_at_rings(a, b, E["rho"], C, E["w"], E["wh"])
        E["nodes"].set_bp(bp_e, b[-1])
        bt_e = bb_e + bp_e
        bt_i = bb_i + E["nodes"].gather_bp(I["rho"])
        new = None
        if push:
            new = {}
            for key, S, pb, gm, dp, bt, da2, q, m in (
                    ("e", E, pb_e, gm_e, dpsi_e, bt_e, da2_e, Q_E, M_E),
                    ("i", I, pb_i, gm_i, dpsi_i, bt_i, da2_i, Q_ION, self.m_i)):
                fr, fu = forces(S["u"], pb, gm, dp, bt, da2, q, m)
                if n == 0:                                                # R8
                    fr_p, fu_p = fr, fu
                else:
                    fr_p, fu_p = state[key]["fr"][S["ids"]], state[key]["fu"][S["ids"]]
                rho_n, u_n, frs, fus = push_ab2(S["rho"], S["u"], fr, fu, fr_p, fu_p, self.dxi)
                ns = {k: np.empty(self.N) for k in ("rho", "u", "fr", "fu")}
                ns["rho"][S["ids"]], ns["u"][S["ids"]] = rho_n, u_n
                ns["fr"][S["ids"]], ns["fu"][S["ids"]] = frs, fus
                new[key] = ns
        check = [psi_e, dpsi_e, dz_e, bt_e, psi_i, dpsi_i, dz_i, bt_i]
        if new is not None:
            check += [new[k][q] for k in ("e", "i") for q in ("rho", "u")]
        if not all(np.all(np.isfinite(c)) for c in check):               # R10
            out["status"] = BREAKDOWN
            return out, None

        def by_id(S, x):
            y = np.empty(self.N)
            y[S["ids"]] = x
            return y

        for key, S, psi, dp, dz, bt in (("", E, psi_e, dpsi_e, dz_e, bt_e),
                                        ("ion_", I, psi_i, dpsi_i, dz_i, bt_i)):
            out.update({key + "psi": by_id(S, psi), key + "er_bt": by_id(S, -dp),
                        key + "ez": by_id(S, -dz), key + "bt": by_id(S, bt),
                        key + "rho": by_id(S, S["rho"]), key + "u": by_id(S, S["u"])})
        out.update(psi_axis=psi_axis, ez_axis=-dz_axis)
        if keep:
            out.update(order=E["ids"], ion_order=I["ids"], A=A, B=B, C=C, M=M, s=s, a=a, b=b,
                       bb=bb_e, psibar=pb_e, ion_psibar=pb_i)
        return out, new

    def run(self, first=0, count=None, state=None, record_stride=1):
        """March slices [first, first+count); lineouts, snapshots of both
        species every record_stride slices, final state, breakdown slice."""
        if count is None:
            count = self.n_xi - first
        if state is None:
            state = self.initial_state()
        rec = {}
        axis = np.full((count, 2), np.nan)
        breakdown = -1
        for k in range(count):
            n = first + k
            out, new = self.slice(n, state, push=(n < self.n_xi - 1))
            if out["status"] != 0:
                breakdown = n
                break
            axis[k] = (out["psi_axis"], out["ez_axis"])
            if record_stride and (n % record_stride == 0 or k == count - 1):
                rec[n] = {q: out[q] for q in out if q not in ("status", "psi_axis", "ez_axis")}
            if new is not None:
                state = new
        return dict(axis=axis, snap=rec, state=state, breakdown=breakdown)
