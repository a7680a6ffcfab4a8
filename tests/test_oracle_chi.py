"""Pins of the oracle's chi = n/gamma deposit (reading R20) against facts
from outside it.

* A single ring between two nodes of a uniform grid deposits c W / V with
  the hat weights and V_g = r_g dr (closed form, exact in binary).
* A ring inside the first node counts wholly to it, over V_0 = r_0^2/2 +
  dr (2 r_0 + r_1)/6.
* Conservation: sum_g V_g chi_g equals sum_j c_j for rings below the last
  node; above it the last node's hat falls off linearly.
* A uniform column at rest (c = w = rho drho) deposits chi = 1 away from
  the axis (the midpoint rule integrates the hat exactly there) and within
  6e-4 at the first node.
* The weight of a ring is n/gamma: w / (gamma - u_z) from eqs.
  plasma_particle_motion_3-4 (gamma and u_z computed from u_r, psibar and
  |a|^2 there, not from psibar alone) equals the oracle's w / psibar;
  planted mistakes (gamma for psibar, a wrong V_0, no fold) fail the pins.
"""
import numpy as np
import pytest

from oracle import wake_oracle as O
from oracle.wake_oracle import LD, chi_deposit, chi_volumes, grid_radii
from paper_2603_16623_amd import workloads as W


def test_single_ring_between_nodes_closed_form():
    gr = grid_radii(8, 2.0)                 # dr = 0.25, nodes 0.125 .. 1.875
    rho = np.array([(gr[1] + gr[2]) / 2])   # 0.5: half way between nodes 1 and 2
    chi = chi_deposit(rho, np.array([1.0]), gr)
    want = np.zeros(8)
    want[1] = 0.5 / (gr[1] * 0.25)
    want[2] = 0.5 / (gr[2] * 0.25)
    assert np.array_equal(chi.astype(np.float64), want)
    V = chi_volumes(gr)
    assert np.array_equal(V[1:-1].astype(np.float64), gr[1:-1] * 0.25)


def test_axis_fold_and_first_volume():
    gr = grid_radii(8, 2.0)
    chi = chi_deposit(np.array([0.05]), np.array([3.0]), gr)
    v0 = gr[0] ** 2 / 2 + 0.25 * (2 * gr[0] + gr[1]) / 6
    assert abs(float(chi[0]) - 3.0 / v0) <= 1e-15 * 3.0 / v0
    assert np.all(chi[1:] == 0)


def test_conservation_on_random_grids():
    """The hats sum to one below the last node; above it the last node's hat
    falls to zero at r_{n-1} + (r_{n-1} - r_{n-2})."""
    rng = np.random.default_rng(3)
    for trial in range(5):
        gr = np.sort(rng.uniform(0.01, 3.0, 40))
        top = gr[-1] + (gr[-1] - gr[-2])
        rho = np.sort(rng.uniform(0.0, gr[-1], 500))
        c = rng.uniform(0.1, 2.0, 500)
        chi = chi_deposit(rho, c, gr)
        tot = float(np.sum(chi_volumes(gr) * chi))
        assert abs(tot - float(np.sum(c.astype(LD)))) <= 1e-15 * float(np.sum(c))
        # one ring above the last node, a quarter of the way to the top
        r = gr[-1] + 0.25 * (top - gr[-1])
        chi = chi_deposit(np.array([r]), np.array([1.0]), gr)
        assert np.all(chi[:-1] == 0)
        assert abs(float(chi[-1] * chi_volumes(gr)[-1]) - 0.75) <= 1e-14   # r rounded to binary64


def test_uniform_column_at_rest_deposits_one():
    r0, dr = W.uniform_rings(1000, 5.0)
    o = O.RingOracle(r0, dr, 0.02, 4, [])
    out, _ = o.slice(0, o.initial_state(), keep=True)
    gr = grid_radii(50, 4.0)
    chi = o.chi_at(out, gr)
    assert np.max(np.abs(chi[1:] - 1.0)) <= 1e-13
    assert abs(chi[0] - 1.0) <= 6.1e-4


def _gamma_uz(u, psibar, a2):
    """gamma and u_z of an electron (q = -1, m = 1) from eqs.
    plasma_particle_motion_3-4."""
    gamma = (1.0 + u * u + psibar * psibar + 0.5 * a2) / (2.0 * psibar)
    uz = (1.0 + u * u - psibar * psibar + 0.5 * a2) / (2.0 * psibar)
    return gamma, uz


def test_weight_is_n_over_gamma_in_a_driven_column():
    inst = W.small_instance(8, n_rings=257, n_xi=120, n_peak=1.0, laser=True, dxi=0.01)
    o = O.RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources)
    st = o.initial_state()
    for n in range(100):
        _, st = o.slice(n, st)
    out, _ = o.slice(100, st, keep=True)
    ids = out["order"]
    rho = out["rho"][ids]
    gamma, uz = _gamma_uz(out["u"][ids], out["psibar"], out["a2"])
    assert float(np.max(out["a2"])) > 1e-3 and float(np.max(np.abs(out["u"]))) > 1e-3
    c = o.w[ids] / (gamma - uz)                      # n / gamma per ring (eq. fluid_from_mp_1)
    gr = grid_radii(60, 3.3)
    want = chi_deposit(rho, c, gr).astype(np.float64)
    got = o.chi_at(out, gr)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # planted: the weight w / gamma instead of w / psibar
    bad = chi_deposit(rho, o.w[ids] / gamma, gr).astype(np.float64)
    assert np.max(np.abs(bad - want)) > 1e-6 * np.max(np.abs(want))


def test_planted_deposit_mistakes_fail(monkeypatch):
    r0, dr = W.uniform_rings(1000, 5.0)
    gr = grid_radii(50, 4.0)
    c = r0 * dr
    good = O.chi_volumes

    def v_no_axis(radii):                            # V_0 as an interior node's r_0 dr
        v = good(radii)
        v[0] = LD(radii[0]) * (LD(radii[1]) - LD(radii[0]))
        return v

    monkeypatch.setattr(O, "chi_volumes", v_no_axis)
    chi = O.chi_deposit(r0, c, gr)
    assert abs(float(chi[0]) - 1.0) > 1e-2
    monkeypatch.setattr(O, "chi_volumes", good)
    # no fold: rings inside the first node dropped
    inside = r0 >= gr[0]
    chi = O.chi_deposit(r0[inside], c[inside], gr)
    assert abs(float(chi[0]) - 1.0) > 1e-2
