"""Per-field parity norm shared by the GPU parity tests (not a test module).

Per slice, each field is held to 1e-12 of its own scale at that slice
(max_i |gpu - oracle| <= 1e-12 * scale_q) and the margin e / tolerance of
every field is printed.  A field whose scale is below 1e-15 has vanished up
to rounding (the plasma at rest: both sides leave double-double residues of
1e-31..1e-22) and is held to 1e-12 of 1e-15.  The scales:

  psi            max over the rings of |psi| and |psi(0)| (the axis value is
                 the same field at r = 0);
  E_r - B_theta  max |E_r - B_theta| over the rings;
  E_z            max over the rings of |E_z| and |E_z(0)|;
  B_theta        max over the rings of |B_theta| and of the terms it is the
                 sum of: |B^(b)|, |a_{i-1} rho_i|, |b_{i-1} / rho_i| and
                 |C_i|.

B_theta alone takes a wider scale: at ring i it is B^(b) plus the inner-side
value a_{i-1} rho_i + b_{i-1}/rho_i of the two-point recursion plus the
fraction w^_i/w_i of the jump C_i (eq. b_theta_plasma, Sec. "Key algorithmic
adjustments").  These terms cancel: behind a linear driver or under a weak
laser the beam field and the plasma's return current nearly cancel, and in a
perturbed column a_{i-1} rho_i and b_{i-1}/rho_i are 10^3 times their sum.
The unknowns (a, b) of the recursion are binary64 numbers on both sides
(the oracle's are its LU solution refined to the nearest binary64), so an
ulp of a term, not of B_theta, is what either side can resolve.

On a field grid the scale of each field also takes the grid's own values.
"""
import numpy as np

FIELDS = ("psi", "er_bt", "ez", "bt")
TOL_SLICE = 1e-12
TOL_E2E = 1e-8


def say(*a):
    print(*a, flush=True)


FLOOR = 1e-15     # below this a field has vanished up to rounding


def rel(gpu, ref, scale=None):
    """max |gpu - ref| over max |ref| (or the given scale), the scale
    floored at FLOOR."""
    if scale is None:
        scale = float(np.max(np.abs(ref))) if np.size(ref) else 0.0
    return float(np.max(np.abs(gpu - ref))) / max(scale, FLOOR)


def field_scales(ref, grid=None):
    """Scale of each field of one oracle slice (``ref`` from
    RingOracle.slice(keep=True)); ``grid``: the oracle's fields at grid
    nodes of that slice, if any."""
    def m(x):
        x = np.asarray(x)
        return float(np.max(np.abs(x))) if x.size else 0.0
    rho = np.asarray(ref["rho"])[ref["order"]]
    s = {"psi": max(m(ref["psi"]), abs(float(ref["psi_axis"]))),
         "er_bt": m(ref["er_bt"]),
         "ez": max(m(ref["ez"]), abs(float(ref["ez_axis"]))),
         "bt": max(m(ref["bt"]), m(ref["bb"]), m(ref["C"]), m(ref["a"][:-1] * rho),
                   m(ref["b"][:-1] / rho))}
    if grid is not None:
        for q in FIELDS:
            s[q] = max(s[q], m(grid[q]))
    return s


def tol_of(scale):
    return TOL_SLICE * max(scale, FLOOR)


def check_fields(got, ref, scales, label, want=None):
    """Assert every field of ``got`` within 1e-12 of its scale of ``want``
    (default: ``ref``); print the margins (error over tolerance).  Returns
    the margins."""
    want = ref if want is None else want
    margins = {}
    for q in FIELDS:
        e = float(np.max(np.abs(np.asarray(got[q]) - np.asarray(want[q])))) if np.size(want[q]) else 0.0
        margins[q] = e / tol_of(scales[q])
    say(f"  margins {label}: " + " ".join(f"{q}={margins[q]:.3g}" for q in FIELDS)
        + f"  (bt scale / max|bt| = {scales['bt'] / max(float(np.max(np.abs(want['bt']))), 1e-300):.3g})")
    for q in FIELDS:
        assert margins[q] <= 1.0, (label, q, margins[q], scales[q])
    return margins


def check_axis(lp, le, n, ref, scales, label):
    """psi(0) and E_z(0) of slice n against the oracle's, per field."""
    ep = abs(float(lp[n]) - float(ref["psi_axis"])) / tol_of(scales["psi"])
    ee = abs(float(le[n]) - float(ref["ez_axis"])) / tol_of(scales["ez"])
    assert ep <= 1.0 and ee <= 1.0, (label, "axis", ep, ee)


def check_state(st, new, label):
    """Pushed ring state elementwise to 1e-12 of each quantity's largest
    magnitude."""
    for a, b in (("rho", "rho"), ("ur", "u"), ("f_rho", "fr"), ("f_u", "fu")):
        r = rel(st[a], new[b])
        assert r <= TOL_SLICE, (label, a, r)


def pushed_by_device(wk, inst, n, state):
    """The device's own ring state at slice n+1, marched from ``state`` at
    slice n by a context of its own (the current tiling and cooperative
    layout), as a state dict for the oracle.  The second slice of a
    two-slice test is then compared on identical input: the pushed radii of
    rings pushed through the axis or past many neighbours carry the push's
    rounding, which the fields at n+1 amplify (d_rho psi goes as 1/rho)."""
    s = wk.WakeSolver.from_instance(inst, record_stride=1)
    s.wake_set_state(n, state["rho"], state["u"], state["fr"], state["fu"])
    s.wake_solve(n, 1)
    st = s.wake_get_state()
    s.close()
    assert st["slice"] == n + 1
    return st, dict(rho=st["rho"], u=st["ur"], fr=st["f_rho"], fu=st["f_u"])
