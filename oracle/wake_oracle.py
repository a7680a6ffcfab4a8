"""Plain, slow CPU oracle of the gridless quasistatic plasma-ring model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this file; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path.

What it computes (paper: "Gridless quasistatic model", Sec. "Numerical
integration of wakefields", "Key algorithmic adjustments", Fig. 2 right
column, Appendix "Solve recursive system"):  electron plasma rings (q=-1,
m=1) over an immobile ion species, marched in xi = -zeta, one slice at a
time:

  sort rings radially -> gather beam/laser sources -> psi, d_rho psi,
  d_zeta psi -> gamma -> A, B, C -> two-point recursion for B_theta^(p)
  -> Adams-Bashforth-2 push.

Every floating-point quantity is IEEE binary64 except the sums that cancel
(the Gauss/log sums of the psi family, eqs. dpsi_dr and psi, the ion node
fields and the d_zeta psi sum), which are formed in 80-bit extended
precision from prefix sums accumulated in double-double (about 106 bits,
``prefix_sum``) and rounded to binary64 once.  The two-point recursion
(eq. ai_bi with b_0=0, a_N=0) is
solved as the linear system it defines, with LAPACK's banded LU (partial
pivoting); the paper's shooting procedure is kept as ``solve_shooting``.

Readings taken where the paper is silent, garbled or self-inconsistent
(numbered as in the design notes; R16, the parity norm, concerns the tests
only):
  R1  electrons carry q=-1, m=1; psibar = 1 + psi = gamma - u_z.
  R2  d_zeta psi = +sum_{rho_k>rho} q w u/(rho psibar)   (the printed sum is
      its negative; derived by differentiating eq. psi with eq. motion_2).
  R3  ponderomotive term: du_r/dzeta gets +q^2 d_rho|a|^2/(4 m^2 psibar)
      and B_i gets -q^3 w d_rho|a|^2/(4 m^2 rho psibar^2)  (printed sign of
      eq. motion_1 and the missing 1/4 in eq. b_coeffs_2 overruled).
  R4  the extra w/rho prefactor in the source decomposition is dropped.
  R5  modified weight w^_j = w_j/2 - n_j dr_j^2/8, a fixed per-ring constant.
  R6  at ring i: d_rho psi uses S_<i + w^_i;  d_zeta psi gives ring i the
      weight w_i - w^_i;  B^(p)_i = B^- + (w^_i/w_i) C_i.
  R7  ties in rho are ordered by ring id.
  R8  AB2 starts with an Euler step on slice 0 (f_prev := f).
  R9  a ring whose radius becomes negative is reflected: rho, u_r and the
      stored AB2 history change sign.
  R10 psibar <= 0 or any non-finite result stops the solve (breakdown).
  R11 immobile ions: one ion ring per electron ring at its initial radius
      with the same weight; node fields use w^; they are gathered to the
      electron radii by linear interpolation (Sec. "Key algorithmic
      adjustments"), with virtual nodes at rho=0 (d_rho psi = 0) and at the
      plasma edge R_p, and the exact exterior field beyond R_p.
  R12 beam particles are deposited in xi with linear (cloud-in-cell)
      weights onto the slice nodes xi_n = n dxi; radially each particle is a
      thin ring, counted below rho when r_k < rho (strict).
  R13 laser: |a|^2 = a0^2 exp(-2 rho^2/w0^2) exp(-2 (xi-xi_L)^2/L^2).
  R14 (numerics, not model) ln rho is evaluated as ln r0 + log1p((rho-r0)/r0)
      so that its rounding, multiplied by the enclosed charge in eq. psi,
      stays proportional to the ring displacement.
  R15 (numerics) the B^(p) recursion is solved as the linear system it
      defines (eq. ai_bi with b_0 = 0, a_N = 0) by banded LU, followed by
      two steps of iterative refinement whose residuals are accumulated in
      80-bit arithmetic: the binary64 LU alone loses digits with the
      system's conditioning at 10^5 rings.  The paper's shooting procedure
      (Appendix "Solve recursive system") reaches the same solution with a
      loss of about log10(I1(R_p)^2) digits and is kept as solve_shooting.
  R17 fields at radii off the rings (Fig. 2, external grid): the same sums
      with no ring at the radius (no w^ term, no own-ring share), B^(p) from
      the interval's (a, b); a ring at exactly that radius counts as
      outside.  The field grid is uniform with nodes at cell centres
      (g + 1/2) r_max / n_r.
  R20 the susceptibility chi = n/gamma on the laser grid (Fig. 2, Sec.
      "Integration into Wake-T"; the deposit's shape is not given): ring j
      carries chi(rho) rho = (w_j / psibar_j) delta(rho - rho_j), since
      eq. fluid_from_mp_1 gives n/gamma = w / (rho (1 - v_z) gamma) delta and
      (1 - v_z) gamma = gamma - u_z = psibar (eqs. plasma_particle_motion_3-4).
      Deposited with linear (hat) weights W_g between neighbouring nodes, a
      ring inside the first node counting wholly to it (folded at the axis),
      the last node's hat reaching as far above it as the spacing below it,
      each node normalised by V_g = integral of W_g rho drho:
      chi_g = sum_j (w_j / psibar_j) W_g(rho_j) / V_g.  A uniform column at
      rest deposits chi = 1, and sum_g V_g chi_g = sum_j w_j / psibar_j.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_banded

LD = np.longdouble
Q_E = -1.0   # electron charge (R1)
M_E = 1.0    # electron mass
Q_ION = 1.0  # singly charged ions (R11)

BREAKDOWN = -5


# ---------------------------------------------------------------------------
# double-double arithmetic (for psi, whose terms cancel) and accurate sums
# ---------------------------------------------------------------------------
def _two_sum(a, b):
    """a + b = s + e exactly (binary64 arrays; numpy does not contract)."""
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _quick_two_sum(a, b):
    """a + b = s + e exactly when |a| >= |b|."""
    s = a + b
    return s, b - (s - a)


def _split(a):
    """Dekker's split: a = h + l with h, l of at most 26 significand bits."""
    c = 134217729.0 * a
    h = c - (c - a)
    return h, a - h


def _two_prod(a, b):
    """a * b = p + e exactly (Dekker's product, no fused multiply-add)."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    return p, ((ah * bh - p) + ah * bl + al * bh) + al * bl


class DD:
    """Double-double numbers: unevaluated sums hi + lo of binary64 arrays
    (about 106 significand bits), for the psi sums, whose terms cancel."""

    def __init__(self, hi, lo=None):
        self.hi = np.asarray(hi, np.float64)
        self.lo = np.zeros_like(self.hi) if lo is None else np.asarray(lo, np.float64)

    @staticmethod
    def of(x):
        """Exact conversion of a DD, binary64 or 80-bit array (an 80-bit
        value is the sum of two binary64 numbers: 64 significand bits)."""
        if isinstance(x, DD):
            return x
        x = np.asarray(x)
        if x.dtype == LD:
            hi = x.astype(np.float64)
            return DD(hi, (x - hi.astype(LD)).astype(np.float64))
        return DD(x.astype(np.float64))

    def __add__(self, o):
        o = DD.of(o)
        s, e = _two_sum(self.hi, o.hi)
        t, f = _two_sum(self.lo, o.lo)
        s, e = _quick_two_sum(s, e + t)
        return DD(*_quick_two_sum(s, e + f))

    __radd__ = __add__

    def __neg__(self):
        return DD(-self.hi, -self.lo)

    def __sub__(self, o):
        return self + (-DD.of(o))

    def __rsub__(self, o):
        return DD.of(o) + (-self)

    def __mul__(self, o):
        o = DD.of(o)
        p, e = _two_prod(self.hi, o.hi)
        e = e + (self.hi * o.lo + self.lo * o.hi)
        return DD(*_quick_two_sum(p, e))

    __rmul__ = __mul__

    def __getitem__(self, k):
        return DD(self.hi[k], self.lo[k])

    def __len__(self):
        return len(self.hi)

    def ld(self):
        """Rounded to 80-bit extended precision."""
        return self.hi.astype(LD) + self.lo.astype(LD)

    def f64(self):
        """Rounded to binary64."""
        return self.hi + self.lo


def dd_cat(parts):
    parts = [DD.of(p) for p in parts]
    return DD(np.concatenate([np.atleast_1d(p.hi) for p in parts]),
              np.concatenate([np.atleast_1d(p.lo) for p in parts]))


def dd_log(x):
    """ln x of positive binary64 values as double-doubles, from 40-digit
    logarithms (mpmath)."""
    import mpmath
    out_h = np.empty(len(x))
    out_l = np.empty(len(x))
    with mpmath.workdps(40):
        for i, v in enumerate(np.asarray(x, np.float64)):
            l = mpmath.log(mpmath.mpf(float(v)))
            h = float(l)
            out_h[i] = h
            out_l[i] = float(l - h)
    return DD(out_h, out_l)


def prefix_sum(x):
    """Inclusive prefix sums x_0 + ... + x_i (a DD array; x: DD, binary64 or
    80-bit), each the exact sum to about 2^-100 of the magnitudes involved.
    The terms are added in double-double arithmetic over the log2(n) steps
    of a scan (step d adds the running sum d places back): at this
    precision the order of the additions does not show in the result.  (A
    plain 80-bit running sum over 2e5 terms of the psi sums errs by a few
    1e-15, more than 1e-12 of a psi of order 1e-3.)"""
    x = DD.of(x)
    hi, lo = x.hi.copy(), x.lo.copy()
    d = 1
    while d < len(hi):
        t = DD(hi[d:], lo[d:]) + DD(hi[:-d], lo[:-d])
        hi = np.concatenate([hi[:d], t.hi])
        lo = np.concatenate([lo[:d], t.lo])
        d *= 2
    return DD(hi, lo)


def suffix_sum(x):
    """Inclusive suffix sums x_i + ... + x_{n-1}, as prefix_sum."""
    x = DD.of(x)
    r = prefix_sum(DD(x.hi[::-1], x.lo[::-1]))
    return DD(r.hi[::-1], r.lo[::-1])


# ---------------------------------------------------------------------------
# set-up (Sec. "Discretization of plasma species into macroparticles")
# ---------------------------------------------------------------------------
def ring_weights(r0, dr, dens=None):
    """Ring weight w_j = n_j0 rho_j0 dr_j (eq. macroparticle_weight) and the
    modified weight w^_j = w_j/2 - n_j0 dr_j^2/8 (Key algorithmic adjustments,
    reading R5)."""
    n = np.ones_like(r0) if dens is None else np.asarray(dens, np.float64)
    w = n * r0 * dr
    wh = w / 2.0 - n * dr * dr / 8.0
    return w, wh


def _gauss_log_sums(rho_l, w, wh, q, lnr):
    """Fields of one species at its own sorted ring radii.

    eq. dpsi_dr : d_rho psi(rho) = -(1/rho) sum_{rho_k<rho} q w_k
    eq. psi     : psi(rho) = -sum_k q w_k ln max(rho, rho_k)
    At the ring itself the ring contributes w^ to the Gauss sum (R6); psi is
    continuous there.  w, wh: binary64 weights; lnr = ln(rho_l) as DD.
    Returns (psi as DD, d_rho psi in 80-bit, psi on the axis as DD).
    """
    csum = prefix_sum(w)
    below = dd_cat([DD(0.0), csum[:-1]])                          # sum_{k<i} w_k
    wl = lnr * np.asarray(w, np.float64)
    rsum = suffix_sum(wl)                                         # sum_{k>=i}
    above = dd_cat([rsum[1:], DD(0.0)])                           # sum_{k>i}
    dpsi = -q * (below.ld() + np.asarray(wh, LD)) / rho_l
    psi = ((below + np.asarray(w, np.float64)) * lnr + above) * (-q)
    psi_axis = rsum[0:1] * (-q)
    return psi, dpsi, psi_axis


class IonNodes:
    """Immobile ion rings at the initial radii (reading R11)."""

    def __init__(self, r0, w, wh, lnr0):
        """lnr0: ln r0 as DD."""
        psi, dpsi, psi_axis = _gauss_log_sums(r0.astype(LD), w, wh, Q_ION, lnr0)
        self.Q = prefix_sum(w)[len(w) - 1:]
        self.Rp = None
        self.r = None
        self._psi = psi
        self._dpsi = dpsi
        self._psi_axis = psi_axis
        self._r0 = r0

    def finish(self, Rp, lnRp):
        """Rp: the plasma edge; lnRp: its logarithm as DD."""
        self.Rp = LD(Rp)
        self.r = np.concatenate([[LD(0)], self._r0.astype(LD), [self.Rp]])
        self.psi = dd_cat([self._psi_axis, self._psi, self.Q * DD.of(lnRp) * (-Q_ION)])
        self.dpsi = np.concatenate([[LD(0)], self._dpsi,
                                    [-Q_ION * self.Q.ld()[0] / self.Rp]])
        return self

    def at(self, rho, lnrho):
        """Ion psi (DD) and d_rho psi (80-bit) at radii rho (lnrho: their
        logarithms as DD): linear interpolation between the bracketing
        nodes, j = last node with r_j < rho (Key algorithmic adjustments),
        psi as the lower node's value plus t times the step; exact exterior
        field beyond the plasma edge."""
        rho_l = np.asarray(rho).astype(LD)
        j = np.searchsorted(self.r, rho_l, side="left") - 1
        outside = j >= len(self.r) - 1
        jj = np.clip(j, 0, len(self.r) - 2)
        r_lo, r_hi = self.r[jj], self.r[jj + 1]
        t = (rho_l - r_lo) / (r_hi - r_lo)
        psi = self.psi[jj] + (self.psi[jj + 1] - self.psi[jj]) * DD.of(t)
        dpsi = (1 - t) * self.dpsi[jj] + t * self.dpsi[jj + 1]
        if np.any(outside):
            ext = DD.of(lnrho)[outside] * self.Q * (-Q_ION)
            psi.hi[outside] = ext.hi
            psi.lo[outside] = ext.lo
            dpsi[outside] = -Q_ION * self.Q.ld()[0] / rho_l[outside]
        return psi, dpsi


# ---------------------------------------------------------------------------
# sources (Sec. "Numerical integration of wakefields": B_theta^(b) from the
# beam charge; Fig. 2 "gather sources")
# ---------------------------------------------------------------------------
class BeamTable:
    """Per-slice radial charge table of all particle beams (reading R12).

    Lambda_n(rho) = (1/(2 pi dxi)) sum_{k: r_k<rho} q_k w_k c_{k,n}
    with c_{k,n} the linear weight of particle k on node n; then
    B^(b)(rho) = Lambda_n(rho) / rho  (Gauss law of the beam equation).
    """

    def __init__(self, beams, dxi, n_xi):
        self.n_xi = n_xi
        nodes, rs, qs = [], [], []
        for b in beams:
            x, y = np.asarray(b.x, np.float64), np.asarray(b.y, np.float64)
            r = np.sqrt(x * x + y * y)
            t = np.asarray(b.xi, np.float64) / dxi
            n0 = np.floor(t)
            f = t - n0
            qw = b.q * np.asarray(b.w, np.float64)
            for node, c in ((n0, 1.0 - f), (n0 + 1.0, f)):
                keep = (node >= 0) & (node <= n_xi - 1) & (c > 0)
                nodes.append(node[keep].astype(np.int64))
                rs.append(r[keep])
                qs.append(qw[keep] * c[keep])
        if nodes:
            node = np.concatenate(nodes)
            r = np.concatenate(rs)
            qc = np.concatenate(qs)
        else:
            node = np.zeros(0, np.int64)
            r = np.zeros(0)
            qc = np.zeros(0)
        order = np.lexsort((r, node))
        self.node, self.r, self.qc = node[order], r[order], qc[order]
        self.off = np.searchsorted(self.node, np.arange(n_xi + 1), side="left")
        self.inv = LD(1) / (LD(2) * LD(math.pi) * LD(dxi))

    def lam(self, n, rho):
        lo, hi = self.off[n], self.off[n + 1]
        if hi == lo:
            return np.zeros_like(rho)
        cum = np.cumsum(self.qc[lo:hi].astype(LD)) * self.inv
        cnt = np.searchsorted(self.r[lo:hi], rho, side="left")
        out = np.zeros(rho.shape, LD)
        nz = cnt > 0
        out[nz] = cum[cnt[nz] - 1]
        return out.astype(np.float64)


def analytic_lambda(src, xi, rho):
    """Charge within rho of a bi-Gaussian beam per unit xi and radian."""
    s2 = src.sigma_r ** 2
    lon = math.exp(-((xi - src.xi_c) ** 2) / (2.0 * src.sigma_xi ** 2))
    return src.q * src.n_peak * lon * s2 * (-np.expm1(-rho * rho / (2.0 * s2)))


def laser_terms(src, xi, rho):
    """|a|^2 and d_rho |a|^2 of a frozen Gaussian envelope (reading R13)."""
    lon = math.exp(-2.0 * (xi - src.xi_l) ** 2 / (src.L ** 2))
    a2 = src.a0 ** 2 * np.exp(-2.0 * rho * rho / (src.w0 ** 2)) * lon
    return a2, -(4.0 * rho / (src.w0 ** 2)) * a2


# ---------------------------------------------------------------------------
# the per-slice steps
# ---------------------------------------------------------------------------
def ring_log(rho, r0, lnr0):
    """ln(rho) of rings whose initial radius is r0 (lnr0 = ln r0 as DD),
    evaluated as ln r0 + log1p((rho - r0)/r0) with the log1p in 80-bit
    arithmetic (reading R14): the psi sums multiply ln rho by the enclosed
    charge, so its rounding must scale with the ring's displacement, not
    with |ln rho|.  Returns DD."""
    r0_l = np.asarray(r0).astype(LD)
    return DD.of(lnr0) + np.log1p((np.asarray(rho).astype(LD) - r0_l) / r0_l)


def psi_family(rho, w, wh, ions, r0, lnr0):
    """psi and d_rho psi at sorted electron rings plus the ion species
    (eqs. dpsi_dr, psi; species summed after interpolation, R11).  r0 are
    the rings' initial radii, lnr0 their logarithms (DD).  Returns binary64
    (psi, dpsi, psi_axis)."""
    rho_l = rho.astype(LD)
    lnr = ring_log(rho, r0, lnr0)
    psi_e, dpsi_e, axis_e = _gauss_log_sums(rho_l, w, wh, Q_E, lnr)
    psi_i, dpsi_i = ions.at(rho_l, lnr)
    psi = (psi_e + psi_i).f64()
    dpsi = (dpsi_e + dpsi_i).astype(np.float64)
    axis = float((axis_e + ions.psi[0:1]).f64()[0])
    return psi, dpsi, axis


def local_quantities(psi, u, a2):
    """psibar = 1 - (q/m) psi and gamma from eq. plasma_particle_motion_4."""
    psibar = 1.0 - (Q_E / M_E) * psi
    gamma = (1.0 + u * u + psibar * psibar
             + (Q_E * Q_E) / (2.0 * M_E * M_E) * a2) / (2.0 * psibar)
    return psibar, gamma


def dzeta_psi(rho, u, w, wh, psibar):
    """d_zeta psi at sorted rings (eq. dpsi_dzeta with reading R2, R6):
    sum over the rings outside of q w u/(rho psibar), ring itself with
    weight w - w^.  Returns (dzpsi at rings, dzpsi on the axis)."""
    c = (Q_E * u / (rho * psibar)).astype(LD)
    term = w.astype(LD) * c
    rsum = suffix_sum(term).ld()
    above = np.concatenate([rsum[1:], np.zeros(1, LD)])
    own = (w - wh).astype(LD) * c
    return (above + own).astype(np.float64), float(rsum[0]) if len(rsum) else 0.0


def coefficients(rho, u, w, psibar, gamma, dpsi, dzpsi, bb, da2, q=Q_E, m=M_E):
    """A_i, B_i, C_i of eqs. b_coeffs_1-3 (readings R3, R4)."""
    wr = w / rho
    A = wr * (q * q / m) / psibar
    B = (-wr * (q * q / m) * gamma * dpsi / psibar ** 2
         + wr * (q * q / m) * bb / psibar
         - wr * (q ** 3 / (4.0 * m * m)) * da2 / psibar ** 2
         - q * w / rho ** 2 * u * u / psibar ** 2
         + wr * (q * q / m) * u * u * dpsi / psibar ** 3
         - wr * (q * q / m) * u * dzpsi / psibar ** 2)
    C = q * wr * (gamma / psibar - 1.0) - q * wr * u * u / psibar ** 2
    return A, B, C


def transfer(A, B, C, rho):
    """Matrix M_i and offset s_i of eq. ai_bi: x_i = M_i x_{i-1} + s_i."""
    M = np.empty((len(rho), 2, 2))
    M[:, 0, 0] = 1.0 + A * rho / 2.0
    M[:, 0, 1] = A / (2.0 * rho)
    M[:, 1, 0] = -A * rho ** 3 / 2.0
    M[:, 1, 1] = 1.0 - A * rho / 2.0
    s = np.empty((len(rho), 2))
    s[:, 0] = (2.0 * B + A * C) / 4.0
    s[:, 1] = rho * (4.0 * C - 2.0 * B * rho - A * C * rho) / 4.0
    return M, s


def _recursion_banded(M, s):
    """Banded storage and right-hand side of eq. ai_bi with b_0 = 0, a_N = 0."""
    n = M.shape[0]
    nu = 2 * n + 2
    # banded storage with 2 lower and 1 upper diagonals: entry (row r,
    # column c) sits at ab[1 + r - c, c]
    ab = np.zeros((4, nu))
    rhs = np.zeros(nu)
    i = np.arange(1, n + 1)
    ra, rb = 2 * i - 1, 2 * i          # rows of the a_i and b_i equations
    ca, cb = 2 * i - 2, 2 * i - 1      # columns of a_{i-1}, b_{i-1}
    ab[1 + 0 - 1, 1] = 1.0                                   # b_0 = 0
    ab[1 + ra - ca, ca] = -M[:, 0, 0]
    ab[1 + ra - cb, cb] = -M[:, 0, 1]
    ab[1 + ra - 2 * i, 2 * i] = 1.0
    ab[1 + rb - ca, ca] = -M[:, 1, 0]
    ab[1 + rb - cb, cb] = -M[:, 1, 1]
    ab[1 + rb - (2 * i + 1), 2 * i + 1] = 1.0
    rhs[ra] = s[:, 0]
    rhs[rb] = s[:, 1]
    ab[1 + (nu - 1) - 2 * n, 2 * n] = 1.0                    # a_N = 0
    return ab, rhs


def _recursion_residual(M, s, a, b):
    """Residual of eq. ai_bi and the boundary rows in 80-bit arithmetic."""
    L = np.longdouble
    a, b = a.astype(L), b.astype(L)
    Ml, sl = M.astype(L), s.astype(L)
    r = np.zeros(2 * M.shape[0] + 2, dtype=L)
    r[0] = -b[0]
    r[1:-1:2] = sl[:, 0] - (a[1:] - Ml[:, 0, 0] * a[:-1] - Ml[:, 0, 1] * b[:-1])
    r[2:-1:2] = sl[:, 1] - (b[1:] - Ml[:, 1, 0] * a[:-1] - Ml[:, 1, 1] * b[:-1])
    r[-1] = -a[-1]
    return r


def solve_recursion(M, s, refine: int = 2):
    """Solve x_i = M_i x_{i-1} + s_i (i=1..N) with b_0 = 0 and a_N = 0
    (eq. ai_bi) as one banded linear system in (a_0, b_0, ..., a_N, b_N),
    by banded LU, then `refine` steps of iterative refinement with residuals
    accumulated in 80-bit arithmetic (the binary64 LU alone loses digits with
    the system's conditioning at large N; R15).  Returns arrays a, b of
    length N+1."""
    ab, rhs = _recursion_banded(M, s)
    z = solve_banded((2, 1), ab, rhs)
    a, b = z[0::2].copy(), z[1::2].copy()
    if refine:
        az, bz = a.astype(np.longdouble), b.astype(np.longdouble)
        for _ in range(refine):
            r = _recursion_residual(M, s, a, b)
            d = solve_banded((2, 1), ab, r.astype(np.float64))
            az += d[0::2]
            bz += d[1::2]
            a, b = az.astype(np.float64), bz.astype(np.float64)
    return a, b


def solve_shooting(M, s):
    """The paper's appendix procedure: a_i = K_i a_0 + T_i, b_i = U_i a_0 + P_i
    with (K,U) from (1,0) and (T,P) from (0,0), then a_0 = -T_N/K_N."""
    n = M.shape[0]
    KU = np.zeros((n + 1, 2)); KU[0] = (1.0, 0.0)
    TP = np.zeros((n + 1, 2))
    for i in range(1, n + 1):
        KU[i] = M[i - 1] @ KU[i - 1]
        TP[i] = M[i - 1] @ TP[i - 1] + s[i - 1]
    a0 = -TP[n, 0] / KU[n, 0]
    return KU[:, 0] * a0 + TP[:, 0], KU[:, 1] * a0 + TP[:, 1]


def b_plasma_at_rings(a, b, rho, C, w, wh):
    """B^(p) at ring i: the inner-side value a_{i-1} rho_i + b_{i-1}/rho_i
    (eq. b_theta_plasma) plus the fraction w^/w of its jump C_i (R6)."""
    return a[:-1] * rho + b[:-1] / rho + (wh / w) * C


def forces(u, psibar, gamma, dpsi, bt, da2, q=Q_E, m=M_E):
    """Right-hand sides in xi = -zeta of eqs. plasma_particle_motion_1-2
    (reading R3 for the ponderomotive term)."""
    f_rho = u / psibar
    f_u = -((q / m) * (gamma * dpsi / psibar - bt)
            + (q * q) / (4.0 * m * m) * da2 / psibar)
    return f_rho, f_u


def push_ab2(rho, u, fr, fu, fr_p, fu_p, dxi):
    """One second-order Adams-Bashforth step of (rho, u_r) in xi
    (eqs. plasma_particle_motion_1-2; Sec. "Integration into Wake-T"): x +=
    dxi (3/2 f - 1/2 f_prev).  A ring pushed to a negative radius is
    reflected through the axis (reading R9): rho, u_r and the derivatives
    kept as the next step's history change sign.  Returns (rho, u, f_rho,
    f_u) after the step, the last two being the history to keep."""
    rho_n = rho + dxi * (1.5 * fr - 0.5 * fr_p)
    u_n = u + dxi * (1.5 * fu - 0.5 * fu_p)
    frs, fus = np.array(fr, np.float64), np.array(fu, np.float64)
    neg = rho_n < 0                                                   # R9
    rho_n[neg] = -rho_n[neg]
    u_n[neg] = -u_n[neg]
    frs[neg] = -frs[neg]
    fus[neg] = -fus[neg]
    return rho_n, u_n, frs, fus


def grid_radii(n_r, r_max):
    """Nodes of a uniform radial field grid: cell centres (g + 1/2) dr_g,
    dr_g = r_max / n_r (reading R17)."""
    dg = float(r_max) / int(n_r)
    return (np.arange(int(n_r), dtype=np.float64) + 0.5) * dg


def chi_volumes(radii):
    """V_g = integral over rho of W_g(rho) rho for the hat weights of reading
    R20 on ascending nodes r_g (80-bit).  Below the first node W_0 = 1; above
    the last node its hat ends at r_{n-1} + (r_{n-1} - r_{n-2}) (2 r_0 for a
    single node)."""
    r = np.asarray(radii).astype(LD)
    n = len(r)
    top = r[-1] + (r[-1] - r[-2]) if n > 1 else 2 * r[0]
    lo = np.concatenate([[LD(0)], r[:-1]])
    hi = np.concatenate([r[1:], [top]])
    # integral of (rho - a)/(b - a) rho over [a, b] is (b - a)(a + 2b)/6;
    # of (c - rho)/(c - b) rho over [b, c] is (c - b)(2b + c)/6
    lower = (r - lo) * (lo + 2 * r) / 6
    lower[0] = r[0] * r[0] / 2
    upper = (hi - r) * (2 * r + hi) / 6
    return lower + upper


def chi_deposit(rho, c, radii):
    """chi at ascending nodes from rings at radii rho carrying c_j = w_j /
    psibar_j (reading R20): for each node, the sum over the rings in the
    support of its hat of c_j W_g(rho_j), over V_g.  80-bit sums."""
    r = np.asarray(radii).astype(LD)
    rho = np.asarray(rho).astype(LD)
    c = np.asarray(c).astype(LD)
    n = len(r)
    top = r[-1] + (r[-1] - r[-2]) if n > 1 else 2 * r[0]
    V = chi_volumes(radii)
    out = np.zeros(n, LD)
    for g in range(n):
        lo = r[g - 1] if g > 0 else LD(0)
        hi = r[g + 1] if g + 1 < n else top
        below = (rho >= lo) & (rho < r[g]) if g > 0 else (rho < r[g])
        above = (rho >= r[g]) & (rho < hi)
        wl = (rho[below] - lo) / (r[g] - lo) if g > 0 else np.ones(int(np.sum(below)), LD)
        wu = (hi - rho[above]) / (hi - r[g])
        out[g] = (np.sum(c[below] * wl) + np.sum(c[above] * wu)) / V[g]
    return out


# ---------------------------------------------------------------------------
# driver (Fig. 2 right column)
# ---------------------------------------------------------------------------
class RingOracle:
    """One instance: ring set, slice grid and frozen sources."""

    def __init__(self, r0, dr, dxi, n_xi, sources=(), dens=None):
        self.r0 = np.asarray(r0, np.float64)
        self.dr = np.asarray(dr, np.float64)
        self.N = len(self.r0)
        self.dxi = float(dxi)
        self.n_xi = int(n_xi)
        self.w, self.wh = ring_weights(self.r0, self.dr, dens)
        self.Rp = float(self.r0[-1] + self.dr[-1] / 2.0)
        self.lnr0 = dd_log(self.r0)
        self.ions = IonNodes(self.r0, self.w, self.wh, self.lnr0).finish(self.Rp, dd_log([self.Rp]))
        self._grid_logs = {}
        beams = [s for s in sources if getattr(s, "kind", "") == "particles"]
        self.analytic = [s for s in sources if getattr(s, "kind", "") == "gaussian"]
        self.lasers = [s for s in sources if getattr(s, "kind", "") == "laser"]
        self.table = BeamTable(beams, self.dxi, self.n_xi)

    def initial_state(self):
        z = np.zeros(self.N)
        return dict(rho=self.r0.copy(), u=z.copy(), fr=z.copy(), fu=z.copy())

    def sources_at(self, n, rho):
        xi = n * self.dxi
        lam = self.table.lam(n, rho)
        for s in self.analytic:
            lam = lam + analytic_lambda(s, xi, rho)
        bb = lam / rho
        a2 = np.zeros_like(rho)
        da2 = np.zeros_like(rho)
        for s in self.lasers:
            x, dx = laser_terms(s, xi, rho)
            a2 = a2 + x
            da2 = da2 + dx
        return bb, a2, da2

    def slice(self, n, state, push=True, keep=False):
        """Fields at slice n and the state pushed to slice n+1.
        ``state`` arrays are indexed by ring id.  Returns (out, new_state)
        with out['status'] = 0 or BREAKDOWN."""
        ids = np.lexsort((np.arange(self.N), state["rho"]))          # R7
        rho = state["rho"][ids]
        u = state["u"][ids]
        w, wh = self.w[ids], self.wh[ids]
        bb, a2, da2 = self.sources_at(n, rho)
        psi, dpsi, psi_axis = psi_family(rho, w, wh, self.ions, self.r0[ids], self.lnr0[ids])
        psibar, gamma = local_quantities(psi, u, a2)
        out = dict(status=0)
        if not np.all(psibar > 0) or not np.all(np.isfinite(psibar)):  # R10
            out["status"] = BREAKDOWN
            return out, None
        dzpsi, dz_axis = dzeta_psi(rho, u, w, wh, psibar)
        A, B, C = coefficients(rho, u, w, psibar, gamma, dpsi, dzpsi, bb, da2)
        M, s = transfer(A, B, C, rho)
        a, b = solve_recursion(M, s)
        bp = b_plasma_at_rings(a, b, rho, C, w, wh)
        bt = bb + bp
        new = None
        fr = fu = None
        if push:
            fr, fu = forces(u, psibar, gamma, dpsi, bt, da2)
            if n == 0:                                                # R8
                fr_p, fu_p = fr, fu
            else:
                fr_p, fu_p = state["fr"][ids], state["fu"][ids]
            rho_n, u_n, frs, fus = push_ab2(rho, u, fr, fu, fr_p, fu_p, self.dxi)
            new = {k: np.empty(self.N) for k in ("rho", "u", "fr", "fu")}
            new["rho"][ids], new["u"][ids] = rho_n, u_n
            new["fr"][ids], new["fu"][ids] = frs, fus
        check = [psi, dpsi, dzpsi, bt]
        if new is not None:
            check += [new["rho"], new["u"]]
        if not all(np.all(np.isfinite(c)) for c in check):             # R10
            out["status"] = BREAKDOWN
            return out, None

        def by_id(x):
            y = np.empty(self.N)
            y[ids] = x
            return y

        out.update(psi=by_id(psi), er_bt=by_id(-dpsi), ez=by_id(-dzpsi),
                   bt=by_id(bt), rho=by_id(rho), u=by_id(u),
                   psi_axis=psi_axis, ez_axis=-dz_axis)
        if keep:
            out.update(order=ids, A=A, B=B, C=C, M=M, s=s, a=a, b=b,
                       bb=bb, a2=a2, da2=da2, psibar=psibar, gamma=gamma,
                       dpsi_sorted=dpsi, dzpsi_sorted=dzpsi, bp=bp)
        return out, new

    def fields_at(self, n, out, radii):
        """psi, E_r - B_theta, E_z and B_theta of slice n at arbitrary radii
        r > 0 (Sec. "Numerical integration of wakefields": eqs. psi, dpsi_dr,
        dpsi_dzeta and b_theta_plasma hold at any radius of the column once
        the rings are known; Fig. 2, fields on an external grid).  ``out``
        is the slice's result with keep=True.  A radius with k rings
        strictly inside it lies in interval k of the recursion: a ring at
        exactly r counts as outside (reading R17).  Returns a dict of
        binary64 arrays."""
        ids = out["order"]
        rho = out["rho"][ids]
        u = out["u"][ids]
        w = self.w[ids]
        r = np.asarray(radii, np.float64)
        k = np.searchsorted(rho, r, side="left")
        key = r.tobytes()
        if key not in self._grid_logs:
            self._grid_logs = {key: dd_log(r)}
        lnr_g = self._grid_logs[key]
        lnr_k = ring_log(rho, self.r0[ids], self.lnr0[ids])           # R14
        S = dd_cat([DD(0.0), prefix_sum(w)])                          # sum_{j<k} w_j
        T = dd_cat([suffix_sum(lnr_k * w), DD(0.0)])                  # sum_{j>=k} w ln rho
        r_l = r.astype(LD)
        psi_e = (S[k] * lnr_g + T[k]) * (-Q_E)                        # eq. psi
        dpsi_e = -Q_E * S[k].ld() / r_l                               # eq. dpsi_dr
        psi_i, dpsi_i = self.ions.at(r_l, lnr_g)                      # R11
        c = w.astype(LD) * (Q_E * u / (rho * out["psibar"])).astype(LD)
        V = np.concatenate([suffix_sum(c).ld(), np.zeros(1, LD)])     # eq. dpsi_dzeta, R2
        bb, _, _ = self.sources_at(n, r)
        bt = bb + out["a"][k] * r + out["b"][k] / r                   # eq. b_theta_plasma
        return dict(psi=(psi_e + psi_i).f64(),
                    er_bt=(-(dpsi_e + dpsi_i)).astype(np.float64),
                    ez=(-V[k]).astype(np.float64), bt=bt)

    def chi_at(self, out, radii):
        """chi = n/gamma of slice n deposited at ascending grid radii
        (reading R20; Fig. 2 "deposit chi in laser grid").  ``out`` is the
        slice's result with keep=True.  Returns binary64."""
        ids = out["order"]
        rho = out["rho"][ids]
        c = self.w[ids].astype(LD) / np.asarray(out["psibar"]).astype(LD)
        return chi_deposit(rho, c, radii).astype(np.float64)

    def run(self, first=0, count=None, state=None, record_stride=1, grid=None):
        """March slices [first, first+count).  Returns a dict with per-slice
        on-axis lineouts, snapshots every ``record_stride`` slices (by ring
        id), the final state and the breakdown slice (-1 if none); with
        ``grid = (n_r, r_max)`` also the fields at the grid_radii nodes of
        every slice, 'grid' of shape [count][4][n_r] (psi, E_r - B_theta,
        E_z, B_theta), and chi there, 'chi' of shape [count][n_r]."""
        if count is None:
            count = self.n_xi - first
        if state is None:
            state = self.initial_state()
        rec = {}
        axis = np.full((count, 2), np.nan)
        gr = None if grid is None else grid_radii(*grid)
        gfield = None if grid is None else np.full((count, 4, len(gr)), np.nan)
        gchi = None if grid is None else np.full((count, len(gr)), np.nan)
        breakdown = -1
        for k in range(count):
            n = first + k
            out, new = self.slice(n, state, push=(n < self.n_xi - 1), keep=grid is not None)
            if out["status"] != 0:
                breakdown = n
                break
            axis[k] = (out["psi_axis"], out["ez_axis"])
            if grid is not None:
                f = self.fields_at(n, out, gr)
                gfield[k] = [f["psi"], f["er_bt"], f["ez"], f["bt"]]
                gchi[k] = self.chi_at(out, gr)
            if record_stride and (n % record_stride == 0 or k == count - 1):
                rec[n] = {q: out[q] for q in ("psi", "er_bt", "ez", "bt", "rho", "u")}
            if new is not None:
                state = new
        res = dict(axis=axis, snap=rec, state=state, breakdown=breakdown)
        if grid is not None:
            res["grid"] = gfield
            res["chi"] = gchi
        return res
