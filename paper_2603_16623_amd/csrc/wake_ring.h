// Per-ring algebra of the electron rings and the beam-table count, shared by
// the one-species marcher and the two-species (mobile-ion) marcher.
#pragma once
#include "wake_device.h"

// ---------------------------------------------------------------------------
// per-ring algebra
// ---------------------------------------------------------------------------
struct Local {
  double pb, ipb, gm, v, A;
};

// psibar, 1/psibar, gamma (eq. motion_4), v = w u/(rho psibar), A_i
__device__ __forceinline__ Local local_of(double irho, double u, double w, double psi, double a2) {
  Local L;
  L.pb = 1.0 + psi;
  L.ipb = rcp_nr(L.pb);
  L.gm = (1.0 + u * u + L.pb * L.pb + 0.5 * a2) * (0.5 * L.ipb);
  L.v = w * u * irho * L.ipb;
  L.A = w * irho * L.ipb;
  return L;
}

// B_i and C_i of eqs. b_coeffs_2-3 for an electron ring (q=-1, m=1)
__device__ __forceinline__ void ring_BC(double irho, double u, double w, const Local& L, double dpsi,
                                        double dz, double bb, double da2, double& B, double& C) {
  const double wr = w * irho;
  const double ipb2 = L.ipb * L.ipb;
  const double u2 = u * u;
  B = -wr * L.gm * dpsi * ipb2 + wr * bb * L.ipb + 0.25 * wr * da2 * ipb2 + wr * irho * u2 * ipb2 +
      wr * u2 * dpsi * ipb2 * L.ipb - wr * u * dz * ipb2;
  C = -wr * (L.gm * L.ipb - 1.0) + wr * u2 * ipb2;
}

// offset s_i of eq. ai_bi
__device__ __forceinline__ void rec_offset(double A, double B, double C, double rho, double& sa,
                                          double& sb) {
  sa = (2.0 * B + A * C) * 0.25;
  sb = rho * (4.0 * C - 2.0 * B * rho - A * C * rho) * 0.25;
}

// transfer matrix M_i of eq. ai_bi (det M_i = 1)
__device__ __forceinline__ Pack<4> rec_matrix(double A, double rho, double irho) {
  const double h = 0.5 * A * rho;
  return {{1.0 + h, 0.5 * A * irho, -h * rho * rho, 1.0 - h}};
}

__device__ __forceinline__ Pack<4> mat_adj(const Pack<4>& m) {
  return {{m.v[3], -m.v[1], -m.v[2], m.v[0]}};
}

// a / b for double-double a with a precomputed reciprocal ib = 1/b
__device__ __forceinline__ dd dd_div_rcp(dd a, double b, double ib) {
  _Pragma("clang fp contract(off)")
  const double q1 = a.hi * ib;
  const dd r = dd_sub(a, two_prod(q1, b));
  const double q2 = r.hi * ib;
  return fast_two_sum(q1, q2);
}

// Number of entries of the ascending table br[0..m) below r, given that
// the first lo entries are below r: galloping from lo (gallop) or a plain
// binary search of [lo, m).
template <class P>
__device__ __forceinline__ int count_below(P br, int lo, int m, double r, bool gallop) {
  int a, b;
  if (gallop) {
    if (lo >= m || !(br[lo] < r)) return lo;
    a = lo;                            // br[a] < r
    int step = 1;
    for (;;) {
      b = a + step;
      if (b >= m) { b = m; break; }
      if (!(br[b] < r)) break;
      a = b;
      step <<= 1;
    }
    a += 1;                            // answer in [a, b]
  } else {
    a = lo;
    b = m;
  }
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (br[mid] < r) a = mid + 1; else b = mid;
  }
  return a;
}
// The same count for radii met in descending order: hi is the count of the
// previous (larger) radius when gallop is set.
template <class P>
__device__ __forceinline__ int count_below_down(P br, int hi, int m, double r, bool gallop) {
  int a, b;
  if (gallop) {
    if (hi <= 0 || br[hi - 1] < r) return hi;
    b = hi - 1;                        // br[b] >= r: the answer is at most b
    int step = 1;
    for (;;) {
      a = b - step;
      if (a < 0) { a = 0; break; }
      if (br[a] < r) { a += 1; break; }
      b = a;
      step <<= 1;
    }
  } else {
    a = 0;
    b = m;
  }
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (br[mid] < r) a = mid + 1; else b = mid;
  }
  return a;
}
