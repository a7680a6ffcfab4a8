// gfx950 marcher of the two-species gridless model: plasma electrons and
// mobile ions, each discretised into rings (paper, Sec. "Gridless
// quasistatic model" and "Key algorithmic adjustments": every species is
// summed on its own at its own rings, the fields of the other species are
// interpolated linearly between that species' rings, and the ion currents
// are left out of B_theta^(p)).
//
// One workgroup of 1024 threads marches one instance through its slices.
// Per species, thread t owns the C = ceil(N / 1024) consecutive sorted
// positions [tC, tC + C); per-position arrays are stored by slot
// (p % C) * 1024 + p / C, so the k-th positions of a wave are contiguous.
// The sorted radii of both species sit in LDS, where the interval searches
// of the gathers run; node tables, per-position work and ring state live in
// device memory.
//
// Per slice:
//   order    each species' (rho, id) order: the previous one if it still
//            holds, else rounds of wave blocks of 256 positions sorted in
//            LDS and the blocks between them merged (the bitonic network
//            over all positions after three rounds that leave disorder);
//   sums     own psi and d_rho psi at each species' rings (eqs. psi,
//            dpsi_dr; double-double prefix of w and suffix of w ln rho, the
//            ring itself with w^), its axis value, outer edge and exterior
//            field: the node tables;
//   gather   the other species' psi and d_rho psi interpolated at every
//            ring; psibar and gamma with the species' q and m (eq.
//            plasma_particle_motion_4); beam and laser sources; own d_zeta
//            psi (eq. dpsi_dzeta, suffix of q w u / (rho psibar)), then the
//            other species' interpolated;
//   B^(p)    electrons only: A, B, C (eqs. b_coeffs_1-3), the two-point
//            recursion (eq. ai_bi) in Green's-function form (growing mode g,
//            decaying mode h, W = det[g, h], x_i = (h_i E_i - g_i D_i) / W)
//            and B^(p) at the electron rings (eq. b_theta_plasma); the ions
//            take it interpolated between the electron rings;
//   push     fields out, Adams-Bashforth-2 push (eqs.
//            plasma_particle_motion_1-2) of both species with their q and m,
//            reflection through the axis, into the other state buffer.
#include "wake_common.h"
#include "wake_device.h"
#include "wake_ring.h"
#include "wake_ions.h"

#include <math.h>

namespace {

constexpr int NT = WAKE_IONS_NT;
constexpr int NW = NT / 64;
constexpr int NMAX = WAKE_IONS_NMAX;

// dynamic LDS: sorted radii of both species, sort ids, scan area, slice
// constants (analytic source factors, then 16 scalars per species), the
// slice's beam-table radii (when at most WAKE_BCAP of them)
struct IonsLds {
  static constexpr size_t r_off = 0;
  static constexpr size_t id_off = r_off + (size_t)2 * NMAX * sizeof(double);
  static constexpr size_t scan_off = id_off + (size_t)NMAX * sizeof(uint16_t);
  static constexpr size_t misc_off = scan_off + (size_t)NW * 16 * sizeof(double);
  static constexpr size_t br_off = misc_off + 64 * sizeof(double);
  static constexpr size_t bytes = br_off + (size_t)WAKE_BCAP * sizeof(double);
};
static_assert(IonsLds::bytes <= 160 * 1024, "two-species LDS");

// per-species scalars of a slice (at s_misc + 32 + 16 s): psi(0) of the
// species alone (dd), total weight (dd), outer edge, exterior psi at the
// edge (dd), exterior d_rho psi at the edge (dd), d_zeta psi(0) of the species
// alone (dd)
enum { SC_PAH = 0, SC_PAL, SC_QH, SC_QL, SC_EDGE, SC_EPH, SC_EPL, SC_EDP, SC_EDL, SC_DZH, SC_DZL,
       SC_N = 16 };

__device__ __forceinline__ unsigned pslot(int p, int C) { return (unsigned)((p % C) * NT + p / C); }

// Bitonic sort of the keys (kr, ki) of n positions in place (n <= NMAX),
// padded with +inf keys to the next power of two.
__device__ void bitonic_ions(double* kr, uint16_t* ki, int n) {
  int P = 1;
  while (P < n) P <<= 1;
  for (int i = n + (int)threadIdx.x; i < P; i += NT) { kr[i] = INFINITY; ki[i] = 0xFFFF; }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += NT) {
        const int l = i ^ j;
        if (l > i) {
          const double a = kr[i], b = kr[l];
          const uint16_t ia = ki[i], ib = ki[l];
          const bool up = (i & k) == 0;
          const bool sw = up ? key_lt(b, (int32_t)ib, a, (int32_t)ia) : key_lt(a, (int32_t)ia, b, (int32_t)ib);
          if (sw) { kr[i] = b; kr[l] = a; ki[i] = ib; ki[l] = ia; }
        }
      }
      __syncthreads();
    }
  }
}

// (rho, id) order of keys with the id in k (no short-circuit: straight-line
// selects)
__device__ __forceinline__ bool ik_lt(double ra, uint32_t ka, double rb, uint32_t kb) {
  return (ra < rb) | ((ra == rb) & (ka < kb));
}
__device__ __forceinline__ void ik_swap(double& ra, uint32_t& ka, double& rb, uint32_t& kb) {
  const double t = ra; ra = rb; rb = t;
  const uint32_t u = ka; ka = kb; kb = u;
}
// the wave's keys of positions [b0, b0 + 256) (four per lane, +inf past n)
__device__ __forceinline__ void ik_load(const double* kr, const uint16_t* ki, int b0, int n, double* r,
                                        uint32_t* k) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = b0 + 4 * lane + j;
    r[j] = p < n ? kr[p] : INFINITY;
    k[j] = p < n ? (uint32_t)ki[p] : 0xffffffffu;
  }
}
__device__ __forceinline__ void ik_store(double* kr, uint16_t* ki, int b0, int n, const double* r,
                                         const uint32_t* k) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = b0 + 4 * lane + j;
    if (p < n) { kr[p] = r[j]; ki[p] = (uint16_t)k[j]; }
  }
}
// whether the wave's 256 keys are in order
__device__ __forceinline__ bool ik_sorted(const double* r, const uint32_t* k) {
  const int lane = threadIdx.x & 63;
  const double xr = lane_next(r[0]);
  const uint32_t xk = lane_next(k[0]);
  const bool ok = (lane == 63 || !ik_lt(xr, xk, r[3], k[3])) && !ik_lt(r[1], k[1], r[0], k[0]) &&
                  !ik_lt(r[2], k[2], r[1], k[1]) && !ik_lt(r[3], k[3], r[2], k[2]);
  return __all(ok);
}
// compare-exchange stage of a bitonic network at distance d over the wave's
// 256 keys (position 4 lane + j), ascending where (position & kk) == 0
__device__ __forceinline__ void ik_stage(double* r, uint32_t* k, int kk, int d) {
  const int lane = threadIdx.x & 63;
  if (d >= 4) {                       // partner in lane ^ (d / 4), same register
    const int lm = d >> 2;
    const bool lower = (lane & lm) == 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double pr = lane_xor(r[j], lm);
      const uint32_t pq = lane_xor(k[j], lm);
      const bool up = ((4 * lane + j) & kk) == 0;
      if (ik_lt(pr, pq, r[j], k[j]) == (lower == up)) { r[j] = pr; k[j] = pq; }
    }
  } else {                            // partner in this lane
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j & d) continue;
      const int jj = j | d;
      const bool up = ((4 * lane + j) & kk) == 0;
      if (ik_lt(r[jj], k[jj], r[j], k[j]) == up) ik_swap(r[j], k[j], r[jj], k[jj]);
    }
  }
}

// One wave puts positions [b0, b0 + 256) (clipped at n) of the keys in LDS
// in order, in place: odd-even transposition first (a ring displaced by L
// positions is in place after L phases; the order is checked every four
// phases), the full bitonic network after 32 phases.
__device__ void ions_sort_block(double* kr, uint16_t* ki, int b0, int n) {
  const int lane = threadIdx.x & 63;
  double r[4];
  uint32_t k[4];
  ik_load(kr, ki, b0, n, r, k);
  if (ik_sorted(r, k)) return;
  #pragma unroll 1
  for (int it = 0; it < 8; ++it) {
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
      if (ik_lt(r[1], k[1], r[0], k[0])) ik_swap(r[0], k[0], r[1], k[1]);
      if (ik_lt(r[3], k[3], r[2], k[2])) ik_swap(r[2], k[2], r[3], k[3]);
      if (ik_lt(r[2], k[2], r[1], k[1])) ik_swap(r[1], k[1], r[2], k[2]);
      const double nr = lane_next(r[0]), pr = lane_prev(r[3]);
      const uint32_t nq = lane_next(k[0]), pq = lane_prev(k[3]);
      const bool take_next = lane < 63 && ik_lt(nr, nq, r[3], k[3]);    // keep the smaller
      const bool take_prev = lane > 0 && ik_lt(r[0], k[0], pr, pq);     // keep the larger
      if (take_next) { r[3] = nr; k[3] = nq; }
      if (take_prev) { r[0] = pr; k[0] = pq; }
    }
    if (ik_sorted(r, k)) {
      ik_store(kr, ki, b0, n, r, k);
      return;
    }
  }
#pragma unroll
  for (int kk = 2; kk <= 256; kk <<= 1) {
#pragma unroll
    for (int d = kk >> 1; d > 0; d >>= 1) ik_stage(r, k, kk, d);
  }
  ik_store(kr, ki, b0, n, r, k);
}

// One wave merges positions [b0, b0 + 256) (clipped at n) whose halves are
// each in order: position i against 255 - i, then the half-cleaners of a
// bitonic merge.
__device__ void ions_merge_block(double* kr, uint16_t* ki, int b0, int n) {
  const int lane = threadIdx.x & 63;
  double r[4];
  uint32_t k[4];
  ik_load(kr, ki, b0, n, r, k);
  if (ik_sorted(r, k)) return;
  {
    double pr[4];
    uint32_t pq[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {       // lane 63 - lane, register 3 - j
      const uint64_t v = (uint64_t)__double_as_longlong(r[3 - j]);
      uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32), q = k[3 - j];
      lo = lane_xor(lane_xor(lane_xor(lane_xor(lane_xor(lane_xor(lo, 1), 2), 4), 8), 16), 32);
      hi = lane_xor(lane_xor(lane_xor(lane_xor(lane_xor(lane_xor(hi, 1), 2), 4), 8), 16), 32);
      q = lane_xor(lane_xor(lane_xor(lane_xor(lane_xor(lane_xor(q, 1), 2), 4), 8), 16), 32);
      pr[j] = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
      pq[j] = q;
    }
    const bool lower = lane < 32;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (ik_lt(pr[j], pq[j], r[j], k[j]) == lower) { r[j] = pr[j]; k[j] = pq[j]; }
  }
#pragma unroll
  for (int d = 64; d > 0; d >>= 1) ik_stage(r, k, 256, d);
  ik_store(kr, ki, b0, n, r, k);
}

// Order of n nearly sorted keys in LDS (position order), in place, in
// rounds: the wave blocks of 256 positions at 0, 256, ... sorted, those at
// 128, 384, ... (two sorted halves) merged, and the order checked at the
// junctions of the second blocks (every segment between them is sorted).
// A ring that moved more than 128 positions leaves a junction out of order
// for the next round; after three rounds the bitonic network sorts all
// positions.
__device__ void ions_fix_order(double* kr, uint16_t* ki, int n) {
  constexpr int NW = NT / 64;
  static_assert(NMAX <= 64 * 256, "a junction per lane");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  #pragma unroll 1
  for (int round = 0; round < 3; ++round) {
    #pragma unroll 1
    for (int b = wave; b * 256 < n; b += NW) ions_sort_block(kr, ki, b * 256, n);
    __syncthreads();
    #pragma unroll 1
    for (int b = wave; 256 * (b + 1) < n; b += NW) ions_merge_block(kr, ki, 128 + b * 256, n);
    __syncthreads();
    bool out = false;
    const int q = 128 + 256 * lane;
    if (q < n) out = ik_lt(kr[q], ki[q], kr[q - 1], ki[q - 1]);
    if (!__syncthreads_or(out)) return;     // also: every wave has read its junction keys
  }
  bitonic_ions(kr, ki, n);
}

// The interval of radius r among the nodes of species o (node 0 the axis,
// node j = its ring j-1, node N+1 its edge): the lower node is j = cnt, the
// number of its rings below r; t the fraction of the way to node j+1.
// Returns false beyond the edge.
struct Interval {
  int j;
  double t;
};
__device__ __forceinline__ bool interval_of(const double* ro, int N, double edge, double r, int cnt,
                                            Interval& iv) {
  iv.j = cnt;
  const double rl = cnt == 0 ? 0.0 : ro[cnt - 1];
  double rh;
  if (cnt < N) {
    rh = ro[cnt];
  } else {
    if (r > edge) { iv.t = 0.0; return false; }
    rh = edge;
  }
  iv.t = (r - rl) / (rh - rl);
  return true;
}

// ln rho of ring id at radius r as ln r0 + log1p((r - r0)/r0) (its rounding
// scales with the ring's displacement, not with |ln rho|)
__device__ __forceinline__ dd ring_log_id(const double* cst, int N, int id, double r) {
  return dd_add_d({cst[IK_LNH * N + id], cst[IK_LNL * N + id]},
                  log1p_fast((r - cst[IK_R0 * N + id]) * cst[IK_IR0 * N + id]));
}

// t of radius r in the node interval starting at node j of species o (the
// same expression as interval_of)
__device__ __forceinline__ double interval_t(const double* ro, int N, double edge, double r, int j) {
  const double rl = j == 0 ? 0.0 : ro[j - 1];
  const double rh = j < N ? ro[j] : edge;
  return (r - rl) / (rh - rl);
}

__global__ __launch_bounds__(NT) void ions_march_kernel(const WakeIons* __restrict__ insts) {
  const WakeIons& I = insts[blockIdx.x];
  double* const s_r = reinterpret_cast<double*>(wake_lds + IonsLds::r_off);
  uint16_t* const s_id = reinterpret_cast<uint16_t*>(wake_lds + IonsLds::id_off);
  double* const s_scan = reinterpret_cast<double*>(wake_lds + IonsLds::scan_off);
  double* const s_misc = reinterpret_cast<double*>(wake_lds + IonsLds::misc_off);
  double* const s_sc = s_misc + 32;
  double* const s_br = reinterpret_cast<double*>(wake_lds + IonsLds::br_off);

  const int tid = threadIdx.x;
  const int N = I.N, C = I.C;
  const size_t S = (size_t)C * NT;
  const int p0 = tid * C;
  const int cnt = N - p0 < 0 ? 0 : (N - p0 < C ? N - p0 : C);
  if (I.ctl[CTL_BREAK] >= 0) return;
  int cur = I.ctl[CTL_CUR];
  const int end = I.first + I.count;
  const int n_an = I.n_an;
  const double dxi = I.dxi;
  const double* const cst = I.cst;
  const double m_ion = I.m_i;
  const bool has_laser = I.has_laser != 0;   // else |a|^2 and its gradient are 0 (not stored)
  unsigned long long fixups = 0;
  int n = I.first;
  for (; n < end; ++n) {
    const double xi = n * dxi;
    if (tid < n_an) {             // this slice's analytic source factors
      const WakeAnalytic& A = I.an[tid];
      if (A.kind == 2) {
        const double s2 = A.sigma_r * A.sigma_r;
        const double dl = xi - A.xi_c;
        s_misc[3 * tid] = 2.0;
        s_misc[3 * tid + 1] = A.q * A.n_peak * exp(-(dl * dl) / (2.0 * A.sigma_xi * A.sigma_xi)) * s2;
        s_misc[3 * tid + 2] = 1.0 / (2.0 * s2);
      } else {
        const double dl = xi - A.xi_l;
        s_misc[3 * tid] = 3.0;
        s_misc[3 * tid + 1] = A.a0 * A.a0 * exp(-2.0 * dl * dl / (A.L * A.L));
        s_misc[3 * tid + 2] = 2.0 / (A.w0 * A.w0);
      }
    }
    // this slice's beam-table radii into LDS (read after the order phase's
    // barriers; the previous slice's reads ended at its last barrier)
    const int bt0 = I.nb ? I.boff[n] : 0;
    const int bm = I.nb ? I.boff[n + 1] - bt0 : 0;
    const bool b_lds = bm <= WAKE_BCAP;
    if (b_lds)
      for (int i = tid; i < bm; i += NT) s_br[i] = I.br[bt0 + i];
    const double* const stc = I.st[cur];
    double* const stn = I.st[cur ^ 1];

    // ---- order of each species ----
    int bad_order = 0;
    #pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const double* rho_s = stc + (size_t)(s * IS_N + IS_RHO) * N;
      int32_t* const ord = I.ord + (size_t)s * N;
      double* const sr = s_r + s * NMAX;
      #pragma unroll 4
      for (int k = 0; k < cnt; ++k) {
        const int p = p0 + k;
        const int id = ord[p];
        sr[p] = rho_s[id];
        s_id[p] = (uint16_t)id;
      }
      __syncthreads();
      int dis = 0;
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const int p = p0 + k;
        if (p > 0 && !key_lt(sr[p - 1], (int32_t)s_id[p - 1], sr[p], (int32_t)s_id[p])) dis = 1;
      }
      const bool resort = __syncthreads_or(dis) != 0;
      if (resort) {
        ions_fix_order(sr, s_id, N);
        ++fixups;
      }
      int32_t* const sid = I.sid + (size_t)s * S;
      double* const wk = I.work + (size_t)s * IW_N * S;
      const double* const st_s = stc + (size_t)s * IS_N * N;
      // the ring's weights and momentum into the slots of its position (used
      // by most phases; the rest is read through the ring id where needed)
      #pragma unroll 4
      for (int k = 0; k < cnt; ++k) {
        const int p = p0 + k;
        const unsigned sl = k * NT + tid;
        int id = s_id[p];
        // a padding key among the first N positions: a radius that is not a
        // finite number (state injected from device memory) -- stop there
        if (id >= N) { id = 0; bad_order = 1; }
        sid[sl] = id;
        if (resort) ord[p] = id;
        wk[IW_W * S + sl] = cst[IK_W * N + id];
        wk[IW_WH * S + sl] = cst[IK_WH * N + id];
        wk[IW_U * S + sl] = st_s[IS_U * N + id];
      }
      __syncthreads();              // s_id is the next species' too
    }

    // ---- own sums: psi and d_rho psi of each species at its rings ----
    dd sw[2], swl[2];
    for (int s = 0; s < 2; ++s) {
      const double* const wk = I.work + (size_t)s * IW_N * S;
      const int32_t* const sid = I.sid + (size_t)s * S;
      const double* sr = s_r + s * NMAX;
      sw[s] = dd_make(0.0);
      swl[s] = dd_make(0.0);
      #pragma unroll 2
      for (int k = 0; k < cnt; ++k) {
        const unsigned sl = k * NT + tid;
        const double r = sr[p0 + k];
        const double w = wk[IW_W * S + sl];
        const dd lnr = ring_log_id(cst, N, sid[sl], r);
        sw[s] = dd_add_d(sw[s], w);
        swl[s] = dd_add(swl[s], dd_mul_d(lnr, w));
      }
    }
    Pack<4> exP, totP, exS, totS;
    block_prefix_suffix<NT, 4, 4, DD2Op, DD2Op, true>(
        Pack<4>{{sw[0].hi, sw[0].lo, sw[1].hi, sw[1].lo}}, Pack<4>{{0.0, 0.0, 0.0, 0.0}}, DD2Op(),
        Pack<4>{{swl[0].hi, swl[0].lo, swl[1].hi, swl[1].lo}}, Pack<4>{{0.0, 0.0, 0.0, 0.0}}, DD2Op(),
        s_scan, exP, totP, exS, totS);
    #pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const double q = s ? 1.0 : -1.0;
      const double* const wk = I.work + (size_t)s * IW_N * S;
      const int32_t* const sid = I.sid + (size_t)s * S;
      double* const tb = I.tab + (size_t)s * IT_N * S;
      double* const sc = s_sc + SC_N * s;
      const double* sr = s_r + s * NMAX;
      const dd Q = s ? dd{totP.v[2], totP.v[3]} : dd{totP.v[0], totP.v[1]};
      dd below = s ? dd{exP.v[2], exP.v[3]} : dd{exP.v[0], exP.v[1]};
      // sum over positions >= p
      dd rest = dd_add(s ? dd{exS.v[2], exS.v[3]} : dd{exS.v[0], exS.v[1]}, s ? swl[1] : swl[0]);
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const unsigned sl = k * NT + tid;
        const int p = p0 + k;
        const double r = sr[p];
        const double w = wk[IW_W * S + sl], wh = wk[IW_WH * S + sl];
        const int id = sid[sl];
        const dd lnr = ring_log_id(cst, N, id, r);
        const dd above = dd_sub(rest, dd_mul_d(lnr, w));
        // psi = -q ((sum_{k<i} w_k + w_i) ln rho_i + sum_{k>i} w_k ln rho_k)
        dd ps = dd_add(dd_mul(dd_add_d(below, w), lnr), above);
        // d_rho psi = -q (sum_{k<i} w_k + w^_i) / rho_i
        dd dp = dd_div_d(dd_add_d(below, wh), r);
        if (q > 0.0) { ps = dd_neg(ps); dp = dd_neg(dp); }
        tb[IT_PSH * S + sl] = ps.hi;
        tb[IT_PSL * S + sl] = ps.lo;
        tb[IT_DPH * S + sl] = dp.hi;
        tb[IT_DPL * S + sl] = dp.lo;
        below = dd_add_d(below, w);
        rest = above;
        if (p == N - 1) {
          // outer edge: the outermost ring plus half its initial extent, and
          // the exterior field there (-q Q ln r, -q Q / r)
          const double edge = r + cst[IK_DR * N + id] / 2.0;
          const dd lne = dd_add_d(lnr, log1p_fast((edge - r) / r));
          dd eps = dd_mul(Q, lne);
          dd edp = dd_div_d(Q, edge);
          if (q > 0.0) { eps = dd_neg(eps); edp = dd_neg(edp); }
          sc[SC_EDGE] = edge;
          sc[SC_EPH] = eps.hi;
          sc[SC_EPL] = eps.lo;
          sc[SC_EDP] = edp.hi;
          sc[SC_EDL] = edp.lo;
        }
      }
      if (tid == 0) {
        dd pa = s ? dd{totS.v[2], totS.v[3]} : dd{totS.v[0], totS.v[1]};
        if (q > 0.0) pa = dd_neg(pa);
        sc[SC_PAH] = pa.hi;
        sc[SC_PAL] = pa.lo;
        sc[SC_QH] = Q.hi;
        sc[SC_QL] = Q.lo;
      }
    }
    __syncthreads();

    // ---- gather psi, d_rho psi; local quantities, sources; d_zeta psi sums ----
    int bad = bad_order;
    const double* const br = b_lds ? s_br : I.br + bt0;
    const double* const bcq = I.bcum + bt0;
    dd szc0 = dd_make(0.0), szc1 = dd_make(0.0);
    #pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const int o = s ^ 1;
      const double q = s ? 1.0 : -1.0, m = s ? m_ion : 1.0;
      const double qm = q / m, qq2 = (q * q) / (2.0 * m * m);
      const double qo = o ? 1.0 : -1.0;
      double* const wk = I.work + (size_t)s * IW_N * S;
      const int32_t* const sid = I.sid + (size_t)s * S;
      const double* tb = I.tab + (size_t)s * IT_N * S;
      const double* tbo = I.tab + (size_t)o * IT_N * S;
      int32_t* const jx = I.jx + (size_t)s * S;
      const double* sr = s_r + s * NMAX;
      const double* ro = s_r + o * NMAX;
      const double* sco = s_sc + SC_N * o;
      const double edge_o = sco[SC_EDGE];
      const dd Qo = {sco[SC_QH], sco[SC_QL]};
      dd szc = dd_make(0.0);
      int lo = 0, blo = 0;
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const unsigned sl = k * NT + tid;
        const double r = sr[p0 + k];
        const double u = wk[IW_U * S + sl];
        const double w = wk[IW_W * S + sl];
        lo = count_below(ro, lo, N, r, k > 0);
        Interval iv;
        dd pg, dg;
        if (interval_of(ro, N, edge_o, r, lo, iv)) {
          // both in double-double: at a ring of the other species (t = 0 or
          // 1) its node value is taken whole, so the two species' sums
          // cancel there as exactly as they do at rest
          dd pl, ph, dl, dh;
          if (iv.j == 0) {
            pl = {sco[SC_PAH], sco[SC_PAL]};
            dl = dd_make(0.0);
          } else {
            const unsigned u0 = pslot(iv.j - 1, C);
            pl = {tbo[IT_PSH * S + u0], tbo[IT_PSL * S + u0]};
            dl = {tbo[IT_DPH * S + u0], tbo[IT_DPL * S + u0]};
          }
          if (iv.j < N) {
            const unsigned u1 = pslot(iv.j, C);
            ph = {tbo[IT_PSH * S + u1], tbo[IT_PSL * S + u1]};
            dh = {tbo[IT_DPH * S + u1], tbo[IT_DPL * S + u1]};
          } else {
            ph = {sco[SC_EPH], sco[SC_EPL]};
            dh = {sco[SC_EDP], sco[SC_EDL]};
          }
          pg = dd_add(pl, dd_mul_d(dd_sub(ph, pl), iv.t));
          dg = dd_add(dl, dd_mul_d(dd_sub(dh, dl), iv.t));
          jx[sl] = iv.j;
        } else {                  // beyond the other species' edge: its exterior field
          pg = dd_mul(Qo, ring_log_id(cst, N, sid[sl], r));
          dg = dd_div_d(Qo, r);
          if (qo > 0.0) { pg = dd_neg(pg); dg = dd_neg(dg); }
          jx[sl] = -1;
        }
        const double psi = dd_round(dd_add(pg, {tb[IT_PSH * S + sl], tb[IT_PSL * S + sl]}));
        const double dpsi = dd_round(dd_add(dg, {tb[IT_DPH * S + sl], tb[IT_DPL * S + sl]}));
        // beam charge inside r (table entries strictly below), analytic beams, lasers
        double lam = 0.0;
        if (bm > 0) {
          blo = count_below(br, blo, bm, r, k > 0);
          if (blo > 0) lam = bcq[blo - 1];
        }
        double a2 = 0.0, da2 = 0.0;
        #pragma unroll 1
        for (int si = 0; si < n_an; ++si) {
          const double kind = s_misc[3 * si], c0 = s_misc[3 * si + 1], c1 = s_misc[3 * si + 2];
          if (kind == 2.0) {
            lam += c0 * (-expm1(-r * r * c1));
          } else {
            const double x = c0 * exp(-r * r * c1);
            a2 += x;
            da2 += -(2.0 * r * c1) * x;
          }
        }
        const double pb = 1.0 - qm * psi;
        if (!(pb > 0.0) || !isfinite(pb)) bad = 1;
        const double c = q * u / (r * pb);
        szc = dd_add_d(szc, w * c);
        wk[IW_PSI * S + sl] = psi;
        wk[IW_DPSI * S + sl] = dpsi;
        wk[IW_PB * S + sl] = pb;
        wk[IW_BB * S + sl] = lam / r;
        if (has_laser) {
          wk[IW_A2 * S + sl] = a2;
          wk[IW_DA2 * S + sl] = da2;
        }
      }
      if (s) szc1 = szc; else szc0 = szc;
    }
    Pack<4> dzs, dzt;
    dzs = block_suffix<NT, 4>(Pack<4>{{szc0.hi, szc0.lo, szc1.hi, szc1.lo}},
                              Pack<4>{{0.0, 0.0, 0.0, 0.0}}, DD2Op(), s_scan, dzt);
    // own d_zeta psi at each ring: the rings outside with w, the ring itself
    // with w - w^
    #pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const double q = s ? 1.0 : -1.0;
      const double* wk = I.work + (size_t)s * IW_N * S;
      double* const tb = I.tab + (size_t)s * IT_N * S;
      const double* sr = s_r + s * NMAX;
      dd above = s ? dd{dzs.v[2], dzs.v[3]} : dd{dzs.v[0], dzs.v[1]};
      #pragma unroll 1
      for (int k = cnt - 1; k >= 0; --k) {
        const unsigned sl = k * NT + tid;
        const double r = sr[p0 + k];
        const double w = wk[IW_W * S + sl], wh = wk[IW_WH * S + sl];
        const double c = q * wk[IW_U * S + sl] / (r * wk[IW_PB * S + sl]);
        tb[IT_DZ * S + sl] = dd_round(dd_add_d(above, (w - wh) * c));
        above = dd_add_d(above, w * c);
      }
      if (tid == 0) {
        s_sc[SC_N * s + SC_DZH] = s ? dzt.v[2] : dzt.v[0];
        s_sc[SC_N * s + SC_DZL] = s ? dzt.v[3] : dzt.v[1];
      }
    }
    __syncthreads();

    // ---- gather d_zeta psi; electrons: coefficients and chunk transfer ----
    Pack<4> G = mat_ident();
    #pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const int o = s ^ 1;
      double* const wk = I.work + (size_t)s * IW_N * S;
      const double* tb = I.tab + (size_t)s * IT_N * S;
      const double* tbo = I.tab + (size_t)o * IT_N * S;
      const int32_t* jx = I.jx + (size_t)s * S;
      const double* sr = s_r + s * NMAX;
      const double* ro = s_r + o * NMAX;
      const double edge_o = s_sc[SC_N * o + SC_EDGE];
      const double dza_o = dd_round({s_sc[SC_N * o + SC_DZH], s_sc[SC_N * o + SC_DZL]});
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const unsigned sl = k * NT + tid;
        const int j = jx[sl];
        double dz = tb[IT_DZ * S + sl];
        if (j >= 0) {
          const double t = interval_t(ro, N, edge_o, sr[p0 + k], j);
          const double dl = j == 0 ? dza_o : tbo[IT_DZ * S + pslot(j - 1, C)];
          const double dh = j < N ? tbo[IT_DZ * S + pslot(j, C)] : 0.0;
          dz += (1.0 - t) * dl + t * dh;
        }
        wk[IW_DZ * S + sl] = dz;
        if (s == 0) {
          const double r = sr[p0 + k];
          const double w = wk[IW_W * S + sl];
          const double irho = rcp_nr(r);
          const double a2 = has_laser ? wk[IW_A2 * S + sl] : 0.0;
          const double da2 = has_laser ? wk[IW_DA2 * S + sl] : 0.0;
          const Local L = local_of(irho, wk[IW_U * S + sl], w, wk[IW_PSI * S + sl], a2);
          double B, Cc, sa, sb;
          ring_BC(irho, wk[IW_U * S + sl], w, L, wk[IW_DPSI * S + sl], dz, wk[IW_BB * S + sl], da2, B,
                  Cc);
          rec_offset(L.A, B, Cc, r, sa, sb);
          G = mat_mul(rec_matrix(L.A, r, irho), G);
          wk[IW_A * S + sl] = L.A;
          wk[IW_C * S + sl] = Cc;
          wk[IW_SA * S + sl] = sa;
          wk[IW_SB * S + sl] = sb;
        }
      }
    }
    // growing mode at the chunk start, decaying mode at the chunk end
    Pack<4> gp, gt, hx, ht;
    block_prefix_suffix<NT, 4, 4, FwdMatOp, BwdMatOp, true>(
        G, mat_ident(), FwdMatOp(), mat_adj(G), mat_ident(), BwdMatOp(), s_scan, gp, gt, hx, ht);
    const double W = gt.v[0];                 // det[g_N, (0, 1)]
    const double iW = 1.0 / W;
    double* const wke = I.work;
    const double* sre = s_r;
    // g_i and the det-sums of the chunk (E forward, D backward)
    double Ec = 0.0, Dc = 0.0;
    {
      double ga = gp.v[0], gb = gp.v[2];
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const unsigned sl = k * NT + tid;
        const double r = sre[p0 + k];
        wke[IW_GA * S + sl] = ga;
        wke[IW_GB * S + sl] = gb;
        wke[IW_E * S + sl] = Ec;
        const Pack<4> M = rec_matrix(wke[IW_A * S + sl], r, rcp_nr(r));
        const double na = M.v[0] * ga + M.v[1] * gb, nb = M.v[2] * ga + M.v[3] * gb;
        ga = na;
        gb = nb;
        Ec += ga * wke[IW_SB * S + sl] - gb * wke[IW_SA * S + sl];
      }
      double ha = hx.v[1], hb = hx.v[3];
      #pragma unroll 1
      for (int k = cnt - 1; k >= 0; --k) {
        const unsigned sl = k * NT + tid;
        const double r = sre[p0 + k];
        Dc += wke[IW_SA * S + sl] * hb - wke[IW_SB * S + sl] * ha;
        const Pack<4> Mi = mat_adj(rec_matrix(wke[IW_A * S + sl], r, rcp_nr(r)));
        const double na = Mi.v[0] * ha + Mi.v[1] * hb, nb = Mi.v[2] * ha + Mi.v[3] * hb;
        ha = na;
        hb = nb;
      }
    }
    Pack<1> ep, et, dsf, dt;
    block_prefix_suffix<NT, 1, 1, SumOp<1>, SumOp<1>, true>(Pack<1>{{Ec}}, Pack<1>{{0.0}}, SumOp<1>(),
                                                           Pack<1>{{Dc}}, Pack<1>{{0.0}}, SumOp<1>(),
                                                           s_scan, ep, et, dsf, dt);
    const double bN = et.v[0] * iW;           // b_N = E_N / W (a_N = 0)
    {
      // x_{i-1} = (h_{i-1} E_{i-1} - g_{i-1} D_{i-1}) / W and B^(p) at ring i
      double* const tbe = I.tab;
      double ha = hx.v[1], hb = hx.v[3];
      double D = dsf.v[0];
      #pragma unroll 1
      for (int k = cnt - 1; k >= 0; --k) {
        const unsigned sl = k * NT + tid;
        const double r = sre[p0 + k];
        const double irho = rcp_nr(r);
        D += wke[IW_SA * S + sl] * hb - wke[IW_SB * S + sl] * ha;
        const Pack<4> Mi = mat_adj(rec_matrix(wke[IW_A * S + sl], r, irho));
        const double na = Mi.v[0] * ha + Mi.v[1] * hb, nb = Mi.v[2] * ha + Mi.v[3] * hb;
        ha = na;
        hb = nb;
        const double E = ep.v[0] + wke[IW_E * S + sl];
        const double ga = wke[IW_GA * S + sl], gb = wke[IW_GB * S + sl];
        const double a = (ha * E - ga * D) * iW;
        const double b = (hb * E - gb * D) * iW;
        const double w = wke[IW_W * S + sl], wh = wke[IW_WH * S + sl];
        const double bp = a * r + b * irho + (wh / w) * wke[IW_C * S + sl];
        tbe[IT_BP * S + sl] = bp;
        wke[IW_BT * S + sl] = wke[IW_BB * S + sl] + bp;
      }
    }
    __syncthreads();

    // ---- ions: B^(p) interpolated between the electron rings ----
    {
      double* const wki = I.work + (size_t)IW_N * S;
      const int32_t* jxi = I.jx + S;
      const double* tbe = I.tab;
      const double edge_e = s_sc[SC_EDGE];
      const double* sri = s_r + NMAX;
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const unsigned sl = k * NT + tid;
        const int j = jxi[sl];
        double bp;
        if (j >= 0) {
          const double t = interval_t(s_r, N, edge_e, sri[p0 + k], j);
          const double bl = j == 0 ? 0.0 : tbe[IT_BP * S + pslot(j - 1, C)];
          const double bh = j < N ? tbe[IT_BP * S + pslot(j, C)] : bN / edge_e;
          bp = (1.0 - t) * bl + t * bh;
        } else {
          bp = bN / sri[p0 + k];
        }
        wki[IW_BT * S + sl] = wki[IW_BB * S + sl] + bp;
      }
    }

    // ---- fields out, push ----
    const bool do_push = n < I.n_xi - 1;
    const bool rec_snap = I.stride > 0 && (n % I.stride) == 0;
    const bool rec_last = n == end - 1;
    #pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const double q = s ? 1.0 : -1.0, m = s ? m_ion : 1.0;
      const double qm = q / m, q24 = (q * q) / (4.0 * m * m), qq2 = (q * q) / (2.0 * m * m);
      const double* frp = stc + (size_t)(s * IS_N + IS_FR) * N;
      const double* fup = stc + (size_t)(s * IS_N + IS_FU) * N;
      const int32_t* sid = I.sid + (size_t)s * S;
      const double* wk = I.work + (size_t)s * IW_N * S;
      const double* sr = s_r + s * NMAX;
      double* const rn_s = stn + (size_t)(s * IS_N + IS_RHO) * N;
      double* const un_s = stn + (size_t)(s * IS_N + IS_U) * N;
      double* const fr_s = stn + (size_t)(s * IS_N + IS_FR) * N;
      double* const fu_s = stn + (size_t)(s * IS_N + IS_FU) * N;
      double* const snap = rec_snap ? I.snap[s] + (size_t)(n / I.stride) * OUT_N * N : nullptr;
      double* const last = I.last[s];
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const unsigned sl = k * NT + tid;
        const int id = sid[sl];
        const double r = sr[p0 + k];
        const double u = wk[IW_U * S + sl], psi = wk[IW_PSI * S + sl], dpsi = wk[IW_DPSI * S + sl];
        const double ez = -wk[IW_DZ * S + sl], bt = wk[IW_BT * S + sl];
        if (!(isfinite(psi) && isfinite(dpsi) && isfinite(ez) && isfinite(bt))) bad = 1;
        if (rec_snap) {
          snap[OUT_PSI * N + id] = psi; snap[OUT_ERBT * N + id] = -dpsi;
          snap[OUT_EZ * N + id] = ez; snap[OUT_BT * N + id] = bt;
          snap[OUT_RHO * N + id] = r; snap[OUT_UR * N + id] = u;
        }
        if (rec_last) {
          last[OUT_PSI * N + id] = psi; last[OUT_ERBT * N + id] = -dpsi;
          last[OUT_EZ * N + id] = ez; last[OUT_BT * N + id] = bt;
          last[OUT_RHO * N + id] = r; last[OUT_UR * N + id] = u;
        }
        if (do_push) {
          const double pb = wk[IW_PB * S + sl];
          const double a2 = has_laser ? wk[IW_A2 * S + sl] : 0.0;
          const double da2 = has_laser ? wk[IW_DA2 * S + sl] : 0.0;
          const double gm = (1.0 + u * u + pb * pb + qq2 * a2) / (2.0 * pb);   // eq. motion_4
          const double f_r = u / pb;
          const double f_u = -(qm * (gm * dpsi / pb - bt) + q24 * da2 / pb);
          double pr = f_r, pu = f_u;
          if (n > 0) { pr = frp[id]; pu = fup[id]; }
          double rn = r + dxi * (1.5 * f_r - 0.5 * pr);
          double un = u + dxi * (1.5 * f_u - 0.5 * pu);
          double sr_ = f_r, su = f_u;
          if (rn < 0.0) { rn = -rn; un = -un; sr_ = -sr_; su = -su; }
          if (!(isfinite(rn) && isfinite(un))) bad = 1;
          rn_s[id] = rn;
          un_s[id] = un;
          fr_s[id] = sr_;
          fu_s[id] = su;
        }
      }
    }
    if (tid == 0) {
      const dd pa = dd_add({s_sc[SC_PAH], s_sc[SC_PAL]}, {s_sc[SC_N + SC_PAH], s_sc[SC_N + SC_PAL]});
      const dd za = dd_add({s_sc[SC_DZH], s_sc[SC_DZL]}, {s_sc[SC_N + SC_DZH], s_sc[SC_N + SC_DZL]});
      I.axis[2 * n] = dd_round(pa);
      I.axis[2 * n + 1] = -dd_round(za);
    }
    if (__syncthreads_or(bad)) {      // breakdown: stop at this slice, its state kept
      if (tid == 0) { I.ctl[CTL_BREAK] = n; I.ctl[CTL_NEXT] = n; I.ctl[CTL_CUR] = cur; }
      break;
    }
    if (do_push) cur ^= 1;
  }
  if (tid == 0) {
    if (n == end) {
      I.ctl[CTL_CUR] = cur;
      I.ctl[CTL_NEXT] = end;
    }
    atomicAdd(I.cnt + CNT_SLICES, (unsigned long long)(n - I.first));
    atomicAdd(I.cnt + CNT_FIXUPS, fixups);
  }
}

// constants (when asked) and the rest state of both species in buffer 0
__global__ void ions_init_kernel(WakeIons J, const double* __restrict__ r0, const double* __restrict__ dr,
                                 const double* __restrict__ dens, int constants) {
  const int N = J.N;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) {
    J.ctl[CTL_CUR] = 0;
    J.ctl[CTL_BREAK] = -1;
    J.ctl[CTL_NEXT] = 0;
    J.ctl[CTL_FAULT] = 0;
  }
  if (j >= N) return;
  double* const cst = const_cast<double*>(J.cst);
  if (constants) {
    const double r = r0[j], d = dr[j];
    const double nd = dens ? dens[j] : 1.0;
    const double w = nd * r * d;                  // eq. macroparticle_weight
    const dd lr = dd_log(r);
    cst[IK_W * N + j] = w;
    cst[IK_WH * N + j] = w / 2.0 - nd * d * d / 8.0;   // modified self weight
    cst[IK_R0 * N + j] = r;
    cst[IK_IR0 * N + j] = 1.0 / r;
    cst[IK_LNH * N + j] = lr.hi;
    cst[IK_LNL * N + j] = lr.lo;
    cst[IK_DR * N + j] = d;
  }
  const double r = cst[IK_R0 * N + j];
  for (int s = 0; s < 2; ++s) {
    double* const st = J.st[0] + (size_t)s * IS_N * N;
    st[IS_RHO * N + j] = r;
    st[IS_U * N + j] = 0.0;
    st[IS_FR * N + j] = 0.0;
    st[IS_FU * N + j] = 0.0;
    J.ord[(size_t)s * N + j] = j;
  }
}

// rest state of both species of instance blockIdx.y in buffer 0 (control
// words reset), from its constants
__global__ void ions_reset_kernel(const WakeIons* __restrict__ insts) {
  const WakeIons& J = insts[blockIdx.y];
  const int N = J.N;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    J.ctl[CTL_CUR] = 0;
    J.ctl[CTL_BREAK] = -1;
    J.ctl[CTL_NEXT] = 0;
    J.ctl[CTL_FAULT] = 0;
  }
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const double r = J.cst[IK_R0 * N + j];
    for (int s = 0; s < 2; ++s) {
      double* const st = J.st[0] + (size_t)s * IS_N * N;
      st[IS_RHO * N + j] = r;
      st[IS_U * N + j] = 0.0;
      st[IS_FR * N + j] = 0.0;
      st[IS_FU * N + j] = 0.0;
      J.ord[(size_t)s * N + j] = j;
    }
  }
}

__global__ void ions_get_state_kernel(WakeIons J, int sp, double* __restrict__ out) {
  const int N = J.N;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double* st = J.st[J.ctl[CTL_CUR] & 1] + (size_t)sp * IS_N * N;
  for (int q = 0; q < IS_N; ++q) out[(size_t)q * N + j] = st[(size_t)q * N + j];
}

__global__ void ions_set_state_kernel(WakeIons J, int sp, const double* __restrict__ rho,
                                      const double* __restrict__ u, const double* __restrict__ fr,
                                      const double* __restrict__ fu, int slice) {
  const int N = J.N;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = J.ctl[CTL_CUR] & 1;
  if (j < N) {
    double* st = J.st[b] + (size_t)sp * IS_N * N;
    st[IS_RHO * N + j] = rho[j];
    st[IS_U * N + j] = u[j];
    st[IS_FR * N + j] = fr ? fr[j] : 0.0;
    st[IS_FU * N + j] = fu ? fu[j] : 0.0;
    J.ord[(size_t)sp * N + j] = j;      // order found again at the next slice
  }
  if (j == 0) {
    J.ctl[CTL_BREAK] = -1;
    J.ctl[CTL_NEXT] = slice;
    J.ctl[CTL_FAULT] = 0;
  }
}

}  // namespace

size_t ions_lds_bytes() { return IonsLds::bytes; }

hipError_t launch_ions_init(const WakeIons& J, const double* r0, const double* dr, const double* dens,
                            bool constants, hipStream_t s) {
  const int blocks = (J.N + 255) / 256;
  hipLaunchKernelGGL(ions_init_kernel, dim3(blocks), dim3(256), 0, s, J, r0, dr, dens, constants ? 1 : 0);
  return hipGetLastError();
}

hipError_t ions_prepare() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&ions_march_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)IonsLds::bytes);
}

hipError_t launch_ions_march(const WakeIons* d_insts, int n_insts, hipStream_t s) {
  hipLaunchKernelGGL(ions_march_kernel, dim3(n_insts), dim3(NT), IonsLds::bytes, s, d_insts);
  return hipGetLastError();
}

hipError_t launch_ions_reset(const WakeIons* d_insts, int n_insts, hipStream_t s) {
  hipLaunchKernelGGL(ions_reset_kernel, dim3(8, n_insts), dim3(256), 0, s, d_insts);
  return hipGetLastError();
}

hipError_t launch_ions_get_state(const WakeIons& J, int sp, double* out, hipStream_t s) {
  hipLaunchKernelGGL(ions_get_state_kernel, dim3((J.N + 255) / 256), dim3(256), 0, s, J, sp, out);
  return hipGetLastError();
}

hipError_t launch_ions_set_state(const WakeIons& J, int sp, const double* rho, const double* u,
                                 const double* fr, const double* fu, int slice, hipStream_t s) {
  hipLaunchKernelGGL(ions_set_state_kernel, dim3((J.N + 255) / 256), dim3(256), 0, s, J, sp, rho, u, fr,
                     fu, slice);
  return hipGetLastError();
}
