// gfx950 slice marcher of the gridless quasistatic plasma-ring solver.
//
// Model (paper, Sec. "Gridless quasistatic model"): axisymmetric electron
// rings (q=-1, m=1) over immobile ions, marched in xi = -zeta.  Per slice:
// radial order (ring id breaks ties), beam/laser sources, the Gauss/log sums
// for psi and d_rho psi (eqs. dpsi_dr, psi), gamma (eq. motion_4), the
// d_zeta psi sum (eq. dpsi_dzeta with the sign obtained by differentiating
// eq. psi), coefficients A, B, C (eqs. b_coeffs_1-3, ponderomotive term with
// the 1/4 and sign of the physical force), the two-point recursion for
// B_theta^(p) (eq. ai_bi, b_0 = 0, a_N = 0) and the Adams-Bashforth-2 push
// (eqs. motion_1-2).
//
// One workgroup owns one instance and marches its slices; thread t owns the
// C = ceil(N / NT) consecutive sorted positions [t*C, t*C + C), stored in
// slots k*NT + t (coalesced).  Per slice:
//   loop B (forward)  psi, d_rho psi from a double-double prefix of
//                     (w, w ln rho); sources; psibar, gamma, A_i, transfer
//                     matrix M_i; per-thread product of M_i and sum of v_i
//   scan              prefix of the products (growing mode g, g_0 = (1,0))
//                     and of v; suffix of the inverse products (decaying
//                     mode h, h_N = (0,1)) and of v
//   loop C (forward)  g_{i-1} stored; sums of det[g_i, s_i], with s_i affine
//                     in the total V = sum v (s = s0 + V s1)
//   loop D (backward) d_zeta psi, B_i, s_i, sum of det[s_i, h_i]
//   scan              prefix of the det[g, s] sums, suffix of det[s, h]
//   loop E (backward) x_{i-1} = (h_{i-1} E_{i-1} - g_{i-1} D_{i-1}) / W,
//                     W = det[g, h] = a-part of g_N; B^(p), outputs, AB2
//                     push, ln rho of the pushed radius for the next slice.
// This variation-of-parameters form solves the same linear system as the
// paper's shooting (Appendix "Solve recursive system") without its
// exponential loss of digits.  If the pushed radii are out of order, the
// rings that are not already in their final place are compacted, sorted
// and dropped into the freed positions (every other ring keeps its slot).
#include "wake_common.h"
#include "wake_device.h"
#include "wake_launch.h"

#include <math.h>

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
  L.ipb = 1.0 / L.pb;
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

// a / b for double-double a with a precomputed reciprocal ib = 1/b
__device__ __forceinline__ dd dd_div_rcp(dd a, double b, double ib) {
  _Pragma("clang fp contract(off)")
  const double q1 = a.hi * ib;
  const dd r = dd_sub(a, two_prod(q1, b));
  const double q2 = r.hi * ib;
  return fast_two_sum(q1, q2);
}

// ln(rho) of ring `id` as ln r0 + log1p((rho - r0)/r0): its rounding scales
// with the ring's displacement, not with |ln rho| (the psi sums multiply
// ln rho by the enclosed charge).
__device__ __forceinline__ dd ring_log(const WakeInst& I, int id, double rho) {
  const double l1 = log1p((rho - I.r0[id]) * I.ir0[id]);
  return dd_add_d({I.L0h[id], I.L0l[id]}, l1);
}

// Ion psi - psi(0) and d_rho psi at radius r: linear interpolation inside
// the node interval containing r (Sec. "Key algorithmic adjustments"),
// searched from the ring's previous interval h; exact exterior field at and
// beyond the plasma edge.
__device__ __forceinline__ void ion_fields(const WakeInst& I, double r, dd lnr, int& h, dd& ps, dd& dp) {
  if (!(r < I.Rp)) {
    const dd Q = {I.tot0[2], I.tot0[3]};
    ps = dd_sub({I.tot0[0], I.tot0[1]}, dd_mul(Q, lnr));
    dp = dd_neg(dd_div_d(Q, r));
    return;
  }
  const double* R = I.ion;
  const int N = I.N;
  int j = h < 0 ? 0 : (h > N ? N : h);
  if (R[j * WAKE_ION_REC + IR_LO] <= r) {
    if (j < N && !(r < R[(j + 1) * WAKE_ION_REC + IR_LO])) {
      int a = j + 1, b, step = 1;     // lo(a) <= r
      for (;;) {
        b = a + step;
        if (b > N) { b = N + 1; break; }
        if (r < R[b * WAKE_ION_REC + IR_LO]) break;
        a = b;
        step <<= 1;
      }
      while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (R[m * WAKE_ION_REC + IR_LO] <= r) a = m; else b = m;
      }
      j = a;
    }
  } else {
    int b = j, a, step = 1;           // lo(b) > r
    for (;;) {
      a = b - step;
      if (a <= 0) { a = 0; break; }
      if (R[a * WAKE_ION_REC + IR_LO] <= r) break;
      b = a;
      step <<= 1;
    }
    while (b - a > 1) {
      const int m = (a + b) >> 1;
      if (R[m * WAKE_ION_REC + IR_LO] <= r) a = m; else b = m;
    }
    j = a;
  }
  h = j;
  const double* rec = R + j * WAKE_ION_REC;
  const double t = (r - rec[IR_LO]) / (rec[IR_HI] - rec[IR_LO]);
  ps = dd_add_d({rec[IR_PSH], rec[IR_PSL]}, t * rec[IR_DPS]);
  dp = dd_add_d({rec[IR_DPH], rec[IR_DPL]}, t * rec[IR_DDP]);
}

// ---------------------------------------------------------------------------
// ring-set initialisation: weights, ln r0, ion interval records, state
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void wake_init_kernel(WakeInst I, const double* __restrict__ r0,
                                                       const double* __restrict__ dr,
                                                       const double* __restrict__ dens) {
  __shared__ double s_scan[(NT / 64) * 8];
  const int N = I.N;
  const int tid = threadIdx.x;
  double* w_out = const_cast<double*>(I.w);
  double* wh_out = const_cast<double*>(I.wh);
  double* r0_out = const_cast<double*>(I.r0);
  double* ir0_out = const_cast<double*>(I.ir0);
  double* l0h = const_cast<double*>(I.L0h);
  double* l0l = const_cast<double*>(I.L0l);
  double* R = const_cast<double*>(I.ion);
  double* consts = const_cast<double*>(I.tot0);
  dd cS = {0.0, 0.0}, cPT = {0.0, 0.0};
  // phase 1: node values (node j+1 is ring j) into records j+1
  for (int base = 0; base < N; base += NT) {
    const int j = base + tid;
    const bool ok = j < N;
    double w = 0.0, wh = 0.0, r = 1.0;
    dd lr = {0.0, 0.0};
    if (ok) {
      r = r0[j];
      const double d = dr[j];
      const double nd = dens ? dens[j] : 1.0;
      w = nd * r * d;                              // eq. macroparticle_weight
      wh = w / 2.0 - nd * d * d / 8.0;             // modified weight
      lr = dd_log(r);
      w_out[j] = w; wh_out[j] = wh; r0_out[j] = r; ir0_out[j] = 1.0 / r;
      l0h[j] = lr.hi; l0l[j] = lr.lo;
    }
    const dd wl = dd_mul_d(lr, w);
    Pack<4> tot;
    Pack<4> pre = block_prefix<NT, 4>(Pack<4>{{w, 0.0, wl.hi, wl.lo}}, Pack<4>{{0, 0, 0, 0}},
                                      DD2Op(), s_scan, tot);
    const dd S = dd_add(cS, {pre.v[0], pre.v[1]});
    const dd PTi = dd_add(dd_add(cPT, {pre.v[2], pre.v[3]}), wl);
    if (ok) {
      // ion ring j (q=+1) at its own radius with self weight w^
      const dd dp = dd_neg(dd_div_d(dd_add_d(S, wh), r));
      const dd ps = dd_neg(dd_sub(dd_mul(dd_add_d(S, w), lr), PTi));
      double* rec = R + (size_t)(j + 1) * WAKE_ION_REC;
      rec[IR_LO] = r;
      rec[IR_PSH] = ps.hi; rec[IR_PSL] = ps.lo;
      rec[IR_DPH] = dp.hi; rec[IR_DPL] = dp.lo;
      // initial state: position j holds ring j; its interval starts at its node
      const int sl = (j % I.C) * I.nt + j / I.C;
      I.rho[0][sl] = r; I.u[0][sl] = 0.0; I.fr[0][sl] = 0.0; I.fu[0][sl] = 0.0;
      I.id[0][sl] = j; I.hint[0][sl] = j + 1;
    }
    cS = dd_add(cS, {tot.v[0], tot.v[1]});
    cPT = dd_add(cPT, {tot.v[2], tot.v[3]});
  }
  if (tid == 0) {
    R[IR_LO] = 0.0;
    R[IR_PSH] = 0.0; R[IR_PSL] = 0.0; R[IR_DPH] = 0.0; R[IR_DPL] = 0.0;
    consts[0] = cPT.hi; consts[1] = cPT.lo;   // sum_j w_j ln r0_j
    consts[2] = cS.hi; consts[3] = cS.lo;     // total weight Q
    I.ctl[CTL_CUR] = 0;
    I.ctl[CTL_BREAK] = -1;
    I.ctl[CTL_NEXT] = 0;
  }
  __syncthreads();
  // phase 2: interval ends and steps; the last node is the plasma edge
  const double Rp = I.Rp;
  const dd eps = dd_sub(cPT, dd_mul(cS, dd_log(Rp)));
  const dd edp = dd_neg(dd_div_d(cS, Rp));
  for (int j = tid; j <= N; j += NT) {
    double* rec = R + (size_t)j * WAKE_ION_REC;
    double hi, nps_h, nps_l, ndp_h, ndp_l;
    if (j < N) {
      const double* nx = rec + WAKE_ION_REC;
      hi = nx[IR_LO]; nps_h = nx[IR_PSH]; nps_l = nx[IR_PSL]; ndp_h = nx[IR_DPH]; ndp_l = nx[IR_DPL];
    } else {
      hi = Rp; nps_h = eps.hi; nps_l = eps.lo; ndp_h = edp.hi; ndp_l = edp.lo;
    }
    rec[IR_HI] = hi;
    rec[IR_DPS] = dd_round(dd_sub({nps_h, nps_l}, {rec[IR_PSH], rec[IR_PSL]}));
    rec[IR_DDP] = dd_round(dd_sub({ndp_h, ndp_l}, {rec[IR_DPH], rec[IR_DPL]}));
  }
}

// ---------------------------------------------------------------------------
// ring order fix-up
// ---------------------------------------------------------------------------
struct MaxKeyOp {   // (rho, id) maximum
  __device__ __forceinline__ Pack<2> operator()(const Pack<2>& a, const Pack<2>& b) const {
    return key_lt(a.v[0], (int32_t)a.v[1], b.v[0], (int32_t)b.v[1]) ? b : a;
  }
};
struct MinKeyOp {   // (rho, id) minimum
  __device__ __forceinline__ Pack<2> operator()(const Pack<2>& a, const Pack<2>& b) const {
    return key_lt(b.v[0], (int32_t)b.v[1], a.v[0], (int32_t)a.v[1]) ? b : a;
  }
};

// Bitonic sort of n keys (rho, id, slot) in place, over P = next power of two
// slots (the caller pads slots [n, P) with +inf keys).
template <int NT>
__device__ void bitonic_keys(double* kr, int32_t* ki, int32_t* ks, int P) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P; i += NT) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const bool lt = key_lt(kr[j], ki[j], kr[i], ki[i]);
          if (up ? lt : !lt) {
            const double tr = kr[i]; kr[i] = kr[j]; kr[j] = tr;
            const int32_t ti = ki[i]; ki[i] = ki[j]; ki[j] = ti;
            const int32_t ts = ks[i]; ks[i] = ks[j]; ks[j] = ts;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Sort the M compacted keys in sk[0]: pieces of WAKE_SORTCAP sorted in LDS,
// then pairwise merges by rank (each key's place in the other run found by
// binary search).  Returns the buffer index holding the result.
template <int NT>
__device__ int sort_keys_global(const WakeInst& I, int M, double* kr, int32_t* ki, int32_t* ks) {
  for (int c0 = 0; c0 < M; c0 += WAKE_SORTCAP) {
    const int len = min(WAKE_SORTCAP, M - c0);
    int P = 1;
    while (P < len) P <<= 1;
    for (int i = threadIdx.x; i < P; i += NT) {
      if (i < len) { kr[i] = I.sk_r[0][c0 + i]; ki[i] = I.sk_i[0][c0 + i]; ks[i] = I.sk_s[0][c0 + i]; }
      else { kr[i] = INFINITY; ki[i] = 0x7fffffff - i; ks[i] = -1; }
    }
    __syncthreads();
    bitonic_keys<NT>(kr, ki, ks, P);
    for (int i = threadIdx.x; i < len; i += NT) {
      I.sk_r[0][c0 + i] = kr[i]; I.sk_i[0][c0 + i] = ki[i]; I.sk_s[0][c0 + i] = ks[i];
    }
    __syncthreads();
  }
  int src = 0;
  for (int run = WAKE_SORTCAP; run < M; run <<= 1) {
    const int dst = 1 - src;
    const double* ar = I.sk_r[src];
    const int32_t* ai = I.sk_i[src];
    for (int e = threadIdx.x; e < M; e += NT) {
      const int base = (e / (2 * run)) * (2 * run);
      const int inA = e - base < run;
      const int ob = inA ? base + run : base;                    // the other run
      const int ol = inA ? min(run, max(0, M - ob)) : run;
      const double r = ar[e];
      const int32_t id = ai[e];
      int lo = 0, hi = ol;                                       // other keys below this key
      while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (key_lt(ar[ob + m], ai[ob + m], r, id)) lo = m + 1; else hi = m;
      }
      const int own = inA ? e - base : e - base - run;
      const int o = base + own + lo;
      I.sk_r[dst][o] = r; I.sk_i[dst][o] = id; I.sk_s[dst][o] = I.sk_s[src][e];
    }
    __syncthreads();
    src = dst;
  }
  return src;
}

// Put buffer `buf` in (rho, id) order.  Rings that are already in their
// final position (key above every key before and below every key after)
// keep their slot; the others are compacted in position order, sorted, and
// written into the freed positions.  Moves the state and the ln rho scratch;
// `tmp` is the other state buffer (free at this point).  Uniform result:
// true if any ring moved.
template <int NT>
__device__ __noinline__ bool fix_order(const WakeInst& I, int buf, int tmp, double* s_scan,
                                       unsigned char* region) {
  const int tid = threadIdx.x;
  const int N = I.N, C = I.C;
  const int cnt = max(0, min(C, N - tid * C));
  // chunk extremes
  Pack<2> mx = {{-INFINITY, -2147483648.0}}, mn = {{INFINITY, 2147483647.0}};
  #pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const int sl = k * NT + tid;
    const Pack<2> key = {{I.rho[buf][sl], (double)I.id[buf][sl]}};
    mx = MaxKeyOp()(mx, key);
    mn = MinKeyOp()(mn, key);
  }
  Pack<2> before, tb, after, ta;
  block_prefix_suffix<NT, 2, 2>(mx, Pack<2>{{-INFINITY, -2147483648.0}}, MaxKeyOp(), mn,
                                Pack<2>{{INFINITY, 2147483647.0}}, MinKeyOp(), s_scan, before, tb,
                                after, ta);
  // below every later key (backward), above every earlier key (forward)
  Pack<2> sm = after;
  #pragma unroll 1
  for (int k = cnt - 1; k >= 0; --k) {
    const int sl = k * NT + tid;
    const Pack<2> key = {{I.rho[buf][sl], (double)I.id[buf][sl]}};
    I.flag[sl] = key_lt(key.v[0], (int32_t)key.v[1], sm.v[0], (int32_t)sm.v[1]) ? 1 : 0;
    sm = MinKeyOp()(sm, key);
  }
  Pack<2> pm = before;
  double oop = 0.0;
  #pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const int sl = k * NT + tid;
    const Pack<2> key = {{I.rho[buf][sl], (double)I.id[buf][sl]}};
    const bool ok = I.flag[sl] && key_lt(pm.v[0], (int32_t)pm.v[1], key.v[0], (int32_t)key.v[1]);
    I.flag[sl] = ok ? 1 : 0;
    if (!ok) oop += 1.0;
    pm = MaxKeyOp()(pm, key);
  }
  Pack<1> tot;
  const Pack<1> j0p = block_prefix<NT, 1>(Pack<1>{{oop}}, Pack<1>{{0.0}}, SumOp<1>(), s_scan, tot);
  const int M = (int)tot.v[0];
  if (M == 0) return false;
  const bool in_lds = M <= WAKE_SORTCAP;
  double* kr = reinterpret_cast<double*>(region);
  int32_t* ki = reinterpret_cast<int32_t*>(kr + WAKE_SORTCAP);
  int32_t* ks = ki + WAKE_SORTCAP;
  int j = (int)j0p.v[0];
  #pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const int sl = k * NT + tid;
    if (I.flag[sl]) continue;
    I.free_slot[j] = sl;
    const double r = I.rho[buf][sl];
    const int32_t id = I.id[buf][sl];
    if (in_lds) { kr[j] = r; ki[j] = id; ks[j] = sl; }
    else { I.sk_r[0][j] = r; I.sk_i[0][j] = id; I.sk_s[0][j] = sl; }
    ++j;
  }
  __syncthreads();
  const double* Kr;
  const int32_t* Ki;
  const int32_t* Ks;
  if (in_lds) {
    int P = 1;
    while (P < M) P <<= 1;
    for (int i = M + tid; i < P; i += NT) { kr[i] = INFINITY; ki[i] = 0x7fffffff - i; ks[i] = -1; }
    __syncthreads();
    bitonic_keys<NT>(kr, ki, ks, P);
    Kr = kr; Ki = ki; Ks = ks;
  } else {
    const int b = sort_keys_global<NT>(I, M, kr, ki, ks);
    Kr = I.sk_r[b]; Ki = I.sk_i[b]; Ks = I.sk_s[b];
  }
  // j-th smallest out-of-place ring -> j-th freed position (via tmp)
  for (int q = tid; q < M; q += NT) {
    const int src = Ks[q], dst = I.free_slot[q];
    I.rho[tmp][dst] = Kr[q]; I.id[tmp][dst] = Ki[q];
    I.u[tmp][dst] = I.u[buf][src]; I.fr[tmp][dst] = I.fr[buf][src]; I.fu[tmp][dst] = I.fu[buf][src];
    I.hint[tmp][dst] = I.hint[buf][src];
    I.g0[dst] = I.lnh[src]; I.g1[dst] = I.lnl[src];
  }
  __syncthreads();
  for (int q = tid; q < M; q += NT) {
    const int dst = I.free_slot[q];
    I.rho[buf][dst] = I.rho[tmp][dst]; I.id[buf][dst] = I.id[tmp][dst];
    I.u[buf][dst] = I.u[tmp][dst]; I.fr[buf][dst] = I.fr[tmp][dst]; I.fu[buf][dst] = I.fu[tmp][dst];
    I.hint[buf][dst] = I.hint[tmp][dst];
    I.lnh[dst] = I.g0[dst]; I.lnl[dst] = I.g1[dst];
  }
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// the slice marcher
// ---------------------------------------------------------------------------
struct FwdMatSumOp {  // (forward matrix product: earlier applied first, running sum)
  __device__ __forceinline__ Pack<5> operator()(const Pack<5>& a, const Pack<5>& b) const {
    Pack<4> m = mat_mul({{b.v[0], b.v[1], b.v[2], b.v[3]}}, {{a.v[0], a.v[1], a.v[2], a.v[3]}});
    return {{m.v[0], m.v[1], m.v[2], m.v[3], a.v[4] + b.v[4]}};
  }
};
struct BwdMatSumOp {  // (index-order product of inverse transfers, running sum)
  __device__ __forceinline__ Pack<5> operator()(const Pack<5>& lo, const Pack<5>& hi) const {
    Pack<4> m = mat_mul({{lo.v[0], lo.v[1], lo.v[2], lo.v[3]}}, {{hi.v[0], hi.v[1], hi.v[2], hi.v[3]}});
    return {{m.v[0], m.v[1], m.v[2], m.v[3], lo.v[4] + hi.v[4]}};
  }
};
struct DDSumOp {      // one double-double sum
  __device__ __forceinline__ Pack<2> operator()(const Pack<2>& a, const Pack<2>& b) const {
    const dd s = dd_add({a.v[0], a.v[1]}, {b.v[0], b.v[1]});
    return {{s.hi, s.lo}};
  }
};

template <int NT>
struct MarchLds {
  static constexpr int NW = NT / 64;
  static constexpr size_t region_bytes() {
    const size_t beam = 2 * WAKE_BCAP * sizeof(double);
    const size_t sort = WAKE_SORTCAP * (sizeof(double) + 2 * sizeof(int32_t));
    const size_t nb = NT * (sizeof(double) + sizeof(int32_t));
    size_t m = beam > sort ? beam : sort;
    return m > nb ? m : nb;
  }
  static constexpr size_t bytes() { return sizeof(double) * (NW * 16 + 64) + region_bytes(); }
};

template <int NT>
__device__ void march(const WakeInst& I, unsigned char* smem) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x;
  const int N = I.N;
  const int C = I.C;
  const int cnt = max(0, min(C, N - tid * C));   // rings owned by this thread

  double* s_scan = reinterpret_cast<double*>(smem);       // NW * 16
  double* s_misc = s_scan + NW * 16;                       // 64
  unsigned char* region = reinterpret_cast<unsigned char*>(s_misc + 64);
  double* s_br = reinterpret_cast<double*>(region);        // beam radii
  double* s_bc = s_br + WAKE_BCAP;                         // beam cumulative charge

  if (I.ctl[CTL_BREAK] >= 0) return;
  int cur = I.ctl[CTL_CUR];
  __syncthreads();
  fix_order<NT>(I, cur, 1 - cur, s_scan, region);   // injected states may be unsorted
  const dd tot0 = {I.tot0[0], I.tot0[1]};
  const double dxi = I.dxi;

  // per-thread sums of (w, w ln rho) for the next slice's prefix
  dd sw = {0.0, 0.0}, swl = {0.0, 0.0};
  bool have_ln = false;

  for (int step = 0; step < I.count; ++step) {
    const int n = I.first + step;
    const double xi = n * dxi;
    const bool do_push = n < I.n_xi - 1;
    const bool rec_snap = I.stride > 0 && (n % I.stride) == 0;
    const bool rec_last = step == I.count - 1;
    const int nb = 1 - cur;
    double* const rho_c = I.rho[cur];
    double* const u_c = I.u[cur];
    const int32_t* const id_c = I.id[cur];
    int32_t* const hint_c = I.hint[cur];

    // ---- loop A: ln rho of every ring (only when not carried over) ----
    if (!have_ln) {
      sw = {0.0, 0.0};
      swl = {0.0, 0.0};
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const int sl = k * NT + tid;
        const int id = id_c[sl];
        const double w = I.w[id];
        const dd lr = ring_log(I, id, rho_c[sl]);
        I.lnh[sl] = lr.hi;
        I.lnl[sl] = lr.lo;
        sw = dd_add_d(sw, w);
        swl = dd_add(swl, dd_mul_d(lr, w));
      }
    }
    // ---- Gauss/log prefix: sum_{k<i} w_k, sum_{k<i} w_k ln rho_k ----
    Pack<4> t4;
    const Pack<4> pre = block_prefix<NT, 4>(Pack<4>{{sw.hi, sw.lo, swl.hi, swl.lo}},
                                            Pack<4>{{0, 0, 0, 0}}, DD2Op(), s_scan, t4);
    const dd totl = {t4.v[2], t4.v[3]};
    const double psi_axis = dd_round(dd_sub(totl, tot0));

    // ---- this slice's analytic source constants (slice-dependent factors) ----
    // beams: lam += c0 * (-expm1(-rho^2 * c1)); lasers: |a|^2 = c0 exp(-rho^2 c1)
    if (tid < I.n_an) {
      const WakeAnalytic& A = I.an[tid];
      if (A.kind == 2) {
        const double s2 = A.sigma_r * A.sigma_r;
        const double dl = xi - A.xi_c;
        const double lon = exp(-(dl * dl) / (2.0 * A.sigma_xi * A.sigma_xi));
        s_misc[3 * tid] = 2.0;
        s_misc[3 * tid + 1] = A.q * A.n_peak * lon * s2;
        s_misc[3 * tid + 2] = 1.0 / (2.0 * s2);
      } else {
        const double dl = xi - A.xi_l;
        const double lon = exp(-2.0 * dl * dl / (A.L * A.L));
        s_misc[3 * tid] = 3.0;
        s_misc[3 * tid + 1] = A.a0 * A.a0 * lon;
        s_misc[3 * tid + 2] = 2.0 / (A.w0 * A.w0);
      }
    }
    const int n_an = I.n_an;

    // ---- stage this slice's beam table ----
    const int bt0 = I.nb ? I.boff[n] : 0;
    const int bm = I.nb ? I.boff[n + 1] - bt0 : 0;
    const bool staged = bm <= WAKE_BCAP;
    if (bm > 0 && staged) {
      for (int i = tid; i < bm; i += NT) { s_br[i] = I.br[bt0 + i]; s_bc[i] = I.bcum[bt0 + i]; }
    }
    __syncthreads();

    // ---- loop B: psi family, sources, local quantities, transfer product ----
    dd S = {pre.v[0], pre.v[1]}, PT = {pre.v[2], pre.v[3]};
    Pack<4> P = mat_ident();
    double vs = 0.0, bad = 0.0;
    int blo = 0;
    #pragma unroll 1
    for (int k = 0; k < cnt; ++k) {
      const int sl = k * NT + tid;
      const double rho = rho_c[sl], u = u_c[sl];
      const int id = id_c[sl];
      int h = hint_c[sl];
      const double w = I.w[id], wh = I.wh[id];
      const dd lnr = {I.lnh[sl], I.lnl[sl]};
      const double irho = 1.0 / rho;
      const dd PTi = dd_add(PT, dd_mul_d(lnr, w));
      const dd pe = dd_sub(dd_mul(dd_add_d(S, w), lnr), PTi);    // psi_e - sum w ln rho
      const dd de = dd_div_rcp(dd_add_d(S, wh), rho, irho);         // d_rho psi_e (self w^)
      dd ips, idp;
      ion_fields(I, rho, lnr, h, ips, idp);
      const double psi = dd_round(dd_add(pe, ips)) + psi_axis;
      const double dpsi = dd_round(dd_add(de, idp));
      S = dd_add_d(S, w);
      PT = PTi;
      // beam charge inside rho (strictly below), analytic beams, lasers
      double lam = 0.0;
      if (bm > 0) {
        int c = 0;
        if (staged) {
          int lo = blo, hi = bm;
          while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if (s_br[m] < rho) lo = m + 1; else hi = m;
          }
          c = lo;
          blo = lo;
          if (c > 0) lam = s_bc[c - 1];
        } else {
          int lo = 0, hi = bm;
          while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if (I.br[bt0 + m] < rho) lo = m + 1; else hi = m;
          }
          c = lo;
          if (c > 0) lam = I.bcum[bt0 + c - 1];
        }
      }
      double aa = 0.0, dda = 0.0;
#pragma unroll 1
      for (int s = 0; s < n_an; ++s) {
        const double kind = s_misc[3 * s], c0 = s_misc[3 * s + 1], c1 = s_misc[3 * s + 2];
        if (kind == 2.0) {
          lam += c0 * (-expm1(-rho * rho * c1));
        } else {
          const double x = c0 * exp(-rho * rho * c1);
          aa += x;
          dda += -(2.0 * rho * c1) * x;
        }
      }
      const double bb = lam * irho;
      const Local L = local_of(irho, u, w, psi, aa);
      if (!(L.pb > 0.0)) bad = 1.0;
      P = mat_mul(rec_matrix(L.A, rho, irho), P);
      vs += L.v;
      I.psi[sl] = psi;
      I.dpsi[sl] = dpsi;
      I.bb[sl] = bb;
      if (I.has_laser) { I.a2[sl] = aa; I.da2[sl] = dda; }
      hint_c[sl] = h;
    }

    // ---- growing mode g (prefix) and decaying mode h (suffix) ----
    Pack<5> gp, gt, hs, ht;
    block_prefix_suffix<NT, 5, 5>(Pack<5>{{P.v[0], P.v[1], P.v[2], P.v[3], vs}},
                                  Pack<5>{{1.0, 0.0, 0.0, 1.0, 0.0}}, FwdMatSumOp(),
                                  Pack<5>{{P.v[3], -P.v[1], -P.v[2], P.v[0], vs}},   // adj(P)
                                  Pack<5>{{1.0, 0.0, 0.0, 1.0, 0.0}}, BwdMatSumOp(), s_scan, gp, gt,
                                  hs, ht);
    const double W = gt.v[0];                 // det[g_N, (0,1)]
    const double iW = 1.0 / W;
    const double Vtot = gt.v[4];
    const double hea = hs.v[1], heb = hs.v[3];   // h at the end of this chunk
    const double Vafter = hs.v[4];

    // ---- loop C: store g_{i-1}; sums of det[g_i, s0_i], det[g_i, s1_i] ----
    double ga = gp.v[0], gb = gp.v[2];
    double V = gp.v[4];
    double le0 = 0.0, le1 = 0.0;
    #pragma unroll 1
    for (int k = 0; k < cnt; ++k) {
      const int sl = k * NT + tid;
      const double rho = rho_c[sl], u = u_c[sl];
      const int id = id_c[sl];
      const double w = I.w[id], wh = I.wh[id];
      const double psi = I.psi[sl], dpsi = I.dpsi[sl], bb = I.bb[sl];
      const double a2 = I.has_laser ? I.a2[sl] : 0.0, da2 = I.has_laser ? I.da2[sl] : 0.0;
      const double irho = 1.0 / rho;
      const Local L = local_of(irho, u, w, psi, a2);
      I.g0[sl] = ga;
      I.g1[sl] = gb;
      const Pack<4> M = rec_matrix(L.A, rho, irho);
      const double na = M.v[0] * ga + M.v[1] * gb;
      const double nbg = M.v[2] * ga + M.v[3] * gb;
      ga = na;
      gb = nbg;
      V += L.v;
      const double dz0 = V - (w - wh) * u * irho * L.ipb;    // d_zeta psi + V_total
      double B0, C;
      ring_BC(irho, u, w, L, dpsi, dz0, bb, da2, B0, C);
      const double B1 = w * irho * u * L.ipb * L.ipb;         // dB/dV_total
      double s0a, s0b;
      rec_offset(L.A, B0, C, rho, s0a, s0b);
      const double s1a = 0.5 * B1, s1b = -0.5 * rho * rho * B1;
      le0 += ga * s0b - gb * s0a;
      le1 += ga * s1b - gb * s1a;
    }

    // ---- loop D: sum of det[s_i, h_i] ----
    double ha = hea, hb = heb;
    double Vgt = Vafter;
    double lds = 0.0;
    #pragma unroll 1
    for (int k = cnt - 1; k >= 0; --k) {
      const int sl = k * NT + tid;
      const double rho = rho_c[sl], u = u_c[sl];
      const int id = id_c[sl];
      const double w = I.w[id], wh = I.wh[id];
      const double psi = I.psi[sl], dpsi = I.dpsi[sl], bb = I.bb[sl];
      const double a2 = I.has_laser ? I.a2[sl] : 0.0, da2 = I.has_laser ? I.da2[sl] : 0.0;
      const double irho = 1.0 / rho;
      const Local L = local_of(irho, u, w, psi, a2);
      const double dz = -(Vgt + (w - wh) * u * irho * L.ipb);
      double B, C;
      ring_BC(irho, u, w, L, dpsi, dz, bb, da2, B, C);
      double sa, sb;
      rec_offset(L.A, B, C, rho, sa, sb);
      lds += sa * hb - sb * ha;
      const double hh = 0.5 * L.A * rho;
      const double na = (1.0 - hh) * ha - (0.5 * L.A * irho) * hb;
      const double nbh = (hh * rho * rho) * ha + (1.0 + hh) * hb;
      ha = na;
      hb = nbh;
      Vgt += L.v;
    }
    Pack<2> ep, et;
    Pack<1> dsf, dt;
    block_prefix_suffix<NT, 2, 1>(Pack<2>{{le0, le1}}, Pack<2>{{0.0, 0.0}}, SumOp<2>(),
                                  Pack<1>{{lds}}, Pack<1>{{0.0}}, SumOp<1>(), s_scan, ep, et, dsf, dt);

    // ---- loop E: B^(p), outputs, push ----
    ha = hea; hb = heb;
    Vgt = Vafter;
    double D = dsf.v[0];
    double E = (ep.v[0] + le0) + Vtot * (ep.v[1] + le1);
    double disorder = 0.0;
    double nxt_r = INFINITY;
    int32_t nxt_i = 0x7fffffff;
    dd sw2 = {0.0, 0.0}, swl2 = {0.0, 0.0};
    double* const rho_n = I.rho[nb];
    double* const u_n = I.u[nb];
    #pragma unroll 1
    for (int k = cnt - 1; k >= 0; --k) {
      const int sl = k * NT + tid;
      const double rho = rho_c[sl], u = u_c[sl];
      const int id = id_c[sl];
      const double w = I.w[id], wh = I.wh[id];
      const double psi = I.psi[sl], dpsi = I.dpsi[sl], bb = I.bb[sl];
      const double a2 = I.has_laser ? I.a2[sl] : 0.0, da2 = I.has_laser ? I.da2[sl] : 0.0;
      const double ga0 = I.g0[sl], gb0 = I.g1[sl];
      const double irho = 1.0 / rho;
      const Local L = local_of(irho, u, w, psi, a2);
      const double dz = -(Vgt + (w - wh) * u * irho * L.ipb);
      double B, C;
      ring_BC(irho, u, w, L, dpsi, dz, bb, da2, B, C);
      double sa, sb;
      rec_offset(L.A, B, C, rho, sa, sb);
      const double ds = sa * hb - sb * ha;                 // det[s_i, h_i]
      const Pack<4> M = rec_matrix(L.A, rho, irho);
      const double gia = M.v[0] * ga0 + M.v[1] * gb0;
      const double gib = M.v[2] * ga0 + M.v[3] * gb0;
      const double e = gia * sb - gib * sa;                // det[g_i, s_i]
      D += ds;                                             // D_{i-1}
      E -= e;                                              // E_{i-1}
      const double hh = 0.5 * L.A * rho;
      const double hpa = (1.0 - hh) * ha - (0.5 * L.A * irho) * hb;   // h_{i-1}
      const double hpb = (hh * rho * rho) * ha + (1.0 + hh) * hb;
      const double a = (hpa * E - ga0 * D) * iW;
      const double b = (hpb * E - gb0 * D) * iW;
      const double bp = a * rho + b * irho + (wh / w) * C;
      const double bt = bb + bp;
      const double ez = -dz;
      if (!(isfinite(psi) && isfinite(dpsi) && isfinite(ez) && isfinite(bt))) bad = 1.0;
      if (rec_snap) {
        double* sp = I.snap + (size_t)(n / I.stride) * OUT_N * N;
        sp[OUT_PSI * N + id] = psi; sp[OUT_ERBT * N + id] = -dpsi;
        sp[OUT_EZ * N + id] = ez; sp[OUT_BT * N + id] = bt;
        sp[OUT_RHO * N + id] = rho; sp[OUT_UR * N + id] = u;
      }
      if (rec_last) {
        double* sp = I.last;
        sp[OUT_PSI * N + id] = psi; sp[OUT_ERBT * N + id] = -dpsi;
        sp[OUT_EZ * N + id] = ez; sp[OUT_BT * N + id] = bt;
        sp[OUT_RHO * N + id] = rho; sp[OUT_UR * N + id] = u;
      }
      if (do_push) {
        const double f_r = u * L.ipb;
        const double f_u = L.gm * dpsi * L.ipb - bt - 0.25 * da2 * L.ipb;
        double pr = f_r, pu = f_u;
        if (n > 0) { pr = I.fr[cur][sl]; pu = I.fu[cur][sl]; }
        double rn = rho + dxi * (1.5 * f_r - 0.5 * pr);
        double un = u + dxi * (1.5 * f_u - 0.5 * pu);
        double sr = f_r, su = f_u;
        if (rn < 0.0) { rn = -rn; un = -un; sr = -sr; su = -su; }
        if (!(isfinite(rn) && isfinite(un))) bad = 1.0;
        rho_n[sl] = rn; u_n[sl] = un; I.fr[nb][sl] = sr; I.fu[nb][sl] = su;
        I.id[nb][sl] = id; I.hint[nb][sl] = hint_c[sl];
        const dd lr = ring_log(I, id, rn);
        I.lnh[sl] = lr.hi;
        I.lnl[sl] = lr.lo;
        sw2 = dd_add_d(sw2, w);
        swl2 = dd_add(swl2, dd_mul_d(lr, w));
        if (!key_lt(rn, id, nxt_r, nxt_i)) disorder = 1.0;
        nxt_r = rn;
        nxt_i = id;
      }
      ha = hpa;
      hb = hpb;
      Vgt += L.v;
    }
    // order across chunk boundaries
    double* s_fr = reinterpret_cast<double*>(region);
    int32_t* s_fi = reinterpret_cast<int32_t*>(s_fr + NT);
    if (do_push) {
      __syncthreads();
      s_fr[tid] = nxt_r;      // this chunk's first pushed key (+inf if empty)
      s_fi[tid] = nxt_i;
      __syncthreads();
      if (cnt > 0 && tid + 1 < NT && (tid + 1) * C < N) {
        const int sl_last = (cnt - 1) * NT + tid;
        const double lr = rho_n[sl_last];
        const int32_t li = I.id[nb][sl_last];
        if (!key_lt(lr, li, s_fr[tid + 1], s_fi[tid + 1])) disorder = 1.0;
      }
    }
    Pack<2> red;
    block_prefix<NT, 2>(Pack<2>{{bad, disorder}}, Pack<2>{{0.0, 0.0}}, SumOp<2>(), s_scan, red);
    if (tid == 0) { I.axis[2 * n] = psi_axis; I.axis[2 * n + 1] = Vtot; }
    if (red.v[0] != 0.0) {
      if (tid == 0) { I.ctl[CTL_BREAK] = n; I.ctl[CTL_CUR] = cur; I.ctl[CTL_NEXT] = n; }
      return;
    }
    if (!do_push) {
      if (tid == 0) { I.ctl[CTL_CUR] = cur; I.ctl[CTL_NEXT] = n + 1; }
      return;
    }
    cur = nb;
    sw = sw2;
    swl = swl2;
    have_ln = true;
    if (red.v[1] != 0.0 && fix_order<NT>(I, cur, 1 - cur, s_scan, region)) {
      // the chunks changed: rebuild the per-thread sums from the moved ln rho
      sw = {0.0, 0.0};
      swl = {0.0, 0.0};
      #pragma unroll 1
      for (int k = 0; k < cnt; ++k) {
        const int sl = k * NT + tid;
        const double w = I.w[I.id[cur][sl]];
        sw = dd_add_d(sw, w);
        swl = dd_add(swl, dd_mul_d(dd{I.lnh[sl], I.lnl[sl]}, w));
      }
    }
    __syncthreads();
  }
  if (tid == 0) { I.ctl[CTL_CUR] = cur; I.ctl[CTL_NEXT] = I.first + I.count; }
}

// 2 waves per SIMD: up to 256 VGPRs per lane, no spills
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
void wake_march_kernel(const WakeInst* __restrict__ insts, int n_insts, int32_t* counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_idx;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= n_insts) return;   // every workgroup leaves once the queue is empty
    if (insts[idx].nt == NT) march<NT>(insts[idx], smem);
    __syncthreads();
  }
}

__global__ void counter_zero_kernel(int32_t* p) {
  if (threadIdx.x == 0) p[0] = 0;
}

// ---------------------------------------------------------------------------
// state transfers by ring id, reset
// ---------------------------------------------------------------------------
__global__ void state_by_id_kernel(WakeInst I, double* rho, double* u, double* fr, double* fu) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= I.N) return;
  const int c = I.ctl[CTL_CUR];
  const int sl = (p % I.C) * I.nt + p / I.C;
  const int i = I.id[c][sl];
  if (rho) rho[i] = I.rho[c][sl];
  if (u) u[i] = I.u[c][sl];
  if (fr) fr[i] = I.fr[c][sl];
  if (fu) fu[i] = I.fu[c][sl];
}

// Injected state (by id) at position = id in buffer 0; the marcher orders
// it before its first slice.  Interval hints start at the rings' nodes.
__global__ void state_set_kernel(WakeInst I, const double* rho, const double* u, const double* fr,
                                 const double* fu, int slice) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) { I.ctl[CTL_CUR] = 0; I.ctl[CTL_BREAK] = -1; I.ctl[CTL_NEXT] = slice; }
  if (i >= I.N) return;
  const int sl = (i % I.C) * I.nt + i / I.C;
  I.rho[0][sl] = rho[i];
  I.u[0][sl] = u[i];
  I.fr[0][sl] = fr ? fr[i] : 0.0;
  I.fu[0][sl] = fu ? fu[i] : 0.0;
  I.id[0][sl] = i;
  I.hint[0][sl] = i + 1;
}

// Back to the state at slice 0 (rings at rest at their initial radii);
// one workgroup per instance.
__global__ void state_reset_kernel(const WakeInst* __restrict__ insts, int n_insts) {
  const WakeInst& I = insts[blockIdx.x];
  for (int j = threadIdx.x; j < I.N; j += blockDim.x) {
    const int sl = (j % I.C) * I.nt + j / I.C;
    I.rho[0][sl] = I.r0[j];
    I.u[0][sl] = 0.0;
    I.fr[0][sl] = 0.0;
    I.fu[0][sl] = 0.0;
    I.id[0][sl] = j;
    I.hint[0][sl] = j + 1;
  }
  if (threadIdx.x == 0) { I.ctl[CTL_CUR] = 0; I.ctl[CTL_BREAK] = -1; I.ctl[CTL_NEXT] = 0; }
}

// ---------------------------------------------------------------------------
// host-callable launchers
// ---------------------------------------------------------------------------
hipError_t launch_init(const WakeInst& I, const double* r0, const double* dr, const double* dens,
                       hipStream_t s) {
  hipLaunchKernelGGL((wake_init_kernel<256>), dim3(1), dim3(256), 0, s, I, r0, dr, dens);
  return hipGetLastError();
}

hipError_t launch_reset(const WakeInst* d_insts, int n_insts, hipStream_t s) {
  if (n_insts <= 0) return hipSuccess;
  hipLaunchKernelGGL(state_reset_kernel, dim3(n_insts), dim3(256), 0, s, d_insts, n_insts);
  return hipGetLastError();
}

hipError_t launch_state_by_id(const WakeInst& I, double* rho, double* u, double* fr, double* fu,
                              hipStream_t s) {
  hipLaunchKernelGGL(state_by_id_kernel, dim3((I.N + 255) / 256), dim3(256), 0, s, I, rho, u, fr, fu);
  return hipGetLastError();
}

hipError_t launch_state_set(const WakeInst& I, const double* rho, const double* u, const double* fr,
                            const double* fu, int slice, hipStream_t s) {
  hipLaunchKernelGGL(state_set_kernel, dim3((I.N + 255) / 256), dim3(256), 0, s, I, rho, u, fr, fu,
                     slice);
  return hipGetLastError();
}

#define WAKE_THREADS(X) X(256) X(512) X(1024)

size_t march_lds_bytes(int nt) {
#define X(a) \
  if (nt == a) return MarchLds<a>::bytes();
  WAKE_THREADS(X)
#undef X
  return 0;
}

hipError_t launch_march(int nt, const WakeInst* d_insts, int n_insts, int32_t* counter, int grid,
                        hipStream_t s) {
#define X(a)                                                                                      \
  if (nt == a) {                                                                                  \
    hipLaunchKernelGGL(counter_zero_kernel, dim3(1), dim3(64), 0, s, counter);                     \
    hipLaunchKernelGGL((wake_march_kernel<a>), dim3(grid), dim3(a), MarchLds<a>::bytes(), s,       \
                       d_insts, n_insts, counter);                                                 \
    return hipGetLastError();                                                                     \
  }
  WAKE_THREADS(X)
#undef X
  return hipErrorInvalidValue;
}

int march_occupancy(int nt) {
  int nb = 0;
#define X(a)                                                                                      \
  if (nt == a) {                                                                                  \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, wake_march_kernel<a>, a,                \
                                                     MarchLds<a>::bytes()) != hipSuccess)         \
      return 0;                                                                                   \
    return nb;                                                                                    \
  }
  WAKE_THREADS(X)
#undef X
  return 0;
}

hipError_t march_prepare(int nt) {
#define X(a)                                                                                      \
  if (nt == a)                                                                                    \
    return hipFuncSetAttribute((const void*)wake_march_kernel<a>,                                 \
                               hipFuncAttributeMaxDynamicSharedMemorySize,                        \
                               (int)MarchLds<a>::bytes());
  WAKE_THREADS(X)
#undef X
  return hipErrorInvalidValue;
}

bool march_threads_ok(int nt) {
#define X(a) \
  if (nt == a) return true;
  WAKE_THREADS(X)
#undef X
  return false;
}
