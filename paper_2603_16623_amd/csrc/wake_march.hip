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
// The recursion x_i = M_i x_{i-1} + s_i (x = (a, b), det M_i = 1) is solved
// in Green's-function form: with the growing mode g (g_0 = (1, 0),
// g_i = M_i g_{i-1}), the decaying mode h (h_N = (0, 1), h_{i-1} = M_i^-1
// h_i) and W = det[g, h] = a-part of g_N,
//   x_i = (h_i E_i - g_i D_i) / W,  E_i = sum_{j<=i} det[g_j, s_j],
//                                    D_i = sum_{j>i}  det[s_j, h_j].
// It solves the same linear system as the paper's shooting (Appendix "Solve
// recursive system") without its exponential loss of digits.
//
// One workgroup owns one instance and marches its slices; thread t owns the
// C = ceil(N / NT) consecutive sorted positions [t*C, t*C + C), stored in
// slots k*NT + t (coalesced).  Two passes over the rings per slice:
//   pass B (forward)  psi, d_rho psi from a double-double prefix of
//                     (w, w ln rho); sources; psibar, gamma, A_i, M_i; the
//                     chunk product G of the M_i and the chunk sum of v_i;
//                     lambda = sum_i G_i^T J s_i with G_i the product up to
//                     ring i and J s = (s_b, -s_a), split as lambda0 +
//                     c lambda1 because s_i is affine in the one unknown
//                     c = -(v of this chunk and every later one).
//   scan              prefix of (G, v) (g at the chunk start), suffix of
//                     (G^-1, v) (h at the chunk end).  The chunk's sums are
//                     then det-sums without another pass:
//                     sum det[g_i, s_i] = g_start . lambda,
//                     sum det[s_i, h_i] = -(G^-1 h_end) . lambda.
//   scan              prefix of the det[g, s] sums, suffix of det[s, h].
//   pass E (backward) s_i again, g and h stepped back by M_i^-1, x_{i-1},
//                     B^(p), outputs, AB2 push, ln rho of the pushed radius.
// If the pushed radii are out of order, runs of positions that must be
// permuted among themselves are found (a run boundary sits where every key
// before is below every key after); short runs are ranked in place, the
// rings of long runs are compacted, sorted and dropped into their freed
// positions.
#include "wake_common.h"
#include "wake_device.h"
#include "wake_cluster.h"
#include "wake_ring.h"
#include "wake_launch.h"

#include <math.h>

// A per-instance array seen as uniform: its base in scalar registers and in
// the global address space, indexed with 32-bit element offsets (loads and
// stores then take the scalar-base + vector-offset form).
template <class T>
struct GA {
  WAKE_GLOBAL T* p;
  __device__ __forceinline__ T operator[](uint32_t i) const {
    return *reinterpret_cast<WAKE_GLOBAL T*>(reinterpret_cast<WAKE_GLOBAL char*>(p) +
                                            i * (uint32_t)sizeof(T));
  }
  __device__ __forceinline__ void st(uint32_t i, T v) const {
    *reinterpret_cast<WAKE_GLOBAL T*>(reinterpret_cast<WAKE_GLOBAL char*>(p) +
                                     i * (uint32_t)sizeof(T)) = v;
  }
};
template <class T>
__device__ __forceinline__ GA<T> uview(const T* q) {
  const uint64_t v = reinterpret_cast<uint64_t>(q);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  GA<T> g;
  g.p = reinterpret_cast<WAKE_GLOBAL T*>(((uint64_t)hi << 32) | lo);
  return g;
}
__device__ __forceinline__ double uni(double x) {
  const uint64_t v = __double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// 16-B chunk of a record (two doubles), moved by one 16-B load or store.
typedef double D2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ D2 d2(double x, double y) {
  D2 r;
  r.x = x;
  r.y = y;
  return r;
}
// A record array kept as planes of 16-B chunks: chunk c of record i sits at
// c * ps + i (ps = slots per plane), so a wave's accesses to one chunk are
// contiguous 16-B lanes.  One uniform base per array.
struct PV {
  GA<D2> g;
  uint32_t ps;
  __device__ __forceinline__ D2 ld(uint32_t c, uint32_t i) const { return g[c * ps + i]; }
  __device__ __forceinline__ void st(uint32_t c, uint32_t i, D2 v) const { g.st(c * ps + i, v); }
  // one double of a chunk (half 0: x, 1: y), an 8-B access
  __device__ __forceinline__ double ldh(uint32_t c, uint32_t i, int half) const {
    return *reinterpret_cast<WAKE_GLOBAL double*>(reinterpret_cast<WAKE_GLOBAL char*>(g.p) +
                                                 (c * ps + i) * 16u + half * 8u);
  }
  __device__ __forceinline__ void sth(uint32_t c, uint32_t i, int half, double v) const {
    *reinterpret_cast<WAKE_GLOBAL double*>(reinterpret_cast<WAKE_GLOBAL char*>(g.p) + (c * ps + i) * 16u +
                                          half * 8u) = v;
  }
  // word i of the plane of 4-B words that starts where chunk c would
  __device__ __forceinline__ int32_t ldi(uint32_t c, uint32_t i) const {
    return reinterpret_cast<WAKE_GLOBAL const int32_t*>(g.p)[4u * c * ps + i];
  }
  __device__ __forceinline__ void sti(uint32_t c, uint32_t i, int32_t v) const {
    reinterpret_cast<WAKE_GLOBAL int32_t*>(g.p)[4u * c * ps + i] = v;
  }
};
__device__ __forceinline__ PV pview(const double* p, uint32_t ps) {
  PV v;
  v.g = uview(reinterpret_cast<const D2*>(p));
  v.ps = __builtin_amdgcn_readfirstlane(ps);
  return v;
}
// sort keys of the ring at slot sl of a state buffer
__device__ __forceinline__ double st_rho(const PV& S, unsigned sl) { return S.ldh(RS_RU, sl, 0); }
__device__ __forceinline__ int32_t st_hs(const PV& S, unsigned sl) { return S.ldi(RS_W, sl); }
// the ring's ion-interval hint (instances without the LDS node table)
__device__ __forceinline__ int32_t st_hint(const PV& S, unsigned sl) { return S.ldi(RS_W, S.ps + sl); }

// ln(rho) of the ring with home slot hs as ln r0 + log1p((rho - r0)/r0): its
// rounding scales with the ring's displacement, not with |ln rho| (the psi
// sums multiply ln rho by the enclosed charge).  r: (r0, 1/r0), l: ln r0.
__device__ __forceinline__ dd ring_log(D2 r, D2 l, double rho) {
  const double l1 = log1p_fast((rho - r.x) * r.y);
  return dd_add_d({l.x, l.y}, l1);
}

template <int NT>
__device__ __forceinline__ int32_t id_of(int32_t hs, int C) {
  return (hs & (NT - 1)) * C + (hs >> __builtin_ctz(NT));
}

// slot of position p (member g = p / (C nt) of a cooperative instance uses
// the single-workgroup layout shifted by g C nt; g = 0 otherwise)
__device__ __forceinline__ unsigned slot_of(int p, int C, int nt) {
  const int P = C * nt, g = p / P, q = p - g * P;
  return (unsigned)(g * P + (q % C) * nt + q / C);
}
// position of slot s (the ring id of home slot s)
__device__ __forceinline__ int pos_of_slot(int s, int C, int nt) {
  const int P = C * nt, g = s / P, r = s - g * P;
  return g * P + (r % nt) * C + r / nt;
}

// Ion psi - psi(0) and d_rho psi at radius r: linear interpolation inside
// the node interval containing r (Sec. "Key algorithmic adjustments"),
// searched from the ring's previous interval h; exact exterior field at and
// beyond the plasma edge.
// Ion fields need: the records R, their count N, the plasma edge Rp and the
// exterior constants (sum w ln r0 as dd, Q as dd).
struct IonView {
  GA<double> R;
  int N;
  double Rp;
  dd T0, Q;
};

// The record of the interval a hint points at (loaded ahead of its use).
__device__ __forceinline__ void ion_load(const IonView& V, int h, double* q) {
  const int j = h < 0 ? 0 : (h > V.N ? V.N : h);
#pragma unroll
  for (int i = 0; i < WAKE_ION_REC; ++i) q[i] = V.R[j * WAKE_ION_REC + i];
}

// q: the record ion_load gave for the same hint h.
__device__ __forceinline__ void ion_fields(const IonView& V, double r, dd lnr, int& h, double* q, dd& ps,
                                           dd& dp) {
  if (!(r < V.Rp)) {
    ps = dd_sub(V.T0, dd_mul(V.Q, lnr));
    dp = dd_neg(dd_div_d(V.Q, r));
    return;
  }
  const GA<double>& R = V.R;
  const int N = V.N;
  int j = h < 0 ? 0 : (h > N ? N : h);
  if (!(q[IR_LO] <= r && r < q[IR_HI])) {
    if (q[IR_LO] <= r) {
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
#pragma unroll
    for (int i = 0; i < WAKE_ION_REC; ++i) q[i] = R[j * WAKE_ION_REC + i];
  }
  h = j;
  const double t = (r - q[IR_LO]) * rcp_nr(q[IR_HI] - q[IR_LO]);
  ps = dd_add_d({q[IR_PSH], q[IR_PSL]}, t * q[IR_DPS]);
  dp = dd_add_d({q[IR_DPH], q[IR_DPL]}, t * q[IR_DDP]);
}

// Ion interval of radius r from the interval nodes kept in LDS as floats
// (node j = lower end of record j, j = 0..N): the largest j with
// node_j <= r in float, by a gallop from the guess j then bisection.  The
// record's exact double bounds confirm it when it is used (a radius within
// a float ulp of a node can land one interval off; the exact search in
// ion_fields then corrects it).
__device__ __forceinline__ int ion_find(const float* nodes, int N, double r, int j) {
  const float x = (float)r;
  j = j < 0 ? 0 : (j > N ? N : j);
  int a, b;
  if (nodes[j] <= x) {
    a = j;                                   // nodes[a] <= x
    int step = 1;
    for (;;) {
      b = a + step;
      if (b > N) { b = N + 1; break; }
      if (x < nodes[b]) break;
      a = b;
      step <<= 1;
    }
  } else {
    b = j;                                   // nodes[b] > x
    int step = 1;
    for (;;) {
      a = b - step;
      if (a <= 0) { a = 0; break; }
      if (nodes[a] <= x) break;
      b = a;
      step <<= 1;
    }
  }
  while (b - a > 1) {
    const int m = (a + b) >> 1;
    if (nodes[m] <= x) a = m; else b = m;
  }
  return a;
}
// ---------------------------------------------------------------------------
// ring-set initialisation: weights, ln r0, ion interval records, state
// ---------------------------------------------------------------------------
// Three kernels over the rings' blocks of NT (in ring order), then one
// over the intervals.  Block b's (w, w ln r0) totals go to tmp[4b..4b+3];
// the serial pass turns them into exclusive offsets, in the order a single
// workgroup marching block by block would have summed them.
template <int NT>
__global__ __launch_bounds__(NT) void init_rings_kernel(WakeInst I, const double* __restrict__ r0,
                                                        const double* __restrict__ dr,
                                                        const double* __restrict__ dens, double* tmp) {
  __shared__ double s_scan[(NT / 64) * 8];
  const int N = I.N;
  const int j = blockIdx.x * NT + threadIdx.x;
  D2* cst = reinterpret_cast<D2*>(const_cast<double*>(I.cst));
  D2* st = reinterpret_cast<D2*>(I.st[0]);
  int32_t* st_w = reinterpret_cast<int32_t*>(I.st[0]);
  const size_t PS = (size_t)I.G * I.C * I.nt;      // slots per plane
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
    const unsigned hs = slot_of(j, I.C, I.nt);   // home slot of ring j
    cst[RC_W * PS + hs] = d2(w, wh);
    cst[RC_R0 * PS + hs] = d2(r, 1.0 / r);
    cst[RC_LN * PS + hs] = d2(lr.hi, lr.lo);
    // initial state: position j holds ring j; its interval starts at its node
    st[RS_RU * PS + hs] = d2(r, 0.0);
    st[RS_F * PS + hs] = d2(0.0, 0.0);
    st[RS_LN * PS + hs] = d2(lr.hi, lr.lo);
    st_w[4 * RS_W * PS + hs] = (int32_t)hs;
    st_w[4 * RS_W * PS + PS + hs] = j + 1;
  }
  const dd wl = dd_mul_d(lr, w);
  Pack<4> tot;
  block_prefix<NT, 4>(Pack<4>{{w, 0.0, wl.hi, wl.lo}}, Pack<4>{{0, 0, 0, 0}}, DD2Op(), s_scan, tot);
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) tmp[4 * blockIdx.x + i] = tot.v[i];
}

// One thread: block totals to exclusive offsets, the totals, record 0, control.
__global__ void init_offsets_kernel(WakeInst I, double* tmp, int n_blocks) {
  if (threadIdx.x != 0) return;
  dd cS = {0.0, 0.0}, cPT = {0.0, 0.0};
  for (int b = 0; b < n_blocks; ++b) {
    const dd tS = {tmp[4 * b], tmp[4 * b + 1]}, tPT = {tmp[4 * b + 2], tmp[4 * b + 3]};
    tmp[4 * b] = cS.hi; tmp[4 * b + 1] = cS.lo; tmp[4 * b + 2] = cPT.hi; tmp[4 * b + 3] = cPT.lo;
    cS = dd_add(cS, tS);
    cPT = dd_add(cPT, tPT);
  }
  double* R = const_cast<double*>(I.ion);
  double* consts = const_cast<double*>(I.tot0);
  R[IR_LO] = 0.0;
  R[IR_PSH] = 0.0; R[IR_PSL] = 0.0; R[IR_DPH] = 0.0; R[IR_DPL] = 0.0;
  consts[0] = cPT.hi; consts[1] = cPT.lo;   // sum_j w_j ln r0_j
  consts[2] = cS.hi; consts[3] = cS.lo;     // total weight Q
  I.ctl[CTL_CUR] = 0;
  I.ctl[CTL_BREAK] = -1;
  I.ctl[CTL_NEXT] = 0;
  I.ctl[CTL_FAULT] = 0;
}

// Node values of the ion rings (node j+1 is ring j) into records j+1.
template <int NT>
__global__ __launch_bounds__(NT) void init_nodes_kernel(WakeInst I, const double* __restrict__ tmp) {
  __shared__ double s_scan[(NT / 64) * 8];
  const int N = I.N;
  const int j = blockIdx.x * NT + threadIdx.x;
  const D2* cst = reinterpret_cast<const D2*>(I.cst);
  const size_t PS = (size_t)I.G * I.C * I.nt;
  const bool ok = j < N;
  double w = 0.0, wh = 0.0, r = 1.0;
  dd lr = {0.0, 0.0};
  if (ok) {
    const unsigned hs = slot_of(j, I.C, I.nt);
    const D2 kw = cst[RC_W * PS + hs], kr = cst[RC_R0 * PS + hs], kl = cst[RC_LN * PS + hs];
    w = kw.x; wh = kw.y; r = kr.x; lr = {kl.x, kl.y};
  }
  const dd wl = dd_mul_d(lr, w);
  Pack<4> tot;
  const Pack<4> pre = block_prefix<NT, 4>(Pack<4>{{w, 0.0, wl.hi, wl.lo}}, Pack<4>{{0, 0, 0, 0}},
                                          DD2Op(), s_scan, tot);
  const dd cS = {tmp[4 * blockIdx.x], tmp[4 * blockIdx.x + 1]};
  const dd cPT = {tmp[4 * blockIdx.x + 2], tmp[4 * blockIdx.x + 3]};
  const dd S = dd_add(cS, {pre.v[0], pre.v[1]});
  const dd PTi = dd_add(dd_add(cPT, {pre.v[2], pre.v[3]}), wl);
  if (ok) {
    // ion ring j (q=+1) at its own radius with self weight w^
    const dd dp = dd_neg(dd_div_d(dd_add_d(S, wh), r));
    const dd ps = dd_neg(dd_sub(dd_mul(dd_add_d(S, w), lr), PTi));
    double* rec = const_cast<double*>(I.ion) + (size_t)(j + 1) * WAKE_ION_REC;
    rec[IR_LO] = r;
    rec[IR_PSH] = ps.hi; rec[IR_PSL] = ps.lo;
    rec[IR_DPH] = dp.hi; rec[IR_DPL] = dp.lo;
  }
}

// Interval ends and steps; the last node is the plasma edge.
__global__ void init_intervals_kernel(WakeInst I) {
  const int N = I.N;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > N) return;
  double* R = const_cast<double*>(I.ion);
  const dd cPT = {I.tot0[0], I.tot0[1]}, cS = {I.tot0[2], I.tot0[3]};
  double* rec = R + (size_t)j * WAKE_ION_REC;
  double hi, nps_h, nps_l, ndp_h, ndp_l;
  if (j < N) {
    const double* nx = rec + WAKE_ION_REC;
    hi = nx[IR_LO]; nps_h = nx[IR_PSH]; nps_l = nx[IR_PSL]; ndp_h = nx[IR_DPH]; ndp_l = nx[IR_DPL];
  } else {
    const double Rp = I.Rp;
    const dd eps = dd_sub(cPT, dd_mul(cS, dd_log(Rp)));
    const dd edp = dd_neg(dd_div_d(cS, Rp));
    hi = Rp; nps_h = eps.hi; nps_l = eps.lo; ndp_h = edp.hi; ndp_l = edp.lo;
  }
  rec[IR_HI] = hi;
  rec[IR_DPS] = dd_round(dd_sub({nps_h, nps_l}, {rec[IR_PSH], rec[IR_PSL]}));
  rec[IR_DDP] = dd_round(dd_sub({ndp_h, ndp_l}, {rec[IR_DPH], rec[IR_DPL]}));
}

// ---------------------------------------------------------------------------
// ring order
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

// Fallback order of a cooperative instance, by segments.  A segment
// boundary sits before position p when every key before p is below every
// key from p on; the rings between consecutive boundaries are permuted
// among themselves.  Rings alone in their segment keep their positions; the
// others (M of them) are compacted in position order, sorted together by
// member 0 in LDS, and put back into the positions they left, in order (the
// segments follow each other in key order, so the j-th smallest goes to the
// j-th freed position).  Two exchanges of totals and three fenced ones, in
// place of the bitonic network's one per stage, which remains for M beyond
// the LDS sort (cap bytes at byte offset lo, 16 per key).  Returns the
// barrier count, -1 when a member gave up.
template <int NT>
__device__ __noinline__ int cl_segments(const WAKE_GLOBAL WakeInst* Ig, Cluster cl, int xo, int oko, int lo,
                                        int cap) {
  const WakeInst& I = *(const WakeInst*)Ig;
  double* const s_x = reinterpret_cast<double*>(wake_lds + xo);
  int* const s_ok = reinterpret_cast<int*>(wake_lds + oko);
  constexpr int NW = NT / 64;
  double* const s_scanA = reinterpret_cast<double*>(wake_lds);          // the slice scans' areas
  double* const s_scanB = s_scanA + NW * 16;
  const int tid = threadIdx.x;
  const int N = I.N, C = I.C, P = C * NT;
  const double iC = 1.0 / (double)C, iP = 1.0 / (double)P;
  const int goff = cl.g * P;
  const int Ng = min(P, N - goff);
  const int q0 = tid * C;
  const int cnt = max(0, min(C, Ng - q0));
  double* const L_r = reinterpret_cast<double*>(wake_lds + lo);
  uint64_t* const L_k = reinterpret_cast<uint64_t*>(wake_lds + lo + 8 * P);
  WAKE_GLOBAL int32_t* const perm = gptr(I.perm);
  // this member's keys by position, in the current order
  #pragma unroll 1
  for (int k0 = 0; k0 < cnt; k0 += 8) {
    int src[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) src[j] = k0 + j < cnt ? perm[goff + (k0 + j) * NT + tid] : -1;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (src[j] < 0) continue;
      L_r[q0 + k0 + j] = gptr(I.gk_r)[src[j]];
      L_k[q0 + k0 + j] = ((uint64_t)(uint32_t)gptr(I.gk_i)[src[j]] << 32) | (uint32_t)src[j];
    }
  }
  __syncthreads();
  const Pack<2> k_lo = {{-INFINITY, -2147483648.0}}, k_hi = {{INFINITY, 2147483647.0}};
  // suffix minima inside the chunk, its maximum and minimum
  double sr[16];
  int32_t si[16];
  Pack<2> mx = k_lo, mn = k_hi;
#pragma unroll
  for (int k = 15; k >= 0; --k) {
    if (k < cnt) {
      const Pack<2> x = {{L_r[q0 + k], (double)(int32_t)(L_k[q0 + k] >> 32)}};
      mx = MaxKeyOp()(mx, x);
      mn = MinKeyOp()(mn, x);
    }
    sr[k] = mn.v[0];
    si[k] = (int32_t)mn.v[1];
  }
  Pack<2> tmx, tmn;
  const Pack<2> bmx = block_prefix<NT, 2>(mx, k_lo, MaxKeyOp(), s_scanA, tmx);   // before the chunk
  const Pack<2> bmn = block_suffix<NT, 2>(mn, k_hi, MinKeyOp(), s_scanB, tmn);   // after the chunk
  if (!cl_gather<4, false>(cl, Pack<4>{{tmx.v[0], tmx.v[1], tmn.v[0], tmn.v[1]}}, s_x, s_ok)) return -1;
  Pack<2> gmx, gtot, gmn, gtot2;
  cl_prefix<2, 4>(s_x, 0, cl.g, cl.G, k_lo, MaxKeyOp(), gmx, gtot);    // earlier members
  cl_suffix<2, 4>(s_x, 2, cl.g, cl.G, k_hi, MinKeyOp(), gmn, gtot2);   // later members
  // boundary before position q0 + k: max of every key before it below min
  // of every key from it on; a ring is alone in its segment when there are
  // boundaries before it and after it
  const Pack<2> after = MinKeyOp()(bmn, gmn);
  Pack<2> pm = MaxKeyOp()(gmx, bmx);
  const Pack<2> from0 = MinKeyOp()(Pack<2>{{sr[0], (double)si[0]}}, after);   // every key from q0 on
  bool bnd = key_lt(pm.v[0], (int32_t)pm.v[1], from0.v[0], (int32_t)from0.v[1]);
  uint32_t bad = 0;             // bit k: ring at q0 + k moves
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (k < cnt) {
      pm = MaxKeyOp()(pm, Pack<2>{{L_r[q0 + k], (double)(int32_t)(L_k[q0 + k] >> 32)}});
      const Pack<2> m = k + 1 < cnt ? Pack<2>{{sr[k + 1], (double)si[k + 1]}} : after;
      const Pack<2> sm = MinKeyOp()(m, after);
      const bool nb = key_lt(pm.v[0], (int32_t)pm.v[1], sm.v[0], (int32_t)sm.v[1]);
      if (!(bnd && nb)) bad |= 1u << k;
      bnd = nb;
    }
  }
  const double nbad = (double)__builtin_popcount(bad);
  Pack<1> tb;
  const Pack<1> ob = block_prefix<NT, 1>(Pack<1>{{nbad}}, Pack<1>{{0.0}}, SumOp<1>(), s_scanA, tb);
  if (!cl_gather<1, false>(cl, tb, s_x, s_ok)) return -1;
  Pack<1> om, mt;
  cl_prefix<1, 1>(s_x, 0, cl.g, cl.G, Pack<1>{{0.0}}, SumOp<1>(), om, mt);
  const int M = (int)mt.v[0];
  int P2 = 1;
  while (P2 < M) P2 <<= 1;
  if (16 * P2 > cap) return cl_bitonic<NT>(Ig, cl, xo, oko);     // every member takes the same branch
  // compaction in position order: key, slot, and the position it leaves
  WAKE_GLOBAL double* const br = gptr(I.bt_r);
  WAKE_GLOBAL int32_t* const bi = gptr(I.bt_i);
  WAKE_GLOBAL int32_t* const bs = gptr(I.bt_s);
  WAKE_GLOBAL int32_t* const fp = gptr(I.sm_i);
  int j = (int)om.v[0] + (int)ob.v[0];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (bad & (1u << k)) {
      br[j] = L_r[q0 + k];
      bi[j] = (int32_t)(L_k[q0 + k] >> 32);
      bs[j] = (int32_t)(uint32_t)L_k[q0 + k];
      fp[j] = goff + q0 + k;
      ++j;
    }
  }
  if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
  if (cl.g == 0) {
    double* const K_r = L_r;
    int32_t* const K_i = reinterpret_cast<int32_t*>(K_r + P2);
    int32_t* const K_s = K_i + P2;
    for (int i = tid; i < P2; i += NT) {
      K_r[i] = i < M ? br[i] : INFINITY;
      K_i[i] = i < M ? bi[i] : 0x7fffffff;
      K_s[i] = i < M ? bs[i] : -1;
    }
    __syncthreads();
    bitonic_keys<NT>(K_r, K_i, K_s, P2);
    for (int i = tid; i < M; i += NT) bs[i] = K_s[i];
  }
  if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
  // the j-th smallest moving ring to the j-th freed position (this member's)
  const int m0 = (int)om.v[0], m1 = m0 + (int)tb.v[0];
  for (int i = m0 + tid; i < m1; i += NT) perm[cl_slot<NT>(fp[i], C, P, iC, iP)] = bs[i];
  return cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok) ? cl.round : -1;
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

// Runs.  A run boundary sits before position p when every key before p is
// below every key from p on; the rings between consecutive boundaries are
// permuted among themselves.  Runs of one ring stay; runs of up to
// WAKE_SEGMAX rings are ranked by counting; the rings of longer runs are
// compacted, sorted together and placed into their freed positions in order
// (each long run keeps its position range, so the j-th smallest goes to the
// j-th freed position).

// Slot form of position p: (p % C) * NT + p / C, with p / C from a
// reciprocal estimate corrected to the exact quotient.
template <int NT>
__device__ __forceinline__ int pos_index(int p, int C, double iC) {
  int q = (int)((double)p * iC);
  if (q * C > p) --q;
  else if ((q + 1) * C <= p) ++q;
  return (p - q * C) * NT + q;
}

struct MaxIntOp {
  __device__ __forceinline__ Pack<1> operator()(const Pack<1>& a, const Pack<1>& b) const {
    return a.v[0] < b.v[0] ? b : a;
  }
};
struct MinIntOp {
  __device__ __forceinline__ Pack<1> operator()(const Pack<1>& a, const Pack<1>& b) const {
    return b.v[0] < a.v[0] ? b : a;
  }
};

// Order fix-up with the keys in global memory (instances with C > CMAX).
// The keys of the ring at position (t, k) are the current buffer's rho and
// id at slot k*NT + t.  Same runs, ranks and long-run sort as the LDS
// version; prefix maxima, boundaries and run starts go through global
// scratch (sm_r/sm_i, flag, cls); the permutation (slot form) is written to
// the global array perm.
template <int NT>
__device__ __noinline__ void fix_order_big(const WakeInst& I, int buf, double* s_scan,
                                           double* s_scan2, unsigned char* region) {
  const int tid = threadIdx.x;
  const int N = I.N, C = I.C;
  const double iC = 1.0 / (double)C;
  const int p0 = tid * C;
  const int cnt = max(0, min(C, N - p0));
  const PV SB = pview(I.st[buf], (uint32_t)(C * NT));
  const GA<double> PMR = uview(I.sm_r);
  const GA<int32_t> PMI = uview(I.sm_i), FL = uview(I.flag), CL = uview(I.cls), PERM = uview(I.perm);
  // chunk extremes; maximum key before each position of the chunk
  Pack<2> mx = {{-INFINITY, -2147483648.0}}, mn = {{INFINITY, 2147483647.0}};
  #pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const unsigned sl = k * NT + tid;
    PMR.st(sl, mx.v[0]);
    PMI.st(sl, (int32_t)mx.v[1]);
    const Pack<2> key = {{st_rho(SB, sl), (double)id_of<NT>(st_hs(SB, sl), C)}};
    mx = MaxKeyOp()(mx, key);
    mn = MinKeyOp()(mn, key);
  }
  Pack<2> before, tb, after, ta;
  block_prefix_suffix<NT, 2, 2, MaxKeyOp, MinKeyOp, false>(
      mx, Pack<2>{{-INFINITY, -2147483648.0}}, MaxKeyOp(), mn, Pack<2>{{INFINITY, 2147483647.0}},
      MinKeyOp(), s_scan, before, tb, after, ta);
  // run boundaries, first and last of the chunk
  Pack<2> sm = after;
  int lb = -1, fb = N;
  #pragma unroll 1
  for (int k = cnt - 1; k >= 0; --k) {
    const unsigned sl = k * NT + tid;
    const Pack<2> key = {{st_rho(SB, sl), (double)id_of<NT>(st_hs(SB, sl), C)}};
    sm = MinKeyOp()(sm, key);
    const Pack<2> pm = MaxKeyOp()(before, Pack<2>{{PMR[sl], (double)PMI[sl]}});
    const bool b = (p0 + k == 0) || key_lt(pm.v[0], (int32_t)pm.v[1], sm.v[0], (int32_t)sm.v[1]);
    FL.st(sl, b ? 1 : 0);
    if (b) {
      if (lb < 0) lb = p0 + k;
      fb = p0 + k;
    }
  }
  Pack<1> ain, at_, ein, et_;
  block_prefix_suffix<NT, 1, 1, MaxIntOp, MinIntOp, false>(
      Pack<1>{{(double)lb}}, Pack<1>{{-1.0}}, MaxIntOp(), Pack<1>{{(double)fb}}, Pack<1>{{(double)N}},
      MinIntOp(), s_scan2, ain, at_, ein, et_);
  // run start of each position
  int a = (int)ain.v[0];
  #pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const unsigned sl = k * NT + tid;
    if (FL[sl]) a = p0 + k;
    CL.st(sl, a);
  }
  // classify backward (run end = first boundary after the position); short
  // runs ranked here; long-run positions marked -1
  int e = (int)ein.v[0];
  double nlong = 0.0;
  #pragma unroll 1
  for (int k = cnt - 1; k >= 0; --k) {
    const int p = p0 + k;
    const unsigned sl = k * NT + tid;
    const int ra = CL[sl];
    if (e - ra == 1) {
      PERM.st(sl, (int32_t)sl);
    } else if (e - ra <= WAKE_SEGMAX) {
      const double r = st_rho(SB, sl);
      const int32_t id = id_of<NT>(st_hs(SB, sl), C);
      const int qi = pos_index<NT>(ra, C, iC);
      int qk = qi / NT, qt = qi % NT;
      int rank = 0;
      #pragma unroll 1
      for (int q = ra; q < e; q += 4) {
        unsigned x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {      // past the run end: compare with itself
          x[i] = q + i < e ? (unsigned)(qk * NT + qt) : sl;
          if (++qk == C) { qk = 0; ++qt; }
        }
        double xr[4];
        int32_t xh[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) { xr[i] = st_rho(SB, x[i]); xh[i] = st_hs(SB, x[i]); }
#pragma unroll
        for (int i = 0; i < 4; ++i) rank += key_lt(xr[i], id_of<NT>(xh[i], C), r, id) ? 1 : 0;
      }
      PERM.st((unsigned)pos_index<NT>(ra + rank, C, iC), (int32_t)sl);
    } else {
      CL.st(sl, -1);
      nlong += 1.0;
    }
    if (FL[sl]) e = p;
  }
  Pack<1> tot;
  const Pack<1> j0p = block_prefix<NT, 1>(Pack<1>{{nlong}}, Pack<1>{{0.0}}, SumOp<1>(), s_scan, tot);
  const int M = (int)tot.v[0];
  if (M > 0) {
    // rings of the long runs, compacted in position order; their freed
    // positions (slot form) in free_slot
    double* zr = reinterpret_cast<double*>(region);
    int32_t* zi = reinterpret_cast<int32_t*>(zr + WAKE_SORTCAP);
    int32_t* zs = zi + WAKE_SORTCAP;
    const bool in_lds = M <= WAKE_SORTCAP;
    int j = (int)j0p.v[0];
    #pragma unroll 1
    for (int k = 0; k < cnt; ++k) {
      const unsigned sl = k * NT + tid;
      if (CL[sl] != -1) continue;
      I.free_slot[j] = (int32_t)sl;
      const double r = st_rho(SB, sl);
      const int32_t id = id_of<NT>(st_hs(SB, sl), C);
      if (in_lds) { zr[j] = r; zi[j] = id; zs[j] = (int32_t)sl; }
      else { I.sk_r[0][j] = r; I.sk_i[0][j] = id; I.sk_s[0][j] = (int32_t)sl; }
      ++j;
    }
    __syncthreads();
    if (in_lds) {
      int P = 1;
      while (P < M) P <<= 1;
      for (int i = M + tid; i < P; i += NT) { zr[i] = INFINITY; zi[i] = 0x7fffffff - i; zs[i] = -1; }
      __syncthreads();
      bitonic_keys<NT>(zr, zi, zs, P);
      for (int q = tid; q < M; q += NT) PERM.st((unsigned)I.free_slot[q], zs[q]);
    } else {
      const int b = sort_keys_global<NT>(I, M, zr, zi, zs);
      for (int q = tid; q < M; q += NT) PERM.st((unsigned)I.free_slot[q], I.sk_s[b][q]);
    }
  }
  __syncthreads();
}


// Order fix-up in LDS (C <= CMAX).  The keys of the rings at every position
// are in LDS in slot form (position (t, k) of thread t at index k*NT + t):
// kr (radius), ki (id).  Builds perm[k*NT + t] = slot, in the current buffer,
// of the ring at sorted position (t, k).  Nothing in global memory moves.
// Run boundaries come from register prefix maxima, run extents from a scan
// of the first and last boundary of each chunk; short runs are ranked by
// counting, long runs sorted together.
// (rho, id) order of packed keys: k = id << 16 | slot, so that equal radii
// fall back to the ring id.
__device__ __forceinline__ bool pk_lt(double ra, uint32_t ka, double rb, uint32_t kb) {
  return (ra < rb) | ((ra == rb) & (ka < kb));     // no short-circuit: straight-line selects
}

// One wave puts the positions [b0, b0 + 256) (clipped at N) in (rho, id)
// order: four keys per lane, read through the current order perm, sorted by
// a bitonic network over registers and lane exchanges, written back as the
// new order of these positions.  A block already in order is left alone.
template <int NT>
__device__ __forceinline__ void sort_block_wave(int b0, int N, int C, double iC, const double* kr,
                                                const uint16_t* ki, uint16_t* perm) {
  const int lane = threadIdx.x & 63;
  double r[4];
  uint32_t k[4];
  int sl[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = b0 + 4 * lane + j;
    sl[j] = -1;
    r[j] = INFINITY;
    k[j] = 0xffffffffu;
    if (p < N) {
      sl[j] = pos_index<NT>(p, C, iC);
      const unsigned src = perm[sl[j]];
      r[j] = kr[src];
      k[j] = ((uint32_t)ki[src] << 16) | src;
    }
  }
  bool ok = !pk_lt(r[1], k[1], r[0], k[0]) && !pk_lt(r[2], k[2], r[1], k[1]) &&
            !pk_lt(r[3], k[3], r[2], k[2]);
  const double nr = __shfl_down(r[0], 1, 64);
  const uint32_t nk = __shfl_down(k[0], 1, 64);
  if (lane < 63) ok = ok && !pk_lt(nr, nk, r[3], k[3]);
  if (__all(ok)) return;
  // Odd-even transposition first: the rings of a run of length L reach
  // their places within L phases and never cross a run boundary, so blocks
  // with short runs (the common case) are done after a few phases.  Order
  // checked every four phases; a block still out of order after 32 phases
  // goes through the full bitonic network.
  #pragma unroll 1
  for (int it = 0; it < 8; ++it) {
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
      // even phase: (0,1) (2,3); odd phase: (1,2) and (3 | next lane's 0)
#pragma unroll
      for (int j = 0; j < 4; j += 2) {
        if (pk_lt(r[j + 1], k[j + 1], r[j], k[j])) {
          const double tr = r[j]; r[j] = r[j + 1]; r[j + 1] = tr;
          const uint32_t tk = k[j]; k[j] = k[j + 1]; k[j + 1] = tk;
        }
      }
      if (pk_lt(r[2], k[2], r[1], k[1])) {
        const double tr = r[1]; r[1] = r[2]; r[2] = tr;
        const uint32_t tk = k[1]; k[1] = k[2]; k[2] = tk;
      }
      const double nr = lane_next(r[0]), pr = lane_prev(r[3]);
      const uint32_t nq = lane_next(k[0]), pq = lane_prev(k[3]);
      const bool take_next = lane < 63 && pk_lt(nr, nq, r[3], k[3]);    // keep the smaller
      const bool take_prev = lane > 0 && pk_lt(r[0], k[0], pr, pq);     // keep the larger
      if (take_next) { r[3] = nr; k[3] = nq; }
      if (take_prev) { r[0] = pr; k[0] = pq; }
    }
    bool in_order = !pk_lt(r[1], k[1], r[0], k[0]) && !pk_lt(r[2], k[2], r[1], k[1]) &&
                    !pk_lt(r[3], k[3], r[2], k[2]);
    const double xr = lane_next(r[0]);
    const uint32_t xq = lane_next(k[0]);
    if (lane < 63) in_order = in_order && !pk_lt(xr, xq, r[3], k[3]);
    if (__all(in_order)) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (sl[j] >= 0) perm[sl[j]] = (uint16_t)(k[j] & 0xffffu);
      return;
    }
  }
#pragma unroll
  for (int kk = 2; kk <= 256; kk <<= 1) {
#pragma unroll
    for (int d = kk >> 1; d > 0; d >>= 1) {
      if (d >= 4) {                 // partner in lane ^ (d / 4), same register
        const int lm = d >> 2;
        const bool lower = (lane & lm) == 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double pr = lane_xor(r[j], lm);
          const uint32_t pq = lane_xor(k[j], lm);
          const bool up = ((4 * lane + j) & kk) == 0;
          if (pk_lt(pr, pq, r[j], k[j]) == (lower == up)) { r[j] = pr; k[j] = pq; }
        }
      } else {                      // partner in this lane
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (j & d) continue;
          const int jj = j | d;
          const bool up = ((4 * lane + j) & kk) == 0;
          if (pk_lt(r[jj], k[jj], r[j], k[j]) == up) {
            const double tr = r[j]; r[j] = r[jj]; r[jj] = tr;
            const uint32_t tk = k[j]; k[j] = k[jj]; k[jj] = tk;
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (sl[j] >= 0) perm[sl[j]] = (uint16_t)(k[j] & 0xffffu);
}

// Value of lane 63 - lane of the wave (rows mirrored by DPP, then rows and
// halves swapped).
__device__ __forceinline__ uint32_t lane_rev(uint32_t x) {
  const int lane = threadIdx.x & 63;
  x = __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, true);     // row_mirror: lane ^ 15 in the row
  const auto a = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  x = (lane & 16) ? a[0] : a[1];
  const auto b = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return (lane & 32) ? b[0] : b[1];
}
__device__ __forceinline__ double lane_rev(double x) {
  const uint64_t v = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = lane_rev((uint32_t)v), hi = lane_rev((uint32_t)(v >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One wave merges the positions [b0, b0 + 256) (clipped at N) whose two
// halves [b0, b0 + 128) and [b0 + 128, b0 + 256) are each in order: four
// keys per lane, the first stage compares position i with 255 - i (the
// second half taken in reverse makes the block bitonic), then the seven
// half-cleaning stages of a bitonic merge; written back as the new order of
// these positions.  A block already in order is left alone.
template <int NT>
__device__ __forceinline__ void merge_block_wave(int b0, int N, int C, double iC, const double* kr,
                                                 const uint16_t* ki, uint16_t* perm) {
  const int lane = threadIdx.x & 63;
  double r[4];
  uint32_t k[4];
  int sl[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = b0 + 4 * lane + j;
    sl[j] = -1;
    r[j] = INFINITY;
    k[j] = 0xffffffffu;
    if (p < N) {
      sl[j] = pos_index<NT>(p, C, iC);
      const unsigned src = perm[sl[j]];
      r[j] = kr[src];
      k[j] = ((uint32_t)ki[src] << 16) | src;
    }
  }
  {
    const double xr = lane_next(r[0]);
    const uint32_t xk = lane_next(k[0]);
    const bool ok = (lane == 63 || !pk_lt(xr, xk, r[3], k[3])) && !pk_lt(r[1], k[1], r[0], k[0]) &&
                    !pk_lt(r[2], k[2], r[1], k[1]) && !pk_lt(r[3], k[3], r[2], k[2]);
    if (__all(ok)) return;
  }
  // position 4 lane + j against 255 - (4 lane + j): lane 63 - lane, register 3 - j
  {
    double pr[4];
    uint32_t pq[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) { pr[j] = lane_rev(r[3 - j]); pq[j] = lane_rev(k[3 - j]); }
    const bool lower = lane < 32;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (pk_lt(pr[j], pq[j], r[j], k[j]) == lower) { r[j] = pr[j]; k[j] = pq[j]; }
  }
#pragma unroll
  for (int d = 64; d > 0; d >>= 1) {
    if (d >= 4) {                   // partner in lane ^ (d / 4), same register
      const int lm = d >> 2;
      const bool lower = (lane & lm) == 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double pr = lane_xor(r[j], lm);
        const uint32_t pq = lane_xor(k[j], lm);
        if (pk_lt(pr, pq, r[j], k[j]) == lower) { r[j] = pr; k[j] = pq; }
      }
    } else {                        // partner in this lane
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j & d) continue;
        const int jj = j | d;
        if (pk_lt(r[jj], k[jj], r[j], k[j])) {
          const double tr = r[j]; r[j] = r[jj]; r[jj] = tr;
          const uint32_t tk = k[j]; k[j] = k[jj]; k[jj] = tk;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (sl[j] >= 0) perm[sl[j]] = (uint16_t)(k[j] & 0xffffu);
}

// Whether any of bits lo..hi (inclusive, lo <= hi) of a bit array is set.
__device__ __forceinline__ bool bits_any(const uint64_t* m, int lo, int hi) {
  #pragma unroll 1
  for (int w = lo >> 6; w <= (hi >> 6); ++w) {
    uint64_t x = m[w];
    if (w == (hi >> 6) && (hi & 63) < 63) x &= (2ull << (hi & 63)) - 1ull;
    if (w == (lo >> 6)) x &= ~0ull << (lo & 63);
    if (x) return true;
  }
  return false;
}

// Key at position p through the order perm, as sort_block_wave compares them.
template <int NT>
__device__ __forceinline__ void key_at(int p, int C, double iC, const double* kr, const uint16_t* ki,
                                       const uint16_t* perm, double& r, uint32_t& k) {
  const unsigned src = perm[pos_index<NT>(p, C, iC)];
  r = kr[src];
  k = ((uint32_t)ki[src] << 16) | src;
}

// Order fix-up for nearly sorted keys in LDS: blocks of 256 positions sorted
// by single waves, first at offsets 0, 256, 512, ... and then at 128, 384,
// ... (the second phase's blocks are two sorted halves, merged).  If no ring
// is more than 128 positions from its place in the order,
// the two phases leave the whole sequence sorted (with the keys cut at any
// threshold, the mixed zone left by the first phase lies inside one block
// of the second).  Up to two such rounds; returns whether the order is
// complete (else the caller runs the general fix-up).
//
// dmask (optional): the push's disorder flags, bit t set if thread t's
// chunk had a pair of positions out of order (inside it, or its last
// position against the next chunk's first).  The first round then sorts
// only the blocks of the first phase whose chunks flagged disorder (the
// others are in order), only the blocks of the second phase over a junction
// of the first phase's blocks left out of order, and checks the order at
// the junctions of the second phase's blocks alone: every segment between
// them is sorted, so the sequence is in order when they are.
template <int NT>
__device__ __noinline__ bool fix_order_blocks(const WakeInst& I, const double* kr, const uint16_t* ki,
                                              uint16_t* perm, const uint64_t* dmask) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int N = I.N, C = I.C;
  const double iC = 1.0 / (double)C;
  const int p0 = tid * C;
  const int cnt = max(0, min(C, N - p0));
  for (int k = 0; k < cnt; ++k) perm[k * NT + tid] = (uint16_t)(k * NT + tid);
  __syncthreads();
  int round = 0;
  if (dmask) {
    round = 1;
    // the first phase's blocks with flagged chunks, one block per lane
    uint64_t bm;
    {
      const int b0 = lane << 8;
      bm = __ballot(b0 < N && bits_any(dmask, b0 / C, min((b0 + 255) / C, NT - 1)));
    }
    int seen = 0;
    #pragma unroll 1
    while (bm) {
      const int b = __builtin_ctzll(bm);
      bm &= bm - 1;
      if (seen++ % NW == wave) sort_block_wave<NT>(b * 256, N, C, iC, kr, ki, perm);
    }
    __syncthreads();
    // junctions q = 256 (j + 1) of the first phase's blocks, one per lane
    bool out = false;
    {
      const int q = 256 * (lane + 1);
      if (q < N) {
        double ra, rb;
        uint32_t ka, kb;
        key_at<NT>(q - 1, C, iC, kr, ki, perm, ra, ka);
        key_at<NT>(q, C, iC, kr, ki, perm, rb, kb);
        out = pk_lt(rb, kb, ra, ka);
      }
    }
    uint64_t jm = __ballot(out);
    seen = 0;
    #pragma unroll 1
    while (jm) {
      const int b = __builtin_ctzll(jm);
      jm &= jm - 1;
      if (seen++ % NW == wave) merge_block_wave<NT>(128 + b * 256, N, C, iC, kr, ki, perm);
    }
    __syncthreads();
    // junctions 128 + 256 j of the second phase's blocks
    out = false;
    {
      const int q = 128 + 256 * lane;
      if (q < N) {
        double ra, rb;
        uint32_t ka, kb;
        key_at<NT>(q - 1, C, iC, kr, ki, perm, ra, ka);
        key_at<NT>(q, C, iC, kr, ki, perm, rb, kb);
        out = pk_lt(rb, kb, ra, ka);
      }
    }
    if (!__ballot(out)) return true;     // the same keys in every wave: a uniform answer
    __syncthreads();                      // every wave has read the keys before a block moves
  }
  #pragma unroll 1
  for (; round < 2; ++round) {
    #pragma unroll 1
    for (int b = wave; b * 256 < N; b += NW) sort_block_wave<NT>(b * 256, N, C, iC, kr, ki, perm);
    __syncthreads();
    #pragma unroll 1
    for (int b = wave; 128 + b * 256 < N; b += NW) merge_block_wave<NT>(128 + b * 256, N, C, iC, kr, ki, perm);
    __syncthreads();
    // in order? (this chunk, and its last position against the next chunk's first)
    int bad = 0;
    if (cnt > 0) {
      unsigned src = perm[tid];
      double pr = kr[src];
      uint32_t pq = ((uint32_t)ki[src] << 16) | src;
      const int m = p0 + cnt < N ? cnt + 1 : cnt;
      #pragma unroll 1
      for (int k = 1; k < m; ++k) {
        const unsigned sl = k < cnt ? k * NT + tid : tid + 1;
        src = perm[sl];
        const double r = kr[src];
        const uint32_t q = ((uint32_t)ki[src] << 16) | src;
        if (pk_lt(r, q, pr, pq)) bad = 1;
        pr = r;
        pq = q;
      }
    }
    if (!__syncthreads_or(bad)) return true;
  }
  return false;
}

template <int NT, int CMAX>
__device__ __noinline__ void fix_order_lds(const WakeInst& I, double* s_scan, double* s_scan2,
                                           unsigned char* region, const double* kr,
                                           const uint16_t* ki, uint16_t* zf, uint16_t* perm) {
  const int tid = threadIdx.x;
  const int N = I.N, C = I.C;
  const double iC = 1.0 / (double)C;
  const int p0 = tid * C;
  const int cnt = max(0, min(C, N - p0));
  Pack<2> mx = {{-INFINITY, -2147483648.0}}, mn = {{INFINITY, 2147483647.0}};
  double pr[CMAX > 0 ? CMAX : 1];
  int32_t pi[CMAX > 0 ? CMAX : 1];      // maximum key before each position of the chunk
#pragma unroll
  for (int k = 0; k < CMAX; ++k) {
    if (k < cnt) {
      pr[k] = mx.v[0];
      pi[k] = (int32_t)mx.v[1];
      const Pack<2> key = {{kr[k * NT + tid], (double)ki[k * NT + tid]}};
      mx = MaxKeyOp()(mx, key);
      mn = MinKeyOp()(mn, key);
    }
  }
  Pack<2> before, tb, after, ta;
  block_prefix_suffix<NT, 2, 2, MaxKeyOp, MinKeyOp, false>(
      mx, Pack<2>{{-INFINITY, -2147483648.0}}, MaxKeyOp(), mn, Pack<2>{{INFINITY, 2147483647.0}},
      MinKeyOp(), s_scan, before, tb, after, ta);
  // run boundaries of the chunk (bit k: boundary before position p0 + k)
  Pack<2> sm = after;
  unsigned bits = 0;
#pragma unroll
  for (int k = CMAX - 1; k >= 0; --k) {
    if (k < cnt) {
      const Pack<2> key = {{kr[k * NT + tid], (double)ki[k * NT + tid]}};
      sm = MinKeyOp()(sm, key);
      const Pack<2> pm = MaxKeyOp()(before, Pack<2>{{pr[k], (double)pi[k]}});
      const bool b = (p0 + k == 0) || key_lt(pm.v[0], (int32_t)pm.v[1], sm.v[0], (int32_t)sm.v[1]);
      bits |= (unsigned)b << k;
    }
  }
  // last boundary at or before each chunk, first one after it
  const double lb = bits ? (double)(p0 + 31 - __builtin_clz(bits)) : -1.0;
  const double fb = bits ? (double)(p0 + __builtin_ctz(bits)) : (double)N;
  Pack<1> ain, at_, ein, et_;
  block_prefix_suffix<NT, 1, 1, MaxIntOp, MinIntOp, false>(
      Pack<1>{{lb}}, Pack<1>{{-1.0}}, MaxIntOp(), Pack<1>{{fb}}, Pack<1>{{(double)N}}, MinIntOp(),
      s_scan2, ain, at_, ein, et_);
  // classify; rings of short runs placed here
  unsigned lng = 0;
  double nlong = 0.0;
  #pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const int p = p0 + k;
    const unsigned own = (unsigned)(k * NT + tid);
    const unsigned below = bits & ((2u << k) - 1u);           // boundaries at or before p
    const unsigned above = bits & ~((2u << k) - 1u);          // boundaries after p
    const int a = below ? p0 + 31 - __builtin_clz(below) : (int)ain.v[0];
    const int e = above ? p0 + __builtin_ctz(above) : (int)ein.v[0];
    if (e - a == 1) { perm[own] = (uint16_t)own; continue; }
    if (e - a <= WAKE_SEGMAX) {
      const double r = kr[own];
      const int32_t id = ki[own];
      int qi = pos_index<NT>(a, C, iC);
      int qk = qi / NT, qt = qi % NT;                          // NT is a power of two
      int rank = 0;
      #pragma unroll 1
      for (int q = a; q < e; q += 4) {
        int x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {       // past the run end: compare with itself
          x[i] = q + i < e ? qk * NT + qt : (int)own;
          if (++qk == C) { qk = 0; ++qt; }
        }
        double xr[4];
        int32_t xi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) { xr[i] = kr[x[i]]; xi[i] = ki[x[i]]; }
#pragma unroll
        for (int i = 0; i < 4; ++i) rank += key_lt(xr[i], xi[i], r, id) ? 1 : 0;
      }
      perm[pos_index<NT>(a + rank, C, iC)] = (uint16_t)own;
    } else {
      lng |= 1u << k;
      nlong += 1.0;
    }
  }
  Pack<1> tot;
  const Pack<1> j0p = block_prefix<NT, 1>(Pack<1>{{nlong}}, Pack<1>{{0.0}}, SumOp<1>(), s_scan, tot);
  const int M = (int)tot.v[0];
  if (M > 0) {
    // rings of the long runs, compacted in position order; sorted keys in
    // zr/zi/zs (slots), their freed positions in zf (LDS index form)
    double* zr = reinterpret_cast<double*>(region);
    int32_t* zi = reinterpret_cast<int32_t*>(zr + WAKE_SORTCAP);
    int32_t* zs = zi + WAKE_SORTCAP;
    const bool in_lds = M <= WAKE_SORTCAP;
    int j = (int)j0p.v[0];
    #pragma unroll 1
    for (int k = 0; k < cnt; ++k) {
      if (!((lng >> k) & 1u)) continue;
      const int own = k * NT + tid;
      if (in_lds) { zf[j] = (uint16_t)own; zr[j] = kr[own]; zi[j] = ki[own]; zs[j] = own; }
      else { I.free_slot[j] = own; I.sk_r[0][j] = kr[own]; I.sk_i[0][j] = ki[own]; I.sk_s[0][j] = own; }
      ++j;
    }
    __syncthreads();
    if (in_lds) {
      int P = 1;
      while (P < M) P <<= 1;
      for (int i = M + tid; i < P; i += NT) { zr[i] = INFINITY; zi[i] = 0x7fffffff - i; zs[i] = -1; }
      __syncthreads();
      bitonic_keys<NT>(zr, zi, zs, P);
      for (int q = tid; q < M; q += NT) perm[zf[q]] = (uint16_t)zs[q];
    } else {
      const int b = sort_keys_global<NT>(I, M, zr, zi, zs);
      for (int q = tid; q < M; q += NT) perm[I.free_slot[q]] = (uint16_t)I.sk_s[b][q];
    }
  }
  __syncthreads();
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
// Cooperative instances: the transfer products and the source det-sums of
// all members from one exchange.  Member m publishes (G_m, V_m), its
// transfer product and v-sum in FwdMatSumOp form, and four vectors summed
// over its chunks: A = sum Gl^T mu, B = sum Gl^T l1, A' = sum K^T mu,
// B' = sum K^T l1 (Gl: the member's transfers before the chunk; K = adj(G)
// Hl with G the chunk's product and Hl the member's inverse transfers after
// it; l1: the part of the chunk's lambda that multiplies c; mu = lambda0 -
// (v of the chunk and of the member's later chunks) l1).  With gin the
// growing mode entering member m, hin the decaying mode leaving it and Vm
// the v-sum of the members after it, the member's sums of det[g_i, s_i] and
// det[s_i, h_i] are gin.A - Vm gin.B and -hin.A' + Vm hin.B'.  Every member
// forms from the gathered packs (NFT doubles each) its exclusive prefix pg
// and suffix sg of the transfers (inverse transfers from the adjugates of
// the published products, det = 1), their totals, and the det-sums of the
// members before it (e_in) and after it (d_in).  Lane l of each wave takes
// members MPL l .. MPL l + MPL-1 (G <= 64 MPL).
struct FwdMatSumOp;
struct BwdMatSumOp;
template <int NFT, class FOp, class BOp, int MPL>
__device__ __forceinline__ void cl_transfer_scan(const double* s_x, int g, int G, Pack<5>& pg, Pack<5>& gt,
                                                 Pack<5>& sg, Pack<5>& ht, double& e_in, double& d_in) {
  const int lane = threadIdx.x & 63;
  const Pack<5> I5 = {{1.0, 0.0, 0.0, 1.0, 0.0}};
  const FOp fop;
  const BOp bop;
  auto fwd_of = [&](int m) {
    const double* q = s_x + m * NFT;
    return Pack<5>{{q[0], q[1], q[2], q[3], q[4]}};
  };
  auto bwd_of = [&](int m) {
    const double* q = s_x + m * NFT;
    return Pack<5>{{q[3], -q[1], -q[2], q[0], q[4]}};
  };
  Pack<5> bf = I5, bb = I5;
#pragma unroll
  for (int j = 0; j < MPL; ++j)
    if (MPL * lane + j < G) bf = fop(bf, fwd_of(MPL * lane + j));
#pragma unroll
  for (int j = MPL - 1; j >= 0; --j)
    if (MPL * lane + j < G) bb = bop(bwd_of(MPL * lane + j), bb);
  const Pack<5> incF = wave_prefix_incl(bf, fop), incB = wave_suffix_incl(bb, bop);
  Pack<5> exF, exB;                     // the members before this lane's, after them
#pragma unroll
  for (int i = 0; i < 5; ++i) { exF.v[i] = lane_prev(incF.v[i]); exB.v[i] = lane_next(incB.v[i]); }
  if (lane == 0) exF = I5;
  if (lane == 63) exB = I5;
  gt = lane_pack(incF, 63);
  ht = lane_pack(incB, 0);
  double vm[MPL], dtm[MPL], etm[MPL];
  Pack<5> pg_l = I5, sg_l = I5;
  Pack<5> x = exB;
#pragma unroll
  for (int j = MPL - 1; j >= 0; --j) {  // descending: the suffix after each member
    const int m = MPL * lane + j;
    vm[j] = x.v[4];
    dtm[j] = 0.0;
    if (m < G) {
      const double* q = s_x + m * NFT;
      const double h0 = x.v[1], h1 = x.v[3];
      dtm[j] = -(h0 * q[9] + h1 * q[10]) + x.v[4] * (h0 * q[11] + h1 * q[12]);
      if (m == g) sg_l = x;
      x = bop(bwd_of(m), x);
    }
  }
  x = exF;
#pragma unroll
  for (int j = 0; j < MPL; ++j) {       // ascending: the prefix before each member
    const int m = MPL * lane + j;
    etm[j] = 0.0;
    if (m < G) {
      const double* q = s_x + m * NFT;
      const double g0 = x.v[0], g1 = x.v[2];
      etm[j] = (g0 * q[5] + g1 * q[6]) - vm[j] * (g0 * q[7] + g1 * q[8]);
      if (m == g) pg_l = x;
      x = fop(x, fwd_of(m));
    }
  }
  static_assert(MPL == 1 || MPL == 4, "one or four members per lane");
  double esum = etm[0], dsum = dtm[0];
  if constexpr (MPL == 4) {
    esum = (etm[0] + etm[1]) + (etm[2] + etm[3]);
    dsum = (dtm[0] + dtm[1]) + (dtm[2] + dtm[3]);
  }
  const Pack<1> eI = wave_prefix_incl(Pack<1>{{esum}}, SumOp<1>());
  const Pack<1> dI = wave_suffix_incl(Pack<1>{{dsum}}, SumOp<1>());
  double e_own = lane_prev(eI.v[0]), d_own = lane_next(dI.v[0]);
  if (lane == 0) e_own = 0.0;
  if (lane == 63) d_own = 0.0;
  const int lg = g / MPL, jg = g % MPL;
#pragma unroll
  for (int j = 0; j < MPL; ++j) {
    if (j < jg) e_own += etm[j];
    if (j > jg) d_own += dtm[j];
  }
  e_in = lane_pack(Pack<1>{{e_own}}, lg).v[0];
  d_in = lane_pack(Pack<1>{{d_own}}, lg).v[0];
  pg = lane_pack(pg_l, lg);
  sg = lane_pack(sg_l, lg);
}

struct SliceHeadOp {  // (w, w ln rho) as double-doubles, then two flag counts
  __device__ __forceinline__ Pack<6> operator()(const Pack<6>& a, const Pack<6>& b) const {
    const dd x = dd_add_fast({a.v[0], a.v[1]}, {b.v[0], b.v[1]});
    const dd y = dd_add_fast({a.v[2], a.v[3]}, {b.v[2], b.v[3]});
    return {{x.hi, x.lo, y.hi, y.lo, a.v[4] + b.v[4], a.v[5] + b.v[5]}};
  }
};

template <int NT>
struct MarchLds {
  static constexpr int NW = NT / 64;
  // rings per thread up to which the keys of every position live in LDS
  static constexpr int CMAX = 16;
  static constexpr int KCAP = NT * CMAX;
  static constexpr size_t region_bytes() {
    const size_t beam = 2 * WAKE_BCAP * sizeof(double);
    const size_t sort = WAKE_SORTCAP * (sizeof(double) + 2 * sizeof(int32_t));
    return beam > sort ? beam : sort;
  }
  // two scan areas, analytic constants, first keys of the chunks
  static constexpr size_t head_bytes() {
    return sizeof(double) * (2 * NW * 16 + 64 + NT) + sizeof(int32_t) * NT;
  }
  // per position (slot form): key radius, key id, slot of the ring
  // (permutation); freed positions of long runs
  static constexpr size_t key_bytes() {
    return (size_t)KCAP * (sizeof(double) + 2 * sizeof(uint16_t)) +
           (size_t)WAKE_SORTCAP * sizeof(uint16_t);
  }
  // ion interval nodes as floats (instances with keys in LDS: N <= KCAP)
  static constexpr size_t ion_bytes() { return ((size_t)(KCAP + 1) * sizeof(float) + 15) & ~(size_t)15; }
  static constexpr size_t bytes() { return head_bytes() + key_bytes() + region_bytes() + ion_bytes(); }
};
// one workgroup's LDS must fit the 160 KiB of a compute unit
static_assert(MarchLds<256>::bytes() <= 160 * 1024, "LDS layout too large");
static_assert(MarchLds<512>::bytes() <= 160 * 1024, "LDS layout too large");
// the block fix-up checks one junction of 256-position blocks per lane
static_assert(MarchLds<256>::KCAP <= 64 * 256 && MarchLds<512>::KCAP <= 64 * 256, "junctions per lane");
// a cooperative member gathers the packs of every member into its key area
static_assert(MarchLds<256>::key_bytes() >= WAKE_CL_GMAX * 16 * sizeof(double), "pack area");
// field-grid variant: the LDS left beside the layout holds the node records
// of grids up to grid_lds_nodes nodes (else they are read from device memory)
template <int NT>
constexpr int grid_lds_nodes() {
  return (int)((160 * 1024 - MarchLds<NT>::bytes() - 512) / (WAKE_GRID_TAB * sizeof(double)));
}
template <int NT>
constexpr size_t grid_lds_bytes() {
  return (size_t)grid_lds_nodes<NT>() * WAKE_GRID_TAB * sizeof(double);
}

// This slice's analytic source factors (beams: lam += c0 (1 - exp(-rho^2 c1));
// lasers: |a|^2 = c0 exp(-rho^2 c1)) and beam-table entries into LDS.
template <int NT>
__device__ __forceinline__ void stage_analytic(const WakeInst& I, int n, double* s_misc) {
  const int tid = threadIdx.x;
  const double xi = n * I.dxi;
  if (tid < I.n_an) {
    const WAKE_GLOBAL WakeAnalytic& A = gptr(I.an)[tid];
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
}
template <int NT>
__device__ __forceinline__ void stage_slice(const WakeInst& I, int n, double* s_misc, double* s_br,
                                            double* s_bc) {
  const int tid = threadIdx.x;
  stage_analytic<NT>(I, n, s_misc);
  if (I.nb) {
    const int bt0 = __builtin_amdgcn_readfirstlane(gptr(I.boff)[n]);
    const int bm = __builtin_amdgcn_readfirstlane(gptr(I.boff)[n + 1]) - bt0;
    const WAKE_GLOBAL double* br = gptr(I.br) + bt0;
    const WAKE_GLOBAL double* bc = gptr(I.bcum) + bt0;
    if (bm <= WAKE_BCAP)
      for (int i = tid; i < bm; i += NT) { s_br[i] = br[i]; s_bc[i] = bc[i]; }
  }
}

// The beam-table entries of a slice that one thread stages in LDS, fetched
// into registers ahead of the store (the fetch for slice n+1 is issued when
// pass E of slice n starts, the store follows the pass).
template <int NT>
struct BeamStage {
  static constexpr int BPT = (WAKE_BCAP + NT - 1) / NT;
  double r[BPT], c[BPT];
  int m;                 // entries of the slice; more than WAKE_BCAP: read from global memory
};
template <int NT>
__device__ __forceinline__ void beam_fetch(const WakeInst& I, int n, BeamStage<NT>& b) {
  b.m = 0;
  if (!I.nb) return;
  const int bt0 = __builtin_amdgcn_readfirstlane(gptr(I.boff)[n]);
  b.m = __builtin_amdgcn_readfirstlane(gptr(I.boff)[n + 1]) - bt0;
  if (b.m > WAKE_BCAP) return;
  const WAKE_GLOBAL double* br = gptr(I.br) + bt0;
  const WAKE_GLOBAL double* bc = gptr(I.bcum) + bt0;
#pragma unroll
  for (int q = 0; q < BeamStage<NT>::BPT; ++q) {
    const int i = threadIdx.x + q * NT;
    b.r[q] = 0.0;
    b.c[q] = 0.0;
    if (i < b.m) { b.r[q] = br[i]; b.c[q] = bc[i]; }
  }
}
template <int NT>
__device__ __forceinline__ void beam_store(const BeamStage<NT>& b, double* s_br, double* s_bc) {
  if (b.m > WAKE_BCAP) return;
#pragma unroll
  for (int q = 0; q < BeamStage<NT>::BPT; ++q) {
    const int i = threadIdx.x + q * NT;
    if (i < b.m) { s_br[i] = b.r[q]; s_bc[i] = b.c[q]; }
  }
}

// Per-thread sums of (w, w ln rho) over the rings at this thread's
// positions (ln rho of each ring taken from its slot).  Eight rings at a
// time: their slots and home slots (from the ring ids in LDS when the order
// is there, else from the home-slot words), then (w, w^) and ln rho, so each
// batch costs one round of independent loads (two without the LDS ids).
template <int NT>
__device__ __forceinline__ void chunk_sums(const WakeInst& I, int cur, int cnt, int goff, uint32_t ps,
                                           bool ident, bool lds_perm, const uint16_t* perm,
                                           const uint16_t* ki, dd& sw, dd& swl) {
  const int tid = threadIdx.x;
  const int C = I.C;
  const double iC = 1.0 / (double)C;
  const unsigned smax = ps - 1;
  const PV SC = pview(I.st[cur], ps), KC = pview(I.cst, ps);
  sw = {0.0, 0.0};
  swl = {0.0, 0.0};
  #pragma unroll 1
  for (int k0 = 0; k0 < cnt; k0 += 8) {
    unsigned s[8], hs[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const unsigned sl = (k0 + j) * NT + tid;
      s[j] = 0;
      hs[j] = 0;
      if (k0 + j < cnt) {
        s[j] = ident ? goff + sl : min(lds_perm ? (unsigned)perm[sl] : (unsigned)gptr(I.perm)[goff + sl], smax);
        hs[j] = lds_perm ? (unsigned)pos_index<NT>(ki[s[j]], C, iC) : (unsigned)st_hs(SC, s[j]);
      }
    }
    double w[8];
    D2 l[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      w[j] = k0 + j < cnt ? KC.ldh(RC_W, hs[j], 0) : 0.0;
      l[j] = k0 + j < cnt ? SC.ld(RS_LN, s[j]) : d2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (k0 + j < cnt) {
        sw = dd_add_d(sw, w[j]);
        swl = dd_add_fast(swl, dd_mul_d(dd{l[j].x, l[j].y}, w[j]));
      }
    }
  }
}

// CL: member `member` of a cooperative instance (I.G workgroups); its
// positions and slots start at goff = member * C * NT, and the slice scans
// and the order fix-up span all members.
// ---------------------------------------------------------------------------
// radial field grid (Fig. 2: fields on an external grid): the ring solve's
// sums evaluated at the uniform nodes r_g = (g + 1/2) dg, g < ng.  A node in
// (rho_{p-1}, rho_p] lies in interval p of the recursion: below it the
// rings before position p, at and above it the rest.
// ---------------------------------------------------------------------------
// Radius of node g: rad[g] for explicit nodes, else (g + 1/2) dg.
__device__ __forceinline__ double grid_node_r(int g, double dg, const WAKE_GLOBAL double* rad) {
  return rad ? rad[g] : ((double)g + 0.5) * dg;
}

// The largest node g with r_g <= x (-1 if none), decided on the node radii
// themselves so that neighbouring intervals split the nodes exactly
// (explicit radii: a binary search; uniform nodes: a guess corrected on the
// radii).
__device__ __forceinline__ int grid_last_below(double x, double dg, double idg, int ng,
                                               const WAKE_GLOBAL double* rad) {
  if (rad) {
    int a = 0, b = ng;                         // nodes at or below x: [0, a)
    while (a < b) {
      const int m = (a + b) >> 1;
      if (rad[m] <= x) a = m + 1; else b = m;
    }
    return a - 1;
  }
  if (!(x >= 0.5 * dg)) return -1;
  const double t = floor(x * idg - 0.5);      // a guess; the node radii decide
  int g = t >= (double)(ng - 1) ? ng - 1 : (int)t;
  if (g < -1) g = -1;
  while (g + 1 < ng && ((double)(g + 1) + 0.5) * dg <= x) ++g;
  while (g >= 0 && ((double)g + 0.5) * dg > x) --g;
  return g;
}

// Per-node hand-over scratch of a slice: 6 chunks of two doubles per node:
// [0] sum of w below, [1] sum of w ln rho below (pass B); [2] (E_z sum at
// and above, a), [3] (b, owner thread) (pass E); [4], [5] the owner's
// partial sums at and above the node of c = w / psibar and c rho (double-
// double; the chi deposit).
constexpr int GS = 6;

// The nodes a slice hands over in pass E: nr real nodes (uniform or explicit
// radii) and, when chi is deposited, one virtual node above the last, at
// r_{nr-1} + (r_{nr-1} - r_{nr-2}) (2 r_0 for a single node), where the last
// node's hat ends.
struct GridNodes {
  const WAKE_GLOBAL double* rad;
  double dg, idg, top;
  int nr, nh;
  __device__ __forceinline__ double r(int g) const { return g < nr ? grid_node_r(g, dg, rad) : top; }
  __device__ __forceinline__ int last_below(double x) const {
    int g = grid_last_below(x, dg, idg, nr, rad);
    if (g == nr - 1 && nh > nr && top <= x) g = nr;
    return g;
  }
};

// psi (eq. psi) and E_r - B_theta = -d_rho psi (eq. dpsi_dr, no ring at r)
// at node g (radius r) of an interval with the sums S, P of weight and
// w ln rho below it.  t0, t1, t2: the node's record (ln r and the immobile
// ions' psi - psi(0) and d_rho psi there, dd pairs, fixed for the solve);
// out: the slice's [4][ng] block.
__device__ __forceinline__ void grid_node_psi(WAKE_GLOBAL double* out, int ng, int g, double r, D2 t0,
                                              D2 t1, D2 t2, dd S, dd P, double psi_axis) {
  const dd pe = dd_add_fast(dd_mul(S, dd{t0.x, t0.y}), dd_neg(P));
  const dd de = dd_div_rcp(S, r, rcp_nr(r));
  out[g] = dd_round(dd_add_fast(pe, dd{t1.x, t1.y})) + psi_axis;
  out[ng + g] = -dd_round(dd_add_fast(de, dd{t2.x, t2.y}));
}

// E_z (eq. dpsi_dzeta: the rings at and above the interval) and
// B_theta = B^(b) + a r + b/r (eq. b_theta_plasma) at node g.
__device__ __forceinline__ void grid_node_b(WAKE_GLOBAL double* out, int ng, int g, double r, double ez,
                                            double a, double b, double bb) {
  const double ir = rcp_nr(r);
  out[2 * ng + g] = ez;
  out[3 * ng + g] = bb + (a * r + b * ir);
}

// chi = n/gamma (reading R20) at the nodes g0, g0 + NT, ... below g1 of a
// slice: a node's full sums D, E of c = w / psibar and c rho at and above it
// are its owner's partial sums plus the owner's later chunks (thr) and, on a
// cooperative instance, the later members (msuf, in LDS); the hats' sums are
// differences of neighbouring nodes' full sums (the virtual node past the
// last included), over the hats' volumes.  all0: the sum of c over every
// ring.  Not inlined: its temporaries stay out of the march's registers.
template <int NT, bool CL>
__device__ __noinline__ void chi_nodes(WAKE_GLOBAL double* gout, int ngB, const WAKE_GLOBAL D2* gscr,
                                       const WAKE_GLOBAL double* thr, const double* msuf, int n_thr,
                                       GridNodes GN, int g0, int g1, dd all0) {
  auto full = [&](int x, dd& d0, dd& d1) {
    const D2 o = gscr[GS * x + 3], p0s = gscr[GS * x + 4], p1s = gscr[GS * x + 5];
    // every node is handed over each slice; the bound keeps a node left
    // unhanded (radii that are not numbers) inside the arrays
    const int ow = (o.y >= 0.0 && o.y < (double)(n_thr)) ? (int)o.y : 0;
    const WAKE_GLOBAL double* t = thr + 4 * (size_t)ow;
    d0 = dd_add({p0s.x, p0s.y}, {t[0], t[1]});
    d1 = dd_add({p1s.x, p1s.y}, {t[2], t[3]});
    if (CL) {
      const double* ms = msuf + 4 * (ow / NT);
      d0 = dd_add(d0, {ms[0], ms[1]});
      d1 = dd_add(d1, {ms[2], ms[3]});
    }
  };
  #pragma unroll 1
  for (int g = g0; g < g1; g += NT) {
    const double rg = GN.r(g), rp = GN.r(g + 1);
    dd D0g, D1g, D0p, D1p;
    full(g, D0g, D1g);
    full(g + 1, D0p, D1p);
    // above the node: sum over [r_g, r_+) of c (r_+ - rho) / (r_+ - r_g)
    dd up = dd_sub(dd_mul_d(dd_sub(D0g, D0p), rp), dd_sub(D1g, D1p));
    up = dd_div_d(up, rp - rg);
    dd lowr;
    double V;
    if (g == 0) {                        // inside the first node: all of it
      lowr = dd_sub(all0, D0g);
      V = 0.5 * rg * rg;
    } else {
      const double rm = GN.r(g - 1);
      dd D0m, D1m;
      full(g - 1, D0m, D1m);
      lowr = dd_sub(dd_sub(D1m, D1g), dd_mul_d(dd_sub(D0m, D0g), rm));
      lowr = dd_div_d(lowr, rg - rm);
      V = (rg - rm) * (rm + 2.0 * rg) / 6.0;
    }
    V += (rp - rg) * (2.0 * rg + rp) / 6.0;
    gout[4 * ngB + g] = dd_round(dd_div_d(dd_add(lowr, up), V));
  }
}

// charge of the analytic beams inside r (staged constants of the slice)
__device__ __forceinline__ double analytic_lam(const double* s_misc, int n_an, double r) {
  double lam = 0.0;
  #pragma unroll 1
  for (int si = 0; si < n_an; ++si)
    if (s_misc[3 * si] == 2.0) lam += s_misc[3 * si + 1] * (-expm1(-r * r * s_misc[3 * si + 2]));
  return lam;
}

template <int NT, bool CL, int GM>
__device__ __forceinline__ void march(const WakeInst& I, int member, const int32_t* queue, unsigned char* smem) {
  // GM: 0 no field grid, 1 field grid, 2 field grid with the chi deposit
  constexpr bool GRID = GM > 0;
  constexpr bool CHI = GM > 1;
  constexpr int NW = NT / 64;
  constexpr int CMAX = MarchLds<NT>::CMAX;
  constexpr int KCAP = MarchLds<NT>::KCAP;
  const int tid = threadIdx.x;
  const int N = I.N;
  const int C = I.C;
  const int P = C * NT;                          // positions per member
  const int goff = CL ? member * P : 0;          // this member's first position / slot
  const int Ng = CL ? min(P, N - goff) : N;      // positions of this member
  const int p0 = tid * C;
  const int cnt = max(0, min(C, Ng - p0));   // rings owned by this thread
  const double iC = 1.0 / (double)C, iP = 1.0 / (double)P;
  // ring id of home slot hs
#define WAKE_ID(hs) (CL ? cl_id<NT>((hs), C, P, iP) : id_of<NT>((hs), C))

  double* s_scanA = reinterpret_cast<double*>(smem);      // NW * 16
  double* s_scanB = s_scanA + NW * 16;                     // NW * 16
  double* s_misc = s_scanB + NW * 16;                      // 64
  double* s_fr = s_misc + 64;                              // NT: first pushed key of each chunk
  int32_t* s_fi = reinterpret_cast<int32_t*>(s_fr + NT);  // NT
  double* s_kr = reinterpret_cast<double*>(smem + MarchLds<NT>::head_bytes());
  uint16_t* s_ki = reinterpret_cast<uint16_t*>(s_kr + KCAP);
  uint16_t* s_perm = s_ki + KCAP;
  uint16_t* s_zf = s_perm + KCAP;
  unsigned char* region = smem + MarchLds<NT>::head_bytes() + MarchLds<NT>::key_bytes();
  double* s_br = reinterpret_cast<double*>(region);        // beam radii
  double* s_bc = s_br + WAKE_BCAP;                         // beam cumulative charge
  float* s_ion = reinterpret_cast<float*>(region + MarchLds<NT>::region_bytes());   // ion nodes
  // keys and ring order in LDS (else the order is fixed in global memory)
  const bool lds_keys = !CL && C <= CMAX;
  const uint32_t ps = (uint32_t)(CL ? I.G * P : P);   // slots of the instance
  const unsigned smax = ps - 1;                        // last slot
  const GA<int32_t> gperm = uview(I.perm);
  // slot, in the current buffer, of the ring at this member's position of
  // slot-form index sl
#define WAKE_SLOT(sl) (ident ? (unsigned)(goff + (sl)) \
                             : min(lds_keys ? (unsigned)s_perm[sl] : (unsigned)gperm[goff + (sl)], smax))
  Cluster cl;
  cl.g = member;
  cl.G = CL ? I.G : 1;
  cl.round = 0;
  cl.xd = I.xd;
  cl.xc = I.xc;
  cl.queue = queue;
  if (CL) cl_start(cl);
  double* const s_x = s_kr;                                   // gathered packs (cooperative)
  int* const s_ok = reinterpret_cast<int*>(s_misc + 62);
  uint64_t* const s_dmask = reinterpret_cast<uint64_t*>(s_misc + 32);   // NW words: the push's disorder flags
  // the same two as byte offsets into the LDS, for the cooperative fix-ups
  const int xo = (int)MarchLds<NT>::head_bytes();
  const int oko = (int)(reinterpret_cast<unsigned char*>(s_ok) - smem);
  // cooperative member-local fix-up rounds in LDS: the key area after the
  // gathered packs (WAKE_CL_GMAX members x 16 doubles)
  const int lo = xo + WAKE_CL_GMAX * 16 * (int)sizeof(double);
  const int lo_cap = (int)MarchLds<NT>::key_bytes() - WAKE_CL_GMAX * 16 * (int)sizeof(double);

  if (__builtin_amdgcn_readfirstlane(I.ctl[CTL_BREAK]) >= 0) return;
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
  const int64_t budget = I.budget;
  int cur = __builtin_amdgcn_readfirstlane(I.ctl[CTL_CUR]);
  double rho_mprev = -1.0;   // field grid, cooperative: radius at the previous member's last position
  double rho_mlast = -1.0;   // field grid, cooperative: radius at this member's last position
  __syncthreads();
  // the ring at this thread's k-th position (slot s of the current buffer)
  // is not the one the push wrote there: the chunk's order changed
#define WAKE_MOVED(s, k) ((int)(s) != goff + (k) * NT + tid)
  // injected states may be unsorted
  bool ident = true;
  bool push_keys = false;   // cooperative: the push's first and last keys of the member are in LDS
  bool moved = false;       // a chunk holds rings of another chunk after the fix-up
  if (CL) {
    #pragma unroll 1
    for (int k = 0; k < cnt; ++k) {
      const unsigned sl = goff + k * NT + tid;
      const PV SB = pview(I.st[cur], ps);
      gptr(I.gk_r)[sl] = st_rho(SB, sl);
      gptr(I.gk_i)[sl] = WAKE_ID(st_hs(SB, sl));
    }
    int r = cl_fix<NT>(as_global(I), cl, xo, oko);
    if (r >= 0 && (r & 1)) {      // the block rounds left disorder
      cl.round = r >> 1;
      r = C <= 16 && 16 * P <= lo_cap ? cl_segments<NT>(as_global(I), cl, xo, oko, lo, lo_cap)
                                      : cl_bitonic<NT>(as_global(I), cl, xo, oko);
      if (r >= 0) r <<= 1;
    }
    if (r < 0) {
      if (tid == 0 && member == 0) I.ctl[CTL_FAULT] = 1;
      return;
    }
    cl.round = r >> 1;
    ident = false;
    for (int k = 0; k < cnt; ++k) moved |= WAKE_MOVED(gperm[goff + k * NT + tid], k);
  } else if (lds_keys) {
    #pragma unroll 1
    for (int k = 0; k < cnt; ++k) {
      const unsigned sl = k * NT + tid;
      const PV SB = pview(I.st[cur], ps);
      s_kr[sl] = st_rho(SB, sl);
      s_ki[sl] = (uint16_t)id_of<NT>(st_hs(SB, sl), C);
    }
    __syncthreads();
    fix_order_lds<NT, CMAX>(I, s_scanB, s_scanA, region, s_kr, s_ki, s_zf, s_perm);
    ident = false;
    for (int k = 0; k < cnt; ++k) moved |= WAKE_MOVED(s_perm[k * NT + tid], k);
  } else {
    fix_order_big<NT>(I, cur, s_scanB, s_scanA, region);
    ident = false;
    for (int k = 0; k < cnt; ++k) moved |= WAKE_MOVED(gperm[k * NT + tid], k);
  }
  const dd tot0 = {uni(I.tot0[0]), uni(I.tot0[1])};
  const double dxi = I.dxi;
  IonView IV;
  IV.R = uview(I.ion);
  IV.N = N;
  IV.Rp = I.Rp;
  IV.T0 = tot0;
  IV.Q = {uni(I.tot0[2]), uni(I.tot0[3])};
  const PV KC = pview(I.cst, ps), SCR = pview(I.sc, ps);
  const GA<double> A2 = uview(I.a2), DA2 = uview(I.da2);
  const int n_an = I.n_an;
  const bool has_laser = I.has_laser != 0;
  // ion interval nodes in LDS (float) for the interval search of pass B;
  // read there after the slice-head scan's barriers
  const bool lds_ion = N <= KCAP;      // the interval nodes fit the LDS table
  int hint0 = goff + p0 + 1;           // interval of the thread's first ring (at rest: its node's)
  // field-grid node records in the LDS beyond the layout (read after the
  // slice-head scan's barriers)
  const bool grid_lds = GRID && I.grid_n > 0 && !I.grid_off && I.grid_n <= grid_lds_nodes<NT>();
  D2* const s_gt = reinterpret_cast<D2*>(smem + MarchLds<NT>::bytes());
  if (grid_lds) {
    const WAKE_GLOBAL D2* const t = reinterpret_cast<const WAKE_GLOBAL D2*>(gptr(I.grid_tab));
    for (int i = tid; i < 3 * I.grid_n; i += NT) s_gt[i] = t[i];
  }
  if (lds_ion)
    for (int j = tid; j <= N; j += NT) s_ion[j] = (float)IV.R[j * WAKE_ION_REC + IR_LO];

  // The per-thread sums of (w, w ln rho), ln rho as the state carries it.
  // The sums in the order the march itself would have left them in (so that
  // a solve split over several launches is bitwise the one-launch solve):
  // chunks whose order the fix-up changed sum forward, the others backward
  // as the push does.
  dd sw = {0.0, 0.0}, swl = {0.0, 0.0};
  if (moved) {
    chunk_sums<NT>(I, cur, cnt, goff, ps, ident, lds_keys, s_perm, s_ki, sw, swl);
  } else {
    #pragma unroll 1
    for (int k = cnt - 1; k >= 0; --k) {
      const unsigned sl = k * NT + tid;
      const unsigned s = WAKE_SLOT(sl);
      const PV SB = pview(I.st[cur], ps);
      const double w = KC.ldh(RC_W, (unsigned)st_hs(SB, s), 0);
      const D2 l = SB.ld(RS_LN, s);
      sw = dd_add_d(sw, w);
      swl = dd_add_fast(swl, dd_mul_d(dd{l.x, l.y}, w));
    }
  }
  // sums of the thread's own rings in the push's order (what a fix-up that
  // leaves the chunk with its own rings falls back to)
  dd sw_push = sw, swl_push = swl;
  int n = I.first;
  int end = I.first + I.count;
  if (n < end) stage_slice<NT>(I, n, s_misc, s_br, s_bc);
  double bad = 0.0, dis = 0.0;
  int fix_rounds = 0;          // consecutive fix-up rounds at this slice head
  int cl_rounds = 0;           // of which over all members (cooperative)
  int unpushed = cur;          // buffer with the unpushed state of slice n-1

  for (;;) {
    // ---- Gauss/log prefix sum_{k<i} (w_k, w_k ln rho_k); flags of slice n-1 ----
    Pack<6> t6;
    double my_dis = 0.0, bnd = 0.0;   // cooperative: this member's disorder, member boundaries out of order
    Pack<6> pre = block_prefix<NT, 6, SliceHeadOp, false>(
        Pack<6>{{sw.hi, sw.lo, swl.hi, swl.lo, bad, dis}}, Pack<6>{{0, 0, 0, 0, 0, 0}},
        SliceHeadOp(), s_scanA, t6);
    if (CL) {
      // members' totals, their first and last keys in the current order (run
      // boundaries between members) and the time budget
      Pack<11> mine;
#pragma unroll
      for (int i = 0; i < 6; ++i) mine.v[i] = t6.v[i];
      if (tid == 0) {
        if (push_keys) {       // the push's keys of the first and the last position, kept in LDS
          mine.v[6] = s_fr[0];
          mine.v[7] = (double)s_fi[0];
          mine.v[8] = s_misc[48];
          mine.v[9] = s_misc[49];
        } else {
          const int ql = Ng - 1;
          const unsigned sf = WAKE_SLOT(0u), sL = WAKE_SLOT((unsigned)((ql % C) * NT + ql / C));
          mine.v[6] = gptr(I.gk_r)[sf];
          mine.v[7] = (double)gptr(I.gk_i)[sf];
          mine.v[8] = gptr(I.gk_r)[sL];
          mine.v[9] = (double)gptr(I.gk_i)[sL];
        }
        mine.v[10] = (budget > 0 && n > I.first &&
                      (int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) >= budget) ? 1.0 : 0.0;
      }
      if (!cl_gather<11, false>(cl, mine, s_x, s_ok)) {
        if (tid == 0 && member == 0) I.ctl[CTL_FAULT] = 1;
        return;
      }
      Pack<6> pg;
      my_dis = t6.v[5];
      if (cl.G <= 64) cl_prefix<6, 11, SliceHeadOp, 1>(s_x, 0, member, cl.G, Pack<6>{{0, 0, 0, 0, 0, 0}}, SliceHeadOp(), pg, t6);
      else cl_prefix<6, 11>(s_x, 0, member, cl.G, Pack<6>{{0, 0, 0, 0, 0, 0}}, SliceHeadOp(), pg, t6);
      pre = SliceHeadOp()(pg, pre);
      if constexpr (GRID) {
        rho_mprev = member > 0 ? s_x[(member - 1) * 11 + 8] : -1.0;
        rho_mlast = s_x[member * 11 + 8];
      }
      // a member out of time; boundaries between members out of order (thread
      // m looks at member m and the one after it)
      bool m_stop = false, m_bnd = false;
      if (tid < cl.G) {
        const int m = tid;
        m_stop = s_x[m * 11 + 10] != 0.0;
        m_bnd = m + 1 < cl.G && key_lt(s_x[(m + 1) * 11 + 6], (int32_t)s_x[(m + 1) * 11 + 7], s_x[m * 11 + 8],
                                       (int32_t)s_x[m * 11 + 9]);
      }
      bnd = __syncthreads_or(m_bnd) ? 1.0 : 0.0;
      const bool stop = __syncthreads_or(m_stop) != 0;
      t6.v[5] += bnd;
      if (stop && t6.v[4] == 0.0) end = n;
    }
    if (t6.v[4] != 0.0) {     // slice n-1 broke down: stop there
      if (tid == 0 && member == 0) { I.ctl[CTL_BREAK] = n - 1; I.ctl[CTL_CUR] = unpushed; I.ctl[CTL_NEXT] = n - 1; }
      return;
    }
    if (n == end) break;
    if (t6.v[5] != 0.0) {     // pushed radii out of order: new order, then redo the prefix
      bool restage = true;    // the general fix-ups use the beam-table area of LDS
      double still = 0.0;      // cooperative: this member still out of order after the round
      if (tid == 0 && member == 0) atomicAdd(I.cnt + CNT_FIXUPS, 1ull);
      if (CL) {
        // disorder inside members only: up to two member-local block rounds
        // (members in order skip them); across member boundaries, or left
        // over, block rounds over all members; after two of these that leave
        // disorder the sort by segments, then the bitonic network
        restage = false;
        if (bnd == 0.0 && fix_rounds < 2 && cl_rounds == 0) {
          if (my_dis == 0.0) {
            ++fix_rounds;
            dis = 0.0;
            continue;
          }
          if (tid == 0) atomicAdd(I.cnt + CNT_CL_LOCAL, 1ull);
          still = (16 * P <= lo_cap ? cl_fix_local_lds<NT>(as_global(I), member, ident, lo)
                                    : cl_fix_local<NT>(as_global(I), member, ident)) ? 1.0 : 0.0;
        } else {
          int r = -1;
          if (tid == 0 && member == 0)
            atomicAdd(I.cnt + (cl_rounds < 2 ? CNT_CL_ROUNDS
                               : cl_rounds == 2 && C <= 16 && 16 * P <= lo_cap ? CNT_CL_SEGMENTS
                                                                                : CNT_CL_BITONIC), 1ull);
          if (cl_rounds < 2) {
            r = cl_fix_round<NT>(as_global(I), cl, xo, oko, ident, 16 * P <= lo_cap ? lo : -1);
            if (r >= 0) {
              still = (r & 1) ? 1.0 : 0.0;
              r >>= 1;
            }
          } else if (cl_rounds == 2 && C <= 16 && 16 * P <= lo_cap) {
            r = cl_segments<NT>(as_global(I), cl, xo, oko, lo, lo_cap);
          } else {             // exact in any case: the round after it finds the order complete
            r = cl_bitonic<NT>(as_global(I), cl, xo, oko);
          }
          if (r < 0) {
            if (tid == 0 && member == 0) I.ctl[CTL_FAULT] = 1;
            return;
          }
          cl.round = r;
          ++cl_rounds;
        }
        ++fix_rounds;
      } else if (lds_keys) {
        restage = !fix_order_blocks<NT>(I, s_kr, s_ki, s_perm, s_dmask);
        if (restage) {
          if (tid == 0) atomicAdd(I.cnt + CNT_GENERAL, 1ull);
          fix_order_lds<NT, CMAX>(I, s_scanB, s_scanA, region, s_kr, s_ki, s_zf, s_perm);
        }
      } else {
        if (tid == 0) atomicAdd(I.cnt + CNT_GENERAL, 1ull);
        fix_order_big<NT>(I, cur, s_scanB, s_scanA, region);
      }
      ident = false;
      push_keys = false;
      // chunks whose order changed sum again
      bool changed = false;
      for (int k = 0; k < cnt; ++k)
        changed |= WAKE_MOVED(lds_keys ? (int32_t)s_perm[k * NT + tid] : gperm[goff + k * NT + tid], k);
      // (a chunk back to its push order after a later round takes the push's sums again)
      if (changed) {
        chunk_sums<NT>(I, cur, cnt, goff, ps, ident, lds_keys, s_perm, s_ki, sw, swl);
      } else {
        sw = sw_push;
        swl = swl_push;
      }
      if (restage) stage_slice<NT>(I, n, s_misc, s_br, s_bc);
      dis = still;
      continue;
    }
    fix_rounds = 0;
    cl_rounds = 0;
    const double psi_axis = dd_round(dd_sub({t6.v[2], t6.v[3]}, tot0));
    const bool do_push = n < I.n_xi - 1;
    const bool rec_snap = I.stride > 0 && (n % I.stride) == 0;
    const bool rec_last = n == end - 1;
    const int nb = 1 - cur;
    const PV Sc = pview(I.st[cur], ps), Sn = pview(I.st[nb], ps);
    int bt0 = 0, bm = 0;
    if (I.nb) {
      bt0 = __builtin_amdgcn_readfirstlane(gptr(I.boff)[n]);
      bm = __builtin_amdgcn_readfirstlane(gptr(I.boff)[n + 1]) - bt0;
    }
    const bool staged = bm <= WAKE_BCAP;
    // the slice's table: staged in LDS, or (too long) in device memory; the
    // two are searched by separate code so each takes its own instructions
    const WAKE_GLOBAL double* const gR = gptr(I.br) + bt0;
    const WAKE_GLOBAL double* const gQ = gptr(I.bcum) + bt0;

    // ---- pass B: psi family, sources, local quantities, chunk sums ----
    dd S = {pre.v[0], pre.v[1]}, PT = {pre.v[2], pre.v[3]};
    Pack<4> G = mat_ident();
    double Vw = 0.0;
    double l0a = 0.0, l0b = 0.0, l1a = 0.0, l1b = 0.0;
    bad = 0.0;
    int blo = 0;
    // loads run ahead: the state of ring k+2 and the constants and ion
    // record of ring k+1 are requested while ring k is computed
    D2 x_ru = d2(1.0, 0.0), x_ln = d2(0.0, 0.0), z_ru = d2(1.0, 0.0), z_ln = d2(0.0, 0.0);
    int32_t x_hs = 0, z_hs = 0;                      // home slots
    int x_hn = 0, z_hn = 0;                          // interval hints (no LDS node table)
    D2 x_wc = d2(0.0, 0.0);                          // (w, w^) of ring k+1
    double x_q[WAKE_ION_REC];
    if (cnt > 0) {
      const unsigned s = WAKE_SLOT(tid);
      x_ru = Sc.ld(RS_RU, s); x_ln = Sc.ld(RS_LN, s); x_hs = st_hs(Sc, s);
      if (!lds_ion) x_hn = st_hint(Sc, s);
    }
    if (cnt > 1) {
      const unsigned s = WAKE_SLOT(NT + tid);
      z_ru = Sc.ld(RS_RU, s); z_ln = Sc.ld(RS_LN, s); z_hs = st_hs(Sc, s);
      if (!lds_ion) z_hn = st_hint(Sc, s);
    }
    // ion interval of the next ring: searched in LDS from the interval of
    // the ring before it (sorted order; the first ring from the interval of
    // the thread's first ring at the previous slice), its records requested
    // one ring ahead; without the LDS table the ring's own interval at the
    // previous slice
    int jn = 0;
    if (cnt > 0) {
      x_wc = KC.ld(RC_W, (unsigned)x_hs);
      jn = lds_ion ? ion_find(s_ion, N, x_ru.x, hint0) : x_hn;
      ion_load(IV, jn, x_q);
    }
    // field grid: the interval owning each node hands the node its sums
    // (pass B: weight and w ln rho below it; pass E: the E_z sum and the
    // B^(p) coefficients); every thread then evaluates nodes.  gb_lo: the
    // last node at or below the previous position, gb_next its successor's
    // radius (a ring at or above it owns nodes)
    // this slice's nodes: entries [gofs, gofs + ngB) of a per-slice node
    // set, else the context's nodes (fields of slice n at 4 n grid_n)
    const size_t gofs = !GRID ? 0 : I.grid_off ? (size_t)gptr(I.grid_off)[n] : (size_t)n * (size_t)I.grid_n;
    const int ngB = !GRID ? 0 : I.grid_off ? gptr(I.grid_off)[n + 1] - (int)gofs : I.grid_n;
    const WAKE_GLOBAL double* const grB =
        (GRID && I.grid_rad) ? gptr(I.grid_rad) + (I.grid_off ? gofs : 0) : nullptr;
    const double dgB = I.grid_dr, idgB = 1.0 / dgB;
    WAKE_GLOBAL D2* const gscr = reinterpret_cast<WAKE_GLOBAL D2*>(gptr(I.grid_scr));
    int gb_lo = -1;
    double gb_next = INFINITY;
    if (GRID && ngB > 0 && cnt > 0) {
      double rb = -1.0;
      if (tid > 0) rb = Sc.ld(RS_RU, WAKE_SLOT((unsigned)((C - 1) * NT + tid - 1))).x;
      else if (CL) rb = rho_mprev;
      gb_lo = grid_last_below(rb, dgB, idgB, ngB, grB);
      gb_next = gb_lo + 1 < ngB ? grid_node_r(gb_lo + 1, dgB, grB) : INFINITY;
    }
    #pragma unroll 1
    for (int k = 0; k < cnt; ++k) {
      const unsigned sl = k * NT + tid;
      const double rho = x_ru.x, u = x_ru.y;
      const int32_t hs = x_hs;
      int h = jn;
      const dd lnr = {x_ln.x, x_ln.y};
      const double w = x_wc.x, wh = x_wc.y;
      double q[WAKE_ION_REC];
#pragma unroll
      for (int i = 0; i < WAKE_ION_REC; ++i) q[i] = x_q[i];
      x_ru = z_ru; x_ln = z_ln; x_hs = z_hs; x_hn = z_hn;
      if (k + 2 < cnt) {
        const unsigned s = WAKE_SLOT(sl + 2 * NT);
        z_ru = Sc.ld(RS_RU, s); z_ln = Sc.ld(RS_LN, s); z_hs = st_hs(Sc, s);
        if (!lds_ion) z_hn = st_hint(Sc, s);
      }
      if (k + 1 < cnt) {
        x_wc = KC.ld(RC_W, (unsigned)x_hs);
        jn = lds_ion ? ion_find(s_ion, N, x_ru.x, h) : x_hn;
        ion_load(IV, jn, x_q);
      }
      const double irho = rcp_nr(rho);
      const dd PTi = dd_add_fast(PT, dd_mul_d(lnr, w));
      const dd pe = dd_add_fast(dd_mul(dd_add_d(S, w), lnr), dd_neg(PTi));    // psi_e - sum w ln rho
      const dd de = dd_div_rcp(dd_add_d(S, wh), rho, irho);         // d_rho psi_e (self w^)
      dd ips, idp;
      ion_fields(IV, rho, lnr, h, q, ips, idp);
      const double psi = dd_round(dd_add_fast(pe, ips)) + psi_axis;
      const double dpsi = dd_round(dd_add_fast(de, idp));
      if (GRID && rho >= gb_next) {
        // nodes of interval p = (rho_{p-1}, rho_p]: the sums below position p
        const int ghi = grid_last_below(rho, dgB, idgB, ngB, grB);
        #pragma unroll 1
        for (int g = gb_lo + 1; g <= ghi; ++g) {
          gscr[GS * g] = d2(S.hi, S.lo);
          gscr[GS * g + 1] = d2(PT.hi, PT.lo);
        }
        gb_lo = ghi;
        gb_next = gb_lo + 1 < ngB ? grid_node_r(gb_lo + 1, dgB, grB) : INFINITY;
      }
      S = dd_add_d(S, w);
      PT = PTi;
      // beam charge inside rho (strictly below), analytic beams, lasers
      double lam = 0.0;
      if (bm > 0) {
        if (staged) {
          blo = count_below(s_br, blo, bm, rho, k > 0);
          if (blo > 0) lam = s_bc[blo - 1];
        } else {
          blo = count_below(gR, blo, bm, rho, k > 0);
          if (blo > 0) lam = gQ[blo - 1];
        }
      }
      double aa = 0.0, dda = 0.0;
      #pragma unroll 1
      for (int si = 0; si < n_an; ++si) {
        const double kind = s_misc[3 * si], c0 = s_misc[3 * si + 1], c1 = s_misc[3 * si + 2];
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
      G = mat_mul(rec_matrix(L.A, rho, irho), G);
      Vw += L.v;
      // s_i with d_zeta psi = (Vw - own) + c: s = s0 + c s1
      const double dz0 = Vw - (w - wh) * u * irho * L.ipb;
      double B0, Cc;
      ring_BC(irho, u, w, L, dpsi, dz0, bb, dda, B0, Cc);
      const double beta = w * irho * u * L.ipb * L.ipb;     // -dB/d(d_zeta psi)
      double s0a, s0b;
      rec_offset(L.A, B0, Cc, rho, s0a, s0b);
      const double s1a = -0.5 * beta, s1b = 0.5 * rho * rho * beta;
      l0a += G.v[0] * s0b - G.v[2] * s0a;
      l0b += G.v[1] * s0b - G.v[3] * s0a;
      l1a += G.v[0] * s1b - G.v[2] * s1a;
      l1b += G.v[1] * s1b - G.v[3] * s1a;
      SCR.st(SC_PSI, goff + sl, d2(psi, dpsi));
      if (has_laser) { A2.st(goff + sl, aa); DA2.st(goff + sl, dda); }
      // the ring's interval: its hint at the next slice (the thread's first
      // ring: the next slice's search starts there)
      if (!lds_ion) Sn.sti(RS_W, Sn.ps + goff + sl, h);
      if (k == 0) hint0 = h;
    }
    if (GRID && ngB > 0 && cnt > 0 && p0 + cnt == Ng && (!CL || member == cl.G - 1)) {
      // nodes beyond the last ring: every ring below them
      #pragma unroll 1
      for (int g = gb_lo + 1; g < ngB; ++g) {
        gscr[GS * g] = d2(S.hi, S.lo);
        gscr[GS * g + 1] = d2(PT.hi, PT.lo);
      }
    }
    // this member's nodes (all of them for a single workgroup)
    int g_begin = 0, g_end = ngB;
    if (GRID && CL && ngB > 0) {
      g_begin = grid_last_below(rho_mprev, dgB, idgB, ngB, grB) + 1;
      if (member < cl.G - 1) g_end = grid_last_below(rho_mlast, dgB, idgB, ngB, grB) + 1;
    }

    // ---- growing mode g (prefix) and decaying mode h (suffix) ----
    Pack<5> gp, gt, hx, ht;
    block_prefix_suffix<NT, 5, 5, FwdMatSumOp, BwdMatSumOp, false>(
        Pack<5>{{G.v[0], G.v[1], G.v[2], G.v[3], Vw}}, Pack<5>{{1.0, 0.0, 0.0, 1.0, 0.0}},
        FwdMatSumOp(), Pack<5>{{G.v[3], -G.v[1], -G.v[2], G.v[0], Vw}},
        Pack<5>{{1.0, 0.0, 0.0, 1.0, 0.0}}, BwdMatSumOp(), s_scanB, gp, gt, hx, ht);
    if (GRID && ngB > 0) {
      // psi, E_r - B_theta and the beam field at this member's nodes (the
      // scans' barriers order the sums written in pass B before these reads)
      const WAKE_GLOBAL D2* const gtab = reinterpret_cast<const WAKE_GLOBAL D2*>(gptr(I.grid_tab)) +
                                         (I.grid_off ? 3 * gofs : 0);
      WAKE_GLOBAL double* const gout = gptr(I.grid) + 5 * gofs;
      #pragma unroll 1
      for (int g = g_begin + tid; g < g_end; g += NT) {
        const double r = grid_node_r(g, dgB, grB);
        D2 t0, t1, t2;
        if (grid_lds) {
          t0 = s_gt[3 * g]; t1 = s_gt[3 * g + 1]; t2 = s_gt[3 * g + 2];
        } else {
          t0 = gtab[3 * g]; t1 = gtab[3 * g + 1]; t2 = gtab[3 * g + 2];
        }
        const D2 sS = gscr[GS * g], sP = gscr[GS * g + 1];
        grid_node_psi(gout, ngB, g, r, t0, t1, t2, dd{sS.x, sS.y}, dd{sP.x, sP.y}, psi_axis);
        double lam = 0.0;
        if (bm > 0) {
          int cb;
          if (staged) {
            cb = count_below(s_br, 0, bm, r, false);
            if (cb > 0) lam = s_bc[cb - 1];
          } else {
            cb = count_below(gR, 0, bm, r, false);
            if (cb > 0) lam = gQ[cb - 1];
          }
        }
        lam += analytic_lam(s_misc, n_an, r);
        gout[3 * ngB + g] = lam * rcp_nr(r);     // B^(b); pass E adds B^(p)
      }
    }
    double e_in = 0.0, d_in = 0.0;       // cooperative: det-sums of the members before / after
    if (CL) {
      // one exchange for the members' transfer products and det-sums: this
      // chunk's parts of the member's A, B, A', B' (Gl, Hl: the member's
      // transfers before the chunk and inverse transfers after it)
      const double vl = Vw + hx.v[4];
      const double mua = l0a - vl * l1a, mub = l0b - vl * l1b;
      const double k0 = G.v[3] * hx.v[0] - G.v[1] * hx.v[2], k1 = G.v[3] * hx.v[1] - G.v[1] * hx.v[3];
      const double k2 = -G.v[2] * hx.v[0] + G.v[0] * hx.v[2], k3 = -G.v[2] * hx.v[1] + G.v[0] * hx.v[3];
      Pack<8> part = {{gp.v[0] * mua + gp.v[2] * mub, gp.v[1] * mua + gp.v[3] * mub,
                       gp.v[0] * l1a + gp.v[2] * l1b, gp.v[1] * l1a + gp.v[3] * l1b,
                       k0 * mua + k2 * mub, k1 * mua + k3 * mub, k0 * l1a + k2 * l1b, k1 * l1a + k3 * l1b}};
      Pack<8> ab;
      block_prefix<NT, 8, SumOp<8>, false>(part, Pack<8>{{0, 0, 0, 0, 0, 0, 0, 0}}, SumOp<8>(), s_scanA, ab);
      Pack<13> mine;
#pragma unroll
      for (int i = 0; i < 5; ++i) mine.v[i] = gt.v[i];
#pragma unroll
      for (int i = 0; i < 8; ++i) mine.v[5 + i] = ab.v[i];
      if (!cl_gather<13, false>(cl, mine, s_x, s_ok)) {
        if (tid == 0 && member == 0) I.ctl[CTL_FAULT] = 1;
        return;
      }
      Pack<5> pg, sg;
      if (cl.G <= 64) cl_transfer_scan<13, FwdMatSumOp, BwdMatSumOp, 1>(s_x, member, cl.G, pg, gt, sg, ht, e_in, d_in);
      else cl_transfer_scan<13, FwdMatSumOp, BwdMatSumOp, 4>(s_x, member, cl.G, pg, gt, sg, ht, e_in, d_in);
      gp = FwdMatSumOp()(pg, gp);
      hx = BwdMatSumOp()(hx, sg);
    }
    const double W = gt.v[0];                 // det[g_N, (0,1)]
    const double iW = 1.0 / W;
    const double Vtot = gt.v[4];
    const double Vafter = hx.v[4];
    const double gsa = gp.v[0], gsb = gp.v[2];    // g at the chunk start
    const double hea = hx.v[1], heb = hx.v[3];    // h at the chunk end
    const double c = -(Vw + Vafter);
    const double la = l0a + c * l1a, lb = l0b + c * l1b;
    const double le = gsa * la + gsb * lb;        // sum of det[g_i, s_i] over the chunk
    const double hsa = G.v[3] * hea - G.v[1] * heb;   // h at the chunk start
    const double hsb = -G.v[2] * hea + G.v[0] * heb;
    const double lds = -(hsa * la + hsb * lb);     // sum of det[s_i, h_i] over the chunk
    Pack<1> ep, et, dsf, dt;
    block_prefix_suffix<NT, 1, 1, SumOp<1>, SumOp<1>, false>(
        Pack<1>{{le}}, Pack<1>{{0.0}}, SumOp<1>(), Pack<1>{{lds}}, Pack<1>{{0.0}}, SumOp<1>(),
        s_scanA, ep, et, dsf, dt);
    if (CL) {
      ep.v[0] = e_in + ep.v[0];
      dsf.v[0] = dsf.v[0] + d_in;
    }

    // ---- pass E: B^(p), outputs, push ----
    // the next slice's beam-table entries, fetched now and stored after the pass
    const bool stage_next = do_push && n + 1 < end;
    BeamStage<NT> nbs;
    nbs.m = 0;
    if (stage_next) beam_fetch<NT>(I, n + 1, nbs);
    double ga = G.v[0] * gsa + G.v[1] * gsb;      // g at the chunk end
    double gb = G.v[2] * gsa + G.v[3] * gsb;
    double ha = hea, hb = heb;
    double Vgt = Vafter;
    double E = ep.v[0] + le;
    double D = dsf.v[0];
    double nxt_r = INFINITY, last_r = INFINITY;
    int32_t nxt_i = 0x7fffffff, last_i = 0x7fffffff;
    dd sw2 = {0.0, 0.0}, swl2 = {0.0, 0.0};
    double dis_l = 0.0;
    // loads run ahead (the march goes backward): the state of ring k-2 and
    // the constants of ring k-1 are requested while ring k is computed
    D2 y_ru = d2(1.0, 0.0), y_f = d2(0.0, 0.0), y_ps = d2(0.0, 0.0), y_ln = d2(0.0, 0.0);   // ring k-1
    int32_t y_hs = 0;
    D2 v_ru = d2(1.0, 0.0), v_f = d2(0.0, 0.0), v_ps = d2(0.0, 0.0), v_ln = d2(0.0, 0.0);   // ring k-2
    int32_t v_hs = 0;
    int bhi = 0;                // beam-table entries below the ring (pass B's count, met downward)
    D2 c_w = d2(1.0, 0.0);      // ring k-1
    if (cnt > 0) {
      const unsigned sl = (cnt - 1) * NT + tid;
      const unsigned s = WAKE_SLOT(sl);
      y_ru = Sc.ld(RS_RU, s); y_f = Sc.ld(RS_F, s); y_ln = Sc.ld(RS_LN, s);
      y_ps = SCR.ld(SC_PSI, goff + sl);
      y_hs = st_hs(Sc, s);
    }
    if (cnt > 1) {
      const unsigned sl = (cnt - 2) * NT + tid;
      const unsigned s = WAKE_SLOT(sl);
      v_ru = Sc.ld(RS_RU, s); v_f = Sc.ld(RS_F, s); v_ln = Sc.ld(RS_LN, s);
      v_ps = SCR.ld(SC_PSI, goff + sl);
      v_hs = st_hs(Sc, s);
    }
    if (cnt > 0) c_w = KC.ld(RC_W, (unsigned)y_hs);
    // field grid: ge_hi the last node at or below the current ring, ge_top
    // its radius (a previous ring below it means the interval owns nodes).
    // chi (fixed node sets): the nodes also take the sums of c = w / psibar
    // and c rho at and above them within this chunk, and who handed them.
    const bool chi = CHI && ngB > 0 && !I.grid_off && I.grid_chi;
    GridNodes GN;
    GN.rad = grB;
    GN.dg = dgB;
    GN.idg = idgB;
    GN.nr = ngB;
    GN.nh = chi ? ngB + 1 : ngB;
    GN.top = 0.0;
    if (chi) {
      const double rl = grid_node_r(ngB - 1, dgB, grB);
      GN.top = ngB > 1 ? rl + (rl - grid_node_r(ngB - 2, dgB, grB)) : 2.0 * rl;
    }
    const double owner = (double)(member * NT + tid);
    dd cg0 = {0.0, 0.0}, cg1 = {0.0, 0.0};
    int ge_hi = -1;
    double ge_top = -INFINITY, g_lo_r = -1.0;
    if (GRID && ngB > 0 && cnt > 0) {
      if (tid > 0) g_lo_r = Sc.ld(RS_RU, WAKE_SLOT((unsigned)((C - 1) * NT + tid - 1))).x;
      else if (CL) g_lo_r = rho_mprev;
      ge_hi = GN.last_below(y_ru.x);
      if (p0 + cnt == Ng && (!CL || member == cl.G - 1)) {
        // nodes beyond the last ring: interval N (a_N = 0, no ring outside)
        const double a = (ha * E - ga * D) * iW, b = (hb * E - gb * D) * iW;
        #pragma unroll 1
        for (int g = ge_hi + 1; g < GN.nh; ++g) {
          gscr[GS * g + 2] = d2(Vgt, a);
          gscr[GS * g + 3] = d2(b, owner);
          if (CHI) {
            gscr[GS * g + 4] = d2(0.0, 0.0);
            gscr[GS * g + 5] = d2(0.0, 0.0);
          }
        }
      }
      ge_top = ge_hi >= 0 ? GN.r(ge_hi) : -INFINITY;
    }
    #pragma unroll 1
    for (int k = cnt - 1; k >= 0; --k) {
      const unsigned sl = k * NT + tid;
      const double rho = y_ru.x, u = y_ru.y, fr_p = y_f.x, fu_p = y_f.y;
      const int32_t hs = y_hs;
      const double psi = y_ps.x, dpsi = y_ps.y;
      const double w = c_w.x, wh = c_w.y;
      const dd lr0 = {y_ln.x, y_ln.y};
      y_ru = v_ru; y_f = v_f; y_hs = v_hs; y_ps = v_ps; y_ln = v_ln;
      if (k > 1) {
        const unsigned sp = sl - 2 * NT;
        const unsigned s = WAKE_SLOT(sp);
        v_ru = Sc.ld(RS_RU, s); v_f = Sc.ld(RS_F, s); v_ln = Sc.ld(RS_LN, s);
        v_ps = SCR.ld(SC_PSI, goff + sp);
        v_hs = st_hs(Sc, s);
      }
      if (k > 0) c_w = KC.ld(RC_W, (unsigned)y_hs);
      const double a2 = has_laser ? A2[goff + sl] : 0.0, da2 = has_laser ? DA2[goff + sl] : 0.0;
      const double irho = rcp_nr(rho);
      // B^(b) as pass B formed it: the table count, then the analytic beams
      double lam = 0.0;
      if (bm > 0) {
        if (staged) {
          bhi = count_below_down(s_br, bhi, bm, rho, k < cnt - 1);
          if (bhi > 0) lam = s_bc[bhi - 1];
        } else {
          bhi = count_below_down(gR, bhi, bm, rho, k < cnt - 1);
          if (bhi > 0) lam = gQ[bhi - 1];
        }
      }
      #pragma unroll 1
      for (int si = 0; si < n_an; ++si)
        if (s_misc[3 * si] == 2.0) lam += s_misc[3 * si + 1] * (-expm1(-rho * rho * s_misc[3 * si + 2]));
      const double bb = lam * irho;
      const Local L = local_of(irho, u, w, psi, a2);
      const double dz = -(Vgt + (w - wh) * u * irho * L.ipb);
      double B, Cc;
      ring_BC(irho, u, w, L, dpsi, dz, bb, da2, B, Cc);
      double sa, sb;
      rec_offset(L.A, B, Cc, rho, sa, sb);
      D += sa * hb - sb * ha;                              // D_{i-1} (det[s_i, h_i])
      E -= ga * sb - gb * sa;                              // E_{i-1} (det[g_i, s_i])
      const double hh = 0.5 * L.A * rho, q = 0.5 * L.A * irho, pp = hh * rho * rho;
      const double nga = (1.0 - hh) * ga - q * gb, ngb = pp * ga + (1.0 + hh) * gb;   // M_i^-1 g_i
      const double nha = (1.0 - hh) * ha - q * hb, nhb = pp * ha + (1.0 + hh) * hb;   // M_i^-1 h_i
      ga = nga; gb = ngb; ha = nha; hb = nhb;
      const double a = (ha * E - ga * D) * iW;
      const double b = (hb * E - gb * D) * iW;
      const double bp = a * rho + b * irho + wh * rcp_nr(w) * Cc;
      const double bt = bb + bp;
      const double ez = -dz;
      if (!(isfinite(psi) && isfinite(dpsi) && isfinite(ez) && isfinite(bt))) bad = 1.0;
      const int32_t id = WAKE_ID(hs);
      if (rec_snap) {
        WAKE_GLOBAL double* sp = gptr(I.snap) + (size_t)(n / I.stride) * OUT_N * N;
        sp[OUT_PSI * N + id] = psi; sp[OUT_ERBT * N + id] = -dpsi;
        sp[OUT_EZ * N + id] = ez; sp[OUT_BT * N + id] = bt;
        sp[OUT_RHO * N + id] = rho; sp[OUT_UR * N + id] = u;
      }
      if (rec_last) {
        WAKE_GLOBAL double* sp = gptr(I.last);
        sp[OUT_PSI * N + id] = psi; sp[OUT_ERBT * N + id] = -dpsi;
        sp[OUT_EZ * N + id] = ez; sp[OUT_BT * N + id] = bt;
        sp[OUT_RHO * N + id] = rho; sp[OUT_UR * N + id] = u;
      }
      if (do_push) {
        const double f_r = u * L.ipb;
        const double f_u = L.gm * dpsi * L.ipb - bt - 0.25 * da2 * L.ipb;
        double pr = f_r, pu = f_u;
        if (n > 0) { pr = fr_p; pu = fu_p; }
        double rn = rho + dxi * (1.5 * f_r - 0.5 * pr);
        double un = u + dxi * (1.5 * f_u - 0.5 * pu);
        double sr = f_r, su = f_u;
        if (rn < 0.0) { rn = -rn; un = -un; sr = -sr; su = -su; }
        if (!(isfinite(rn) && isfinite(un))) bad = 1.0;
        // ln rho moves with the ring: the old value plus log1p of the step
        const dd lr = dd_add_d(lr0, log1p_fast((rn - rho) * irho));
        Sn.st(RS_RU, goff + sl, d2(rn, un));
        Sn.st(RS_F, goff + sl, d2(sr, su));
        Sn.st(RS_LN, goff + sl, d2(lr.hi, lr.lo));
        Sn.sti(RS_W, goff + sl, hs);
        sw2 = dd_add_d(sw2, w);
        swl2 = dd_add_fast(swl2, dd_mul_d(lr, w));
        if (lds_keys) { s_kr[sl] = rn; s_ki[sl] = (uint16_t)id; }
        if (CL) { gptr(I.gk_r)[goff + sl] = rn; gptr(I.gk_i)[goff + sl] = id; }
        if (!key_lt(rn, id, nxt_r, nxt_i)) dis_l = 1.0;
        if (k == cnt - 1) { last_r = rn; last_i = id; }
        nxt_r = rn;
        nxt_i = id;
      }
      Vgt += L.v;
      if (GRID) {
        if (CHI && chi) {
          const double c = w * L.ipb;
          cg0 = dd_add_d(cg0, c);
          cg1 = dd_add(cg1, two_prod(c, rho));
        }
        const double rlo = k > 0 ? y_ru.x : g_lo_r;
        if (rlo < ge_top) {
          // nodes of interval p = (rho_{p-1}, rho_p]
          const int glo = GN.last_below(rlo) + 1;
          #pragma unroll 1
          for (int g = glo; g <= ge_hi; ++g) {
            gscr[GS * g + 2] = d2(Vgt, a);
            gscr[GS * g + 3] = d2(b, owner);
            if (CHI) {
              gscr[GS * g + 4] = d2(cg0.hi, cg0.lo);
              gscr[GS * g + 5] = d2(cg1.hi, cg1.lo);
            }
          }
          ge_hi = glo - 1;
          ge_top = ge_hi >= 0 ? GN.r(ge_hi) : -INFINITY;
        }
      }
    }
    if (tid == 0 && member == 0) { gptr(I.axis)[2 * n] = psi_axis; gptr(I.axis)[2 * n + 1] = Vtot; }
    // order across chunk boundaries: this chunk's first pushed key (+inf if
    // empty) against the previous chunk's last one
    s_fr[tid] = nxt_r;
    s_fi[tid] = nxt_i;
    if (CL && do_push && cnt > 0 && p0 + cnt == Ng) { s_misc[48] = last_r; s_misc[49] = (double)last_i; }
    if (stage_next) {
      __syncthreads();        // every wave is done with this slice's table and constants
      stage_analytic<NT>(I, n + 1, s_misc);
      beam_store<NT>(nbs, s_br, s_bc);
    }
    // out of time: this slice is the launch's last (one clock read, broadcast;
    // cooperative members decide together at the next slice head)
    if (tid == 0)
      s_misc[63] = !CL && budget > 0 && (int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) >= budget ? 1.0 : 0.0;
    __syncthreads();
    if (s_misc[63] != 0.0) end = n + 1;
    if (GRID && ngB > 0) {
      // E_z and B_theta at this member's nodes (after the barrier above)
      WAKE_GLOBAL double* const gout = gptr(I.grid) + 5 * gofs;
      #pragma unroll 1
      for (int g = g_begin + tid; g < g_end; g += NT) {
        const double r = grid_node_r(g, dgB, grB);
        const D2 e0 = gscr[GS * g + 2], e1 = gscr[GS * g + 3];
        grid_node_b(gout, ngB, g, r, e0.x, e0.y, e1.x, gout[3 * ngB + g]);
      }
      if (CHI && chi) {
        // chi = n/gamma (reading R20): each node's owner adds the sums of
        // the chunks after its own; the hats' sums are differences of the
        // full sums D, E (c and c rho at and above a node) of neighbouring
        // nodes
        Pack<4> tot;
        const Pack<4> later = block_suffix<NT, 4>(Pack<4>{{cg0.hi, cg0.lo, cg1.hi, cg1.lo}},
                                                  Pack<4>{{0.0, 0.0, 0.0, 0.0}}, DD2Op(), s_scanA, tot);
        WAKE_GLOBAL double* const thr = gptr(I.grid_thr);
        #pragma unroll
        for (int i = 0; i < 4; ++i) thr[4 * (size_t)(member * NT + tid) + i] = later.v[i];
        dd all0 = {tot.v[0], tot.v[1]};
        const double* msuf = nullptr;          // sums of the members after each member
        if (CL) {
          // member totals (the fenced form: the nodes' partial sums and the
          // threads' suffixes become visible to every member)
          if (!cl_gather<4, true>(cl, tot, s_x, s_ok)) {
            if (tid == 0 && member == 0) I.ctl[CTL_FAULT] = 1;
            return;
          }
          if (tid == 0) {
            Pack<4> run = {{0.0, 0.0, 0.0, 0.0}};
            for (int m = cl.G - 1; m >= 0; --m) {
              const Pack<4> x = {{s_x[4 * m], s_x[4 * m + 1], s_x[4 * m + 2], s_x[4 * m + 3]}};
              #pragma unroll
              for (int i = 0; i < 4; ++i) s_x[4 * m + i] = run.v[i];
              run = DD2Op()(x, run);
            }
            #pragma unroll
            for (int i = 0; i < 4; ++i) s_x[4 * cl.G + i] = run.v[i];
          }
          __syncthreads();
          all0 = {s_x[4 * cl.G], s_x[4 * cl.G + 1]};
          msuf = s_x;
        } else {
          __syncthreads();
        }
        chi_nodes<NT, CL>(gout, ngB, gscr, thr, msuf, (CL ? cl.G : 1) * NT, GN, g_begin + tid, g_end, all0);
      }
    }
    if (do_push && cnt > 0 && tid + 1 < NT && !key_lt(last_r, last_i, s_fr[tid + 1], s_fi[tid + 1]))
      dis_l = 1.0;
    dis = dis_l;
    if (!CL && lds_keys) {    // the chunks' flags for the fix-up at the next slice head
      const uint64_t m = __ballot(dis_l != 0.0);
      if ((tid & 63) == 0) s_dmask[tid >> 6] = m;
    }
    unpushed = cur;
    if (do_push) {
      // the pushed rings sit at the slots of this slice's positions
      cur = nb;
      ident = true;
      push_keys = CL;
      sw = sw2;
      swl = swl2;
      sw_push = sw2;
      swl_push = swl2;
    }
    ++n;
  }
  if (tid == 0 && member == 0) {
    I.ctl[CTL_CUR] = cur;
    I.ctl[CTL_NEXT] = end;
    atomicAdd(I.cnt + CNT_SLICES, (unsigned long long)(end - I.first));
    if (CL) atomicAdd(I.cnt + CNT_CL_MEETINGS, (unsigned long long)cl.round);
  }
#undef WAKE_SLOT
#undef WAKE_ID
#undef WAKE_MOVED
}

// the cooperative march as a function of its own (its registers stay out of
// the single-workgroup march, which is inlined into the kernel)
template <int NT, int GM>
__device__ __noinline__ void march_member(const WAKE_GLOBAL WakeInst* I, int member, const int32_t* queue) {
  march<NT, true, GM>(*(const WakeInst*)I, member, queue, wake_lds);
}

#ifndef WAKE_WAVES_PER_EU
#define WAKE_WAVES_PER_EU 2
#endif
// WAKE_WAVES_PER_EU waves per SIMD (2: up to 256 VGPRs per lane)
template <int NT, int GM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAKE_WAVES_PER_EU)))
void wake_march_kernel(const WakeInst* __restrict__ insts, int n_insts, int n_tasks, int32_t* counter) {
  unsigned char* const smem = wake_lds;
  __shared__ int s_idx;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(s_idx);
    __syncthreads();
    if (idx >= n_tasks) return;   // every workgroup leaves once the queue is empty
    // task idx: member idx - task0 of the last instance with task0 <= idx
    int lo = 0, hi = n_insts;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (__builtin_amdgcn_readfirstlane(insts[mid].task0) <= idx) lo = mid; else hi = mid;
    }
    const WakeInst& I = insts[lo];
    if (I.nt == NT) {
      if (I.G > 1) march_member<NT, GM>(as_global(I), idx - I.task0, counter);
      else march<NT, false, GM>(I, 0, counter, smem);
    }
    __syncthreads();
  }
}

__global__ void counter_zero_kernel(int32_t* p) {
  if (threadIdx.x == 0) p[0] = 0;
}

// barrier words of the cooperative instances of a launch start at zero
// and their packs carry no stamp of this launch's rounds
__global__ void cluster_reset_kernel(const WakeInst* __restrict__ insts, int n_insts) {
  for (int i = threadIdx.x; i < n_insts; i += blockDim.x) {
    const int G = insts[i].G;
    if (G <= 1) continue;
    insts[i].xc[0] = 0; insts[i].xc[1] = 0; insts[i].xc[2] = 0;
    for (int k = 0; k < 2 * G; ++k) insts[i].xd[cl_stamp_at(G, k / G, k % G)] = -1.0;
  }
}

// ---------------------------------------------------------------------------
// state transfers by ring id, reset
// ---------------------------------------------------------------------------
__global__ void state_by_id_kernel(WakeInst I, double* rho, double* u, double* fr, double* fu) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= I.N) return;
  const int c = I.ctl[CTL_CUR];
  const unsigned sl = slot_of(p, I.C, I.nt);
  const size_t PS = (size_t)I.G * I.C * I.nt;
  const D2* r = reinterpret_cast<const D2*>(I.st[c]) + sl;
  const int hs = reinterpret_cast<const int32_t*>(I.st[c])[4 * RS_W * PS + sl];
  const int i = pos_of_slot(hs, I.C, I.nt);
  if (rho) rho[i] = r[RS_RU * PS].x;
  if (u) u[i] = r[RS_RU * PS].y;
  if (fr) fr[i] = r[RS_F * PS].x;
  if (fu) fu[i] = r[RS_F * PS].y;
}

// Injected state (by id) at position = id in buffer 0; the marcher orders
// it before its first slice.  Interval hints start at the rings' nodes.
__global__ void state_set_kernel(WakeInst I, const double* rho, const double* u, const double* fr,
                                 const double* fu, int slice) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) { I.ctl[CTL_CUR] = 0; I.ctl[CTL_BREAK] = -1; I.ctl[CTL_NEXT] = slice; I.ctl[CTL_FAULT] = 0; }
  if (i >= I.N) return;
  const unsigned sl = slot_of(i, I.C, I.nt);
  const size_t PS = (size_t)I.G * I.C * I.nt;
  D2* r = reinterpret_cast<D2*>(I.st[0]) + sl;
  const D2* k = reinterpret_cast<const D2*>(I.cst) + sl;
  const dd lr = ring_log(k[RC_R0 * PS], k[RC_LN * PS], rho[i]);
  r[RS_RU * PS] = d2(rho[i], u[i]);
  r[RS_F * PS] = d2(fr ? fr[i] : 0.0, fu ? fu[i] : 0.0);
  r[RS_LN * PS] = d2(lr.hi, lr.lo);
  int32_t* wd = reinterpret_cast<int32_t*>(I.st[0]) + 4 * RS_W * PS;
  wd[sl] = (int32_t)sl;
  wd[PS + sl] = i + 1;
}

// Back to the state at slice 0 (rings at rest at their initial radii);
// one workgroup per instance.
__global__ void state_reset_kernel(const WakeInst* __restrict__ insts, int n_insts) {
  const WakeInst& I = insts[blockIdx.x];
  for (int j = threadIdx.x; j < I.N; j += blockDim.x) {
    const unsigned sl = slot_of(j, I.C, I.nt);
    const size_t PS = (size_t)I.G * I.C * I.nt;
    D2* r = reinterpret_cast<D2*>(I.st[0]) + sl;
    const D2* k = reinterpret_cast<const D2*>(I.cst) + sl;
    r[RS_RU * PS] = d2(k[RC_R0 * PS].x, 0.0);
    r[RS_F * PS] = d2(0.0, 0.0);
    r[RS_LN * PS] = k[RC_LN * PS];
    int32_t* wd = reinterpret_cast<int32_t*>(I.st[0]) + 4 * RS_W * PS;
    wd[sl] = (int32_t)sl;
    wd[PS + sl] = j + 1;
  }
  if (threadIdx.x == 0) { I.ctl[CTL_CUR] = 0; I.ctl[CTL_BREAK] = -1; I.ctl[CTL_NEXT] = 0; I.ctl[CTL_FAULT] = 0; }
}

// Control words of a list of instances into one buffer (4 words each).
__global__ void ctl_gather_kernel(const WakeInst* __restrict__ insts, int n, int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int w = 0; w < CTL_NWORDS; ++w) out[i * CTL_NWORDS + w] = insts[i].ctl[w];
}

// ---------------------------------------------------------------------------
// host-callable launchers
// ---------------------------------------------------------------------------
hipError_t launch_ctl_gather(const WakeInst* d_insts, int n, int32_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ctl_gather_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_insts, n, out);
  return hipGetLastError();
}

hipError_t launch_init(const WakeInst& I, const double* r0, const double* dr, const double* dens,
                       hipStream_t s) {
  // block totals / offsets in the fix-up's scratch (4 doubles per block of 256 rings)
  const int nb = (I.N + 255) / 256;
  double* tmp = I.sm_r;
  hipLaunchKernelGGL((init_rings_kernel<256>), dim3(nb), dim3(256), 0, s, I, r0, dr, dens, tmp);
  hipLaunchKernelGGL(init_offsets_kernel, dim3(1), dim3(64), 0, s, I, tmp, nb);
  hipLaunchKernelGGL((init_nodes_kernel<256>), dim3(nb), dim3(256), 0, s, I, (const double*)tmp);
  hipLaunchKernelGGL(init_intervals_kernel, dim3((I.N + 1 + 255) / 256), dim3(256), 0, s, I);
  return hipGetLastError();
}

// Field-grid node table: ln r_g and the immobile ions' psi - psi(0) and
// d_rho psi at r_g (the same interpolation as at the rings), dd pairs.  The
// table is made once per grid, so psi's interpolation is carried out in
// double-double throughout: the weight t = (r - lo)/(hi - lo) from exact
// differences and the step between the nodes' double-double values (at the
// rings the step is rounded to double, which resolves psi to ~1e-16 of the
// step; nodes between rings at rest see psi of order w dr^2 only).
__global__ void grid_init_kernel(WakeInst I, double* tab, int n_entries) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_entries) return;
  const double r = I.grid_rad ? I.grid_rad[g] : ((double)g + 0.5) * I.grid_dr;
  const dd l = dd_log(r);
  IonView IV;
  IV.R = uview(I.ion);
  IV.N = I.N;
  IV.Rp = I.Rp;
  IV.T0 = {I.tot0[0], I.tot0[1]};
  IV.Q = {I.tot0[2], I.tot0[3]};
  int h = 0;
  double q[WAKE_ION_REC];
  ion_load(IV, h, q);
  dd ps, dp;
  ion_fields(IV, r, l, h, q, ps, dp);
  if (r < I.Rp) {
    const dd a = two_sum(r, -q[IR_LO]);            // r - lo, exact
    const dd b = two_sum(q[IR_HI], -q[IR_LO]);     // hi - lo, exact
    dd t = dd_div_d(a, b.hi);
    t = dd_add_d(t, -t.hi * b.lo / b.hi);          // a / (b.hi + b.lo) to second order
    dd nxt;                                         // psi - psi(0) at the upper node
    if (h < I.N) {
      nxt = {I.ion[(size_t)(h + 1) * WAKE_ION_REC + IR_PSH], I.ion[(size_t)(h + 1) * WAKE_ION_REC + IR_PSL]};
    } else {                                        // the plasma edge: exterior value there
      nxt = dd_sub(IV.T0, dd_mul(IV.Q, dd_log(I.Rp)));
    }
    const dd lo_ps = {q[IR_PSH], q[IR_PSL]};
    ps = dd_add(lo_ps, dd_mul(dd_sub(nxt, lo_ps), t));
  }
  double* t = tab + (size_t)WAKE_GRID_TAB * g;
  t[0] = l.hi; t[1] = l.lo;
  t[2] = ps.hi; t[3] = ps.lo;
  t[4] = dp.hi; t[5] = dp.lo;
}

hipError_t launch_grid_init(const WakeInst& I, double* tab, int n_entries, hipStream_t s) {
  if (n_entries <= 0) return hipSuccess;
  hipLaunchKernelGGL(grid_init_kernel, dim3((n_entries + 255) / 256), dim3(256), 0, s, I, tab, n_entries);
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

#define WAKE_THREADS(X) X(256) X(512)

size_t march_lds_bytes(int nt) {
#define X(a) \
  if (nt == a) return MarchLds<a>::bytes();
  WAKE_THREADS(X)
#undef X
  return 0;
}

hipError_t launch_march(int nt, const WakeInst* d_insts, int n_insts, int n_tasks, int32_t* counter,
                        int grid, int grid_mode, hipStream_t s) {
#define X(a)                                                                                      \
  if (nt == a) {                                                                                  \
    hipLaunchKernelGGL(counter_zero_kernel, dim3(1), dim3(64), 0, s, counter);                     \
    hipLaunchKernelGGL(cluster_reset_kernel, dim3(1), dim3(256), 0, s, d_insts, n_insts);          \
    if (grid_mode == 2)                                                                           \
      hipLaunchKernelGGL((wake_march_kernel<a, 2>), dim3(grid), dim3(a),                          \
                         MarchLds<a>::bytes() + grid_lds_bytes<a>(), s, d_insts, n_insts, n_tasks, \
                         counter);                                                                \
    else if (grid_mode == 1)                                                                      \
      hipLaunchKernelGGL((wake_march_kernel<a, 1>), dim3(grid), dim3(a),                          \
                         MarchLds<a>::bytes() + grid_lds_bytes<a>(), s, d_insts, n_insts, n_tasks, \
                         counter);                                                                \
    else                                                                                          \
      hipLaunchKernelGGL((wake_march_kernel<a, 0>), dim3(grid), dim3(a), MarchLds<a>::bytes(),    \
                         s, d_insts, n_insts, n_tasks, counter);                                  \
    return hipGetLastError();                                                                     \
  }
  WAKE_THREADS(X)
#undef X
  return hipErrorInvalidValue;
}

int march_cmax(int nt) {
#define X(a) \
  if (nt == a) return MarchLds<a>::CMAX;
  WAKE_THREADS(X)
#undef X
  return 0;
}

int march_occupancy(int nt) {
  int nb = 0;
#define X(a)                                                                                      \
  if (nt == a) {                                                                                  \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, wake_march_kernel<a, 0>, a,         \
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
  if (nt == a) {                                                                                  \
    hipError_t e = hipFuncSetAttribute((const void*)wake_march_kernel<a, 0>,                      \
                                       hipFuncAttributeMaxDynamicSharedMemorySize,                \
                                       (int)MarchLds<a>::bytes());                                \
    if (e != hipSuccess) return e;                                                                \
    e = hipFuncSetAttribute((const void*)wake_march_kernel<a, 1>,                                 \
                            hipFuncAttributeMaxDynamicSharedMemorySize,                           \
                            (int)(MarchLds<a>::bytes() + grid_lds_bytes<a>()));                   \
    if (e != hipSuccess) return e;                                                                \
    return hipFuncSetAttribute((const void*)wake_march_kernel<a, 2>,                              \
                               hipFuncAttributeMaxDynamicSharedMemorySize,                        \
                               (int)(MarchLds<a>::bytes() + grid_lds_bytes<a>()));                \
  }
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
