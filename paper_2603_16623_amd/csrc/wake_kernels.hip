// gfx950 kernels of the gridless quasistatic plasma-ring solver.
//
// Model (paper, Sec. "Gridless quasistatic model"): axisymmetric electron
// rings (q=-1, m=1) over immobile ions, marched in xi = -zeta.  Per slice:
// radial sort (ring id breaks ties), beam/laser sources, the Gauss/log sums
// for psi and d_rho psi (eqs. dpsi_dr, psi), gamma (eq. motion_4), the
// d_zeta psi sum (eq. dpsi_dzeta, derived sign), coefficients A, B, C
// (eqs. b_coeffs_1-3, ponderomotive term with the 1/4 of eq. motion_1 and
// the physical sign), the two-point recursion for B_theta^(p) (eq. ai_bi,
// b_0 = 0, a_N = 0) and the Adams-Bashforth-2 push (eqs. motion_1-2).
//
// One workgroup owns one instance and marches all of its slices.  Rings
// sit in sorted order; thread t of a tile owns K consecutive rings.  Per
// slice two passes run over the tiles:
//   pass 1 (forward)  double-double prefix of (w, w ln rho) -> psi, d_rho psi;
//                     gamma, A, M_i; prefix product of M_i (growing mode g,
//                     g_0 = (1,0)); prefix of v_i = w u/(rho psibar);
//                     prefix sums E0, E1 of det[g_i, s_i] where s_i is
//                     affine in the (not yet known) total V = sum v.
//   pass 2 (backward) suffix product of M_i^-1 (decaying mode h, h_N=(0,1)),
//                     suffix of v -> d_zeta psi, B_i, s_i; suffix D of
//                     det[s_i, h_i]; then x_{i-1} = (h_{i-1} E_{i-1} -
//                     g_{i-1} D_{i-1}) / W with W = det[g, h] = a-part of
//                     g_N; B^(p), outputs, push.
// This Green's-function form of the recursion solves the same linear
// system as the paper's shooting (Appendix) without its exponential loss
// of digits.  The cancelling Gauss/log sums run in double-double.
#include "wake_common.h"
#include "wake_device.h"

#include <math.h>

#define WAKE_SORT_CAP 2048   // beam entries per slice sorted in LDS

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ion_fields(const WakeInst& I, double r, dd lnr, dd& ps, dd& dp) {
  // Ion psi - psi(0) and d_rho psi at radius r: linear interpolation between
  // the node j with r_j < r <= r_{j+1} (Sec. "Key algorithmic adjustments"),
  // exact exterior field beyond the plasma edge.
  const dd Q = {I.tot0[2], I.tot0[3]};
  if (r > I.Rp) {
    dd qlr = dd_mul(Q, lnr);
    ps = dd_sub({I.tot0[0], I.tot0[1]}, qlr);
    dp = dd_neg(dd_div_d(Q, r));
    return;
  }
  int b = (int)(r * I.lut_scale);
  b = b < 0 ? 0 : (b > I.lut_n - 1 ? I.lut_n - 1 : b);
  int lo = I.ion_lut[b > 0 ? b - 1 : 0];
  int hi = I.ion_lut[b + 2 < I.lut_n ? b + 2 : I.lut_n];
  // smallest idx in [lo, hi] with ion_r[idx] >= r
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (I.ion_r[mid] < r) lo = mid + 1; else hi = mid;
  }
  // r > 0 always has ion_r[0] = 0 below it; a zero or NaN radius (a
  // breakdown, flagged by the caller) must still index inside the table
  int j = lo - 1;
  j = j < 0 ? 0 : (j > I.N ? I.N : j);
  const double r0 = I.ion_r[j], r1 = I.ion_r[j + 1];
  const double t = (r - r0) / (r1 - r0);
  const dd p0 = {I.ion_ps_hi[j], I.ion_ps_lo[j]}, p1 = {I.ion_ps_hi[j + 1], I.ion_ps_lo[j + 1]};
  const dd d0 = {I.ion_dp_hi[j], I.ion_dp_lo[j]}, d1 = {I.ion_dp_hi[j + 1], I.ion_dp_lo[j + 1]};
  ps = dd_add(p0, dd_mul_d(dd_sub(p1, p0), t));
  dp = dd_add(d0, dd_mul_d(dd_sub(d1, d0), t));
}

// ln(rho) of ring `id` as ln r0 + log1p((rho - r0)/r0): accurate relative to
// the ring's displacement, which keeps the psi sums (where ln rho is
// multiplied by the enclosed charge) free of log rounding.
__device__ __forceinline__ dd ring_log(const WakeInst& I, int id, double rho) {
  const double r0 = I.ion_r[id + 1];
  const double l1 = log1p((rho - r0) / r0);
  return dd_add_d({I.L0_hi[id], I.L0_lo[id]}, l1);
}

// Coefficients of eqs. b_coeffs_1-3 for an electron ring (q=-1, m=1).
__device__ __forceinline__ void ring_coeffs(double rho, double u, double w, double pb, double gm,
                                            double dpsi, double dz, double bb, double da2,
                                            double& A, double& B, double& C) {
  const double wr = w / rho;
  const double ipb = 1.0 / pb;
  const double ipb2 = ipb * ipb;
  const double u2 = u * u;
  A = wr * ipb;
  B = -wr * gm * dpsi * ipb2 + wr * bb * ipb + 0.25 * wr * da2 * ipb2 + (wr / rho) * u2 * ipb2 +
      wr * u2 * dpsi * ipb2 * ipb - wr * u * dz * ipb2;
  C = -wr * (gm * ipb - 1.0) + wr * u2 * ipb2;
}

__device__ __forceinline__ void rec_offset(double A, double B, double C, double rho, double& sa,
                                           double& sb) {
  sa = (2.0 * B + A * C) * 0.25;
  sb = rho * (4.0 * C - 2.0 * B * rho - A * C * rho) * 0.25;
}

__device__ __forceinline__ Pack<4> rec_matrix(double A, double rho) {
  const double h = 0.5 * A * rho;
  return {{1.0 + h, A / (2.0 * rho), -h * rho * rho, 1.0 - h}};
}

__device__ __forceinline__ double gamma_of(double u, double pb, double a2) {
  return (1.0 + u * u + pb * pb + 0.5 * a2) / (2.0 * pb);
}

// ---------------------------------------------------------------------------
// ring-set initialisation: weights, ion node tables, initial state
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
  double* ion_r = const_cast<double*>(I.ion_r);
  double* dph = const_cast<double*>(I.ion_dp_hi);
  double* dpl = const_cast<double*>(I.ion_dp_lo);
  double* psh = const_cast<double*>(I.ion_ps_hi);
  double* psl = const_cast<double*>(I.ion_ps_lo);
  double* consts = const_cast<double*>(I.tot0);
  double* l0h = const_cast<double*>(I.L0_hi);
  double* l0l = const_cast<double*>(I.L0_lo);
  dd cS = {0.0, 0.0}, cPT = {0.0, 0.0};
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
      w_out[j] = w;
      wh_out[j] = wh;
      l0h[j] = lr.hi;
      l0l[j] = lr.lo;
    }
    const dd wl = dd_mul_d(lr, w);
    Pack<4> tot;
    Pack<4> pre = block_prefix<NT, 4>(Pack<4>{{w, 0.0, wl.hi, wl.lo}}, Pack<4>{{0, 0, 0, 0}},
                                      DD2Op(), s_scan, tot);
    const dd S = dd_add(cS, {pre.v[0], pre.v[1]});
    const dd PTi = dd_add(dd_add(cPT, {pre.v[2], pre.v[3]}), wl);
    if (ok) {
      // ion ring j (q=+1) at its own radius, self weight w^
      const dd dp = dd_neg(dd_div_d(dd_add_d(S, wh), r));
      const dd ps = dd_neg(dd_sub(dd_mul(dd_add_d(S, w), lr), PTi));
      ion_r[j + 1] = r;
      dph[j + 1] = dp.hi; dpl[j + 1] = dp.lo;
      psh[j + 1] = ps.hi; psl[j + 1] = ps.lo;
      I.rho[0][j] = r;
      I.u[0][j] = 0.0;
      I.fr[0][j] = 0.0;
      I.fu[0][j] = 0.0;
      I.id[0][j] = j;
    }
    cS = dd_add(cS, {tot.v[0], tot.v[1]});
    cPT = dd_add(cPT, {tot.v[2], tot.v[3]});
  }
  if (tid == 0) {
    // virtual nodes: axis and plasma edge
    ion_r[0] = 0.0;
    dph[0] = 0.0; dpl[0] = 0.0; psh[0] = 0.0; psl[0] = 0.0;
    const double Rp = I.Rp;
    ion_r[N + 1] = Rp;
    const dd dp = dd_neg(dd_div_d(cS, Rp));
    const dd ps = dd_sub(cPT, dd_mul(cS, dd_log(Rp)));
    dph[N + 1] = dp.hi; dpl[N + 1] = dp.lo;
    psh[N + 1] = ps.hi; psl[N + 1] = ps.lo;
    consts[0] = cPT.hi; consts[1] = cPT.lo;   // sum_j w_j ln r0_j
    consts[2] = cS.hi; consts[3] = cS.lo;     // total weight Q
    I.ctl[CTL_CUR] = 0;
    I.ctl[CTL_BREAK] = -1;
    I.ctl[CTL_NEXT] = 0;
  }
}

// lut[b] = number of ion nodes with radius < b * Rp / lut_n
__global__ void wake_lut_kernel(WakeInst I) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > I.lut_n) return;
  const double x = (double)b / I.lut_scale;
  int lo = 0, hi = I.N + 2;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (I.ion_r[mid] < x) lo = mid + 1; else hi = mid;
  }
  const_cast<int32_t*>(I.ion_lut)[b] = lo;
}

// ---------------------------------------------------------------------------
// beam table: linear (cloud-in-cell) weights in xi onto the slice nodes,
// per-slice radius order, cumulative charge
// ---------------------------------------------------------------------------
struct BeamParts {
  const double *x, *y, *xi, *w, *q;
  int64_t n;
};

__device__ __forceinline__ void particle_entries(const BeamParts& P, int64_t k, double dxi, int n_xi,
                                                 double& r, int& n0, double& c0, double& c1) {
  {
#pragma clang fp contract(off)
    const double x = P.x[k], y = P.y[k];
    r = __builtin_sqrt(x * x + y * y);
  }
  const double t = P.xi[k] / dxi;
  const double fl = floor(t);
  const double f = t - fl;
  c0 = 1.0 - f;
  c1 = f;
  n0 = (fl < -2.0) ? -2 : (fl > (double)n_xi + 1.0 ? n_xi + 1 : (int)fl);
}

__global__ void beam_count_kernel(BeamParts P, double dxi, int n_xi, int32_t* __restrict__ cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  double r, c0, c1;
  int n0;
  particle_entries(P, k, dxi, n_xi, r, n0, c0, c1);
  if (n0 >= 0 && n0 <= n_xi - 1 && c0 > 0.0) atomicAdd(&cnt[n0], 1);
  if (n0 + 1 >= 0 && n0 + 1 <= n_xi - 1 && c1 > 0.0) atomicAdd(&cnt[n0 + 1], 1);
}

template <int NT>
__global__ __launch_bounds__(NT) void exclusive_scan_kernel(const int32_t* __restrict__ in, int n,
                                                            int32_t* __restrict__ out) {
  __shared__ double s_scan[(NT / 64) * 8];
  double carry = 0.0;
  for (int base = 0; base < n; base += NT) {
    const int i = base + threadIdx.x;
    const double v = i < n ? (double)in[i] : 0.0;
    Pack<1> tot;
    Pack<1> pre = block_prefix<NT, 1>(Pack<1>{{v}}, Pack<1>{{0.0}}, SumOp<1>(), s_scan, tot);
    if (i < n) out[i] = (int32_t)(carry + pre.v[0]);
    carry += tot.v[0];
  }
  if (threadIdx.x == 0) out[n] = (int32_t)carry;
}

__global__ void beam_scatter_kernel(BeamParts P, double dxi, int n_xi, const int32_t* __restrict__ poff,
                                    int32_t* __restrict__ cursor, double* __restrict__ er,
                                    double* __restrict__ eq, int64_t* __restrict__ ek) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  double r, c0, c1;
  int n0;
  particle_entries(P, k, dxi, n_xi, r, n0, c0, c1);
  const double qw = P.q[k] * P.w[k];
  if (n0 >= 0 && n0 <= n_xi - 1 && c0 > 0.0) {
    const int e = poff[n0] + atomicAdd(&cursor[n0], 1);
    er[e] = r; eq[e] = qw * c0; ek[e] = 2 * k;
  }
  if (n0 + 1 >= 0 && n0 + 1 <= n_xi - 1 && c1 > 0.0) {
    const int e = poff[n0 + 1] + atomicAdd(&cursor[n0 + 1], 1);
    er[e] = r; eq[e] = qw * c1; ek[e] = 2 * k + 1;
  }
}

__device__ __forceinline__ bool ent_lt(double ra, int64_t ka, double rb, int64_t kb) {
  return ra < rb || (ra == rb && ka < kb);
}

__global__ void pow2_kernel(const int32_t* __restrict__ cnt, int n, int32_t* __restrict__ cnt2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cnt[i];
  int p = c > 0 ? 1 : 0;
  while (p < c) p <<= 1;
  cnt2[i] = p;
}

// One workgroup per slice: bitonic sort of the slice's entries by (r, key)
// over its power-of-two padded segment (in LDS when it fits, else in
// global memory), then the cumulative charge / (2 pi dxi).
template <int NT>
__global__ __launch_bounds__(NT) void beam_sort_kernel(const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ poff, double* er,
                                                       double* eq, int64_t* ek, double inv2pidxi,
                                                       double* __restrict__ br,
                                                       double* __restrict__ bcum) {
  __shared__ double s_r[WAKE_SORT_CAP];
  __shared__ double s_q[WAKE_SORT_CAP];
  __shared__ int64_t s_k[WAKE_SORT_CAP];
  __shared__ double s_scan[(NT / 64) * 8];
  const int nd = blockIdx.x;
  const int b0 = off[nd], m = off[nd + 1] - b0;
  const int pb = poff[nd], p2 = poff[nd + 1] - pb;
  if (m == 0) return;
  const bool in_lds = p2 <= WAKE_SORT_CAP;
  double* R = in_lds ? s_r : er + pb;
  double* Qv = in_lds ? s_q : eq + pb;
  int64_t* Kv = in_lds ? s_k : ek + pb;
  for (int i = threadIdx.x; i < p2; i += NT) {
    if (i < m) {
      if (in_lds) { s_r[i] = er[pb + i]; s_q[i] = eq[pb + i]; s_k[i] = ek[pb + i]; }
    } else {
      R[i] = INFINITY; Qv[i] = 0.0; Kv[i] = INT64_MAX - i;
    }
  }
  __syncthreads();
  for (int size = 2; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < p2; i += NT) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const bool lt = ent_lt(R[j], Kv[j], R[i], Kv[i]);
          if (up ? lt : !lt) {
            const double tr = R[i]; R[i] = R[j]; R[j] = tr;
            const double tq = Qv[i]; Qv[i] = Qv[j]; Qv[j] = tq;
            const int64_t tk = Kv[i]; Kv[i] = Kv[j]; Kv[j] = tk;
          }
        }
      }
      __syncthreads();
    }
  }
  double carry = 0.0;
  for (int base = 0; base < m; base += NT) {
    const int i = base + threadIdx.x;
    const double v = i < m ? Qv[i] : 0.0;
    Pack<1> tot;
    Pack<1> pre = block_prefix<NT, 1>(Pack<1>{{v}}, Pack<1>{{0.0}}, SumOp<1>(), s_scan, tot);
    if (i < m) {
      br[b0 + i] = R[i];
      bcum[b0 + i] = (carry + pre.v[0] + v) * inv2pidxi;
    }
    carry += tot.v[0];
  }
}

// ---------------------------------------------------------------------------
// the slice marcher
// ---------------------------------------------------------------------------
struct MatSumOp {  // (forward matrix product, running sum)
  __device__ __forceinline__ Pack<5> operator()(const Pack<5>& a, const Pack<5>& b) const {
    Pack<4> ma = {{a.v[0], a.v[1], a.v[2], a.v[3]}}, mb = {{b.v[0], b.v[1], b.v[2], b.v[3]}};
    Pack<4> m = mat_mul(mb, ma);
    return {{m.v[0], m.v[1], m.v[2], m.v[3], a.v[4] + b.v[4]}};
  }
};
struct BwdMatSumOp {  // (index-order product of inverse transfers, running sum)
  __device__ __forceinline__ Pack<5> operator()(const Pack<5>& lo, const Pack<5>& hi) const {
    Pack<4> ma = {{lo.v[0], lo.v[1], lo.v[2], lo.v[3]}}, mb = {{hi.v[0], hi.v[1], hi.v[2], hi.v[3]}};
    Pack<4> m = mat_mul(ma, mb);
    return {{m.v[0], m.v[1], m.v[2], m.v[3], lo.v[4] + hi.v[4]}};
  }
};

template <int NT, int K>
struct Lds {
  static constexpr int T = NT * K;
  static constexpr int NW = NT / 64;
  static constexpr size_t bytes() {
    return sizeof(double) * (NW * 8 + 64 + 2 * WAKE_BCAP + T) + sizeof(int32_t) * 2 * T;
  }
};

// total sum_j w_j ln rho_j of the state in buffer `buf` (double-double)
template <int NT, int K>
__device__ dd total_wlnr(const WakeInst& I, int buf, double* s_scan) {
  constexpr int T = NT * K;
  dd acc = {0.0, 0.0};
  for (int base = threadIdx.x * K; base < I.N; base += T) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int p = base + k;
      if (p < I.N) {
        const int id = I.id[buf][p];
        acc = dd_add(acc, dd_mul_d(ring_log(I, id, I.rho[buf][p]), I.w[id]));
      }
    }
  }
  Pack<2> tot;
  block_prefix<NT, 2>(Pack<2>{{acc.hi, acc.lo}}, Pack<2>{{0.0, 0.0}},
                      [](const Pack<2>& a, const Pack<2>& b) {
                        dd s = dd_add({a.v[0], a.v[1]}, {b.v[0], b.v[1]});
                        return Pack<2>{{s.hi, s.lo}};
                      },
                      s_scan, tot);
  return {tot.v[0], tot.v[1]};
}

// one merge round over LDS keys: pairs of sorted runs of length `run`
// become runs of 2*run; thread t produces outputs [t*K, t*K+K).
template <int NT, int K>
__device__ __forceinline__ void lds_merge_round(double* kr, int32_t* ki, int32_t* kp, int run) {
  const int out0 = threadIdx.x * K;
  const int base = (out0 / (2 * run)) * (2 * run);
  const int d = out0 - base;
  const int A = base, B = base + run;
  const bool ordered = key_lt(kr[B - 1], ki[B - 1], kr[B], ki[B]);
  double orr[K];
  int32_t oi[K], op[K];
  if (!ordered) {
    int lo = d > run ? d - run : 0, hi = d < run ? d : run;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (key_lt(kr[A + mid], ki[A + mid], kr[B + d - 1 - mid], ki[B + d - 1 - mid])) lo = mid + 1;
      else hi = mid;
    }
    int i = lo, j = d - lo;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool takeA = i < run && (j >= run || key_lt(kr[A + i], ki[A + i], kr[B + j], ki[B + j]));
      const int s = takeA ? A + i : B + j;
      orr[k] = kr[s]; oi[k] = ki[s]; op[k] = kp[s];
      if (takeA) ++i; else ++j;
    }
  }
  __syncthreads();
  if (!ordered) {
#pragma unroll
    for (int k = 0; k < K; ++k) { kr[out0 + k] = orr[k]; ki[out0 + k] = oi[k]; kp[out0 + k] = op[k]; }
  }
  __syncthreads();
}

// Sort the T keys of one tile (positions [tb, tb+T) of buffer `src`,
// padded past N) in LDS.  On return kr/ki/kp hold the sorted tile.
template <int NT, int K>
__device__ void lds_sort_tile(const WakeInst& I, int src, int tb, double* kr, int32_t* ki, int32_t* kp) {
  constexpr int T = NT * K;
  double r[K];
  int32_t id[K], ps[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int p = tb + threadIdx.x * K + k;
    if (p < I.N) { r[k] = I.rho[src][p]; id[k] = I.id[src][p]; }
    else { r[k] = INFINITY; id[k] = I.N + p; }
    ps[k] = p;
  }
  // insertion sort of the thread's K keys
#pragma unroll
  for (int a = 1; a < K; ++a) {
#pragma unroll
    for (int b = a; b > 0; --b) {
      if (key_lt(r[b], id[b], r[b - 1], id[b - 1])) {
        double tr = r[b]; r[b] = r[b - 1]; r[b - 1] = tr;
        int32_t ti = id[b]; id[b] = id[b - 1]; id[b - 1] = ti;
        int32_t tp = ps[b]; ps[b] = ps[b - 1]; ps[b - 1] = tp;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    kr[threadIdx.x * K + k] = r[k]; ki[threadIdx.x * K + k] = id[k]; kp[threadIdx.x * K + k] = ps[k];
  }
  __syncthreads();
  for (int run = K; run < T; run <<= 1) lds_merge_round<NT, K>(kr, ki, kp, run);
}

// Merge two adjacent sorted runs [a0, a0+la) and [a0+la, a0+la+lb) of the
// global key arrays (src) into tmp, then copy back.
template <int NT, int K>
__device__ void global_merge_pair(double* kr, int32_t* ki, int32_t* kp, double* tr, int32_t* ti,
                                  int32_t* tp, int a0, int la, int lb) {
  constexpr int T = NT * K;
  const int L = la + lb;
  const int B = a0 + la;
  for (int c0 = 0; c0 < L; c0 += T) {
    const int d = c0 + threadIdx.x * K;
    if (d < L) {
      int lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key_lt(kr[a0 + mid], ki[a0 + mid], kr[B + d - 1 - mid], ki[B + d - 1 - mid])) lo = mid + 1;
        else hi = mid;
      }
      int i = lo, j = d - lo;
      for (int k = 0; k < K && d + k < L; ++k) {
        const bool takeA = i < la && (j >= lb || key_lt(kr[a0 + i], ki[a0 + i], kr[B + j], ki[B + j]));
        const int s = takeA ? a0 + i : B + j;
        tr[a0 + d + k] = kr[s]; ti[a0 + d + k] = ki[s]; tp[a0 + d + k] = kp[s];
        if (takeA) ++i; else ++j;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < L; i += NT) {
    kr[a0 + i] = tr[a0 + i]; ki[a0 + i] = ti[a0 + i]; kp[a0 + i] = tp[a0 + i];
  }
  __syncthreads();
}

// Reorder the state from buffer src into buffer dst by (rho, id).
template <int NT, int K>
__device__ void sort_state(const WakeInst& I, int src, int dst, double* kr, int32_t* ki, int32_t* kp) {
  constexpr int T = NT * K;
  const int N = I.N;
  const int ntiles = (N + T - 1) / T;
  if (ntiles == 1) {
    lds_sort_tile<NT, K>(I, src, 0, kr, ki, kp);
    for (int p = threadIdx.x; p < N; p += NT) {
      const int o = kp[p];
      I.rho[dst][p] = kr[p]; I.id[dst][p] = ki[p];
      I.u[dst][p] = I.u[src][o]; I.fr[dst][p] = I.fr[src][o]; I.fu[dst][p] = I.fu[src][o];
    }
    __syncthreads();
    return;
  }
  double* gr = I.skey_r[0]; int32_t* gi = I.skey_i[0]; int32_t* gp = I.skey_p[0];
  for (int tl = 0; tl < ntiles; ++tl) {
    lds_sort_tile<NT, K>(I, src, tl * T, kr, ki, kp);
    for (int i = threadIdx.x; i < T; i += NT) {
      const int p = tl * T + i;
      if (p < N) { gr[p] = kr[i]; gi[p] = ki[i]; gp[p] = kp[i]; }
    }
    __syncthreads();
  }
  // block odd-even transposition with merge-split of adjacent tiles
  for (;;) {
    bool changed = false;
    for (int par = 0; par < 2; ++par) {
      for (int j = par; j + 1 < ntiles; j += 2) {
        const int a0 = j * T;
        const int lb = min(T, N - (j + 1) * T);
        if (key_lt(gr[a0 + T], gi[a0 + T], gr[a0 + T - 1], gi[a0 + T - 1])) {
          global_merge_pair<NT, K>(gr, gi, gp, I.skey_r[1], I.skey_i[1], I.skey_p[1], a0, T, lb);
          changed = true;
        }
      }
      __syncthreads();
    }
    if (!changed) break;
  }
  for (int p = threadIdx.x; p < N; p += NT) {
    const int o = gp[p];
    I.rho[dst][p] = gr[p]; I.id[dst][p] = gi[p];
    I.u[dst][p] = I.u[src][o]; I.fr[dst][p] = I.fr[src][o]; I.fu[dst][p] = I.fu[src][o];
  }
  __syncthreads();
}

// Is buffer `buf` in (rho, id) order?  Uniform result.
template <int NT>
__device__ bool state_sorted(const WakeInst& I, int buf, double* s_scan) {
  double bad = 0.0;
  for (int p = threadIdx.x; p + 1 < I.N; p += NT)
    if (!key_lt(I.rho[buf][p], I.id[buf][p], I.rho[buf][p + 1], I.id[buf][p + 1])) bad = 1.0;
  Pack<1> tot;
  block_prefix<NT, 1>(Pack<1>{{bad}}, Pack<1>{{0.0}}, SumOp<1>(), s_scan, tot);
  return tot.v[0] == 0.0;
}

template <int NT, int K>
__device__ void march(const WakeInst& I, unsigned char* smem) {
  constexpr int T = NT * K;
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x;
  const int N = I.N;
  const int ntiles = (N + T - 1) / T;
  const bool multi = ntiles > 1;

  double* s_scan = reinterpret_cast<double*>(smem);  // NW*8
  double* s_misc = s_scan + NW * 8;                   // 64
  double* s_br = s_misc + 64;                         // BCAP
  double* s_bc = s_br + WAKE_BCAP;                    // BCAP
  double* s_kr = s_bc + WAKE_BCAP;                    // T
  int32_t* s_ki = reinterpret_cast<int32_t*>(s_kr + T);  // T
  int32_t* s_kp = s_ki + T;                              // T

  if (I.ctl[CTL_BREAK] >= 0) return;
  int cur = I.ctl[CTL_CUR];
  __syncthreads();
  // the state must start sorted (fresh rings are; injected states may not be)
  if (!state_sorted<NT>(I, cur, s_scan)) {
    sort_state<NT, K>(I, cur, 1 - cur, s_kr, s_ki, s_kp);
    cur = 1 - cur;
  }
  dd tot = total_wlnr<NT, K>(I, cur, s_scan);
  const dd tot0 = {I.tot0[0], I.tot0[1]};

  // per-ring registers of the current tile (resident across both passes
  // when the instance is one tile)
  double rho[K], u[K], w[K], wh[K], psi[K], dpsi[K], bb[K], g0[K], g1[K], e0[K], e1[K], a2[K],
      da2[K];
  int32_t id[K];
  Pack<4> Pch;   // this thread's transfer product for the tile
  double vch;    // this thread's sum of v for the tile

  for (int step = 0; step < I.count; ++step) {
    const int n = I.first + step;
    const double xi = n * I.dxi;
    const bool do_push = n < I.n_xi - 1;
    const bool rec_snap = I.stride > 0 && (n % I.stride) == 0;
    const bool rec_last = step == I.count - 1;
    const double psi_axis = dd_round(dd_sub(tot, tot0));
    const int nb = 1 - cur;

    // ---- stage this slice's beam table ----
    const int bt0 = I.nb ? I.boff[n] : 0;
    const int bm = I.nb ? I.boff[n + 1] - bt0 : 0;
    const bool staged = bm <= WAKE_BCAP;
    if (bm > 0 && staged) {
      for (int i = tid; i < bm; i += NT) { s_br[i] = I.br[bt0 + i]; s_bc[i] = I.bcum[bt0 + i]; }
    }
    __syncthreads();

    // ================= pass 1: forward over tiles =================
    dd cS = {0.0, 0.0}, cPT = {0.0, 0.0};
    double gc0 = 1.0, gc1 = 0.0;   // g at the start of the tile
    double cV = 0.0, cE0 = 0.0, cE1 = 0.0;
    double bad = 0.0;
    for (int tl = 0; tl < ntiles; ++tl) {
      const int base = tl * T + tid * K;
      dd lnr[K];
      dd sw = {0.0, 0.0}, swl = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int p = base + k;
        const bool ok = p < N;
        rho[k] = ok ? I.rho[cur][p] : 1.0;
        u[k] = ok ? I.u[cur][p] : 0.0;
        id[k] = ok ? I.id[cur][p] : -1;
        w[k] = ok ? I.w[id[k]] : 0.0;
        wh[k] = ok ? I.wh[id[k]] : 0.0;
        lnr[k] = ok ? ring_log(I, id[k], rho[k]) : dd{0.0, 0.0};
        sw = dd_add_d(sw, w[k]);
        swl = dd_add(swl, dd_mul_d(lnr[k], w[k]));
      }
      // ---- sources: beam charge within rho, laser envelope ----
      {
        int cnt[K];
#pragma unroll
        for (int k = 0; k < K; ++k) cnt[k] = 0;
        if (bm > 0) {
          if (staged) {
            int lo0 = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
              int lo = lo0, hi = bm;
              while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_br[mid] < rho[k]) lo = mid + 1; else hi = mid;
              }
              cnt[k] = lo;
              lo0 = (base + k < N) ? lo : lo0;
            }
          } else {
            for (int c0 = 0; c0 < bm; c0 += WAKE_BCAP) {
              const int cl = min(WAKE_BCAP, bm - c0);
              __syncthreads();
              for (int i = tid; i < cl; i += NT) s_br[i] = I.br[bt0 + c0 + i];
              __syncthreads();
#pragma unroll
              for (int k = 0; k < K; ++k) {
                if (s_br[0] < rho[k]) {
                  int lo = 0, hi = cl;
                  while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_br[mid] < rho[k]) lo = mid + 1; else hi = mid;
                  }
                  cnt[k] = c0 + lo;
                }
              }
            }
            __syncthreads();
          }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          double lam = 0.0;
          if (cnt[k] > 0) lam = staged ? s_bc[cnt[k] - 1] : I.bcum[bt0 + cnt[k] - 1];
          double aa = 0.0, dda = 0.0;
          for (int s = 0; s < I.n_an; ++s) {
            const WakeAnalytic& S = I.an[s];
            if (S.kind == 2) {
              const double s2 = S.sigma_r * S.sigma_r;
              const double dl = xi - S.xi_c;
              const double lon = exp(-(dl * dl) / (2.0 * S.sigma_xi * S.sigma_xi));
              lam += S.q * S.n_peak * lon * s2 * (-expm1(-rho[k] * rho[k] / (2.0 * s2)));
            } else {
              const double dl = xi - S.xi_l;
              const double lon = exp(-2.0 * dl * dl / (S.L * S.L));
              const double x = S.a0 * S.a0 * exp(-2.0 * rho[k] * rho[k] / (S.w0 * S.w0)) * lon;
              aa += x;
              dda += -(4.0 * rho[k] / (S.w0 * S.w0)) * x;
            }
          }
          bb[k] = lam / rho[k];
          a2[k] = aa;
          da2[k] = dda;
        }
      }
      // ---- Gauss/log sums (double-double prefix) ----
      Pack<4> t4;
      Pack<4> pre = block_prefix<NT, 4>(Pack<4>{{sw.hi, sw.lo, swl.hi, swl.lo}},
                                        Pack<4>{{0, 0, 0, 0}}, DD2Op(), s_scan, t4);
      dd S = dd_add(cS, {pre.v[0], pre.v[1]});
      dd PT = dd_add(cPT, {pre.v[2], pre.v[3]});
      cS = dd_add(cS, {t4.v[0], t4.v[1]});
      cPT = dd_add(cPT, {t4.v[2], t4.v[3]});
      Pch = mat_ident();
      vch = 0.0;
      double pbk[K], vk[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool ok = base + k < N;
        const dd PTi = dd_add(PT, dd_mul_d(lnr[k], w[k]));
        // electron psi - sum_j w_j ln rho_j and d_rho psi (self weight w^)
        const dd pe = dd_sub(dd_mul(dd_add_d(S, w[k]), lnr[k]), PTi);
        const dd de = dd_div_d(dd_add_d(S, wh[k]), rho[k]);
        dd ips, idp;
        if (ok) ion_fields(I, rho[k], lnr[k], ips, idp);
        else { ips = {0.0, 0.0}; idp = {0.0, 0.0}; }
        psi[k] = dd_round(dd_add(pe, ips)) + psi_axis;
        dpsi[k] = dd_round(dd_add(de, idp));
        S = dd_add_d(S, w[k]);
        PT = PTi;
        const double pb = 1.0 + psi[k];
        if (ok && !(pb > 0.0)) bad = 1.0;
        const double gm = gamma_of(u[k], pb, a2[k]);
        const double v = ok ? w[k] * u[k] / (rho[k] * pb) : 0.0;
        const double A = ok ? w[k] / (rho[k] * pb) : 0.0;
        pbk[k] = pb;
        vk[k] = v;
        Pch = mat_mul(rec_matrix(A, rho[k]), Pch);
        vch += v;
        (void)gm;
      }
      // ---- growing mode g (prefix product) and prefix of v ----
      Pack<5> t5;
      Pack<5> gp = block_prefix<NT, 5>(Pack<5>{{Pch.v[0], Pch.v[1], Pch.v[2], Pch.v[3], vch}},
                                       Pack<5>{{1.0, 0.0, 0.0, 1.0, 0.0}}, MatSumOp(), s_scan, t5);
      double ga = gp.v[0] * gc0 + gp.v[1] * gc1;
      double gb = gp.v[2] * gc0 + gp.v[3] * gc1;
      double V = cV + gp.v[4];
      {
        const double na = t5.v[0] * gc0 + t5.v[1] * gc1;
        const double nbv = t5.v[2] * gc0 + t5.v[3] * gc1;
        gc0 = na; gc1 = nbv;
        cV += t5.v[4];
      }
      double le0 = 0.0, le1 = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool ok = base + k < N;
        g0[k] = ga; g1[k] = gb;   // g_{i-1}
        const double pb = pbk[k];
        const double A = ok ? w[k] / (rho[k] * pb) : 0.0;
        const Pack<4> M = rec_matrix(A, rho[k]);
        const double na = M.v[0] * ga + M.v[1] * gb;
        const double nbv = M.v[2] * ga + M.v[3] * gb;
        ga = na; gb = nbv;        // g_i
        V += vk[k];
        double x0 = 0.0, x1 = 0.0;
        if (ok) {
          const double gm = gamma_of(u[k], pb, a2[k]);
          const double c = 1.0 - wh[k] / w[k];
          const double dz0 = V - c * vk[k];     // d_zeta psi + V_total
          double Aa, B0, C;
          ring_coeffs(rho[k], u[k], w[k], pb, gm, dpsi[k], dz0, bb[k], da2[k], Aa, B0, C);
          const double B1 = (w[k] / rho[k]) * u[k] / (pb * pb);
          double s0a, s0b;
          rec_offset(Aa, B0, C, rho[k], s0a, s0b);
          const double s1a = 0.5 * B1, s1b = -0.5 * rho[k] * rho[k] * B1;
          x0 = ga * s0b - gb * s0a;   // det[g_i, s0_i]
          x1 = ga * s1b - gb * s1a;   // det[g_i, s1_i]
        }
        e0[k] = x0; e1[k] = x1;
        le0 += x0; le1 += x1;
      }
      Pack<2> t2;
      Pack<2> ep = block_prefix<NT, 2>(Pack<2>{{le0, le1}}, Pack<2>{{0.0, 0.0}}, SumOp<2>(), s_scan, t2);
      double E0 = cE0 + ep.v[0], E1 = cE1 + ep.v[1];
      cE0 += t2.v[0]; cE1 += t2.v[1];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double x0 = e0[k], x1 = e1[k];
        e0[k] = E0; e1[k] = E1;   // exclusive: E_{i-1}
        E0 += x0; E1 += x1;
      }
      if (multi) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int p = base + k;
          if (p < N) {
            I.scr[SC_PSI * N + p] = psi[k]; I.scr[SC_DPSI * N + p] = dpsi[k];
            I.scr[SC_BB * N + p] = bb[k];
            I.scr[SC_G0 * N + p] = g0[k]; I.scr[SC_G1 * N + p] = g1[k];
            I.scr[SC_E0 * N + p] = e0[k]; I.scr[SC_E1 * N + p] = e1[k];
            if (I.has_laser) { I.scr[SC_A2 * N + p] = a2[k]; I.scr[SC_DA2 * N + p] = da2[k]; }
          }
        }
        double* ts = I.tscr + ((size_t)tl * NT + tid) * 5;
        ts[0] = Pch.v[0]; ts[1] = Pch.v[1]; ts[2] = Pch.v[2]; ts[3] = Pch.v[3]; ts[4] = vch;
      }
    }
    const double Vtot = cV;
    const double W = gc0;   // det[g_N, h_N] with h_N = (0, 1)
    const double iW = 1.0 / W;

    // ================= pass 2: backward over tiles =================
    double hc0 = 0.0, hc1 = 1.0;   // h at the end of the tile
    double cVs = 0.0, cD = 0.0;
    dd swl_next = {0.0, 0.0};
    double disorder = 0.0;
    double nxt_r = INFINITY;       // first ring of the following tile (new radius)
    int32_t nxt_i = 0x7fffffff;
    for (int tl = ntiles - 1; tl >= 0; --tl) {
      const int base = tl * T + tid * K;
      if (multi) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int p = base + k;
          const bool ok = p < N;
          rho[k] = ok ? I.rho[cur][p] : 1.0;
          u[k] = ok ? I.u[cur][p] : 0.0;
          id[k] = ok ? I.id[cur][p] : -1;
          w[k] = ok ? I.w[id[k]] : 0.0;
          wh[k] = ok ? I.wh[id[k]] : 0.0;
          psi[k] = ok ? I.scr[SC_PSI * N + p] : 0.0;
          dpsi[k] = ok ? I.scr[SC_DPSI * N + p] : 0.0;
          bb[k] = ok ? I.scr[SC_BB * N + p] : 0.0;
          g0[k] = ok ? I.scr[SC_G0 * N + p] : 0.0;
          g1[k] = ok ? I.scr[SC_G1 * N + p] : 0.0;
          e0[k] = ok ? I.scr[SC_E0 * N + p] : 0.0;
          e1[k] = ok ? I.scr[SC_E1 * N + p] : 0.0;
          a2[k] = (ok && I.has_laser) ? I.scr[SC_A2 * N + p] : 0.0;
          da2[k] = (ok && I.has_laser) ? I.scr[SC_DA2 * N + p] : 0.0;
        }
        const double* ts = I.tscr + ((size_t)tl * NT + tid) * 5;
        Pch = {{ts[0], ts[1], ts[2], ts[3]}};
        vch = ts[4];
      }
      // decaying mode h: suffix of the inverse transfers (det M = 1, so the
      // inverse of the thread's product is its adjugate)
      Pack<5> t5;
      Pack<5> hs = block_suffix<NT, 5>(
          Pack<5>{{Pch.v[3], -Pch.v[1], -Pch.v[2], Pch.v[0], vch}}, Pack<5>{{1.0, 0.0, 0.0, 1.0, 0.0}},
          BwdMatSumOp(), s_scan, t5);
      double ha = hs.v[0] * hc0 + hs.v[1] * hc1;
      double hb = hs.v[2] * hc0 + hs.v[3] * hc1;
      double Vgt = cVs + hs.v[4];
      {
        const double na = t5.v[0] * hc0 + t5.v[1] * hc1;
        const double nbv = t5.v[2] * hc0 + t5.v[3] * hc1;
        hc0 = na; hc1 = nbv;
        cVs += t5.v[4];
      }
      double hp0[K], hp1[K], dzk[K], Ck[K], ds[K];
      double lds = 0.0;
#pragma unroll
      for (int k = K - 1; k >= 0; --k) {
        const bool ok = base + k < N;
        const double pb = 1.0 + psi[k];
        const double gm = gamma_of(u[k], pb, a2[k]);
        const double v = ok ? w[k] * u[k] / (rho[k] * pb) : 0.0;
        const double A = ok ? w[k] / (rho[k] * pb) : 0.0;
        const double hh = 0.5 * A * rho[k];
        // h_{i-1} = M_i^{-1} h_i
        const double na = (1.0 - hh) * ha - (A / (2.0 * rho[k])) * hb;
        const double nbv = (hh * rho[k] * rho[k]) * ha + (1.0 + hh) * hb;
        double dz = 0.0, C = 0.0, x = 0.0;
        if (ok) {
          const double c = 1.0 - wh[k] / w[k];
          dz = -(Vgt + c * v);
          double Aa, B;
          ring_coeffs(rho[k], u[k], w[k], pb, gm, dpsi[k], dz, bb[k], da2[k], Aa, B, C);
          double sa, sb;
          rec_offset(Aa, B, C, rho[k], sa, sb);
          x = sa * hb - sb * ha;   // det[s_i, h_i]
        }
        Vgt += v;
        hp0[k] = na; hp1[k] = nbv;
        dzk[k] = dz; Ck[k] = C; ds[k] = x;
        lds += x;
        ha = na; hb = nbv;
      }
      Pack<1> t1;
      Pack<1> dsf = block_suffix<NT, 1>(Pack<1>{{lds}}, Pack<1>{{0.0}}, SumOp<1>(), s_scan, t1);
      double D = cD + dsf.v[0];
      cD += t1.v[0];
      double nr[K];
#pragma unroll
      for (int k = K - 1; k >= 0; --k) {
        const int p = base + k;
        const bool ok = p < N;
        D += ds[k];                               // D_{i-1} = sum_{k>=i} det[s_k, h_k]
        const double E = e0[k] + Vtot * e1[k];    // E_{i-1}
        const double a = (hp0[k] * E - g0[k] * D) * iW;
        const double b = (hp1[k] * E - g1[k] * D) * iW;
        nr[k] = INFINITY;
        if (!ok) continue;
        const double bp = a * rho[k] + b / rho[k] + (wh[k] / w[k]) * Ck[k];
        const double bt = bb[k] + bp;
        const double ez = -dzk[k];
        if (!(isfinite(psi[k]) && isfinite(dpsi[k]) && isfinite(ez) && isfinite(bt))) bad = 1.0;
        if (rec_snap) {
          double* sp = I.snap + (size_t)(n / I.stride) * OUT_N * N;
          sp[OUT_PSI * N + id[k]] = psi[k]; sp[OUT_ERBT * N + id[k]] = -dpsi[k];
          sp[OUT_EZ * N + id[k]] = ez; sp[OUT_BT * N + id[k]] = bt;
          sp[OUT_RHO * N + id[k]] = rho[k]; sp[OUT_UR * N + id[k]] = u[k];
        }
        if (rec_last) {
          double* sp = I.last;
          sp[OUT_PSI * N + id[k]] = psi[k]; sp[OUT_ERBT * N + id[k]] = -dpsi[k];
          sp[OUT_EZ * N + id[k]] = ez; sp[OUT_BT * N + id[k]] = bt;
          sp[OUT_RHO * N + id[k]] = rho[k]; sp[OUT_UR * N + id[k]] = u[k];
        }
        if (do_push) {
          const double pb = 1.0 + psi[k];
          const double gm = gamma_of(u[k], pb, a2[k]);
          const double f_r = u[k] / pb;
          const double f_u = gm * dpsi[k] / pb - bt - 0.25 * da2[k] / pb;
          double pr = f_r, pu = f_u;
          if (n > 0) { pr = I.fr[cur][p]; pu = I.fu[cur][p]; }
          double rn = rho[k] + I.dxi * (1.5 * f_r - 0.5 * pr);
          double un = u[k] + I.dxi * (1.5 * f_u - 0.5 * pu);
          double sr = f_r, su = f_u;
          if (rn < 0.0) { rn = -rn; un = -un; sr = -sr; su = -su; }
          if (!(isfinite(rn) && isfinite(un))) bad = 1.0;
          I.rho[nb][p] = rn; I.u[nb][p] = un; I.fr[nb][p] = sr; I.fu[nb][p] = su;
          I.id[nb][p] = id[k];
          nr[k] = rn;
          swl_next = dd_add(swl_next, dd_mul_d(ring_log(I, id[k], rn), w[k]));
        }
      }
      if (do_push) {
        // disorder of the pushed radii, within the thread and across neighbours
        double fr0 = INFINITY, lr0 = INFINITY;
        int32_t fi0 = 0x7fffffff, li0 = 0x7fffffff;
        bool have = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (base + k >= N) continue;
          if (have && !key_lt(lr0, li0, nr[k], id[k])) disorder = 1.0;
          if (!have) { fr0 = nr[k]; fi0 = id[k]; }
          lr0 = nr[k]; li0 = id[k]; have = true;
        }
        __syncthreads();
        s_kr[tid] = fr0; s_ki[tid] = fi0;
        __syncthreads();
        if (have) {
          const double nxr = tid + 1 < NT ? s_kr[tid + 1] : nxt_r;
          const int32_t nxi = tid + 1 < NT ? s_ki[tid + 1] : nxt_i;
          const bool next_valid = tid + 1 < NT ? (base + K < N) : (tl + 1 < ntiles);
          if (next_valid && !key_lt(lr0, li0, nxr, nxi)) disorder = 1.0;
        }
        nxt_r = s_kr[0]; nxt_i = s_ki[0];
        __syncthreads();
      }
    }
    // ---- slice reduction: next total, breakdown, disorder ----
    Pack<4> red;
    block_prefix<NT, 4>(Pack<4>{{swl_next.hi, swl_next.lo, bad, disorder}}, Pack<4>{{0, 0, 0, 0}},
                        [](const Pack<4>& a, const Pack<4>& b) {
                          dd s = dd_add({a.v[0], a.v[1]}, {b.v[0], b.v[1]});
                          return Pack<4>{{s.hi, s.lo, a.v[2] + b.v[2], a.v[3] + b.v[3]}};
                        },
                        s_scan, red);
    if (tid == 0) { I.axis[2 * n] = psi_axis; I.axis[2 * n + 1] = Vtot; }
    if (red.v[2] != 0.0) {
      if (tid == 0) { I.ctl[CTL_BREAK] = n; I.ctl[CTL_CUR] = cur; I.ctl[CTL_NEXT] = n; }
      return;
    }
    if (!do_push) {
      if (tid == 0) { I.ctl[CTL_CUR] = cur; I.ctl[CTL_NEXT] = n + 1; }
      return;   // last slice of the window: nothing left to march
    }
    if (red.v[3] != 0.0) {
      sort_state<NT, K>(I, nb, cur, s_kr, s_ki, s_kp);   // cur stays the same buffer
    } else {
      cur = nb;
    }
    tot = {red.v[0], red.v[1]};
    __syncthreads();
  }
  if (tid == 0) { I.ctl[CTL_CUR] = cur; I.ctl[CTL_NEXT] = I.first + I.count; }
}

template <int NT, int K>
__global__ __launch_bounds__(NT) void wake_march_kernel(const WakeInst* __restrict__ insts, int n_insts,
                                                        int32_t* counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_idx;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= n_insts) return;   // every workgroup leaves once the queue is empty
    march<NT, K>(insts[idx], smem);
    __syncthreads();
  }
}

__global__ void wake_zero_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// By-id copies of the sorted state (for wake_get_state)
__global__ void state_by_id_kernel(WakeInst I, double* rho, double* u, double* fr, double* fu) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= I.N) return;
  const int c = I.ctl[CTL_CUR];
  const int i = I.id[c][p];
  if (rho) rho[i] = I.rho[c][p];
  if (u) u[i] = I.u[c][p];
  if (fr) fr[i] = I.fr[c][p];
  if (fu) fu[i] = I.fu[c][p];
}

// Injected state (by id) written in id order into buffer 0; the marcher
// sorts it before its first slice.
__global__ void state_set_kernel(WakeInst I, const double* rho, const double* u, const double* fr,
                                 const double* fu, int slice) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) { I.ctl[CTL_CUR] = 0; I.ctl[CTL_BREAK] = -1; I.ctl[CTL_NEXT] = slice; }
  if (i >= I.N) return;
  I.rho[0][i] = rho[i];
  I.u[0][i] = u[i];
  I.fr[0][i] = fr ? fr[i] : 0.0;
  I.fu[0][i] = fu ? fu[i] : 0.0;
  I.id[0][i] = i;
}

// Back to the state at slice 0 (rings at rest at their initial radii);
// one workgroup per instance.
__global__ void state_reset_kernel(const WakeInst* __restrict__ insts, int n_insts) {
  const WakeInst& I = insts[blockIdx.x];
  for (int j = threadIdx.x; j < I.N; j += blockDim.x) {
    I.rho[0][j] = I.ion_r[j + 1];
    I.u[0][j] = 0.0;
    I.fr[0][j] = 0.0;
    I.fu[0][j] = 0.0;
    I.id[0][j] = j;
  }
  if (threadIdx.x == 0) { I.ctl[CTL_CUR] = 0; I.ctl[CTL_BREAK] = -1; I.ctl[CTL_NEXT] = 0; }
}

// ---------------------------------------------------------------------------
// host-callable launchers (used by wake_api.cpp)
// ---------------------------------------------------------------------------
#include "wake_launch.h"

hipError_t launch_init(const WakeInst& I, const double* r0, const double* dr, const double* dens,
                       hipStream_t s) {
  hipLaunchKernelGGL((wake_init_kernel<256>), dim3(1), dim3(256), 0, s, I, r0, dr, dens);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = (I.lut_n + 1 + 255) / 256;
  hipLaunchKernelGGL(wake_lut_kernel, dim3(nb), dim3(256), 0, s, I);
  return hipGetLastError();
}

hipError_t launch_beam_table(const double* x, const double* y, const double* xi, const double* w,
                             const double* q, int64_t np, double dxi, int n_xi, int32_t* cnt,
                             int32_t* cnt2, int32_t* cursor, int32_t* off, int32_t* poff, double* er,
                             double* eq, int64_t* ek, double* br, double* bcum, hipStream_t s) {
  BeamParts P = {x, y, xi, w, q, np};
  const int zb = (n_xi + 1 + 255) / 256;
  hipLaunchKernelGGL(wake_zero_kernel, dim3(zb), dim3(256), 0, s, cnt, n_xi + 1);
  hipLaunchKernelGGL(wake_zero_kernel, dim3(zb), dim3(256), 0, s, cursor, n_xi + 1);
  const int pb = (int)((np + 255) / 256);
  if (np > 0) hipLaunchKernelGGL(beam_count_kernel, dim3(pb), dim3(256), 0, s, P, dxi, n_xi, cnt);
  hipLaunchKernelGGL(pow2_kernel, dim3(zb), dim3(256), 0, s, cnt, n_xi, cnt2);
  hipLaunchKernelGGL((exclusive_scan_kernel<1024>), dim3(1), dim3(1024), 0, s, cnt, n_xi, off);
  hipLaunchKernelGGL((exclusive_scan_kernel<1024>), dim3(1), dim3(1024), 0, s, cnt2, n_xi, poff);
  if (np > 0)
    hipLaunchKernelGGL(beam_scatter_kernel, dim3(pb), dim3(256), 0, s, P, dxi, n_xi, poff, cursor, er,
                       eq, ek);
  hipLaunchKernelGGL((beam_sort_kernel<256>), dim3(n_xi), dim3(256), 0, s, off, poff, er, eq, ek,
                     1.0 / (2.0 * M_PI * dxi), br, bcum);
  return hipGetLastError();
}

hipError_t launch_reset(const WakeInst* d_insts, int n_insts, hipStream_t s) {
  if (n_insts <= 0) return hipSuccess;
  hipLaunchKernelGGL(state_reset_kernel, dim3(n_insts), dim3(256), 0, s, d_insts, n_insts);
  return hipGetLastError();
}

hipError_t launch_zero(int32_t* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(wake_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
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

template <int NT, int K>
static hipError_t launch_march_t(const WakeInst* d_insts, int n_insts, int32_t* counter, int grid,
                                 hipStream_t s) {
  const size_t lds = Lds<NT, K>::bytes();
  hipLaunchKernelGGL(wake_zero_kernel, dim3(1), dim3(64), 0, s, counter, 1);
  hipLaunchKernelGGL((wake_march_kernel<NT, K>), dim3(grid), dim3(NT), lds, s, d_insts, n_insts,
                     counter);
  return hipGetLastError();
}

template <int NT, int K>
static int occupancy_t() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, wake_march_kernel<NT, K>, NT,
                                                   Lds<NT, K>::bytes()) != hipSuccess)
    return 0;
  return nb;
}

template <int NT, int K>
static hipError_t set_lds_attr_t() {
  return hipFuncSetAttribute((const void*)wake_march_kernel<NT, K>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)Lds<NT, K>::bytes());
}

#define WAKE_CONFIGS(X) X(256, 2) X(256, 4) X(256, 8) X(512, 2) X(512, 4) X(1024, 2)

int march_config_count() {
  int n = 0;
#define X(a, b) ++n;
  WAKE_CONFIGS(X)
#undef X
  return n;
}

int march_config(int idx, int* nt, int* k) {
  int i = 0;
#define X(a, b) \
  if (i++ == idx) { *nt = a; *k = b; return 0; }
  WAKE_CONFIGS(X)
#undef X
  return -1;
}

hipError_t launch_march(int nt, int k, const WakeInst* d_insts, int n_insts, int32_t* counter, int grid,
                        hipStream_t s) {
#define X(a, b) \
  if (nt == a && k == b) return launch_march_t<a, b>(d_insts, n_insts, counter, grid, s);
  WAKE_CONFIGS(X)
#undef X
  return hipErrorInvalidValue;
}

int march_occupancy(int nt, int k) {
#define X(a, b) \
  if (nt == a && k == b) return occupancy_t<a, b>();
  WAKE_CONFIGS(X)
#undef X
  return 0;
}

hipError_t march_prepare(int nt, int k) {
#define X(a, b) \
  if (nt == a && k == b) return set_lds_attr_t<a, b>();
  WAKE_CONFIGS(X)
#undef X
  return hipErrorInvalidValue;
}
