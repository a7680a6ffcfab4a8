// Device-side building blocks for the gfx950 ring solver: double-double
// arithmetic, 64-wide wavefront and workgroup scans, and ring-key order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// ---------------------------------------------------------------------------
// double-double (unevaluated sum hi + lo) arithmetic.  Contraction of a
// multiply into an addition is forbidden inside every helper: after
// inlining, `a + b` in two_sum would otherwise fuse with a caller's product
// b = x*y into fma(x, y, a), and the error term would no longer describe the
// rounded sum.  The product error uses an explicit fma.
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd dd_make(double a) { return {a, 0.0}; }

__device__ __forceinline__ dd two_sum(double a, double b) {
  _Pragma("clang fp contract(off)")
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  _Pragma("clang fp contract(off)")
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
  _Pragma("clang fp contract(off)")
  double p = a * b;
  double e = __builtin_fma(a, b, -p);
  return {p, e};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
  _Pragma("clang fp contract(off)")
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

__device__ __forceinline__ dd dd_add_d(dd a, double b) {
  _Pragma("clang fp contract(off)")
  dd s = two_sum(a.hi, b);
  s.lo += a.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  _Pragma("clang fp contract(off)")
  dd p = two_prod(a.hi, b);
  p.lo = __builtin_fma(a.lo, b, p.lo);
  return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd dd_div_d(dd a, double b) {
  _Pragma("clang fp contract(off)")
  double q1 = a.hi / b;
  dd r = dd_sub(a, two_prod(q1, b));
  double q2 = r.hi / b;
  return fast_two_sum(q1, q2);
}

__device__ __forceinline__ double dd_round(dd a) {
  _Pragma("clang fp contract(off)") return a.hi + a.lo; }

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  _Pragma("clang fp contract(off)")
  dd p = two_prod(a.hi, b.hi);
  p.lo = __builtin_fma(a.hi, b.lo, __builtin_fma(a.lo, b.hi, p.lo));
  return fast_two_sum(p.hi, p.lo);
}

// exp(x) to double-double accuracy (|x| < 700): x = k ln2 + t with
// |t| <= ln2/2, Taylor series of e^t in double-double, scaled by 2^k.
__device__ inline dd dd_exp(double x) {
  _Pragma("clang fp contract(off)")
  const dd LN2 = {6.93147180559945286227e-01, 2.31904681384629955842e-17};
  const double kf = rint(x / LN2.hi);
  const dd t = dd_sub(dd_make(x), dd_mul_d(LN2, kf));
  dd term = {1.0, 0.0}, sum = {1.0, 0.0};
  for (int n = 1; n <= 27; ++n) {
    term = dd_div_d(dd_mul(term, t), (double)n);
    sum = dd_add(sum, term);
  }
  const int k = (int)kf;
  return {ldexp(sum.hi, k), ldexp(sum.lo, k)};
}

// ln(r) to double-double accuracy for r > 0: one Newton step on e^y = r
// from the binary64 logarithm.
__device__ inline dd dd_log(double r) {
  _Pragma("clang fp contract(off)")
  const double y = log(r);
  const dd e = dd_exp(y);
  const dd d = dd_sub(dd_make(r), e);
  return two_sum(y, d.hi / e.hi);
}

// ---------------------------------------------------------------------------
// packs of doubles moved through cross-lane shuffles and LDS
// ---------------------------------------------------------------------------
template <int NF>
struct Pack {
  double v[NF];
};

template <int NF>
__device__ __forceinline__ Pack<NF> shfl_up_pack(const Pack<NF>& p, int d) {
  Pack<NF> r;
#pragma unroll
  for (int i = 0; i < NF; ++i) r.v[i] = __shfl_up(p.v[i], d, 64);
  return r;
}

template <int NF>
__device__ __forceinline__ Pack<NF> shfl_down_pack(const Pack<NF>& p, int d) {
  Pack<NF> r;
#pragma unroll
  for (int i = 0; i < NF; ++i) r.v[i] = __shfl_down(p.v[i], d, 64);
  return r;
}

// Exclusive prefix over the workgroup in thread order.  op(earlier, later)
// must be associative; ident must satisfy op(ident, x) == x exactly.
// `lds` holds NT/64 packs.  Every thread also receives the total.  With
// TAIL = false the closing barrier is left out: the caller must not write
// `lds` again before another barrier has been passed by every thread.
template <int NT, int NF, class Op, bool TAIL = true>
__device__ __forceinline__ Pack<NF> block_prefix(const Pack<NF>& x, const Pack<NF>& ident, Op op,
                                                 double* lds, Pack<NF>& total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  Pack<NF> inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    Pack<NF> o = shfl_up_pack(inc, d);
    if (lane >= d) inc = op(o, inc);
  }
  Pack<NF> ex = shfl_up_pack(inc, 1);
  if (lane == 0) ex = ident;
  if (lane == 63) {
#pragma unroll
    for (int i = 0; i < NF; ++i) lds[wv * NF + i] = inc.v[i];
  }
  __syncthreads();
  Pack<NF> pre = ident, tot;
  #pragma unroll 1
  for (int w = 0; w < NW; ++w) {
    Pack<NF> s;
#pragma unroll
    for (int i = 0; i < NF; ++i) s.v[i] = lds[w * NF + i];
    if (w < wv) pre = op(pre, s);
    tot = (w == 0) ? s : op(tot, s);
  }
  if (TAIL) __syncthreads();
  total = tot;
  return op(pre, ex);
}

// Exclusive suffix over the workgroup: result for thread t combines the
// elements of threads t+1 .. NT-1 in thread order, op(lower, higher).
template <int NT, int NF, class Op>
__device__ __forceinline__ Pack<NF> block_suffix(const Pack<NF>& x, const Pack<NF>& ident, Op op,
                                                 double* lds, Pack<NF>& total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  Pack<NF> inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    Pack<NF> o = shfl_down_pack(inc, d);
    if (lane + d < 64) inc = op(inc, o);
  }
  Pack<NF> ex = shfl_down_pack(inc, 1);
  if (lane == 63) ex = ident;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NF; ++i) lds[wv * NF + i] = inc.v[i];
  }
  __syncthreads();
  Pack<NF> suf = ident, tot;
  #pragma unroll 1
  for (int w = NW - 1; w >= 0; --w) {
    Pack<NF> s;
#pragma unroll
    for (int i = 0; i < NF; ++i) s.v[i] = lds[w * NF + i];
    if (w > wv) suf = op(s, suf);
    tot = (w == NW - 1) ? s : op(s, tot);
  }
  __syncthreads();
  total = tot;
  return op(ex, suf);
}

// A prefix (in thread order, opP(earlier, later)) of xp and a suffix
// (opS(lower, higher)) of xs in one pass: one pair of barriers for both.
// `lds` holds NT/64 * (NP + NS) doubles.  TAIL as for block_prefix.
template <int NT, int NP, int NS, class OpP, class OpS, bool TAIL = true>
__device__ __forceinline__ void block_prefix_suffix(const Pack<NP>& xp, const Pack<NP>& idP, OpP opP,
                                                    const Pack<NS>& xs, const Pack<NS>& idS, OpS opS,
                                                    double* lds, Pack<NP>& exP, Pack<NP>& totP,
                                                    Pack<NS>& exS, Pack<NS>& totS) {
  constexpr int NW = NT / 64;
  constexpr int NF = NP + NS;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  Pack<NP> ip = xp;
  Pack<NS> is = xs;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    Pack<NP> o = shfl_up_pack(ip, d);
    Pack<NS> q = shfl_down_pack(is, d);
    if (lane >= d) ip = opP(o, ip);
    if (lane + d < 64) is = opS(is, q);
  }
  Pack<NP> ep = shfl_up_pack(ip, 1);
  Pack<NS> es = shfl_down_pack(is, 1);
  if (lane == 0) ep = idP;
  if (lane == 63) es = idS;
  if (lane == 63) {
#pragma unroll
    for (int i = 0; i < NP; ++i) lds[wv * NF + i] = ip.v[i];
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NS; ++i) lds[wv * NF + NP + i] = is.v[i];
  }
  __syncthreads();
  Pack<NP> pre = idP, tp;
  Pack<NS> suf = idS, ts;
  #pragma unroll 1
  for (int w = 0; w < NW; ++w) {
    Pack<NP> a;
#pragma unroll
    for (int i = 0; i < NP; ++i) a.v[i] = lds[w * NF + i];
    if (w < wv) pre = opP(pre, a);
    tp = (w == 0) ? a : opP(tp, a);
  }
  #pragma unroll 1
  for (int w = NW - 1; w >= 0; --w) {
    Pack<NS> a;
#pragma unroll
    for (int i = 0; i < NS; ++i) a.v[i] = lds[w * NF + NP + i];
    if (w > wv) suf = opS(a, suf);
    ts = (w == NW - 1) ? a : opS(a, ts);
  }
  if (TAIL) __syncthreads();
  exP = opP(pre, ep);
  totP = tp;
  exS = opS(es, suf);
  totS = ts;
}

// sums of packs (commutative), used with the scans above
template <int NF>
struct SumOp {
  __device__ __forceinline__ Pack<NF> operator()(const Pack<NF>& a, const Pack<NF>& b) const {
    Pack<NF> r;
#pragma unroll
    for (int i = 0; i < NF; ++i) r.v[i] = a.v[i] + b.v[i];
    return r;
  }
};

// pairs of double-doubles: (hi0, lo0, hi1, lo1)
struct DD2Op {
  __device__ __forceinline__ Pack<4> operator()(const Pack<4>& a, const Pack<4>& b) const {
    dd x = dd_add({a.v[0], a.v[1]}, {b.v[0], b.v[1]});
    dd y = dd_add({a.v[2], a.v[3]}, {b.v[2], b.v[3]});
    return {{x.hi, x.lo, y.hi, y.lo}};
  }
};

// 2x2 matrices stored (m00, m01, m10, m11).
__device__ __forceinline__ Pack<4> mat_mul(const Pack<4>& a, const Pack<4>& b) {
  return {{a.v[0] * b.v[0] + a.v[1] * b.v[2], a.v[0] * b.v[1] + a.v[1] * b.v[3],
           a.v[2] * b.v[0] + a.v[3] * b.v[2], a.v[2] * b.v[1] + a.v[3] * b.v[3]}};
}

// forward transfer: earlier applied first -> later * earlier
struct FwdMatOp {
  __device__ __forceinline__ Pack<4> operator()(const Pack<4>& earlier, const Pack<4>& later) const {
    return mat_mul(later, earlier);
  }
};

// backward transfer in index order: lower applied last -> lower * higher
struct BwdMatOp {
  __device__ __forceinline__ Pack<4> operator()(const Pack<4>& lower, const Pack<4>& higher) const {
    return mat_mul(lower, higher);
  }
};

__device__ __forceinline__ Pack<4> mat_ident() { return {{1.0, 0.0, 0.0, 1.0}}; }

// ---------------------------------------------------------------------------
// ring order: radius, then ring id
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool key_lt(double ra, int32_t ia, double rb, int32_t ib) {
  return ra < rb || (ra == rb && ia < ib);
}
