// Device-side building blocks for the gfx950 ring solver: double-double
// arithmetic, 64-wide wavefront and workgroup scans, and ring-key order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// The workgroup's dynamic LDS, named once so that code reached through a
// call (not only the kernel itself) addresses it as LDS rather than through
// flat pointers.
extern __shared__ __align__(16) unsigned char wake_lds[];

#define WAKE_GLOBAL __attribute__((address_space(1)))
// A device array's pointer in the global address space (64-bit indexing), so
// that its accesses take global rather than flat instructions (a flat access
// waits for both the memory and the LDS counters).
template <class T>
__device__ __forceinline__ WAKE_GLOBAL T* gptr(T* q) {
  return reinterpret_cast<WAKE_GLOBAL T*>(reinterpret_cast<uint64_t>(q));
}
// An object in device memory handed to a function that is not inlined, typed
// so that the callee reads it with global instructions.
template <class T>
__device__ __forceinline__ const WAKE_GLOBAL T* as_global(const T& x) {
  return (const WAKE_GLOBAL T*)&x;
}

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

// Sum with one two_sum of the high parts and the low parts added in
// double: the error stays within a few units of 2^-104 (|a| + |b|), which
// is all the field sums need (they end rounded to double).
__device__ __forceinline__ dd dd_add_fast(dd a, dd b) {
  _Pragma("clang fp contract(off)")
  dd s = two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return fast_two_sum(s.hi, s.lo);
}

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (e = 1 - x r, r += r e): within about an ulp of the rounded quotient,
// without the IEEE division sequence.  x = 0 or +-inf give NaN.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
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

// ln(1 + d) for d > -1 in a few dozen operations, to a few ulp:
// 1 + d = m + c exactly (two_sum), m = 2^k f with f in [sqrt(1/2), sqrt(2)),
// ln f = 2 atanh(s) with s = (f - 1) / (f + 1) (|s| < 0.172) summed by its
// Taylor series through s^25 (the next term is below 2^-64 of the sum), and
// ln(1 + d) = k ln 2 + ln f + c / m.  m <= 0 gives NaN.
__device__ __forceinline__ double log1p_fast(double d) {
  _Pragma("clang fp contract(off)")
  if (fabs(d) < 0.03125) {
    // small steps (the push's common case): 2 atanh(s), s = d / (2 + d),
    // without the range reduction; |s| < 0.016, so the series' first
    // omitted term, 2 s z^5 / 11, is below 1e-19 of the result
    const double s = d * rcp_nr(2.0 + d);
    const double z = s * s;
    double p = 1.0 / 9.0;
    p = __builtin_fma(p, z, 1.0 / 7.0);
    p = __builtin_fma(p, z, 1.0 / 5.0);
    p = __builtin_fma(p, z, 1.0 / 3.0);
    const double two_s = s + s;
    return __builtin_fma(two_s * z, p, two_s);
  }
  const dd mc = two_sum(1.0, d);
  const double m = mc.hi;
  int k = __builtin_amdgcn_frexp_exp(m);
  double f = __builtin_amdgcn_frexp_mant(m);            // [0.5, 1)
  if (f < 0.70710678118654752440) { f = f + f; k -= 1; }
  const double s = (f - 1.0) * rcp_nr(f + 1.0);
  const double z = s * s;
  double p = 1.0 / 25.0;
  p = __builtin_fma(p, z, 1.0 / 23.0);
  p = __builtin_fma(p, z, 1.0 / 21.0);
  p = __builtin_fma(p, z, 1.0 / 19.0);
  p = __builtin_fma(p, z, 1.0 / 17.0);
  p = __builtin_fma(p, z, 1.0 / 15.0);
  p = __builtin_fma(p, z, 1.0 / 13.0);
  p = __builtin_fma(p, z, 1.0 / 11.0);
  p = __builtin_fma(p, z, 1.0 / 9.0);
  p = __builtin_fma(p, z, 1.0 / 7.0);
  p = __builtin_fma(p, z, 1.0 / 5.0);
  p = __builtin_fma(p, z, 1.0 / 3.0);
  const double two_s = s + s;
  const double lf = __builtin_fma(two_s * z, p, two_s);     // 2 s (1 + z p)
  const double LN2_HI = 6.93147180559945286227e-01, LN2_LO = 2.31904681384629955842e-17;
  const double kd = (double)k;
  const double tail = __builtin_fma(kd, LN2_LO, lf + mc.lo * rcp_nr(m));
  const double r = __builtin_fma(kd, LN2_HI, tail);
  return m > 0.0 ? r : __builtin_nan("");
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
// single values moved between lanes of a wave
// ---------------------------------------------------------------------------
// Value of lane (lane ^ lm) of the wave, lm in {1, 2, 4, 8, 16, 32}, by
// register-level moves (DPP within rows of 16 lanes, lane-swap instructions
// across rows and halves) rather than through the LDS crossbar.
__device__ __forceinline__ uint32_t lane_xor(uint32_t x, int lm) {
  const int lane = threadIdx.x & 63;
  switch (lm) {
    case 1: return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);   // quad_perm 1,0,3,2
    case 2: return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true);   // quad_perm 2,3,0,1
    case 4: {
      const uint32_t up = __builtin_amdgcn_mov_dpp(x, 0x104, 0xF, 0xF, true);   // from lane + 4
      const uint32_t dn = __builtin_amdgcn_mov_dpp(x, 0x114, 0xF, 0xF, true);   // from lane - 4
      return (lane & 4) ? dn : up;
    }
    case 8: return __builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, true);  // rotate row by 8
    case 16: {
      const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
      return (lane & 16) ? r[0] : r[1];
    }
    default: {
      const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
      return (lane & 32) ? r[0] : r[1];
    }
  }
}
// Value of the next (lane + 1) or previous (lane - 1) lane of the wave (a
// whole-wave DPP shift; the last / first lane reads 0).
__device__ __forceinline__ uint32_t lane_next(uint32_t x) { return __builtin_amdgcn_mov_dpp(x, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ uint32_t lane_prev(uint32_t x) { return __builtin_amdgcn_mov_dpp(x, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ double lane_next(double x) {
  const uint64_t v = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = lane_next((uint32_t)v), hi = lane_next((uint32_t)(v >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double lane_prev(double x) {
  const uint64_t v = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = lane_prev((uint32_t)v), hi = lane_prev((uint32_t)(v >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double lane_xor(double x, int lm) {
  const uint64_t v = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = lane_xor((uint32_t)v, lm), hi = lane_xor((uint32_t)(v >> 32), lm);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// ---------------------------------------------------------------------------
// packs of doubles moved through cross-lane shuffles and LDS
// ---------------------------------------------------------------------------
template <int NF>
struct Pack {
  double v[NF];
};

// ---------------------------------------------------------------------------
// Wave-level scans on DPP row shifts (lanes of a 16-lane row) and lane reads
// (across rows), then one LDS exchange of the wave totals per workgroup.
// ---------------------------------------------------------------------------
// DPP move of each double of a pack (two 32-bit halves).  CTRL 0x110 + d:
// lane i reads lane i - d of its row; 0x100 + d: lane i + d; 0x138 / 0x130:
// the previous / next lane of the wave.  Lanes with no source read 0.  A
// DPP read from a lane that is switched off reads 0 too, so these moves are
// always evaluated with the whole wave active, never as one operand of ?:
// or && (which evaluates it under a partial mask).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int NF>
__device__ __forceinline__ Pack<NF> dpp_pack(const Pack<NF>& p) {
  Pack<NF> r;
#pragma unroll
  for (int i = 0; i < NF; ++i) r.v[i] = dpp_d<CTRL>(p.v[i]);
  return r;
}
// the pack of lane l (l uniform over the wave)
template <int NF>
__device__ __forceinline__ Pack<NF> lane_pack(const Pack<NF>& p, int l) {
  Pack<NF> r;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const long long v = __double_as_longlong(p.v[i]);
    const int lo = __builtin_amdgcn_readlane((int)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    r.v[i] = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  }
  return r;
}
template <int NF>
__device__ __forceinline__ Pack<NF> pick(bool c, const Pack<NF>& a, const Pack<NF>& b) {
  Pack<NF> r;
#pragma unroll
  for (int i = 0; i < NF; ++i) r.v[i] = c ? a.v[i] : b.v[i];
  return r;
}

// Inclusive prefix within each 16-lane row over the first M lanes of the
// row (M <= 16), op(earlier, later).
template <int M, int NF, class Op>
__device__ __forceinline__ Pack<NF> row_prefix_incl(Pack<NF> inc, Op op) {
  const int lr = threadIdx.x & 15;
  if (M > 1) { const Pack<NF> o = dpp_pack<0x111>(inc); if (lr >= 1) inc = op(o, inc); }
  if (M > 2) { const Pack<NF> o = dpp_pack<0x112>(inc); if (lr >= 2) inc = op(o, inc); }
  if (M > 4) { const Pack<NF> o = dpp_pack<0x114>(inc); if (lr >= 4) inc = op(o, inc); }
  if (M > 8) { const Pack<NF> o = dpp_pack<0x118>(inc); if (lr >= 8) inc = op(o, inc); }
  return inc;
}
// Inclusive suffix within each row over its first M lanes, op(lower, higher).
template <int M, int NF, class Op>
__device__ __forceinline__ Pack<NF> row_suffix_incl(Pack<NF> inc, Op op) {
  const int lr = threadIdx.x & 15;
  if (M > 1) { const Pack<NF> o = dpp_pack<0x101>(inc); if (lr + 1 < M) inc = op(inc, o); }
  if (M > 2) { const Pack<NF> o = dpp_pack<0x102>(inc); if (lr + 2 < M) inc = op(inc, o); }
  if (M > 4) { const Pack<NF> o = dpp_pack<0x104>(inc); if (lr + 4 < M) inc = op(inc, o); }
  if (M > 8) { const Pack<NF> o = dpp_pack<0x108>(inc); if (lr + 8 < M) inc = op(inc, o); }
  return inc;
}
// Inclusive prefix over the 64 lanes of the wave.
template <int NF, class Op>
__device__ __forceinline__ Pack<NF> wave_prefix_incl(const Pack<NF>& x, Op op) {
  Pack<NF> inc = row_prefix_incl<16>(x, op);
  const int row = (threadIdx.x & 63) >> 4;
  const Pack<NF> t0 = lane_pack(inc, 15), t1 = lane_pack(inc, 31), t2 = lane_pack(inc, 47);
  const Pack<NF> t01 = op(t0, t1);
  const Pack<NF> t012 = op(t01, t2);
  const Pack<NF> pre = pick(row == 1, t0, pick(row == 2, t01, t012));
  if (row > 0) inc = op(pre, inc);
  return inc;
}
// Inclusive suffix over the 64 lanes of the wave.
template <int NF, class Op>
__device__ __forceinline__ Pack<NF> wave_suffix_incl(const Pack<NF>& x, Op op) {
  Pack<NF> inc = row_suffix_incl<16>(x, op);
  const int row = (threadIdx.x & 63) >> 4;
  const Pack<NF> t1 = lane_pack(inc, 16), t2 = lane_pack(inc, 32), t3 = lane_pack(inc, 48);
  const Pack<NF> t23 = op(t2, t3);
  const Pack<NF> t123 = op(t1, t23);
  const Pack<NF> post = pick(row == 0, t123, pick(row == 1, t23, t3));
  if (row < 3) inc = op(inc, post);
  return inc;
}
// Combined wave totals, read by every lane from `lds` (NW packs of NF,
// starting at lds + off, stride S): exclusive prefix for this wave and the
// total.  NW <= 16.
template <int NW, int NF, class Op>
__device__ __forceinline__ void waves_prefix(const double* lds, int off, int S, const Pack<NF>& ident, Op op,
                                             Pack<NF>& pre, Pack<NF>& total) {
  const int lane = threadIdx.x & 63;
  Pack<NF> a = ident;
  if (lane < NW) {
#pragma unroll
    for (int i = 0; i < NF; ++i) a.v[i] = lds[lane * S + off + i];
  }
  a = row_prefix_incl<NW>(a, op);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  pre = wv > 0 ? lane_pack(a, wv - 1) : ident;
  total = lane_pack(a, NW - 1);
}
template <int NW, int NF, class Op>
__device__ __forceinline__ void waves_suffix(const double* lds, int off, int S, const Pack<NF>& ident, Op op,
                                             Pack<NF>& suf, Pack<NF>& total) {
  const int lane = threadIdx.x & 63;
  Pack<NF> a = ident;
  if (lane < NW) {
#pragma unroll
    for (int i = 0; i < NF; ++i) a.v[i] = lds[lane * S + off + i];
  }
  a = row_suffix_incl<NW>(a, op);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  suf = wv < NW - 1 ? lane_pack(a, wv + 1) : ident;
  total = lane_pack(a, 0);
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
  const Pack<NF> inc = wave_prefix_incl(x, op);
  const Pack<NF> sh = dpp_pack<0x138>(inc);       // outside any condition: every lane active
  const Pack<NF> ex = pick(lane == 0, ident, sh);
  if (lane == 63) {
#pragma unroll
    for (int i = 0; i < NF; ++i) lds[wv * NF + i] = inc.v[i];
  }
  __syncthreads();
  Pack<NF> pre;
  waves_prefix<NW, NF>(lds, 0, NF, ident, op, pre, total);
  if (TAIL) __syncthreads();
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
  const Pack<NF> inc = wave_suffix_incl(x, op);
  const Pack<NF> sh = dpp_pack<0x130>(inc);
  const Pack<NF> ex = pick(lane == 63, ident, sh);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NF; ++i) lds[wv * NF + i] = inc.v[i];
  }
  __syncthreads();
  Pack<NF> suf;
  waves_suffix<NW, NF>(lds, 0, NF, ident, op, suf, total);
  __syncthreads();
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
  const Pack<NP> ip = wave_prefix_incl(xp, opP);
  const Pack<NS> is = wave_suffix_incl(xs, opS);
  const Pack<NP> shp = dpp_pack<0x138>(ip);
  const Pack<NS> shs = dpp_pack<0x130>(is);
  const Pack<NP> ep = pick(lane == 0, idP, shp);
  const Pack<NS> es = pick(lane == 63, idS, shs);
  if (lane == 63) {
#pragma unroll
    for (int i = 0; i < NP; ++i) lds[wv * NF + i] = ip.v[i];
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NS; ++i) lds[wv * NF + NP + i] = is.v[i];
  }
  __syncthreads();
  Pack<NP> pre;
  Pack<NS> suf;
  waves_prefix<NW, NP>(lds, 0, NF, idP, opP, pre, totP);
  waves_suffix<NW, NS>(lds, NP, NF, idS, opS, suf, totS);
  if (TAIL) __syncthreads();
  exP = opP(pre, ep);
  exS = opS(es, suf);
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
