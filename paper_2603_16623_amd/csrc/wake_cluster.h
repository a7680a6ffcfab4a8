// Cooperative instances (device side): G workgroups march one instance that
// is too large for one workgroup's LDS.  Member g owns the sorted positions
// [g*P, g*P + P) (P = C * NT).  Per slice the members meet twice (slice
// head; transfer products with the coefficients of their source det-sums) to
// exchange their scan totals, and a few more times when the order needs
// fixing; the order
// fix-up works on keys and permutation in device memory.
//
// Barrier.  Each member publishes a pack (agent-scope atomic stores, which
// write through to the point where all XCDs meet), waits for those stores to
// complete and then stores the round number in its stamp word (the pack's
// last word, or a word beside the other members' stamps in instances of many
// members); thread m of every member polls member m's stamp until it reads the
// round, and once every stamp has been seen the member reads all the packs
// with agent-scope atomic loads, consecutive lanes on consecutive words (a
// wave's loads then fetch each line of the packs once, where one thread per
// pack made every member fetch every line once per word: at 196 members that
// was ~5x10^5 requests on 392 lines per meeting).  There is no shared arrival
// counter.  Packs alternate between two buffers by round; a
// member writes buffer b again only two rounds later, when every member has
// read it (it could not have passed the round in between otherwise).  The per-slice exchanges carry
// nothing but their packs and take no cache maintenance.  The fenced form,
// used by the order fix-up, also hands over plain device-memory data (keys,
// permutation, ring state that changes member): a release fence before the
// arrival writes the XCD's L2 back, an acquire fence after the wait drops
// its stale lines; both act on the whole L2 of the XCD, so they are kept off
// the every-slice path.
//
// Wait bounds.  Once every member of the instance has started, a wait longer
// than WAKE_CL_WAIT_TICKS sets the give-up word, and every member then leaves
// the instance (reported as a device error).  Before that, a member waits for
// workgroups of the launch to finish earlier tasks and take up the missing
// members (the queue hands out tasks in order, so they come): the bound then
// counts from the last task taken from the queue and is WAKE_CL_START_TICKS.
// No wave can wait forever.
#pragma once
#include "wake_common.h"
#include "wake_device.h"

#define WAKE_CL_GMAX WAKE_CL_MEMBERS       // members per instance at most (four per lane of a wave)
static_assert(WAKE_CL_GMAX <= 256, "member scans combine four members per lane");
#define WAKE_CL_WAIT_TICKS 200000000ll     // 2 s of the 100 MHz clock
#define WAKE_CL_START_TICKS 3000000000ll   // 30 s without a task taken

struct Cluster {
  int g, G;      // this member, members
  int round;     // barriers passed in this launch
  double* xd;    // [2][G][16] packs, then [2][G] stamps (see cl_stamp_at)
  int32_t* xc;   // [1] give-up, [2] members started
  const int32_t* queue;   // task queue counter of the launch
};

// Index in xd of member m's stamp word in buffer buf.  Below
// WAKE_CL_DENSE_STAMPS members it is the pack's last word (word 15); from
// there on the stamps sit side by side after the packs, eight to a 64-B
// line, so a wave's polls fetch eight stamps per request (with 196 members
// the polls of every member on every other member's line had become the
// meetings' main cost; with 40, stamps sharing lines made the stores of the
// last arrivals slower instead).
#define WAKE_CL_DENSE_STAMPS 64
__device__ __forceinline__ size_t cl_stamp_at(int G, int buf, int m) {
  return G >= WAKE_CL_DENSE_STAMPS ? (size_t)32 * G + (size_t)buf * G + m : ((size_t)buf * G + m) * 16 + 15;
}

// Counts the member in as started (once per launch, before its first
// exchange).
__device__ __forceinline__ void cl_start(Cluster& cl) {
  if (threadIdx.x == 0) atomicAdd(cl.xc + 2, 1);
}

// One thread waits (bounded) until the stamp word of another member's pack
// reads `want`.  1 when it did, 0 when a member gave up (or this wait gave
// up and told the others).  The give-up word and the bounds are looked at
// every sixteenth poll.
__device__ __noinline__ int cl_await(const WAKE_GLOBAL double* sp, double want, WAKE_GLOBAL int32_t* xc,
                                     const WAKE_GLOBAL int32_t* queue, int G) {
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  bool all_in = false;
  int q_last = -1;
  for (int it = 1;; ++it) {
    if (__hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want) return 1;
    if ((it & 15) == 0) {
      if (__hip_atomic_load(xc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 0;
      const uint64_t now = __builtin_amdgcn_s_memrealtime();
      if (!all_in) {
        all_in = __hip_atomic_load(xc + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= G;
        const int q = __hip_atomic_load(queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (all_in || q != q_last) { q_last = q; t0 = now; }
      }
      if ((int64_t)(now - t0) > (all_in ? WAKE_CL_WAIT_TICKS : WAKE_CL_START_TICKS)) {
        __hip_atomic_store(xc + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// All-gather of NF doubles per member; member m's pack lands at s_x[m * NF].
// Every thread of every member calls it at the same point of the march.
// Thread 0 writes the member's pack (write-through stores), waits for them
// to complete and then writes the pack's stamp, the round number; thread m
// waits for member m's stamp of this round; then the member's threads copy
// all packs, word by word across the lanes.  There is no shared counter:
// every member's arrival is its own word.  FENCED also
// publishes the plain device-memory writes before it (release fence before
// the stamp) and makes the others' visible after it (acquire fence).
// Returns false when a member gave up.
template <int NF, bool FENCED = true>
__device__ __forceinline__ bool cl_gather(Cluster& cl, const Pack<NF>& mine, double* s_x, int* s_ok) {
  static_assert(NF <= 15, "exchange packs hold 15 doubles and the stamp");
  const int buf = cl.round & 1;
  const double stamp = (double)cl.round;
  WAKE_GLOBAL double* const xd = gptr(cl.xd);
  if (threadIdx.x == 0) *s_ok = 1;
  __syncthreads();                                   // this member's writes of the round are issued
  if (threadIdx.x == 0) {
    WAKE_GLOBAL double* slot = xd + ((size_t)buf * cl.G + cl.g) * 16;
#pragma unroll
    for (int i = 0; i < NF; ++i) __hip_atomic_store(slot + i, mine.v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (FENCED) {
      // release only: the XCD's L2 written back (the member's plain stores
      // are there after the barrier); the acquire half comes after the wait
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    } else {
      // the pack's write-through stores complete before its stamp
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_s_waitcnt(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    __hip_atomic_store(xd + cl_stamp_at(cl.G, buf, cl.g), stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const int m = threadIdx.x;
  if (m < cl.G) {
    if (!cl_await(xd + cl_stamp_at(cl.G, buf, m), stamp, gptr(cl.xc), gptr(cl.queue), cl.G)) *s_ok = 0;
  }
  __syncthreads();                                   // every stamp of the round seen
  if (*s_ok) {
    const WAKE_GLOBAL double* base = xd + (size_t)buf * cl.G * 16;
    for (int i = threadIdx.x; i < cl.G * 16; i += blockDim.x) {
      const int f = i & 15;
      if (f < NF) s_x[(i >> 4) * NF + f] = __hip_atomic_load(base + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  const int ok = *s_ok;
  if (FENCED) {
    if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // stale lines dropped
    __syncthreads();
  }
  ++cl.round;
  return ok != 0;
}

// Exclusive prefix over members (op(earlier, later)) of the packs gathered at
// s_x (field offset off, NFT doubles per member) for member g, and the total.
// G <= 64 MPL: lane l of each wave combines members MPL l .. MPL l + MPL-1
// in order (ident beyond the last member, which op absorbs exactly), a wave
// scan runs over the lanes, and member g's prefix is the lanes before its
// own followed by the members of its lane below it.  MPL = 1 (G <= 64)
// leaves out the serial steps on either side of the wave scan.
template <int NF, int NFT, class Op, int MPL = 4>
__device__ __forceinline__ void cl_prefix(const double* s_x, int off, int g, int G, const Pack<NF>& ident,
                                          Op op, Pack<NF>& pre, Pack<NF>& tot) {
  const int lane = threadIdx.x & 63;
  Pack<NF> blk = ident;
#pragma unroll
  for (int j = 0; j < MPL; ++j) {
    const int m = MPL * lane + j;
    if (m < G) {
      Pack<NF> x;
#pragma unroll
      for (int i = 0; i < NF; ++i) x.v[i] = s_x[m * NFT + off + i];
      blk = op(blk, x);
    }
  }
  const Pack<NF> inc = wave_prefix_incl(blk, op);
  const int lg = g / MPL;
  const Pack<NF> before = lane_pack(inc, lg > 0 ? lg - 1 : 0);
  Pack<NF> p = lg > 0 ? before : ident;
  for (int m = MPL * lg; m < g; ++m) {
    Pack<NF> x;
#pragma unroll
    for (int i = 0; i < NF; ++i) x.v[i] = s_x[m * NFT + off + i];
    p = op(p, x);
  }
  pre = p;
  tot = lane_pack(inc, 63);
}
// Exclusive suffix over members (op(lower, higher)) and the total, with the
// same grouping of four members per lane.
template <int NF, int NFT, class Op>
__device__ __forceinline__ void cl_suffix(const double* s_x, int off, int g, int G, const Pack<NF>& ident,
                                          Op op, Pack<NF>& suf, Pack<NF>& tot) {
  const int lane = threadIdx.x & 63;
  Pack<NF> blk = ident;
#pragma unroll
  for (int j = 3; j >= 0; --j) {
    const int m = 4 * lane + j;
    if (m < G) {
      Pack<NF> x;
#pragma unroll
      for (int i = 0; i < NF; ++i) x.v[i] = s_x[m * NFT + off + i];
      blk = op(x, blk);
    }
  }
  const Pack<NF> inc = wave_suffix_incl(blk, op);
  const int lg = g >> 2;
  const Pack<NF> after = lane_pack(inc, lg < 63 ? lg + 1 : 63);
  Pack<NF> p = lg < 63 ? after : ident;
  const int top = min(4 * lg + 3, G - 1);
  for (int m = top; m > g; --m) {
    Pack<NF> x;
#pragma unroll
    for (int i = 0; i < NF; ++i) x.v[i] = s_x[m * NFT + off + i];
    p = op(x, p);
  }
  suf = p;
  tot = lane_pack(inc, 0);
}

// Slot of position p in the cooperative layout (P = C * NT), quotients from
// reciprocal estimates corrected to the exact ones.
__device__ __forceinline__ int cl_div(int a, int b, double ib) {
  int q = (int)((double)a * ib);
  if (q * b > a) --q;
  else if ((q + 1) * b <= a) ++q;
  return q;
}
template <int NT>
__device__ __forceinline__ int cl_slot(int p, int C, int P, double iC, double iP) {
  const int g = cl_div(p, P, iP);
  const int q = p - g * P;
  const int t = cl_div(q, C, iC);
  return g * P + (q - t * C) * NT + t;
}
// Ring id of home slot hs (the inverse of cl_slot).
template <int NT>
__device__ __forceinline__ int32_t cl_id(int32_t hs, int C, int P, double iP) {
  const int g = cl_div(hs, P, iP);
  const int r = hs - g * P;
  return g * P + (r & (NT - 1)) * C + (r >> __builtin_ctz(NT));
}

// (rho, id) order with the slot carried in the low word: k = id << 32 | slot.
__device__ __forceinline__ bool k64_lt(double ra, uint64_t ka, double rb, uint64_t kb) {
  return (ra < rb) | ((ra == rb) & (ka < kb));
}
__device__ __forceinline__ uint64_t lane_xor64(uint64_t x, int lm) {
  return ((uint64_t)lane_xor((uint32_t)(x >> 32), lm) << 32) | lane_xor((uint32_t)x, lm);
}
__device__ __forceinline__ uint64_t lane_next64(uint64_t x) {
  return ((uint64_t)lane_next((uint32_t)(x >> 32)) << 32) | lane_next((uint32_t)x);
}
__device__ __forceinline__ uint64_t lane_prev64(uint64_t x) {
  return ((uint64_t)lane_prev((uint32_t)(x >> 32)) << 32) | lane_prev((uint32_t)x);
}

// One wave sorts 256 keys held four per lane (lane l: keys 4l..4l+3) by
// (radius, 64-bit word with the id in the high half): odd-even
// transposition for up to 32 phases, then a bitonic network.  Returns false
// when they were in order already (nothing moved).
__device__ __forceinline__ bool sort_regs256(double* r, uint64_t* k) {
  const int lane = threadIdx.x & 63;
  bool ok = !k64_lt(r[1], k[1], r[0], k[0]) && !k64_lt(r[2], k[2], r[1], k[1]) &&
            !k64_lt(r[3], k[3], r[2], k[2]);
  {
    const double nr = lane_next(r[0]);
    const uint64_t nk = lane_next64(k[0]);
    if (lane < 63) ok = ok && !k64_lt(nr, nk, r[3], k[3]);
  }
  if (__all(ok)) return false;
  bool done = false;
  #pragma unroll 1
  for (int it = 0; it < 8 && !done; ++it) {
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
#pragma unroll
      for (int j = 0; j < 4; j += 2) {
        if (k64_lt(r[j + 1], k[j + 1], r[j], k[j])) {
          const double tr = r[j]; r[j] = r[j + 1]; r[j + 1] = tr;
          const uint64_t tk = k[j]; k[j] = k[j + 1]; k[j + 1] = tk;
        }
      }
      if (k64_lt(r[2], k[2], r[1], k[1])) {
        const double tr = r[1]; r[1] = r[2]; r[2] = tr;
        const uint64_t tk = k[1]; k[1] = k[2]; k[2] = tk;
      }
      const double nr = lane_next(r[0]), pr = lane_prev(r[3]);
      const uint64_t nq = lane_next64(k[0]), pq = lane_prev64(k[3]);
      const bool take_next = lane < 63 && k64_lt(nr, nq, r[3], k[3]);
      const bool take_prev = lane > 0 && k64_lt(r[0], k[0], pr, pq);
      if (take_next) { r[3] = nr; k[3] = nq; }
      if (take_prev) { r[0] = pr; k[0] = pq; }
    }
    bool in_order = !k64_lt(r[1], k[1], r[0], k[0]) && !k64_lt(r[2], k[2], r[1], k[1]) &&
                    !k64_lt(r[3], k[3], r[2], k[2]);
    const double xr = lane_next(r[0]);
    const uint64_t xq = lane_next64(k[0]);
    if (lane < 63) in_order = in_order && !k64_lt(xr, xq, r[3], k[3]);
    done = __all(in_order);
  }
  if (!done) {
#pragma unroll
    for (int kk = 2; kk <= 256; kk <<= 1) {
#pragma unroll
      for (int d = kk >> 1; d > 0; d >>= 1) {
        if (d >= 4) {
          const int lm = d >> 2;
          const bool lower = (lane & lm) == 0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double pr = lane_xor(r[j], lm);
            const uint64_t pq = lane_xor64(k[j], lm);
            const bool up = ((4 * lane + j) & kk) == 0;
            if (k64_lt(pr, pq, r[j], k[j]) == (lower == up)) { r[j] = pr; k[j] = pq; }
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (j & d) continue;
            const int jj = j | d;
            const bool up = ((4 * lane + j) & kk) == 0;
            if (k64_lt(r[jj], k[jj], r[j], k[j]) == up) {
              const double tr = r[j]; r[j] = r[jj]; r[jj] = tr;
              const uint64_t tk = k[j]; k[j] = k[jj]; k[jj] = tk;
            }
          }
        }
      }
    }
  }
  return true;
}

// One wave puts the positions [b0, b0 + 256) of a cooperative instance in
// order: keys by slot in device memory (gk_r, gk_i), order perm by position
// slot; only the positions in [w_lo, w_hi) are written back (a block that
// two members sort alike, each keeping its own positions), and with src_at
// the order is read from that array by position instead of from perm.
template <int NT>
__device__ __noinline__ void cl_sort_block(int b0, int N, int C, int P, double iC, double iP,
                                           const WAKE_GLOBAL double* gk_r, const WAKE_GLOBAL int32_t* gk_i,
                                           WAKE_GLOBAL int32_t* perm, int w_lo = 0, int w_hi = 0x7fffffff,
                                           const WAKE_GLOBAL int32_t* src_at = nullptr) {
  const int lane = threadIdx.x & 63;
  double r[4];
  uint64_t k[4];
  int sl[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = b0 + 4 * lane + j;
    sl[j] = -1;
    r[j] = INFINITY;
    k[j] = ~0ull;
    if (p < N) {
      sl[j] = cl_slot<NT>(p, C, P, iC, iP);
      const int src = src_at ? src_at[p] : perm[sl[j]];
      r[j] = gk_r[src];
      k[j] = ((uint64_t)(uint32_t)gk_i[src] << 32) | (uint32_t)src;
    }
  }
  if (!sort_regs256(r, k)) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = b0 + 4 * lane + j;
    if (sl[j] >= 0 && p >= w_lo && p < w_hi) perm[sl[j]] = (int32_t)(uint32_t)(k[j] & 0xffffffffull);
  }
}

// The same for keys held by position in LDS (L_r, L_k, positions [0, n)).
__device__ __noinline__ void lds_sort_block(int b0, int n, double* L_r, uint64_t* L_k) {
  const int lane = threadIdx.x & 63;
  double r[4];
  uint64_t k[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = b0 + 4 * lane + j;
    r[j] = p < n ? L_r[p] : INFINITY;
    k[j] = p < n ? L_k[p] : ~0ull;
  }
  if (!sort_regs256(r, k)) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = b0 + 4 * lane + j;
    if (p < n) { L_r[p] = r[j]; L_k[p] = k[j]; }
  }
}

// Whether this thread's positions (and the position after them) are out of
// order in the cooperative order perm; with within, the position after the
// member's last one (the next member's first) is left out.  Slots are read
// eight at a time, then their keys, so each batch costs two rounds of
// independent loads.
template <int NT>
__device__ __forceinline__ int cl_chunk_disordered(const WakeInst& I, int goff, int cnt, int C, int P,
                                                   double iC, double iP, bool within = false) {
  const int tid = threadIdx.x;
  const int N = I.N;
  if (cnt <= 0) return 0;
  const int p0 = goff + tid * C;
  const int m = p0 + cnt < (within ? min(N, goff + P) : N) ? cnt + 1 : cnt;
  int bad = 0;
  double pr = -INFINITY;
  int32_t pi = -1;
  #pragma unroll 1
  for (int k0 = 0; k0 < m; k0 += 8) {
    int src[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + j;
      src[j] = -1;
      if (k < m) src[j] = gptr(I.perm)[k < cnt ? goff + k * NT + tid : cl_slot<NT>(p0 + k, C, P, iC, iP)];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (src[j] < 0) continue;
      const double r = gptr(I.gk_r)[src[j]];
      const int32_t id = gptr(I.gk_i)[src[j]];
      if (k0 + j > 0 && key_lt(r, id, pr, pi)) bad = 1;
      pr = r;
      pi = id;
    }
  }
  return bad;
}

// Fallback order of a cooperative instance: a bitonic sort of every position
// in device memory (keys copied out in position order, padded to the next
// power of two with keys above every ring), one barrier per network stage.
template <int NT>
__device__ __noinline__ int cl_bitonic(const WAKE_GLOBAL WakeInst* Ig, Cluster cl, int xo, int oko) {
  const WakeInst& I = *(const WakeInst*)Ig;
  double* const s_x = reinterpret_cast<double*>(wake_lds + xo);
  int* const s_ok = reinterpret_cast<int*>(wake_lds + oko);
  const int N = I.N, C = I.C, P = C * NT;
  const double iC = 1.0 / (double)C, iP = 1.0 / (double)P;
  const int P2 = N <= 1 ? 1 : 1 << (32 - __builtin_clz((unsigned)(N - 1)));
  const int gt = cl.g * NT + threadIdx.x, nth = cl.G * NT;
  for (int p = gt; p < P2; p += nth) {
    if (p < N) {
      const int src = gptr(I.perm)[cl_slot<NT>(p, C, P, iC, iP)];
      gptr(I.bt_r)[p] = gptr(I.gk_r)[src];
      gptr(I.bt_i)[p] = gptr(I.gk_i)[src];
      gptr(I.bt_s)[p] = src;
    } else {
      gptr(I.bt_r)[p] = INFINITY;
      gptr(I.bt_i)[p] = 0x7fffffff;
      gptr(I.bt_s)[p] = -1;
    }
  }
  if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
  for (int kk = 2; kk <= P2; kk <<= 1) {
    for (int d = kk >> 1; d > 0; d >>= 1) {
      const int ld = __builtin_ctz((unsigned)d);
      for (int i = gt; i < P2 / 2; i += nth) {
        const int a = ((i >> ld) << (ld + 1)) | (i & (d - 1)), b = a | d;
        const bool up = (a & kk) == 0;
        const double ra = gptr(I.bt_r)[a], rb = gptr(I.bt_r)[b];
        const int32_t ia = gptr(I.bt_i)[a], ib = gptr(I.bt_i)[b];
        if (key_lt(rb, ib, ra, ia) == up) {
          const int32_t sa = gptr(I.bt_s)[a], sb = gptr(I.bt_s)[b];
          gptr(I.bt_r)[a] = rb; gptr(I.bt_r)[b] = ra;
          gptr(I.bt_i)[a] = ib; gptr(I.bt_i)[b] = ia;
          gptr(I.bt_s)[a] = sb; gptr(I.bt_s)[b] = sa;
        }
      }
      if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
    }
  }
  for (int p = gt; p < N; p += nth) gptr(I.perm)[cl_slot<NT>(p, C, P, iC, iP)] = gptr(I.bt_s)[p];
  return cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok) ? cl.round : -1;
}

// Order fix-up of a cooperative instance from its keys by slot (gk_r, gk_i):
// writes perm (position slot -> slot).  Blocks of 256 positions sorted by
// single waves of all members at offsets 0, 256, ... and then 128, 384, ...
// (the two phases order every ring within 128 positions of its place), the
// order checked across all positions, at most two such rounds.  Returns -1
// when a member gave up, else twice the barrier count plus whether disorder
// remains (the caller then runs a fallback sort).
template <int NT>
__device__ __noinline__ int cl_fix(const WAKE_GLOBAL WakeInst* Ig, Cluster cl, int xo, int oko) {
  const WakeInst& I = *(const WakeInst*)Ig;
  double* const s_x = reinterpret_cast<double*>(wake_lds + xo);
  int* const s_ok = reinterpret_cast<int*>(wake_lds + oko);
  const int tid = threadIdx.x;
  const int N = I.N, C = I.C, P = C * NT;
  const double iC = 1.0 / (double)C, iP = 1.0 / (double)P;
  const int goff = cl.g * P;
  const int Ng = min(P, N - goff);
  const int cnt = max(0, min(C, Ng - tid * C));
  for (int k = 0; k < cnt; ++k) gptr(I.perm)[goff + k * NT + tid] = goff + k * NT + tid;
  if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
  constexpr int NW = NT / 64;
  const int wave = tid >> 6;
  #pragma unroll 1
  for (int round = 0; round < 2; ++round) {
    #pragma unroll 1
    for (int b = wave; b * 256 < Ng; b += NW) cl_sort_block<NT>(goff + b * 256, N, C, P, iC, iP, gptr(I.gk_r), gptr(I.gk_i), gptr(I.perm));
    if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
    #pragma unroll 1
    for (int b = wave; 128 + b * 256 < Ng; b += NW)
      cl_sort_block<NT>(goff + 128 + b * 256, N, C, P, iC, iP, gptr(I.gk_r), gptr(I.gk_i), gptr(I.perm));
    if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
    // in order? this thread's positions and the position after them
    int bad = cl_chunk_disordered<NT>(I, goff, cnt, C, P, iC, iP);
    bad = __syncthreads_or(bad);
    if (!cl_gather<1>(cl, Pack<1>{{(double)bad}}, s_x, s_ok)) return -1;
    double any = 0.0;
    for (int m = 0; m < cl.G; ++m) any += s_x[m];
    if (any == 0.0) return 2 * cl.round;
  }
  return 2 * cl.round + 1;
}

// One in-loop round of the cooperative fix-up over all members (first: this
// member's order starts from the identity of the pushed rings).  Each member
// sorts the blocks at offsets 0, 256, ... of its own range (member ranges are
// multiples of 256 positions) after a local barrier, then, between two
// barriers of all members, the blocks at 128, 384, ... that start in its
// range; the last of these straddles the next member.  Returns -1 when a
// member gave up, else twice the barrier count plus whether this member's
// positions (and the first of the next member) are still out of order; the
// next slice-head exchange sums that flag.
template <int NT>
__device__ __noinline__ int cl_fix_round(const WAKE_GLOBAL WakeInst* Ig, Cluster cl, int xo, int oko, bool first,
                                         int lo) {
  const WakeInst& I = *(const WakeInst*)Ig;
  double* const s_x = reinterpret_cast<double*>(wake_lds + xo);
  int* const s_ok = reinterpret_cast<int*>(wake_lds + oko);
  const int tid = threadIdx.x;
  const int N = I.N, C = I.C, P = C * NT;
  const double iC = 1.0 / (double)C, iP = 1.0 / (double)P;
  const int goff = cl.g * P;
  const int Ng = min(P, N - goff);
  const int cnt = max(0, min(C, Ng - tid * C));
  constexpr int NW = NT / 64;
  const int wave = tid >> 6;
  if (lo >= 0) {
    // the same blocks with the interior ones sorted in LDS first; after the
    // meeting the two members a boundary block straddles both sort it, from
    // the same keys to the same order, and each writes back its own
    // positions only, so no second meeting has to publish them; the order
    // across member boundaries is checked at the next slice head
    // (the order of the first and last 128 positions of every member also by
    // position in bt_s, which no member writes again before the next slice
    // head: the straddling sorts read that copy, so one member's write-back
    // cannot change the other's input)
    cl_lds_blocks<NT>(I, cl.g, first, lo, false, gptr(I.bt_s));
    if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
    if (wave == 0 && goff + Ng < N)
      cl_sort_block<NT>(goff + Ng - 128, N, C, P, iC, iP, gptr(I.gk_r), gptr(I.gk_i), gptr(I.perm), goff, goff + Ng,
                        gptr(I.bt_s));
    if (wave == 1 && goff > 0)
      cl_sort_block<NT>(goff - 128, N, C, P, iC, iP, gptr(I.gk_r), gptr(I.gk_i), gptr(I.perm), goff, goff + Ng,
                        gptr(I.bt_s));
    __syncthreads();
    const int bl = cl_chunk_disordered<NT>(I, goff, cnt, C, P, iC, iP, true);
    return 2 * cl.round + (__syncthreads_or(bl) ? 1 : 0);
  }
  if (first)           // later rounds continue from the order the previous one left
    for (int k = 0; k < cnt; ++k) gptr(I.perm)[goff + k * NT + tid] = goff + k * NT + tid;
  __syncthreads();
  #pragma unroll 1
  for (int b = wave; b * 256 < Ng; b += NW)
    cl_sort_block<NT>(goff + b * 256, N, C, P, iC, iP, gptr(I.gk_r), gptr(I.gk_i), gptr(I.perm));
  if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
  #pragma unroll 1
  for (int b = wave; 128 + b * 256 < Ng; b += NW)
    cl_sort_block<NT>(goff + 128 + b * 256, N, C, P, iC, iP, gptr(I.gk_r), gptr(I.gk_i), gptr(I.perm));
  if (!cl_gather<1>(cl, Pack<1>{{0.0}}, s_x, s_ok)) return -1;
  const int b_ = cl_chunk_disordered<NT>(I, goff, cnt, C, P, iC, iP);
  return 2 * cl.round + (__syncthreads_or(b_) ? 1 : 0);
}

// One member-local round of the in-loop fix-up, for disorder inside this
// member's range while the order across member boundaries holds: the blocks
// at offsets 0, 256, ... and then 128, 384, ... of the member's own range,
// less the one that straddles the next member, between the member's own
// barriers; the member's keys and order are its own writes, so no exchange
// is needed.  Returns whether the member's positions are still out of order.
template <int NT>
__device__ __noinline__ int cl_fix_local(const WAKE_GLOBAL WakeInst* Ig, int g, bool first) {
  const WakeInst& I = *(const WakeInst*)Ig;
  const int tid = threadIdx.x;
  const int N = I.N, C = I.C, P = C * NT;
  const double iC = 1.0 / (double)C, iP = 1.0 / (double)P;
  const int goff = g * P;
  const int Ng = min(P, N - goff);
  const int cnt = max(0, min(C, Ng - tid * C));
  const int lim = goff + Ng == N ? Ng : Ng - 256;   // phase-two blocks starting below lim lie inside
  constexpr int NW = NT / 64;
  const int wave = tid >> 6;
  if (first)
    for (int k = 0; k < cnt; ++k) gptr(I.perm)[goff + k * NT + tid] = goff + k * NT + tid;
  __syncthreads();
  #pragma unroll 1
  for (int b = wave; b * 256 < Ng; b += NW)
    cl_sort_block<NT>(goff + b * 256, N, C, P, iC, iP, gptr(I.gk_r), gptr(I.gk_i), gptr(I.perm));
  __syncthreads();
  #pragma unroll 1
  for (int b = wave; 128 + b * 256 < lim; b += NW)
    cl_sort_block<NT>(goff + 128 + b * 256, N, C, P, iC, iP, gptr(I.gk_r), gptr(I.gk_i), gptr(I.perm));
  __syncthreads();
  const int b_ = cl_chunk_disordered<NT>(I, goff, cnt, C, P, iC, iP, true);
  return __syncthreads_or(b_);
}

// Block phases over this member's own positions with its keys copied into
// LDS by position (radius; id and slot in one 64-bit word) at byte offset lo
// of the dynamic LDS (16 bytes per position): the blocks at offsets 0, 256,
// ... and then 128, 384, ... of the member's range, less the one that
// straddles the next member, sorted there, and the order written back to
// perm.  Loads batched: slots, then keys.  With check, returns whether the
// member's positions are still out of order (the position after its last is
// the next member's, checked elsewhere).
template <int NT>
__device__ __forceinline__ int cl_lds_blocks(const WakeInst& I, int g, bool first, int lo, bool check,
                                             WAKE_GLOBAL int32_t* stage = nullptr) {
  const int tid = threadIdx.x;
  const int N = I.N, C = I.C, P = C * NT;
  const int goff = g * P;
  const int Ng = min(P, N - goff);
  const int cnt = max(0, min(C, Ng - tid * C));
  const int lim = goff + Ng == N ? Ng : Ng - 256;   // phase-two blocks starting below lim lie inside
  constexpr int NW = NT / 64;
  const int wave = tid >> 6;
  double* const L_r = reinterpret_cast<double*>(wake_lds + lo);
  uint64_t* const L_k = reinterpret_cast<uint64_t*>(wake_lds + lo + 8 * P);
  WAKE_GLOBAL int32_t* const perm = gptr(I.perm);
  const WAKE_GLOBAL double* const gr = gptr(I.gk_r);
  const WAKE_GLOBAL int32_t* const gi = gptr(I.gk_i);
  #pragma unroll 1
  for (int k0 = 0; k0 < cnt; k0 += 8) {
    int src[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int sl = goff + (k0 + j) * NT + tid;
      src[j] = -1;
      if (k0 + j < cnt) src[j] = first ? sl : perm[sl];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (src[j] < 0) continue;
      const int q = tid * C + k0 + j;
      L_r[q] = gr[src[j]];
      L_k[q] = ((uint64_t)(uint32_t)gi[src[j]] << 32) | (uint32_t)src[j];
    }
  }
  __syncthreads();
  #pragma unroll 1
  for (int b = wave; b * 256 < Ng; b += NW) lds_sort_block(b * 256, Ng, L_r, L_k);
  __syncthreads();
  #pragma unroll 1
  for (int b = wave; 128 + b * 256 < lim; b += NW) lds_sort_block(128 + b * 256, Ng, L_r, L_k);
  __syncthreads();
  int bad = 0;
  #pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    const int q = tid * C + k;
    if (check && q + 1 < Ng && k64_lt(L_r[q + 1], L_k[q + 1], L_r[q], L_k[q])) bad = 1;
    const int32_t v = (int32_t)(uint32_t)(L_k[q] & 0xffffffffull);
    perm[goff + k * NT + tid] = v;
    if (stage && (q < 128 || q >= Ng - 128)) stage[goff + q] = v;
  }
  return __syncthreads_or(bad);
}

// The member-local round in LDS (cl_fix_local's blocks).
template <int NT>
__device__ __noinline__ int cl_fix_local_lds(const WAKE_GLOBAL WakeInst* Ig, int g, bool first, int lo) {
  return cl_lds_blocks<NT>(*(const WakeInst*)Ig, g, first, lo, true);
}
