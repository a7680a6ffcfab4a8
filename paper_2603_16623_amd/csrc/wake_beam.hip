// gfx950 kernels that build the per-slice beam table of the ring solver:
// linear (cloud-in-cell) weights of every particle on the slice nodes
// xi_n = n dxi, entries grouped by slice, sorted by radius (then particle),
// and the cumulative charge q w c / (2 pi dxi) inside each radius, so that
// B_theta^(b) at a ring is (charge below its radius) / radius (Gauss law of
// the beam equation, Sec. "Numerical integration of wakefields").
#include "wake_common.h"
#include "wake_device.h"
#include "wake_launch.h"

#include <math.h>

#include <mutex>

#define WAKE_SORT_CAP 2048   // beam entries per slice sorted in LDS

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

__global__ void wake_zero_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
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

hipError_t launch_zero(int32_t* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(wake_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scratch of the beam-table build for callers that cannot allocate device
// memory (wake_prepare_noalloc): every GPU holds its own copy of this array
// until the process ends; calls on one GPU share it.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[WAKE_NOALLOC_SCRATCH];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[256];     // device address of `scratch`, per device
}  // namespace

hipError_t beam_scratch(int dev, void** p, size_t* bytes) {
  if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    // the array's name is a host-side stand-in: its device address on this
    // device comes from the runtime, once
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = q;
  }
  *p = g_scratch_ptr[dev];
  *bytes = WAKE_NOALLOC_SCRATCH;
  return hipSuccess;
}
