// Host runtime of the C ABI in include/wake.h: argument checking, device
// memory (one arena per context), beam-table build and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/wake.h"
#include "wake_common.h"
#include "wake_launch.h"
#include "wake_runtime.h"

namespace {

int g_nt = 512;      // workgroup threads of new contexts (slot layout)
int g_wpc = 0;       // workgroups per compute unit of persistent launches (0: occupancy)
int g_cl_rings = 0;  // rings per thread of cooperative instances (0: 8)
int g_cl_min = 0;    // ring count from which instances are cooperative (0: beyond one workgroup's LDS keys)
bool g_tuned = false;   // a tuning table is installed
wake_tuning g_tuning;   // per ring-count bucket: threads, cooperative rings per thread


}  // namespace

// Most members of one instance: the member scans' limit, and the
// workgroups of nt threads the current device holds at once (members of an
// instance must be resident together).
// The installed tuning's layout for N rings (false when none is installed).
static bool tuned_layout(int N, Layout* L) {
  if (!g_tuned) return false;
  int b = 0;
  while (b + 1 < g_tuning.n_buckets && N >= g_tuning.lo[b + 1]) ++b;
  L->nt = g_tuning.threads[b];
  L->rpt = g_tuning.rings_per_thread[b];
  L->min_n = L->rpt > 0 ? 1 : INT32_MAX;
  return true;
}

extern "C" int wake_set_tuning(const wake_tuning* t) {
  if (!t) {
    g_tuned = false;
    return WAKE_OK;
  }
  if (t->n_buckets < 1 || t->n_buckets > WAKE_TUNE_BUCKETS || t->lo[0] != 0) return WAKE_EINVAL;
  for (int b = 0; b < t->n_buckets; ++b) {
    if (b > 0 && !(t->lo[b] > t->lo[b - 1])) return WAKE_EINVAL;
    if (!march_threads_ok(t->threads[b]) || t->rings_per_thread[b] < 0 || t->rings_per_thread[b] > 4096)
      return WAKE_EINVAL;
  }
  for (int b = 0; b < t->n_buckets; ++b) HIP_TRY(march_prepare(t->threads[b]));
  g_tuning = *t;
  g_tuned = true;
  return WAKE_OK;
}

extern "C" int wake_get_tuning(wake_tuning* t) {
  if (!t) return WAKE_EINVAL;
  if (!g_tuned) return WAKE_ESTATE;
  *t = g_tuning;
  return WAKE_OK;
}

extern "C" int wake_get_threads(wake_ctx* c, int32_t* threads) {
  if (!c || !threads) return WAKE_EINVAL;
  *threads = c->I.nt;
  return WAKE_OK;
}

static int members_max(int nt) {
  static int cached[3] = {0, 0, 0};
  const int k = nt == 256 ? 0 : nt == 512 ? 1 : 2;
  if (cached[k] == 0) {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
      cu = 1;
    const int occ = std::max(1, march_occupancy(nt));
    cached[k] = std::max(1, std::min(WAKE_CL_MEMBERS, occ * cu));
  }
  return cached[k];
}

Layout layout_default(int nt) { return Layout{nt, g_cl_rings, g_cl_min}; }

Layout layout_for(int N) {
  Layout L;
  if (tuned_layout(N, &L)) return L;
  return layout_default(g_nt);
}

// Layout of an instance of N rings: one workgroup with C = ceil(N / nt)
// rings per thread while the keys of every position fit its LDS (and N is
// below the cooperative threshold), else G members of C rings per thread
// (G at most members_max).
void layout_of(int N, const Layout& L, int* C, int* G) {
  const int nt = L.nt;
  const int kcap = march_cmax(nt) * nt;
  const int min_n = L.min_n > 0 ? L.min_n : kcap + 1;
  if (N >= min_n && N > nt) {
    const int gm = members_max(nt);
    int c = std::max(L.rpt > 0 ? L.rpt : 8, (N + gm * nt - 1) / (gm * nt));
    const int g = (N + c * nt - 1) / (c * nt);
    if (g > 1) { *C = c; *G = g; return; }
  }
  *C = (N + nt - 1) / nt;
  *G = 1;
}

namespace {

static size_t pow2_at_least(size_t n) {
  size_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Bytes of the per-context arena (mirrors the carving in wake_create).
// S = slots of the per-ring arrays (G * C * nt >= N).
size_t arena_bytes(int N, int n_xi, int stride, const Layout& L) {
  int Ci = 0, Gi = 1;
  layout_of(N, L, &Ci, &Gi);
  const size_t S = (size_t)Gi * Ci * L.nt;
  const size_t n_rec = stride > 0 ? (size_t)(n_xi + stride - 1) / stride : 0;
  size_t d = 0, i = 0;
  d += 2 * RC_CHUNKS * S;                   // constants by home slot
  d += WAKE_ION_REC * (size_t)(N + 1);      // ion interval records
  d += 4;                                   // tot0, Q
  d += 2 * RS_DOUBLES * S;                  // state, two buffers
  d += (2 * SC_CHUNKS + 2) * S;             // slice scratch, laser terms
  d += 1 * S;                               // fix-up: suffix minimum
  i += 4 * S;                               // fix-up: order, prefix max id, flags, run starts
  d += 2 * (size_t)N;                       // sort keys x2
  i += 4 * (size_t)N + (size_t)N;           // sort ids/slots x2, free slots
  d += 2 * (size_t)n_xi;                    // axis
  d += n_rec * OUT_N * (size_t)N;           // snapshots
  d += OUT_N * (size_t)N;                   // last
  i += CTL_NWORDS;                          // ctl
  d += CNT_N;                               // event counters
  d += 4 * (size_t)N;                       // staging
  if (Gi > 1) {                             // cooperative: exchange, keys, fallback sort
    const size_t P2 = pow2_at_least((size_t)N);
    d += 2 * (size_t)Gi * 17 + S + P2;
    i += 4 + S + 2 * P2;
  }
  return d * 8 + i * 4 + 64 * 256;          // + alignment slack
}

}  // namespace

struct wake_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<wake_ctx*> ctxs;
  WakeInst* d_insts = nullptr;     // descriptors of eager solves
  int32_t* d_counter = nullptr;
  WakeInst* d_ginsts = nullptr;    // descriptors the captured graph reads (written by capture only)
  int32_t* d_gcounter = nullptr;
  WakeIons* d_jinsts = nullptr;    // two-species records of eager solves
  WakeIons* d_gjinsts = nullptr;   // two-species records the captured graph reads
  int cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool holds = false;      // the contexts count this batch
};

int dev_err(hipError_t e) { return e == hipErrorOutOfMemory ? WAKE_ENOMEM : WAKE_EDEVICE; }

extern "C" const char* wake_strerror(int code) {
  switch (code) {
    case WAKE_OK: return "ok";
    case WAKE_EINVAL: return "invalid argument";
    case WAKE_ENOMEM: return "out of memory";
    case WAKE_EDEVICE: return "HIP runtime error";
    case WAKE_ESTATE: return "call out of order";
    case WAKE_EBREAKDOWN: return "quasistatic breakdown (psibar <= 0 or non-finite value)";
    case WAKE_ENOTREC: return "slice not recorded";
    default: return "unknown error";
  }
}

int64_t ctx_footprint(int32_t n_rings, int32_t n_xi, int64_t n_particles, int32_t record_stride,
                      const Layout& L) {
  if (n_rings <= 0 || n_xi <= 0 || n_particles < 0 || record_stride < 0) return -1;
  int64_t b = (int64_t)arena_bytes(n_rings, n_xi, record_stride, L);
  // persistent beam table: offsets + (r, cumulative charge) per entry
  b += 4 * (int64_t)(n_xi + 1) + 16 * 2 * n_particles + 1024;
  // transient build buffers (particles, counts, padded entries)
  b += 40 * n_particles + 20 * (int64_t)(n_xi + 1) + 24 * 4 * n_particles + 2048;
  b += sizeof(WakeInst) + 512;
  return b;
}

extern "C" int64_t wake_footprint(int32_t n_rings, int32_t n_xi, int64_t n_particles,
                                  int32_t record_stride) {
  if (n_rings <= 0) return -1;
  return ctx_footprint(n_rings, n_xi, n_particles, record_stride, layout_for(n_rings));
}

static void release(wake_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->arena.base) (void)hipFree(c->arena.base);
  if (c->beam_mem && !c->beam_external) (void)hipFree(c->beam_mem);
  if (c->grid_mem) (void)hipFree(c->grid_mem);
  if (c->d_inst) (void)hipFree(c->d_inst);
  if (c->d_counter) (void)hipFree(c->d_counter);
  if (c->d_J) (void)hipFree(c->d_J);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" void wake_destroy(wake_ctx* ctx) { release(ctx); }

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// The plasma column and window of a new context (wake_plasma, wake_domain).
static int check_column(const wake_plasma* plasma, const wake_domain* dom) {
  if (!plasma || !dom || plasma->n_rings <= 0 || !plasma->r0 || !plasma->dr) return WAKE_EINVAL;
  const int N = plasma->n_rings;
  if (N > (1 << 28)) return WAKE_EINVAL;
  if (!finite_pos(dom->dxi) || dom->n_xi <= 0 || dom->record_stride < 0) return WAKE_EINVAL;
  // ring geometry: r0_j = sum_{k<j} dr_k + dr_j/2, strictly increasing
  double edge = 0.0;
  for (int j = 0; j < N; ++j) {
    const double d = plasma->dr[j], r = plasma->r0[j];
    if (!finite_pos(d) || !finite_pos(r)) return WAKE_EINVAL;
    if (j > 0 && !(r > plasma->r0[j - 1])) return WAKE_EINVAL;
    const double want = edge + 0.5 * d;
    if (std::fabs(r - want) > 1e-9 * want) return WAKE_EINVAL;
    if (plasma->dens && !finite_pos(plasma->dens[j])) return WAKE_EINVAL;
    edge += d;
  }
  return WAKE_OK;
}

// A new context with its stream (nothing allocated on the device yet).
static int ctx_new(wake_ctx** out, void* hip_stream) {
  wake_ctx* c = new (std::nothrow) wake_ctx();
  if (!c) return WAKE_ENOMEM;
  std::memset(&c->I, 0, sizeof(WakeInst));
  std::memset(&c->J, 0, sizeof(WakeIons));
  if (hipGetDevice(&c->device) != hipSuccess) { release(c); return WAKE_EDEVICE; }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      release(c);
      return WAKE_EDEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return WAKE_OK;
}

int ctx_create(wake_ctx** out, const wake_plasma* plasma, const wake_domain* dom, void* hip_stream,
               const Layout& L) {
  const int nt = L.nt;
  if (!out) return WAKE_EINVAL;
  if (!march_threads_ok(nt)) return WAKE_EINVAL;
  *out = nullptr;
  int rc = check_column(plasma, dom);
  if (rc != WAKE_OK) return rc;
  const int N = plasma->n_rings;
  wake_ctx* c = nullptr;
  rc = ctx_new(&c, hip_stream);
  if (rc != WAKE_OK) return rc;
  WakeInst& I = c->I;
  I.N = N;
  I.n_xi = dom->n_xi;
  I.stride = dom->record_stride;
  I.dxi = dom->dxi;
  I.Rp = plasma->r0[N - 1] + plasma->dr[N - 1] / 2.0;
  I.inv2pidxi = 1.0 / (2.0 * M_PI * I.dxi);
  I.nt = nt;
  layout_of(N, L, &I.C, &I.G);
  const size_t S = (size_t)I.G * I.C * I.nt;
  const size_t bytes = arena_bytes(N, I.n_xi, I.stride, L);
  hipError_t e = hipMalloc(&c->arena.base, bytes);
  if (e != hipSuccess) { c->arena.base = nullptr; release(c); return dev_err(e); }
  c->arena.size = bytes;
  Arena& A = c->arena;
  const size_t n_rec = I.stride > 0 ? (size_t)(I.n_xi + I.stride - 1) / I.stride : 0;
  I.cst = A.take<double>((size_t)2 * RC_CHUNKS * S);
  I.ion = A.take<double>((size_t)WAKE_ION_REC * (N + 1));
  I.tot0 = A.take<double>(4);
  for (int b = 0; b < 2; ++b) I.st[b] = A.take<double>((size_t)RS_DOUBLES * S);
  I.sc = A.take<double>((size_t)2 * SC_CHUNKS * S);
  I.a2 = A.take<double>(S);
  I.da2 = A.take<double>(S);
  I.perm = A.take<int32_t>(S);
  I.sm_r = A.take<double>(S);
  I.sm_i = A.take<int32_t>(S);
  I.flag = A.take<int32_t>(S);
  I.cls = A.take<int32_t>(S);
  for (int b = 0; b < 2; ++b) {
    I.sk_r[b] = A.take<double>(N);
    I.sk_i[b] = A.take<int32_t>(N);
    I.sk_s[b] = A.take<int32_t>(N);
  }
  I.free_slot = A.take<int32_t>(N);
  I.axis = A.take<double>(2 * (size_t)I.n_xi);
  I.snap = n_rec ? A.take<double>(n_rec * OUT_N * N) : nullptr;
  I.last = A.take<double>((size_t)OUT_N * N);
  I.ctl = A.take<int32_t>(CTL_NWORDS);
  I.cnt = A.take<unsigned long long>(CNT_N);
  c->staging = A.take<double>(4 * (size_t)N);
  if (I.G > 1) {
    const size_t P2 = pow2_at_least((size_t)N);
    I.xd = A.take<double>((size_t)2 * I.G * 17);   // packs and stamps
    I.xc = A.take<int32_t>(4);
    I.gk_r = A.take<double>(S);
    I.gk_i = A.take<int32_t>(S);
    I.bt_r = A.take<double>(P2);
    I.bt_i = A.take<int32_t>(P2);
    I.bt_s = A.take<int32_t>(P2);
  }
  if (A.used > A.size) { release(c); return WAKE_ENOMEM; }
  e = hipMalloc(&c->d_inst, sizeof(WakeInst));
  if (e == hipSuccess) e = hipMalloc(&c->d_counter, 64);
  if (e != hipSuccess) { release(c); return dev_err(e); }
  // upload the ring geometry into the staging area and build constants
  double* d_r0 = c->staging;
  double* d_dr = c->staging + N;
  double* d_dn = plasma->dens ? c->staging + 2 * (size_t)N : nullptr;
  e = hipMemcpyAsync(d_r0, plasma->r0, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_dr, plasma->dr, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && d_dn)
    e = hipMemcpyAsync(d_dn, plasma->dens, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(I.axis, 0, sizeof(double) * 2 * I.n_xi, c->stream);
  if (e == hipSuccess) e = launch_zero(reinterpret_cast<int32_t*>(I.cnt), 2 * CNT_N, c->stream);
  if (e == hipSuccess) e = launch_init(I, d_r0, d_dr, d_dn, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) { release(c); return dev_err(e); }
  *out = c;
  return WAKE_OK;
}

extern "C" int wake_create(wake_ctx** out, const wake_plasma* plasma, const wake_domain* dom,
                           void* hip_stream) {
  if (!plasma || plasma->n_rings <= 0) return out ? (*out = nullptr, WAKE_EINVAL) : WAKE_EINVAL;
  return ctx_create(out, plasma, dom, hip_stream, layout_for(plasma->n_rings));
}

// ---------------------------------------------------------------------------
// two-species contexts: plasma electrons and mobile ions
// ---------------------------------------------------------------------------
extern "C" int wake_create_mobile_ions(wake_ctx** out, const wake_plasma* plasma, double ion_mass,
                                       const wake_domain* dom, void* hip_stream) {
  if (!out) return WAKE_EINVAL;
  *out = nullptr;
  int rc = check_column(plasma, dom);
  if (rc != WAKE_OK) return rc;
  if (!finite_pos(ion_mass) || plasma->n_rings > WAKE_IONS_NMAX) return WAKE_EINVAL;
  const int N = plasma->n_rings;
  wake_ctx* c = nullptr;
  rc = ctx_new(&c, hip_stream);
  if (rc != WAKE_OK) return rc;
  c->two_species = true;
  WakeInst& I = c->I;
  WakeIons& J = c->J;
  I.N = J.N = N;
  I.n_xi = J.n_xi = dom->n_xi;
  I.stride = J.stride = dom->record_stride;
  I.dxi = J.dxi = dom->dxi;
  I.Rp = plasma->r0[N - 1] + plasma->dr[N - 1] / 2.0;
  I.inv2pidxi = 1.0 / (2.0 * M_PI * I.dxi);
  I.nt = WAKE_IONS_NT;
  I.G = 1;
  I.C = J.C = (N + WAKE_IONS_NT - 1) / WAKE_IONS_NT;
  J.m_i = ion_mass;
  const size_t S = (size_t)J.C * WAKE_IONS_NT;
  const size_t n_rec = I.stride > 0 ? (size_t)(I.n_xi + I.stride - 1) / I.stride : 0;
  // sizes first (a null arena only counts), then the real carve
  for (int pass = 0; pass < 2; ++pass) {
    Arena& A = c->arena;
    if (pass == 1) {
      const size_t bytes = A.used + 256;
      A = Arena();
      hipError_t e = hipMalloc(&A.base, bytes);
      if (e != hipSuccess) { A.base = nullptr; release(c); return dev_err(e); }
      A.size = bytes;
    }
    J.cst = A.take<double>((size_t)IK_N * N);
    for (int b = 0; b < 2; ++b) J.st[b] = A.take<double>((size_t)2 * IS_N * N);
    J.ord = A.take<int32_t>((size_t)2 * N);
    J.sid = A.take<int32_t>(2 * S);
    J.jx = A.take<int32_t>(2 * S);
    J.tab = A.take<double>((size_t)2 * IT_N * S);
    J.work = A.take<double>((size_t)2 * IW_N * S);
    J.axis = A.take<double>(2 * (size_t)I.n_xi);
    for (int sp = 0; sp < 2; ++sp) {
      J.snap[sp] = n_rec ? A.take<double>(n_rec * OUT_N * N) : nullptr;
      J.last[sp] = A.take<double>((size_t)OUT_N * N);
    }
    J.ctl = A.take<int32_t>(CTL_NWORDS);
    J.cnt = A.take<unsigned long long>(CNT_N);
    c->staging = A.take<double>(4 * (size_t)N);
  }
  // the electrons' outputs and the control words are read through I
  I.axis = J.axis;
  I.snap = J.snap[0];
  I.last = J.last[0];
  I.ctl = J.ctl;
  I.cnt = J.cnt;
  hipError_t e = hipMalloc(&c->d_J, sizeof(WakeIons));
  if (e != hipSuccess) { c->d_J = nullptr; release(c); return dev_err(e); }
  double* d_r0 = c->staging;
  double* d_dr = c->staging + N;
  double* d_dn = plasma->dens ? c->staging + 2 * (size_t)N : nullptr;
  e = hipMemcpyAsync(d_r0, plasma->r0, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_dr, plasma->dr, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && d_dn)
    e = hipMemcpyAsync(d_dn, plasma->dens, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(J.axis, 0, sizeof(double) * 2 * I.n_xi, c->stream);
  if (e == hipSuccess) e = launch_zero(reinterpret_cast<int32_t*>(J.cnt), 2 * CNT_N, c->stream);
  if (e == hipSuccess) e = ions_prepare();
  if (e == hipSuccess) e = launch_ions_init(J, d_r0, d_dr, d_dn, true, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) { release(c); return dev_err(e); }
  *out = c;
  return WAKE_OK;
}

// march a two-species context: its record (with the sources and beam table
// the context gathered in I) to the device, one workgroup
WakeIons ions_record(const wake_ctx* c, int first, int count) {
  WakeIons J = c->J;
  const WakeInst& I = c->I;
  J.first = first;
  J.count = count;
  J.nb = I.nb;
  J.n_an = I.n_an;
  J.has_laser = I.has_laser;
  for (int k = 0; k < WAKE_MAX_ANALYTIC; ++k) J.an[k] = I.an[k];
  J.boff = I.boff;
  J.br = I.br;
  J.bcum = I.bcum;
  return J;
}

static int ions_launch(wake_ctx* c, int first, int count) {
  c->J = ions_record(c, first, count);
  HIP_TRY(hipMemcpyAsync(c->d_J, &c->J, sizeof(WakeIons), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(launch_ions_march(c->d_J, 1, c->stream));
  return WAKE_OK;
}

extern "C" int wake_add_beam(wake_ctx* c, const wake_source* s) {
  if (!c || !s) return WAKE_EINVAL;
  if (c->prepared) return WAKE_ESTATE;
  WakeInst& I = c->I;
  if (s->kind == WAKE_BEAM_PARTICLES) {
    if (s->n < 0 || !std::isfinite(s->q)) return WAKE_EINVAL;
    if (s->n > 0 && (!s->x || !s->y || !s->xi || !s->w)) return WAKE_EINVAL;
    if ((int64_t)c->px.size() + s->n > (int64_t)1 << 29) return WAKE_EINVAL;
    for (int64_t k = 0; k < s->n; ++k)
      if (!std::isfinite(s->x[k]) || !std::isfinite(s->y[k]) || !std::isfinite(s->xi[k]) ||
          !std::isfinite(s->w[k]))
        return WAKE_EINVAL;
    try {
      c->px.insert(c->px.end(), s->x, s->x + s->n);
      c->py.insert(c->py.end(), s->y, s->y + s->n);
      c->pxi.insert(c->pxi.end(), s->xi, s->xi + s->n);
      c->pw.insert(c->pw.end(), s->w, s->w + s->n);
      c->pq.insert(c->pq.end(), (size_t)s->n, s->q);
    } catch (...) {
      return WAKE_ENOMEM;
    }
    return WAKE_OK;
  }
  if (s->kind != WAKE_BEAM_GAUSSIAN && s->kind != WAKE_LASER_GAUSSIAN) return WAKE_EINVAL;
  if (I.n_an >= WAKE_MAX_ANALYTIC) return WAKE_EINVAL;
  WakeAnalytic a;
  std::memset(&a, 0, sizeof(a));
  a.kind = s->kind;
  if (s->kind == WAKE_BEAM_GAUSSIAN) {
    if (!std::isfinite(s->q) || !std::isfinite(s->n_peak) || !finite_pos(s->sigma_r) ||
        !finite_pos(s->sigma_xi) || !std::isfinite(s->xi_c))
      return WAKE_EINVAL;
    a.q = s->q; a.n_peak = s->n_peak; a.sigma_r = s->sigma_r; a.sigma_xi = s->sigma_xi; a.xi_c = s->xi_c;
  } else {
    if (!std::isfinite(s->a0) || !finite_pos(s->w0) || !finite_pos(s->L) || !std::isfinite(s->xi_l))
      return WAKE_EINVAL;
    a.a0 = s->a0; a.w0 = s->w0; a.L = s->L; a.xi_l = s->xi_l;
    I.has_laser = 1;
  }
  I.an[I.n_an++] = a;
  return WAKE_OK;
}

// Carving of the persistent beam table (offsets per slice, then the radii
// and cumulative charges of up to ne entries) and of the build's scratch
// (particle copies, per-slice counts, padded entries).  With A.base null
// only the sizes are computed.
struct TableParts {
  int32_t* off;
  double *br, *bc;
};
static TableParts carve_table(Arena& A, int n_xi, int64_t ne) {
  TableParts t;
  t.off = A.take<int32_t>(n_xi + 1);
  t.br = A.take<double>(std::max<int64_t>(ne, 1));
  t.bc = A.take<double>(std::max<int64_t>(ne, 1));
  return t;
}
struct BuildParts {
  double *x, *y, *xi, *w, *q;
  int32_t *cnt, *cnt2, *cursor, *poff;
  double *er, *eq;
  int64_t* ek;
};
static BuildParts carve_build(Arena& A, int n_xi, int64_t np) {
  const int64_t npad = 4 * np + 4;      // power-of-two padded entries
  BuildParts b;
  b.x = A.take<double>(np);
  b.y = A.take<double>(np);
  b.xi = A.take<double>(np);
  b.w = A.take<double>(np);
  b.q = A.take<double>(np);
  b.cnt = A.take<int32_t>(n_xi + 1);
  b.cnt2 = A.take<int32_t>(n_xi + 1);
  b.cursor = A.take<int32_t>(n_xi + 1);
  b.poff = A.take<int32_t>(n_xi + 1);
  b.er = A.take<double>(npad);
  b.eq = A.take<double>(npad);
  b.ek = A.take<int64_t>(npad);
  return b;
}

// The beam table of a context (step a1) and the rest of wake_prepare.
// table / scratch: device memory for the table and for the build, or null
// to allocate them here (the table then belongs to the context, the
// scratch to this call).
static int prepare_impl(wake_ctx* c, char* table, size_t table_bytes, char* scratch,
                        size_t scratch_bytes) {
  HIP_TRY(hipSetDevice(c->device));
  WakeInst& I = c->I;
  const int64_t np = (int64_t)c->px.size();
  const int n_xi = I.n_xi;
  const int64_t ne = 2 * np;            // at most two nodes per particle
  Arena P;
  carve_table(P, n_xi, ne);
  const size_t pbytes = P.used + 256;
  Arena B;
  if (np > 0) carve_build(B, n_xi, np);
  const size_t tbytes = B.used + 256;
  if (table && table_bytes < pbytes) return WAKE_EINVAL;
  if (scratch && np > 0 && scratch_bytes < tbytes) return WAKE_EINVAL;
  char* tmp = nullptr;
  if (!table) {
    HIP_TRY(hipMalloc(&c->beam_mem, pbytes));
    c->beam_external = false;
  } else {
    c->beam_mem = table;
    c->beam_external = true;
  }
  P = Arena();
  P.base = c->beam_mem;
  P.size = pbytes;
  const TableParts T = carve_table(P, n_xi, ne);
  I.boff = T.off;
  I.br = T.br;
  I.bcum = T.bc;
  I.nb = (int32_t)ne;
  hipError_t e = hipSuccess;
  if (np > 0) {
    if (!scratch) {
      e = hipMalloc(&tmp, tbytes);
      if (e != hipSuccess) return dev_err(e);
    }
    B = Arena();
    B.base = scratch ? scratch : tmp;
    B.size = tbytes;
    const BuildParts b = carve_build(B, n_xi, np);
    const size_t sz = sizeof(double) * np;
    e = hipMemcpyAsync(b.x, c->px.data(), sz, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.y, c->py.data(), sz, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.xi, c->pxi.data(), sz, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.w, c->pw.data(), sz, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.q, c->pq.data(), sz, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = launch_beam_table(b.x, b.y, b.xi, b.w, b.q, np, I.dxi, n_xi, b.cnt, b.cnt2, b.cursor, T.off,
                            b.poff, b.er, b.eq, b.ek, T.br, T.bc, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return dev_err(e);
    // the table holds only entries that landed on a node
    int32_t total = 0;
    HIP_TRY(hipMemcpy(&total, I.boff + n_xi, sizeof(int32_t), hipMemcpyDeviceToHost));
    I.nb = total;
  } else {
    HIP_TRY(launch_zero(T.off, n_xi + 1, c->stream));
    I.nb = 0;
  }
  if (!table) {               // the particles' host copies are no longer needed
    std::vector<double>().swap(c->px);
    std::vector<double>().swap(c->py);
    std::vector<double>().swap(c->pxi);
    std::vector<double>().swap(c->pw);
    std::vector<double>().swap(c->pq);
  }
  if (!c->two_species) HIP_TRY(march_prepare(I.nt));   // the two-species marcher is set up at creation
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->prepared = true;
  return WAKE_OK;
}

extern "C" int wake_prepare(wake_ctx* c) {
  if (!c) return WAKE_EINVAL;
  if (c->prepared) return WAKE_OK;
  const int r = prepare_impl(c, nullptr, 0, nullptr, 0);
  if (r != WAKE_OK && c->beam_mem) {      // nothing of a failed attempt stays
    (void)hipFree(c->beam_mem);
    c->beam_mem = nullptr;
  }
  return r;
}

extern "C" int wake_prepare_noalloc(wake_ctx* c, void* table, int64_t table_bytes) {
  if (!c || !table || table_bytes <= 0) return WAKE_EINVAL;
  if (c->prepared) return WAKE_OK;
  if ((int64_t)c->px.size() > WAKE_NOALLOC_PARTICLES || c->I.n_xi > WAKE_NOALLOC_SLICES)
    return WAKE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  void* scr = nullptr;
  size_t scr_bytes = 0;
  HIP_TRY(beam_scratch(c->device, &scr, &scr_bytes));
  const int r = prepare_impl(c, static_cast<char*>(table), (size_t)table_bytes, static_cast<char*>(scr),
                             scr_bytes);
  if (r != WAKE_OK) {                     // the table stays the caller's
    c->beam_mem = nullptr;
    c->beam_external = false;
  }
  return r;
}

int drain(wake_ctx* c) {
  if (c->pending) {
    HIP_TRY(hipStreamSynchronize(c->pending));
    c->pending = nullptr;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return WAKE_OK;
}

static int read_ctl(wake_ctx* c, int32_t ctl[CTL_NWORDS]) {
  int r = drain(c);
  if (r != WAKE_OK) return r;
  HIP_TRY(hipMemcpy(ctl, c->I.ctl, sizeof(int32_t) * CTL_NWORDS, hipMemcpyDeviceToHost));
  return ctl[CTL_FAULT] ? WAKE_EDEVICE : WAKE_OK;
}

static int launch_one(wake_ctx* c, int first, int count) {
  WakeInst& I = c->I;
  I.first = first;
  I.count = count;
  I.task0 = 0;
  HIP_TRY(hipMemcpyAsync(c->d_inst, &I, sizeof(WakeInst), hipMemcpyHostToDevice, c->stream));
  const int mode = I.grid_n > 0 ? (I.grid_chi && !I.grid_off ? 2 : 1) : 0;
  HIP_TRY(launch_march(I.nt, c->d_inst, 1, I.G, c->d_counter, I.G, mode, c->stream));
  return WAKE_OK;
}

// Per-slice trace of a solve (WAKE_TRACE set in the environment: "1" or
// "stderr" writes to stderr, anything else names a file appended to): the
// solve marches one slice per launch, each timed with HIP events, and one
// line per slice gives the context, slice, GPU time, whether the slice began
// with an order fix-up and the breakdown slice.  Results are bitwise those of
// an untraced solve (launch splits do not change them).  Synchronous.
static int traced_solve(wake_ctx* c, int first, int count, const char* where) {
  FILE* f = (!std::strcmp(where, "1") || !std::strcmp(where, "stderr")) ? stderr : std::fopen(where, "a");
  if (!f) return WAKE_EINVAL;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int r = WAKE_OK;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  for (int n = first; he == hipSuccess && r == WAKE_OK && n < first + count; ++n) {
    unsigned long long fx0 = 0, fx1 = 0;
    he = hipMemcpy(&fx0, c->I.cnt + CNT_FIXUPS, sizeof(fx0), hipMemcpyDeviceToHost);
    if (he == hipSuccess) he = hipEventRecord(e0, c->stream);
    if (he != hipSuccess) break;
    r = c->two_species ? ions_launch(c, n, 1) : launch_one(c, n, 1);
    if (r != WAKE_OK) break;
    he = hipEventRecord(e1, c->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    int32_t ctl[CTL_NWORDS];
    if (he == hipSuccess) he = hipMemcpy(ctl, c->I.ctl, sizeof(ctl), hipMemcpyDeviceToHost);
    if (he == hipSuccess) he = hipMemcpy(&fx1, c->I.cnt + CNT_FIXUPS, sizeof(fx1), hipMemcpyDeviceToHost);
    if (he != hipSuccess) break;
    std::fprintf(f, "wake_trace ctx=%p rings=%d slice=%d us=%.2f fixup=%llu breakdown=%d\n", (void*)c,
                 c->I.N, n, ms * 1e3, fx1 - fx0, ctl[CTL_BREAK]);
    if (ctl[CTL_BREAK] >= 0) break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (f != stderr) std::fclose(f);
  else std::fflush(f);
  if (he != hipSuccess) return dev_err(he);
  return r;
}

extern "C" int wake_solve(wake_ctx* c, int32_t first, int32_t count) {
  if (!c) return WAKE_EINVAL;
  if (count < 0 || first < 0 || (int64_t)first + count > c->I.n_xi) return WAKE_EINVAL;
  if (first != c->next) return WAKE_ESTATE;
  if (count == 0) return WAKE_OK;
  HIP_TRY(hipSetDevice(c->device));
  int r = drain(c);
  if (r != WAKE_OK) return r;
  r = wake_prepare(c);
  if (r != WAKE_OK) return r;
  const char* trace = std::getenv("WAKE_TRACE");
  if (trace && *trace)
    r = traced_solve(c, first, count, trace);
  else
    r = c->two_species ? ions_launch(c, first, count) : launch_one(c, first, count);
  if (r != WAKE_OK) return r;
  c->next = first + count;
  return WAKE_OK;
}

extern "C" int wake_counters(wake_ctx* c, int64_t* out, int32_t n, int32_t reset) {
  if (!c || n < 0 || (n > 0 && !out)) return WAKE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  int r = drain(c);
  if (r != WAKE_OK) return r;
  unsigned long long h[CNT_N];
  HIP_TRY(hipMemcpy(h, c->I.cnt, sizeof(h), hipMemcpyDeviceToHost));
  for (int i = 0; i < n && i < CNT_N; ++i) out[i] = (int64_t)h[i];
  for (int i = CNT_N; i < n; ++i) out[i] = 0;
  if (reset) {
    HIP_TRY(launch_zero(reinterpret_cast<int32_t*>(c->I.cnt), 2 * CNT_N, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return WAKE_OK;
}

extern "C" int wake_sync(wake_ctx* c) {
  if (!c) return WAKE_EINVAL;
  return drain(c);
}

extern "C" int wake_status(wake_ctx* c, int32_t* brk, int32_t* next) {
  if (!c) return WAKE_EINVAL;
  int32_t ctl[CTL_NWORDS];
  int r = read_ctl(c, ctl);
  if (r != WAKE_OK) return r;
  if (ctl[CTL_BREAK] >= 0) c->next = ctl[CTL_NEXT];
  if (brk) *brk = ctl[CTL_BREAK];
  if (next) *next = ctl[CTL_BREAK] >= 0 ? ctl[CTL_NEXT] : c->next;
  return WAKE_OK;
}

static int copy_out(double* dst, const double* src, size_t n, int dev, hipStream_t s) {
  if (!dst) return WAKE_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, sizeof(double) * n,
                         dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  return WAKE_OK;
}

// Recorded fields of one species (snapshots snap, last slice last).
static int fields_of(wake_ctx* c, const double* snap, const double* last, int32_t slice, double* psi,
                     double* erbt, double* ez, double* bt, double* rho, double* ur, int32_t dev) {
  const WakeInst& I = c->I;
  int32_t ctl[CTL_NWORDS];
  int r = read_ctl(c, ctl);
  if (r != WAKE_OK) return r;
  const int brk = ctl[CTL_BREAK];
  const double* base;
  if (slice == -1) {
    if (c->next == 0 && brk < 0) return WAKE_ESTATE;
    if (brk >= 0) return WAKE_EBREAKDOWN;
    base = last;
  } else {
    if (slice < 0 || slice >= I.n_xi) return WAKE_EINVAL;
    if (brk >= 0 && slice >= brk) return WAKE_EBREAKDOWN;
    if (slice >= c->next || slice < c->valid_from) return WAKE_ESTATE;
    if (I.stride <= 0 || slice % I.stride != 0) return WAKE_ENOTREC;
    base = snap + (size_t)(slice / I.stride) * OUT_N * I.N;
  }
  const size_t N = I.N;
  double* outs[OUT_N] = {psi, erbt, ez, bt, rho, ur};
  for (int q = 0; q < OUT_N; ++q) {
    r = copy_out(outs[q], base + q * N, N, dev, c->stream);
    if (r != WAKE_OK) return r;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return WAKE_OK;
}

extern "C" int wake_fields(wake_ctx* c, int32_t slice, double* psi, double* erbt, double* ez,
                           double* bt, double* rho, double* ur, int32_t dev) {
  if (!c) return WAKE_EINVAL;
  return fields_of(c, c->I.snap, c->I.last, slice, psi, erbt, ez, bt, rho, ur, dev);
}

extern "C" int wake_species_fields(wake_ctx* c, int32_t species, int32_t slice, double* psi,
                                   double* erbt, double* ez, double* bt, double* rho, double* ur,
                                   int32_t dev) {
  if (!c || species < 0 || species > 1 || (species == 1 && !c->two_species)) return WAKE_EINVAL;
  if (species == 0) return wake_fields(c, slice, psi, erbt, ez, bt, rho, ur, dev);
  return fields_of(c, c->J.snap[1], c->J.last[1], slice, psi, erbt, ez, bt, rho, ur, dev);
}

// Drop a context's field grid (device memory released).
static int grid_clear(wake_ctx* c) {
  WakeInst& I = c->I;
  if (c->grid_mem) {
    HIP_TRY(hipFree(c->grid_mem));
    c->grid_mem = nullptr;
  }
  c->grid_off_h.clear();
  I.grid_n = 0;
  I.grid_dr = 0.0;
  I.grid = nullptr;
  I.grid_tab = nullptr;
  I.grid_scr = nullptr;
  I.grid_rad = nullptr;
  I.grid_off = nullptr;
  I.grid_thr = nullptr;
  return WAKE_OK;
}

// Common set-up of a field grid: n_fields node-slices of fields (5 doubles
// each: psi, E_r - B_theta, E_z, B_theta, chi), n_tab node records,
// hand-over scratch for max_nodes nodes of a slice and the virtual node above
// them (12 doubles each), the chi deposit's per-thread sums (4 doubles per
// thread of the instance), extra doubles for radii and int32 words for
// offsets copied in.  Unmarched slices read as NaN.  The caller fills the
// radii / offsets and then calls grid_finish.
static int grid_alloc(wake_ctx* c, size_t n_fields, size_t n_tab, int max_nodes, size_t n_rad,
                      size_t n_off, double** rad, int32_t** off) {
  WakeInst& I = c->I;
  const size_t n_scr = 12 * ((size_t)max_nodes + 1);
  const size_t n_thr = 4 * (size_t)I.nt * (size_t)I.G;
  const size_t nd = 5 * n_fields + WAKE_GRID_TAB * n_tab + n_scr + n_thr + n_rad + (n_off + 1) / 2;
  HIP_TRY(hipMalloc(&c->grid_mem, sizeof(double) * nd));
  I.grid_n = max_nodes;
  I.grid = c->grid_mem;
  I.grid_tab = c->grid_mem + 5 * n_fields;
  I.grid_scr = c->grid_mem + 5 * n_fields + WAKE_GRID_TAB * n_tab;
  I.grid_thr = I.grid_scr + n_scr;
  double* tail = I.grid_thr + n_thr;
  *rad = n_rad ? tail : nullptr;
  *off = n_off ? reinterpret_cast<int32_t*>(tail + n_rad) : nullptr;
  HIP_TRY(hipMemsetAsync(c->grid_mem, 0xFF, sizeof(double) * 5 * n_fields, c->stream));
  HIP_TRY(hipMemsetAsync(I.grid_scr, 0, sizeof(double) * (n_scr + n_thr), c->stream));
  return WAKE_OK;
}

static int grid_finish(wake_ctx* c, size_t n_tab) {
  WakeInst& I = c->I;
  HIP_TRY(launch_grid_init(I, const_cast<double*>(I.grid_tab), (int)n_tab, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return WAKE_OK;
}

// checks shared by the grid set-up calls
static int grid_begin(wake_ctx* c) {
  if (!c || c->two_species) return WAKE_EINVAL;
  if (c->next != 0 || c->batches > 0) return WAKE_ESTATE;
  HIP_TRY(hipSetDevice(c->device));
  int r = drain(c);
  if (r != WAKE_OK) return r;
  return grid_clear(c);
}

extern "C" int wake_set_grid(wake_ctx* c, int32_t n_r, double r_max) {
  if (!c || c->two_species) return WAKE_EINVAL;
  if (n_r < 0 || n_r > (1 << 20) || (n_r > 0 && !finite_pos(r_max))) return WAKE_EINVAL;
  int r = grid_begin(c);
  if (r != WAKE_OK) return r;
  if (n_r == 0) return WAKE_OK;
  WakeInst& I = c->I;
  double* rad;
  int32_t* off;
  r = grid_alloc(c, (size_t)n_r * (size_t)I.n_xi, n_r, n_r, 0, 0, &rad, &off);
  if (r != WAKE_OK) { grid_clear(c); return r; }
  I.grid_dr = r_max / (double)n_r;
  r = grid_finish(c, n_r);
  if (r != WAKE_OK) grid_clear(c);
  return r;
}

extern "C" int wake_set_grid_radii(wake_ctx* c, int64_t n_nodes, const double* radii,
                                   const int64_t* slice_off) {
  if (!c || c->two_species) return WAKE_EINVAL;
  if (n_nodes < 0 || (n_nodes > 0 && !radii)) return WAKE_EINVAL;
  const int n_xi = c->I.n_xi;
  int max_nodes = 0;
  if (!slice_off) {
    if (n_nodes > (1 << 20)) return WAKE_EINVAL;
    for (int64_t g = 0; g < n_nodes; ++g)
      if (!finite_pos(radii[g]) || (g > 0 && !(radii[g] > radii[g - 1]))) return WAKE_EINVAL;
    max_nodes = (int)n_nodes;
  } else {
    if (n_nodes > (1 << 28) || slice_off[0] != 0 || slice_off[n_xi] != n_nodes) return WAKE_EINVAL;
    for (int n = 0; n < n_xi; ++n) {
      const int64_t k0 = slice_off[n], k1 = slice_off[n + 1];
      if (k1 < k0 || k1 - k0 > (1 << 20)) return WAKE_EINVAL;
      for (int64_t g = k0; g < k1; ++g)
        if (!finite_pos(radii[g]) || (g > k0 && radii[g] < radii[g - 1])) return WAKE_EINVAL;
      max_nodes = std::max(max_nodes, (int)(k1 - k0));
    }
  }
  int r = grid_begin(c);
  if (r != WAKE_OK) return r;
  if (n_nodes == 0) return WAKE_OK;
  WakeInst& I = c->I;
  const size_t n_fields = slice_off ? (size_t)n_nodes : (size_t)n_nodes * (size_t)n_xi;
  double* rad;
  int32_t* off;
  r = grid_alloc(c, n_fields, (size_t)n_nodes, max_nodes, (size_t)n_nodes,
                 slice_off ? (size_t)n_xi + 1 : 0, &rad, &off);
  if (r != WAKE_OK) { grid_clear(c); return r; }
  hipError_t e = hipMemcpyAsync(rad, radii, sizeof(double) * n_nodes, hipMemcpyHostToDevice, c->stream);
  I.grid_rad = rad;
  if (slice_off && e == hipSuccess) {
    try {
      c->grid_off_h.assign(slice_off, slice_off + n_xi + 1);
    } catch (...) {
      grid_clear(c);
      return WAKE_ENOMEM;
    }
    e = hipMemcpyAsync(off, c->grid_off_h.data(), sizeof(int32_t) * (n_xi + 1), hipMemcpyHostToDevice,
                       c->stream);
    I.grid_off = off;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) { grid_clear(c); return dev_err(e); }
  r = grid_finish(c, (size_t)n_nodes);
  if (r != WAKE_OK) grid_clear(c);
  return r;
}

extern "C" int wake_set_grid_beam(wake_ctx* c) {
  if (!c || c->two_species) return WAKE_EINVAL;
  if (c->next != 0 || c->batches > 0) return WAKE_ESTATE;
  int r = wake_prepare(c);                        // the beam table is the node set
  if (r != WAKE_OK) return r;
  r = grid_begin(c);
  if (r != WAKE_OK) return r;
  WakeInst& I = c->I;
  if (I.nb <= 0) return WAKE_EINVAL;
  try {
    c->grid_off_h.resize((size_t)I.n_xi + 1);
  } catch (...) {
    return WAKE_ENOMEM;
  }
  HIP_TRY(hipMemcpy(c->grid_off_h.data(), I.boff, sizeof(int32_t) * (I.n_xi + 1), hipMemcpyDeviceToHost));
  int max_nodes = 0;
  for (int n = 0; n < I.n_xi; ++n) max_nodes = std::max(max_nodes, c->grid_off_h[n + 1] - c->grid_off_h[n]);
  double* rad;
  int32_t* off;
  r = grid_alloc(c, (size_t)I.nb, (size_t)I.nb, max_nodes, 0, 0, &rad, &off);
  if (r != WAKE_OK) { grid_clear(c); return r; }
  I.grid_rad = I.br;
  I.grid_off = I.boff;
  r = grid_finish(c, (size_t)I.nb);
  if (r != WAKE_OK) grid_clear(c);
  return r;
}

// first entry and node count of a slice's grid nodes
static void grid_slice(const wake_ctx* c, int slice, size_t* first, size_t* count) {
  if (c->grid_off_h.empty()) {
    *first = (size_t)slice * (size_t)c->I.grid_n;
    *count = (size_t)c->I.grid_n;
  } else {
    *first = (size_t)c->grid_off_h[slice];
    *count = (size_t)(c->grid_off_h[slice + 1] - c->grid_off_h[slice]);
  }
}

extern "C" int wake_grid_nodes(wake_ctx* c, int32_t slice, int64_t* count, double* radii) {
  if (!c || !count) return WAKE_EINVAL;
  const WakeInst& I = c->I;
  if (!c->grid_mem) return WAKE_ESTATE;
  if (slice < 0 || slice >= I.n_xi) return WAKE_EINVAL;
  size_t first, cnt;
  grid_slice(c, slice, &first, &cnt);
  *count = (int64_t)cnt;
  if (!radii || cnt == 0) return WAKE_OK;
  if (!I.grid_rad) {
    for (size_t g = 0; g < cnt; ++g) radii[g] = ((double)g + 0.5) * I.grid_dr;
    return WAKE_OK;
  }
  HIP_TRY(hipSetDevice(c->device));
  int r = drain(c);
  if (r != WAKE_OK) return r;
  const double* src = I.grid_rad + (c->grid_off_h.empty() ? 0 : first);
  HIP_TRY(hipMemcpy(radii, src, sizeof(double) * cnt, hipMemcpyDeviceToHost));
  return WAKE_OK;
}

extern "C" int wake_grid_fields(wake_ctx* c, int32_t slice, double* psi, double* erbt, double* ez,
                                double* bt, int32_t dev) {
  if (!c) return WAKE_EINVAL;
  const WakeInst& I = c->I;
  if (!c->grid_mem) return WAKE_ESTATE;
  int32_t ctl[CTL_NWORDS];
  int r = read_ctl(c, ctl);
  if (r != WAKE_OK) return r;
  const int brk = ctl[CTL_BREAK];
  if (slice == -1) {
    if (brk >= 0) return WAKE_EBREAKDOWN;
    if (c->next == 0) return WAKE_ESTATE;
    slice = c->next - 1;
  }
  if (slice < 0 || slice >= I.n_xi) return WAKE_EINVAL;
  if (brk >= 0 && slice >= brk) return WAKE_EBREAKDOWN;
  if (slice >= c->next || slice < c->valid_from) return WAKE_ESTATE;
  size_t first, ng;
  grid_slice(c, slice, &first, &ng);
  const double* base = I.grid + 5 * first;
  double* outs[4] = {psi, erbt, ez, bt};
  for (int q = 0; q < 4; ++q) {
    r = copy_out(outs[q], base + q * ng, ng, dev, c->stream);
    if (r != WAKE_OK) return r;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return WAKE_OK;
}

extern "C" int wake_set_grid_chi(wake_ctx* c, int32_t on) {
  if (!c || c->two_species) return WAKE_EINVAL;
  if (c->next != 0 || c->batches > 0) return WAKE_ESTATE;
  HIP_TRY(hipSetDevice(c->device));
  int r = drain(c);
  if (r != WAKE_OK) return r;
  c->I.grid_chi = on ? 1 : 0;
  return WAKE_OK;
}

extern "C" int wake_grid_chi(wake_ctx* c, int32_t slice, double* chi, int32_t dev) {
  if (!c) return WAKE_EINVAL;
  const WakeInst& I = c->I;
  if (!c->grid_mem || !c->grid_off_h.empty() || !I.grid_chi) return WAKE_ESTATE;
  int32_t ctl[CTL_NWORDS];
  int r = read_ctl(c, ctl);
  if (r != WAKE_OK) return r;
  const int brk = ctl[CTL_BREAK];
  if (slice == -1) {
    if (brk >= 0) return WAKE_EBREAKDOWN;
    if (c->next == 0) return WAKE_ESTATE;
    slice = c->next - 1;
  }
  if (slice < 0 || slice >= I.n_xi) return WAKE_EINVAL;
  if (brk >= 0 && slice >= brk) return WAKE_EBREAKDOWN;
  if (slice >= c->next || slice < c->valid_from) return WAKE_ESTATE;
  size_t first, ng;
  grid_slice(c, slice, &first, &ng);
  r = copy_out(chi, I.grid + 5 * first + 4 * ng, ng, dev, c->stream);
  if (r != WAKE_OK) return r;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return WAKE_OK;
}

extern "C" int wake_lineout(wake_ctx* c, double* psi_axis, double* ez_axis, int32_t dev) {
  if (!c) return WAKE_EINVAL;
  int r = drain(c);
  if (r != WAKE_OK) return r;
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const size_t n = c->I.n_xi;
  if (psi_axis)
    HIP_TRY(hipMemcpy2DAsync(psi_axis, sizeof(double), c->I.axis, 2 * sizeof(double), sizeof(double),
                             n, kind, c->stream));
  if (ez_axis)
    HIP_TRY(hipMemcpy2DAsync(ez_axis, sizeof(double), c->I.axis + 1, 2 * sizeof(double),
                             sizeof(double), n, kind, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return WAKE_OK;
}

// Ring state of species sp (0: electrons; 1: the ions of a two-species
// context) at the next slice.
static int get_state_of(wake_ctx* c, int sp, int32_t* slice, double* rho, double* ur, double* f_rho,
                        double* f_u, int32_t dev) {
  int32_t brk = -1, next = 0;
  int r = wake_status(c, &brk, &next);
  if (r != WAKE_OK) return r;
  const size_t N = c->I.N;
  double* st = c->staging;
  if (c->two_species)
    HIP_TRY(launch_ions_get_state(c->J, sp, st, c->stream));
  else
    HIP_TRY(launch_state_by_id(c->I, st, st + N, st + 2 * N, st + 3 * N, c->stream));
  double* outs[4] = {rho, ur, f_rho, f_u};
  for (int q = 0; q < 4; ++q) {
    r = copy_out(outs[q], st + q * N, N, dev, c->stream);
    if (r != WAKE_OK) return r;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (slice) *slice = next;
  return WAKE_OK;
}

static int set_state_of(wake_ctx* c, int sp, int32_t slice, const double* rho, const double* ur,
                        const double* f_rho, const double* f_u, int32_t dev) {
  if (!rho || !ur) return WAKE_EINVAL;
  if (slice < 0 || slice >= c->I.n_xi) return WAKE_EINVAL;
  const size_t N = c->I.N;
  if (!dev) {
    for (size_t i = 0; i < N; ++i)
      if (!finite_pos(rho[i]) || !std::isfinite(ur[i])) return WAKE_EINVAL;
  }
  HIP_TRY(hipSetDevice(c->device));
  int r = drain(c);
  if (r != WAKE_OK) return r;
  double* st = c->staging;
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIP_TRY(hipMemcpyAsync(st, rho, sizeof(double) * N, kind, c->stream));
  HIP_TRY(hipMemcpyAsync(st + N, ur, sizeof(double) * N, kind, c->stream));
  if (f_rho) HIP_TRY(hipMemcpyAsync(st + 2 * N, f_rho, sizeof(double) * N, kind, c->stream));
  if (f_u) HIP_TRY(hipMemcpyAsync(st + 3 * N, f_u, sizeof(double) * N, kind, c->stream));
  if (c->two_species)
    HIP_TRY(launch_ions_set_state(c->J, sp, st, st + N, f_rho ? st + 2 * N : nullptr,
                                  f_u ? st + 3 * N : nullptr, slice, c->stream));
  else
    HIP_TRY(launch_state_set(c->I, st, st + N, f_rho ? st + 2 * N : nullptr,
                             f_u ? st + 3 * N : nullptr, slice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->next = slice;
  c->valid_from = slice;
  return WAKE_OK;
}

extern "C" int wake_get_state(wake_ctx* c, int32_t* slice, double* rho, double* ur, double* f_rho,
                              double* f_u, int32_t dev) {
  if (!c) return WAKE_EINVAL;
  return get_state_of(c, 0, slice, rho, ur, f_rho, f_u, dev);
}

extern "C" int wake_set_state(wake_ctx* c, int32_t slice, const double* rho, const double* ur,
                              const double* f_rho, const double* f_u, int32_t dev) {
  if (!c) return WAKE_EINVAL;
  return set_state_of(c, 0, slice, rho, ur, f_rho, f_u, dev);
}

extern "C" int wake_get_species_state(wake_ctx* c, int32_t species, int32_t* slice, double* rho,
                                      double* ur, double* f_rho, double* f_u, int32_t dev) {
  if (!c || species < 0 || species > 1 || (species == 1 && !c->two_species)) return WAKE_EINVAL;
  return get_state_of(c, species, slice, rho, ur, f_rho, f_u, dev);
}

extern "C" int wake_set_species_state(wake_ctx* c, int32_t species, int32_t slice, const double* rho,
                                      const double* ur, const double* f_rho, const double* f_u,
                                      int32_t dev) {
  if (!c || species < 0 || species > 1 || (species == 1 && !c->two_species)) return WAKE_EINVAL;
  return set_state_of(c, species, slice, rho, ur, f_rho, f_u, dev);
}

extern "C" int wake_reset(wake_ctx* c) {
  if (!c) return WAKE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  int r = drain(c);
  if (r != WAKE_OK) return r;
  if (c->two_species) {
    HIP_TRY(launch_ions_init(c->J, nullptr, nullptr, nullptr, false, c->stream));
  } else {
    HIP_TRY(hipMemcpyAsync(c->d_inst, &c->I, sizeof(WakeInst), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_reset(c->d_inst, 1, c->stream));
  }
  c->next = 0;
  c->valid_from = 0;
  return WAKE_OK;
}

// ---------------------------------------------------------------------------
// tiling: workgroup threads (fixed per context at creation) and workgroups
// per compute unit of persistent launches
// ---------------------------------------------------------------------------
static const int kThreads[] = {256, 512};

extern "C" int wake_tiling_count(void) { return 2; }

extern "C" int wake_tiling_get(int32_t idx, int32_t* nt, int32_t* wpc) {
  if (!nt || !wpc || idx < 0 || idx >= 2) return WAKE_EINVAL;
  *nt = kThreads[idx];
  *wpc = march_occupancy(kThreads[idx]);
  return WAKE_OK;
}

extern "C" int wake_set_tiling(int32_t nt, int32_t wpc) {
  if (!march_threads_ok(nt) || wpc < 0 || wpc > 32) return WAKE_EINVAL;
  HIP_TRY(march_prepare(nt));
  g_nt = nt;
  g_wpc = wpc;
  return WAKE_OK;
}

extern "C" int wake_set_cluster(int32_t rings_per_thread, int32_t min_rings) {
  if (rings_per_thread < 0 || rings_per_thread > 4096 || min_rings < 0) return WAKE_EINVAL;
  g_cl_rings = rings_per_thread;
  g_cl_min = min_rings;
  return WAKE_OK;
}

extern "C" int wake_get_layout(wake_ctx* c, int32_t* workgroups, int32_t* rings_per_thread) {
  if (!c) return WAKE_EINVAL;
  if (workgroups) *workgroups = c->I.G;
  if (rings_per_thread) *rings_per_thread = c->I.C;
  return WAKE_OK;
}

extern "C" int wake_get_tiling(int32_t* nt, int32_t* wpc) {
  if (!nt || !wpc) return WAKE_EINVAL;
  *nt = g_nt;
  *wpc = g_wpc;
  return WAKE_OK;
}

extern "C" int wake_tiling_occupancy(int32_t nt, int32_t wpc) {
  (void)wpc;
  if (!march_threads_ok(nt)) return WAKE_EINVAL;
  if (march_prepare(nt) != hipSuccess) return WAKE_EDEVICE;
  return march_occupancy(nt);
}

// persistent grid for nt-thread workgroups
int march_grid(int nt, int n_insts, int dev) {
  const int occ = std::max(1, march_occupancy(nt));
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
    cu = 1;
  const int wpc = g_wpc > 0 ? std::min(g_wpc, occ) : occ;
  return std::max(1, std::min(n_insts, wpc * cu));
}

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
static void batch_release(wake_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_insts) (void)hipFree(b->d_insts);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->d_ginsts) (void)hipFree(b->d_ginsts);
  if (b->d_gcounter) (void)hipFree(b->d_gcounter);
  if (b->d_jinsts) (void)hipFree(b->d_jinsts);
  if (b->d_gjinsts) (void)hipFree(b->d_gjinsts);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  if (b->holds)
    for (wake_ctx* c : b->ctxs) --c->batches;
  delete b;
}

extern "C" void wake_batch_destroy(wake_batch* b) { batch_release(b); }

extern "C" int wake_batch_create(wake_batch** out, wake_ctx* const* ctxs, int32_t n, void* stream) {
  if (!out) return WAKE_EINVAL;
  *out = nullptr;
  if (!ctxs || n <= 0) return WAKE_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return WAKE_EINVAL;
  wake_batch* b = new (std::nothrow) wake_batch();
  if (!b) return WAKE_ENOMEM;
  b->device = ctxs[0]->device;
  for (int i = 0; i < n; ++i) {
    if (ctxs[i]->device != b->device) { batch_release(b); return WAKE_EINVAL; }
    int r = wake_prepare(ctxs[i]);
    if (r != WAKE_OK) { batch_release(b); return r; }
  }
  b->ctxs.assign(ctxs, ctxs + n);
  if (stream) {
    b->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      batch_release(b);
      return WAKE_EDEVICE;
    }
    b->own_stream = true;
  }
  b->cap = n;
  if (hipMalloc(&b->d_insts, sizeof(WakeInst) * n) != hipSuccess ||
      hipMalloc(&b->d_counter, 64) != hipSuccess ||
      hipMalloc(&b->d_ginsts, sizeof(WakeInst) * n) != hipSuccess ||
      hipMalloc(&b->d_gcounter, 64) != hipSuccess ||
      hipMalloc(&b->d_jinsts, sizeof(WakeIons) * n) != hipSuccess ||
      hipMalloc(&b->d_gjinsts, sizeof(WakeIons) * n) != hipSuccess) {
    batch_release(b);
    return WAKE_ENOMEM;
  }
  for (wake_ctx* c : b->ctxs) ++c->batches;
  b->holds = true;
  *out = b;
  return WAKE_OK;
}

// Fill the device descriptor array with (first, count) per instance, longest
// first.  Returns the number of instances with work.
static int batch_stage(wake_batch* b, int32_t n_slices, bool from_zero, std::vector<WakeInst>& v,
                       std::vector<WakeIons>& vj) {
  v.clear();
  vj.clear();
  for (wake_ctx* c : b->ctxs) {
    const int first = from_zero ? 0 : c->next;
    int count = c->I.n_xi - first;
    if (n_slices >= 0) count = std::min(count, (int)n_slices);
    if (count <= 0) continue;
    if (c->two_species) {
      vj.push_back(ions_record(c, first, count));
      continue;
    }
    WakeInst I = c->I;
    I.first = first;
    I.count = count;
    v.push_back(I);
  }
  std::stable_sort(v.begin(), v.end(), [](const WakeInst& a, const WakeInst& c) {
    return (int64_t)a.N * a.count > (int64_t)c.N * c.count;
  });
  std::stable_sort(vj.begin(), vj.end(), [](const WakeIons& a, const WakeIons& c) {
    return (int64_t)a.N * a.count > (int64_t)c.N * c.count;
  });
  assign_tasks(v);
  return (int)(v.size() + vj.size());
}

// one persistent launch per distinct workgroup size present in v (the
// descriptors are already at d_insts; each launch takes the instances of its
// size from the shared queue)
int assign_tasks(std::vector<WakeInst>& v) {
  int t = 0;
  for (WakeInst& I : v) {
    I.task0 = t;
    t += I.G;
  }
  return t;
}

// (task0 already assigned; a cooperative instance's members need their G
// workgroups resident together, so the grid never drops below the largest G)
hipError_t launch_insts(const std::vector<WakeInst>& v, const WakeInst* d_insts, int32_t* d_counter,
                        int dev, int grid_override, hipStream_t s) {
  int n_tasks = 0;
  for (const WakeInst& I : v) n_tasks += I.G;
  for (int nt : kThreads) {
    int n = 0, gmax = 1;
    int mode = 0;
    for (const WakeInst& I : v)
      if (I.nt == nt) {
        n += I.G;
        gmax = std::max(gmax, (int)I.G);
        if (I.grid_n > 0) mode = std::max(mode, I.grid_chi && !I.grid_off ? 2 : 1);
      }
    if (n == 0) continue;
    int g = grid_override > 0 ? std::min(grid_override, n) : march_grid(nt, n, dev);
    g = std::max(g, gmax);
    hipError_t e = launch_march(nt, d_insts, (int)v.size(), n_tasks, d_counter, g, mode, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// the one-species persistent launches, then one workgroup per two-species
// instance (longest first)
static hipError_t batch_launch(wake_batch* b, const std::vector<WakeInst>& v,
                               const std::vector<WakeIons>& vj, int grid_override, bool graph) {
  if (!v.empty()) {
    hipError_t e = launch_insts(v, graph ? b->d_ginsts : b->d_insts, graph ? b->d_gcounter : b->d_counter,
                                b->device, grid_override, b->stream);
    if (e != hipSuccess) return e;
  }
  if (!vj.empty()) return launch_ions_march(graph ? b->d_gjinsts : b->d_jinsts, (int)vj.size(), b->stream);
  return hipSuccess;
}

extern "C" int wake_batch_solve(wake_batch* b, int32_t n_slices) {
  if (!b) return WAKE_EINVAL;
  HIP_TRY(hipSetDevice(b->device));
  for (wake_ctx* c : b->ctxs) {
    int r = drain(c);
    if (r != WAKE_OK) return r;
  }
  std::vector<WakeInst> v;
  std::vector<WakeIons> vj;
  const int n = batch_stage(b, n_slices, false, v, vj);
  if (n == 0) return WAKE_OK;
  if (!v.empty())
    HIP_TRY(hipMemcpyAsync(b->d_insts, v.data(), sizeof(WakeInst) * v.size(), hipMemcpyHostToDevice,
                           b->stream));
  if (!vj.empty())
    HIP_TRY(hipMemcpyAsync(b->d_jinsts, vj.data(), sizeof(WakeIons) * vj.size(), hipMemcpyHostToDevice,
                           b->stream));
  HIP_TRY(batch_launch(b, v, vj, 0, false));
  for (wake_ctx* c : b->ctxs) {
    int count = c->I.n_xi - c->next;
    if (n_slices >= 0) count = std::min(count, (int)n_slices);
    if (count > 0) c->next += count;
    c->pending = b->stream;
  }
  return WAKE_OK;
}

extern "C" int wake_batch_capture(wake_batch* b, int32_t grid) {
  if (!b) return WAKE_EINVAL;
  HIP_TRY(hipSetDevice(b->device));
  for (wake_ctx* c : b->ctxs) {
    int r = drain(c);
    if (r != WAKE_OK) return r;
  }
  std::vector<WakeInst> v;
  std::vector<WakeIons> vj;
  const int n = batch_stage(b, -1, true, v, vj);
  if (n == 0) return WAKE_EINVAL;
  // the graph reads descriptors of its own: eager solves of the batch
  // between a capture and its replays rewrite only d_insts / d_jinsts
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (!v.empty())
    HIP_TRY(hipMemcpy(b->d_ginsts, v.data(), sizeof(WakeInst) * v.size(), hipMemcpyHostToDevice));
  if (!vj.empty())
    HIP_TRY(hipMemcpy(b->d_gjinsts, vj.data(), sizeof(WakeIons) * vj.size(), hipMemcpyHostToDevice));
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  if (!v.empty()) e = launch_reset(b->d_ginsts, (int)v.size(), b->stream);
  if (e == hipSuccess && !vj.empty()) e = launch_ions_reset(b->d_gjinsts, (int)vj.size(), b->stream);
  if (e == hipSuccess) e = batch_launch(b, v, vj, grid, true);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return dev_err(e != hipSuccess ? e : e2);
  }
  b->graph = graph;
  HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  for (wake_ctx* c : b->ctxs) {
    c->next = 0;
    c->valid_from = 0;
  }
  return WAKE_OK;
}

extern "C" int wake_batch_replay(wake_batch* b) {
  if (!b || !b->exec) return WAKE_ESTATE;
  HIP_TRY(hipSetDevice(b->device));
  HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  for (wake_ctx* c : b->ctxs) {
    c->next = c->I.n_xi;
    c->valid_from = 0;
    c->pending = b->stream;
  }
  return WAKE_OK;
}

extern "C" int wake_batch_sync(wake_batch* b) {
  if (!b) return WAKE_EINVAL;
  HIP_TRY(hipStreamSynchronize(b->stream));
  return WAKE_OK;
}
