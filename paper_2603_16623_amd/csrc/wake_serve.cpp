// Request server of the C ABI (include/wake.h, "Served form"): continuous
// batching of independent solves.
//
// Requests are queued on the host (inputs copied).  Each step admits queued
// requests in arrival order while their device footprint (wake_footprint)
// fits the budget, marches every resident request by up to slices_per_step
// slices in one persistent launch (one workgroup per request, the same
// kernels as a single solve), and retires the requests that reached the end
// of their window or broke down: their on-axis lineout and final fields are
// copied to the host and their device memory released.  A request's result
// does not depend on the other requests in the mix: the march of one
// instance reads and writes only its own memory, and a solve split into
// several launches is bitwise the one-launch solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/wake.h"
#include "wake_common.h"
#include "wake_launch.h"
#include "wake_runtime.h"

namespace {

struct Request {
  int64_t ticket = 0;
  std::vector<double> r0, dr, dens;
  wake_domain dom{};
  std::vector<wake_source> src;
  std::vector<std::vector<double>> pdata;   // particle arrays of the sources, 4 per source
  int64_t n_particles = 0;
  int64_t footprint = 0;
};

struct Active {
  int64_t ticket;
  wake_ctx* ctx;
  int64_t footprint;
};

struct Result {
  int32_t status = WAKE_OK;
  int32_t breakdown = -1;
  int32_t N = 0, n_xi = 0;
  std::vector<double> axis;   // [n_xi][2]
  std::vector<double> last;   // [6][N]
};

}  // namespace

struct wake_server {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  wake_server_config cfg{};
  int64_t next_ticket = 1;
  int64_t in_use = 0;
  int64_t marched = 0;        // ring-slice updates marched so far
  std::deque<Request> queue;
  std::vector<Active> active;
  std::unordered_map<int64_t, Result> done;
  WakeInst* d_insts = nullptr;
  int32_t* d_counter = nullptr;
  int32_t* d_ctl = nullptr;
  int cap = 0;
  std::vector<int32_t> h_ctl;
};

static void server_release(wake_server* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (Active& a : s->active) wake_destroy(a.ctx);
  if (s->d_insts) (void)hipFree(s->d_insts);
  if (s->d_counter) (void)hipFree(s->d_counter);
  if (s->d_ctl) (void)hipFree(s->d_ctl);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

extern "C" void wake_server_destroy(wake_server* s) { server_release(s); }

extern "C" int wake_server_create(wake_server** out, const wake_server_config* cfg, void* hip_stream) {
  if (!out) return WAKE_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->slices_per_step <= 0 || cfg->device_bytes <= 0 || cfg->max_active < 0 ||
      cfg->ring_slices_per_step < 0 || cfg->step_us < 0)
    return WAKE_EINVAL;
  int cur_nt = 0, cur_wpc = 0;
  (void)wake_get_tiling(&cur_nt, &cur_wpc);
  const int nt = cfg->threads != 0 ? cfg->threads : cur_nt;
  if (wake_tiling_occupancy(nt, 0) < 0) return WAKE_EINVAL;
  wake_server* s = new (std::nothrow) wake_server();
  if (!s) return WAKE_ENOMEM;
  s->cfg = *cfg;
  s->cfg.threads = nt;
  if (hipGetDevice(&s->device) != hipSuccess) { server_release(s); return WAKE_EDEVICE; }
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      server_release(s);
      return WAKE_EDEVICE;
    }
    s->own_stream = true;
  }
  if (hipMalloc(&s->d_counter, 64) != hipSuccess) { server_release(s); return WAKE_ENOMEM; }
  *out = s;
  return WAKE_OK;
}

extern "C" int wake_server_submit(wake_server* s, const wake_plasma* plasma, const wake_domain* dom,
                                  const wake_source* sources, int32_t n_sources, int64_t* ticket) {
  if (!s || !plasma || !dom || !ticket || n_sources < 0 || (n_sources > 0 && !sources))
    return WAKE_EINVAL;
  const int N = plasma->n_rings;
  if (N <= 0 || !plasma->r0 || !plasma->dr || dom->n_xi <= 0 || dom->record_stride < 0)
    return WAKE_EINVAL;
  Request q;
  try {
    q.r0.assign(plasma->r0, plasma->r0 + N);
    q.dr.assign(plasma->dr, plasma->dr + N);
    if (plasma->dens) q.dens.assign(plasma->dens, plasma->dens + N);
    q.dom = *dom;
    for (int i = 0; i < n_sources; ++i) {
      wake_source w = sources[i];
      if (w.kind == WAKE_BEAM_PARTICLES) {
        if (w.n < 0 || (w.n > 0 && (!w.x || !w.y || !w.xi || !w.w))) return WAKE_EINVAL;
        const double* arrs[4] = {w.x, w.y, w.xi, w.w};
        for (int a = 0; a < 4; ++a) q.pdata.emplace_back(arrs[a], arrs[a] + w.n);
        q.n_particles += w.n;
      }
      q.src.push_back(w);
    }
  } catch (...) {
    return WAKE_ENOMEM;
  }
  q.footprint = ctx_footprint(N, dom->n_xi, q.n_particles, dom->record_stride,
                              layout_default(s->cfg.threads));
  if (q.footprint < 0) return WAKE_EINVAL;
  q.ticket = s->next_ticket++;
  *ticket = q.ticket;
  s->queue.push_back(std::move(q));
  return WAKE_OK;
}

// Build a context for a queued request (on the server stream).
static int admit(wake_server* s, Request& q, wake_ctx** out) {
  wake_plasma pl;
  pl.n_rings = (int32_t)q.r0.size();
  pl.r0 = q.r0.data();
  pl.dr = q.dr.data();
  pl.dens = q.dens.empty() ? nullptr : q.dens.data();
  wake_ctx* c = nullptr;
  int r = ctx_create(&c, &pl, &q.dom, s->stream, layout_default(s->cfg.threads));
  if (r != WAKE_OK) return r;
  size_t pd = 0;
  for (wake_source w : q.src) {
    if (w.kind == WAKE_BEAM_PARTICLES) {
      w.x = q.pdata[pd].data(); w.y = q.pdata[pd + 1].data();
      w.xi = q.pdata[pd + 2].data(); w.w = q.pdata[pd + 3].data();
      pd += 4;
    }
    r = wake_add_beam(c, &w);
    if (r != WAKE_OK) { wake_destroy(c); return r; }
  }
  r = wake_prepare(c);
  if (r != WAKE_OK) { wake_destroy(c); return r; }
  *out = c;
  return WAKE_OK;
}

static int retire(wake_server* s, size_t i, int32_t brk) {
  Active a = s->active[i];
  wake_ctx* c = a.ctx;
  Result res;
  res.N = c->I.N;
  res.n_xi = c->I.n_xi;
  res.breakdown = brk;
  res.status = brk >= 0 ? WAKE_EBREAKDOWN : WAKE_OK;
  try {
    res.axis.resize(2 * (size_t)res.n_xi);
    if (brk < 0) res.last.resize((size_t)OUT_N * res.N);
  } catch (...) {
    return WAKE_ENOMEM;
  }
  HIP_TRY(hipMemcpyAsync(res.axis.data(), c->I.axis, sizeof(double) * res.axis.size(),
                         hipMemcpyDeviceToHost, s->stream));
  if (brk < 0)
    HIP_TRY(hipMemcpyAsync(res.last.data(), c->I.last, sizeof(double) * res.last.size(),
                           hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  wake_destroy(c);
  s->in_use -= a.footprint;
  s->done[a.ticket] = std::move(res);
  s->active.erase(s->active.begin() + i);
  return WAKE_OK;
}

extern "C" int wake_server_step(wake_server* s, int32_t* n_active, int32_t* n_queued, int32_t* n_done) {
  if (!s) return WAKE_EINVAL;
  HIP_TRY(hipSetDevice(s->device));
  // admission, in arrival order, by device footprint and by workgroups: the
  // resident requests' workgroups (G each) must fit one persistent launch,
  // so that every request marches for the whole step
  const int slots = march_grid(s->cfg.threads, 1 << 30, s->device);
  int used = 0;
  for (const Active& a : s->active) used += a.ctx->I.G;
  while (!s->queue.empty()) {
    if (s->cfg.max_active > 0 && (int)s->active.size() >= s->cfg.max_active) break;
    Request& q = s->queue.front();
    int qc = 0, qg = 1;
    layout_of((int)q.r0.size(), layout_default(s->cfg.threads), &qc, &qg);
    if (used + qg > slots && !s->active.empty()) break;
    const bool fits = s->in_use + q.footprint <= s->cfg.device_bytes;
    if (!fits && !s->active.empty()) break;
    wake_ctx* c = nullptr;
    const int r = fits ? admit(s, q, &c) : WAKE_ENOMEM;
    if (r != WAKE_OK) {           // never runnable: report it as the request's result
      Result res;
      res.status = r;
      res.N = (int32_t)q.r0.size();
      res.n_xi = q.dom.n_xi;
      s->done[q.ticket] = std::move(res);
      s->queue.pop_front();
      continue;
    }
    s->active.push_back({q.ticket, c, q.footprint});
    s->in_use += q.footprint;
    used += c->I.G;
    s->queue.pop_front();
  }
  int32_t retired = 0;
  if (!s->active.empty()) {
    // one persistent launch over every resident request; with a step length,
    // each request's share of it (workgroups that fit / resident requests)
    int64_t budget = 0;
    if (s->cfg.step_us > 0) {
      int tasks = 0;
      for (const Active& a : s->active) tasks += a.ctx->I.G;
      const double share = std::min(1.0, (double)slots / (double)tasks);
      budget = std::max<int64_t>(1, (int64_t)(s->cfg.step_us * 100.0 * share));   // 100 MHz ticks
    }
    std::vector<WakeInst> v;
    std::vector<int> count(s->active.size(), 0);
    for (size_t i = 0; i < s->active.size(); ++i) {
      wake_ctx* c = s->active[i].ctx;
      int k = s->cfg.slices_per_step;
      if (s->cfg.ring_slices_per_step > 0)
        k = (int)std::min<int64_t>(k, std::max<int64_t>(1, s->cfg.ring_slices_per_step / c->I.N));
      const int cnt = std::min(k, c->I.n_xi - c->next);
      count[i] = cnt;
      WakeInst I = c->I;
      I.first = c->next;
      I.count = cnt;
      I.budget = budget;
      v.push_back(I);
    }
    const int n = (int)v.size();
    if (n > s->cap) {
      if (s->d_insts) (void)hipFree(s->d_insts);
      if (s->d_ctl) (void)hipFree(s->d_ctl);
      s->d_insts = nullptr;
      s->d_ctl = nullptr;
      const int cap = std::max(n, 2 * s->cap);
      HIP_TRY(hipMalloc(&s->d_insts, sizeof(WakeInst) * cap));
      HIP_TRY(hipMalloc(&s->d_ctl, sizeof(int32_t) * CTL_NWORDS * cap));
      s->cap = cap;
    }
    // order of the queue: longest remaining work first (the instance order
    // inside a launch changes no result)
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return (int64_t)v[a].N * v[a].count > (int64_t)v[b].N * v[b].count;
    });
    std::vector<WakeInst> vs(n);
    for (int i = 0; i < n; ++i) vs[i] = v[order[i]];
    assign_tasks(vs);
    HIP_TRY(hipMemcpyAsync(s->d_insts, vs.data(), sizeof(WakeInst) * n, hipMemcpyHostToDevice,
                           s->stream));
    HIP_TRY(launch_insts(vs, s->d_insts, s->d_counter, s->device, 0, s->stream));
    HIP_TRY(launch_ctl_gather(s->d_insts, n, s->d_ctl, s->stream));
    s->h_ctl.resize((size_t)CTL_NWORDS * n);
    HIP_TRY(hipMemcpyAsync(s->h_ctl.data(), s->d_ctl, sizeof(int32_t) * CTL_NWORDS * n,
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::vector<int32_t> brk(s->active.size(), -1);
    for (int j = 0; j < n; ++j) {
      const int i = order[j];
      const int32_t* w = &s->h_ctl[(size_t)CTL_NWORDS * j];
      wake_ctx* c = s->active[i].ctx;
      brk[i] = w[CTL_BREAK];
      const int nx = w[CTL_NEXT];
      s->marched += (int64_t)std::max(0, nx - c->next) * c->I.N;
      c->next = nx;
    }
    for (size_t i = s->active.size(); i-- > 0;) {
      wake_ctx* c = s->active[i].ctx;
      if (brk[i] >= 0 || c->next >= c->I.n_xi) {
        const int r = retire(s, i, brk[i]);
        if (r != WAKE_OK) return r;
        ++retired;
      }
    }
  }
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  if (n_done) *n_done = retired;
  return WAKE_OK;
}

extern "C" int wake_server_result(wake_server* s, int64_t ticket, int32_t* breakdown_slice,
                                  double* psi_axis, double* ez_axis, double* psi, double* er_minus_bt,
                                  double* ez, double* bt, double* rho, double* ur) {
  if (!s) return WAKE_EINVAL;
  auto it = s->done.find(ticket);
  if (it == s->done.end()) return ticket > 0 && ticket < s->next_ticket ? WAKE_ESTATE : WAKE_EINVAL;
  Result& res = it->second;
  if (breakdown_slice) *breakdown_slice = res.breakdown;
  const int status = res.status;
  if (status == WAKE_OK || status == WAKE_EBREAKDOWN) {
    for (int i = 0; i < res.n_xi; ++i) {
      if (psi_axis) psi_axis[i] = res.axis[2 * (size_t)i];
      if (ez_axis) ez_axis[i] = res.axis[2 * (size_t)i + 1];
    }
    if (status == WAKE_OK) {
      double* outs[OUT_N] = {psi, er_minus_bt, ez, bt, rho, ur};
      for (int q = 0; q < OUT_N; ++q)
        if (outs[q]) std::memcpy(outs[q], res.last.data() + (size_t)q * res.N, sizeof(double) * res.N);
    }
  }
  s->done.erase(it);
  return status;
}

extern "C" int wake_server_stats(wake_server* s, int64_t* bytes_in_use, int32_t* n_active,
                                 int32_t* n_queued, int32_t* n_results, int64_t* ring_slices) {
  if (!s) return WAKE_EINVAL;
  if (ring_slices) *ring_slices = s->marched;
  if (bytes_in_use) *bytes_in_use = s->in_use;
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  if (n_results) *n_results = (int32_t)s->done.size();
  return WAKE_OK;
}

extern "C" int wake_server_ready(wake_server* s, int64_t* tickets, int32_t cap, int32_t* n) {
  if (!s || !n || cap < 0 || (cap > 0 && !tickets)) return WAKE_EINVAL;
  int32_t k = 0;
  for (const auto& kv : s->done) {
    if (k >= cap) break;
    tickets[k++] = kv.first;
  }
  *n = k;
  return WAKE_OK;
}
