// Autotuner of the C ABI (include/wake.h, "Autotuner"): measures candidate
// layouts of the marcher per ring-count bucket on the caller's instances and
// installs the fastest as the tuning that new contexts take.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <vector>

#include "../../include/wake.h"
#include "wake_common.h"
#include "wake_launch.h"
#include "wake_runtime.h"

namespace {

const int kLo[WAKE_TUNE_BUCKETS] = {0, 2048, 4096, 8192, 16384, 32768, 65536, 131072};

struct Cand {
  int nt, rpt;
};

// Candidate layouts for a bucket whose instances have nmin..nmax rings: one
// workgroup where the keys of every position fit its LDS, cooperative
// members of 512 threads where the ring counts exceed 2048.
std::vector<Cand> candidates(int nmin, int nmax) {
  std::vector<Cand> v;
  for (int nt : {256, 512})
    if (nmax <= march_cmax(nt) * nt) v.push_back({nt, 0});
  if (nmin > 2048)
    for (int rpt : {1, 2, 4, 8})
      if (nmin > rpt * 512) v.push_back({512, rpt});
  if (v.empty()) v.push_back({512, 8});
  return v;
}

struct Owned {
  std::vector<wake_ctx*> ctxs;
  wake_batch* batch = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~Owned() {
    if (batch) wake_batch_destroy(batch);
    for (wake_ctx* c : ctxs) wake_destroy(c);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// Ring-slice updates per second of the instances idx marched together through
// their first min(slices, n_xi) slices with layout L (the faster of two runs).
int measure(const wake_plasma* plasmas, const wake_domain* domains, const wake_source* const* sources,
            const int32_t* n_sources, const std::vector<int>& idx, int slices, const Layout& L,
            hipStream_t stream, double* rate) {
  Owned o;
  double work = 0.0;
  for (int i : idx) {
    wake_domain dom = domains[i];
    dom.record_stride = 0;
    wake_ctx* c = nullptr;
    int r = ctx_create(&c, &plasmas[i], &dom, stream, L);
    if (r != WAKE_OK) return r;
    o.ctxs.push_back(c);
    for (int k = 0; k < n_sources[i]; ++k) {
      r = wake_add_beam(c, &sources[i][k]);
      if (r != WAKE_OK) return r;
    }
    r = wake_prepare(c);
    if (r != WAKE_OK) return r;
    work += (double)plasmas[i].n_rings * std::min(slices, dom.n_xi);
  }
  int r = wake_batch_create(&o.batch, o.ctxs.data(), (int32_t)o.ctxs.size(), stream);
  if (r != WAKE_OK) return r;
  HIP_TRY(hipEventCreate(&o.ev[0]));
  HIP_TRY(hipEventCreate(&o.ev[1]));
  float best = 0.0f;
  for (int run = 0; run < 2; ++run) {
    if (run > 0)
      for (wake_ctx* c : o.ctxs) {
        r = wake_reset(c);
        if (r != WAKE_OK) return r;
      }
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipEventRecord(o.ev[0], stream));
    r = wake_batch_solve(o.batch, slices);
    if (r != WAKE_OK) return r;
    HIP_TRY(hipEventRecord(o.ev[1], stream));
    HIP_TRY(hipEventSynchronize(o.ev[1]));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, o.ev[0], o.ev[1]));
    if (run == 0 || ms < best) best = ms;
  }
  *rate = best > 0.0f ? work / (best * 1e-3) : 0.0;
  return WAKE_OK;
}

}  // namespace

extern "C" int wake_autotune(const wake_plasma* plasmas, const wake_domain* domains,
                             const wake_source* const* sources, const int32_t* n_sources, int32_t n,
                             int32_t slices, void* hip_stream, wake_tuning* out) {
  if (!plasmas || !domains || n <= 0 || slices <= 0 || !out || !n_sources) return WAKE_EINVAL;
  for (int i = 0; i < n; ++i)
    if (plasmas[i].n_rings <= 0 || n_sources[i] < 0 || (n_sources[i] > 0 && (!sources || !sources[i])))
      return WAKE_EINVAL;
  hipStream_t stream = (hipStream_t)hip_stream;
  bool own = false;
  if (!stream) {
    HIP_TRY(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    own = true;
  }
  wake_tuning t{};
  t.n_buckets = WAKE_TUNE_BUCKETS;
  int status = WAKE_OK;
  for (int b = 0; b < WAKE_TUNE_BUCKETS && status == WAKE_OK; ++b) {
    t.lo[b] = kLo[b];
    t.threads[b] = 512;
    t.rings_per_thread[b] = kLo[b] < 8192 ? 0 : 8;
    t.rate[b] = 0.0;
    const int hi = b + 1 < WAKE_TUNE_BUCKETS ? kLo[b + 1] : INT_MAX;
    std::vector<int> idx;
    int nmin = INT_MAX, nmax = 0;
    for (int i = 0; i < n; ++i) {
      const int N = plasmas[i].n_rings;
      if (N >= kLo[b] && N < hi) {
        idx.push_back(i);
        nmin = std::min(nmin, N);
        nmax = std::max(nmax, N);
      }
    }
    if (idx.empty()) continue;
    for (const Cand& c : candidates(nmin, nmax)) {
      const Layout L{c.nt, c.rpt, c.rpt > 0 ? 1 : INT32_MAX};
      double rate = 0.0;
      status = measure(plasmas, domains, sources, n_sources, idx, slices, L, stream, &rate);
      if (status != WAKE_OK) break;
      if (rate > t.rate[b]) {
        t.rate[b] = rate;
        t.threads[b] = c.nt;
        t.rings_per_thread[b] = c.rpt;
      }
    }
  }
  if (own) (void)hipStreamDestroy(stream);
  if (status != WAKE_OK) return status;
  status = wake_set_tuning(&t);
  if (status == WAKE_OK) *out = t;
  return status;
}
