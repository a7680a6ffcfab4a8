// Host runtime internals shared by the C ABI (wake_api.cpp) and the
// request server (wake_serve.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/wake.h"
#include "wake_common.h"
#include "wake_ions.h"

// bump allocation of one context's device arena (256-B aligned pieces)
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  template <class T>
  T* take(size_t n) {
    used = (used + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + used);
    used += n * sizeof(T);
    return p;
  }
};

struct wake_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  WakeInst I;
  WakeInst* d_inst = nullptr;
  int32_t* d_counter = nullptr;
  Arena arena;
  double* staging = nullptr;   // 4N doubles
  // beam table (persistent part)
  char* beam_mem = nullptr;
  bool beam_external = false;      // beam_mem belongs to the caller (wake_prepare_noalloc)
  // pending particle sources (host copies until the table is built)
  std::vector<double> px, py, pxi, pw, pq;
  double* grid_mem = nullptr;  // field grid: fields, node records, hand-over scratch, radii, offsets
  std::vector<int32_t> grid_off_h; // per-slice node sets: host copy of the offsets (empty: fixed nodes)
  bool prepared = false;
  int batches = 0;                 // batches that hold this context
  int next = 0;
  int valid_from = 0;              // first slice whose records belong to the current state's march
  hipStream_t pending = nullptr;   // batch stream that last marched this context
  // two-species context (electrons and mobile ions): its own instance
  // record and marcher; I keeps the sources, beam table, outputs of the
  // electrons and control words
  bool two_species = false;
  WakeIons J;
  WakeIons* d_J = nullptr;
};


int dev_err(hipError_t e);

#define HIP_TRY(x)                              \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return dev_err(e_);   \
  } while (0)

// wait for every stream that may still work on the context
int drain(wake_ctx* c);
// persistent grid for nt-thread workgroups over n instances
int march_grid(int nt, int n_insts, int dev);
// How a context is laid out: workgroup threads, rings per thread of
// cooperative members (0: 8) and the ring count from which contexts are
// cooperative (0: beyond one workgroup's LDS keys; INT32_MAX: never).
struct Layout {
  int nt, rpt, min_n;
};
// the layout of wake_set_tiling / wake_set_cluster for nt-thread workgroups
Layout layout_default(int nt);
// the layout a new context of N rings takes (the installed tuning, else the
// tiling and cluster settings)
Layout layout_for(int N);
// layout of an instance (rings per thread C, workgroups G)
void layout_of(int N, const Layout& L, int* C, int* G);
// first task of each descriptor (members of a cooperative instance are G
// consecutive tasks); returns the number of tasks
int assign_tasks(std::vector<WakeInst>& v);
// one persistent launch per distinct workgroup size over the descriptors v
// (already copied to d_insts, tasks assigned)
hipError_t launch_insts(const std::vector<WakeInst>& v, const WakeInst* d_insts, int32_t* d_counter,
                        int dev, int grid_override, hipStream_t s);
// a two-species context's record for a march of slices [first, first+count)
// (its sources and beam table taken from I)
WakeIons ions_record(const wake_ctx* c, int first, int count);
// context creation / footprint with an explicit workgroup size
int ctx_create(wake_ctx** out, const wake_plasma* plasma, const wake_domain* dom, void* hip_stream,
               const Layout& L);
int64_t ctx_footprint(int32_t n_rings, int32_t n_xi, int64_t n_particles, int32_t record_stride,
                      const Layout& L);
