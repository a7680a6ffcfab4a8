// Host-callable kernel launchers (defined in wake_march.hip, wake_beam.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "wake_common.h"

hipError_t launch_init(const WakeInst& I, const double* r0, const double* dr, const double* dens,
                       hipStream_t s);
hipError_t launch_beam_table(const double* x, const double* y, const double* xi, const double* w,
                             const double* q, int64_t np, double dxi, int n_xi, int32_t* cnt,
                             int32_t* cnt2, int32_t* cursor, int32_t* off, int32_t* poff, double* er,
                             double* eq, int64_t* ek, double* br, double* bcum, hipStream_t s);
hipError_t launch_zero(int32_t* p, int n, hipStream_t s);
// Device scratch of the beam-table build for callers that cannot allocate:
// a file-scope device array of WAKE_NOALLOC_SCRATCH bytes, its address on
// device `dev` (which must be current) looked up once per device.
#define WAKE_NOALLOC_SCRATCH ((size_t)24 << 20)
#define WAKE_NOALLOC_PARTICLES 131072
#define WAKE_NOALLOC_SLICES 131072
hipError_t beam_scratch(int dev, void** p, size_t* bytes);
hipError_t launch_state_by_id(const WakeInst& I, double* rho, double* u, double* fr, double* fu,
                              hipStream_t s);
hipError_t launch_state_set(const WakeInst& I, const double* rho, const double* u, const double* fr,
                            const double* fu, int slice, hipStream_t s);
hipError_t launch_reset(const WakeInst* d_insts, int n_insts, hipStream_t s);
hipError_t launch_ctl_gather(const WakeInst* d_insts, int n, int32_t* out, hipStream_t s);

// marcher: workgroups of nt threads (256 or 512)
bool march_threads_ok(int nt);
size_t march_lds_bytes(int nt);
// grid_mode: 0 the plain variant; 1 the variant that also evaluates the
// fields at the instances' grid nodes; 2 that one with the chi deposit (for
// instances whose grid deposits chi).  Instances without a grid march in the
// grid variants as in the plain one, instances without the deposit in
// variant 2 as in variant 1.
hipError_t launch_march(int nt, const WakeInst* d_insts, int n_insts, int n_tasks, int32_t* counter,
                        int grid, int grid_mode, hipStream_t s);
// field-grid node records of I's grid (ln r_g, ion fields at r_g) for its
// n_entries nodes (per-slice node sets: every entry)
hipError_t launch_grid_init(const WakeInst& I, double* tab, int n_entries, hipStream_t s);
int march_occupancy(int nt);
int march_cmax(int nt);     // rings per thread up to which the keys of every position fit LDS
hipError_t march_prepare(int nt);
