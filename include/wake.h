/*
 * wake.h - C ABI of the MI355X (gfx950) gridless quasistatic plasma-ring
 * wake solver.
 *
 * The model is the paper's gridless quasistatic model ("Gridless
 * quasistatic model for efficient simulation of plasma-based
 * accelerators", Sec. "Gridless quasistatic model" and Appendix "Solve
 * recursive system"): an axisymmetric electron plasma, discretised into
 * delta-function rings (Sec. "Discretization of plasma species into
 * macroparticles"), over an immobile ion species, responds to frozen
 * ultra-relativistic beams and a frozen laser envelope.  The window is
 * marched in xi = -zeta (normalised units: lengths in k_p^-1, densities in
 * n0) one slice at a time: sort rings radially, gather sources, compute
 * psi, d_rho psi, d_zeta psi (eqs. dpsi_dr, psi, dpsi_dzeta), gamma
 * (eq. plasma_particle_motion_4), B_theta^(p) from the two-point recursion
 * (eqs. b_theta_plasma, ai_bi, b_coeffs_1-3) and push (r, u_r) with
 * second-order Adams-Bashforth (eqs. plasma_particle_motion_1-2).
 *
 * Conventions.  Electrons carry q = -1, m = 1, so psibar = 1 + psi.
 * Fields are reported at slice nodes xi_n = n * dxi, n = 0 .. n_xi-1, at
 * every ring, indexed by ring id (its index in the wake_plasma arrays):
 *   psi, E_r - B_theta (= -d_rho psi), E_z (= d_xi psi), B_theta,
 * and on the axis psi(0) and E_z(0) for every slice.
 *
 * Errors.  Every int-returning call returns WAKE_OK (0) or a negative
 * wake_status; no C++ exception crosses this boundary.  Every computation
 * runs in HIP kernels on the device current at wake_create; there is no CPU
 * path.  A context is used from one host thread at a time.
 *
 * Memory.  Pointers passed in are owned by the caller.  Host input arrays
 * are copied before the call returns.  Output pointers are host memory
 * unless the call's dst_is_device flag is set, in which case they are
 * device pointers on the context's device (e.g. torch tensor data).
 */
#ifndef WAKE_H
#define WAKE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wake_ctx wake_ctx;
typedef struct wake_batch wake_batch;

enum wake_status {
  WAKE_OK = 0,
  WAKE_EINVAL = -1,      /* an argument is out of range or inconsistent */
  WAKE_ENOMEM = -2,      /* device or host allocation failed */
  WAKE_EDEVICE = -3,     /* a HIP runtime call failed */
  WAKE_ESTATE = -4,      /* call out of order (e.g. slice not yet solved) */
  WAKE_EBREAKDOWN = -5,  /* psibar <= 0 or a non-finite value: the quasistatic
                            description broke down; the solve stopped there */
  WAKE_ENOTREC = -6      /* the requested slice was not recorded */
};

enum wake_source_kind {
  WAKE_BEAM_PARTICLES = 1, /* macroparticles (x, y, xi, w) with charge q each */
  WAKE_BEAM_GAUSSIAN = 2,  /* analytic bi-Gaussian density n_peak exp(-r^2/2sr^2 - (xi-xi_c)^2/2sx^2) */
  WAKE_LASER_GAUSSIAN = 3  /* frozen envelope |a|^2 = a0^2 exp(-2 r^2/w0^2 - 2 (xi-xi_l)^2/L^2) */
};

/* Plasma column (Sec. "Discretization of plasma species into macroparticles").
 * Ring j starts at r0[j] = sum_{k<j} dr[k] + dr[j]/2 (checked to 1e-9
 * relative), carries weight w_j = dens[j] r0[j] dr[j] (eq. macroparticle_weight)
 * and the modified self weight w_j/2 - dens[j] dr[j]^2/8 (Sec. "Key
 * algorithmic adjustments").  Immobile ions sit at the same radii with the
 * same weights.  r0 must be strictly increasing, dr > 0, dens > 0. */
typedef struct {
  int32_t n_rings;
  const double *r0;   /* [n_rings] host */
  const double *dr;   /* [n_rings] host */
  const double *dens; /* [n_rings] host, NULL = uniform density 1 */
} wake_plasma;

/* Longitudinal window: fields at xi_n = n * dxi for n = 0 .. n_xi-1
 * (the plasma is unperturbed at xi = 0, Fig. 2 "initialize at zeta = 0").
 * record_stride > 0 keeps a full snapshot (all six ring quantities) every
 * record_stride slices; 0 keeps only the last solved slice. */
typedef struct {
  double dxi;
  int32_t n_xi;
  int32_t record_stride;
} wake_domain;

/* One driver or witness.  Beams are ultra-relativistic and frozen
 * (Sec. "Theoretical framework"); B_theta^(b) at a ring is the beam charge
 * inside its radius over the radius (Gauss law of the beam equation).
 * Particles are deposited in xi with linear weights onto the slice nodes.
 * Fields not used by `kind` are ignored. */
typedef struct {
  int32_t kind;                  /* wake_source_kind */
  double q;                      /* charge of each beam particle (-1: electrons) */
  int64_t n;                     /* number of particles (PARTICLES) */
  const double *x, *y, *xi, *w;  /* [n] host: positions and number weights (n0 k_p^-3) */
  double n_peak, sigma_r, sigma_xi, xi_c; /* GAUSSIAN beam */
  double a0, w0, L, xi_l;        /* LASER_GAUSSIAN */
} wake_source;

/* Create a solver for one plasma column and window on the current HIP
 * device.  hip_stream: a hipStream_t to run on, or NULL for a stream of the
 * context's own.  Uploads the rings and builds the weights and ion tables
 * on the device.  *out is NULL on failure. */
int wake_create(wake_ctx **out, const wake_plasma *plasma, const wake_domain *domain,
                void *hip_stream);

/* Add one source; only before the first wake_solve / wake_prepare.
 * At most 8 analytic sources (Gaussian beams and lasers together). */
int wake_add_beam(wake_ctx *ctx, const wake_source *src);

/* Build the beam table and everything else the march needs (done
 * implicitly by the first wake_solve).  Synchronous. */
int wake_prepare(wake_ctx *ctx);

/* wake_prepare for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same beam table, built into `table`, device memory on the context's
 * device owned by the caller (at least 4 (n_xi + 1) + 32 n_particles + 1024
 * bytes, n_particles = every particle added with wake_add_beam; it must stay
 * valid until wake_destroy, which does not free it), with the build staged
 * in a device array the library holds on each GPU until the process ends
 * (24 MiB; at most 131072 particles and 131072 slices).  The call allocates
 * no device memory.  WAKE_EINVAL for a null table, a table too small or
 * sizes beyond those limits; WAKE_OK with nothing done when the context is
 * already prepared.  Every call on a GPU shares that GPU's staging array:
 * calls that overlap on one GPU (several host threads) race.  Synchronous.
 * A context prepared this way solves, batches and serves as after
 * wake_prepare, with the same results. */
int wake_prepare_noalloc(wake_ctx *ctx, void *table, int64_t table_bytes);

/* March slices [first_slice, first_slice + n_slices) on the context's
 * stream (asynchronous): per slice the sort, sources, psi family, gamma,
 * d_zeta psi, the coefficients and two-point recursion of B_theta^(p) and
 * the push of Fig. 2 (right column) and Sec. "Numerical integration of
 * wakefields" (eqs. dpsi_dr, psi, dpsi_dzeta, b_coeffs_1-3, ai_bi,
 * plasma_particle_motion_1-4).  first_slice must equal the context's next slice
 * (0 after create, the end of the previous solve, or the slice given to
 * wake_set_state).  A breakdown stops the march at its slice and is
 * reported by wake_status / wake_fields.  With WAKE_TRACE set in the
 * environment ("1" or "stderr": standard error; otherwise a file name,
 * appended to) the solve is traced: one launch per slice, synchronous, and
 * one line per slice with its GPU time (HIP events), whether it began with
 * an order fix-up and the breakdown slice; the results are bitwise those of
 * an untraced solve. */
int wake_solve(wake_ctx *ctx, int32_t first_slice, int32_t n_slices);

/* Fields at the rings of one solved slice, indexed by ring id: psi,
 * E_r - B_theta, E_z, B_theta, and the ring radius and radial momentum at
 * that slice (the gauge relations eqs. lorentz_gauge_1-2 turn the solve's
 * psi, d_rho psi and d_zeta psi into E_r - B_theta = -d_rho psi and
 * E_z = -d_zeta psi; B_theta = B^(b) + B^(p), eq. b_theta_plasma).  slice = -1 means the last slice of the most recent solve;
 * otherwise the slice must be a recorded one (multiple of record_stride) and
 * marched from the current state (WAKE_ESTATE for slices before the slice
 * of the last wake_set_state).  NULL outputs are skipped.  Synchronizes the
 * context's stream. */
int wake_fields(wake_ctx *ctx, int32_t slice, double *psi, double *er_minus_bt, double *ez,
                double *bt, double *rho, double *ur, int32_t dst_is_device);

/* Radial field grid (Fig. 2 of the paper, the fields on an external grid
 * that couples the plasma to the beams; eqs. psi, dpsi_dr, dpsi_dzeta and
 * b_theta_plasma hold at any radius once the rings of a slice are known).
 * n_r uniform nodes at cell centres r_g = (g + 1/2) r_max / n_r,
 * g = 0..n_r-1; every marched slice also writes psi, E_r - B_theta, E_z
 * and B_theta at them (4 n_r doubles per slice, n_xi slices, held on the
 * device by the context; not counted by wake_footprint).  A node with k
 * rings strictly inside it takes the sums of the rings below and above,
 * with no ring at the node; a ring exactly at a node counts as outside it.
 * Only before the first solve and while no batch holds the context
 * (WAKE_ESTATE otherwise); n_r = 0 removes the grid.  n_r <= 2^20,
 * r_max > 0 finite (WAKE_EINVAL); WAKE_ENOMEM if the device memory is not
 * there.  A batch marches contexts with and without grids together.  The
 * served form (wake_server_*) has no grid.  Synchronous. */
int wake_set_grid(wake_ctx *ctx, int32_t n_r, double r_max);

/* chi = n/gamma (the plasma susceptibility the laser envelope solver takes,
 * Fig. 2 "deposit chi in laser grid", Sec. "Integration into Wake-T") at the
 * nodes of a uniform or fixed-radii grid for one solved slice [n_r]: each
 * ring carries w / psibar (n/gamma of eq. fluid_from_mp_1 with (1 - v_z)
 * gamma = psibar), deposited with linear (hat) weights between neighbouring
 * nodes (a ring inside the first node wholly to it; the last node's hat
 * reaching as far above it as the spacing below it) and normalised by each
 * hat's integral of rho drho, so that a uniform plasma at rest gives 1.
 * Slice and errors as wake_grid_fields; WAKE_ESTATE unless the deposit was
 * switched on (wake_set_grid_chi) and for per-slice node sets
 * (wake_set_grid_radii with offsets, wake_set_grid_beam), which deposit no
 * chi.  Synchronizes. */
int wake_grid_chi(wake_ctx *ctx, int32_t slice, double *chi, int32_t dst_is_device);
/* Switch the chi deposit on (on != 0) or off for the context's grids (off
 * after wake_create; Fig. 2 deposits chi when there is a laser).  Only
 * before the first solve and while no batch holds the context
 * (WAKE_ESTATE). */
int wake_set_grid_chi(wake_ctx *ctx, int32_t on);

/* Field grid at radii the caller gives (Sec. "Key algorithmic adjustments":
 * the sums give the plasma fields at any radius, so they can be sampled with
 * any radial resolution; the node rule is wake_set_grid's).  slice_off NULL:
 * the same n_nodes radii at every slice, strictly increasing, > 0, finite,
 * n_nodes <= 2^20.  Otherwise slice_off holds n_xi + 1 offsets (slice_off[0]
 * = 0, non-decreasing, slice_off[n_xi] = n_nodes <= 2^28, at most 2^20 per
 * slice) and slice n takes radii[slice_off[n] .. slice_off[n+1]), ascending
 * within the slice (equal radii allowed), > 0, finite.  n_nodes = 0 removes
 * the grid.  Same call order, memory and errors as wake_set_grid; radii
 * and offsets are copied.  Synchronous. */
int wake_set_grid_radii(wake_ctx *ctx, int64_t n_nodes, const double *radii,
                        const int64_t *slice_off);

/* Field grid at the beam particles' own radii: slice n's nodes are the
 * entries of slice n in the beam table (every macroparticle added with
 * wake_add_beam that deposits on that slice node, at its radius, ascending;
 * a particle between two slice nodes appears at both), so the fields reach
 * the particles with no radial grid (the direct beam-plasma coupling Sec.
 * "Integration into Wake-T" names).  Prepares the context (wake_prepare) if
 * it is not yet.  WAKE_EINVAL without particles; otherwise as
 * wake_set_grid.  Synchronous. */
int wake_set_grid_beam(wake_ctx *ctx);

/* Node count of a slice's grid (uniform and fixed grids: every slice the
 * same) and, if radii is not NULL, their radii (host memory, count
 * doubles).  WAKE_ESTATE without a grid.  Synchronizes. */
int wake_grid_nodes(wake_ctx *ctx, int32_t slice, int64_t *count, double *radii);

/* Grid fields of one solved slice [the slice's node count each, in node
 * order], read out per slice (slice = -1: the slice before the context's
 * next slice, i.e. the last slice of the most recent solve).  WAKE_ESTATE without a grid,
 * for a slice at or after the next slice, or before the slice of the last
 * wake_set_state (not marched from the current state); WAKE_EBREAKDOWN at
 * or after a breakdown.  NULL outputs are skipped.  Synchronizes the
 * context's stream. */
int wake_grid_fields(wake_ctx *ctx, int32_t slice, double *psi, double *er_minus_bt, double *ez,
                     double *bt, int32_t dst_is_device);

/* psi(0) and E_z(0) of every slice [n_xi each]; slices not solved yet hold
 * stale values.  Synchronizes. */
int wake_lineout(wake_ctx *ctx, double *psi_axis, double *ez_axis, int32_t dst_is_device);

/* Ring state at the context's next slice, indexed by ring id: radius,
 * radial momentum and the Adams-Bashforth history (d rho/d xi and
 * d u_r/d xi of the previous slice).  *slice receives the next slice.
 * Synchronizes. */
int wake_get_state(wake_ctx *ctx, int32_t *slice, double *rho, double *ur, double *f_rho,
                   double *f_u, int32_t dst_is_device);

/* Replace the ring state (by ring id) and make `slice` the next slice.
 * f_rho/f_u may be NULL (zero history; slice 0 ignores it anyway).
 * Radii must be > 0 and finite. */
int wake_set_state(wake_ctx *ctx, int32_t slice, const double *rho, const double *ur,
                   const double *f_rho, const double *f_u, int32_t src_is_device);

/* Back to slice 0 with the rings at rest (asynchronous). */
int wake_reset(wake_ctx *ctx);

/* Breakdown slice (-1 if none) and next slice.  Synchronizes. */
int wake_status(wake_ctx *ctx, int32_t *breakdown_slice, int32_t *next_slice);

/* Wait for the context's stream. */
int wake_sync(wake_ctx *ctx);

/* Event counters of the context's marches, summed since creation (or the
 * last reset), a trace of what the march did: [0] slices marched, [1] order
 * fix-ups at slice heads (pushed radii out of order), [2] general fix-ups
 * after the block rounds failed (one workgroup); cooperative instances: [3]
 * member-local rounds (one per member that sorts), [4] rounds over all
 * members, [5] sorts by segments, [6] bitonic fallbacks, [7] meetings of the
 * members through device memory.  The first min(n, 8) go to out (more are
 * zero); reset != 0 zeroes them.  Synchronizes. */
int wake_counters(wake_ctx *ctx, int64_t *out, int32_t n, int32_t reset);

/* Device bytes a context of this size holds (for admission control). */
int64_t wake_footprint(int32_t n_rings, int32_t n_xi, int64_t n_particles, int32_t record_stride);

void wake_destroy(wake_ctx *ctx);
const char *wake_strerror(int code);

/* ---------------------------------------------------------------------
 * Mobile ions (paper, Sec. "Key algorithmic adjustments": several plasma
 * species, the ions included, each summed on its own at its own rings; the
 * beam-driven benchmark of Sec. "Validation benchmarks" moves the ions).  A
 * two-species context holds the electrons (species 0: q = -1, m = 1) and
 * singly charged ions of mass ion_mass electron masses (species 1: q = +1,
 * psibar = 1 - psi / ion_mass), both starting at rest at the column's radii
 * with the column's weights.  Per slice each species is sorted and its psi,
 * d_rho psi and d_zeta psi sums formed at its own rings (eqs. psi, dpsi_dr,
 * dpsi_dzeta); at the rings of the other species they are interpolated
 * linearly between that species' rings, with nodes at the axis (its psi(0),
 * d_rho psi = 0, its d_zeta psi(0), B^(p) = 0) and at its outer edge (its
 * outermost ring's radius plus half that ring's initial extent dr: the
 * exterior field -q Q ln r, -q Q / r, d_zeta psi = 0, B^(p) = b_N / r) and
 * the exterior field beyond the edge.  B_theta^(p) comes from the electrons
 * alone (eqs. b_coeffs_1-3, ai_bi: the ion currents are neglected) and
 * reaches the ions by the same interpolation.  Both species are pushed with
 * their q and m (eqs. plasma_particle_motion_1-4).  psi(0) and E_z(0) of the
 * lineout are the sums over both species.
 *
 * The context is a wake_ctx: wake_add_beam, wake_prepare(_noalloc),
 * wake_solve, wake_status, wake_lineout, wake_reset, wake_sync,
 * wake_counters (slices, order fix-ups), wake_get_layout / wake_get_threads
 * and wake_destroy work on it as on any context; wake_fields,
 * wake_get_state and wake_set_state act on the electrons; the calls below
 * reach either species.  It has no field grid (wake_set_grid: WAKE_EINVAL)
 * and is not a request of the served form.  One workgroup of 1024 threads
 * marches it, alone or in a batch (wake_batch_*: batches may mix one- and
 * two-species contexts; each result equals the context's alone);
 * n_rings <= 8192 and ion_mass > 0 finite (WAKE_EINVAL otherwise).
 * --------------------------------------------------------------------- */
int wake_create_mobile_ions(wake_ctx **out, const wake_plasma *plasma, double ion_mass,
                            const wake_domain *domain, void *hip_stream);
/* wake_fields of species 0 (electrons) or 1 (ions; WAKE_EINVAL on a
 * one-species context), by ring id of that species. */
int wake_species_fields(wake_ctx *ctx, int32_t species, int32_t slice, double *psi,
                        double *er_minus_bt, double *ez, double *bt, double *rho, double *ur,
                        int32_t dst_is_device);
/* wake_get_state / wake_set_state of one species.  Setting either species
 * makes `slice` the next slice of both (set both to start a two-species
 * march from a given state) and clears a breakdown. */
int wake_get_species_state(wake_ctx *ctx, int32_t species, int32_t *slice, double *rho, double *ur,
                           double *f_rho, double *f_u, int32_t dst_is_device);
int wake_set_species_state(wake_ctx *ctx, int32_t species, int32_t slice, const double *rho,
                           const double *ur, const double *f_rho, const double *f_u,
                           int32_t src_is_device);

/* ---------------------------------------------------------------------
 * Tiling of the marcher.  A workgroup of `threads` threads owns one instance;
 * thread t owns the ceil(n_rings / threads) consecutive rings (in radial
 * order) starting at t * ceil(n_rings / threads).  `threads` is fixed for a
 * context when it is created (256 or 512; a workgroup of 1024 threads holds
 * four waves per SIMD, which leaves the marcher 128 registers per lane: it
 * spilled 167-404 of them and marched slower, so it is not offered).
 * Persistent launches place
 * `wgs_per_cu` workgroups on each compute unit (0: as many as fit).  The
 * choice changes summation order only (results agree to rounding).
 * wake_tiling_get returns the threads of entry `index` and how many such
 * workgroups fit on one compute unit.
 * --------------------------------------------------------------------- */
int wake_tiling_count(void);
int wake_tiling_get(int32_t index, int32_t *threads, int32_t *wgs_per_cu);
int wake_set_tiling(int32_t threads, int32_t wgs_per_cu);
int wake_get_tiling(int32_t *threads, int32_t *wgs_per_cu);
/* workgroups of `threads` threads resident per compute unit (occupancy) */
int wake_tiling_occupancy(int32_t threads, int32_t wgs_per_cu);

/* ---------------------------------------------------------------------
 * Cooperative instances (the large-ring-count path).  A context with more
 * rings than one workgroup can keep ordered in LDS (more than 16 * threads)
 * is marched by G workgroups
 * together, member g owning the sorted positions [g P, g P + P), P = C *
 * threads, with C = max(rings_per_thread, ceil(n_rings / (M threads)))
 * and G = ceil(n_rings / P) <= M, M = the smaller of 256 and the
 * workgroups of that size the device holds at once.  Per slice the members exchange their
 * scan totals through device memory (three all-gathers) and fix the ring
 * order on keys in device memory; the order is the same and the fields
 * agree with a single workgroup's to rounding.  The members of one instance
 * must be resident together: launches always place at least G workgroups.
 * wake_set_cluster(rings_per_thread, min_rings) applies to contexts
 * created from now on: rings_per_thread 0 = 8; min_rings 0 = the LDS limit
 * above, otherwise contexts of at least min_rings rings are cooperative
 * (when that gives G >= 2).  A member that waits more than 2 s at a barrier
 * stops the instance, which then reports WAKE_EDEVICE.
 * --------------------------------------------------------------------- */
int wake_set_cluster(int32_t rings_per_thread, int32_t min_rings);
/* workgroups (G) and rings per thread (C) of a context */
int wake_get_layout(wake_ctx *ctx, int32_t *workgroups, int32_t *rings_per_thread);

/* ---------------------------------------------------------------------
 * Autotuner of the layout per ring-count bucket (the batched form's
 * "rings per workgroup and LDS tiling").  Bucket b holds ring counts in
 * [lo[b], lo[b+1]) (the last has no upper end); a context created while a
 * tuning is installed takes its bucket's workgroup threads (256 or 512: the
 * LDS tiling of the marcher) and rings per thread of cooperative
 * members (0: one workgroup per context, never cooperative; else
 * cooperative from the moment it gives two or more members).  Tiling and
 * cluster settings apply to contexts only while no tuning is installed; the
 * served form keeps its own threads.  Any choice gives the same results to
 * rounding; the same choice gives bitwise the same results.
 * --------------------------------------------------------------------- */
#define WAKE_TUNE_BUCKETS 8
typedef struct {
  int32_t n_buckets;
  int32_t lo[WAKE_TUNE_BUCKETS];               /* lo[0] = 0, increasing */
  int32_t threads[WAKE_TUNE_BUCKETS];
  int32_t rings_per_thread[WAKE_TUNE_BUCKETS];
  double rate[WAKE_TUNE_BUCKETS];              /* measured ring-slice updates/s of the choice
                                                  (0: bucket not measured, default layout) */
} wake_tuning;

/* Measure and install a tuning.  The n instances (plasma, domain, sources as
 * for wake_create / wake_add_beam; sources[i] points at n_sources[i]
 * sources; host arrays) are grouped into the buckets lo = 0, 2048, 4096,
 * 8192, 16384, 32768, 65536, 131072 rings; for every bucket with instances,
 * each candidate layout (one workgroup of 256 or 512 threads where
 * the keys of every position fit its LDS; cooperative members of 512
 * threads with 1, 2, 4 or 8 rings per thread where the ring counts exceed
 * 2048) marches all of the bucket's instances together through their first
 * min(slices, n_xi) slices in one persistent launch, twice, and the larger
 * ring-slice rate wins (the earlier candidate on a tie, so the choice
 * follows from the measurements).  Buckets without instances take 512
 * threads, one workgroup below 8192 rings, else eight rings per member
 * thread.  *out receives the installed tuning.  Synchronous; allocates and
 * frees contexts of its own on hip_stream (NULL: a stream of its own). */
int wake_autotune(const wake_plasma *plasmas, const wake_domain *domains,
                  const wake_source *const *sources, const int32_t *n_sources, int32_t n,
                  int32_t slices, void *hip_stream, wake_tuning *out);
/* Install a tuning (t = NULL removes it).  WAKE_EINVAL for a malformed one. */
int wake_set_tuning(const wake_tuning *t);
/* The installed tuning; WAKE_ESTATE when none is. */
int wake_get_tuning(wake_tuning *t);
/* Workgroup threads of a context's layout. */
int wake_get_threads(wake_ctx *ctx, int32_t *threads);

/* ---------------------------------------------------------------------
 * Batched form: many independent contexts (same device) marched by one
 * persistent launch; workgroups take instances longest-first from a device
 * counter.  Two-species contexts of the batch follow in one launch of a
 * workgroup each (longest first).  Per-instance results equal those of
 * solving alone with the same tiling.
 * --------------------------------------------------------------------- */
int wake_batch_create(wake_batch **out, wake_ctx *const *ctxs, int32_t n, void *hip_stream);
/* Advance every instance by up to n_slices (-1: to its window end) from its
 * next slice.  Asynchronous on the batch stream. */
int wake_batch_solve(wake_batch *b, int32_t n_slices);
/* Capture "reset every instance to slice 0, then march the whole window"
 * into a HIP graph (grid = workgroups resident on the device, or
 * `grid` if > 0); wake_batch_replay launches it. */
int wake_batch_capture(wake_batch *b, int32_t grid);
int wake_batch_replay(wake_batch *b);
int wake_batch_sync(wake_batch *b);
void wake_batch_destroy(wake_batch *b);

/* ---------------------------------------------------------------------
 * Served form: continuous batching of independent solves (a parameter scan
 * issuing requests of different ring counts and window lengths).  Requests
 * are queued with their inputs copied; each wake_server_step admits queued
 * requests in arrival order while their device footprint (wake_footprint at
 * the server's tiling) fits device_bytes (a request larger than the whole
 * budget is admitted alone when nothing else is resident), marches every
 * resident request by up to slices_per_step slices in one persistent launch,
 * and retires those that reached their window end or broke down (on-axis
 * lineout and final fields copied to the host, device memory released).
 * Ring state stays on the device between steps.  A request's result is
 * bitwise the result of solving it alone with wake_solve.  One host thread
 * at a time per server.
 * --------------------------------------------------------------------- */
typedef struct wake_server wake_server;

typedef struct {
  int32_t threads;          /* workgroup threads of the server's contexts (0: current tiling) */
  int32_t slices_per_step;  /* most slices a resident request advances per step (> 0) */
  int32_t max_active;       /* cap on resident requests (0: none) */
  int64_t device_bytes;     /* device-memory budget of the resident requests (> 0) */
  int64_t ring_slices_per_step; /* per-request work per step: a request of N rings advances
                                   max(1, ring_slices_per_step / N) slices (at most
                                   slices_per_step), so that small requests are not held to
                                   the pace of large ones; 0: slices_per_step for all */
  int32_t step_us;          /* wall-clock length of a step (0: none): each request stops after
                               the slice that exhausts its share of it (the step length, shared
                               when more requests are resident than workgroups fit) */
} wake_server_config;

int wake_server_create(wake_server **out, const wake_server_config *cfg, void *hip_stream);
/* Queue one solve (sources as for wake_add_beam).  *ticket names it. */
int wake_server_submit(wake_server *s, const wake_plasma *plasma, const wake_domain *domain,
                       const wake_source *sources, int32_t n_sources, int64_t *ticket);
/* Admit, march one step, retire (synchronous).  Counts after the step:
 * resident, still queued, retired by this step. */
int wake_server_step(wake_server *s, int32_t *n_active, int32_t *n_queued, int32_t *n_done);
/* Result of a retired request, then released: returns WAKE_OK, WAKE_EBREAKDOWN
 * (lineout up to the breakdown slice, no final fields), another negative
 * status if it could not run, or WAKE_ESTATE if not retired yet.  Lineout
 * [n_xi] each; final fields at the last slice by ring id [n_rings] each;
 * NULL skips. */
int wake_server_result(wake_server *s, int64_t ticket, int32_t *breakdown_slice, double *psi_axis,
                       double *ez_axis, double *psi, double *er_minus_bt, double *ez, double *bt,
                       double *rho, double *ur);
/* Device bytes held by resident requests, resident / queued requests,
 * results waiting to be fetched, ring-slice updates marched so far. */
int wake_server_stats(wake_server *s, int64_t *bytes_in_use, int32_t *n_active, int32_t *n_queued,
                      int32_t *n_results, int64_t *ring_slices);
/* Tickets whose results are ready (not yet fetched), up to cap of them;
 * *n receives how many were written. */
int wake_server_ready(wake_server *s, int64_t *tickets, int32_t cap, int32_t *n);
void wake_server_destroy(wake_server *s);

#ifdef __cplusplus
}
#endif

#endif /* WAKE_H */
