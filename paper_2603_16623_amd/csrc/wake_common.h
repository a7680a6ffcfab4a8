// Internal data layout shared by the host runtime and the gfx950 kernels of
// the gridless ring solver.  Not part of the public ABI (include/wake.h).
#pragma once
#include <stdint.h>

#define WAKE_MAX_ANALYTIC 8   // analytic beams + lasers per instance
#define WAKE_BCAP 1024        // beam-table entries staged in LDS per slice
#define WAKE_SORTCAP 1024     // rings of long disordered runs sorted in LDS in one piece
#define WAKE_SEGMAX 64        // disordered runs up to this length are ranked in place
#define WAKE_ION_REC 8        // doubles per ion interval record
#define WAKE_CL_MEMBERS 256   // workgroups of one cooperative instance at most
#define WAKE_GRID_TAB 6       // doubles per field-grid node record

// Control words of one instance (device memory, int32).
enum { CTL_CUR = 0, CTL_BREAK = 1, CTL_NEXT = 2, CTL_FAULT = 3, CTL_NWORDS = 4 };
// Event counters of one instance (device memory, 64-bit), summed over its
// marches: slices marched, order fix-ups at slice heads, general fix-ups
// after the block rounds (one workgroup), and for cooperative instances the
// member-local rounds (per member that sorts), rounds over all members,
// sorts by segments, bitonic fallbacks and meetings.
enum { CNT_SLICES = 0, CNT_FIXUPS, CNT_GENERAL, CNT_CL_LOCAL, CNT_CL_ROUNDS, CNT_CL_SEGMENTS,
       CNT_CL_BITONIC, CNT_CL_MEETINGS, CNT_N };

// Ion interval record j (j = 0..N), nodes 0 = axis, j = r0[j-1], N+1 = R_p:
// [node_j, node_{j+1}), psi-psi(0) at node j (dd), its step to node j+1,
// d_rho psi at node j (dd), its step.
enum { IR_LO = 0, IR_HI, IR_PSH, IR_PSL, IR_DPS, IR_DPH, IR_DPL, IR_DDP };

struct WakeAnalytic {
  int32_t kind;     // 2 = bi-Gaussian beam, 3 = Gaussian laser envelope
  int32_t pad;
  double q, n_peak, sigma_r, sigma_xi, xi_c;  // beam
  double a0, w0, L, xi_l;                     // laser
};

// One instance as the kernels see it.  All pointers are device pointers.
//
// Slot layout.  A workgroup of nt threads owns the instance; thread t owns
// the C = ceil(N / nt) consecutive sorted positions [t*C, t*C + C).  Per-ring
// arrays are stored by slot: position p sits in slot (p % C) * nt + p / C,
// so that thread t reads its k-th ring at slot k*nt + t and the lanes of a
// wavefront touch consecutive addresses.
//
// Home slot.  Ring id i has home slot hs(i) = (i % C) * nt + i / C, the slot
// of position i; its constants (weights, r0, ln r0) are stored at hs(i).
// The state stores hs instead of the id (id = (hs % nt) * C + hs / nt), so
// that while rings stay near their initial order the constant gathers of a
// wavefront stay contiguous.
//
// Cooperative instances.  An instance too large for one workgroup's LDS is
// marched by G workgroups (members) together; member g owns the positions
// [g*P, g*P + P), P = C * nt, and inside that range uses the layout above
// shifted by g*P (slot g*P + (q % C) * nt + q / C for q = p - g*P).  With
// G = 1 this is the layout above.  Members exchange their scan totals and
// meet at barriers through device memory.
//
// Order.  Rings are kept in (rho, id) order.  A slice whose pushed radii come
// out of order only computes the new order as a permutation (sorted position
// -> slot), in LDS when the keys of every position fit there, else in global
// memory; the next slice reads through it and writes its pushed rings at the
// slots of the new positions.
struct WakeInst {
  int32_t N;          // rings
  int32_t n_xi;       // slices of the window
  int32_t first;      // first slice marched by this launch
  int32_t count;      // number of slices marched by this launch
  int32_t stride;     // snapshot every `stride` slices (0: none)
  int32_t n_an;       // analytic sources
  int32_t has_laser;  // any laser among the analytic sources
  int32_t nt;         // workgroup threads of the slot layout
  int32_t C;          // rings per thread (ceil(N / nt) for a single workgroup)
  int32_t G;          // workgroups per instance (1, or a cooperative cluster)
  int32_t task0;      // first task of this instance in its launch queue
  int32_t nb;         // beam-table entries
  double dxi, Rp, inv2pidxi;
  int64_t budget;     // wall-clock budget of this launch in 100 MHz ticks (0: none):
                      // the march stops after the slice that exhausts it
  WakeAnalytic an[WAKE_MAX_ANALYTIC];
  // per-ring constants by home slot (RC_* chunks)
  const double *cst;
  const double *ion;          // [N+1][WAKE_ION_REC]
  const double *tot0;         // [4]: sum_j w_j ln r0_j (dd), total weight Q (dd)
  // beam table (CSR over slices)
  const int32_t *boff;        // [n_xi + 1]
  const double *br, *bcum;    // [nb]
  // ring state by slot, two buffers (RS_* chunks): rho, u_r, AB2 history,
  // ln rho (dd), home slot, ion-interval search hint.  A slice reads
  // the rings of its sorted positions from the current buffer (through the
  // order permutation) and writes them to the slots of those positions in
  // the other buffer.
  double *st[2];
  // slice scratch by position slot (SC_* chunks): psi, d_rho psi, B^(b);
  // laser |a|^2 and d_rho |a|^2
  double *sc, *a2, *da2;
  // order fix-up with global keys: ring order (sorted position, slot form ->
  // slot), prefix maximum keys, run boundaries, run starts / long-run marks,
  // long-run sort keys
  int32_t *perm;
  double *sm_r;
  int32_t *sm_i, *flag, *cls;
  double *sk_r[2];
  int32_t *sk_i[2], *sk_s[2];
  int32_t *free_slot;
  // cooperative instances: exchange packs [2][G][16] and stamps [2][G], control words
  // (barrier arrivals, give-up flag), sort keys by slot, fallback sort arrays
  // of the next power of two >= N
  double *xd;
  int32_t *xc;
  double *gk_r;
  int32_t *gk_i;
  double *bt_r;
  int32_t *bt_i, *bt_s;
  // outputs
  double *axis;               // [n_xi][2]: psi(0), E_z(0)
  double *snap;               // [n_rec][6][N] by ring id
  double *last;               // [6][N] by ring id: last marched slice
  int32_t *ctl;               // [CTL_NWORDS]
  unsigned long long *cnt;    // [CNT_N]
  // radial field grid (none while grid_n is 0): nodes r_g = (g + 1/2)
  // grid_dr, g < grid_n; fields of every slice [n_xi][5][grid_n] (psi,
  // E_r - B_theta, E_z, B_theta, chi); per node [grid_n][WAKE_GRID_TAB]: ln r_g,
  // the ions' psi - psi(0) and d_rho psi at r_g, as dd pairs
  int32_t grid_n;
  double grid_dr;
  double *grid;
  const double *grid_tab;
  double *grid_scr;           // [grid_n + 1][12]: the owning interval's sums handed to each node
  // explicit node radii (null: the uniform nodes above).  Without grid_off
  // the same grid_n radii (ascending) serve every slice; with it, slice n's
  // nodes are entries grid_off[n] .. grid_off[n+1]-1 (ascending within the
  // slice), node records and fields are per entry (the slice's fields at
  // grid + 5 grid_off[n], [5][count], chi not deposited) and grid_n is the
  // most nodes a slice has
  const double *grid_rad;
  const int32_t *grid_off;
  // chi deposit on fixed node sets (when grid_chi is set): per thread of the
  // instance (G nt of them), the sums of c and c rho of the chunks after its
  // own (dd pairs)
  double *grid_thr;
  int32_t grid_chi;
};

// Per-ring records, stored as planes of 16-B chunks of two doubles: chunk c
// of slot i at element c * S + i of the array (S = C * nt slots), so that a
// wave reads one chunk of 64 consecutive slots as contiguous 16-B lanes.
// The state ends with two planes of 4-B words where chunk RS_W would start
// (int32 4 * RS_W * S): the ring's home slot at word i, and at word S + i
// its ion interval at the previous slice (kept for instances whose ion nodes
// are not staged in LDS).  A state buffer holds RS_DOUBLES * S doubles.
enum { RS_RU = 0, RS_F, RS_LN, RS_W, RS_DOUBLES = 2 * RS_W + 1 };   // (rho, u_r) (f_rho, f_u) (ln rho); hs, hint
enum { RC_W = 0, RC_R0, RC_LN, RC_CHUNKS };             // (w, w^) (r0, 1/r0) (ln r0)
enum { SC_PSI = 0, SC_CHUNKS };                         // (psi, d_rho psi)

// Quantities of a snapshot, in this order: psi, E_r - B_theta, E_z,
// B_theta, rho, u_r.
enum { OUT_PSI = 0, OUT_ERBT, OUT_EZ, OUT_BT, OUT_RHO, OUT_UR, OUT_N };
