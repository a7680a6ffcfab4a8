// Internal data layout shared by the host runtime and the gfx950 kernels of
// the gridless ring solver.  Not part of the public ABI (include/wake.h).
#pragma once
#include <stdint.h>

#define WAKE_MAX_ANALYTIC 8   // analytic beams + lasers per instance
#define WAKE_BCAP 2048        // beam-table entries staged in LDS per chunk
#define WAKE_NSCR 9           // per-ring scratch arrays of the multi-tile path

// Scratch array slots (multi-tile path), each [N] doubles by sorted position.
enum { SC_PSI = 0, SC_DPSI, SC_BB, SC_G0, SC_G1, SC_E0, SC_E1, SC_A2, SC_DA2 };

// Control words of one instance (device memory, int32).
enum { CTL_CUR = 0, CTL_BREAK = 1, CTL_NEXT = 2, CTL_NWORDS = 4 };

struct WakeAnalytic {
  int32_t kind;     // 2 = bi-Gaussian beam, 3 = Gaussian laser envelope
  int32_t pad;
  double q, n_peak, sigma_r, sigma_xi, xi_c;  // beam
  double a0, w0, L, xi_l;                     // laser
};

// One instance as the kernels see it.  All pointers are device pointers.
struct WakeInst {
  int32_t N;          // rings
  int32_t n_xi;       // slices of the window
  int32_t first;      // first slice marched by this launch
  int32_t count;      // number of slices marched by this launch
  int32_t stride;     // snapshot every `stride` slices (0: none)
  int32_t n_an;       // analytic sources
  int32_t has_laser;  // any laser among the analytic sources
  int32_t lut_n;      // buckets of the ion-node lookup table
  int32_t nb;         // beam-table entries
  int32_t pad;
  double dxi, Rp, Q, lut_scale;   // lut_scale = lut_n / Rp
  double inv2pidxi;               // 1 / (2 pi dxi)
  WakeAnalytic an[WAKE_MAX_ANALYTIC];
  // constants by ring id: weight, modified weight, ln r0 (double-double)
  const double *w, *wh;
  const double *L0_hi, *L0_lo;
  // ion nodes (N+2): radius, d_rho psi (dd), psi - psi(0) (dd)
  const double *ion_r, *ion_dp_hi, *ion_dp_lo, *ion_ps_hi, *ion_ps_lo;
  const double *tot0;             // [2]: sum_j w_j ln r0_j (dd)
  const int32_t *ion_lut;         // [lut_n + 1]
  // beam table (CSR over slices)
  const int32_t *boff;            // [n_xi + 1]
  const double *br, *bcum;        // [nb]
  // ring state, two buffers, by sorted position
  double *rho[2], *u[2], *fr[2], *fu[2];
  int32_t *id[2];
  // multi-tile scratch
  double *scr;                    // [WAKE_NSCR][N]
  double *tscr;                   // [tiles][threads][5]
  double *skey_r[2];              // [N] global merge buffers (multi-tile sort)
  int32_t *skey_i[2], *skey_p[2];
  // outputs
  double *axis;                   // [n_xi][2]: psi(0), E_z(0)
  double *snap;                   // [n_rec][6][N] by ring id
  double *last;                   // [6][N] by ring id: last marched slice
  int32_t *ctl;                   // [CTL_NWORDS]
};

// Quantities of a snapshot, in this order: psi, E_r - B_theta, E_z,
// B_theta, rho, u_r.
enum { OUT_PSI = 0, OUT_ERBT, OUT_EZ, OUT_BT, OUT_RHO, OUT_UR, OUT_N };
