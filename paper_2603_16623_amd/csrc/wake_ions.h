// Internal layout of two-species instances (plasma electrons and mobile
// ions), shared by the host runtime and the gfx950 kernels.  Not part of the
// public ABI (include/wake.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wake_common.h"

#define WAKE_IONS_NT 1024      // workgroup threads of the two-species marcher
#define WAKE_IONS_NMAX 8192    // rings per species (the sorted radii of both species sit in LDS)

// per-ring constants by ring id (both species start at the same radii with
// the same weights): w, w^, r0, 1/r0, ln r0 (dd), dr
enum { IK_W = 0, IK_WH, IK_R0, IK_IR0, IK_LNH, IK_LNL, IK_DR, IK_N };
// ring state planes by ring id: rho, u_r, and the Adams-Bashforth history
enum { IS_RHO = 0, IS_U, IS_FR, IS_FU, IS_N };
// node tables of a species by slot: its own psi (dd), d_rho psi (dd) and
// d_zeta psi at its rings; B^(p) at the electron rings
enum { IT_PSH = 0, IT_PSL, IT_DPH, IT_DPL, IT_DZ, IT_BP, IT_N };
// per-position work by slot: the ring's weights and momentum gathered at
// the slice head (w, w^, u_r), the fields (total of both species), psibar,
// the beam field, the laser's |a|^2 and its gradient (with a laser only);
// for the electrons the recursion's A_i, C_i, offset s_i, growing mode g
// before ring i and the det-sum E before it.  ln rho, gamma and the
// interpolation parameters are formed again where they are used.
enum { IW_W = 0, IW_WH, IW_U, IW_PSI, IW_DPSI, IW_DZ, IW_BT, IW_PB, IW_BB, IW_A2, IW_DA2, IW_A, IW_C,
       IW_SA, IW_SB, IW_GA, IW_GB, IW_E, IW_N };

// One two-species instance as the kernels see it.  All pointers are device
// pointers.  Species 0 are the electrons (q = -1, m = 1), species 1 the
// ions (q = +1, m = m_i).  Per species, thread t of the workgroup owns the
// C = ceil(N / 1024) consecutive sorted positions [tC, tC + C); position p
// is stored at slot (p % C) * 1024 + p / C (S = 1024 C slots per plane).
struct WakeIons {
  int32_t N, n_xi, first, count, stride, C;
  int32_t nb, n_an, has_laser, pad;
  double dxi, m_i;
  WakeAnalytic an[WAKE_MAX_ANALYTIC];
  const int32_t* boff;        // beam table (CSR over slices)
  const double *br, *bcum;
  const double* cst;          // [IK_N][N]
  double* st[2];              // two buffers, each [2 species][IS_N][N]
  int32_t* ord;               // [2][N] ring ids in the latest sorted order (by position)
  int32_t* sid;               // [2][S] ring id of each position, by slot
  int32_t* jx;                // [2][S] rings of the other species below each ring (-1: beyond
                              //        its edge), by slot
  double* tab;                // [2][IT_N][S]
  double* work;               // [2][IW_N][S]
  double* axis;               // [n_xi][2]: psi(0), E_z(0)
  double* snap[2];            // per species [n_rec][OUT_N][N] by ring id
  double* last[2];            // per species [OUT_N][N]: the last marched slice
  int32_t* ctl;               // [CTL_NWORDS]; CTL_CUR is the state buffer of the next slice
  unsigned long long* cnt;    // [CNT_N]: slices marched, order fix-ups
};

hipError_t launch_ions_init(const WakeIons& J, const double* r0, const double* dr, const double* dens,
                            bool constants, hipStream_t s);
// the marcher's LDS allowance on the current device (before its first launch there)
hipError_t ions_prepare();
hipError_t launch_ions_march(const WakeIons* d_insts, int n_insts, hipStream_t s);
// back to slice 0 with both species at rest, for n records in device memory
// (the records' own fields are read on the device: capturable)
hipError_t launch_ions_reset(const WakeIons* d_insts, int n_insts, hipStream_t s);
// ring state of species sp at the next slice to out [4][N] (rho, u_r, f_rho, f_u)
hipError_t launch_ions_get_state(const WakeIons& J, int sp, double* out, hipStream_t s);
// replace species sp's state (f_rho/f_u may be null: zero) and make `slice` the next slice
hipError_t launch_ions_set_state(const WakeIons& J, int sp, const double* rho, const double* u,
                                 const double* fr, const double* fu, int slice, hipStream_t s);
size_t ions_lds_bytes();
