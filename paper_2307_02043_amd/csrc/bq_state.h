// Per-system BiCGSTAB state kept in device memory (all scalars FP64), and
// the argument blocks of the Green's-operator passes.
#pragma once

#include "bq_common.h"

namespace bq {

enum SysStatus : int {
  SYS_RUNNING = 0,
  SYS_CONVERGED = 1,
  SYS_NOTCONV = 2,
  SYS_BREAKDOWN = 3,
  SYS_NONFINITE = 4,
};

struct SysState {
  double rho_x, rho_y;          // rho = <rhat, r> of the previous iteration
  double rhon_x, rhon_y;        // rho_new
  double alpha_x, alpha_y;
  double omega_x, omega_y;
  double beta_x, beta_y;
  double bnorm2;                // ||b||^2
  double res;                   // last relative (recursive) residual
  int status;
  int iters;
  int sflag;                    // converged on the half step ||s||
  int first;                    // no iteration done yet
  double tol;
  int max_iter;
  int mvs;                      // solver matvecs done (G applications)
  double brk;                   // |rho|, |<rhat, v>| or |omega| below this: breakdown
};

// Which systems a solver pass works on.
enum RunMask : int { RUN_ALL = 0, RUN_ACTIVE = 1, RUN_ACTIVE_NOT_S = 2 };

__device__ inline bool sys_skip(const SysState* st, int mask, int b) {
  if (mask == RUN_ALL || st == nullptr) return false;
  const SysState& s = st[b];
  if (s.status != SYS_RUNNING) return true;
  if (mask == RUN_ACTIVE_NOT_S && s.sflag) return true;
  return false;
}

// Prologue of the forward z pass: what field the Green's operator acts on.
enum ZfMode : int {
  ZF_XV = 0,       // x . v
  ZF_XUIN = 1,     // x . u_in (plane wave generated in-register)
  ZF_DETCONJ = 2,  // S^T conj(r_det): conj of the detector image on z = N-1
  ZF_V = 3,        // v
  ZF_VCONJ = 4,    // conj(v)
  ZF_XP_UPD = 5,   // BiCGSTAB direction update fused in: p = r + beta (p - omega v)
                   // (p = r on the first iteration) written back, then x . p
};

// Epilogue of the inverse z pass.
enum ZiMode : int {
  ZI_G = 0,         // out = G w
  ZI_GCONJ = 1,     // out = conj(G w)
  ZI_AV_RHAT = 2,   // out = v - G w ; partial <rhat, out>
  ZI_AS_TS = 3,     // out = s - G w ; partials <out, s>, <out, out>
  ZI_G_NORM = 4,    // out = out2 = G w ; partial ||out||^2
  ZI_RES_NORM = 5,  // out = out2 = b - e0 + G w (e0 in vz; b = bsrc, or the
                    // plane wave from inc when bsrc is null) ; partial ||out||^2
};

template <typename T>
struct PassArgs {
  int N, B;
  int mask;                    // RunMask
  const SysState* state;
  // z-forward prologue
  int zf_mode;
  const T* xpot;               // scattering potential, N^3 real
  const C<T>* vin;             // B x N^3
  const C<T>* rdet;            // B x N^2 detector residual
  const C<double>* inc;        // B x 3 x N plane-wave factors (x, y, z)
  C<T>* pio;                   // ZF_XP_UPD: p (read, then overwritten)
  const C<T>* rvec;            // ZF_XP_UPD: r
  const C<T>* vvec;            // ZF_XP_UPD: v of the previous iteration
  // intermediates
  C<T>* zh;                    // B x 2 x N^3
  C<T>* xh;                    // B x 4 x N^3 (split xy path)
  const C<T>* ghat;            // 8 x N^3 parity-class transfer function
  const C<T>* twN;             // W_N^k, k < N
  const C<T>* twH;             // exp(-i pi n / N), n < N
  // z-inverse epilogue
  int zi_mode;
  const C<T>* vz;              // v (ZI_AV_RHAT), s (ZI_AS_TS) or e0 (ZI_RES_NORM)
  const C<T>* bsrc;            // right-hand side b (ZI_RES_NORM), null: plane wave
  const C<T>* rhat;
  C<T>* out;
  C<T>* out2;
  double* partial;             // B x NP x 4
  int xy_fused;                // use the LDS-resident plane pass when available
  // launch shapes chosen by the autotuner (0: default); host side only
  int xtile;                   // rows per workgroup of the x passes
  int zf_threads;              // threads per workgroup of the padded z-forward pass
};

}  // namespace bq
