// The DIRK/Picard solver object (shared by the single-instance and the
// batched drivers).
#pragma once
#include "internal.h"

struct bgk_solver {
  const tgs_dag* dag = nullptr;
  bgk_solver_opts opts{};
  int S = 1;
  double A[4][4] = {}, b[4] = {}, c[4] = {};
  bool stiffly_accurate = true;
  // linear-combination coefficients over {f^k, f^(1..S)}
  double qcoef[4][5] = {}, Fcoef[4][5] = {}, ncoef[5] = {};
  double* fk = nullptr;          // copy of f^k
  double* fst[4] = {};           // converged stage values
  double* fping = nullptr;       // previous iterate (lagged facets / FP32 form)
  double* q = nullptr;           // stage source
  float* d32 = nullptr;          // FP32 correction traces
  double* U[2] = {};             // moments ping-pong
  double* mcoef = nullptr;
  double* mtab = nullptr;        // factorised Maxwellian tables (tensor grids)
  double* pr = nullptr;          // per-axis projections (PROJECTED mode)
  double* bcd = nullptr;         // dense boundary data [n_bfaces][n_fp][n_v]
  double* nu = nullptr;
  double* partial = nullptr;
  double* ratio = nullptr;       // [4]
  int32_t* status = nullptr;     // [2]
  unsigned long long* numax = nullptr;
  uint8_t* sticky = nullptr;     // MATCHED nodes held on DIRECT for the stage
  // pinned host mirror: ratio[4], numax bits, status[2]
  double* h_info = nullptr;
  hipEvent_t ev[4] = {};  // kernel timing: before maxw, before sweep, before moments, after
};

namespace bgk {
int set_tableau(bgk_solver* s, int tab);
}  // namespace bgk
