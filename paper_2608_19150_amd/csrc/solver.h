// The DIRK/Picard solver object (shared by the single-instance and the
// batched drivers).
#pragma once
#include <vector>

#include "internal.h"

// A captured chunk of Picard iterations, keyed by everything the captured
// launches depend on: the stage, the moments' buffer parity and the buffers
// read and written at the chunk's start.
struct ChunkKey {
  int stage, ucur;
  const void *prev, *out, *fk, *q;
  bool operator==(const ChunkKey& o) const {
    return stage == o.stage && ucur == o.ucur && prev == o.prev && out == o.out && fk == o.fk &&
           q == o.q;
  }
};

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
  double* msplit = nullptr;      // chunk sums of the velocity-split moment pass (or null)
  double* ratio = nullptr;       // [4]
  int32_t* status = nullptr;     // [2]
  unsigned long long* numax = nullptr;
  uint8_t* sticky = nullptr;     // MATCHED nodes held on DIRECT for the stage
  // pinned host mirror: ratio[4], numax bits, status[2]
  double* h_info = nullptr;
  hipEvent_t ev[4] = {};  // kernel timing: before maxw, before sweep, before moments, after
  // device control block of the chunked iteration: int32 [0] done (0 running,
  // 1 converged, 2 failed), [1] iterations of the stage, [2] MATCHED
  // fallbacks of the stage, [3] error code, [4] non-physical nodes; double at
  // byte 32: the last max ratio
  int32_t* ctl = nullptr;
  hipStream_t cap = nullptr;  // capture stream (graph mode)
  std::vector<std::pair<ChunkKey, hipGraphExec_t>> graphs;
};

namespace bgk {
int set_tableau(bgk_solver* s, int tab);
}  // namespace bgk
