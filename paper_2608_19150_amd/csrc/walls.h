// Wall boundary data for the solver (walls.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/bgktgs.h"

namespace bgk {

const tgs_dag* walls_dag(const tgs_walls* w);
// fills the wall rows of bc_dense [n_bfaces][n_fp][n_v] from f (sweep layout)
// (a non-null `skip` turns the launch into a no-op while *skip is nonzero)
int launch_wall_values(const tgs_walls* w, const double* f, double* bc_dense, hipStream_t stream,
                       const int32_t* skip = nullptr);
// bc_dense[bf][p][j] = Maxwellian of bc_coef[bf][p] at velocity j, every facet
int launch_bc_dense(const tgs_dag* d, const double* bc_coef, double* bc_dense,
                    hipStream_t stream);

}  // namespace bgk
