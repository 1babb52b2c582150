// fgh_batch.hpp -- host-side queries shared by the serving loop and the solver drivers.
#pragma once
#include <stdint.h>

namespace fgh {

// FGH_BATCH=0 turns shared launches (and the server's grouping by size class) off.
bool batching_enabled();

// Whether FP32-refined solves with this grid, rule and solver run their inner loops in shared
// launches under fgh_solve_batch (size-specialised passes along every axis; CG or Eyre-Milton).
bool batch_shares_launches(int d, const int32_t* N, int rule, int precision, int solver);

// Contrast C/c of a packed phase table: the largest eigenvalue of its blocks over the smallest
// (0 if a block is not positive definite or the table is not finite).
double phase_table_contrast(int d, const double* table, int n_phases);

}  // namespace fgh
