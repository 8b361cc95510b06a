// Tuning table for the persistent launches of the large-order path.
#pragma once

namespace submat {

// Workgroups per compute unit for the persistent large-order kernels of a
// chunk whose largest submatrix order is max_m.
int tuned_blocks_per_cu(int max_m, int fp64);

// Workgroups per compute unit for the tridiagonal eigensolver (the
// workgroups of a compute unit share its LDS).
int tuned_eig_blocks_per_cu(int max_m);

// Panel width and workgroups per compute unit of the tridiagonal reduction
// for a chunk whose largest order is max_m, in FP64 or FP32.
int tuned_reduction_nb(int max_m, int fp64);
int tuned_reduction_per_cu(int max_m, int fp64);

// Largest order of the one-wavefront (Jacobi) bucket, 1..64.
int tuned_small_max();

// Reloads the table: from the file named by SUBMAT_TUNE_FILE when use_file
// (built-in defaults when unset, unreadable or empty), else the defaults.
void reload_tuning(bool use_file);

// Whether the current table came from a file.
bool tuning_from_file();

}  // namespace submat
