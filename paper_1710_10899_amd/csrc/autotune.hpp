// Tuning table for the persistent launches of the large-order path.
#pragma once

namespace submat {

// Workgroups per compute unit for the persistent large-order kernels of a
// chunk whose largest submatrix order is max_m.
int tuned_blocks_per_cu(int max_m, int fp64);

// Workgroups per compute unit for the tridiagonal eigensolver (the
// workgroups of a compute unit share its LDS).
int tuned_eig_blocks_per_cu(int max_m);

// Reloads the table: from the file named by SUBMAT_TUNE_FILE when use_file
// (built-in defaults when unset, unreadable or empty), else the defaults.
void reload_tuning(bool use_file);

// Whether the current table came from a file.
bool tuning_from_file();

}  // namespace submat
