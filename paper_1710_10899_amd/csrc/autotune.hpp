// Tuning table for the persistent launches of the large-order path.
#pragma once

namespace submat {

// Workgroups per compute unit for the persistent large-order kernels of a
// chunk whose largest submatrix order is max_m.
int tuned_blocks_per_cu(int max_m, int fp64);

// Blocks per compute unit for the QL kernel (one wave per block; the
// blocks of a compute unit share its LDS).
int tuned_ql_blocks_per_cu(int max_m);

// Reloads the table from the file named by SUBMAT_TUNE_FILE (if set).
void reload_tuning();

}  // namespace submat
