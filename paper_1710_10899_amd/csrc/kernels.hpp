// Host-side launch interface between the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace submat {

// Status counter slots (int64 each) in the per-device status block.
enum StatusSlot : int {
  ST_NONPOS = 0,      // submatrices with an eigenvalue <= 0
  ST_FALLBACK = 1,    // submatrices redone in FP64 by the mixed path
  ST_UNCONV = 2,      // eigensolver did not converge
  ST_INVITER = 3,     // eigenvectors computed by inverse iteration (eigenvalue clusters)
  ST_STALE = 4,       // columns whose order exceeds what the plan was built for (NaN output)
  ST_PATTERN = 5,     // calls whose pattern failed device-side validation (no output written)
  ST_DONE = 6,        // columns whose output (forward column or adjoint terms) was written
  ST_NSLOTS = 64,
};


// Pattern error bits written by the plan kernel.
enum PatternBits : uint32_t {
  PAT_ROWPTR = 1u,   // rowptr not 0..nnz non-decreasing
  PAT_RANGE = 2u,    // column index out of range
  PAT_ORDER = 4u,    // row not strictly increasing
  PAT_ASYM = 8u,     // (i,j) stored but (j,i) not
  PAT_NODIAG = 16u,  // diagonal not stored
};

// ---- plan / utility kernels (plan.hip) ----
hipError_t launch_plan_pattern(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz,
                               int32_t* m_out, int32_t* c_out, uint32_t* err, hipStream_t s);
hipError_t launch_fill_zero(void* ptr, int64_t bytes, hipStream_t s);
hipError_t launch_reset_status(int64_t* status, int32_t* counters, int ncounters, hipStream_t s);

// ---- one-wavefront Jacobi path (small.hip) ----
// Spectral function applied to every submatrix (codes match the ABI's).
enum FnKind : int { FN_INV_ROOT = 0, FN_ROOT = 1, FN_POWER = 2 };
struct SpecFn {
  int kind;      // FnKind
  int p;         // root order (the two root functions)
  double alpha;  // exponent (real power)
};

struct SmallArgs {
  const int32_t* rowptr;
  const int32_t* colind;
  const void* vals;      // value type vdtype
  int vdtype;            // 0 = f64, 1 = f32
  const int32_t* items;  // columns on this path, largest m first
  const int32_t* cidx;   // c_j per column
  int n_items;
  int mmax;              // largest m among items
  SpecFn fn;
  int mixed;             // 1: FP32 bulk with FP64 redo of flagged submatrices
  double kappa_max;
  void* x;               // forward output (nullptr in backward)
  const void* gx;        // backward input (nullptr in forward)
  void* ga;              // backward output, accumulated (zeroed by the caller)
  int64_t* status;
  int32_t* work_ctr;     // zeroed before the launch
  int grid;              // persistent grid size
  double* dout;          // backward, deterministic: D_j is written here (m x m, column-major)
  const int64_t* doff;   //   at dout + doff[j] instead of being scatter-added,
  const int32_t* dld;    //   in a slot planned for order dld[j]
  const uint32_t* pattern_err;  // device-side pattern validation bits of this call (nullptr: validated
                                // at plan build); nonzero: the launch writes nothing
};
hipError_t launch_small(const SmallArgs& a, hipStream_t s);

// ---- forward without allocation (noalloc.hip) ----
// Largest n of the entry point that allocates nothing, and its per-device
// scratch: status slots, the pattern error word, a work counter, m_j, c_j.
constexpr int32_t kNoAllocMaxN = 1 << 20;
int noalloc_forward(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n, int64_t nnz,
                    SpecFn fn, int32_t vdtype, int mixed, double kappa_max, void* x, int num_cus, hipStream_t s,
                    int64_t** status_out);

// ---- deterministic adjoint assembly (adjoint_reduce.hip) ----
struct DetReduceArgs {
  const int32_t* rowptr;
  const int32_t* colind;
  const int32_t* tpos;    // transpose position of every stored entry
  int32_t n;
  int32_t phase;          // columns j with dphase[j] == phase contribute
  const int32_t* dphase;  // per column: the phase whose launch leaves D_j in memory
  const int32_t* dld;     // per column: leading dimension of D_j
  const int64_t* doff;    // per column: offset of D_j from base (elements, or bytes when bytes_off)
  const void* base;
  int bytes_off;
  void* ga;               // accumulated in place (zeroed at the start of the call)
};
hipError_t launch_adjoint_reduce(const DetReduceArgs& a, int vdtype, int num_cus, hipStream_t s);
// upper entries of grad_a += their lower mirrors (after the lower-triangle
// scatter-adds of every phase)
hipError_t launch_adjoint_mirror(const int32_t* rowptr, const int32_t* colind, const int32_t* tpos, int n,
                                 void* ga, int vdtype, int num_cus, hipStream_t s);

// ---- large-order path (large.hip) ----
struct LargeArgs {
  const int32_t* rowptr;
  const int32_t* colind;
  const int32_t* tpos;    // per stored entry: position of its transpose entry
  const void* vals;
  int vdtype;
  const int32_t* items;   // chunk items -> column id
  const int32_t* cidx;    // c_j per column
  const int32_t* ldm;     // per item: leading dimension (padded order)
  // All offsets are in BYTES, so an FP32 and an FP64 view of one slot start
  // at the same address.
  const int64_t* off;     // per item: S and W slab offset
  const int64_t* qoff;    // per item: Q slab offset (workspace or saved buffer)
  const int64_t* voff;    // per item: offset of its e / tau vectors
  const int64_t* doff;    // per item: offset of d (eigenvalues after the eigensolver)
  const int64_t* eoff;    // per item: offset of its scratch (eigensolver, back-transformation)
  int n_items;
  int max_m;
  void* S;                // slab base (gathered S_j, then the Householder vectors)
  void* Q;                // slab base (Z, then the eigenvectors Q1 Z)
  void* W;                // slab base (panel W of the reduction, adjoint scratch)
  void* d;                // per item vectors (eigenvalues after the eigensolver)
  void* e;
  void* tau;
  void* escr;             // scratch of the eigensolver and the back-transformation
  int32_t* flags;         // per item: bit0 nonpositive, bit1 fallback, bit2 unconverged
  SpecFn fn;
  double kappa_max;
  double cluster_tol;     // relative eigenvalue gap below which inverse iteration is used
  int lds_limit;          // device limit on LDS bytes per workgroup
  int panel_rows;         // reduction: rows of the panel kept in LDS (set by its launcher)
  int panel_off;          // reduction: offset (doubles) of that copy after the row partials
  int nb;                 // reduction: panel width (even, 2..48)
  int red_per_cu;         // reduction: workgroups per compute unit its LDS is laid out for (1 or 2)
  void* x;                // forward output (value type vdtype)
  const void* gx;         // backward input
  void* ga;               // backward output (accumulated)
  int64_t* status;
  int32_t* work_ctr;
  int grid;
  int fp64;               // 1: compute in FP64, 0: FP32
  int only_flagged;       // 1: process only items whose fallback flag is set
  int det;                // backward: leave D_j (FP64, lower triangle) in the W slab instead of
                          // scatter-adding it (deterministic assembly afterwards)
  int xcd_queues;         // unit launches: work_ctr holds kXcdQueues counters, one queue per XCD
};
enum LargeFlags : int32_t { LF_NONPOS = 1, LF_FALLBACK = 2, LF_UNCONV = 4 };

hipError_t launch_gather_large(const LargeArgs& a, hipStream_t s);
hipError_t launch_tridiagonalise(const LargeArgs& a, hipStream_t s);
// Workgroups per compute unit of the reduction: per_cu, lowered until each
// workgroup's LDS share holds its fixed part and min(nb, max_m) panel rows.
int reduction_fit_per_cu(int max_m, int nb, int fp64, int64_t lds_limit, int per_cu);
int back_blocks_per_cu();       // the same for the back-transformation
int adjoint_blocks_per_cu();    // and for the adjoint
hipError_t launch_tridiag_eig(const LargeArgs& a, hipStream_t s);
hipError_t launch_eig_orth(const LargeArgs& a, hipStream_t s);
// back-transformation Q = Q1 Z: VT = V T^T per item and reflector block,
// then the blocks applied per (item, column block) unit
hipError_t launch_back_prep(const LargeArgs& a, hipStream_t s);
hipError_t launch_back_apply(const LargeArgs& a, hipStream_t s);
int back_apply_units(int n_items, int max_m);  // units of launch_back_apply
constexpr int kXcdQueueCount = 8;               // work queues of a unit launch with xcd_queues
size_t eig_lds_bytes(int max_m);
size_t apply_scratch_elems(int ld);  // scratch elements per item of the back-transformation
hipError_t launch_apply_column(const LargeArgs& a, hipStream_t s);
// the forward's column from the reflectors and Z, without forming Q
// (one wavefront per submatrix)
hipError_t launch_column_factored(const LargeArgs& a, hipStream_t s);
int column_waves_per_cu();
// adjoint: a, b and Ms per item; T1 = Q Ms and D = T1 Q^T (lower) over
// (item, column block) units (units: back_apply_units); D into grad_a
hipError_t launch_adjoint_prep(const LargeArgs& a, hipStream_t s);
hipError_t launch_adjoint_product(const LargeArgs& a, int lower, hipStream_t s);
hipError_t launch_adjoint_scatter(const LargeArgs& a, hipStream_t s);

}  // namespace submat
