// Sparse products and Krylov loops around the submatrix method's result
// (krylov.hip): shared declarations for the host orchestration in api.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace submat {

// CSR matrix for the row-wise product y[i] = sum_{q in row i} vals[q] x[colind[q]]
struct SpmvArgs {
  const int32_t* rowptr;
  const int32_t* colind;
  const double* vals;
  int n;
  int lanes;  // lanes per row (power of two, 4..64)
};

// Scratch of the deterministic grid reductions
struct KrylovScratch {
  double* partials;  // reduction_blocks() doubles
  uint32_t* ticket;  // zero between reductions
};

// Scalars of a CG solve, in device memory
struct CgState {
  double rr;     // r . r
  double pq;     // p . (B p)
  double beta;   // rr_new / rr
  double bnorm;  // ||r_0|| = ||b'||
  double tol;    // relative residual threshold
  int32_t iters;
  int32_t done;
  int32_t breakdown;  // p . B p <= 0 or a non-finite residual
  int32_t pad;
};

int spmv_lanes(double mean_row);
int reduction_blocks();
hipError_t launch_transpose_positions(const int32_t* rowptr, const int32_t* colind, int n, int32_t* tpos,
                                      hipStream_t s);
hipError_t launch_gather_transpose(const int32_t* tpos, const double* vals, int64_t nnz, double* out, hipStream_t s);
hipError_t launch_spmv(const SpmvArgs& a, const double* x, double* y, double c, const double* sv, const int32_t* done,
                       hipStream_t s);
hipError_t launch_dot(const double* a, const double* b, int64_t n, KrylovScratch& k, double* out, const int32_t* done,
                      hipStream_t s);
hipError_t launch_scale(const double* x, double* y, int64_t n, const double* num, const double* den, int sqrt_den,
                        hipStream_t s);
hipError_t launch_random_vector(double* v, int64_t n, uint64_t seed, hipStream_t s);
hipError_t launch_gemv_t(const double* V, int64_t n, int ncol, const double* w, double* h, hipStream_t s);
hipError_t launch_gemv_n_sub(const double* V, int64_t n, int ncol, const double* h, double* w, double* alpha, int j,
                             hipStream_t s);
hipError_t launch_tridiag_max(const double* a, const double* b2, int k, double* out, hipStream_t s);
hipError_t launch_cg_start(double* x, const double* r, double* p, int64_t n, CgState* st, KrylovScratch& k,
                           hipStream_t s);
hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q, int64_t n, CgState* st,
                            KrylovScratch& k, hipStream_t s);
hipError_t launch_cg_direction(double* p, const double* r, int64_t n, const CgState* st, hipStream_t s);

hipError_t launch_densify(const int32_t* rowptr, const int32_t* colind, const double* vals, int n, int colbased,
                          double* D, hipStream_t s);
hipError_t launch_residual_fro2(const double* T, int n, KrylovScratch& k, double* out, hipStream_t s);

}  // namespace submat
