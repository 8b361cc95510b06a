// Sparse products and Krylov loops that consume the submatrix method's
// result (gfx950, wave64, FP64):
//   * the residual metric of Section 4.1, ||X^p A - I||_2 = sqrt(lambda_max(R^T R)),
//     by Lanczos on R^T R applied matrix-free (R v = X^p (A v) - v);
//   * the preconditioned CG of Section 4.4 on K^T A K y = K^T b, x = K y.
// Every loop body is a short sequence of kernels; reductions are
// deterministic (per-block partials summed in a fixed order by the block
// that finishes last), and every kernel of the CG loop reads a device flag
// and returns at once after convergence, so the host can enqueue iterations
// in batches and only poll a scalar.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "krylov.hpp"

namespace submat {

constexpr int kKB = 256;            // threads per block
constexpr int kKW = 64;             // wave size
constexpr int kRedGrid = 512;       // blocks of a reduction (partials buffer size)

__device__ __forceinline__ double kwave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kKW);
  return v;
}

// Sum of a block's per-thread values (kKB threads), valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = kwave_sum(v);
  const int w = threadIdx.x / kKW;
  if ((threadIdx.x & (kKW - 1)) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kKB / kKW; ++i) t += sh[i];
  return t;
}

// Deterministic grid reduction tail: every block deposits its partial; the
// block that arrives last (ticket) sums all partials in index order and
// returns true in thread 0 with the total in *total. The ticket is reset for
// the next reduction.
__device__ bool grid_reduce_last(double part, double* partials, uint32_t* ticket, double* total) {
  __shared__ bool s_last;
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = part;
    __threadfence();
    const uint32_t t = atomicAdd(ticket, 1u);
    s_last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double v = 0.0;
  if (threadIdx.x < kKW) {
    for (int i = threadIdx.x; i < (int)gridDim.x; i += kKW) v += partials[i];
    v = kwave_sum(v);
  }
  if (threadIdx.x == 0) {
    *total = v;
    *ticket = 0u;
  }
  return threadIdx.x == 0;
}

// ----------------------------------------------------------- pattern helpers
// tpos[q] = position of the entry (colind[q], i) for q in row i; the
// pattern is structurally symmetric (validated), so it exists.
__global__ __launch_bounds__(kKB) void k_transpose_positions(const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ colind, int n,
                                                             int32_t* __restrict__ tpos) {
  const int row = (int)((blockIdx.x * (int64_t)kKB + threadIdx.x) / kKW);
  const int lane = threadIdx.x & (kKW - 1);
  if (row >= n) return;
  for (int q = rowptr[row] + lane; q < rowptr[row + 1]; q += kKW) {
    const int j = colind[q];
    int lo = rowptr[j], hi = rowptr[j + 1] - 1, pos = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int c = colind[mid];
      if (c == row) { pos = mid; break; }
      if (c < row) lo = mid + 1; else hi = mid - 1;
    }
    tpos[q] = pos;
  }
}

// out[q] = vals[tpos[q]]: the value array of M^T on the same pattern.
__global__ __launch_bounds__(kKB) void k_gather_transpose(const int32_t* __restrict__ tpos,
                                                          const double* __restrict__ vals, int64_t nnz,
                                                          double* __restrict__ out) {
  for (int64_t q = blockIdx.x * (int64_t)kKB + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * kKB)
    out[q] = vals[tpos[q]];
}

// ------------------------------------------------------------------- SpMV
// y[i] = sum_{q in row i} vals[q] x[colind[q]] + c * s[i] (s may be null).
// L lanes per row (64 / L rows per wave); the lanes of a row stride over its
// entries so that vals and colind are read in coalesced runs.
template <int L>
__global__ __launch_bounds__(kKB) void k_spmv(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                              const double* __restrict__ vals, const double* __restrict__ x,
                                              double* __restrict__ y, int n, double c, const double* __restrict__ s,
                                              const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int64_t g = blockIdx.x * (int64_t)kKB + threadIdx.x;
  const int row = (int)(g / L);
  const int sub = threadIdx.x & (L - 1);
  double acc = 0.0;
  if (row < n) {
    const int q1 = rowptr[row + 1];
    for (int q = rowptr[row] + sub; q < q1; q += L) acc = fma(vals[q], x[colind[q]], acc);
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kKW);
  if (row < n && sub == 0) y[row] = s ? fma(c, s[row], acc) : acc;
}

// ---------------------------------------------------------------- vectors
// out = a . b (deterministic)
__global__ __launch_bounds__(kKB) void k_dot(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                             double* partials, uint32_t* ticket, double* out,
                                             const int32_t* __restrict__ done) {
  __shared__ double sh[kKB / kKW];
  if (done && *done) return;
  double v = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB)
    v = fma(a[i], b[i], v);
  v = block_sum(v, sh);
  double tot;
  if (grid_reduce_last(v, partials, ticket, &tot)) *out = tot;
}

// y = a * x with a = num[0] / den[0] (or sqrt(den[0]) when sqrt_den), read
// from device memory; a non-positive denominator gives y = 0; num null
// reads as 1, den null as no division.
__global__ __launch_bounds__(kKB) void k_scale(const double* __restrict__ x, double* __restrict__ y, int64_t n,
                                               const double* __restrict__ num, const double* __restrict__ den,
                                               int sqrt_den) {
  double a = num ? *num : 1.0;
  if (den) {
    const double d = sqrt_den ? sqrt(*den) : *den;
    a = d > 0.0 ? a / d : 0.0;
  }
  for (int64_t i = blockIdx.x * (int64_t)kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) y[i] = a * x[i];
}

// Seeded start vector: splitmix64 of (seed, i) mapped to [-1, 1).
__global__ __launch_bounds__(kKB) void k_random_vector(double* __restrict__ v, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// ----------------------------------------------------------------- Lanczos
// h[c] = V[:, c] . w for c < ncol (one block per column; V column-major, ld n)
__global__ __launch_bounds__(kKB) void k_gemv_t(const double* __restrict__ V, int64_t n, int ncol,
                                                const double* __restrict__ w, double* __restrict__ h) {
  __shared__ double sh[kKB / kKW];
  const int c = blockIdx.x;
  if (c >= ncol) return;
  const double* v = V + (int64_t)c * n;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kKB) acc = fma(v[i], w[i], acc);
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) h[c] = acc;
}

// w -= V[:, :ncol] h; alpha[j] += h[j] (the reorthogonalisation's correction
// of the Lanczos coefficient, applied by block 0) when alpha is given.
__global__ __launch_bounds__(kKB) void k_gemv_n_sub(const double* __restrict__ V, int64_t n, int ncol,
                                                    const double* __restrict__ h, double* __restrict__ w,
                                                    double* alpha, int j) {
  for (int64_t i = blockIdx.x * (int64_t)kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) {
    double acc = 0.0;
    for (int c = 0; c < ncol; ++c) acc = fma(V[(int64_t)c * n + i], h[c], acc);
    w[i] -= acc;
  }
  if (alpha && blockIdx.x == 0 && threadIdx.x == 0) alpha[j] += h[j];
}

// Largest eigenvalue of the k x k symmetric tridiagonal matrix (diagonal a,
// squared off-diagonal b2[0..k-2]) by multisection with Sturm counts: one wave, each
// round splits the bracket into 65 parts (lane l tests point l + 1), so 10
// rounds narrow it by 65^10 ~ 1e18.
__device__ int sturm_below(const double* a, const double* b2, int k, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    d = (a[i] - x) - (i ? b2[i - 1] / d : 0.0);
    if (fabs(d) < 1e-300) d = -1e-300;
    cnt += d < 0.0;
  }
  return cnt;
}

__global__ __launch_bounds__(kKW) void k_tridiag_max(const double* __restrict__ a, const double* __restrict__ b2,
                                                     int k, double* __restrict__ out) {
  const int lane = threadIdx.x;
  double lo = 0.0, hi = 0.0;
  {  // Gershgorin bracket
    double glo = 1e300, ghi = -1e300;
    for (int i = lane; i < k; i += kKW) {
      const double r = (i ? sqrt(b2[i - 1]) : 0.0) + (i + 1 < k ? sqrt(b2[i]) : 0.0);
      glo = fmin(glo, a[i] - r);
      ghi = fmax(ghi, a[i] + r);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      glo = fmin(glo, __shfl_xor(glo, off, kKW));
      ghi = fmax(ghi, __shfl_xor(ghi, off, kKW));
    }
    const double pad = 1e-14 * fmax(fabs(glo), fabs(ghi)) + 1e-300;
    lo = glo - pad;
    hi = ghi + pad;
  }
  for (int round = 0; round < 12; ++round) {
    const double step = (hi - lo) / (kKW + 1);
    const double x = lo + (lane + 1) * step;
    const int below = sturm_below(a, b2, k, x);
    // the largest eigenvalue lies above the points with count < k and at or
    // below the first point with count == k
    const unsigned long long full = __ballot(below >= k);
    const int first = full ? __ffsll((long long)full) - 1 : kKW;
    const double nlo = first == 0 ? lo : lo + first * step;
    const double nhi = first == kKW ? hi : lo + (first + 1) * step;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) *out = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------- CG
// State layout in device memory (doubles, then ints): see CgState.
// x += alpha p, r -= alpha q with alpha = rr / pq; then rr' = r . r, beta =
// rr' / rr, iteration count, convergence flag (||r|| <= tol ||b||).
__global__ __launch_bounds__(kKB) void k_cg_update(double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   int64_t n, CgState* st, double* partials, uint32_t* ticket) {
  __shared__ double sh[kKB / kKW];
  if (st->done) return;
  const double pq = st->pq;
  const double alpha = pq > 0.0 ? st->rr / pq : 0.0;  // breakdown leaves x and r as they are
  double v = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    v = fma(ri, ri, v);
  }
  v = block_sum(v, sh);
  double rr_new;
  if (grid_reduce_last(v, partials, ticket, &rr_new)) {
    if (!(pq > 0.0)) {  // the operator is not positive definite: stop, uncounted
      st->done = 1;
      st->breakdown = 1;
    } else {
      const double rr = st->rr;
      st->beta = rr_new / rr;
      st->rr = rr_new;
      st->iters += 1;
      if (sqrt(rr_new) <= st->tol * st->bnorm) {
        st->done = 1;
      } else if (!isfinite(rr_new)) {
        st->done = 1;
        st->breakdown = 1;
      }
    }
  }
}

// p = r + beta p
__global__ __launch_bounds__(kKB) void k_cg_direction(double* __restrict__ p, const double* __restrict__ r, int64_t n,
                                                      const CgState* st) {
  if (st->done) return;
  const double beta = st->beta;
  for (int64_t i = blockIdx.x * (int64_t)kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB)
    p[i] = fma(beta, p[i], r[i]);
}

// rr = r . r, bnorm = sqrt(rr), p = r, x = 0 (the CG start from x0 = 0)
__global__ __launch_bounds__(kKB) void k_cg_start(double* __restrict__ x, const double* __restrict__ r,
                                                  double* __restrict__ p, int64_t n, CgState* st,
                                                  double* partials, uint32_t* ticket) {
  __shared__ double sh[kKB / kKW];
  double v = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) {
    const double ri = r[i];
    p[i] = ri;
    x[i] = 0.0;
    v = fma(ri, ri, v);
  }
  v = block_sum(v, sh);
  double rr;
  if (grid_reduce_last(v, partials, ticket, &rr)) {
    st->rr = rr;
    st->bnorm = sqrt(rr);
    st->iters = 0;
    st->breakdown = 0;
    st->done = rr == 0.0 ? 1 : 0;
  }
}

// ------------------------------------------------------------ launchers
static int grid_for(int64_t n) {
  const int64_t g = (n + kKB - 1) / kKB;
  return (int)(g < kRedGrid ? (g > 0 ? g : 1) : kRedGrid);
}

hipError_t launch_transpose_positions(const int32_t* rowptr, const int32_t* colind, int n, int32_t* tpos,
                                      hipStream_t s) {
  const int64_t threads = (int64_t)n * kKW;
  hipLaunchKernelGGL(k_transpose_positions, dim3((unsigned)((threads + kKB - 1) / kKB)), dim3(kKB), 0, s, rowptr,
                     colind, n, tpos);
  return hipGetLastError();
}

hipError_t launch_gather_transpose(const int32_t* tpos, const double* vals, int64_t nnz, double* out,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_gather_transpose, dim3(grid_for(nnz) * 4), dim3(kKB), 0, s, tpos, vals, nnz, out);
  return hipGetLastError();
}

int spmv_lanes(double mean_row) {
  if (mean_row > 48) return 64;
  if (mean_row > 24) return 32;
  if (mean_row > 12) return 16;
  if (mean_row > 6) return 8;
  return 4;
}

hipError_t launch_spmv(const SpmvArgs& a, const double* x, double* y, double c, const double* sv, const int32_t* done,
                       hipStream_t s) {
  const int64_t threads = (int64_t)a.n * a.lanes;
  const dim3 grid((unsigned)((threads + kKB - 1) / kKB)), block(kKB);
  switch (a.lanes) {
    case 4: hipLaunchKernelGGL(k_spmv<4>, grid, block, 0, s, a.rowptr, a.colind, a.vals, x, y, a.n, c, sv, done); break;
    case 8: hipLaunchKernelGGL(k_spmv<8>, grid, block, 0, s, a.rowptr, a.colind, a.vals, x, y, a.n, c, sv, done); break;
    case 16: hipLaunchKernelGGL(k_spmv<16>, grid, block, 0, s, a.rowptr, a.colind, a.vals, x, y, a.n, c, sv, done); break;
    case 32: hipLaunchKernelGGL(k_spmv<32>, grid, block, 0, s, a.rowptr, a.colind, a.vals, x, y, a.n, c, sv, done); break;
    default: hipLaunchKernelGGL(k_spmv<64>, grid, block, 0, s, a.rowptr, a.colind, a.vals, x, y, a.n, c, sv, done); break;
  }
  return hipGetLastError();
}

hipError_t launch_dot(const double* a, const double* b, int64_t n, KrylovScratch& k, double* out,
                      const int32_t* done, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(grid_for(n)), dim3(kKB), 0, s, a, b, n, k.partials, k.ticket, out, done);
  return hipGetLastError();
}

hipError_t launch_scale(const double* x, double* y, int64_t n, const double* num, const double* den, int sqrt_den,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kKB), 0, s, x, y, n, num, den, sqrt_den);
  return hipGetLastError();
}

hipError_t launch_random_vector(double* v, int64_t n, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_random_vector, dim3(grid_for(n)), dim3(kKB), 0, s, v, n, seed);
  return hipGetLastError();
}

hipError_t launch_gemv_t(const double* V, int64_t n, int ncol, const double* w, double* h, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_t, dim3(ncol), dim3(kKB), 0, s, V, n, ncol, w, h);
  return hipGetLastError();
}

hipError_t launch_gemv_n_sub(const double* V, int64_t n, int ncol, const double* h, double* w, double* alpha, int j,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_n_sub, dim3(grid_for(n)), dim3(kKB), 0, s, V, n, ncol, h, w, alpha, j);
  return hipGetLastError();
}

hipError_t launch_tridiag_max(const double* a, const double* b2, int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag_max, dim3(1), dim3(kKW), 0, s, a, b2, k, out);
  return hipGetLastError();
}

hipError_t launch_cg_start(double* x, const double* r, double* p, int64_t n, CgState* st, KrylovScratch& k,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_cg_start, dim3(grid_for(n)), dim3(kKB), 0, s, x, r, p, n, st, k.partials, k.ticket);
  return hipGetLastError();
}

hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q, int64_t n, CgState* st,
                            KrylovScratch& k, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update, dim3(grid_for(n)), dim3(kKB), 0, s, x, r, p, q, n, st, k.partials, k.ticket);
  return hipGetLastError();
}

hipError_t launch_cg_direction(double* p, const double* r, int64_t n, const CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_direction, dim3(grid_for(n)), dim3(kKB), 0, s, p, r, n, st);
  return hipGetLastError();
}

int reduction_blocks() { return kRedGrid; }

}  // namespace submat

namespace submat {

// ------------------------------------------------------------ refinement
// Dense row-major n x n image of a CSR value array: column-based
// (segment j = column j, colbased = 1) or row-based. The target is zeroed
// first by the caller.
__global__ __launch_bounds__(kKB) void k_densify(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                                 const double* __restrict__ vals, int n, int colbased,
                                                 double* __restrict__ D) {
  const int seg = (int)((blockIdx.x * (int64_t)kKB + threadIdx.x) / kKW);
  const int lane = threadIdx.x & (kKW - 1);
  if (seg >= n) return;
  for (int q = rowptr[seg] + lane; q < rowptr[seg + 1]; q += kKW) {
    const int64_t r = colbased ? colind[q] : seg, c = colbased ? seg : colind[q];
    D[r * n + c] = vals[q];
  }
}

// out = ||T - I||_F^2 over a dense row-major n x n matrix (deterministic)
__global__ __launch_bounds__(kKB) void k_residual_fro2(const double* __restrict__ T, int n, double* partials,
                                                       uint32_t* ticket, double* out) {
  __shared__ double sh[kKB / kKW];
  const int64_t nn = (int64_t)n * n;
  double v = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)kKB + threadIdx.x; e < nn; e += (int64_t)gridDim.x * kKB) {
    const int64_t i = e / n, j = e - i * n;
    const double d = T[e] - (i == j ? 1.0 : 0.0);
    v = fma(d, d, v);
  }
  v = block_sum(v, sh);
  double tot;
  if (grid_reduce_last(v, partials, ticket, &tot)) *out = tot;
}

hipError_t launch_densify(const int32_t* rowptr, const int32_t* colind, const double* vals, int n, int colbased,
                          double* D, hipStream_t s) {
  const int64_t threads = (int64_t)n * kKW;
  hipLaunchKernelGGL(k_densify, dim3((unsigned)((threads + kKB - 1) / kKB)), dim3(kKB), 0, s, rowptr, colind, vals, n,
                     colbased, D);
  return hipGetLastError();
}

hipError_t launch_residual_fro2(const double* T, int n, KrylovScratch& k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_residual_fro2, dim3(kRedGrid), dim3(kKB), 0, s, T, n, k.partials, k.ticket, out);
  return hipGetLastError();
}

}  // namespace submat
