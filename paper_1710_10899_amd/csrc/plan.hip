// Pattern analysis (Section 3.1 needs R_j; Section 3.3 needs R_j.indexof(j))
// and small utility kernels.
#include "common.hpp"
#include "kernels.hpp"

namespace submat {

// One thread per row j: m_j, c_j = position of j in its segment, and the
// conditions under which Algorithms 1 and 2 are defined (sorted unique
// in-range indices, symmetric pattern, stored diagonal).
__global__ void k_plan_pattern(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                               int32_t n, int64_t nnz, int32_t* __restrict__ m_out,
                               int32_t* __restrict__ c_out, uint32_t* __restrict__ err) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0 && (rowptr[0] != 0 || (int64_t)rowptr[n] != nnz)) atomicOr(err, (uint32_t)PAT_ROWPTR);
  if (j >= n) return;
  const int64_t a = rowptr[j], b = rowptr[j + 1];
  m_out[j] = 0;
  c_out[j] = -1;
  if (a < 0 || b < a || b > nnz) {
    atomicOr(err, (uint32_t)PAT_ROWPTR);
    return;
  }
  uint32_t bits = 0;
  int prev = -1;
  int c = -1;
  for (int64_t q = a; q < b; ++q) {
    const int i = colind[q];
    if (i < 0 || i >= n) { bits |= PAT_RANGE; break; }
    if (i <= prev) { bits |= PAT_ORDER; break; }
    prev = i;
    if (i == (int)j) c = (int)(q - a);
    // symmetric pattern: j must be stored in row i
    const int64_t ia = rowptr[i], ib = rowptr[i + 1];
    if (ia < 0 || ib < ia || ib > nnz) { bits |= PAT_ROWPTR; break; }
    int64_t lo = ia, hi = ib - 1;
    bool found = false;
    while (lo <= hi) {
      const int64_t mid = (lo + hi) >> 1;
      const int v = colind[mid];
      if (v == (int)j) { found = true; break; }
      if (v < (int)j) lo = mid + 1; else hi = mid - 1;
    }
    if (!found) bits |= PAT_ASYM;
  }
  if (c < 0 && !(bits & (PAT_RANGE | PAT_ORDER))) bits |= PAT_NODIAG;
  if (bits) atomicOr(err, bits);
  m_out[j] = (int32_t)(b - a);
  c_out[j] = c;
}

hipError_t launch_plan_pattern(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz,
                               int32_t* m_out, int32_t* c_out, uint32_t* err, hipStream_t s) {
  const int bs = 256;
  const int grid = (int)((n + bs - 1) / bs);
  hipLaunchKernelGGL(k_plan_pattern, dim3(grid), dim3(bs), 0, s, rowptr, colind, n, nnz, m_out, c_out, err);
  return hipGetLastError();
}

// Plain fill kernel (kept out of memset nodes so that captured graphs replay
// it reliably).
__global__ void k_fill_zero(uint64_t* __restrict__ p, int64_t nwords, uint8_t* __restrict__ tail, int ntail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) p[i] = 0;
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void* ptr, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  const int64_t nwords = bytes / 8;
  const int ntail = (int)(bytes - nwords * 8);
  int64_t g = (nwords + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(256), 0, s, (uint64_t*)ptr, nwords,
                     (uint8_t*)ptr + nwords * 8, ntail);
  return hipGetLastError();
}

__global__ void k_reset_status(int64_t* __restrict__ status, int32_t* __restrict__ counters, int ncounters) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ST_NSLOTS) status[i] = 0;
  for (int k = i; k < ncounters; k += gridDim.x * blockDim.x) counters[k] = 0;
}

hipError_t launch_reset_status(int64_t* status, int32_t* counters, int ncounters, hipStream_t s) {
  int g = (ncounters + 255) / 256;
  if (g < 1) g = 1;
  if (g > 64) g = 64;
  hipLaunchKernelGGL(k_reset_status, dim3(g), dim3(256), 0, s, status, counters, ncounters);
  return hipGetLastError();
}

}  // namespace submat
