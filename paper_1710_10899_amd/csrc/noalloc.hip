// Forward of the one-wavefront path without any device allocation, for
// callers that cannot allocate (HIP graph capture, tight serving loops).
//
// Every column j (Sections 3.1-3.4) runs through the same kernels as the
// planned path: the pattern kernel writes m_j, c_j = R_j.indexof(j) and the
// validation bits, and the one-wavefront Jacobi kernel takes the columns in
// index order (no bucketing, no LPT order: that needs the orders on the
// host). Device memory beyond the caller's inputs and outputs lives in one
// file-scope array, `scratch`; its device address is looked up once per
// device with hipGetSymbolAddress and only that address is handed to
// kernels. Layout (bytes):
//   [0, 512)        status slots (ST_NSLOTS int64)
//   [512, 516)      pattern validation bits of the call
//   [516, 520)      work counter of the Jacobi launch
//   [1024, +4 N)    m_j,  N = kNoAllocMaxN
//   [.., +4 N)      c_j
// Calls on one device share the array: calls that overlap in time on one
// device race, and every call clears what must start at zero (status, the
// error word, the counter) with a fill kernel (no memset node).
#include <map>
#include <mutex>

#include "../../include/submat.h"
#include "common.hpp"
#include "kernels.hpp"

namespace submat {

constexpr size_t kNoAllocHeader = 1024;
constexpr size_t kNoAllocScratchBytes = kNoAllocHeader + 8 * (size_t)kNoAllocMaxN;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;   // device -> address of that device's `scratch`

// Address of `scratch` on the current device (looked up on first use there).
int scratch_address(unsigned char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SUBMAT_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return SUBMAT_EHIP;
    }
    it = g_scratch_ptr.emplace(dev, (unsigned char*)ptr).first;
  }
  *out = it->second;
  return SUBMAT_OK;
}
}  // namespace

__global__ void k_noalloc_clear(int64_t* status, uint32_t* err, int32_t* ctr) {
  const int i = threadIdx.x;
  if (i < ST_NSLOTS) status[i] = 0;
  if (i == 0) {
    *err = 0u;
    *ctr = 0;
  }
}

int noalloc_forward(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n, int64_t nnz,
                    SpecFn fn, int32_t vdtype, int mixed, double kappa_max, void* x, int num_cus, hipStream_t s,
                    int64_t** status_out) {
  if (n < 1 || n > kNoAllocMaxN) return SUBMAT_ETOOBIG;
  unsigned char* base = nullptr;
  if (scratch_address(&base)) return SUBMAT_EHIP;
  int64_t* status = (int64_t*)base;
  uint32_t* err = (uint32_t*)(base + 512);
  int32_t* ctr = (int32_t*)(base + 516);
  int32_t* m = (int32_t*)(base + kNoAllocHeader);
  int32_t* c = m + kNoAllocMaxN;
  hipLaunchKernelGGL(k_noalloc_clear, dim3(1), dim3(ST_NSLOTS), 0, s, status, err, ctr);
  if (hipGetLastError() != hipSuccess) return SUBMAT_EHIP;
  if (launch_plan_pattern(rowptr, colind, n, nnz, m, c, err, s) != hipSuccess) return SUBMAT_EHIP;
  SmallArgs sa{};
  sa.rowptr = rowptr;
  sa.colind = colind;
  sa.vals = vals;
  sa.vdtype = vdtype;
  sa.items = nullptr;   // column it is item it
  sa.cidx = c;
  sa.n_items = n;
  sa.mmax = 64;         // any order up to 64; larger ones are NaN and counted
  sa.fn = fn;
  sa.mixed = mixed;
  sa.kappa_max = kappa_max;
  sa.x = x;
  sa.status = status;
  sa.work_ctr = ctr;
  int g = num_cus * 8;
  sa.grid = g > n ? n : g;
  sa.pattern_err = err;
  if (launch_small(sa, s) != hipSuccess) return SUBMAT_EHIP;
  *status_out = status;
  return SUBMAT_OK;
}

}  // namespace submat
