// Device helpers shared by the submatrix-method kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace submat {

constexpr int kWave = 64;

template <class T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 1.1102230246251565e-16; };
template <> struct Eps<float> { static constexpr double v = 5.9604644775390625e-08; };

// f(lambda) = lambda^(-1/p): one root (correctly rounded sqrt for p = 2)
// followed by one division.
__device__ __forceinline__ double inv_root_p(double lam, int p) {
  if (p == 1) return 1.0 / lam;
  if (p == 2) return 1.0 / sqrt(lam);
  if (p == 3) return 1.0 / cbrt(lam);
  return 1.0 / pow(lam, 1.0 / (double)p);
}

// lambda^(1/p)
__device__ __forceinline__ double root_p(double lam, int p) {
  if (p == 1) return lam;
  if (p == 2) return sqrt(lam);
  if (p == 3) return cbrt(lam);
  return pow(lam, 1.0 / (double)p);
}

// Divided difference of f(x) = x^(-1/p) at lambda_k, lambda_l written in
// alpha = lambda^(1/p): -1 / (a_k a_l sum_{i<p} a_k^i a_l^(p-1-i)).
// Free of cancellation, and equal to f'(lambda) when a_k == a_l.
__device__ __forceinline__ double divdiff(double ak, double al, int p) {
  double h = 1.0, alp = 1.0;
  for (int q = 1; q < p; ++q) {
    alp *= al;
    h = ak * h + alp;
  }
  return -1.0 / (ak * al * h);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Block-wide sum over NW waves; `red` is LDS scratch of >= NW doubles.
// All threads get the result.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

// Position of `key` in the sorted int array r[0..m) or -1 (binary search).
__device__ __forceinline__ int find_sorted(const int* r, int m, int key) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (r[mid] < key) lo = mid + 1; else hi = mid;
  }
  return (m > 0 && r[lo] == key) ? lo : -1;
}

// Persistent-kernel work distribution: next item index for the block. The
// value is the same in every lane; readfirstlane lets the compiler keep it,
// and everything derived from it (sizes, offsets, slab pointers), in scalar
// registers.
__device__ __forceinline__ int next_item(int* ctr, int* s_slot) {
  __syncthreads();
  if (threadIdx.x == 0) *s_slot = atomicAdd(ctr, 1);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*s_slot);
}

template <class T>
__device__ __forceinline__ void atomic_add_val(T* p, T v) {
  atomicAdd(p, v);
}

}  // namespace submat
