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

// The spectral functions (inverse p-th root of Sections 3-4; p-th root and
// real power of the subsection on other matrix operations), evaluated in
// FP64 whatever the storage type.
__device__ __forceinline__ double spec_f(double lam, const SpecFn& f) {
  if (f.kind == FN_ROOT) return root_p(lam, f.p);
  if (f.kind == FN_POWER) return pow(lam, f.alpha);
  return inv_root_p(lam, f.p);
}

// Per-eigenvalue node from which the divided differences work:
// alpha = lambda^(1/p) for the two root functions, lambda itself for a real
// power.
__device__ __forceinline__ double spec_node(double lam, const SpecFn& f) {
  return f.kind == FN_POWER ? lam : root_p(lam, f.p);
}

// Divided difference G = (f(lambda_k) - f(lambda_l)) / (lambda_k - lambda_l),
// f'(lambda) when equal, from the nodes of spec_node, in forms without
// cancellation:
//   inverse root: -1 / (a_k a_l h),  h = sum_{i<p} a_k^i a_l^(p-1-i)
//   root:          1 / h            (a_k - a_l = (a_k^p - a_l^p) / h)
//   power:         lambda_l^alpha expm1(alpha t) / (lambda_k - lambda_l),
//                  t = log(lambda_k / lambda_l), since
//                  lambda_k^alpha = lambda_l^alpha exp(alpha t); t is taken
//                  as log1p(d), d = (lambda_k - lambda_l) / lambda_l, for
//                  |d| < 1/2 (exact difference, full relative accuracy of a
//                  small t) and as the log of the ratio otherwise (where
//                  log1p of a d near -1 would lose digits).
// The power form is a separate instantiation (POW) in the kernels, so that
// its transcendental calls do not raise the register count of the others.
__device__ __forceinline__ double root_divdiff(double xk, double xl, const SpecFn& f) {
  double h = 1.0, alp = 1.0;
  for (int q = 1; q < f.p; ++q) {
    alp *= xl;
    h = xk * h + alp;
  }
  return f.kind == FN_ROOT ? 1.0 / h : -1.0 / (xk * xl * h);
}
// pwl = lambda_l^alpha, formed once per eigenvalue by the caller.
__device__ __forceinline__ double power_divdiff(double xk, double xl, double pwl, double alpha) {
  const double diff = xk - xl;
  if (diff == 0.0) return alpha * pwl / xl;
  const double d = diff / xl;
  const double t = fabs(d) < 0.5 ? log1p(d) : log(xk / xl);
  return pwl * expm1(alpha * t) / diff;
}
template <bool POW>
__device__ __forceinline__ double spec_divdiff(double xk, double xl, double pwl, const SpecFn& f) {
  return POW ? power_divdiff(xk, xl, pwl, f.alpha) : root_divdiff(xk, xl, f);
}

// Lane exchange by DPP (the VALU reads its operand from another lane of the
// same row of 16 lanes, without an LDS round trip). gfx9 DPP control codes:
// quad_perm [l0, l1, l2, l3] = l0 | l1 << 2 | l2 << 4 | l3 << 6;
// row_half_mirror (lane i <-> 7 - i within each group of 8) = 0x141.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of G consecutive lanes (G = 1, 2, 4 or 8). Each
// step adds the partner lane's value; IEEE addition is commutative, so every
// lane of a group ends with the same bits.
// g must be the same in every lane of the wave (the branches are uniform).
__device__ __forceinline__ double group_sum(double v, int g) {
  if (g >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]: lane ^ 1
  if (g >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]: lane ^ 2
  if (g >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror: the other quad of the 8
  return v;
}

// Value of lane l (a compile-time-uniform lane index), broadcast to every lane.
__device__ __forceinline__ double read_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Wave-wide reductions: within each row of 16 lanes by DPP exchanges (lane ^ 1,
// lane ^ 2, the other quad of 8, the other 8 of 16: every lane of a row ends
// with the same bits, the operation being commutative), then the four rows'
// values from lanes 0, 16, 32, 48 combined in that order in every lane.
template <class Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = op(v, dpp_f64<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = op(v, dpp_f64<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = op(v, dpp_f64<0x141>(v));  // row_half_mirror
  v = op(v, dpp_f64<0x140>(v));  // row_mirror
  return op(op(op(read_lane(v, 0), read_lane(v, 16)), read_lane(v, 32)), read_lane(v, 48));
}
__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double x, double y) { return x + y; });
}
__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce(v, [](double x, double y) { return fmin(x, y); });
}
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, [](double x, double y) { return fmax(x, y); });
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

// Work queues grouped by XCD for launches over (item, block) units, item-
// major (u = it * ncb + cb): queue q holds the items it = q, q + 8, ... A
// workgroup takes units from the queue of the XCD it runs on (the XCC_ID
// hardware register), then from the others in turn, so every unit is taken
// exactly once whatever the placement, and the units of one item, taken at
// about the same time by workgroups of one XCD, share that XCD's L2.
// ctrs: kXcdQueues counters, zero at launch. Returns u, or -1 once every
// queue is drained. `q` (thread 0's) carries the current queue between calls.
constexpr int kXcdQueues = 8;
__device__ __forceinline__ int xcc_id() {
  // s_getreg_b32 of HW_REG_XCC_ID (id 20), bits 3:0
  return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & (kXcdQueues - 1);
}
__device__ __forceinline__ int next_unit_xcd(int* ctrs, int n_items, int ncb, int* s_slot, int& q) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int res = -1;
    for (int t = 0; t < kXcdQueues; ++t) {
      const int qq = (q + t) & (kXcdQueues - 1);
      const int nq = (n_items - qq + kXcdQueues - 1) / kXcdQueues;  // items of queue qq
      const int l = atomicAdd(&ctrs[qq], 1);
      if (l < nq * ncb) {
        res = (qq + kXcdQueues * (l / ncb)) * ncb + (l % ncb);
        q = qq;
        break;
      }
    }
    *s_slot = res;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*s_slot);
}

template <class T>
__device__ __forceinline__ void atomic_add_val(T* p, T v) {
  atomicAdd(p, v);
}

}  // namespace submat
