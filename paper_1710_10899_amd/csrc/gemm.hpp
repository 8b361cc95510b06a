// Workgroup-level GEMM on the MFMA 16x16x4 instructions (FP64 and FP32),
// for the dense products inside one submatrix: the blocked accumulation of
// the Householder reflectors, the rank-2k trailing update of the reduction
// and the two products of the adjoint.
//
//   C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C
//
// All matrices column-major in global memory (L2-resident slabs). The
// workgroup (NW waves) walks C in BM x BN tiles, BM = 64, BN = 16 * NW;
// wave w owns the 32 x 32 block (w % 2, w / 2) of the tile as 2 x 2 MFMA
// output tiles. Operand tiles of depth BK = 16 are staged through LDS,
// k-major, so that every lane reads its MFMA operand without bank
// conflicts.
//
// MFMA 16x16x4 lane layout (checked on the device): for lane l,
// A operand = A[l % 16][l / 16], B operand = B[l / 16][l % 16];
// accumulator register r holds D[row][l % 16] with row = 4 * (l / 16) + r
// for the FP32 instruction and row = l / 16 + 4 * r for the FP64 one.
#pragma once

#include "common.hpp"

namespace submat {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
template <> struct Mfma<double> {
  typedef mf_d4 acc_t;
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef mf_f4 acc_t;
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

constexpr int kGemmBM = 64;
constexpr int kGemmBK = 16;

// LDS elements of T needed by wg_gemm with NW waves.
template <int NW> constexpr int gemm_lds_elems() { return kGemmBK * kGemmBM + kGemmBK * 16 * NW; }

// TA: op(A) = A^T (A stored K x M); TB: op(B) = B^T (B stored N x K).
// LOWER: tiles lying entirely above the diagonal of C are skipped (for
// symmetric results kept in the lower triangle).
// Must be called by every thread of the workgroup (contains barriers).
template <class T, int NW, bool TA, bool TB, bool LOWER = false>
__device__ void wg_gemm(int M, int N, int K, T alpha, const T* __restrict__ A, int lda,
                        const T* __restrict__ B, int ldb, T beta, T* __restrict__ C, int ldc, T* smem) {
  constexpr int BM = kGemmBM, BK = kGemmBK, BN = 16 * NW, NT = NW * kWave;
  typedef typename Mfma<T>::acc_t acc_t;
  T* As = smem;            // [BK][BM]
  T* Bs = smem + BK * BM;  // [BK][BN]
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int wr = wv & 1, wc = wv >> 1;
  const int li = lane & 15, lk = lane >> 4;
  for (int i0 = 0; i0 < M; i0 += BM) {
    for (int j0 = 0; j0 < N; j0 += BN) {
      if (LOWER && j0 >= i0 + BM) continue;
      acc_t acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
      for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        // A tile: op(A)[i0 .. i0+BM) x [k0 .. k0+BK)
        for (int q = tid; q < BM * BK; q += NT) {
          int kq, iq;
          if (TA) { iq = q / BK; kq = q - iq * BK; }   // contiguous along k in storage
          else { kq = q / BM; iq = q - kq * BM; }      // contiguous along i in storage
          const int gi = i0 + iq, gk = k0 + kq;
          T v = T(0);
          if (gi < M && gk < K) v = TA ? A[(int64_t)gi * lda + gk] : A[(int64_t)gk * lda + gi];
          As[kq * BM + iq] = v;
        }
        // B tile: op(B)[k0 .. k0+BK) x [j0 .. j0+BN)
        for (int q = tid; q < BN * BK; q += NT) {
          int kq, jq;
          if (TB) { kq = q / BN; jq = q - kq * BN; }   // contiguous along j in storage
          else { jq = q / BK; kq = q - jq * BK; }      // contiguous along k in storage
          const int gj = j0 + jq, gk = k0 + kq;
          T v = T(0);
          if (gj < N && gk < K) v = TB ? B[(int64_t)gk * ldb + gj] : B[(int64_t)gj * ldb + gk];
          Bs[kq * BN + jq] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          T av[2], bv[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) av[a] = As[(kk + lk) * BM + wr * 32 + a * 16 + li];
#pragma unroll
          for (int b = 0; b < 2; ++b) bv[b] = Bs[(kk + lk) * BN + wc * 32 + b * 16 + li];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::step(av[a], bv[b], acc[a][b]);
        }
      }
      // epilogue
#pragma unroll
      for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int gj = j0 + wc * 32 + b * 16 + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gi = i0 + wr * 32 + a * 16 + Mfma<T>::row(lk, r);
            if (gi < M && gj < N) {
              T* cp = C + (int64_t)gj * ldc + gi;
              *cp = (beta == T(0)) ? alpha * acc[a][b][r] : alpha * acc[a][b][r] + beta * *cp;
            }
          }
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace submat
