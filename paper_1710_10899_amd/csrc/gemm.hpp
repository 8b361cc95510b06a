// Workgroup-level GEMM on the MFMA 16x16x4 instructions (FP64 and FP32),
// for the dense products inside one submatrix: the blocked accumulation of
// the Householder reflectors, the rank-2k trailing update of the reduction
// and the two products of the adjoint.
//
//   C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C
//
// All matrices column-major in global memory. The workgroup (NW waves)
// walks C in BM x BN tiles, BM = 32 * TM, BN = 8 * NW * TN; wave w owns the
// (16 TM) x (16 TN) block (w % 2, w / 2) of the tile as TM x TN MFMA output
// tiles (2 x 2 by default; larger blocks read each operand fewer times). Operand tiles of depth BK = 16 are staged through LDS,
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

// LDS layout of a staged operand tile follows its order in global memory,
// so that both the store (consecutive threads, consecutive addresses) and
// the MFMA operand read are free of bank conflicts:
//  * contiguous along i (or j): k-major rows [BK][W + 16]; the stride is 16
//    doubles off a multiple of the bank width, so the four k-rows one MFMA
//    read touches fall in different bank halves;
//  * contiguous along k: k-minor rows [W][BK + 1]; the odd stride spreads the
//    16 rows of one MFMA read over distinct banks.
constexpr int kGemmPad = 16;
template <int W> constexpr int tile_elems_major() { return kGemmBK * (W + kGemmPad); }
template <int W> constexpr int tile_elems_minor() { return W * (kGemmBK + 1); }
template <int W> constexpr int tile_elems() {
  return tile_elems_major<W>() > tile_elems_minor<W>() ? tile_elems_major<W>() : tile_elems_minor<W>();
}
// LDS elements of T needed by wg_gemm with NW waves and TM x TN tiles per wave.
template <int NW, int TM = 2, int TN = 2> constexpr int gemm_lds_elems() {
  return tile_elems<32 * TM>() + tile_elems<8 * NW * TN>();
}

// TA: op(A) = A^T (A stored K x M); TB: op(B) = B^T (B stored N x K).
// LOWER: tiles lying entirely above the diagonal of C are skipped (for
// symmetric results kept in the lower triangle).
// Must be called by every thread of the workgroup (contains barriers).
// PF: k-tiles fetched ahead into registers while the current one is
// multiplied (0, 1 or 2; each costs 6-8 registers). Two tiles in flight
// cover the HBM latency, which exceeds the MFMA time of one 16-deep k-tile.
// ZA, ZB: triangles of the operands that hold zeros in memory (the caller
// guarantees it), whose products are skipped; the result is unchanged:
//   ZA = 1: op(A)[i][k] = 0 for k < i;  ZA = 2: op(A)[i][k] = 0 for k > i;
//   ZB = 1: op(B)[k][j] = 0 for k < j.
// A tile's k-range is cut to the k that can meet a nonzero, and a wave's
// 16 x 16 block skips the 4-deep k-slices that meet only zeros.
template <class T, int NW, bool TA, bool TB, bool LOWER = false, int PF = 1, int TM = 2, int TN = 2, int ZA = 0,
          int ZB = 0>
__device__ void wg_gemm(int M, int N, int K, T alpha, const T* __restrict__ A, int lda,
                        const T* __restrict__ B, int ldb, T beta, T* __restrict__ C, int ldc, T* smem) {
  static_assert(PF >= 0 && PF <= 2, "prefetch depth 0..2");
  static_assert(ZA >= 0 && ZA <= 2 && ZB >= 0 && ZB <= 1, "zero-triangle modes");
  constexpr int BM = 32 * TM, BK = kGemmBK, BN = 8 * NW * TN, NT = NW * kWave;
  constexpr int WM = 16 * TM, WN = 16 * TN;  // one wave's block of C
  constexpr int AL = BM * BK / NT, BL = BN * BK / NT;  // tile elements per thread
  constexpr int NS = PF > 1 ? PF : 1;                  // register slots
  typedef typename Mfma<T>::acc_t acc_t;
  // A tile: k-major unless A is transposed (then contiguous along k);
  // B tile: k-major if B is transposed (contiguous along j), else k-minor.
  constexpr int SA = TA ? BK + 1 : BM + kGemmPad;
  constexpr int SB = TB ? BN + kGemmPad : BK + 1;
  T* As = smem;
  T* Bs = smem + tile_elems<BM>();
  auto a_at = [&](int kq, int iq) -> T& { return TA ? As[iq * SA + kq] : As[kq * SA + iq]; };
  auto b_at = [&](int kq, int jq) -> T& { return TB ? Bs[kq * SB + jq] : Bs[jq * SB + kq]; };
  // an opaque copy of the thread index keeps the compiler from hoisting this
  // product's index arithmetic out of the caller's loops (where the
  // hoisted values of several products would stay live at once)
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int wr = wv & 1, wc = wv >> 1;
  const int li = lane & 15, lk = lane >> 4;
  // element q of a tile -> (k, i) position; storage order follows the
  // contiguous direction of the operand in memory
  auto a_pos = [&](int q, int& kq, int& iq) {
    if (TA) { iq = q / BK; kq = q - iq * BK; } else { kq = q / BM; iq = q - kq * BM; }
  };
  auto b_pos = [&](int q, int& kq, int& jq) {
    if (TB) { kq = q / BN; jq = q - kq * BN; } else { jq = q / BK; kq = q - jq * BK; }
  };
  for (int i0 = 0; i0 < M; i0 += BM) {
    for (int j0 = 0; j0 < N; j0 += BN) {
      if (LOWER && j0 >= i0 + BM) continue;
      // 16 x 16 output blocks of this wave that hold no element of C (past
      // M or N, or above the diagonal for LOWER) take no MFMA: the tests
      // are uniform over the wave
      bool live[TM][TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int r0 = i0 + wr * WM + a * 16, c0 = j0 + wc * WN + b * 16;
          live[a][b] = r0 < M && c0 < N && (!LOWER || c0 <= r0 + 15);
        }
      }
      acc_t acc[TM][TN];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
      // k-range [kb, ke) of this tile: outside it every product meets a zero
      // of the operands' triangles (kb stays a multiple of BK)
      int kb = 0, ke = K;
      if (ZA == 1) kb = i0;
      if (ZB == 1 && j0 > kb) kb = j0;
      kb = kb / BK * BK;
      if (ZA == 2 && i0 + BM < ke) ke = i0 + BM;
      T ra[NS][AL], rb[NS][BL];
      auto fetch = [&](int slot, int k0) {
#pragma unroll
        for (int e = 0; e < AL; ++e) {
          int kq, iq;
          a_pos(tid + e * NT, kq, iq);
          const int gi = i0 + iq, gk = k0 + kq;
          ra[slot][e] = (gi < M && gk < K) ? (TA ? A[(int64_t)gi * lda + gk] : A[(int64_t)gk * lda + gi]) : T(0);
        }
#pragma unroll
        for (int e = 0; e < BL; ++e) {
          int kq, jq;
          b_pos(tid + e * NT, kq, jq);
          const int gj = j0 + jq, gk = k0 + kq;
          rb[slot][e] = (gj < N && gk < K) ? (TB ? B[(int64_t)gk * ldb + gj] : B[(int64_t)gj * ldb + gk]) : T(0);
        }
      };
      // one k-tile: registers of `slot` into LDS, then (after refilling the
      // slot with tile k0 + PF*BK) its MFMAs
      auto step = [&](int slot, int k0) {
        if (PF == 0) fetch(0, k0);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < AL; ++e) {
          int kq, iq;
          a_pos(tid + e * NT, kq, iq);
          a_at(kq, iq) = ra[slot][e];
        }
#pragma unroll
        for (int e = 0; e < BL; ++e) {
          int kq, jq;
          b_pos(tid + e * NT, kq, jq);
          b_at(kq, jq) = rb[slot][e];
        }
        __syncthreads();
        if (PF > 0 && k0 + PF * BK < ke) fetch(slot, k0 + PF * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          T av[TM], bv[TN];
#pragma unroll
          for (int a = 0; a < TM; ++a) av[a] = a_at(kk + lk, wr * WM + a * 16 + li);
#pragma unroll
          for (int b = 0; b < TN; ++b) bv[b] = b_at(kk + lk, wc * WN + b * 16 + li);
          const int ks = k0 + kk;  // this slice: k in [ks, ks + 4)
#pragma unroll
          for (int a = 0; a < TM; ++a) {
#pragma unroll
            for (int b = 0; b < TN; ++b) {
              // wave-uniform: the slice meets only zeros of A's or B's triangle
              const int r0 = i0 + wr * WM + a * 16, c0 = j0 + wc * WN + b * 16;
              const bool zero = (ZA == 1 && ks + 4 <= r0) || (ZA == 2 && ks > r0 + 15) || (ZB == 1 && ks + 4 <= c0);
              if (live[a][b] && !zero) acc[a][b] = Mfma<T>::step(av[a], bv[b], acc[a][b]);
            }
          }
        }
      };
      if (PF >= 1 && kb < ke) fetch(0, kb);
      if (PF >= 2 && kb + BK < ke) fetch(NS - 1, kb + BK);
      if (PF >= 2) {
        for (int k0 = kb; k0 < ke; k0 += 2 * BK) {
          step(0, k0);
          if (k0 + BK < ke) step(NS - 1, k0 + BK);
        }
      } else {
        for (int k0 = kb; k0 < ke; k0 += BK) step(0, k0);
      }
      // epilogue
#pragma unroll
      for (int a = 0; a < TM; ++a) {
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int gj = j0 + wc * WN + b * 16 + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gi = i0 + wr * WM + a * 16 + Mfma<T>::row(lk, r);
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

// Symmetric rank-2K update of the lower tiles of C (column-major, ldc):
//   C += alpha (V W^T + W V^T),  V, W: M x K column-major (ldv, ldw),
// as one product with inner dimension 2K (k-tiles of [V | W] against
// [W | V]), so that C is read and written once. Tiles entirely above the
// diagonal are skipped. Must be called by every thread of the workgroup.
template <class T, int NW>
__device__ void wg_syr2k_lower(int M, int K, T alpha, const T* __restrict__ V, int ldv, const T* __restrict__ W,
                               int ldw, T* __restrict__ C, int ldc, T* smem) {
  constexpr int BM = kGemmBM, BK = kGemmBK, BN = 16 * NW, NT = NW * kWave;
  constexpr int AL = BM * BK / NT, BL = BN * BK / NT;
  typedef typename Mfma<T>::acc_t acc_t;
  // both operand tiles are contiguous along i / j: k-major LDS layout
  constexpr int SA = BM + kGemmPad, SB = BN + kGemmPad;
  T* As = smem;
  T* Bs = smem + tile_elems<BM>();
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));  // see wg_gemm
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int wr = wv & 1, wc = wv >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int nk1 = (K + BK - 1) / BK;  // k-tiles per half
  for (int i0 = 0; i0 < M; i0 += BM) {
    for (int j0 = 0; j0 < M; j0 += BN) {
      if (j0 >= i0 + BM) continue;
      bool live[2][2];  // this wave's 16 x 16 blocks that meet the lower triangle of C
#pragma unroll
      for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int r0 = i0 + wr * 32 + a * 16, c0 = j0 + wc * 32 + b * 16;
          live[a][b] = r0 < M && c0 < M && c0 <= r0 + 15;
        }
      }
      acc_t acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
      // the next k-tile is fetched into registers while the current one is
      // multiplied; first half: V against W, second half: W against V
      T ra[AL], rb[BL];
      auto fetch = [&](int kt) {
        const bool second = kt >= nk1;
        const int k0 = (second ? kt - nk1 : kt) * BK;
        const T* Asrc = second ? W : V;
        const T* Bsrc = second ? V : W;
        const int lda = second ? ldw : ldv, ldb = second ? ldv : ldw;
#pragma unroll
        for (int e = 0; e < AL; ++e) {
          const int q = tid + e * NT, kq = q / BM, iq = q - kq * BM;
          const int gi = i0 + iq, gk = k0 + kq;
          ra[e] = (gi < M && gk < K) ? Asrc[(int64_t)gk * lda + gi] : T(0);
        }
#pragma unroll
        for (int e = 0; e < BL; ++e) {
          const int q = tid + e * NT, kq = q / BN, jq = q - kq * BN;
          const int gj = j0 + jq, gk = k0 + kq;
          rb[e] = (gj < M && gk < K) ? Bsrc[(int64_t)gk * ldb + gj] : T(0);
        }
      };
      fetch(0);
      for (int kt = 0; kt < 2 * nk1; ++kt) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < AL; ++e) {
          const int q = tid + e * NT, kq = q / BM, iq = q - kq * BM;
          As[kq * SA + iq] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < BL; ++e) {
          const int q = tid + e * NT, kq = q / BN, jq = q - kq * BN;
          Bs[kq * SB + jq] = rb[e];
        }
        __syncthreads();
        if (kt + 1 < 2 * nk1) fetch(kt + 1);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          T av[2], bv[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) av[a] = As[(kk + lk) * SA + wr * 32 + a * 16 + li];
#pragma unroll
          for (int b = 0; b < 2; ++b) bv[b] = Bs[(kk + lk) * SB + wc * 32 + b * 16 + li];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              if (live[a][b]) acc[a][b] = Mfma<T>::step(av[a], bv[b], acc[a][b]);
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int gj = j0 + wc * 32 + b * 16 + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gi = i0 + wr * 32 + a * 16 + Mfma<T>::row(lk, r);
            if (gi < M && gj < M) {
              T* cp = C + (int64_t)gj * ldc + gi;
              *cp = alpha * acc[a][b][r] + *cp;
            }
          }
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace submat
