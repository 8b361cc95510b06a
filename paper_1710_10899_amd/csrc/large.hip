// Large-order path (m > 64): one workgroup per submatrix.
//
//   gather      S_j from CSR into an HBM slab (Section 3.1), symmetrised
//   tridiag     blocked Householder reduction S = Q1 T Q1^T (lower form): per
//               panel of NB columns a lower-triangle symv per column, and one
//               rank-2*NB trailing update on MFMA
//   eig         T = Z diag(lambda) Z^T in FP64: Sturm-count bisection
//               with Newton steps for the eigenvalues, twisted factorisation / inverse iteration for
//               the eigenvectors, local reorthogonalisation (Z into the Q
//               slab)
//   back        Q = Q1 Z: the reflectors applied to Z in compact-WY blocks
//               of 128 (two 64-column factors merged), products on MFMA
//   column      x = Q (f(lambda) o Q[c,:]^T) into X's value segment
//               (Sections 3.3-3.4)
//   adjoint     D = Q sym(G o (a b^T)) Q^T on MFMA, scattered into dA's
//               stored pairs
//
// Slabs are column-major with leading dimension ldm (the order rounded up
// to a multiple of 16). After the reduction column k of the S slab holds the
// full Householder vector v_k (zeros above row k+1, 1 at row k+1).
#include <math.h>

#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "gemm.hpp"
#include "kernels.hpp"

namespace submat {

constexpr int kBlock = 256;
constexpr int kNW = kBlock / kWave;
// The back-transformation runs 4-wave workgroups, two per compute unit:
// one item's serial WY-factor steps overlap the other's products.
constexpr int kBackBlock = 256;
constexpr int kBackNW = kBackBlock / kWave;
constexpr int kBackPerCU = 2;
// The adjoint likewise (its products prefetch one k-tile ahead, which keeps
// it within the registers of two waves per SIMD).
constexpr int kAdjBlock = 256;
constexpr int kAdjNW = kAdjBlock / kWave;
constexpr int kAdjPerCU = 2;
// Panel width of the reduction: a launch parameter (LargeArgs::nb, even,
// 8..kNBMax; the tuning table's default 16 was measured best of 8..48 at
// orders ~400 with two workgroups per compute unit).
constexpr int kNBMax = 48;

template <class T> __device__ __forceinline__ T* at(void* base, int64_t off_bytes) {
  return (T*)((char*)base + off_bytes);
}
template <class T> __device__ __forceinline__ const T* at(const void* base, int64_t off_bytes) {
  return (const T*)((const char*)base + off_bytes);
}

// A column whose order no longer fits the slot and LDS sizes its plan was
// built for (the caller changed a pattern under a cached plan) is not
// computed: every kernel skips it, and the output kernels write NaN over its
// segment and count it.
__device__ __forceinline__ bool order_mismatch(const LargeArgs& a, int m, int ld) { return m > ld || m > a.max_m; }

__device__ __forceinline__ bool skip_item(const LargeArgs& a, int it) {
  const int fl = a.flags[it];
  if (a.only_flagged) return !(fl & LF_FALLBACK);
  return !a.fp64 && (fl & LF_FALLBACK);  // the FP32 pass leaves flagged items to FP64
}

// ---------------------------------------------------------------- gather
template <class T, class VT>
__global__ __launch_bounds__(kBlock) void k_gather_large(LargeArgs a) {
  // LDS: R (max_m ints), then one column buffer of max_m doubles per wave
  extern __shared__ double gdyn[];
  __shared__ int s_item;
  int* R = (int*)gdyn;
  const VT* vals = (const VT*)a.vals;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  double* col = gdyn + (a.max_m + 1) / 2 + (size_t)wv * a.max_m;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) continue;
    T* S = at<T>(a.S, a.off[it]);
    for (int i = tid; i < m; i += kBlock) R[i] = a.colind[a0 + i];
    __syncthreads();
    // Column k of (S + S^T)/2 is built in LDS from row R[k] of A (the
    // partner A[R[l]][R[k]] of each stored A[R[k]][R[l]] is at its
    // transpose position) and stored with contiguous writes; the padding
    // rows and columns of the ld x ld slot are zero.
    for (int k = wv; k < ld; k += kNW) {
      T* dst = S + (int64_t)k * ld;
      if (k >= m) {
        for (int l = lane; l < ld; l += kWave) dst[l] = T(0);
        continue;
      }
      for (int l = lane; l < m; l += kWave) col[l] = 0.0;
      __builtin_amdgcn_wave_barrier();
      const int r = R[k];
      const int s0 = a.rowptr[r], s1 = a.rowptr[r + 1];
      for (int q = s0 + lane; q < s1; q += kWave) {
        const int l = find_sorted(R, m, a.colind[q]);
        if (l >= 0) col[l] = 0.5 * ((double)vals[q] + (double)vals[a.tpos[q]]);
      }
      __builtin_amdgcn_wave_barrier();
      for (int l = lane; l < ld; l += kWave) dst[l] = l < m ? (T)col[l] : T(0);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- symmetric matvec
// The reduction runs with 4-wave workgroups, two per compute unit (two waves
// per SIMD): while one item waits on a column's serial steps (norm,
// reflector, barriers), the other streams its trailing matrix.
constexpr int kRedNW = 4;
// workgroups per compute unit the LDS budget is shared by: a template
// parameter of the kernel (1 or 2, LargeArgs::red_per_cu at launch)
constexpr int kRedBlock = kRedNW * kWave;
// y = A v for a symmetric n x n matrix given by its lower triangle (column
// major, leading dimension ld), v and y in LDS, called by the whole
// workgroup. The columns are cut into strips of kStrip; wave w
// takes strips w, 2*NW-1-w, 2*NW+w, ... (balanced over the triangle). For a
// strip the lanes run down the rows r >= c0 in groups of 64; each lane loads
// kStrip elements of its row (one coalesced column segment per load) and
//   * adds sum_c A[r][c] v[c] to its wave's row partial spart[w][r];
//   * accumulates A[r][c] v[r] (r > c) for each of the strip's columns,
//     reduced across the wave at the end of the strip.
// After a barrier, y = sum over waves of the partials, in a fixed order
// (deterministic), is formed by the caller.
constexpr int kStrip = 8;
// row groups of 64 per strip iteration of the symv, by element type (two for
// both: four groups of 4-byte elements raised the FP32 reduction's register
// use past what three workgroups per compute unit allow, and were slower,
// 141.9 against 137.0 ms on the 6656-column workload; three groups of 8-byte
// elements fit two FP64 workgroups per compute unit without spills but took
// 156.0 against 150.5 ms)
template <class T> constexpr int kSymvGroups = 2;
template <> constexpr int kSymvGroups<float> = 2;

// Column-dot reduction of a strip: 64 lanes each hold kStrip partials. Lane
// l keeps the strip's columns in slots permuted by u -> u ^ p(l), with
// p(l) = sum over halving steps h of h * bit(l, h * 64 / kStrip). Then each
// halving step is the same for every lane, x[q] += x'[q + h] from the lane
// across that bit, and after the steps slot 0 of lane l holds a partial of
// column p(l) over the lanes that differ in the remaining low bits.
__device__ __forceinline__ int strip_perm(int lane) {
  int p = 0;
#pragma unroll
  for (int h = kStrip / 2; h >= 1; h >>= 1) p += (lane & (h * (kWave / kStrip))) ? h : 0;
  return p;
}
__device__ __forceinline__ double wave_strip_sum(double (&x)[kStrip]) {
#pragma unroll
  for (int h = kStrip / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int q = 0; q < h; ++q) x[q] += __shfl_xor(x[q + h], h * (kWave / kStrip));
  }
  double t = x[0];
#pragma unroll
  for (int bit = kWave / kStrip / 2; bit >= 1; bit >>= 1) t += __shfl_xor(t, bit);
  return t;
}

// Column dots of strip [c0, c0 + kStrip) of a panel P (n rows, ncol
// columns, leading dimension ld): z[c] = P[:, c]^T v, with the lane
// partials and the reduction of the symv's strips.
// Rows [0, nl) of the panel are read from its LDS copy L (row-major, stride
// pld = nb + 1, the panel's column c at L[row * pld + c]), the rest from
// global memory. The odd stride spreads the lanes of a column read over the
// LDS banks.
template <class T>
__device__ __forceinline__ void panel_strip_dots(const T* __restrict__ P, int ld, int n, int ncol, int c0,
                                                 const double* __restrict__ v, double* z, int lane, int pl,
                                                 const double* __restrict__ L, int nl, int pld) {
  double cd[kStrip];
  int col[kStrip];
#pragma unroll
  for (int u = 0; u < kStrip; ++u) {
    const int c = c0 + (u ^ pl);
    cd[u] = 0.0;
    col[u] = (c < ncol ? c : c0) * ld;
  }
  for (int r = lane; r < nl; r += kWave) {
    const double vr = v[r];
#pragma unroll
    for (int u = 0; u < kStrip; ++u) {
      const int c = c0 + (u ^ pl);
      cd[u] = fma(c < ncol ? L[r * pld + (c < ncol ? c : 0)] : 0.0, vr, cd[u]);
    }
  }
  for (int r = nl + lane; r - lane < n; r += 2 * kWave) {
    const int r2 = r + kWave;
    const bool in = r < n, in2 = r2 < n;
    const uint32_t ra = in ? r : n - 1, rb = in2 ? r2 : n - 1;  // past the end: the last row (see the symv)
    double av[kStrip], aw[kStrip];
#pragma unroll
    for (int u = 0; u < kStrip; ++u) {
      av[u] = (double)P[(uint32_t)col[u] + ra];
      aw[u] = (double)P[(uint32_t)col[u] + rb];
    }
    const double vr = in ? v[r] : 0.0, vr2 = in2 ? v[r2] : 0.0;
#pragma unroll
    for (int u = 0; u < kStrip; ++u) {
      const bool cok = c0 + (u ^ pl) < ncol;
      cd[u] = fma(cok ? av[u] : 0.0, vr, cd[u]);
      cd[u] = fma(cok ? aw[u] : 0.0, vr2, cd[u]);
    }
  }
  const double tot = wave_strip_sum(cd);
  if ((lane & (kWave / kStrip - 1)) == 0 && c0 + pl < ncol) z[c0 + pl] = tot;
}

// The strips of the symv of the trailing matrix A (n x n, lower triangle)
// and, first in the schedule, the strips of the panel dots z1 = Wp^T v and
// z2 = Vp^T v (npc columns each, n rows, leading dimension ld).
template <class T, int RG>
__device__ void symv_lower_strips(const T* __restrict__ A, int ld, int n, const double* __restrict__ v,
                                  double* spart, int max_m, const T* __restrict__ Vp, const T* __restrict__ Wp,
                                  int npc, double* z1, double* z2, const double* __restrict__ Vl,
                                  const double* __restrict__ Wl, int nl, int pld) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int pl = strip_perm(lane);
  double* my = spart + (int64_t)wv * max_m;
  for (int r = lane; r < n; r += kWave) my[r] = 0.0;
  const int nps = (npc + kStrip - 1) / kStrip;
  const int nextra = 2 * nps;
  const int nstrip = nextra + (n + kStrip - 1) / kStrip;
  for (int t = 0;; ++t) {
    const int s = t * kRedNW + ((t & 1) ? (kRedNW - 1 - wv) : wv);
    if (s >= nstrip) break;
    if (s < nextra) {
      const bool isw = s < nps;
      panel_strip_dots(isw ? Wp : Vp, ld, n, npc, (isw ? s : s - nps) * kStrip, v, isw ? z1 : z2, lane, pl,
                       isw ? Wl : Vl, nl, pld);
      continue;
    }
    const int c0 = (s - nextra) * kStrip;
    double vc[kStrip], cd[kStrip];
    int col[kStrip];  // element offsets of the slot columns from the uniform base A
#pragma unroll
    for (int u = 0; u < kStrip; ++u) {
      const int c = c0 + (u ^ pl);
      vc[u] = (c < n) ? v[c] : 0.0;
      cd[u] = 0.0;
      col[u] = (c < n ? c : c0) * ld;
    }
    // RG groups of 64 rows per iteration: RG * kStrip loads in flight per
    // lane (more groups for 4-byte elements, so that the bytes in flight
    // match the FP64 pass's)
    for (int r = c0 + lane; r - lane < n; r += RG * kWave) {
      double av[RG][kStrip];
      bool in[RG];
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        // unconditional loads (rows past the end read the column's last row,
        // whose cache line the in-range lanes fetch anyway; columns past the
        // end read column c0) and masked values: no branch per load
        in[g] = r + g * kWave < n;
        const uint32_t rg = in[g] ? r + g * kWave : n - 1;
#pragma unroll
        for (int u = 0; u < kStrip; ++u) av[g][u] = (double)A[(uint32_t)col[u] + rg];
      }
#pragma unroll
      for (int g = 0; g < RG; ++g) {
#pragma unroll
        for (int u = 0; u < kStrip; ++u) {
          const bool cok = c0 + (u ^ pl) < n;
          av[g][u] = (in[g] && cok) ? av[g][u] : 0.0;
        }
      }
      double vr[RG], racc[RG];
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        vr[g] = in[g] ? v[r + g * kWave] : 0.0;
        racc[g] = 0.0;
      }
      if (r - lane >= c0 + kStrip) {  // the whole first group lies below the diagonal block
#pragma unroll
        for (int u = 0; u < kStrip; ++u) {
          racc[0] = fma(av[0][u], vc[u], racc[0]);
          cd[u] = fma(av[0][u], vr[0], cd[u]);
        }
      } else {
#pragma unroll
        for (int u = 0; u < kStrip; ++u) {
          const int c = c0 + (u ^ pl);
          const double a_ = (r >= c) ? av[0][u] : 0.0;
          racc[0] = fma(a_, vc[u], racc[0]);
          cd[u] = fma((r > c) ? a_ : 0.0, vr[0], cd[u]);
        }
      }
      // the other groups start 64 rows lower or more, below the diagonal block
#pragma unroll
      for (int g = 1; g < RG; ++g) {
#pragma unroll
        for (int u = 0; u < kStrip; ++u) {
          racc[g] = fma(av[g][u], vc[u], racc[g]);
          cd[u] = fma(av[g][u], vr[g], cd[u]);
        }
      }
#pragma unroll
      for (int g = 0; g < RG; ++g)
        if (in[g]) my[r + g * kWave] += racc[g];
    }
    const double tot = wave_strip_sum(cd);
    if ((lane & (kWave / kStrip - 1)) == 0 && c0 + pl < n) my[c0 + pl] += tot;
  }
}

// acc - sum_{c<i} (P[c*ld] a[c] + Q[c*ld] b[c]) with eight loads in flight
// (P, Q: the same row of two column-major panels).
template <class T>
__device__ __forceinline__ double panel_correct(const T* __restrict__ P, const T* __restrict__ Q, int64_t ld,
                                                const double* a, const double* b, int i, double acc) {
  double acc1 = 0.0;
  int c = 0;
  for (; c + 4 <= i; c += 4) {
    double p[4], q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      p[u] = (double)P[(int64_t)(c + u) * ld];
      q[u] = (double)Q[(int64_t)(c + u) * ld];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc = fma(-p[u], a[c + u], acc);
      acc1 = fma(-q[u], b[c + u], acc1);
    }
  }
  for (; c < i; ++c) {
    acc = fma(-(double)P[(int64_t)c * ld], a[c], acc);
    acc1 = fma(-(double)Q[(int64_t)c * ld], b[c], acc1);
  }
  return acc + acc1;
}

// ------------------------------------------------------- tridiagonalise
// Blocked Householder reduction (lower form), panel width NB; V (the
// Householder vectors, in S) and W (in the W slab) hold the current panel.
// Column k = k0 + i:
//  (2) its reflector (v, tau, beta) from the column brought up to date with
//      the panel's earlier vectors, A[k:, k] - V W[k,:]^T - W V[k,:]^T;
//  (3) y = A22 v with A22 the trailing matrix as it stood at the start of
//      the panel, z1 = W^T v, z2 = V^T v, then y -= V z1 + W z2;
//  (5) w = tau y - (tau/2)(tau y . v) v into column i of W.
// The pass of (3) that reads the rows of V and W also brings the next
// column up to date from the same loads (its term for v, w follows in (5)),
// so the next reflector takes its column from LDS: one dependent global
// round trip per column besides the symv. After the panel,
// A22 -= V W^T + W V^T on MFMA over the tiles that meet the lower triangle;
// only the lower triangle is ever read.
// Outputs: d[0..m), e[0..m-1), tau[0..m-2) and v_k in column k of S.
constexpr int kRedRows = 8;  // rows per thread in the row passes
static_assert(kRedRows * kRedBlock >= 2048, "row passes cover the largest supported order");

// y -= sum_{c<i} P[c] z1[c] + Q[c] z2[c] and an -= sum_{c<i} P[c] wr[c] +
// Q[c] vr[c] from one set of loads (P, Q: the same row of V and W).
template <class T>
__device__ __forceinline__ void panel_correct2(const T* __restrict__ P, const T* __restrict__ Q, int64_t ld,
                                               const double* z1, const double* z2, const double* wr,
                                               const double* vr, int i, double& y, double& an) {
  double y1 = 0.0, a1 = 0.0;
  int c = 0;
  for (; c + 4 <= i; c += 4) {
    double p[4], q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      p[u] = (double)P[(int64_t)(c + u) * ld];
      q[u] = (double)Q[(int64_t)(c + u) * ld];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      y = fma(-p[u], z1[c + u], y);
      y1 = fma(-q[u], z2[c + u], y1);
      an = fma(-p[u], wr[c + u], an);
      a1 = fma(-q[u], vr[c + u], a1);
    }
  }
  for (; c < i; ++c) {
    const double p = (double)P[(int64_t)c * ld], q = (double)Q[(int64_t)c * ld];
    y = fma(-p, z1[c], y);
    y1 = fma(-q, z2[c], y1);
    an = fma(-p, wr[c], an);
    a1 = fma(-q, vr[c], a1);
  }
  y += y1;
  an += a1;
}

template <class T, int PERCU>
__global__ __launch_bounds__(kRedBlock, PERCU) void k_tridiagonalise(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  __shared__ double red[kRedNW];
  __shared__ double vk[kNBMax], wk[kNBMax], z1[kNBMax], z2[kNBMax];
  const int nb = a.nb, pld = a.nb + 1;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  // LDS: v, then one region holding the symv's per-wave row partials
  // (kRedNW rows of max_m; row 0 becomes y = A22 v, row 1 then the next
  // column) and, during the trailing update only, the GEMM staging tiles
  double* sv = dyn;
  double* spart = dyn + a.max_m;
  double* sy = spart;
  double* sa = spart + a.max_m;
  T* gsm = (T*)spart;
  // LDS copy of the current panel's V and W on its first pc rows (row k0 + 1
  // onwards), so that the panel dots and the corrections of most rows do
  // not go back to global memory
  const int pc = a.panel_rows;
  double* Vl = spart + (int64_t)a.panel_off;
  double* Wl = Vl + (int64_t)pc * pld;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) continue;
    T* S = at<T>(a.S, a.off[it]);
    T* Wb = at<T>(a.W, a.off[it]);  // W: column c at Wb + c*ld, rows indexed globally
    T* d = at<T>(a.d, a.doff[it]);
    T* e = at<T>(a.e, a.voff[it]);
    T* tau = at<T>(a.tau, a.voff[it]);
    for (int k0 = 0; k0 + 2 < m; k0 += nb) {
      const int nbt = (m - 2 - k0) < nb ? (m - 2 - k0) : nb;
      for (int i = 0; i < nbt; ++i) {
        const int k = k0 + i;
        const int n2 = m - k - 1;
        const bool fuse_next = i + 1 < nbt;  // the next column belongs to this panel
        // row k+1 of the panel: the next column's coefficients
        if (fuse_next && tid < i) {
          vk[tid] = (double)S[(int64_t)(k0 + tid) * ld + (k + 1)];
          wk[tid] = (double)Wb[(int64_t)tid * ld + (k + 1)];
        }
        // (2) reflector from x = A[k+1:, k]; the panel's first column comes
        // from the slab (as left by the trailing update), the others from sa
        T* x = S + (int64_t)k * ld + (k + 1);
        double part = 0.0, alpha, dkk;
        if (i == 0) {
          for (int q = 1 + tid; q < n2; q += kRedBlock) part += (double)x[q] * (double)x[q];
          alpha = (double)x[0];  // read before the barrier: x[0] is overwritten below
          dkk = (double)S[(int64_t)k * ld + k];
        } else {
          for (int q = 1 + tid; q < n2; q += kRedBlock) part += sa[q + 1] * sa[q + 1];
          alpha = sa[1];
          dkk = sa[0];
        }
        const double sigma = block_sum<kRedNW>(part, red);
        double beta, tk, scale;
        if (sigma == 0.0) {
          beta = alpha; tk = 0.0; scale = 0.0;
        } else {
          const double nrm = sqrt(alpha * alpha + sigma);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tk = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        for (int q = tid; q < n2; q += kRedBlock) {
          const double xq = (i == 0) ? (double)x[q] : sa[q + 1];
          const double vq = (q == 0) ? 1.0 : xq * scale;
          sv[q] = vq;
          x[q] = (T)vq;
          if (i + q < pc) Vl[(i + q) * pld + i] = (double)(T)vq;
        }
        if (tid == 0) {
          d[k] = (T)dkk;
          e[k] = (T)beta;
          tau[k] = (T)tk;
        }
        __syncthreads();
        // column k above row k+1 becomes the zero part of v_k
        for (int q = tid; q <= k; q += kRedBlock) S[(int64_t)k * ld + q] = T(0);
        // (3) y = A22 v, lower triangle only: every element is read once and
        // serves both y[r] += A[r][c] v[c] and y[c] += A[r][c] v[r]; the
        // panel dots z1 = W^T v, z2 = V^T v run as extra strips.
        const int nl = pc - i > 0 ? (pc - i < n2 ? pc - i : n2) : 0;  // cached rows of this column
        symv_lower_strips<T, kSymvGroups<T>>(S + (int64_t)(k + 1) * ld + (k + 1), ld, n2, sv, spart, a.max_m,
                          S + (int64_t)k0 * ld + (k + 1), Wb + (k + 1), i, z1, z2, Vl + i * pld,
                          Wl + i * pld, nl, pld);
        __syncthreads();
        // each thread sums its rows' partials (fixed order), applies
        // y -= V z1 + W z2 and, from the same loads, the next column's
        // update by the panel's earlier vectors. sy aliases row 0 of spart
        // and every thread reads and writes only its own rows (the same rows
        // in (5) below, so no barrier separates the two passes); the partial
        // of tau y . v over those rows is formed on the way.
        double an[kRedRows];
        double pv = 0.0;
#pragma unroll
        for (int rr = 0; rr < kRedRows; ++rr) {
          const int r = tid + rr * kRedBlock;
          an[rr] = 0.0;
          if (r < n2) {
            double acc = spart[r];
#pragma unroll
            for (int w = 1; w < kRedNW; ++w) acc += spart[(int64_t)w * a.max_m + r];
            const bool cached = r < nl;
            if (fuse_next) {
              double nx = (double)S[(int64_t)(k + 1) * ld + (k + 1 + r)];
              if (i > 0) {
                if (cached)
                  panel_correct2(Vl + (i + r) * pld, Wl + (i + r) * pld, 1, z1, z2, wk, vk, i, acc, nx);
                else
                  panel_correct2(S + (int64_t)k0 * ld + (k + 1 + r), Wb + (k + 1 + r), ld, z1, z2, wk, vk, i, acc,
                                 nx);
              }
              an[rr] = nx;
            } else if (i > 0) {
              acc = cached ? panel_correct(Vl + (i + r) * pld, Wl + (i + r) * pld, 1, z1, z2, i, acc)
                           : panel_correct(S + (int64_t)k0 * ld + (k + 1 + r), Wb + (k + 1 + r), ld, z1, z2, i, acc);
            }
            sy[r] = acc;
            pv = fma(tk * acc, sv[r], pv);
          }
        }
        // (5) w = tau y - (tau/2)(tau y . v) v into column i of W; the next
        // column takes the term of v_k, w_k: -v w[0] - w v[0], v[0] = 1
        // (block_sum's barriers also publish sy[0])
        const double Kc = 0.5 * tk * block_sum<kRedNW>(pv, red);
        const double w0 = tk * sy[0] - Kc * sv[0];
#pragma unroll
        for (int rr = 0; rr < kRedRows; ++rr) {
          const int r = tid + rr * kRedBlock;
          if (r < n2) {
            const double wr = tk * sy[r] - Kc * sv[r];
            Wb[(int64_t)i * ld + (k + 1 + r)] = (T)wr;
            if (i + r < pc) Wl[(i + r) * pld + i] = (double)(T)wr;
            if (fuse_next) sa[r] = an[rr] - sv[r] * w0 - wr;
          }
        }
        __syncthreads();
      }
      // trailing update A22 -= V W^T + W V^T (lower tiles)
      const int c0 = k0 + nbt;
      const int M = m - c0;
      if (M > 0) {
        const T* V2 = S + (int64_t)k0 * ld + c0;
        const T* W2 = Wb + c0;
        T* C = S + (int64_t)c0 * ld + c0;
        wg_syr2k_lower<T, kRedNW>(M, nbt, T(-1), V2, ld, W2, ld, C, ld, gsm);
      }
    }
    if (tid == 0) {
      if (m >= 2) {
        d[m - 2] = S[(int64_t)(m - 2) * ld + (m - 2)];
        e[m - 2] = S[(int64_t)(m - 2) * ld + (m - 1)];
        tau[m - 2] = T(0);
      }
      d[m - 1] = S[(int64_t)(m - 1) * ld + (m - 1)];
      e[m - 1] = T(0);
    }
    __syncthreads();
    // the last two columns carry no reflector: zero them
    for (int q = tid; q < 2 * m; q += kRedBlock) {
      const int c = q < m ? m - 2 : m - 1;
      const int r = q < m ? q : q - m;
      if (c >= 0) S[(int64_t)c * ld + r] = T(0);
    }
  }
}

// --------------------------------------------- tridiagonal eigensolver
// Eigen-decomposition of T = tridiag(e, d, e) in FP64 (Section 3.2 leaves
// the dense eigensolver open; this is Sturm-count bisection with Newton
// steps, twisted factorisations and inverse iteration):
//  * off-diagonals below eps * sqrt(|d_i d_i+1|) are set to zero, which
//    splits T into unreduced blocks; eigenvalue index j belongs to the block
//    holding row j;
//  * eigenvalue j: a bracket from Sturm counts of its block (one lane per
//    eigenvalue), from Gershgorin bounds down to a few ulps; on an unsplit
//    T, once the bracket holds eigenvalue j alone, Newton steps on
//    log det(T - xI) choose the trial points;
//  * eigenvector of an eigenvalue whose neighbours in its block are further
//    than ctol * ||T|| away: twisted factorisation T - lambda I =
//    N_r D_r N_r^T with the twist r minimising |gamma_r|, then
//    z_r = 1, z_i = -L_i z_i+1 (i < r), z_i+1 = -U_i z_i (i >= r);
//  * a cluster of closer eigenvalues is handled by one lane, member after
//    member: inverse iteration with LDL^T solves from a seeded start vector,
//    each iterate orthogonalised (modified Gram-Schmidt) against the
//    cluster's earlier vectors, with perturbed shifts for coincident values.
// Eigenvalues replace d (ascending within each block). Two FP64 m x m
// scratch arrays Z and U hold the factors, lane j owning column j (element
// (i, j) at i*ld + j, so the lanes' accesses to one component coalesce);
// eigenvector j ends normalised in column j of Z.
constexpr int kEigBlock = 256;
constexpr int kEigNW = kEigBlock / kWave;
constexpr double kUnitRoundoff = 1.1102230246251565e-16;  // 2^-53
constexpr double kSafeMin = 2.2250738585072014e-308;
constexpr int kInvIterMax = 5;
constexpr int kOrthB = 16;  // eigenvectors per block of the local reorthogonalisation
static_assert(kOrthB * kOrthB == kEigBlock, "one thread per entry of a block Gram matrix");

// Counter-based uniform deviate in (-1, 1): the splitmix64 finaliser
// (Steele, Lea, Flood 2014) of a 64-bit key.
__device__ __forceinline__ double hash_unit(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// 1/q from the hardware reciprocal and two Newton steps (relative error a
// few ulps; |q| >= pivmin >= the smallest normal, so 1/q is finite).
__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// Number of eigenvalues of block [s, t) below x (Sturm sequence of the
// LDL^T factorisation of T - xI; tiny pivots replaced by -pivmin, so that
// |e^2 / q| <= e^2 / pivmin stays finite).
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int s, int t, double x,
                                           double pivmin) {
  double q = d[s] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = s + 1; i < t; ++i) {
    q = fma(-e2[i - 1], recip(q), d[i] - x);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// The same count over a whole unsplit T (rows 0..m, m the same in every
// lane): uniform bounds give scalar loop control and constant LDS offsets.
// After the guard |q| >= pivmin > 0, so q < 0 is its sign bit.
__device__ __forceinline__ int sturm_count_all(const double* d, const double* e2, int m, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = (int)((uint32_t)__double2hiint(q) >> 31);
#pragma unroll 4
  for (int i = 1; i < m; ++i) {
    q = fma(-e2[i - 1], recip(q), d[i] - x);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (int)((uint32_t)__double2hiint(q) >> 31);
  }
  return cnt;
}

// The count of sturm_count_all at two points x1, x2 in one pass over T (the
// two recurrences are independent, so their latencies overlap), each with
// the logarithmic derivative sd = sum_i q_i'/q_i = d/dx log det(T - xI) =
// -sum_l 1/(lambda_l - x), from q_i' = -1 + e_{i-1}^2 q_{i-1}' / q_{i-1}^2
// (a Newton step for an eigenvalue is -1/sd). The pivots are those of
// sturm_count_all. Guarded pivots or overflow make sd infinite or NaN,
// which the caller rejects.
__device__ __forceinline__ void sturm_newton_all2(const double* d, const double* e2, int m, double x1, double x2,
                                                  double pivmin, int& c1, int& c2, double& sd1, double& sd2) {
  double q1 = d[0] - x1, q2 = d[0] - x2;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  if (fabs(q2) < pivmin) q2 = -pivmin;
  int n1 = (int)((uint32_t)__double2hiint(q1) >> 31), n2 = (int)((uint32_t)__double2hiint(q2) >> 31);
  double qp1 = -1.0, qp2 = -1.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 2
  for (int i = 1; i < m; ++i) {
    const double ee = e2[i - 1], di = d[i];
    const double r1 = recip(q1), r2 = recip(q2);
    s1 = fma(qp1, r1, s1);
    s2 = fma(qp2, r2, s2);
    const double t1 = ee * r1, t2 = ee * r2;
    qp1 = fma(t1 * r1, qp1, -1.0);
    qp2 = fma(t2 * r2, qp2, -1.0);
    q1 = fma(-ee, r1, di - x1);
    q2 = fma(-ee, r2, di - x2);
    if (fabs(q1) < pivmin) q1 = -pivmin;
    if (fabs(q2) < pivmin) q2 = -pivmin;
    n1 += (int)((uint32_t)__double2hiint(q1) >> 31);
    n2 += (int)((uint32_t)__double2hiint(q2) >> 31);
  }
  sd1 = fma(qp1, recip(q1), s1);
  sd2 = fma(qp2, recip(q2), s2);
  c1 = n1;
  c2 = n2;
}

// Sturm-safeguarded Newton search for eigenvalue k of an unsplit T: the
// bracket [lo, hi] (counts clo <= k < chi) is kept exactly as in bisection
// and the search ends on the same width test; only the next trial point
// differs. While the bracket holds more than eigenvalue k, it is the
// midpoint. Once it holds k alone, it is the Newton point x - 1/sd if that
// lies inside and the Newton steps at least halve every two iterations.
// Newton from one side never closes the far end, so when the step is within
// the tolerance, the trial point goes across the eigenvalue towards the open
// end by (|step| + g) 2^j, j counting such probes.
struct EigSearch {
  double lo, hi, x, w1, w2;
  int clo, chi, k, npr;
  bool done;
};

__device__ __forceinline__ bool search_stop(const EigSearch& S, double atol) {
  return S.hi - S.lo <= 4.0 * kUnitRoundoff * fmax(fabs(S.lo), fabs(S.hi)) + atol || !(S.x > S.lo && S.x < S.hi);
}

// Start from the multisection counts msc[0..nm) at glo + (i + 1) hstep: the
// last point with count <= k, and the next one.
__device__ __forceinline__ void search_init(EigSearch& S, int k, const int* msc, double glo, double ghi, double hstep,
                                            int m, double atol) {
  constexpr int nm = kEigBlock;
  int a2 = 0, b2 = nm;
  while (a2 < b2) {
    const int mid = (a2 + b2) >> 1;
    if (msc[mid] <= k) a2 = mid + 1;
    else b2 = mid;
  }
  // points 0..a2-1 have count <= k, point a2 (if any) has count > k
  S.lo = a2 > 0 ? glo + a2 * hstep : glo;
  S.hi = a2 < nm ? glo + (a2 + 1) * hstep : ghi;
  S.clo = a2 > 0 ? msc[a2 - 1] : 0;
  S.chi = a2 < nm ? msc[a2] : m;
  S.x = 0.5 * (S.lo + S.hi);
  S.w1 = S.w2 = INFINITY;
  S.npr = 0;
  S.k = k;
  S.done = search_stop(S, atol);
}

__device__ __forceinline__ void search_update(EigSearch& S, int cnt, double sd, double atol) {
  const bool up = cnt > S.k;
  if (up) {
    S.hi = S.x;
    S.chi = cnt;
  } else {
    S.lo = S.x;
    S.clo = cnt;
  }
  const double g = 2.0 * kUnitRoundoff * fmax(fabs(S.lo), fabs(S.hi)) + 0.5 * atol;
  const double step = -1.0 / sd;
  const double st = fabs(step);
  const bool iso = S.chi - S.clo == 1;
  const double xb = 0.5 * (S.lo + S.hi);
  double xn = xb, wn = fabs(xb - S.x);
  if (iso && !(st > 2.0 * g)) {
    const double pr = S.x + (up ? -1.0 : 1.0) * (st + g) * ldexp(1.0, S.npr);
    if (pr > S.lo && pr < S.hi) {
      xn = pr;
      wn = S.w1;
      ++S.npr;
    } else {
      S.npr = 0;
    }
  } else {
    S.npr = 0;
    const double xt = S.x + step;
    if (iso && xt > S.lo && xt < S.hi && !(st > 0.5 * S.w2)) {
      xn = xt;
      wn = st;
    }
  }
  S.w2 = S.w1;
  S.w1 = wn;
  S.x = xn;
  S.done = search_stop(S, atol);
}

__device__ __forceinline__ double guard_pivot(double D, double tol) {
  return fabs(D) < tol ? (D < 0.0 ? -tol : tol) : D;
}

// Twisted-factorisation eigenvector of block [s, t) for shift lam, left
// unnormalised in column jj of Z (z_r = 1). Returns false when the result
// is not finite or its residual |gamma_r| / ||z|| is not small.
__device__ bool twisted_vector(const double* d, const double* e, int s, int t, double lam, double tol,
                               double rtol, double* Z, double* U, int ld, int jj, double& nrm2) {
  double Dp = guard_pivot(d[s] - lam, tol);
  for (int i = s; i < t - 1; ++i) {
    const double L = e[i] / Dp;
    Z[(int64_t)i * ld + jj] = L;
    Dp = guard_pivot((d[i + 1] - lam) - L * e[i], tol);
  }
  double Dm = guard_pivot(d[t - 1] - lam, tol);
  double gbest = fabs(Dm - (t - 1 > s ? Z[(int64_t)(t - 2) * ld + jj] * e[t - 2] : 0.0));
  int r = t - 1;
  for (int i = t - 2; i >= s; --i) {
    const double Ui = e[i] / Dm;
    U[(int64_t)i * ld + jj] = Ui;
    Dm = guard_pivot((d[i] - lam) - Ui * e[i], tol);
    const double g = fabs(Dm - (i > s ? Z[(int64_t)(i - 1) * ld + jj] * e[i - 1] : 0.0));
    if (g < gbest) {
      gbest = g;
      r = i;
    }
  }
  double n2 = 1.0, zn = 1.0;
  for (int i = t - 2; i >= s; --i) {
    if (i < r) {
      const double z = -Z[(int64_t)i * ld + jj] * zn;
      Z[(int64_t)i * ld + jj] = z;
      n2 = fma(z, z, n2);
      zn = z;
    }
  }
  Z[(int64_t)r * ld + jj] = 1.0;
  double zp = 1.0;
  for (int i = s; i < t - 1; ++i) {
    if (i >= r) {
      const double z = -U[(int64_t)i * ld + jj] * zp;
      Z[(int64_t)(i + 1) * ld + jj] = z;
      n2 = fma(z, z, n2);
      zp = z;
    }
  }
  nrm2 = n2;
  return isfinite(n2) && gbest <= rtol * sqrt(n2);
}

// Inverse iteration for the k eigenvalues lam[j0 .. j0+k) of block [s, t),
// one lane, member by member; results (unit norm) in columns j0.. of Z.
// Column j of U holds the iterate, column j of Z the LDL^T multipliers
// until the member is done. Returns the number of members that did not
// converge.
__device__ int cluster_vectors(const double* d, const double* e, const double* lam, int s, int t, int j0, int k,
                               double tol, double rtol, double* Z, double* U, int ld, uint64_t seed) {
  int bad = 0;
  double lprev = 0.0;
  for (int c = 0; c < k; ++c) {
    const int jc = j0 + c;
    double lc = lam[jc];
    if (c > 0) {
      const double pert = 10.0 * kUnitRoundoff * fmax(fabs(lc), tol);
      if (lc - lprev < pert) lc = lprev + pert;
    }
    lprev = lc;
    double* y = U + jc;
    double* L = Z + jc;
    double nb = 0.0;
    for (int i = s; i < t; ++i) {
      const double b = hash_unit(seed ^ ((uint64_t)jc << 32) ^ (uint64_t)i);
      y[(int64_t)i * ld] = b;
      nb = fma(b, b, nb);
    }
    double sc = 1.0 / sqrt(nb);
    for (int i = s; i < t; ++i) y[(int64_t)i * ld] *= sc;
    int conv = 0;
    for (int iter = 0; iter < kInvIterMax && conv < 2; ++iter) {
      // (T - lc I) y <- y: LDL^T without pivoting (guarded pivots)
      double D = guard_pivot(d[s] - lc, tol);
      double w = y[(int64_t)s * ld];
      for (int i = s; i < t - 1; ++i) {
        const double Li = e[i] / D;
        L[(int64_t)i * ld] = Li;
        y[(int64_t)i * ld] = w / D;
        w = y[(int64_t)(i + 1) * ld] - Li * w;
        D = guard_pivot((d[i + 1] - lc) - Li * e[i], tol);
      }
      double yi = w / D;
      y[(int64_t)(t - 1) * ld] = yi;
      for (int i = t - 2; i >= s; --i) {
        yi = y[(int64_t)i * ld] - L[(int64_t)i * ld] * yi;
        y[(int64_t)i * ld] = yi;
      }
      // orthogonalise against the cluster's finished vectors
      for (int q = 0; q < c; ++q) {
        const double* zq = Z + (j0 + q);
        double dot = 0.0;
        for (int i = s; i < t; ++i) dot = fma(y[(int64_t)i * ld], zq[(int64_t)i * ld], dot);
        for (int i = s; i < t; ++i) y[(int64_t)i * ld] = fma(-dot, zq[(int64_t)i * ld], y[(int64_t)i * ld]);
      }
      double n2 = 0.0;
      for (int i = s; i < t; ++i) n2 = fma(y[(int64_t)i * ld], y[(int64_t)i * ld], n2);
      const double nrm = sqrt(n2);
      // the start had unit norm, so 1/nrm estimates the residual
      if (isfinite(nrm) && nrm > 0.0 && 1.0 <= rtol * nrm) ++conv;
      sc = (isfinite(nrm) && nrm > 0.0) ? 1.0 / nrm : 0.0;
      for (int i = s; i < t; ++i) y[(int64_t)i * ld] *= sc;
    }
    if (conv == 0) ++bad;
    for (int i = s; i < t; ++i) L[(int64_t)i * ld] = y[(int64_t)i * ld];
  }
  return bad;
}

template <class T>
__global__ __launch_bounds__(kEigBlock) void k_tridiag_eig(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  __shared__ double red[4 * kEigNW];
  __shared__ int ired[2 * kEigNW];
  __shared__ int msc[kEigBlock];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int M = a.max_m;
  double* d = dyn;
  double* e = dyn + M;
  double* e2 = dyn + 2 * M;  // e^2 during bisection, then 1/||z|| per eigenvector
  double* lam = dyn + 3 * M;
  int* bs = (int*)(dyn + 4 * M);  // start of the unreduced block holding row i
  int* be = bs + M;               // its end (exclusive)
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) continue;
    T* dg = at<T>(a.d, a.doff[it]);
    const T* eg = at<T>((const void*)a.e, a.voff[it]);
    double* Z = at<double>(a.escr, a.eoff[it]);
    double* U = Z + (int64_t)ld * ld;
    for (int i = tid; i < m; i += kEigBlock) {
      const double di = (double)dg[i];
      double ei = 0.0;
      if (i + 1 < m) {
        ei = (double)eg[i];
        const double dn = (double)dg[i + 1];
        if (fabs(ei) <= kUnitRoundoff * sqrt(fabs(di)) * sqrt(fabs(dn))) ei = 0.0;
      }
      d[i] = di;
      e[i] = ei;
      e2[i] = ei * ei;
    }
    __syncthreads();
    double tn = 0.0, glo = INFINITY, ghi = -INFINITY, emax2 = 0.0;
    for (int i = tid; i < m; i += kEigBlock) {
      const double el = i > 0 ? fabs(e[i - 1]) : 0.0, er = fabs(e[i]);
      tn = fmax(tn, fabs(d[i]) + el + er);
      glo = fmin(glo, d[i] - el - er);
      ghi = fmax(ghi, d[i] + el + er);
      emax2 = fmax(emax2, e2[i]);
    }
    tn = wave_max(tn);
    glo = wave_min(glo);
    ghi = wave_max(ghi);
    emax2 = wave_max(emax2);
    if (lane == 0) {
      red[wv] = tn;
      red[kEigNW + wv] = glo;
      red[2 * kEigNW + wv] = ghi;
      red[3 * kEigNW + wv] = emax2;
    }
    if (tid == 0) {
      int st = 0;
      for (int i = 0; i < m; ++i) {
        bs[i] = st;
        if (e[i] == 0.0) st = i + 1;
      }
      int en = m;
      for (int i = m - 1; i >= 0; --i) {
        if (e[i] == 0.0) en = i + 1;
        be[i] = en;
      }
    }
    __syncthreads();
    tn = red[0];
    glo = red[kEigNW];
    ghi = red[2 * kEigNW];
    emax2 = red[3 * kEigNW];
    for (int w = 1; w < kEigNW; ++w) {
      tn = fmax(tn, red[w]);
      glo = fmin(glo, red[kEigNW + w]);
      ghi = fmax(ghi, red[2 * kEigNW + w]);
      emax2 = fmax(emax2, red[3 * kEigNW + w]);
    }
    const double pivmin = kSafeMin * fmax(1.0, emax2);
    const double pad = 2.0 * kUnitRoundoff * tn * m + 4.0 * pivmin;
    glo -= pad;
    ghi += pad;
    // eigenvalues: one lane each, to a few ulps or 1e-3 eps ||T||
    const double atol = 1e-3 * kUnitRoundoff * tn + pivmin;
    // multisection start for an unsplit T: counts at kEigBlock evenly
    // spaced points (one Sturm pass per thread) narrow every bracket by a
    // factor kEigBlock + 1 before the bisection
    const bool one_block = be[0] == m;
    const double hstep = (ghi - glo) / (kEigBlock + 1);
    if (one_block) msc[tid] = sturm_count_all(d, e2, m, glo + (tid + 1) * hstep, pivmin);
    __syncthreads();
    if (one_block) {
      // a lane searches eigenvalues jj and jj + kEigBlock together: their
      // Sturm chains are interleaved in one pass over T (two independent
      // dependency chains, the d / e^2 loads shared)
      for (int jj = tid; jj < m; jj += 2 * kEigBlock) {
        const int j2 = jj + kEigBlock;
        EigSearch S1, S2;
        search_init(S1, jj, msc, glo, ghi, hstep, m, atol);
        if (j2 < m) {
          search_init(S2, j2, msc, glo, ghi, hstep, m, atol);
        } else {
          S2 = S1;
          S2.done = true;
        }
        for (int iter = 0; iter < 256 && !(S1.done && S2.done); ++iter) {
          int c1, c2;
          double sd1, sd2;
          sturm_newton_all2(d, e2, m, S1.x, S2.done ? S1.x : S2.x, pivmin, c1, c2, sd1, sd2);
          if (!S1.done) search_update(S1, c1, sd1, atol);
          if (!S2.done) search_update(S2, c2, sd2, atol);
        }
        lam[jj] = 0.5 * (S1.lo + S1.hi);
        if (j2 < m) lam[j2] = 0.5 * (S2.lo + S2.hi);
      }
    } else {
      for (int jj = tid; jj < m; jj += kEigBlock) {
        const int s = bs[jj], t = be[jj], k = jj - s;
        double lo = glo, hi = ghi;
        for (int iter = 0; iter < 256; ++iter) {
          const double mid = 0.5 * (lo + hi);
          if (hi - lo <= 4.0 * kUnitRoundoff * fmax(fabs(lo), fabs(hi)) + atol || !(mid > lo && mid < hi)) break;
          const int cnt = sturm_count(d, e2, s, t, mid, pivmin);
          if (cnt > k) hi = mid;
          else lo = mid;
        }
        lam[jj] = 0.5 * (lo + hi);
      }
    }
    __syncthreads();
    // eigenvectors
    const double ctol = a.cluster_tol * tn;
    const double tol = kUnitRoundoff * fmax(tn, kSafeMin);
    const double rtol = 16.0 * kUnitRoundoff * fmax(tn, kSafeMin) * m;
    const uint64_t seed = 0x5A17B0D1ull * (uint64_t)(j + 1);
    int ninv = 0, bad = 0;
    for (int jj = tid; jj < m; jj += kEigBlock) {
      const int s = bs[jj], t = be[jj];
      const bool wp = jj > s && lam[jj] - lam[jj - 1] <= ctol;
      const bool wn = jj + 1 < t && lam[jj + 1] - lam[jj] <= ctol;
      double sc = 1.0;
      if (!wp && !wn) {
        double n2 = 0.0;
        if (twisted_vector(d, e, s, t, lam[jj], tol, rtol, Z, U, ld, jj, n2)) {
          sc = 1.0 / sqrt(n2);
        } else {
          bad += cluster_vectors(d, e, lam, s, t, jj, 1, tol, rtol, Z, U, ld, seed);
          ++ninv;
        }
      } else if (!wp) {
        int k = 1;
        while (jj + k < t && lam[jj + k] - lam[jj + k - 1] <= ctol) ++k;
        bad += cluster_vectors(d, e, lam, s, t, jj, k, tol, rtol, Z, U, ld, seed);
        ninv += k;
      }
      e2[jj] = wp ? 1.0 : sc;  // cluster members are normalised by their leader
    }
    __syncthreads();
    // Column jj of Z still has to be scaled by e2[jj]; the scale goes to row
    // 0 of the U region (dead from here on) and the reorthogonalisation
    // applies it where it reads the column. On a split T the rows outside a
    // vector's block are zeroed here.
    for (int jj = tid; jj < m; jj += kEigBlock) {
      if (!one_block) {
        const int s = bs[jj], t = be[jj];
        for (int i = 0; i < s; ++i) Z[(int64_t)i * ld + jj] = 0.0;
        for (int i = t; i < m; ++i) Z[(int64_t)i * ld + jj] = 0.0;
      }
      U[jj] = e2[jj];
    }
    // eigenvalues, spectrum checks and flags
    double lmin = INFINITY, lmax = -INFINITY;
    for (int jj = tid; jj < m; jj += kEigBlock) {
      const double v = lam[jj];
      lmin = fmin(lmin, v);
      lmax = fmax(lmax, v);
      dg[jj] = (T)v;
    }
    lmin = wave_min(lmin);
    lmax = wave_max(lmax);
    bad = (int)wave_sum((double)bad);
    ninv = (int)wave_sum((double)ninv);
    __syncthreads();
    if (lane == 0) {
      red[wv] = lmin;
      red[kEigNW + wv] = lmax;
      ired[wv] = bad;
      ired[kEigNW + wv] = ninv;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kEigNW; ++w) {
        lmin = fmin(lmin, red[w]);
        lmax = fmax(lmax, red[kEigNW + w]);
      }
      int nbad = 0, nin = 0;
      for (int w = 0; w < kEigNW; ++w) {
        nbad += ired[w];
        nin += ired[kEigNW + w];
      }
      int flags = nbad ? LF_UNCONV : 0;
      // lambda_min <= 0 has no real inverse p-th root; in the FP32 pass an
      // estimated condition number above kappa_max sends the submatrix to
      // the FP64 pass
      if (!a.fp64) {
        if ((flags & LF_UNCONV) || !(lmin > 0.0) || lmax > a.kappa_max * lmin) flags = LF_FALLBACK;
      } else if (!(lmin > 0.0)) {
        flags |= LF_NONPOS;
      }
      a.flags[it] = a.only_flagged ? (flags | LF_FALLBACK) : flags;
      if (flags & LF_NONPOS) atomicAdd((unsigned long long*)&a.status[ST_NONPOS], 1ull);
      if (a.fp64 && (flags & LF_UNCONV)) atomicAdd((unsigned long long*)&a.status[ST_UNCONV], 1ull);
      if (!a.fp64 && (flags & LF_FALLBACK)) atomicAdd((unsigned long long*)&a.status[ST_FALLBACK], 1ull);
      if (nin) atomicAdd((unsigned long long*)&a.status[ST_INVITER], (unsigned long long)nin);
    }
    __syncthreads();
  }
}

// Local reorthogonalisation of the eigenvectors of T, then Z into the Q slab.
// Vectors computed one by one are orthogonal only to about eps ||T|| / gap;
// the error lies mostly along eigenvectors of nearby eigenvalues, i.e. of
// nearby indices. Blocks B of kOrthB consecutive vectors are made
// orthonormal in order, against the previous (finished) block P:
//   pass 1   C = P^T B and H = B^T B (MFMA, both from one read of P and B)
//   small    G = H - C^T C = (B - P C)^T (B - P C), R^T R = G (Cholesky),
//            Rinv = R^-1, D = C Rinv
//   pass 2   B <- B Rinv - P D = (B - P C) R^-1, also stored into Q (type T)
template <class T>
__global__ __launch_bounds__(kEigBlock) void k_eig_orth(LargeArgs a) {
  __shared__ int s_item, s_bad;
  __shared__ double acc_s[kEigNW][2][kOrthB * kOrthB];
  __shared__ double Cs[kOrthB * kOrthB], Gs[kOrthB * kOrthB], Rs[kOrthB * kOrthB], Ri[kOrthB * kOrthB],
      Ds[kOrthB * kOrthB];
  __shared__ double tile[kOrthB * (kWave + 1)];
  __shared__ double bsc[kOrthB];  // column scales of the current block
  typedef Mfma<double>::acc_t acc_t;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int li = lane & 15, lk = lane >> 4;
  const int k = tid / kOrthB, l = tid - k * kOrthB;  // one entry of a 16 x 16 matrix
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) continue;
    T* Qz = at<T>(a.Q, a.qoff[it]);  // Z, column-major, for the back-transformation
    double* Z = at<double>(a.escr, a.eoff[it]);
    // 1/||z|| of each column as left by the eigensolver (row 0 of the U
    // region); a block B is scaled as it is read, P is already final
    const double* zsc = Z + (int64_t)ld * ld;
    if (tid == 0) s_bad = 0;
    for (int j0 = 0; j0 < m; j0 += kOrthB) {
      const int nb = (m - j0) < kOrthB ? (m - j0) : kOrthB;
      double* B = Z + j0;
      const double* P = Z + (j0 - kOrthB);  // used only when j0 > 0
      const bool hasP = j0 > 0;
      if (tid < kOrthB) bsc[tid] = tid < nb ? zsc[j0 + tid] : 0.0;
      const double lsc = li < nb ? zsc[j0 + li] : 0.0;
      // pass 1: wave w takes rows 4w.., 4(w+NW).. (four rows per MFMA step).
      // Loads are unconditional (rows past m read row m - 1, columns past nb
      // lie in the slab's padding, ld being a multiple of 16; without a
      // previous block P reads B) and masked afterwards, so that the
      // unrolled steps keep several loads in flight.
      acc_t cacc = acc_t{0, 0, 0, 0}, hacc = acc_t{0, 0, 0, 0};
      const double* Pr = hasP ? P : B;
      constexpr int kU = 4;  // MFMA steps whose loads are issued together
      for (int i00 = 4 * wv; i00 < m; i00 += 4 * kEigNW * kU) {
        double braw[kU], praw[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int i = i00 + 4 * kEigNW * u + lk;
          const int64_t o = (int64_t)(i < m ? i : m - 1) * ld + li;
          braw[u] = B[o];
          praw[u] = Pr[o];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int i = i00 + 4 * kEigNW * u + lk;
          const bool ok = i < m && li < nb;
          const double bv = ok ? braw[u] * lsc : 0.0;
          const double pv = (hasP && i < m) ? praw[u] : 0.0;
          hacc = Mfma<double>::step(bv, bv, hacc);
          cacc = Mfma<double>::step(pv, bv, cacc);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = Mfma<double>::row(lk, r);
        acc_s[wv][0][row * kOrthB + li] = cacc[r];
        acc_s[wv][1][row * kOrthB + li] = hacc[r];
      }
      __syncthreads();
      double c = 0.0, h = 0.0;
#pragma unroll
      for (int w = 0; w < kEigNW; ++w) {
        c += acc_s[w][0][tid];
        h += acc_s[w][1][tid];
      }
      Cs[tid] = c;
      __syncthreads();
      {
        double g = h;
        for (int q = 0; q < kOrthB; ++q) g = fma(-Cs[q * kOrthB + k], Cs[q * kOrthB + l], g);
        if (k >= nb || l >= nb) g = (k == l) ? 1.0 : 0.0;
        Gs[tid] = g;
      }
      __syncthreads();
      // right-looking Cholesky of G: row kk of R per step
      for (int kk = 0; kk < kOrthB; ++kk) {
        const double piv = Gs[kk * kOrthB + kk];
        if (tid < kOrthB) {
          const double r = sqrt(fmax(piv, kSafeMin));
          Rs[kk * kOrthB + tid] = tid < kk ? 0.0 : (tid == kk ? r : Gs[kk * kOrthB + tid] / r);
        }
        if (tid == 0 && !(piv > 0.25)) s_bad = 1;  // the vectors were far from orthonormal
        __syncthreads();
        if (k > kk && l > kk) Gs[tid] -= Rs[kk * kOrthB + k] * Rs[kk * kOrthB + l];
        __syncthreads();
      }
      // Rinv: lane `tid` solves R x = e_tid by back substitution (its own column)
      if (tid < kOrthB) {
        for (int q = kOrthB - 1; q >= 0; --q) {
          double v = (q == tid) ? 1.0 : 0.0;
          for (int kk = q + 1; kk < kOrthB; ++kk) v = fma(-Rs[q * kOrthB + kk], Ri[kk * kOrthB + tid], v);
          Ri[q * kOrthB + tid] = v / Rs[q * kOrthB + q];
        }
      }
      __syncthreads();
      {
        double dv = 0.0;
        for (int q = 0; q < kOrthB; ++q) dv = fma(Cs[k * kOrthB + q], Ri[q * kOrthB + l], dv);
        Ds[tid] = dv;
      }
      __syncthreads();
      // pass 2 reads B unscaled: (B diag(bsc)) Rinv = B (diag(bsc) Rinv)
      Ri[tid] *= bsc[k];
      __syncthreads();
      // pass 2, 64 rows at a time: thread (row, column); the 16 threads of
      // a row sit in one wave and read the whole row before any of them
      // writes it. The columns go to Q (column-major) through an LDS
      // transpose so that both the reads and the writes coalesce.
      for (int i0 = 0; i0 < m; i0 += kWave) {
        // (each row's 16 values loaded together and unconditionally: rows past
        // m read row m - 1 and are discarded, columns past nb lie in the
        // padding and are masked)
        for (int q = tid; q < kWave * kOrthB; q += kEigBlock) {
          const int ii = q / kOrthB, lq = q - ii * kOrthB, i = i0 + ii;
          const int64_t o = (int64_t)(i < m ? i : m - 1) * ld;
          constexpr int kH = kOrthB / 2;  // values in flight per batch
          double bv[kH];
          double v = 0.0;
#pragma unroll
          for (int h = 0; h < kOrthB; h += kH) {
#pragma unroll
            for (int kk = 0; kk < kH; ++kk) bv[kk] = B[o + h + kk];
#pragma unroll
            for (int kk = 0; kk < kH; ++kk) v = fma(h + kk < nb ? bv[kk] : 0.0, Ri[(h + kk) * kOrthB + lq], v);
          }
          if (hasP) {
#pragma unroll
            for (int h = 0; h < kOrthB; h += kH) {
#pragma unroll
              for (int kk = 0; kk < kH; ++kk) bv[kk] = P[o + h + kk];
#pragma unroll
              for (int kk = 0; kk < kH; ++kk) v = fma(-bv[kk], Ds[(h + kk) * kOrthB + lq], v);
            }
          }
          if (i < m) {
            if (lq < nb) B[(int64_t)i * ld + lq] = v;
          } else {
            v = 0.0;
          }
          tile[lq * (kWave + 1) + ii] = v;
        }
        __syncthreads();
        for (int q = tid; q < kWave * kOrthB; q += kEigBlock) {
          const int lq = q / kWave, ii = q - lq * kWave, i = i0 + ii;
          if (i < m && lq < nb) Qz[(int64_t)(j0 + lq) * ld + i] = (T)tile[lq * (kWave + 1) + ii];
        }
        __syncthreads();
      }
    }
    if (tid == 0 && s_bad) {
      // a block without full rank: the eigensolver failed for this submatrix
      const int fl = a.flags[it];
      if (a.fp64) {
        if (!(fl & LF_UNCONV)) atomicAdd((unsigned long long*)&a.status[ST_UNCONV], 1ull);
        a.flags[it] = fl | LF_UNCONV;
      } else if (!(fl & LF_FALLBACK)) {
        atomicAdd((unsigned long long*)&a.status[ST_FALLBACK], 1ull);
        a.flags[it] = LF_FALLBACK;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------ back-transform
// Q = Q1 Z with Q1 = H_0 H_1 ... H_{m-3} applied to Z in place, block by
// block from the last one. A block of up to kNBq consecutive reflectors
// with vectors V (rows k0+1.., zeros above each vector's first entry) acts
// as H_k0 ... H_k0+nb-1 = I - V T V^T, so
//   Q[k0+1:, :] -= V (T (V^T Q[k0+1:, :])) = V ((V T^T)^T Q[k0+1:, :]).
// T is upper triangular: for a half of kNBh reflectors, T[c][c] = tau_c
// and T[0:c, c] = -tau_c T[0:c, 0:c] (V^T V)[0:c, c] (one wave, in LDS);
// the two halves merge as [[T1, -T1 (V1^T V2) T2], [0, T2]]. All products
// on MFMA; 2 m^3 flops in all.
// Two kernels: k_back_prep forms, per item and block, VT = V T^T into the
// W slab at V's position; k_back_apply then takes (item, kBackCols columns
// of Q) units, independent of each other since the blocks act on the rows:
// each applies every block to its columns, so Q crosses HBM about once per
// block while the V and VT panels, read by all column units of an item,
// come from the caches.
constexpr int kNBq = 128;
constexpr int kNBh = kNBq / 2;
constexpr int kBackCols = 64;
static_assert(kXcdQueues == kXcdQueueCount, "one work queue per XCD on both sides");

size_t apply_scratch_elems(int ld) {
  // G, T, X, then Wm (kNBq x ld) for the column units; ld rounded up to
  // whole column blocks
  const size_t ldc = ((size_t)ld + kBackCols - 1) / kBackCols * kBackCols;
  return 2 * (size_t)kNBq * kNBq + (size_t)kNBh * kNBh + (size_t)kNBq * ldc;
}

// Upper-triangular compact-WY factor of reflectors c0 .. c0+nh-1 of a block
// from its Gram matrix G (column-major, leading dimension kNBq), into
// columns/rows c0.. of Tm (same layout); called by the whole workgroup.
template <class T>
__device__ void wy_factor_half(const T* Gm, T* Tm, const T* tau, int c0, int nh, double* Ts) {
  const int tid = threadIdx.x;
  for (int q = tid; q < kNBh * kNBh; q += kBackBlock) {
    const int c = q / kNBh, r = q - c * kNBh;
    // Ts[c*kNBh + r] = G(c0 + r, c0 + c) for r <= c (the only entries read
    // below), from G's lower triangle: G(c0 + c, c0 + r)
    Ts[q] = (r < nh && c < nh && r <= c) ? (double)Gm[(int64_t)(c0 + r) * kNBq + (c0 + c)] : 0.0;
  }
  __syncthreads();
  // column by column, in place over G: column c of G (rows < c) is read
  // before column c of T replaces it
  if (tid < kWave) {
    for (int c = 0; c < nh; ++c) {
      const double tc = (double)tau[c0 + c];
      double v = 0.0;
      if (tid < c) {
        for (int s2 = tid; s2 < c; ++s2) v = fma(Ts[s2 * kNBh + tid], Ts[c * kNBh + s2], v);
        v = -tc * v;
      }
      __builtin_amdgcn_wave_barrier();
      if (tid < c) Ts[c * kNBh + tid] = v;
      if (tid == c) Ts[c * kNBh + c] = tc;
      if (tid > c && tid < kNBh) Ts[c * kNBh + tid] = 0.0;
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int q = tid; q < kNBh * kNBh; q += kBackBlock) {
    const int c = q / kNBh, r = q - c * kNBh;
    if (r < nh && c < nh) Tm[(int64_t)(c0 + c) * kNBq + (c0 + r)] = (T)Ts[q];
  }
  __syncthreads();
}

template <class T>
__global__ __launch_bounds__(kBackBlock, kBackPerCU) void k_back_prep(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  __shared__ double Ts[kNBh * kNBh];
  const int tid = threadIdx.x;
  T* gsm = (T*)dyn;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (skip_item(a, it)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) continue;
    const T* S = at<T>((const void*)a.S, a.off[it]);
    T* VTs = at<T>(a.W, a.off[it]);
    const T* tau = at<T>((const void*)a.tau, a.voff[it]);
    // scratch (type T): G, T (kNBq x kNBq each), X (kNBh x kNBh)
    T* Gm = at<T>(a.escr, a.eoff[it]);
    T* Tm = Gm + kNBq * kNBq;
    T* Xm = Tm + kNBq * kNBq;
    const int nref = m - 2;
    for (int k0 = 0; k0 < nref; k0 += kNBq) {
      const int nbt = (nref - k0) < kNBq ? (nref - k0) : kNBq;
      const int n2 = m - k0 - 1;
      const int nh1 = nbt < kNBh ? nbt : kNBh, nh2 = nbt - nh1;
      const T* V = S + (int64_t)k0 * ld + (k0 + 1);
      // G = V^T V, lower tiles only (G is symmetric); V's zeros above each
      // vector's first entry are skipped
      wg_gemm<T, kBackNW, true, false, true, 1, 2, 2, 1, 1>(nbt, nbt, n2, T(1), V, ld, V, ld, T(0), Gm, kNBq, gsm);
      for (int q = tid; q < kNBq * kNBq; q += kBackBlock) Tm[q] = T(0);
      __syncthreads();
      wy_factor_half<T>(Gm, Tm, tau + k0, 0, nh1, Ts);
      if (nh2 > 0) {
        wy_factor_half<T>(Gm, Tm, tau + k0, kNBh, nh2, Ts);
        // T12 = -T1 (G12 T2): X = G12 T2, then T12 = -T1 X
        const T* G21 = Gm + kNBh;  // rows kNBh.., columns 0..: G12 = G21^T
        const T* T22 = Tm + (int64_t)kNBh * kNBq + kNBh;
        wg_gemm<T, kBackNW, true, false, false, 1>(nh1, nh2, nh2, T(1), G21, kNBq, T22, kNBq, T(0), Xm, kNBh, gsm);
        wg_gemm<T, kBackNW, false, false, false, 1>(nh1, nh2, nh1, T(-1), Tm, kNBq, Xm, kNBh, T(0),
                                                   Tm + (int64_t)kNBh * kNBq, kNBq, gsm);
      }
      // VT = V T^T (n2 x nbt) over V's position in the W slab: V(r, k) = 0
      // for r < k and T(j, k) = 0 for k < j, so VT(r, j) = 0 for r < j
      wg_gemm<T, kBackNW, false, true, false, 1, 2, 2, 2, 1>(n2, nbt, nbt, T(1), V, ld, Tm, kNBq, T(0),
                                                            VTs + (int64_t)k0 * ld + (k0 + 1), ld, gsm);
    }
  }
}

// Units u = it * ncb + cb over the items and their column blocks (ncb from
// the largest order; units past an item's order are skipped).
template <class T>
__global__ __launch_bounds__(kBackBlock, kBackPerCU) void k_back_apply(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  T* gsm = (T*)dyn;
  const int ncb = (a.max_m + kBackCols - 1) / kBackCols;
  const int nunits = a.n_items * ncb;
  int q = xcc_id();
  for (;;) {
    const int u = a.xcd_queues ? next_unit_xcd(a.work_ctr, a.n_items, ncb, &s_item, q)
                               : next_item(a.work_ctr, &s_item);
    if (u < 0 || u >= nunits) break;
    const int it = u / ncb, cb = u - it * ncb;
    if (skip_item(a, it)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) continue;
    const int c0 = cb * kBackCols;
    if (c0 >= m) continue;
    const int nc = (m - c0) < kBackCols ? (m - c0) : kBackCols;
    const T* S = at<T>((const void*)a.S, a.off[it]);
    const T* VTs = at<T>((const void*)a.W, a.off[it]);
    T* Q = at<T>(a.Q, a.qoff[it]) + (int64_t)c0 * ld;
    // this unit's columns of the kNBq x ld block product Wm
    T* Wm = at<T>(a.escr, a.eoff[it]) + 2 * kNBq * kNBq + kNBh * kNBh + (int64_t)c0 * kNBq;
    const int nref = m - 2;
    for (int t = (nref + kNBq - 1) / kNBq - 1; t >= 0; --t) {
      const int k0 = t * kNBq;
      const int nbt = (nref - k0) < kNBq ? (nref - k0) : kNBq;
      const int n2 = m - k0 - 1;
      const T* V = S + (int64_t)k0 * ld + (k0 + 1);
      const T* VT = VTs + (int64_t)k0 * ld + (k0 + 1);
      T* Qs = Q + (k0 + 1);
      // Wm = VT^T Q_sub (nbt x nc; one 128 x 64 tile, so Q_sub is read once), Q_sub -= V Wm;
      // the zeros of VT(r, j) (r < j) and V(r, k) (r < k) are skipped
      wg_gemm<T, kBackNW, true, false, false, 1, 4, 2, 1, 0>(nbt, nc, n2, T(1), VT, ld, Qs, ld, T(0), Wm, kNBq, gsm);
      wg_gemm<T, kBackNW, false, false, false, 1, 2, 2, 2, 0>(n2, nc, nbt, T(-1), V, ld, Wm, kNBq, T(1), Qs, ld, gsm);
    }
  }
}

// ------------------------------------------------------- apply column
// x[r] = sum_p Q[r][p] f(lambda_p) Q[c][p]; NaN when lambda_min <= 0 or the
// eigensolver did not converge.
template <class T, class VT>
__global__ __launch_bounds__(kBlock) void k_apply_column(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  double* wv = dyn;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (skip_item(a, it)) continue;
    const int fl = a.flags[it];
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) {
      for (int r = tid; r < m; r += kBlock) ((VT*)a.x)[a0 + r] = (VT)NAN;
      if (tid == 0) atomicAdd((unsigned long long*)&a.status[ST_STALE], 1ull);
      continue;
    }
    const int c = a.cidx[j];
    const T* Q = at<T>((const void*)a.Q, a.qoff[it]);
    const T* lam = at<T>((const void*)a.d, a.doff[it]);
    const bool bad = (fl & (LF_NONPOS | LF_UNCONV)) != 0;
    for (int q = tid; q < m; q += kBlock) wv[q] = spec_f((double)lam[q], a.fn) * (double)Q[(int64_t)q * ld + c];
    __syncthreads();
    VT* x = (VT*)a.x + a0;
    for (int r = tid; r < m; r += kBlock) {
      double s = 0.0;
      for (int q = 0; q < m; ++q) s = fma((double)Q[(int64_t)q * ld + r], wv[q], s);
      x[r] = bad ? (VT)NAN : (VT)s;
    }
    if (tid == 0) atomicAdd((unsigned long long*)&a.status[ST_DONE], 1ull);
  }
}

// -------------------------------------------- column from the factors
// Forward without the eigenvector matrix: with Q = Q1 Z and Q1 = H_0 ...
// H_{m-3}, the column is
//   x = Q1 (Z (f(lambda) o (Z^T (Q1^T e_c)))),
// O(m^2) work per submatrix instead of forming Q (2 m^3). One wavefront per
// submatrix; lane l holds the vector's rows l, l + 64, ... in registers.
// Each reflector H_k = I - tau_k v_k v_k^T (v_k in column k of the S slab,
// zero above row k + 1, 1 at row k + 1, zero below row m) costs one wave
// reduction; Z^T u takes the columns of Z eight at a time (one coalesced
// load per column per row group, the strip reduction of the symv), Z y
// walks the columns of Z with y broadcast from LDS.
constexpr int kColWavesPerCU = 16;

// u <- H_k u for one reflector (orders above 16 * 64: the prefetching loop
// below would hold three 32-element vectors per lane)
template <class T, int NPL>
__device__ __forceinline__ void apply_reflector(const T* __restrict__ v, double tk, int m, int lane, double (&u)[NPL]) {
  double d = 0.0;
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    const int r = lane + kWave * i;
    if (r < m) d = fma((double)v[r], u[i], d);
  }
  d = tk * wave_sum(d);
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    const int r = lane + kWave * i;
    if (r < m) u[i] = fma(-d, (double)v[r], u[i]);
  }
}

// u <- H_k u for k = k0, k0 + dk, ..., k1 (inclusive, dk = +1 or -1), each
// H_k = I - tau_k v_k v_k^T with v_k in column k of V (leading dimension ld,
// rows >= m never read). Up to 16 rows per lane the next reflector's column
// is loaded while the current one's dot product is reduced.
template <class T, int NPL>
__device__ __forceinline__ void apply_reflectors(const T* __restrict__ V, const T* __restrict__ tau, int ld, int m,
                                                 int k0, int k1, int dk, int lane, double (&u)[NPL]) {
  if ((k1 - k0) * dk < 0) return;
  if constexpr (NPL > 16) {
    for (int k = k0;; k += dk) {
      apply_reflector<T, NPL>(V + (int64_t)k * ld, (double)tau[k], m, lane, u);
      if (k == k1) break;
    }
    return;
  }
  double vn[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    const int r = lane + kWave * i;
    vn[i] = r < m ? (double)V[(int64_t)k0 * ld + r] : 0.0;
  }
  double tn = (double)tau[k0];
  for (int k = k0;; k += dk) {
    double v[NPL];
#pragma unroll
    for (int i = 0; i < NPL; ++i) v[i] = vn[i];
    const double tk = tn;
    const bool more = k != k1;
    if (more) {
      const T* vc = V + (int64_t)(k + dk) * ld;
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        const int r = lane + kWave * i;
        vn[i] = r < m ? (double)vc[r] : 0.0;
      }
      tn = (double)tau[k + dk];
    }
    double d = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) d = fma(v[i], u[i], d);
    d = tk * wave_sum(d);
#pragma unroll
    for (int i = 0; i < NPL; ++i) u[i] = fma(-d, v[i], u[i]);
    if (!more) break;
  }
}

template <class T, class VT, int NPL>
__global__ __launch_bounds__(kWave) void k_column_factored(LargeArgs a) {
  extern __shared__ double cdyn[];
  __shared__ int s_item;
  const int lane = threadIdx.x;
  const int pl = strip_perm(lane);
  double* yv = cdyn;  // max_m: f(lambda) o (Z^T Q1^T e_c)
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (skip_item(a, it)) continue;
    const int fl = a.flags[it];
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    VT* x = (VT*)a.x + a0;
    if (order_mismatch(a, m, ld) || m > NPL * kWave) {
      for (int r = lane; r < m; r += kWave) x[r] = (VT)NAN;
      if (lane == 0) atomicAdd((unsigned long long*)&a.status[ST_STALE], 1ull);
      continue;
    }
    const int c = a.cidx[j];
    const T* V = at<T>((const void*)a.S, a.off[it]);
    const T* Z = at<T>((const void*)a.Q, a.qoff[it]);
    const T* tau = at<T>((const void*)a.tau, a.voff[it]);
    const T* lam = at<T>((const void*)a.d, a.doff[it]);
    const bool bad = (fl & (LF_NONPOS | LF_UNCONV)) != 0;
    double u[NPL];
#pragma unroll
    for (int i = 0; i < NPL; ++i) u[i] = (lane + kWave * i == c) ? 1.0 : 0.0;
    // u = Q1^T e_c = H_{m-3} ... H_0 e_c
    apply_reflectors<T, NPL>(V, tau, ld, m, 0, m - 3, 1, lane, u);
    // y = f(lambda) o (Z^T u), eight columns of Z per pass
    for (int j0 = 0; j0 < m; j0 += kStrip) {
      double cd[kStrip];
#pragma unroll
      for (int s2 = 0; s2 < kStrip; ++s2) cd[s2] = 0.0;
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        const int r = lane + kWave * i;
        if (r < m) {
#pragma unroll
          for (int s2 = 0; s2 < kStrip; ++s2) {
            const int col = j0 + (s2 ^ pl);
            cd[s2] = fma(col < m ? (double)Z[(int64_t)col * ld + r] : 0.0, u[i], cd[s2]);
          }
        }
      }
      const double tot = wave_strip_sum(cd);
      const int col = j0 + pl;
      if ((lane & (kWave / kStrip - 1)) == 0 && col < m) yv[col] = spec_f((double)lam[col], a.fn) * tot;
    }
    __syncthreads();
    // u = Z y
#pragma unroll
    for (int i = 0; i < NPL; ++i) u[i] = 0.0;
    for (int jj = 0; jj < m; ++jj) {
      const double yj = yv[jj];
      const T* zc = Z + (int64_t)jj * ld;
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        const int r = lane + kWave * i;
        if (r < m) u[i] = fma((double)zc[r], yj, u[i]);
      }
    }
    // x = Q1 u = H_0 ... H_{m-3} u
    apply_reflectors<T, NPL>(V, tau, ld, m, m - 3, 0, -1, lane, u);
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int r = lane + kWave * i;
      if (r < m) x[r] = bad ? (VT)NAN : (VT)u[i];
    }
    if (lane == 0) atomicAdd((unsigned long long*)&a.status[ST_DONE], 1ull);
    __syncthreads();
  }
}

// --------------------------------------------------------------- adjoint
// a = Q^T w, b = Q[c,:]^T, Ms = (G o (a b^T + b a^T))/2, T1 = Q Ms,
// D = T1 Q^T (lower tiles; D is symmetric), then every stored pair
// (R[k], R[l]) at position q receives D[max(k,l)][min(k,l)].
// Four kernels: k_adj_prep per item (a = Q^T w, b = Q[c, :]^T and Ms in the
// S slab), then two products over (item, kBackCols columns) units, which
// read the item's whole Q (or T1) from the caches while each writes only its
// own columns: T1 = Q Ms into the W slab, D = T1 Q^T (lower part) into the
// S slab; k_adj_scatter last, per item, adds D into grad_a (or, in the
// deterministic mode, copies it to FP64 in the W slab).
template <class T, class VT, bool POW>
__global__ __launch_bounds__(kAdjBlock, kAdjPerCU) void k_adj_prep(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  double* w = dyn;
  double* av = w + a.max_m;
  double* bv = av + a.max_m;
  double* alv = bv + a.max_m;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (skip_item(a, it)) continue;
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) {
      for (int r = tid; r < m; r += kAdjBlock) atomicAdd(&((VT*)a.ga)[a0 + r], (VT)NAN);
      if (tid == 0) atomicAdd((unsigned long long*)&a.status[ST_STALE], 1ull);
      continue;
    }
    const int c = a.cidx[j];
    const T* Q = at<T>((const void*)a.Q, a.qoff[it]);
    T* Ms = at<T>(a.S, a.off[it]);
    const T* lam = at<T>((const void*)a.d, a.doff[it]);
    const VT* gx = (const VT*)a.gx + a0;
    for (int i = tid; i < m; i += kAdjBlock) {
      w[i] = (double)gx[i];
      bv[i] = (double)Q[(int64_t)i * ld + c];
      alv[i] = spec_node((double)lam[i], a.fn);
    }
    __syncthreads();
    // a = Q^T w, a wave per column of Q; four row groups' loads issued
    // together (unconditional: rows past m read row m - 1, masked)
    for (int pc = wv; pc < m; pc += kAdjNW) {
      const T* qc = Q + (int64_t)pc * ld;
      double part = 0.0;
      for (int r0 = lane; r0 < m; r0 += 4 * kWave) {
        double qv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + u * kWave;
          qv[u] = (double)qc[r < m ? r : m - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + u * kWave;
          if (r < m) part = fma(qv[u], w[r], part);
        }
      }
      part = wave_sum(part);
      if (lane == 0) av[pc] = part;
    }
    __syncthreads();
    if (POW) {  // lambda^alpha per eigenvalue, into w (no longer needed)
      for (int i = tid; i < m; i += kAdjBlock) w[i] = pow(alv[i], a.fn.alpha);
      __syncthreads();
    }
    for (int l = wv; l < m; l += kAdjNW) {
      const double pwl = POW ? w[l] : 0.0;
      for (int pr = lane; pr < m; pr += kWave) {
        const double g = spec_divdiff<POW>(alv[pr], alv[l], pwl, a.fn);
        Ms[(int64_t)l * ld + pr] = (T)(0.5 * g * (av[pr] * bv[l] + av[l] * bv[pr]));
      }
    }
    __syncthreads();
  }
}

// LOWER = false: T1[:, c0:c0+nc] = Q Ms[:, c0:c0+nc] into the W slab;
// LOWER = true:  D[c0:, c0:c0+nc] = T1[c0:, :] Q[c0:c0+nc, :]^T into the S slab
// (the tiles of the block that meet the lower triangle).
template <class T, bool LOWER>
__global__ __launch_bounds__(kAdjBlock, kAdjPerCU) void k_adj_product(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  T* gsm = (T*)dyn;
  const int ncb = (a.max_m + kBackCols - 1) / kBackCols;
  const int nunits = a.n_items * ncb;
  int q = xcc_id();
  for (;;) {
    const int u = a.xcd_queues ? next_unit_xcd(a.work_ctr, a.n_items, ncb, &s_item, q)
                               : next_item(a.work_ctr, &s_item);
    if (u < 0 || u >= nunits) break;
    const int it = u / ncb, cb = u - it * ncb;
    if (skip_item(a, it)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) continue;
    const int c0 = cb * kBackCols;
    if (c0 >= m) continue;
    const int nc = (m - c0) < kBackCols ? (m - c0) : kBackCols;
    const T* Q = at<T>((const void*)a.Q, a.qoff[it]);
    T* Ms = at<T>(a.S, a.off[it]);
    T* T1 = at<T>(a.W, a.off[it]);
    if (!LOWER)
      wg_gemm<T, kAdjNW, false, false, false, 1, 4, 2>(m, nc, m, T(1), Q, ld, Ms + (int64_t)c0 * ld, ld, T(0),
                                                 T1 + (int64_t)c0 * ld, ld, gsm);
    else
      wg_gemm<T, kAdjNW, false, true, true, 1, 4, 2>(m - c0, nc, m, T(1), T1 + c0, ld, Q + c0, ld, T(0),
                                               Ms + (int64_t)c0 * ld + c0, ld, gsm);
  }
}

template <class T, class VT>
__global__ __launch_bounds__(kAdjBlock, kAdjPerCU) void k_adj_scatter(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  int* R = (int*)dyn;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (skip_item(a, it)) continue;
    const int fl = a.flags[it];
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    if (order_mismatch(a, m, ld)) continue;
    const T* Ms = at<T>((const void*)a.S, a.off[it]);
    const bool bad = (fl & (LF_NONPOS | LF_UNCONV)) != 0;
    if (a.det) {
      // deterministic mode: D (lower triangle, FP64) into this item's W slot
      // (T1 is dead), assembled afterwards in a fixed order
      double* D64 = at<double>(a.W, a.off[it]);
      for (int lo = wv; lo < m; lo += kAdjNW)
        for (int hi = lo + lane; hi < m; hi += kWave)
          D64[(int64_t)lo * ld + hi] = bad ? (double)NAN : (double)Ms[(int64_t)lo * ld + hi];
      if (tid == 0) atomicAdd((unsigned long long*)&a.status[ST_DONE], 1ull);
      continue;
    }
    for (int i = tid; i < m; i += kAdjBlock) R[i] = a.colind[a0 + i];
    __syncthreads();
    VT* ga = (VT*)a.ga;
    // the lower triangle only (column <= row); the upper entries receive
    // their lower mirror's sum after the last phase
    for (int k = wv; k < m; k += kAdjNW) {
      const int r = R[k];
      const int s0 = a.rowptr[r], s1 = a.rowptr[r + 1];
      // four entries per lane and step, their column indices loaded together
      // (entries past the row's end read its last one and are skipped)
      for (int q0 = s0 + lane; q0 < s1; q0 += 4 * kWave) {
        int cq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q0 + u * kWave;
          cq[u] = a.colind[q < s1 ? q : s1 - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q0 + u * kWave;
          if (q < s1 && cq[u] <= r) {
            const int l = find_sorted(R, m, cq[u]);
            if (l >= 0) {
              const int hi = l > k ? l : k, lo = l > k ? k : l;
              atomicAdd(&ga[q], bad ? (VT)NAN : (VT)Ms[(int64_t)lo * ld + hi]);
            }
          }
        }
        if (cq[3] > r) break;  // the row is sorted: the rest lies above the diagonal
      }
    }
    if (tid == 0) atomicAdd((unsigned long long*)&a.status[ST_DONE], 1ull);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launch
static size_t vec_lds(const LargeArgs& a, int nvec, size_t elt) { return (size_t)nvec * a.max_m * elt; }

#define SUBMAT_VT_SWITCH(VTYPE, ...)  \
  do {                                \
    if ((VTYPE) == 0) {               \
      using VT = double;              \
      __VA_ARGS__;                    \
    } else {                          \
      using VT = float;               \
      __VA_ARGS__;                    \
    }                                 \
  } while (0)

hipError_t launch_gather_large(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const size_t lds = ((size_t)(a.max_m + 1) / 2 + (size_t)kNW * a.max_m) * sizeof(double);
  if ((int64_t)lds > a.lds_limit) return hipErrorInvalidValue;
  if (a.fp64) {
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_gather_large<double, VT>), dim3(a.grid), dim3(kBlock), lds, s, a));
  } else {
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_gather_large<float, VT>), dim3(a.grid), dim3(kBlock), lds, s, a));
  }
  return hipGetLastError();
}

int back_blocks_per_cu() { return kBackPerCU; }
int adjoint_blocks_per_cu() { return kAdjPerCU; }

// static LDS of k_tridiagonalise (block_sum scratch, the next column's
// coefficients, panel dots) plus a margin
constexpr size_t kTridiagStaticLds = 4096;

// Rows of the LDS panel copy that a workgroup's share of the LDS holds, with
// per_cu workgroups per compute unit (negative: the fixed part alone does
// not fit that share), up to the largest order.
static int reduction_panel_rows(int max_m, int nb, int fp64, int64_t lds_limit, int per_cu) {
  const size_t part = (size_t)kRedNW * max_m * 8;
  const size_t gemm = fp64 ? gemm_lds_elems<kRedNW>() * sizeof(double) : gemm_lds_elems<kRedNW>() * sizeof(float);
  const size_t base = (size_t)max_m * 8 + (part > gemm ? part : gemm);
  const int64_t left = lds_limit / per_cu - (int64_t)base - (int64_t)kTridiagStaticLds;
  if (left < 0) return -1;
  const int64_t rows = left / (2 * (nb + 1) * (int64_t)sizeof(double));
  return (int)(rows < max_m ? rows : max_m);
}

int reduction_fit_per_cu(int max_m, int nb, int fp64, int64_t lds_limit, int per_cu) {
  // fewer workgroups per compute unit until each one's share of the LDS
  // also holds one panel width of rows of the panel copy (more would not be
  // resident together anyway, and would only cost registers)
  while (per_cu > 1 && reduction_panel_rows(max_m, nb, fp64, lds_limit, per_cu) < std::min(nb, max_m)) --per_cu;
  return per_cu;
}

template <class T, int PERCU>
static void launch_tridiag_t(const LargeArgs& a0, hipStream_t s) {
  LargeArgs a = a0;
  const int pld = a.nb + 1;
  const size_t part = vec_lds(a, kRedNW, 8), gemm = gemm_lds_elems<kRedNW>() * sizeof(T);
  const size_t base = vec_lds(a, 1, 8) + (part > gemm ? part : gemm);
  // the panel copy takes what is left of the workgroup's share of the LDS
  // (PERCU workgroups per compute unit), up to the largest order
  int rows = reduction_panel_rows(a.max_m, a.nb, a.fp64, a.lds_limit, PERCU);
  if (rows < 0) rows = 0;
  a.panel_rows = rows;
  a.panel_off = (int)((part > gemm ? part : gemm) / sizeof(double));
  const size_t lds = base + (size_t)rows * 2 * pld * sizeof(double);
  hipLaunchKernelGGL((k_tridiagonalise<T, PERCU>), dim3(a.grid), dim3(kRedBlock), lds, s, a);
}

hipError_t launch_tridiagonalise(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.nb < 2 || a.nb > kNBMax || (a.nb & 1) || a.red_per_cu < 1 || a.red_per_cu > 4) return hipErrorInvalidValue;
  if (reduction_fit_per_cu(a.max_m, a.nb, a.fp64, a.lds_limit, a.red_per_cu) != a.red_per_cu)
    return hipErrorInvalidValue;  // the caller sizes the grid for the value that fits
  if (a.fp64) {
    switch (a.red_per_cu) {
      case 1: launch_tridiag_t<double, 1>(a, s); break;
      case 2: launch_tridiag_t<double, 2>(a, s); break;
      case 3: launch_tridiag_t<double, 3>(a, s); break;
      default: launch_tridiag_t<double, 4>(a, s); break;
    }
  } else {
    switch (a.red_per_cu) {
      case 1: launch_tridiag_t<float, 1>(a, s); break;
      case 2: launch_tridiag_t<float, 2>(a, s); break;
      case 3: launch_tridiag_t<float, 3>(a, s); break;
      default: launch_tridiag_t<float, 4>(a, s); break;
    }
  }
  return hipGetLastError();
}

size_t eig_lds_bytes(int max_m) { return (size_t)max_m * (4 * sizeof(double) + 2 * sizeof(int)); }

hipError_t launch_tridiag_eig(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const size_t lds = eig_lds_bytes(a.max_m);
  if ((int64_t)lds + 2048 > a.lds_limit) return hipErrorInvalidConfiguration;
  if (a.fp64)
    hipLaunchKernelGGL(k_tridiag_eig<double>, dim3(a.grid), dim3(kEigBlock), lds, s, a);
  else
    hipLaunchKernelGGL(k_tridiag_eig<float>, dim3(a.grid), dim3(kEigBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_eig_orth(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.fp64)
    hipLaunchKernelGGL(k_eig_orth<double>, dim3(a.grid), dim3(kEigBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_eig_orth<float>, dim3(a.grid), dim3(kEigBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_back_prep(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.fp64)
    hipLaunchKernelGGL(k_back_prep<double>, dim3(a.grid), dim3(kBackBlock), gemm_lds_elems<kBackNW>() * 8, s, a);
  else
    hipLaunchKernelGGL(k_back_prep<float>, dim3(a.grid), dim3(kBackBlock), gemm_lds_elems<kBackNW>() * 4, s, a);
  return hipGetLastError();
}

hipError_t launch_back_apply(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if ((int64_t)a.n_items * ((a.max_m + kBackCols - 1) / kBackCols) > INT32_MAX) return hipErrorInvalidValue;
  if (a.fp64)
    hipLaunchKernelGGL(k_back_apply<double>, dim3(a.grid), dim3(kBackBlock), (gemm_lds_elems<kBackNW, 4, 2>() * 8), s, a);
  else
    hipLaunchKernelGGL(k_back_apply<float>, dim3(a.grid), dim3(kBackBlock), (gemm_lds_elems<kBackNW, 4, 2>() * 4), s, a);
  return hipGetLastError();
}

int back_apply_units(int n_items, int max_m) { return n_items * ((max_m + kBackCols - 1) / kBackCols); }

hipError_t launch_apply_column(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const size_t lds = vec_lds(a, 1, 8);
  if (a.fp64) {
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_apply_column<double, VT>), dim3(a.grid), dim3(kBlock), lds, s, a));
  } else {
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_apply_column<float, VT>), dim3(a.grid), dim3(kBlock), lds, s, a));
  }
  return hipGetLastError();
}

template <class T, class VT>
static void dispatch_column_factored(const LargeArgs& a, size_t lds, hipStream_t s) {
  if (a.max_m <= 8 * kWave)
    hipLaunchKernelGGL((k_column_factored<T, VT, 8>), dim3(a.grid), dim3(kWave), lds, s, a);
  else if (a.max_m <= 16 * kWave)
    hipLaunchKernelGGL((k_column_factored<T, VT, 16>), dim3(a.grid), dim3(kWave), lds, s, a);
  else
    hipLaunchKernelGGL((k_column_factored<T, VT, 32>), dim3(a.grid), dim3(kWave), lds, s, a);
}

int column_waves_per_cu() { return kColWavesPerCU; }

hipError_t launch_column_factored(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.max_m > 32 * kWave) return hipErrorInvalidValue;
  const size_t lds = vec_lds(a, 1, 8);
  if (a.fp64) {
    SUBMAT_VT_SWITCH(a.vdtype, (dispatch_column_factored<double, VT>(a, lds, s)));
  } else {
    SUBMAT_VT_SWITCH(a.vdtype, (dispatch_column_factored<float, VT>(a, lds, s)));
  }
  return hipGetLastError();
}

template <class T, bool POW>
static void dispatch_adj_prep(const LargeArgs& a, size_t lds, hipStream_t s) {
  SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_adj_prep<T, VT, POW>), dim3(a.grid), dim3(kAdjBlock), lds, s, a));
}

hipError_t launch_adjoint_prep(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const size_t lds = vec_lds(a, 4, 8);
  const bool pw = a.fn.kind == FN_POWER;
  if (a.fp64)
    pw ? dispatch_adj_prep<double, true>(a, lds, s) : dispatch_adj_prep<double, false>(a, lds, s);
  else
    pw ? dispatch_adj_prep<float, true>(a, lds, s) : dispatch_adj_prep<float, false>(a, lds, s);
  return hipGetLastError();
}

hipError_t launch_adjoint_product(const LargeArgs& a, int lower, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if ((int64_t)a.n_items * ((a.max_m + kBackCols - 1) / kBackCols) > INT32_MAX) return hipErrorInvalidValue;
  if (a.fp64) {
    if (lower)
      hipLaunchKernelGGL((k_adj_product<double, true>), dim3(a.grid), dim3(kAdjBlock), (gemm_lds_elems<kAdjNW, 4, 2>() * 8), s, a);
    else
      hipLaunchKernelGGL((k_adj_product<double, false>), dim3(a.grid), dim3(kAdjBlock), (gemm_lds_elems<kAdjNW, 4, 2>() * 8), s, a);
  } else {
    if (lower)
      hipLaunchKernelGGL((k_adj_product<float, true>), dim3(a.grid), dim3(kAdjBlock), (gemm_lds_elems<kAdjNW, 4, 2>() * 4), s, a);
    else
      hipLaunchKernelGGL((k_adj_product<float, false>), dim3(a.grid), dim3(kAdjBlock), (gemm_lds_elems<kAdjNW, 4, 2>() * 4), s, a);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_scatter(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const size_t lds = (size_t)a.max_m * sizeof(int);
  if (a.fp64) {
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_adj_scatter<double, VT>), dim3(a.grid), dim3(kAdjBlock), lds, s, a));
  } else {
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_adj_scatter<float, VT>), dim3(a.grid), dim3(kAdjBlock), lds, s, a));
  }
  return hipGetLastError();
}

}  // namespace submat
