// Large-order path (m > 64): one workgroup per submatrix for the dense
// stages, one lane per submatrix for the tridiagonal QL iteration.
//
//   gather      S_j from CSR into an HBM slab (Section 3.1), symmetrised
//   tridiag     blocked Householder reduction S = Q1 T Q1^T (lower form): per
//               panel of NB columns a row-parallel symv per column, and one
//               rank-2*NB trailing update on MFMA
//   form_q1     Q1 accumulated explicitly from compact-WY blocks of NB
//               reflectors, products on MFMA
//   ql          implicit QL with Wilkinson shifts on T (d, e in LDS); the
//               eigenvalues replace d and every plane rotation is recorded,
//               sweep by sweep
//   rotations   Q = Q1 * (all rotations): each thread owns a row of Q and
//               applies a batch of K sweeps in one pass over it (sweep s lags
//               sweep s-1 by two columns, so a window of 2K values suffices);
//               rotation coefficients are staged in LDS tables
//   column      x = Q (f(lambda) o Q[c,:]^T) into X's value segment
//               (Sections 3.3-3.4)
//   adjoint     D = Q sym(G o (a b^T)) Q^T on MFMA, scattered into dA's
//               stored pairs
//
// Slabs are column-major with leading dimension ldm (the order rounded up
// to a multiple of 16). After the reduction column k of the S slab holds the
// full Householder vector v_k (zeros above row k+1, 1 at row k+1).
#include <math.h>

#include "common.hpp"
#include "gemm.hpp"
#include "kernels.hpp"

namespace submat {

constexpr int kBlock = 256;
constexpr int kNW = kBlock / kWave;
constexpr int kBigBlock = 512;
constexpr int kBigNW = kBigBlock / kWave;
constexpr int kNB = 32;  // panel width of the reduction and of the WY blocks

template <class T> __device__ __forceinline__ T* at(void* base, int64_t off_bytes) {
  return (T*)((char*)base + off_bytes);
}
template <class T> __device__ __forceinline__ const T* at(const void* base, int64_t off_bytes) {
  return (const T*)((const char*)base + off_bytes);
}

__device__ __forceinline__ bool skip_item(const LargeArgs& a, int it) {
  const int fl = a.flags[it];
  if (a.only_flagged) return !(fl & LF_FALLBACK);
  return !a.fp64 && (fl & LF_FALLBACK);  // the FP32 pass leaves flagged items to FP64
}

// ---------------------------------------------------------------- gather
template <class T, class VT>
__global__ __launch_bounds__(kBlock) void k_gather_large(LargeArgs a) {
  extern __shared__ int R[];  // max_m ints
  __shared__ int s_item;
  const VT* vals = (const VT*)a.vals;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    T* S = at<T>(a.S, a.off[it]);
    for (int i = tid; i < m; i += kBlock) R[i] = a.colind[a0 + i];
    const int64_t tot = (int64_t)ld * ld;
    for (int64_t q = tid; q < tot; q += kBlock) S[q] = T(0);
    __syncthreads();
    for (int k = wv; k < m; k += kNW) {
      const int r = R[k];
      const int s0 = a.rowptr[r], s1 = a.rowptr[r + 1];
      for (int q = s0 + lane; q < s1; q += kWave) {
        const int l = find_sorted(R, m, a.colind[q]);
        if (l >= 0) S[(int64_t)l * ld + k] = (T)vals[q];
      }
    }
    __syncthreads();
    // (S + S^T)/2: wave w owns columns l = w, w+NW, ..., lanes run over k > l
    for (int l = wv; l < m; l += kNW) {
      for (int k = l + 1 + lane; k < m; k += kWave) {
        const T t = T(0.5) * (S[(int64_t)l * ld + k] + S[(int64_t)k * ld + l]);
        S[(int64_t)l * ld + k] = t;
        S[(int64_t)k * ld + l] = t;
      }
    }
  }
}

// ------------------------------------------------------- symmetric matvec
// y = A v for a symmetric n x n matrix given by its lower triangle (column
// major, leading dimension ld), v and y in LDS, called by the whole
// 512-thread workgroup. The columns are cut into strips of kStrip; wave w
// takes strips w, 2*NW-1-w, 2*NW+w, ... (balanced over the triangle). For a
// strip the lanes run down the rows r >= c0 in groups of 64; each lane loads
// kStrip elements of its row (one coalesced column segment per load) and
//   * adds sum_c A[r][c] v[c] to its wave's row partial spart[w][r];
//   * accumulates A[r][c] v[r] (r > c) for each of the strip's columns,
//     reduced across the wave at the end of the strip.
// y = sum over waves of the partials, in a fixed order (deterministic).
constexpr int kStrip = 8;

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

template <class T>
__device__ void symv_lower(const T* __restrict__ A, int ld, int n, const double* __restrict__ v,
                           double* y, double* spart, int max_m) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int pl = strip_perm(lane);
  double* my = spart + (int64_t)wv * max_m;
  for (int r = lane; r < n; r += kWave) my[r] = 0.0;
  const int nstrip = (n + kStrip - 1) / kStrip;
  for (int t = 0;; ++t) {
    const int s = t * kBigNW + ((t & 1) ? (kBigNW - 1 - wv) : wv);
    if (s >= nstrip) break;
    const int c0 = s * kStrip;
    double vc[kStrip], cd[kStrip];
    const T* col[kStrip];
#pragma unroll
    for (int u = 0; u < kStrip; ++u) {
      const int c = c0 + (u ^ pl);
      vc[u] = (c < n) ? v[c] : 0.0;
      cd[u] = 0.0;
      col[u] = A + (int64_t)(c < n ? c : c0) * ld;
    }
    for (int r = c0 + lane; r - lane < n; r += kWave) {
      const bool in = r < n;
      double av[kStrip];
#pragma unroll
      for (int u = 0; u < kStrip; ++u) av[u] = (in && c0 + (u ^ pl) < n) ? (double)col[u][r] : 0.0;
      const double vr = in ? v[r] : 0.0;
      double racc = 0.0;
      if (r - lane >= c0 + kStrip) {  // the whole group lies below the diagonal block
#pragma unroll
        for (int u = 0; u < kStrip; ++u) {
          racc = fma(av[u], vc[u], racc);
          cd[u] = fma(av[u], vr, cd[u]);
        }
      } else {
#pragma unroll
        for (int u = 0; u < kStrip; ++u) {
          const int c = c0 + (u ^ pl);
          const double a_ = (r >= c) ? av[u] : 0.0;
          racc = fma(a_, vc[u], racc);
          cd[u] = fma((r > c) ? a_ : 0.0, vr, cd[u]);
        }
      }
      if (in) my[r] += racc;
    }
    const double tot = wave_strip_sum(cd);
    if ((lane & (kWave / kStrip - 1)) == 0 && c0 + pl < n) my[c0 + pl] += tot;
  }
  __syncthreads();
  // y may alias row 0 of spart: each thread reads and writes only its own r
  for (int r = tid; r < n; r += kBigBlock) {
    double acc = spart[r];
#pragma unroll
    for (int w = 1; w < kBigNW; ++w) acc += spart[(int64_t)w * max_m + r];
    y[r] = acc;
  }
}

// ------------------------------------------------------- tridiagonalise
// Blocked Householder reduction (lower form), panel width NB. Within a
// panel, column k = k0 + i is first brought up to date with the panel's
// earlier vectors (A[k:, k] -= V W[k,:]^T + W V[k,:]^T), its reflector
// (v, tau, beta) is formed, and w = tau (A22 v - V (W^T v) - W (V^T v)),
// w -= (tau/2)(w.v) v, where A22 is the trailing matrix as it stood at the
// start of the panel. After the panel, A22 -= V W^T + W V^T on MFMA over
// the tiles that meet the lower triangle; only the lower triangle is read.
// Outputs: d[0..m), e[0..m-1), tau[0..m-2) and v_k in column k of S.
template <class T>
__global__ __launch_bounds__(kBigBlock) void k_tridiagonalise(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  __shared__ double red[kBigNW];
  __shared__ double vk[kNB], wk[kNB], z1[kNB], z2[kNB];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  // LDS: v, then one region shared by the symv's per-wave row partials
  // (kBigNW rows of max_m; row 0 becomes y = A22 v) and, during the trailing
  // update only, the GEMM staging tiles
  double* sv = dyn;
  double* spart = dyn + a.max_m;
  double* sy = spart;
  T* gsm = (T*)spart;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    T* S = at<T>(a.S, a.off[it]);
    T* Wb = at<T>(a.W, a.off[it]);  // W: column c at Wb + c*ld, rows indexed globally
    T* d = at<T>(a.d, a.doff[it]);
    T* e = at<T>(a.e, a.voff[it]);
    T* tau = at<T>(a.tau, a.voff[it]);
    for (int k0 = 0; k0 + 2 < m; k0 += kNB) {
      const int nbt = (m - 2 - k0) < kNB ? (m - 2 - k0) : kNB;
      for (int i = 0; i < nbt; ++i) {
        const int k = k0 + i;
        const int n2 = m - k - 1;
        // (1) bring column k (rows k..m-1) up to date with the panel's vectors
        if (i > 0) {
          if (tid < i) {
            vk[tid] = (double)S[(int64_t)(k0 + tid) * ld + k];
            wk[tid] = (double)Wb[(int64_t)tid * ld + k];
          }
          __syncthreads();
          for (int r = k + tid; r < m; r += kBigBlock) {
            double acc = (double)S[(int64_t)k * ld + r];
#pragma unroll 1
            for (int c = 0; c < i; ++c)
              acc -= (double)S[(int64_t)(k0 + c) * ld + r] * wk[c] + (double)Wb[(int64_t)c * ld + r] * vk[c];
            S[(int64_t)k * ld + r] = (T)acc;
          }
          __syncthreads();
        }
        // (2) reflector from x = A[k+1:, k]
        T* x = S + (int64_t)k * ld + (k + 1);
        double part = 0.0;
        for (int q = 1 + tid; q < n2; q += kBigBlock) part += (double)x[q] * (double)x[q];
        const double alpha = (double)x[0];   // read before the barrier: x[0] is overwritten below
        const double dkk = (double)S[(int64_t)k * ld + k];
        const double sigma = block_sum<kBigNW>(part, red);
        double beta, tk, scale;
        if (sigma == 0.0) {
          beta = alpha; tk = 0.0; scale = 0.0;
        } else {
          const double nrm = sqrt(alpha * alpha + sigma);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tk = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        for (int q = tid; q < n2; q += kBigBlock) {
          const double vq = (q == 0) ? 1.0 : (double)x[q] * scale;
          sv[q] = vq;
          x[q] = (T)vq;
        }
        if (tid == 0) {
          d[k] = (T)dkk;
          e[k] = (T)beta;
          tau[k] = (T)tk;
        }
        __syncthreads();
        // column k above row k+1 becomes the zero part of v_k
        for (int q = tid; q <= k; q += kBigBlock) S[(int64_t)k * ld + q] = T(0);
        // (3) y = A22 v, A22 = the trailing matrix as it stood at the start
        // of the panel, lower triangle only: every element is read once and
        // serves both y[r] += A[r][c] v[c] and y[c] += A[r][c] v[r].
        symv_lower(S + (int64_t)(k + 1) * ld + (k + 1), ld, n2, sv, sy, spart, a.max_m);
        __syncthreads();
        // (4) y -= V (W^T v) + W (V^T v) over the panel's earlier vectors
        if (i > 0) {
          for (int c = wv; c < i; c += kBigNW) {
            const T* vc = S + (int64_t)(k0 + c) * ld + (k + 1);
            const T* wc = Wb + (int64_t)c * ld + (k + 1);
            double p1 = 0.0, p2 = 0.0;
#pragma unroll 1
            for (int r = lane; r < n2; r += kWave) {
              p1 = fma((double)wc[r], sv[r], p1);
              p2 = fma((double)vc[r], sv[r], p2);
            }
            p1 = wave_sum(p1);
            p2 = wave_sum(p2);
            if (lane == 0) {
              z1[c] = p1;
              z2[c] = p2;
            }
          }
          __syncthreads();
          for (int r = tid; r < n2; r += kBigBlock) {
            double acc = sy[r];
#pragma unroll 1
            for (int c = 0; c < i; ++c)
              acc -= (double)S[(int64_t)(k0 + c) * ld + (k + 1 + r)] * z1[c] +
                     (double)Wb[(int64_t)c * ld + (k + 1 + r)] * z2[c];
            sy[r] = acc;
          }
          __syncthreads();
        }
        // (5) w = tau y - (tau/2)(tau y . v) v into column i of W
        double pv = 0.0;
        for (int r = tid; r < n2; r += kBigBlock) pv = fma(tk * sy[r], sv[r], pv);
        const double Kc = 0.5 * tk * block_sum<kBigNW>(pv, red);
        for (int r = tid; r < n2; r += kBigBlock)
          Wb[(int64_t)i * ld + (k + 1 + r)] = (T)(tk * sy[r] - Kc * sv[r]);
        __syncthreads();
      }
      // trailing update A22 -= V W^T + W V^T (lower tiles)
      const int c0 = k0 + nbt;
      const int M = m - c0;
      if (M > 0) {
        const T* V2 = S + (int64_t)k0 * ld + c0;
        const T* W2 = Wb + c0;
        T* C = S + (int64_t)c0 * ld + c0;
        wg_gemm<T, kBigNW, false, true, true, false>(M, M, nbt, T(-1), V2, ld, W2, ld, T(1), C, ld, gsm);
        wg_gemm<T, kBigNW, false, true, true, false>(M, M, nbt, T(-1), W2, ld, V2, ld, T(1), C, ld, gsm);
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
    for (int q = tid; q < 2 * m; q += kBigBlock) {
      const int c = q < m ? m - 2 : m - 1;
      const int r = q < m ? q : q - m;
      if (c >= 0) S[(int64_t)c * ld + r] = T(0);
    }
  }
}

// ------------------------------------------------------------- form Q1
// Q1 = B_0 B_1 ... with B_t = I - V_t T_t V_t^T the compact-WY form of NB
// consecutive reflectors (T_t upper triangular: T[c][c] = tau_c,
// T[0:c, c] = -tau_c T[0:c, 0:c] (V^T V)[0:c, c]). Backward accumulation
// from the identity: Q22 -= V (T (V^T Q22)) with Q22 = Q[k0+1:, k0+1:].
template <class T>
__global__ __launch_bounds__(kBigBlock) void k_form_q1(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  __shared__ double Gs[kNB * kNB], Ts[kNB * kNB];
  const int tid = threadIdx.x;
  T* gsm = (T*)dyn;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    const T* S = at<T>((const void*)a.S, a.off[it]);
    T* Q = at<T>(a.Q, a.qoff[it]);
    T* Wm = at<T>(a.W, a.off[it]);
    const T* tau = at<T>((const void*)a.tau, a.voff[it]);
    const int64_t tot = (int64_t)ld * ld;
    for (int64_t q = tid; q < tot; q += kBigBlock) {
      const int64_t c = q / ld, r = q - c * ld;
      Q[q] = (r == c && r < m) ? T(1) : T(0);
    }
    __syncthreads();
    const int nref = m - 2;
    if (nref > 0) {
      const int nblk = (nref + kNB - 1) / kNB;
      for (int t = nblk - 1; t >= 0; --t) {
        const int k0 = t * kNB;
        const int nbt = (nref - k0) < kNB ? (nref - k0) : kNB;
        const int n2 = m - k0 - 1;
        const T* V = S + (int64_t)k0 * ld + (k0 + 1);
        // Gram matrix of the block's vectors
        for (int q = tid; q < nbt * nbt; q += kBigBlock) {
          const int r = q / nbt, c = q - r * nbt;
          double g = 0.0;
          if (r <= c) {
            const T* vr = V + (int64_t)r * ld;
            const T* vc = V + (int64_t)c * ld;
            for (int s = c; s < n2; ++s) g = fma((double)vr[s], (double)vc[s], g);
          }
          Gs[r * kNB + c] = g;
        }
        __syncthreads();
        if (tid < kWave) {
          for (int c = 0; c < nbt; ++c) {
            const double tc = (double)tau[k0 + c];
            // T[r][c] for r < c: -tau_c sum_{s=r}^{c-1} T[r][s] G[s][c]
            double v = 0.0;
            if (tid < c) {
              for (int s = tid; s < c; ++s) v = fma(Ts[tid * kNB + s], Gs[s * kNB + c], v);
              v = -tc * v;
            }
            __builtin_amdgcn_wave_barrier();
            if (tid < c) Ts[tid * kNB + c] = v;
            if (tid == c) Ts[c * kNB + c] = tc;
            if (tid > c && tid < kNB) Ts[tid * kNB + c] = 0.0;
            __builtin_amdgcn_wave_barrier();
          }
        }
        __syncthreads();
        // Wm (nbt x n2, ld nbt) = V^T Q22
        T* Q22 = Q + (int64_t)(k0 + 1) * ld + (k0 + 1);
        wg_gemm<T, kBigNW, true, false>(nbt, n2, n2, T(1), V, ld, Q22, ld, T(0), Wm, nbt, gsm);
        // Wm = T Wm, 64 columns at a time through LDS
        for (int c0 = 0; c0 < n2; c0 += 64) {
          const int nc = (n2 - c0) < 64 ? (n2 - c0) : 64;
          for (int q = tid; q < nbt * nc; q += kBigBlock) {
            const int c = q / nbt, r = q - c * nbt;
            gsm[c * kNB + r] = Wm[(int64_t)(c0 + c) * nbt + r];
          }
          __syncthreads();
          for (int q = tid; q < nbt * nc; q += kBigBlock) {
            const int c = q / nbt, r = q - c * nbt;
            double acc = 0.0;
            for (int q2 = r; q2 < nbt; ++q2) acc = fma(Ts[r * kNB + q2], (double)gsm[c * kNB + q2], acc);
            Wm[(int64_t)(c0 + c) * nbt + r] = (T)acc;
          }
          __syncthreads();
        }
        // Q22 -= V Wm
        wg_gemm<T, kBigNW, false, false>(n2, n2, nbt, T(-1), V, ld, Wm, nbt, T(1), Q22, ld, gsm);
      }
    }
  }
}

// ---------------------------------------------------------- QL on T
__device__ __forceinline__ void store_pair(double* p, double c, double s) {
  *(double2*)p = make_double2(c, s);
}
__device__ __forceinline__ void store_pair(float* p, float c, float s) {
  *(float2*)p = make_float2(c, s);
}

// One lane per submatrix, P submatrices per wave, d and e in LDS (FP64).
// Implicit QL with a Wilkinson shift on the unreduced block [l, mm]; each
// sweep runs i = mm-1 down to l and records its rotations (c, s): columns
// (i, i+1) of Q become (c q_i - s q_{i+1}, s q_i + c q_{i+1}).
// Sweep table entry: hi, lo, offset of its first rotation.
template <class T>
__global__ __launch_bounds__(64) void k_tridiag_ql(LargeArgs a) {
  extern __shared__ double dyn[];
  const int P = a.ql_items;
  const int LDL = a.max_m + 1;
  const int lane = threadIdx.x;
  const int it = blockIdx.x * P + lane;
  if (lane >= P || it >= a.n_items) return;
  if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) return;
  const int j = a.items[it];
  const int m = a.rowptr[j + 1] - a.rowptr[j];
  double* d = dyn + (int64_t)lane * LDL;
  double* e = dyn + (int64_t)(P + lane) * LDL;
  T* dg = at<T>(a.d, a.doff[it]);
  const T* eg = at<T>((const void*)a.e, a.voff[it]);
  for (int k = 0; k < m; ++k) {
    d[k] = (double)dg[k];
    e[k] = (double)eg[k];
  }
  T* rot = at<T>(a.rot, a.roff[it]);
  int32_t* sw = a.sweeps + a.swoff[it];
  const int64_t rot_cap = 2 * (int64_t)m * m + 64;
  const int sw_cap = 6 * m + 16;
  const double eps = Eps<T>::v;
  int64_t nrot = 0;
  int nsw = 0;
  int flags = 0;
  e[m - 1] = 0.0;
  for (int l = 0; l < m && !(flags & LF_UNCONV); ++l) {
    int iter = 0;
    for (;;) {
      // first negligible off-diagonal at or after l, eight entries per step
      int mm = m - 1;
      for (int k8 = l; k8 < m - 1; k8 += 8) {
        int hit = -1;
#pragma unroll
        for (int u = 7; u >= 0; --u) {
          const int kk = k8 + u;
          if (kk < m - 1 && fabs(e[kk]) <= eps * (fabs(d[kk]) + fabs(d[kk + 1]))) hit = kk;
        }
        if (hit >= 0) {
          mm = hit;
          break;
        }
      }
      if (mm == l) break;
      if (++iter > 40 || nsw >= sw_cap || nrot + (mm - l) > rot_cap) {
        flags |= LF_UNCONV;
        break;
      }
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      const int64_t base = nrot;
      bool early = false;
      // d[i+1] of iteration i is the d[i] that iteration i+1 read (the sweep
      // only writes d[i+2] before it), so it is carried in a register
      double dnext = d[mm];
      double di = d[mm - 1], ei = e[mm - 1];
      // d[i-1], e[i-1] were read one iteration earlier; d[i-2], e[i-2] are
      // requested now, so no LDS read is waited on in the rotation chain
      double dn = mm - 2 >= l ? d[mm - 2] : 0.0, en = mm - 2 >= l ? e[mm - 2] : 0.0;
      for (int i = mm - 1; i >= l; --i) {
        double dnn = 0.0, enn = 0.0;
        if (i - 2 >= l) { dnn = d[i - 2]; enn = e[i - 2]; }
        const double f = s * ei;
        const double b = c * ei;
        // r = hypot(f, g) and 1/r from one reciprocal square root refined by
        // two Newton steps; the scaled fallback guards against overflow
        const double af = fabs(f), ag = fabs(g);
        const double big = af > ag ? af : ag;
        double rinv;
        if (big > 1e150 || big < 1e-150) {
          r = hypot(f, g);
          rinv = r != 0.0 ? 1.0 / r : 0.0;
        } else {
          const double x2 = fma(f, f, g * g);
          double y = __builtin_amdgcn_rsq(x2);
          double hx = x2 * y;
          y = fma(0.5 * y, fma(-hx, y, 1.0), y);
          hx = x2 * y;
          y = fma(0.5 * y, fma(-hx, y, 1.0), y);
          rinv = y;
          r = x2 * y;
        }
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] = dnext - pp;
          e[mm] = 0.0;
          early = true;
          break;
        }
        s = f * rinv;
        c = g * rinv;
        g = dnext - pp;
        r = (di - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        store_pair(rot + 2 * nrot, (T)c, (T)s);
        ++nrot;
        dnext = di;
        di = dn;
        ei = en;
        dn = dnn;
        en = enn;
      }
      const int cnt = (int)(nrot - base);
      if (cnt > 0) {
        sw[3 * nsw + 0] = mm - 1;
        sw[3 * nsw + 1] = mm - cnt;
        sw[3 * nsw + 2] = (int32_t)base;
        ++nsw;
      }
      if (early) continue;
      d[l] -= pp;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
  a.nsweeps[it] = nsw;
  // spectrum checks: lambda_min <= 0 has no real inverse p-th root; in the
  // FP32 pass an estimated condition number above kappa_max sends the
  // submatrix to the FP64 pass
  double lmin = INFINITY, lmax = -INFINITY;
  for (int k = 0; k < m; ++k) {
    const double v = d[k];
    lmin = fmin(lmin, v);
    lmax = fmax(lmax, v);
    dg[k] = (T)v;
  }
  if (!a.fp64) {
    if ((flags & LF_UNCONV) || !(lmin > 0.0) || lmax > a.kappa_max * lmin) flags = LF_FALLBACK;
  } else if (!(lmin > 0.0)) {
    flags |= LF_NONPOS;
  }
  if (a.only_flagged) a.flags[it] = flags | LF_FALLBACK;
  else a.flags[it] = flags;
  if (flags & LF_NONPOS) atomicAdd((unsigned long long*)&a.status[ST_NONPOS], 1ull);
  if (a.fp64 && (flags & LF_UNCONV)) atomicAdd((unsigned long long*)&a.status[ST_UNCONV], 1ull);
  if (!a.fp64 && (flags & LF_FALLBACK)) atomicAdd((unsigned long long*)&a.status[ST_FALLBACK], 1ull);
  atomicAdd((unsigned long long*)&a.status[ST_ROTWORK], (unsigned long long)(nrot * m));
}

// ------------------------------------------------------ apply rotations
// Q <- Q * G_1 * G_2 * ... (all recorded rotations, in order). A batch of K
// sweeps is applied in one pass over each row: at step t sweep s acts on
// columns (P, P+1), P = H - t + 2s. The logical window slot i (column
// H - t + i) lives in register (i - t) mod 2K, so nothing is shifted; the
// step loop is unrolled over 2K steps per LDS table chunk. Inactive
// (sweep, step) pairs are identity rotations in the table. Each thread
// carries RPT rows, so every coefficient read from LDS serves RPT rows.
template <class T, int K, int RPT>
__global__ __launch_bounds__(kBlock) void k_apply_rotations(LargeArgs a) {
  constexpr int TS = 2 * K;
  __shared__ int s_item;
  __shared__ int s_hi[K], s_lo[K], s_off[K];
  __shared__ T tab[TS][K][2];
  const int tid = threadIdx.x;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (skip_item(a, it)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    T* Q = at<T>(a.Q, a.qoff[it]);
    const T* rot = at<T>((const void*)a.rot, a.roff[it]);
    const int32_t* sw = a.sweeps + a.swoff[it];
    const int nsw = a.nsweeps[it];
    for (int b0 = 0; b0 < nsw; b0 += K) {
      const int nb = (nsw - b0) < K ? (nsw - b0) : K;
      __syncthreads();
      if (tid < K) {
        if (tid < nb) {
          s_hi[tid] = sw[3 * (b0 + tid) + 0];
          s_lo[tid] = sw[3 * (b0 + tid) + 1];
          s_off[tid] = sw[3 * (b0 + tid) + 2];
        } else {
          s_hi[tid] = -1;  // empty sweep: never active
          s_lo[tid] = 1;
          s_off[tid] = 0;
        }
      }
      __syncthreads();
      int H = -1, L = m;
      for (int s = 0; s < K; ++s) {
        if (s_hi[s] >= 0) {
          H = s_hi[s] > H ? s_hi[s] : H;
          L = s_lo[s] < L ? s_lo[s] : L;
        }
      }
      if (H < 0) continue;
      const int tend = H + 2 * K - 1 - L;
      for (int rb = 0; rb < m; rb += kBlock * RPT) {
        int row[RPT];
        bool act[RPT];
        T w[RPT][TS];
        // columns are loaded PF steps before they enter the window
        constexpr int PF = 8;
        T pf[RPT][PF];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          row[u] = rb + tid + u * kBlock;
          act[u] = row[u] < m;
#pragma unroll
          for (int q = 0; q < TS; ++q) w[u][q] = T(0);
          // slot 1 at t = 0 is column H+1 -> register 1
          if (act[u]) w[u][1] = Q[(int64_t)(H + 1) * ld + row[u]];
#pragma unroll
          for (int q = 0; q < PF; ++q) {
            const int col = H - q;
            pf[u][q] = (act[u] && col >= L) ? Q[(int64_t)col * ld + row[u]] : T(0);
          }
        }
        for (int t0 = 0; t0 <= tend; t0 += TS) {
          __syncthreads();
          for (int q = tid; q < TS * K; q += kBlock) {
            const int ts = q / K, s = q - ts * K;
            const int P = H - (t0 + ts) + 2 * s;
            T c = T(1), sn = T(0);
            if (P >= s_lo[s] && P <= s_hi[s]) {
              const int64_t idx = (int64_t)s_off[s] + (s_hi[s] - P);
              c = rot[2 * idx];
              sn = rot[2 * idx + 1];
            }
            tab[ts][s][0] = c;
            tab[ts][s][1] = sn;
          }
          __syncthreads();
#pragma unroll
          for (int ts = 0; ts < TS; ++ts) {
            const int t = t0 + ts;
            if (t <= tend) {
              const int base = H - t;
              // register of logical slot i at this step: (i - ts) mod TS;
              // the column entering now was prefetched into pf[ts % PF]
              if (base >= L) {
#pragma unroll
                for (int u = 0; u < RPT; ++u) w[u][(TS - ts) % TS] = pf[u][ts % PF];
              }
              const int cpf = base - PF;
              if (cpf >= L) {
#pragma unroll
                for (int u = 0; u < RPT; ++u)
                  if (act[u]) pf[u][ts % PF] = Q[(int64_t)cpf * ld + row[u]];
              }
#pragma unroll
              for (int s = 0; s < K; ++s) {
                const int p0 = (2 * s - ts + 2 * TS) % TS, p1 = (2 * s + 1 - ts + 2 * TS) % TS;
                const T c = tab[ts][s][0], sn = tab[ts][s][1];
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                  const T x0 = w[u][p0], x1 = w[u][p1];
                  w[u][p1] = sn * x0 + c * x1;
                  w[u][p0] = c * x0 - sn * x1;
                }
              }
              const int pout = base + TS - 1;
              if (pout <= H + 1 && pout >= L) {
#pragma unroll
                for (int u = 0; u < RPT; ++u)
                  if (act[u]) Q[(int64_t)pout * ld + row[u]] = w[u][(TS - 1 - ts + TS) % TS];
              }
            }
          }
        }
      }
    }
  }
}

// ------------------------------------------------------- apply column
// x[r] = sum_p Q[r][p] f(lambda_p) Q[c][p]; NaN when lambda_min <= 0 or the
// QL iteration did not converge.
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
    const int c = a.cidx[j];
    const T* Q = at<T>((const void*)a.Q, a.qoff[it]);
    const T* lam = at<T>((const void*)a.d, a.doff[it]);
    const bool bad = (fl & (LF_NONPOS | LF_UNCONV)) != 0;
    for (int q = tid; q < m; q += kBlock) wv[q] = inv_root_p((double)lam[q], a.p) * (double)Q[(int64_t)q * ld + c];
    __syncthreads();
    VT* x = (VT*)a.x + a0;
    for (int r = tid; r < m; r += kBlock) {
      double s = 0.0;
      for (int q = 0; q < m; ++q) s = fma((double)Q[(int64_t)q * ld + r], wv[q], s);
      x[r] = bad ? (VT)NAN : (VT)s;
    }
  }
}

// --------------------------------------------------------------- adjoint
// a = Q^T w, b = Q[c,:]^T, Ms = (G o (a b^T + b a^T))/2, T1 = Q Ms,
// D = T1 Q^T (lower tiles; D is symmetric), then every stored pair
// (R[k], R[l]) at position q receives D[max(k,l)][min(k,l)].
template <class T, class VT>
__global__ __launch_bounds__(kBigBlock) void k_adjoint(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  int* R = (int*)dyn;
  double* w = dyn + (a.max_m + 1) / 2 + 1;
  double* av = w + a.max_m;
  double* bv = av + a.max_m;
  double* alv = bv + a.max_m;
  T* gsm = (T*)(alv + a.max_m);
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (skip_item(a, it)) continue;
    const int fl = a.flags[it];
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    const int c = a.cidx[j];
    const T* Q = at<T>((const void*)a.Q, a.qoff[it]);
    T* Ms = at<T>(a.S, a.off[it]);
    T* T1 = at<T>(a.W, a.off[it]);
    const T* lam = at<T>((const void*)a.d, a.doff[it]);
    const bool bad = (fl & (LF_NONPOS | LF_UNCONV)) != 0;
    const VT* gx = (const VT*)a.gx + a0;
    for (int i = tid; i < m; i += kBigBlock) {
      R[i] = a.colind[a0 + i];
      w[i] = (double)gx[i];
      bv[i] = (double)Q[(int64_t)i * ld + c];
      alv[i] = root_p((double)lam[i], a.p);
    }
    __syncthreads();
    for (int pc = wv; pc < m; pc += kBigNW) {
      double part = 0.0;
      for (int r = lane; r < m; r += kWave) part = fma((double)Q[(int64_t)pc * ld + r], w[r], part);
      part = wave_sum(part);
      if (lane == 0) av[pc] = part;
    }
    __syncthreads();
    for (int l = wv; l < m; l += kBigNW) {
      for (int pr = lane; pr < m; pr += kWave) {
        const double g = divdiff(alv[pr], alv[l], a.p);
        Ms[(int64_t)l * ld + pr] = (T)(0.5 * g * (av[pr] * bv[l] + av[l] * bv[pr]));
      }
    }
    __syncthreads();
    wg_gemm<T, kBigNW, false, false>(m, m, m, T(1), Q, ld, Ms, ld, T(0), T1, ld, gsm);
    wg_gemm<T, kBigNW, false, true, true>(m, m, m, T(1), T1, ld, Q, ld, T(0), Ms, ld, gsm);
    VT* ga = (VT*)a.ga;
    for (int k = wv; k < m; k += kBigNW) {
      const int r = R[k];
      const int s0 = a.rowptr[r], s1 = a.rowptr[r + 1];
      for (int q = s0 + lane; q < s1; q += kWave) {
        const int l = find_sorted(R, m, a.colind[q]);
        if (l >= 0) {
          const int hi = l > k ? l : k, lo = l > k ? k : l;
          atomicAdd(&ga[q], bad ? (VT)NAN : (VT)Ms[(int64_t)lo * ld + hi]);
        }
      }
    }
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
  const size_t lds = (size_t)a.max_m * sizeof(int);
  if (a.fp64) {
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_gather_large<double, VT>), dim3(a.grid), dim3(kBlock), lds, s, a));
  } else {
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_gather_large<float, VT>), dim3(a.grid), dim3(kBlock), lds, s, a));
  }
  return hipGetLastError();
}

template <class T>
static void launch_tridiag_t(const LargeArgs& a, hipStream_t s) {
  const size_t part = vec_lds(a, kBigNW, 8), gemm = gemm_lds_elems<kBigNW>() * sizeof(T);
  const size_t lds = vec_lds(a, 1, 8) + (part > gemm ? part : gemm);
  hipLaunchKernelGGL(k_tridiagonalise<T>, dim3(a.grid), dim3(kBigBlock), lds, s, a);
}

hipError_t launch_tridiagonalise(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.fp64) launch_tridiag_t<double>(a, s);
  else launch_tridiag_t<float>(a, s);
  return hipGetLastError();
}

hipError_t launch_form_q1(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.fp64)
    hipLaunchKernelGGL(k_form_q1<double>, dim3(a.grid), dim3(kBigBlock), gemm_lds_elems<kBigNW>() * 8, s, a);
  else
    hipLaunchKernelGGL(k_form_q1<float>, dim3(a.grid), dim3(kBigBlock), gemm_lds_elems<kBigNW>() * 4, s, a);
  return hipGetLastError();
}

int ql_items_per_wave(int max_m, int lds_limit, int blocks_per_cu) {
  // d and e of P submatrices in LDS (FP64), the device's LDS shared by
  // blocks_per_cu blocks
  const int64_t budget = ((int64_t)(lds_limit > 0 ? lds_limit : 65536) - 4096) / blocks_per_cu;
  int p = (int)(budget / (16 * (int64_t)(max_m + 1)));
  if (p > 64) p = 64;
  if (p < 1) p = 1;
  return p;
}

hipError_t launch_tridiag_ql(const LargeArgs& a0, hipStream_t s) {
  if (a0.n_items <= 0) return hipSuccess;
  LargeArgs a = a0;
  a.ql_items = ql_items_per_wave(a.max_m, a.lds_limit, a.ql_bpc > 0 ? a.ql_bpc : 2);
  const int grid = (a.n_items + a.ql_items - 1) / a.ql_items;
  const size_t lds = (size_t)2 * a.ql_items * (a.max_m + 1) * sizeof(double);
  if (a.fp64)
    hipLaunchKernelGGL(k_tridiag_ql<double>, dim3(grid), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL(k_tridiag_ql<float>, dim3(grid), dim3(64), lds, s, a);
  return hipGetLastError();
}

template <class T>
static void launch_rot_t(const LargeArgs& a, hipStream_t s) {
  const bool two = a.max_m > kBlock;
  if (a.rot_batch >= 16) {
    if (two) hipLaunchKernelGGL((k_apply_rotations<T, 16, 2>), dim3(a.grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_apply_rotations<T, 16, 1>), dim3(a.grid), dim3(kBlock), 0, s, a);
  } else {
    if (two) hipLaunchKernelGGL((k_apply_rotations<T, 8, 2>), dim3(a.grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_apply_rotations<T, 8, 1>), dim3(a.grid), dim3(kBlock), 0, s, a);
  }
}

hipError_t launch_apply_rotations(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.fp64) launch_rot_t<double>(a, s);
  else launch_rot_t<float>(a, s);
  return hipGetLastError();
}

hipError_t launch_check_spectrum(const LargeArgs&, hipStream_t) { return hipSuccess; }

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

hipError_t launch_adjoint(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const size_t base = ((size_t)(a.max_m + 1) / 2 + 1) * 8 + vec_lds(a, 4, 8);
  if (a.fp64) {
    const size_t lds = base + gemm_lds_elems<kBigNW>() * sizeof(double);
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_adjoint<double, VT>), dim3(a.grid), dim3(kBigBlock), lds, s, a));
  } else {
    const size_t lds = base + gemm_lds_elems<kBigNW>() * sizeof(float);
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_adjoint<float, VT>), dim3(a.grid), dim3(kBigBlock), lds, s, a));
  }
  return hipGetLastError();
}

}  // namespace submat
