// Large-order path (m > 64): one workgroup per submatrix for the dense
// stages, one lane per submatrix for the tridiagonal QL iteration.
//
//   gather     S_j from CSR into an HBM slab (Section 3.1), symmetrised
//   tridiag    Householder reduction S = Q1 T Q1^T (lower form)
//   form_q1    Q1 accumulated explicitly from the reflectors
//   ql         implicit QL with Wilkinson shifts on T; the eigenvalues replace
//              d and every plane rotation is recorded, sweep by sweep
//   rotations  Q = Q1 * (all rotations): each thread owns rows of Q and applies
//              a batch of K sweeps in one pass over the row (sweep s lags
//              sweep s-1 by two columns, so a window of 2K values suffices)
//   column     x = Q (f(lambda) o Q[c,:]^T) into X's value segment
//              (Sections 3.3-3.4)
//   adjoint    D = Q sym(G o (a b^T)) Q^T scattered into dA's stored pairs
//
// Slabs are column-major with leading dimension ldm (the order rounded up
// to a multiple of 16); element (r, c) of item i is at base + off[i] +
// c*ldm + r.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace submat {

constexpr int kBlock = 256;
constexpr int kNW = kBlock / kWave;

template <class T> __device__ __forceinline__ T* at(void* base, int64_t off_bytes) {
  return (T*)((char*)base + off_bytes);
}
template <class T> __device__ __forceinline__ const T* at(const void* base, int64_t off_bytes) {
  return (const T*)((const char*)base + off_bytes);
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

// ------------------------------------------------------- tridiagonalise
// Unblocked Householder reduction, both triangles kept up to date.
// Step k: v (v0 = 1) maps S[k+1:, k] to beta e_1; p = tau S22 v;
// w = p - (tau/2)(p.v) v; S22 -= v w^T + w v^T.
// Outputs: d[0..m), e[0..m-1), tau[0..m-2), v_k stored in S[k+1:, k].
template <class T>
__global__ __launch_bounds__(kBlock) void k_tridiagonalise(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  __shared__ double red[kNW];
  const int tid = threadIdx.x;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    T* S = at<T>(a.S, a.off[it]);
    T* d = at<T>(a.d, a.doff[it]);
    T* e = at<T>(a.e, a.voff[it]);
    T* tau = at<T>(a.tau, a.voff[it]);
    T* sv = (T*)dyn;
    T* sw = sv + a.max_m;
    for (int k = 0; k + 2 < m; ++k) {
      const int n2 = m - k - 1;
      T* x = S + (int64_t)k * ld + (k + 1);
      double part = 0.0;
      for (int i = 1 + tid; i < n2; i += kBlock) part += (double)x[i] * (double)x[i];
      const double alpha = (double)x[0];  // read before the barrier: x[0] is overwritten below
      const double sigma = block_sum<kNW>(part, red);
      double beta, tk, scale;
      if (sigma == 0.0) {
        beta = alpha; tk = 0.0; scale = 0.0;
      } else {
        const double nrm = sqrt(alpha * alpha + sigma);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tk = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int i = tid; i < n2; i += kBlock) {
        const T vi = (i == 0) ? T(1) : (T)((double)x[i] * scale);
        sv[i] = vi;
        x[i] = vi;
      }
      if (tid == 0) {
        d[k] = S[(int64_t)k * ld + k];
        e[k] = (T)beta;
        tau[k] = (T)tk;
      }
      __syncthreads();
      if (tk != 0.0) {
        // p = tau * S22 v (thread per row)
        T* S22 = S + (int64_t)(k + 1) * ld + (k + 1);
        double pv_part = 0.0;
        for (int i = tid; i < n2; i += kBlock) {
          T acc = T(0);
          for (int jj = 0; jj < n2; ++jj) acc += S22[(int64_t)jj * ld + i] * sv[jj];
          const T pi = (T)tk * acc;
          sw[i] = pi;
          pv_part += (double)pi * (double)sv[i];
        }
        const double Kc = 0.5 * tk * block_sum<kNW>(pv_part, red);
        for (int i = tid; i < n2; i += kBlock) sw[i] = (T)((double)sw[i] - Kc * (double)sv[i]);
        __syncthreads();
        for (int i = tid; i < n2; i += kBlock) {
          const T vi = sv[i], wi = sw[i];
          for (int jj = 0; jj < n2; ++jj) {
            T* q = S22 + (int64_t)jj * ld + i;
            *q = *q - (vi * sw[jj] + wi * sv[jj]);
          }
        }
        __syncthreads();
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
  }
}

// ------------------------------------------------------------- form Q1
// Q1 = H_0 H_1 ... H_{m-3}; backward accumulation from the identity:
// Q[k+1:, k+1:] -= tau_k v_k (v_k^T Q[k+1:, k+1:]).
template <class T>
__global__ __launch_bounds__(kBlock) void k_form_q1(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int m = a.rowptr[j + 1] - a.rowptr[j];
    const int ld = a.ldm[it];
    const T* S = at<T>(a.S, a.off[it]);
    T* Q = at<T>(a.Q, a.qoff[it]);
    const T* tau = at<T>((const void*)a.tau, a.voff[it]);
    T* sv = (T*)dyn;
    T* sy = sv + a.max_m;
    const int64_t tot = (int64_t)ld * ld;
    for (int64_t q = tid; q < tot; q += kBlock) {
      const int64_t c = q / ld, r = q - c * ld;
      Q[q] = (r == c && r < m) ? T(1) : T(0);
    }
    __syncthreads();
    for (int k = m - 3; k >= 0; --k) {
      const T tk = tau[k];
      if (tk == T(0)) continue;
      const int n2 = m - k - 1;
      const T* v = S + (int64_t)k * ld + (k + 1);
      for (int i = tid; i < n2; i += kBlock) sv[i] = v[i];
      __syncthreads();
      T* Q22 = Q + (int64_t)(k + 1) * ld + (k + 1);
      // y_c = sum_i v_i Q22[i][c]: one wave per column, lanes over rows
      for (int c = wv; c < n2; c += kNW) {
        double part = 0.0;
        for (int i = lane; i < n2; i += kWave) part += (double)sv[i] * (double)Q22[(int64_t)c * ld + i];
        part = wave_sum(part);
        if (lane == 0) sy[c] = (T)((double)tk * part);
      }
      __syncthreads();
      for (int i = tid; i < n2; i += kBlock) {
        const T vi = sv[i];
        for (int c = 0; c < n2; ++c) {
          T* q = Q22 + (int64_t)c * ld + i;
          *q = *q - vi * sy[c];
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------- QL on T
// One lane per submatrix. Implicit QL with a Wilkinson shift on the
// unreduced block [l, mm]; each sweep runs i = mm-1 down to l and records
// its rotations (c, s): columns (i, i+1) of Q become
// (c q_i - s q_{i+1}, s q_i + c q_{i+1}). Sweep table entry: hi, lo, offset.
template <class T>
__global__ __launch_bounds__(64) void k_tridiag_ql(LargeArgs a) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= a.n_items) return;
  if (a.only_flagged && !(a.flags[it] & LF_FALLBACK)) return;
  const int j = a.items[it];
  const int m = a.rowptr[j + 1] - a.rowptr[j];
  T* d = at<T>(a.d, a.doff[it]);
  T* e = at<T>(a.e, a.voff[it]);
  T* rot = at<T>(a.rot, a.roff[it]);
  int32_t* sw = a.sweeps + a.swoff[it];
  const int64_t rot_cap = 2 * (int64_t)m * m + 64;
  const int sw_cap = 6 * m + 16;
  const double eps = Eps<T>::v;
  int64_t nrot = 0;
  int nsw = 0;
  int flags = 0;
  e[m - 1] = T(0);
  for (int l = 0; l < m && !(flags & LF_UNCONV); ++l) {
    int iter = 0;
    for (;;) {
      int mm = l;
      for (; mm < m - 1; ++mm) {
        const double dd = fabs((double)d[mm]) + fabs((double)d[mm + 1]);
        if (fabs((double)e[mm]) <= eps * dd) break;
      }
      if (mm == l) break;
      if (++iter > 40 || nsw >= sw_cap || nrot + (mm - l) > rot_cap) {
        flags |= LF_UNCONV;
        break;
      }
      double g = ((double)d[l + 1] - (double)d[l]) / (2.0 * (double)e[l]);
      double r = hypot(g, 1.0);
      g = (double)d[mm] - (double)d[l] + (double)e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      const int64_t base = nrot;
      int i = mm - 1;
      bool early = false;
      double di = (double)d[i], ei = (double)e[i];
      for (; i >= l; --i) {
        // prefetch the next pair while this rotation is formed
        double dn = 0.0, en = 0.0;
        if (i > l) { dn = (double)d[i - 1]; en = (double)e[i - 1]; }
        const double f = s * ei;
        const double b = c * ei;
        r = hypot(f, g);
        e[i + 1] = (T)r;
        if (r == 0.0) {
          d[i + 1] = (T)((double)d[i + 1] - pp);
          e[mm] = T(0);
          early = true;
          break;
        }
        const double rinv = 1.0 / r;
        s = f * rinv;
        c = g * rinv;
        g = (double)d[i + 1] - pp;
        r = (di - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = (T)(g + pp);
        g = c * r - b;
        rot[2 * nrot] = (T)c;
        rot[2 * nrot + 1] = (T)s;
        ++nrot;
        di = dn;
        ei = en;
      }
      const int cnt = (int)(nrot - base);
      if (cnt > 0) {
        sw[3 * nsw + 0] = mm - 1;
        sw[3 * nsw + 1] = mm - cnt;
        sw[3 * nsw + 2] = (int32_t)base;
        ++nsw;
      }
      if (early) continue;
      d[l] = (T)((double)d[l] - pp);
      e[l] = (T)g;
      e[mm] = T(0);
    }
  }
  a.nsweeps[it] = nsw;
  // spectrum checks: lambda_min <= 0 has no real inverse p-th root; in the
  // FP32 pass an estimated condition number above kappa_max sends the
  // submatrix to the FP64 pass
  double lmin = INFINITY, lmax = -INFINITY;
  for (int k = 0; k < m; ++k) {
    const double v = (double)d[k];
    lmin = fmin(lmin, v);
    lmax = fmax(lmax, v);
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
}

// ------------------------------------------------------ apply rotations
// Q <- Q * G_1 * G_2 * ... (all recorded rotations, in order). A batch of K
// sweeps is applied in one pass over each row: at step t sweep s acts on
// columns (P, P+1), P = H - t + 2s, which keeps the per-row window at 2K
// values (slots 2s, 2s+1 for sweep s) in registers.
template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_apply_rotations(LargeArgs a) {
  __shared__ int s_item;
  __shared__ int s_hi[K], s_lo[K], s_off[K];
  const int tid = threadIdx.x;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    const int fl = a.flags[it];
    if (a.only_flagged && !(fl & LF_FALLBACK)) continue;
    if (!a.only_flagged && !a.fp64 && (fl & LF_FALLBACK)) continue;  // redone in FP64
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
#pragma unroll
      for (int s = 0; s < K; ++s) {
        if (s_hi[s] >= 0) {
          H = s_hi[s] > H ? s_hi[s] : H;
          L = s_lo[s] < L ? s_lo[s] : L;
        }
      }
      if (H < 0) continue;
      const int tend = H + 2 * K - 1 - L;
      for (int r = tid; r < m; r += kBlock) {
        T w[2 * K];
#pragma unroll
        for (int q = 0; q < 2 * K; ++q) w[q] = T(0);
        w[1] = Q[(int64_t)(H + 1) * ld + r];
        for (int t = 0; t <= tend; ++t) {
          const int base = H - t;
          if (base >= L) w[0] = Q[(int64_t)base * ld + r];
#pragma unroll
          for (int s = 0; s < K; ++s) {
            const int P = base + 2 * s;
            if (P >= s_lo[s] && P <= s_hi[s]) {
              const int64_t idx = (int64_t)s_off[s] + (s_hi[s] - P);
              const T c = rot[2 * idx], sn = rot[2 * idx + 1];
              const T x0 = w[2 * s], x1 = w[2 * s + 1];
              w[2 * s + 1] = sn * x0 + c * x1;
              w[2 * s] = c * x0 - sn * x1;
            }
          }
          const int pout = base + 2 * K - 1;
          if (pout <= H + 1 && pout >= L) Q[(int64_t)pout * ld + r] = w[2 * K - 1];
#pragma unroll
          for (int q = 2 * K - 1; q > 0; --q) w[q] = w[q - 1];
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
    const int fl = a.flags[it];
    if (a.only_flagged && !(fl & LF_FALLBACK)) continue;
    if (!a.only_flagged && !a.fp64 && (fl & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    const int c = a.cidx[j];
    const T* Q = at<T>(a.Q, a.qoff[it]);
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
// C = A * B (NN) or A * B^T (NT), m x m, column-major, leading dim ld.
// 256 threads, 64x64 output tiles, 4x4 per thread, K steps of 16.
template <class T, bool NT>
__device__ void block_gemm(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C, int m,
                           int ld, T* As, T* Bs) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  for (int ti = 0; ti < m; ti += 64) {
    for (int tj = 0; tj < m; tj += 64) {
      T acc[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = T(0);
      for (int kk = 0; kk < m; kk += 16) {
        __syncthreads();
        for (int q = tid; q < 16 * 64; q += kBlock) {
          const int kq = q >> 6, iq = q & 63;
          const int gi = ti + iq, gk = kk + kq;
          As[kq * 64 + iq] = (gi < m && gk < m) ? A[(int64_t)gk * ld + gi] : T(0);
          const int gj = tj + iq;
          T bv = T(0);
          if (gj < m && gk < m) bv = NT ? B[(int64_t)gk * ld + gj] : B[(int64_t)gj * ld + gk];
          Bs[kq * 64 + iq] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int kq = 0; kq < 16; ++kq) {
          T av[4], bv[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) av[x] = As[kq * 64 + ty * 4 + x];
#pragma unroll
          for (int y = 0; y < 4; ++y) bv[y] = Bs[kq * 64 + tx * 4 + y];
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] += av[x] * bv[y];
        }
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) {
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int gi = ti + ty * 4 + x, gj = tj + tx * 4 + y;
          if (gi < m && gj < m) C[(int64_t)gj * ld + gi] = acc[x][y];
        }
      }
    }
  }
  __syncthreads();
}

template <class T, class VT>
__global__ __launch_bounds__(kBlock) void k_adjoint(LargeArgs a) {
  extern __shared__ double dyn[];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  // dynamic LDS: R (max_m ints, padded to doubles), w, av, bv, alv (max_m doubles each),
  // then two 16x64 GEMM staging tiles of T
  int* R = (int*)dyn;
  double* w = dyn + (a.max_m + 1) / 2 + 1;
  double* av = w + a.max_m;
  double* bv = av + a.max_m;
  double* alv = bv + a.max_m;
  T* As = (T*)(alv + a.max_m);
  T* Bs = As + 16 * 64;
  for (;;) {
    const int it = next_item(a.work_ctr, &s_item);
    if (it >= a.n_items) break;
    const int fl = a.flags[it];
    if (a.only_flagged && !(fl & LF_FALLBACK)) continue;
    if (!a.only_flagged && !a.fp64 && (fl & LF_FALLBACK)) continue;
    const int j = a.items[it];
    const int a0 = a.rowptr[j];
    const int m = a.rowptr[j + 1] - a0;
    const int ld = a.ldm[it];
    const int c = a.cidx[j];
    const T* Q = at<T>(a.Q, a.qoff[it]);
    T* Ms = at<T>(a.S, a.off[it]);
    T* T1 = at<T>(a.W, a.off[it]);
    const T* lam = at<T>((const void*)a.d, a.doff[it]);
    const bool bad = (fl & (LF_NONPOS | LF_UNCONV)) != 0;
    const VT* gx = (const VT*)a.gx + a0;
    for (int i = tid; i < m; i += kBlock) {
      R[i] = a.colind[a0 + i];
      w[i] = (double)gx[i];
      bv[i] = (double)Q[(int64_t)i * ld + c];
      alv[i] = root_p((double)lam[i], a.p);
    }
    __syncthreads();
    // a = Q^T w: one wave per column p
    for (int pc = wv; pc < m; pc += kNW) {
      double part = 0.0;
      for (int r = lane; r < m; r += kWave) part = fma((double)Q[(int64_t)pc * ld + r], w[r], part);
      part = wave_sum(part);
      if (lane == 0) av[pc] = part;
    }
    __syncthreads();
    // Ms[p][l] = (G o (a b^T + b a^T))/2
    for (int l = wv; l < m; l += kNW) {
      for (int pr = lane; pr < m; pr += kWave) {
        const double g = divdiff(alv[pr], alv[l], a.p);
        Ms[(int64_t)l * ld + pr] = (T)(0.5 * g * (av[pr] * bv[l] + av[l] * bv[pr]));
      }
    }
    __syncthreads();
    block_gemm<T, false>(Q, Ms, T1, m, ld, As, Bs);   // T1 = Q Ms
    block_gemm<T, true>(T1, Q, Ms, m, ld, As, Bs);    // D = T1 Q^T (into the Ms slab)
    VT* ga = (VT*)a.ga;
    for (int k = wv; k < m; k += kNW) {
      const int r = R[k];
      const int s0 = a.rowptr[r], s1 = a.rowptr[r + 1];
      for (int q = s0 + lane; q < s1; q += kWave) {
        const int l = find_sorted(R, m, a.colind[q]);
        if (l >= 0) atomicAdd(&ga[q], bad ? (VT)NAN : (VT)Ms[(int64_t)l * ld + k]);
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

hipError_t launch_tridiagonalise(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.fp64)
    hipLaunchKernelGGL(k_tridiagonalise<double>, dim3(a.grid), dim3(kBlock), vec_lds(a, 2, 8), s, a);
  else
    hipLaunchKernelGGL(k_tridiagonalise<float>, dim3(a.grid), dim3(kBlock), vec_lds(a, 2, 4), s, a);
  return hipGetLastError();
}

hipError_t launch_form_q1(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.fp64)
    hipLaunchKernelGGL(k_form_q1<double>, dim3(a.grid), dim3(kBlock), vec_lds(a, 2, 8), s, a);
  else
    hipLaunchKernelGGL(k_form_q1<float>, dim3(a.grid), dim3(kBlock), vec_lds(a, 2, 4), s, a);
  return hipGetLastError();
}

hipError_t launch_tridiag_ql(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const int grid = (a.n_items + 63) / 64;
  if (a.fp64)
    hipLaunchKernelGGL(k_tridiag_ql<double>, dim3(grid), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_tridiag_ql<float>, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_apply_rotations(const LargeArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.fp64) {
    if (a.rot_batch >= 16)
      hipLaunchKernelGGL((k_apply_rotations<double, 16>), dim3(a.grid), dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_apply_rotations<double, 8>), dim3(a.grid), dim3(kBlock), 0, s, a);
  } else {
    if (a.rot_batch >= 16)
      hipLaunchKernelGGL((k_apply_rotations<float, 16>), dim3(a.grid), dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_apply_rotations<float, 8>), dim3(a.grid), dim3(kBlock), 0, s, a);
  }
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
    const size_t lds = base + 2 * 16 * 64 * sizeof(double);
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_adjoint<double, VT>), dim3(a.grid), dim3(kBlock), lds, s, a));
  } else {
    const size_t lds = base + 2 * 16 * 64 * sizeof(float);
    SUBMAT_VT_SWITCH(a.vdtype, hipLaunchKernelGGL((k_adjoint<float, VT>), dim3(a.grid), dim3(kBlock), lds, s, a));
  }
  return hipGetLastError();
}

}  // namespace submat
