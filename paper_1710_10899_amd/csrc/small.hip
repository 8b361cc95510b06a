// One wavefront per submatrix for orders m <= 64: gather S_j from CSR into
// LDS (Section 3.1), one-sided Jacobi eigendecomposition in LDS, f(lambda)
// and the column R_j.indexof(j) (Sections 3.2-3.3), contiguous store into
// X's value segment (Section 3.4). The backward variant forms the
// Daleckii-Krein adjoint from the same eigenpairs and scatter-adds it.
//
// Layout: the working matrix A = S V and V live column-major in LDS
// (leading dimension MMAX+1). Column pairs are visited in round-robin
// tournament order, m/2 disjoint pairs per round; each pair is handled by a
// group of 128/MMAX lanes that split its rows and reduce its Gram sums with
// DPP lane exchanges. Gram entries and the rotation angle are always
// computed in FP64, also when the columns are FP32.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace submat {

template <int MMAX>
struct SmallShared {
  double A[MMAX * (MMAX + 1)];  // working columns / T1 / D (viewed as T or double)
  double V[MMAX * (MMAX + 1)];  // eigenvector columns (viewed as T)
  double lam[MMAX];
  double aa[MMAX];
  double bb[MMAX];
  double al[MMAX];
  double yv[MMAX];
  double dk[MMAX];
  int R[MMAX];
  int item;
};

// S[k][l] = A[R[k]][R[l]] (stored pattern, 0 elsewhere), then (S + S^T)/2.
template <class T, class VT, int MMAX>
__device__ void gather_small(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                             const VT* __restrict__ vals, const int* R, int m, T* A) {
  constexpr int LD = MMAX + 1;
  const int lane = threadIdx.x;
  for (int q = lane; q < m * LD; q += kWave) A[q] = T(0);
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    const int r = R[k];
    const int s0 = rowptr[r], s1 = rowptr[r + 1];
    for (int q = s0 + lane; q < s1; q += kWave) {
      const int l = find_sorted(R, m, colind[q]);
      if (l >= 0) A[l * LD + k] = (T)vals[q];
    }
  }
  __syncthreads();
  // lane l symmetrises the pairs (k, l), k < l: no two lanes touch one pair
  if (lane < m) {
    for (int k = 0; k < lane; ++k) {
      const T t = T(0.5) * (A[lane * LD + k] + A[k * LD + lane]);
      A[lane * LD + k] = t;
      A[k * LD + lane] = t;
    }
  }
  __syncthreads();
}

// One-sided Jacobi on A = S (columns orthogonalised by right rotations,
// accumulated in V). Per round the column pairs of the round-robin
// tournament are disjoint; pair q of a round belongs to the G lanes
// q*G .. q*G + G-1 (G = 8, 4 or 2 for m <= 16, 32, 64: a function of m
// alone, so a submatrix gets the same bits whatever launch it is in), lane r
// of the group taking rows r, r + G, ...
// The group forms the pair's 2 x 2 Gram matrix in FP64 (partial sums, then
// a DPP reduction within the group), every lane of the group derives the
// same rotation from it, and each lane rotates its own rows of both columns
// of A and of V, in place in LDS. On return V holds eigenvectors and
// lam[p] = a_p . v_p the signed eigenvalues. Returns true when a full sweep
// needed no rotation.
template <class T, int MMAX>
__device__ bool jacobi_small(T* A, T* V, int m, double* lam) {
  constexpr int LD = MMAX + 1;
  const int G = m <= 16 ? 8 : (m <= 32 ? 4 : 2);  // lanes per pair
  const int lane = threadIdx.x;
  const int pq = lane / G, r0 = lane - pq * G;
  for (int q = lane; q < m * LD; q += kWave) {
    const int c = q / LD, r = q - c * LD;
    V[q] = (r == c) ? T(1) : T(0);
  }
  __syncthreads();
  const int N = m + (m & 1);
  const double tol = (double)(m > 8 ? m : 8) * Eps<T>::v;
  const double tol2 = tol * tol;
  bool converged = false;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rotated = 0;
    for (int rd = 0; rd < N - 1; ++rd) {
      // circle method: pair 0 = (rd, N-1), pair k = (rd + k, rd - k) mod N-1
      int i1, i2;
      if (pq == 0) {
        i1 = rd;
        i2 = N - 1;
      } else {
        i1 = (rd + pq) % (N - 1);
        i2 = (rd - pq + (N - 1)) % (N - 1);
      }
      const int lo = i1 < i2 ? i1 : i2, hi = i1 < i2 ? i2 : i1;
      const bool act = 2 * pq < N && hi < m;  // the pair exists and is not the odd player's bye
      double sa = 0.0, sb = 0.0, g = 0.0;
      if (act) {
        const T* x = A + lo * LD;
        const T* y = A + hi * LD;
        for (int i = r0; i < m; i += G) {
          const double xi = (double)x[i], yi = (double)y[i];
          sa = fma(xi, xi, sa);
          sb = fma(yi, yi, sb);
          g = fma(xi, yi, g);
        }
      }
      sa = group_sum(sa, G);
      sb = group_sum(sb, G);
      g = group_sum(g, G);
      if (act && g * g > tol2 * sa * sb) {
        const double zeta = (sb - sa) / (2.0 * g);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const T c = (T)cs, s = (T)(cs * t);
        rotated = 1;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          T* X = (w == 0 ? A : V) + lo * LD;
          T* Y = (w == 0 ? A : V) + hi * LD;
          for (int i = r0; i < m; i += G) {
            const T x = X[i], y = Y[i];
            X[i] = c * x - s * y;
            Y[i] = s * x + c * y;
          }
        }
      }
      __syncthreads();
    }
    if (__ballot(rotated) == 0) {
      converged = true;
      break;
    }
  }
  if (lane < m) {
    double l = 0.0;
    for (int i = 0; i < m; ++i) l = fma((double)A[lane * LD + i], (double)V[lane * LD + i], l);
    lam[lane] = l;
  }
  __syncthreads();
  return converged;
}

// x_seg[r] = sum_p V[r][p] f(lambda_p) V[c][p]
template <class T, class VT, int MMAX>
__device__ void finish_forward(const T* V, SmallShared<MMAX>& sh, int m, int c, const SpecFn& fn, bool bad, VT* x_seg) {
  constexpr int LD = MMAX + 1;
  const int lane = threadIdx.x;
  if (lane < m) sh.aa[lane] = spec_f(sh.lam[lane], fn) * (double)V[lane * LD + c];
  __syncthreads();
  if (lane < m) {
    double s = 0.0;
    for (int q = 0; q < m; ++q) s = fma((double)V[q * LD + lane], sh.aa[q], s);
    x_seg[lane] = bad ? (VT)NAN : (VT)s;
  }
  __syncthreads();
}

// D = V (M + M^T)/2 V^T with M = G o (a b^T), a = V^T w, b = V[c, :]^T;
// every stored pair (R[k], R[l]) at position q gets ga[q] += D[k][l].
// The symmetric middle factor Ms is formed in LDS, then D is produced one
// column at a time (y = Ms V[k, :]^T, D[:, k] = V y) and scattered.
// With dout (deterministic mode) D is written there, m x m column-major,
// instead of being scatter-added.
template <class T, class VT, int MMAX, bool POW>
__device__ void finish_backward(const T* V, SmallShared<MMAX>& sh, int m, int c, const SpecFn& fn, bool bad,
                                const VT* __restrict__ w_seg, VT* __restrict__ ga,
                                const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                double* __restrict__ dout) {
  constexpr int LD = MMAX + 1;
  const int lane = threadIdx.x;
  double* Ms = sh.A;  // the working columns are no longer needed
  if (lane < m) sh.bb[lane] = (double)w_seg[lane];
  __syncthreads();
  double a_l = 0.0, b_l = 0.0, al_l = 0.0;
  if (lane < m) {
    for (int r = 0; r < m; ++r) a_l = fma((double)V[lane * LD + r], sh.bb[r], a_l);
    b_l = (double)V[lane * LD + c];
    al_l = spec_node(sh.lam[lane], fn);
  }
  __syncthreads();
  if (lane < m) {
    sh.aa[lane] = a_l;
    sh.bb[lane] = b_l;
    sh.al[lane] = al_l;
    if (POW) sh.yv[lane] = pow(al_l, fn.alpha);  // lambda^alpha; yv is free until the columns of D
  }
  __syncthreads();
  if (lane < m) {
    for (int l = 0; l < m; ++l)
      Ms[l * LD + lane] =
          0.5 * spec_divdiff<POW>(al_l, sh.al[l], POW ? sh.yv[l] : 0.0, fn) * (a_l * sh.bb[l] + sh.aa[l] * b_l);
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    if (lane < m) {
      double y = 0.0;
      for (int l = 0; l < m; ++l) y = fma(Ms[l * LD + lane], (double)V[l * LD + k], y);
      sh.yv[lane] = y;
    }
    __syncthreads();
    if (lane < m) {
      double dk = 0.0;
      for (int q = 0; q < m; ++q) dk = fma((double)V[q * LD + lane], sh.yv[q], dk);
      sh.dk[lane] = dk;
    }
    __syncthreads();
    if (dout) {
      for (int l = lane; l < m; l += kWave) dout[(int64_t)k * m + l] = bad ? (double)NAN : sh.dk[l];
    } else {
      // the lower triangle only (column <= row): D_j is symmetric, and the
      // upper entries receive their lower mirror's sum after the last phase
      const int r = sh.R[k];
      const int s0 = rowptr[r], s1 = rowptr[r + 1];
      for (int q = s0 + lane; q < s1; q += kWave) {
        const int cq = colind[q];
        if (cq > r) break;
        const int l = find_sorted(sh.R, m, cq);
        if (l >= 0) atomicAdd(&ga[q], bad ? (VT)NAN : (VT)sh.dk[l]);
      }
    }
    __syncthreads();
  }
}

// BWD: adjoint instead of forward; POW: the adjoint of a real power
template <class VT, int MMAX, bool BWD, bool POW>
__global__ __launch_bounds__(64) void k_small(SmallArgs args) {
  __shared__ SmallShared<MMAX> sh;
  const VT* vals = (const VT*)args.vals;
  const int lane = threadIdx.x;
  if (args.pattern_err && *args.pattern_err) {
    // the pattern failed the device-side validation of this call: nothing
    // is written (its segment bounds cannot be trusted), one count
    if (blockIdx.x == 0 && lane == 0) atomicAdd((unsigned long long*)&args.status[ST_PATTERN], 1ull);
    return;
  }
  for (;;) {
    const int it = next_item(args.work_ctr, &sh.item);
    if (it >= args.n_items) break;
    const int j = args.items ? args.items[it] : it;
    const int a0 = args.rowptr[j];
    const int m = args.rowptr[j + 1] - a0;
    if (m > MMAX || (BWD && args.dout && m != args.dld[j])) {
      // the order exceeds what this launch was sized for (the pattern changed
      // under a cached plan): no computation, NaN over the segment, counted
      for (int r = lane; r < m; r += kWave) {
        if (BWD) atomicAdd(&((VT*)args.ga)[a0 + r], (VT)NAN);
        else ((VT*)args.x)[a0 + r] = (VT)NAN;
      }
      if (lane == 0) atomicAdd((unsigned long long*)&args.status[ST_STALE], 1ull);
      continue;
    }
    const int c = args.cidx[j];
    if (lane < m) sh.R[lane] = args.colind[a0 + lane];
    __syncthreads();
    bool done = false;
    if (args.mixed) {
      float* A = (float*)sh.A;
      float* V = (float*)sh.V;
      gather_small<float, VT, MMAX>(args.rowptr, args.colind, vals, sh.R, m, A);
      const bool conv = jacobi_small<float, MMAX>(A, V, m, sh.lam);
      const double lmin = wave_min(lane < m ? sh.lam[lane] : INFINITY);
      const double lmax = wave_max(lane < m ? sh.lam[lane] : -INFINITY);
      const bool flagged = !conv || !(lmin > 0.0) || lmax > args.kappa_max * lmin;
      if (!flagged) {
        if (BWD)
          finish_backward<float, VT, MMAX, POW>(V, sh, m, c, args.fn, false, (const VT*)args.gx + a0,
                                           (VT*)args.ga, args.rowptr, args.colind,
                                           args.dout ? args.dout + args.doff[j] : nullptr);
        else
          finish_forward<float, VT, MMAX>(V, sh, m, c, args.fn, false, (VT*)args.x + a0);
        done = true;
      } else if (lane == 0) {
        atomicAdd((unsigned long long*)&args.status[ST_FALLBACK], 1ull);
      }
      __syncthreads();
    }
    if (!done) {
      double* A = sh.A;
      double* V = sh.V;
      gather_small<double, VT, MMAX>(args.rowptr, args.colind, vals, sh.R, m, A);
      const bool conv = jacobi_small<double, MMAX>(A, V, m, sh.lam);
      const double lmin = wave_min(lane < m ? sh.lam[lane] : INFINITY);
      const bool nonpos = !(lmin > 0.0);
      const bool bad = nonpos || !conv;
      if (lane == 0) {
        if (nonpos) atomicAdd((unsigned long long*)&args.status[ST_NONPOS], 1ull);
        if (!conv) atomicAdd((unsigned long long*)&args.status[ST_UNCONV], 1ull);
      }
      if (BWD)
        finish_backward<double, VT, MMAX, POW>(V, sh, m, c, args.fn, bad, (const VT*)args.gx + a0,
                                          (VT*)args.ga, args.rowptr, args.colind,
                                          args.dout ? args.dout + args.doff[j] : nullptr);
      else
        finish_forward<double, VT, MMAX>(V, sh, m, c, args.fn, bad, (VT*)args.x + a0);
    }
    if (lane == 0) atomicAdd((unsigned long long*)&args.status[ST_DONE], 1ull);
  }
}

template <class VT, bool BWD, bool POW>
static hipError_t dispatch_small(const SmallArgs& a, hipStream_t s) {
  const dim3 grid(a.grid), block(64);
  if (a.mmax <= 16)
    hipLaunchKernelGGL((k_small<VT, 16, BWD, POW>), grid, block, 0, s, a);
  else if (a.mmax <= 32)
    hipLaunchKernelGGL((k_small<VT, 32, BWD, POW>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k_small<VT, 64, BWD, POW>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <class VT>
static hipError_t dispatch_small_fn(const SmallArgs& a, hipStream_t s) {
  if (a.gx == nullptr) return dispatch_small<VT, false, false>(a, s);
  if (a.fn.kind == FN_POWER) return dispatch_small<VT, true, true>(a, s);
  return dispatch_small<VT, true, false>(a, s);
}

hipError_t launch_small(const SmallArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.mmax > 64) return hipErrorInvalidValue;
  return a.vdtype == 0 ? dispatch_small_fn<double>(a, s) : dispatch_small_fn<float>(a, s);
}

}  // namespace submat
