// Deterministic assembly of the adjoint (the paper has no gradient; this is
// the order-fixed form of the scatter-add of the Daleckii-Krein terms).
//
// Every column j contributes D_j[k][l] to the stored entry (R_j[k], R_j[l]).
// Instead of atomic adds, the columns of one phase (the one-wavefront launch,
// or one chunk of the large-order path) leave their D_j in memory, and this
// kernel forms, for every stored entry q = (r, c),
//   grad_a[q] += sum over j in R_r and R_c, ascending, of D_j[k][l]
// with k the position of r in R_j and l that of c. Both lists are sorted, so
// the common columns come out of one merge in ascending order; k and l come
// from the transpose positions (the entry (j, r) of column j sits at
// tpos[position of (r, j)]), with no search. The entries (r, c) and (c, r)
// add the same terms in the same order, so grad_a stays exactly symmetric,
// and the result does not depend on how the work was scheduled.
#include "common.hpp"
#include "kernels.hpp"

namespace submat {

constexpr int kRedBlock = 256;
constexpr int kRedWaves = kRedBlock / kWave;

// D_j of phase `phase` lies at base + doff[j] (elements for the one-wavefront
// buffer, bytes for a chunk's slab: `bytes_off`), lower triangle column-major
// with leading dimension dld[j]: D[hi][lo] at lo * ld + hi, always FP64.
template <class VT>
__global__ __launch_bounds__(kRedBlock) void k_adjoint_reduce(DetReduceArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  VT* ga = (VT*)a.ga;
  for (int r = blockIdx.x * kRedWaves + wv; r < a.n; r += gridDim.x * kRedWaves) {
    const int r0 = a.rowptr[r], r1 = a.rowptr[r + 1];
    for (int q = r0 + lane; q < r1; q += kWave) {
      const int c = a.colind[q];
      const int c0 = a.rowptr[c], c1 = a.rowptr[c + 1];
      int i = r0, k = c0;
      double sum = 0.0;
      bool any = false;
      while (i < r1 && k < c1) {
        const int ji = a.colind[i], jk = a.colind[k];
        if (ji == jk) {
          if (a.dphase[ji] == a.phase) {
            const int j0 = a.rowptr[ji], ld = a.dld[ji];
            const int pr = a.tpos[i] - j0, pc = a.tpos[k] - j0;
            const int hi = pr > pc ? pr : pc, lo = pr > pc ? pc : pr;
            const int mj = a.rowptr[ji + 1] - j0;
            if ((a.bytes_off ? mj > ld : mj != ld) || pr < 0 || pc < 0 || hi >= mj) {
              sum = NAN;  // column j no longer fits its slot (pattern changed under the plan)
            } else {
              const int64_t o = a.doff[ji];
              const double* D =
                  a.bytes_off ? (const double*)((const char*)a.base + o) : (const double*)a.base + o;
              sum += D[(int64_t)lo * ld + hi];
            }
            any = true;
          }
          ++i;
          ++k;
        } else if (ji < jk) {
          ++i;
        } else {
          ++k;
        }
      }
      if (any) ga[q] = (VT)((double)ga[q] + sum);
    }
  }
}

// The atomic scatter-adds write the lower triangle (column <= row) only;
// afterwards every upper entry q = (r, c), c > r, adds the value of its
// lower mirror (c, r) at tpos[q]. Upper entries hold zero at that point,
// or NaN where a column marked its segment as not computed.
template <class VT>
__global__ __launch_bounds__(kRedBlock) void k_adjoint_mirror(const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ colind,
                                                              const int32_t* __restrict__ tpos, int n, VT* ga) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  for (int r = blockIdx.x * kRedWaves + wv; r < n; r += gridDim.x * kRedWaves) {
    const int r0 = rowptr[r], r1 = rowptr[r + 1];
    for (int q = r0 + lane; q < r1; q += kWave)
      if (colind[q] > r) ga[q] += ga[tpos[q]];
  }
}

hipError_t launch_adjoint_mirror(const int32_t* rowptr, const int32_t* colind, const int32_t* tpos, int n,
                                 void* ga, int vdtype, int num_cus, hipStream_t s) {
  int g = (n + kRedWaves - 1) / kRedWaves;
  if (g > num_cus * 8) g = num_cus * 8;
  if (g < 1) g = 1;
  if (vdtype == 0)
    hipLaunchKernelGGL(k_adjoint_mirror<double>, dim3(g), dim3(kRedBlock), 0, s, rowptr, colind, tpos, n, (double*)ga);
  else
    hipLaunchKernelGGL(k_adjoint_mirror<float>, dim3(g), dim3(kRedBlock), 0, s, rowptr, colind, tpos, n, (float*)ga);
  return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const DetReduceArgs& a, int vdtype, int num_cus, hipStream_t s) {
  int g = (a.n + kRedWaves - 1) / kRedWaves;
  if (g > num_cus * 8) g = num_cus * 8;
  if (g < 1) g = 1;
  if (vdtype == 0)
    hipLaunchKernelGGL(k_adjoint_reduce<double>, dim3(g), dim3(kRedBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_adjoint_reduce<float>, dim3(g), dim3(kRedBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace submat
