// k-point sampling: the density matrix of the Born-von Karman supercell.
//
// With a k mesh of nk0 x nk1 x nk2 points the density matrix of two orbitals
// depends only on the offset of their cells modulo the BvK supercell of as
// many cells (Methods: the k-sum definition of D, Eq. Eexx).  The caller
// gives it per offset, Dk[r][nt][nt] with r = r0 + nk0 (r1 + nk1 r2); the
// contraction kernels read the supercell matrix
//   Dsc[(t, i)][(u, j)] = Dk[u - t][i][j]   (atom (t, i) = cell t, orbital i)
// as a dense row-major [nk nt][nk nt] block-circulant matrix, written here
// once per set of tensors.  One workgroup per supercell row; the row's nk
// blocks are contiguous rows of Dk, copied with coalesced loads and stores.
#include <algorithm>

#include "lrx_internal.h"

namespace lrx {

namespace {

constexpr int kNT = 256;

__global__ void __launch_bounds__(kNT) k_bvk_expand(const double* __restrict__ Dk, int nk0, int nk1, int nk2,
                                                    int64_t nt, double* __restrict__ Dsc) {
  const int ncell = nk0 * nk1 * nk2;
  const int64_t ns = (int64_t)ncell * nt;
  for (int64_t row = blockIdx.x; row < ns; row += gridDim.x) {
    const int t = (int)(row / nt);
    const int64_t i = row - (int64_t)t * nt;
    const int t0 = t % nk0, t1 = (t / nk0) % nk1, t2 = t / (nk0 * nk1);
    double* out = Dsc + row * ns;
    for (int u = 0; u < ncell; ++u) {
      const int u0 = u % nk0, u1 = (u / nk0) % nk1, u2 = u / (nk0 * nk1);
      const int r = (u0 - t0 + nk0) % nk0 + nk0 * ((u1 - t1 + nk1) % nk1 + nk1 * ((u2 - t2 + nk2) % nk2));
      const double* src = Dk + ((int64_t)r * nt + i) * nt;
      double* dst = out + (int64_t)u * nt;
      for (int64_t j = threadIdx.x; j < nt; j += kNT) dst[j] = src[j];
    }
  }
}

__global__ void k_sub_from(const double* __restrict__ keep, double* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = keep[i] - x[i];
}

}  // namespace

void launch_bvk_expand(const double* Dk, const int* nk, int64_t nt, double* Dsc, hipStream_t s) {
  const int64_t rows = (int64_t)nk[0] * nk[1] * nk[2] * nt;
  const unsigned g = (unsigned)std::min<int64_t>(rows, 65536);
  hipLaunchKernelGGL(k_bvk_expand, dim3(g), dim3(kNT), 0, s, Dk, nk[0], nk[1], nk[2], nt, Dsc);
}

void launch_sub_from(const double* keep, double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((n + kNT - 1) / kNT, 4096);
  hipLaunchKernelGGL(k_sub_from, dim3(g), dim3(kNT), 0, s, keep, x, n);
}

}  // namespace lrx
