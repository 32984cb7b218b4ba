// k-point sampling: checks of the density matrix per Born-von Karman offset,
// and the combination of the two real passes of a complex density matrix.
//
// With a k mesh of nk0 x nk1 x nk2 points the density matrix of two orbitals
// depends only on the offset of their cells modulo the BvK supercell of as
// many cells (Methods: the k-sum definition of D, Eq. Eexx).  The caller
// gives it per offset, Dk[r][nt][nt] with r = r0 + nk0 (r1 + nk1 r2), and the
// kernels read it there directly (d_block): the block of two supercell atoms
// is that of their cells' offset.
#include <algorithm>

#include "lrx_internal.h"

namespace lrx {

namespace {

constexpr int kNT = 256;

__device__ inline bool close_rel(double x, double y) { return fabs(x - y) <= 1e-12 * (fabs(x) + fabs(y)); }

// D(-r) = D(r)^H: Re Dk[-r][j][i] = Re Dk[r][i][j] and Im Dk[-r][j][i] =
// -Im Dk[r][i][j], each pair checked once (from the element that comes first
// in memory; an element that is its own partner is not checked).
__global__ void k_val_herm(const double* __restrict__ Dre, const double* __restrict__ Dim, int nk0, int nk1, int nk2,
                           int64_t nt, int* err) {
  const int64_t nn = nt * nt, n = (int64_t)nk0 * nk1 * nk2 * nn;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / nn);
    const int64_t ij = e - (int64_t)r * nn, i = ij / nt, j = ij - i * nt;
    const int r0 = r % nk0, r1 = (r / nk0) % nk1, r2 = r / (nk0 * nk1);
    const int m = (nk0 - r0) % nk0 + nk0 * ((nk1 - r1) % nk1 + nk1 * ((nk2 - r2) % nk2));
    const int64_t f = (int64_t)m * nn + j * nt + i;   // the partner element
    if (f <= e) continue;
    if (!close_rel(Dre[e], Dre[f])) bad = 1;
    if (Dim && !close_rel(Dim[e], -Dim[f])) bad = 1;
  }
  if (bad) atomicOr(err, kErrDSym);
}

__global__ void k_sub_from(const double* __restrict__ keep, double* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = keep[i] - x[i];
}

}  // namespace

void launch_validate_herm(const double* Dre, const double* Dim, const int* nk, int64_t nt, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_val_herm, dim3(2048), dim3(kNT), 0, s, Dre, Dim, nk[0], nk[1], nk[2], nt, err);
}

void launch_sub_from(const double* keep, double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((n + kNT - 1) / kNT, 4096);
  hipLaunchKernelGGL(k_sub_from, dim3(g), dim3(kNT), 0, s, keep, x, n);
}

}  // namespace lrx
