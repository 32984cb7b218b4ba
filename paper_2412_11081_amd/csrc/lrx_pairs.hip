// Image-pair enumeration: every (first, second, R) with the lattice image R of
// atom `second` inside the cutoff sphere of atom `first` (Methods: each basis
// function carries a combined index of atom and lattice vector, and every
// two-centre block is a function of the displacement between the two).
//
//   r(f, s, R) = (tau_s - tau_f) + R.L,   kept iff |r|^2 < r_c^2,
//
// with R.L = (R_0 L_0 + R_1 L_1) + R_2 L_2 and |r|^2 = (r_x^2 + r_y^2) + r_z^2
// rounded after every operation (no fused multiply-add), so the decision is
// reproducible bit for bit.  Keys come out sorted by (first, second, R
// lexicographic): a first pass counts each atom pair's images, ordered
// prefix sums give each pair its output range, and a second pass writes its
// images in R order.  No atomics: the output does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lrx.h"

namespace {

constexpr int kNT = 256;

struct Cell {
  double L[9];      // rows a1, a2, a3
  double rc2;
  int span[3];      // R_i in [-span_i, span_i]
  int N;
};

__device__ inline bool inside(const double* __restrict__ tau, const Cell& c, int f, int s, int r0, int r1, int r2) {
  double d2 = 0.0;
  double q[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const double sh = __dadd_rn(__dadd_rn(__dmul_rn((double)r0, c.L[x]), __dmul_rn((double)r1, c.L[3 + x])),
                                __dmul_rn((double)r2, c.L[6 + x]));
    q[x] = __dadd_rn(__dadd_rn(tau[3 * s + x], -tau[3 * f + x]), sh);
  }
  d2 = __dadd_rn(__dadd_rn(__dmul_rn(q[0], q[0]), __dmul_rn(q[1], q[1])), __dmul_rn(q[2], q[2]));
  return d2 < c.rc2;
}

// Exclusive scan of one row of kNT-strided values in place (one workgroup);
// returns the row total.  Ordered: wave ballots are not used, only sums of
// integers, which are exact.
__device__ long long row_scan(long long* v, int n, long long* sh) {
  long long carry = 0;
  for (int i0 = 0; i0 < n; i0 += kNT) {
    const int i = i0 + threadIdx.x;
    const long long x = i < n ? v[i] : 0;
    sh[threadIdx.x] = x;
    __syncthreads();
    // Hillis-Steele inclusive scan over the kNT values
    for (int o = 1; o < kNT; o <<= 1) {
      const long long y = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < n) v[i] = carry + sh[threadIdx.x] - x;
    const long long tot = sh[kNT - 1];
    __syncthreads();
    carry += tot;
  }
  return carry;
}

// Workgroup f: images per second atom s (cnt[f N + s]), then the row's
// exclusive prefix sums in place and the row total.
__global__ void __launch_bounds__(kNT) k_enum_count(const double* __restrict__ tau, Cell c, long long* cnt,
                                                    long long* rowtot) {
  __shared__ long long sh[kNT];
  const int f = blockIdx.x, N = c.N;
  long long* row = cnt + (long long)f * N;
  for (int s = threadIdx.x; s < N; s += kNT) {
    long long k = 0;
    for (int r0 = -c.span[0]; r0 <= c.span[0]; ++r0)
      for (int r1 = -c.span[1]; r1 <= c.span[1]; ++r1)
        for (int r2 = -c.span[2]; r2 <= c.span[2]; ++r2) k += inside(tau, c, f, s, r0, r1, r2);
    row[s] = k;
  }
  __syncthreads();
  const long long tot = row_scan(row, N, sh);
  if (threadIdx.x == 0) rowtot[f] = tot;
}

// One workgroup: exclusive prefix sums of the row totals; total at [N].
__global__ void __launch_bounds__(kNT) k_enum_rows(long long* rowtot, int N) {
  __shared__ long long sh[kNT];
  const long long tot = row_scan(rowtot, N, sh);
  if (threadIdx.x == 0) rowtot[N] = tot;
}

// Workgroup f: each second atom's images in R order at its output range.
__global__ void __launch_bounds__(kNT) k_enum_write(const double* __restrict__ tau, Cell c, const long long* cnt,
                                                    const long long* rowoff, int* first, int* second, int* R) {
  const int f = blockIdx.x, N = c.N;
  for (int s = threadIdx.x; s < N; s += kNT) {
    long long pos = rowoff[f] + cnt[(long long)f * N + s];
    for (int r0 = -c.span[0]; r0 <= c.span[0]; ++r0)
      for (int r1 = -c.span[1]; r1 <= c.span[1]; ++r1)
        for (int r2 = -c.span[2]; r2 <= c.span[2]; ++r2)
          if (inside(tau, c, f, s, r0, r1, r2)) {
            first[pos] = f;
            second[pos] = s;
            R[3 * pos] = r0;
            R[3 * pos + 1] = r1;
            R[3 * pos + 2] = r2;
            ++pos;
          }
  }
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" int lrx_enumerate_pairs(int32_t device, int32_t natom, const double* tau, const double* lattice,
                                   double rcut, int64_t capacity, int32_t* first, int32_t* second, int32_t* R,
                                   int64_t* count) {
  if (natom <= 0 || !tau || !lattice || !count || !(rcut > 0) || !std::isfinite(rcut) || capacity < 0)
    return LRX_EINVAL;
  if (capacity > 0 && (!first || !second || !R)) return LRX_EINVAL;
  for (int i = 0; i < 3 * natom; ++i)
    if (!std::isfinite(tau[i])) return LRX_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LRX_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return LRX_EHIP;
  Cell c{};
  std::memcpy(c.L, lattice, sizeof(c.L));
  const double* L = lattice;
  auto cross = [&](int i, int j, double* o) {
    o[0] = L[3 * i + 1] * L[3 * j + 2] - L[3 * i + 2] * L[3 * j + 1];
    o[1] = L[3 * i + 2] * L[3 * j + 0] - L[3 * i + 0] * L[3 * j + 2];
    o[2] = L[3 * i + 0] * L[3 * j + 1] - L[3 * i + 1] * L[3 * j + 0];
  };
  const double vol = std::fabs(L[0] * (L[4] * L[8] - L[5] * L[7]) - L[1] * (L[3] * L[8] - L[5] * L[6]) +
                               L[2] * (L[3] * L[7] - L[4] * L[6]));
  if (!(vol > 0) || !std::isfinite(vol)) return LRX_EINVAL;
  // images within the cutoff of any atom of the cell: |R_i| <= ceil(r_c / h_i) + 1,
  // h_i the distance between the lattice planes spanned by the other two vectors
  for (int i = 0; i < 3; ++i) {
    double x[3];
    cross((i + 1) % 3, (i + 2) % 3, x);
    const double h = vol / std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double sp = std::ceil(rcut / h) + 1.0;
    if (!(sp < 64)) return LRX_EINVAL;   // cell far smaller than the cutoff
    c.span[i] = (int)sp;
  }
  c.rc2 = rcut * rcut;
  c.N = natom;
  const int64_t nn = (int64_t)natom * natom;
  DevBuf dtau, dcnt, drow, dfirst, dsecond, dR;
  auto alloc = [&](DevBuf& b, size_t bytes) { return hipMalloc(&b.p, std::max<size_t>(bytes, 8)) == hipSuccess; };
  if (!alloc(dtau, sizeof(double) * 3 * natom) || !alloc(dcnt, sizeof(long long) * nn) ||
      !alloc(drow, sizeof(long long) * (natom + 1)))
    return LRX_ENOMEM;
  hipStream_t s = nullptr;
  if (hipMemcpy(dtau.p, tau, sizeof(double) * 3 * natom, hipMemcpyHostToDevice) != hipSuccess) return LRX_EHIP;
  hipLaunchKernelGGL(k_enum_count, dim3(natom), dim3(kNT), 0, s, (const double*)dtau.p, c, (long long*)dcnt.p,
                     (long long*)drow.p);
  hipLaunchKernelGGL(k_enum_rows, dim3(1), dim3(kNT), 0, s, (long long*)drow.p, natom);
  long long total = 0;
  if (hipGetLastError() != hipSuccess) return LRX_EHIP;
  if (hipMemcpy(&total, (long long*)drow.p + natom, sizeof(long long), hipMemcpyDeviceToHost) != hipSuccess)
    return LRX_EHIP;
  *count = total;
  if (total > capacity) return total == 0 ? LRX_OK : LRX_EBUDGET;
  if (total == 0) return LRX_OK;
  if (!alloc(dfirst, sizeof(int) * total) || !alloc(dsecond, sizeof(int) * total) || !alloc(dR, sizeof(int) * 3 * total))
    return LRX_ENOMEM;
  hipLaunchKernelGGL(k_enum_write, dim3(natom), dim3(kNT), 0, s, (const double*)dtau.p, c, (const long long*)dcnt.p,
                     (const long long*)drow.p, (int*)dfirst.p, (int*)dsecond.p, (int*)dR.p);
  if (hipGetLastError() != hipSuccess) return LRX_EHIP;
  if (hipMemcpy(first, dfirst.p, sizeof(int) * total, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(second, dsecond.p, sizeof(int) * total, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(R, dR.p, sizeof(int) * 3 * total, hipMemcpyDeviceToHost) != hipSuccess)
    return LRX_EHIP;
  return LRX_OK;
}
