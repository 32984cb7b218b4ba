// Preparation of the C tensor and its derivative from V and the three-centre
// integrals (Eq. C_VA; the gradient after Eq. V_inverse).  For a C key
// (A,F,R) the LRI coefficients of the AO pair (A a, F f) on the ABFs of both
// atoms solve
//
//   M [C^A; C^F] = [(P_A|phi_A phi_F); (P_F|phi_A phi_F)],
//   M = [[V(A,A,0), V(A,F,R)], [V(A,F,R)^T, V(F,F,0)]]   (symmetric positive definite),
//
// and the key's C block is C^A (the first mA rows).  The on-site key (A,A,0)
// uses the ABFs of A alone.  With dV the derivative of V(A,F,R) and dP that
// of the integrals (both with respect to the key's displacement r),
//
//   M dC = -[[0, dV], [dV^T, 0]] [C^A; C^F] + dP,
//
// from the derivative of M^-1 (Eq. V_inverse); on-site blocks do not move
// with their atom, so their dC is zero.
//
// One workgroup per key (a grid of one workgroup per CU takes the keys in
// turn).  For n <= 201 the lower triangle of M is assembled in LDS (packed
// rows, n (n + 1) / 2 doubles, at most 158.6 KiB), factorised in place,
// M = L L^T (right-looking, the trailing update spread over the
// workgroup), and inverted in place, L -> L^-1 (column by column from the
// last, each column a triangular product with the part already inverted,
// eight threads per row).  Larger M go through the workgroup's slice of a
// device workspace: a left-looking factorisation (one thread per row of
// the current column) and L^-1 by forward substitution (one thread per
// column).  M^-1 = L^-T L^-1 then runs on the matrix cores.  The products
// with the right-hand sides -- C = M^-1 (P|phi phi), the derivative
// columns -dV C + dP, and
// dC = M^-1 W -- are GEMMs on the matrix cores.  FP64 throughout; no atomics
// but the error flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lrx.h"

namespace {

constexpr int kPT = 512;
constexpr int kTriMax = 201;                             // largest n whose packed triangle fits the LDS
constexpr int kTriLds = kTriMax * (kTriMax + 1) / 2;     // doubles (162408 bytes)

struct PrepItem {
  int A, F, onsite;
  int64_t t;      // element offset of the integrals (derivatives at 3 t)
  int64_t vAA, vFF, vAF;   // element offsets of V(A,A,0), V(F,F,0), V(A,F,R)
  int64_t c;      // element offset of the output C block (derivatives at 3 c)
};

// L L^T = M for the n x n matrix at M (row-major, in place, lower triangle);
// returns false when a pivot is not positive
__device__ bool cholesky(double* M, int n) {
  const int tid = threadIdx.x;
  bool ok = true;
  for (int j = 0; j < n; ++j) {
    const double* rj = M + (int64_t)j * n;
    for (int i = j + tid; i < n; i += kPT) {
      double* ri = M + (int64_t)i * n;
      double s0 = ri[j], s1 = 0, s2 = 0, s3 = 0;
      int k = 0;
      for (; k + 4 <= j; k += 4) {
        s0 -= ri[k] * rj[k];
        s1 -= ri[k + 1] * rj[k + 1];
        s2 -= ri[k + 2] * rj[k + 2];
        s3 -= ri[k + 3] * rj[k + 3];
      }
      for (; k < j; ++k) s0 -= ri[k] * rj[k];
      ri[j] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    const double djj = rj[j];
    ok = ok && djj > 0.0;
    const double d = djj > 0.0 ? sqrt(djj) : 1.0;
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += kPT) M[(int64_t)i * n + j] /= d;
    if (tid == 0) M[(int64_t)j * n + j] = d;
    __syncthreads();
  }
  return ok;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// Y = L^-1 (lower triangular, n x n, row-major at Y) by forward substitution,
// one thread per column
__device__ void invert_lower(const double* L, int n, double* Y) {
  for (int c = threadIdx.x; c < n; c += kPT) {
    for (int i = 0; i < c; ++i) Y[(int64_t)i * n + c] = 0.0;
    Y[(int64_t)c * n + c] = 1.0 / L[(int64_t)c * n + c];
    for (int i = c + 1; i < n; ++i) {
      const double* li = L + (int64_t)i * n;
      double s0 = 0, s1 = 0;
      int k = c;
      for (; k + 2 <= i; k += 2) {
        s0 -= li[k] * Y[(int64_t)k * n + c];
        s1 -= li[k + 1] * Y[(int64_t)(k + 1) * n + c];
      }
      for (; k < i; ++k) s0 -= li[k] * Y[(int64_t)k * n + c];
      Y[(int64_t)i * n + c] = (s0 + s1) / li[i];
    }
  }
}

// element (i, k), k <= i, of a packed lower triangle
__device__ inline int tri(int i, int k) { return i * (i + 1) / 2 + k; }

// L L^T = M for the packed lower triangle T (LDS) of an n x n matrix, n <=
// kTriMax, in place, right-looking: column j is scaled by the root of its
// updated pivot, then the trailing triangle takes the rank-one update
// T(i,k) -= L(i,j) L(k,j), j < k <= i, eight threads per row; returns
// false when a pivot is not positive
__device__ bool cholesky_tri(double* T, int n) {
  const int tid = threadIdx.x, sub = tid & 7;
  bool ok = true;
  for (int j = 0; j < n; ++j) {
    const double djj = T[tri(j, j)];
    ok = ok && djj > 0.0;
    const double d = djj > 0.0 ? sqrt(djj) : 1.0;
    __syncthreads();   // every thread has read the pivot
    for (int i = j + 1 + tid; i < n; i += kPT) T[tri(i, j)] /= d;
    if (tid == 0) T[tri(j, j)] = d;
    __syncthreads();
    for (int i = j + 1 + (tid >> 3); i < n; i += kPT / 8) {
      const double lij = T[tri(i, j)];
      double* ri = T + tri(i, 0);
      for (int k = j + 1 + sub; k <= i; k += 8) ri[k] -= lij * T[tri(k, j)];
    }
    __syncthreads();
  }
  return ok;
}

// L -> L^-1 for the packed lower triangle T (LDS), in place: for j from the
// last column down, Y(j,j) = 1 / L(j,j) and Y(i,j) = -Y(j,j) sum_{j<k<=i}
// Y(i,k) L(k,j) for i > j (the columns right of j already hold Y); eight
// threads per row take every eighth k and add their partial sums with lane
// shuffles, 64 rows per pass
__device__ void invert_tri(double* T, int n) {
  static_assert(kTriMax - 1 <= 4 * (kPT / 8), "four passes of kPT / 8 rows");
  const int tid = threadIdx.x, sub = tid & 7;
  for (int j = n - 1; j >= 0; --j) {
    const double yjj = 1.0 / T[tri(j, j)];
    double t[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = j + 1 + (tid >> 3) + (kPT / 8) * p;
      double acc = 0.0;
      if (i < n) {
        const double* yi = T + tri(i, 0);
        for (int k = j + 1 + sub; k <= i; k += 8) acc += yi[k] * T[tri(k, j)];
      }
      t[p] = acc;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int o = 4; o > 0; o >>= 1) t[p] += __shfl_xor(t[p], o, 64);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = j + 1 + (tid >> 3) + (kPT / 8) * p;
      if (i < n && sub == 0) T[tri(i, j)] = -yjj * t[p];
    }
    if (tid == 0) T[tri(j, j)] = yjj;
    __syncthreads();
  }
}

// C[i][j] = alpha sum_k A(i,k) B(k,j) (+ Cadd[i][j]) for i < M, j < N on the
// matrix cores; A(i,k) = A[i sai + k sak], B(k,j) = B[k sbk + j sbj].  A
// wave forms one 32 x 32 block at (i0, j0), four 16 x 16 tiles that share
// their A and B fragments; f64 16x16x4 MFMA with lane (q, g):
// A[m = q][k = g], B[k = g][n = q], result r is row g + 4 r.  Operands are
// read from clamped addresses (no branches); the A operand of a k past K is
// zero; rows and columns past M, N are not stored.  The loads of four
// k-steps are issued before their products.
__device__ inline void gemm_block(int M, int N, int K, const double* __restrict__ A, int64_t sai, int64_t sak,
                                  const double* __restrict__ B, int64_t sbk, int64_t sbj, double alpha,
                                  const double* Cadd, int64_t ldadd, double* C, int64_t ldc, int i0, int j0) {
  const int lane = threadIdx.x & 63, q = lane & 15, g = lane >> 4;
  const int ns = (K + 3) >> 2;
  const double* ap[2] = {A + (int64_t)min(i0 + q, M - 1) * sai, A + (int64_t)min(i0 + 16 + q, M - 1) * sai};
  const double* bp[2] = {B + (int64_t)min(j0 + q, N - 1) * sbj, B + (int64_t)min(j0 + 16 + q, N - 1) * sbj};
  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4{0, 0, 0, 0};
  for (int s0 = 0; s0 < ns; s0 += 4) {
    double a[4][2], b[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * (s0 + u) + g, kc = min(k, K - 1);
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const double av = ap[x][(int64_t)kc * sak];
        a[u][x] = k < K ? av : 0.0;
        b[u][x] = bp[x][(int64_t)kc * sbk];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][x], b[u][y], acc[x][y], 0, 0, 0);
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * x + g + 4 * r, j = j0 + 16 * y + q;
        if (i < M && j < N)
          C[(int64_t)i * ldc + j] = alpha * acc[x][y][r] + (Cadd ? Cadd[(int64_t)i * ldadd + j] : 0.0);
      }
}

// one product, its 32 x 32 blocks taken by the workgroup's waves in turn
__device__ void wg_gemm(int M, int N, int K, const double* __restrict__ A, int64_t sai, int64_t sak,
                        const double* __restrict__ B, int64_t sbk, int64_t sbj, double alpha, const double* Cadd,
                        int64_t ldadd, double* C, int64_t ldc) {
  const int w = threadIdx.x >> 6, tm = (M + 31) >> 5, tn = (N + 31) >> 5;
  for (int blk = w; blk < tm * tn; blk += kPT / 64)
    gemm_block(M, N, K, A, sai, sak, B, sbk, sbj, alpha, Cadd, ldadd, C, ldc, 32 * (blk / tn), 32 * (blk % tn));
}

// Mi = L^-T L^-1 for the lower-triangular n x n Y = L^-1 (row-major):
// Mi(i,j) = sum_{k >= max(i,j)} Y[k][i] Y[k][j].  The 32 x 32 blocks on and
// below the diagonal are formed, as in wg_gemm, with their depth starting
// at the block's first row (the terms before it are products with exact
// zeros of Y); a block below the diagonal is also written to its mirror
// position (one writer per element).
__device__ void wg_ltl(int n, const double* __restrict__ Y, double* Mi) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane & 15, g = lane >> 4;
  const int tm = (n + 31) >> 5, ns = (n + 3) >> 2;
  for (int blk = w; blk < tm * (tm + 1) / 2; blk += kPT / 64) {
    int bi = (int)((sqrt(8.0 * blk + 1.0) - 1.0) * 0.5);
    if ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;    // guard the rounding of the root
    if (bi * (bi + 1) / 2 > blk) --bi;
    const int bj = blk - bi * (bi + 1) / 2, i0 = 32 * bi, j0 = 32 * bj;
    const double* ap[2] = {Y + min(i0 + q, n - 1), Y + min(i0 + 16 + q, n - 1)};
    const double* bp[2] = {Y + min(j0 + q, n - 1), Y + min(j0 + 16 + q, n - 1)};
    d4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = d4{0, 0, 0, 0};
    for (int s0 = i0 / 4; s0 < ns; s0 += 4) {
      double a[4][2], b[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 4 * (s0 + u) + g, kc = min(k, n - 1);
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const double av = ap[x][(int64_t)kc * n];
          a[u][x] = k < n ? av : 0.0;
          b[u][x] = bp[x][(int64_t)kc * n];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][x], b[u][y], acc[x][y], 0, 0, 0);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 16 * x + g + 4 * r, j = j0 + 16 * y + q;
          if (i < n && j < n) {
            Mi[(int64_t)i * n + j] = acc[x][y][r];
            if (bi != bj) Mi[(int64_t)j * n + i] = acc[x][y][r];   // a diagonal block holds both
          }
        }
  }
}

// Workspace of a workgroup: L (the factor, in place of M, when n >
// kTriMax), Linv, Minv (each nmax x nmax), then X [n][ld]: C in columns
// [0, K1), the derivative right-hand sides W_x in columns K1 + x K1 + [0,
// K1).  Dynamic LDS: the packed triangle (kTriLds doubles).
__global__ void __launch_bounds__(kPT) k_prep(const PrepItem* __restrict__ items, int nitem, const int* __restrict__ nao,
                                              const int* __restrict__ nabf, const double* __restrict__ Tval,
                                              const double* __restrict__ Tdval, const double* __restrict__ Vval,
                                              const double* __restrict__ Vdval, double* __restrict__ Cval,
                                              double* __restrict__ Cdval, double* __restrict__ ws, int64_t wsStride,
                                              int nmax, int* __restrict__ err) {
  extern __shared__ double tl[];
  double* M = ws + blockIdx.x * wsStride;
  double* Li = M + (int64_t)nmax * nmax;
  double* Mi = Li + (int64_t)nmax * nmax;
  double* X = Mi + (int64_t)nmax * nmax;
  const int tid = threadIdx.x;
  for (int p = blockIdx.x; p < nitem; p += gridDim.x) {
    const PrepItem it = items[p];
    const int mA = nabf[it.A], mF = nabf[it.F], nA = nao[it.A], nF = nao[it.F];
    const int n = it.onsite ? mA : mA + mF, K1 = nA * nF, ld = it.onsite ? K1 : 4 * K1;
    const double* VAA = Vval + it.vAA;
    const double* VFF = Vval + it.vFF;
    const double* VAF = Vval + it.vAF;
    auto mval = [&](int i, int j) {
      if (i < mA) return j < mA ? VAA[i * mA + j] : VAF[i * mF + (j - mA)];
      return j < mA ? VAF[j * mF + (i - mA)] : VFF[(i - mA) * mF + (j - mA)];
    };
    if (n <= kTriMax) {
      // lower triangle in LDS: row i holds j <= i
      for (int e = tid; e < n * (n + 1) / 2; e += kPT) {
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        if (tri(i + 1, 0) <= e) ++i;       // guard the rounding of the root
        if (tri(i, 0) > e) --i;
        tl[e] = mval(i, e - tri(i, 0));
      }
      __syncthreads();
      if (!cholesky_tri(tl, n) && tid == 0) atomicMax(err, 1);
      invert_tri(tl, n);
      for (int64_t e = tid; e < (int64_t)n * n; e += kPT) {
        const int i = (int)(e / n), k = (int)(e % n);
        Li[e] = k <= i ? tl[tri(i, k)] : 0.0;
      }
    } else {
      for (int64_t e = tid; e < (int64_t)n * n; e += kPT) M[e] = mval((int)(e / n), (int)(e % n));
      __syncthreads();
      if (!cholesky(M, n) && tid == 0) atomicMax(err, 1);
      invert_lower(M, n, Li);
    }
    __syncthreads();
    // M^-1 = L^-T L^-1: Mi(i,j) = sum_k Li[k][i] Li[k][j]
    wg_ltl(n, Li, Mi);
    __syncthreads();
    // C = M^-1 (P|phi phi)  [n][K1]
    const double* T = Tval + it.t;
    wg_gemm(n, K1, n, Mi, n, 1, T, K1, 1, 1.0, nullptr, 0, X, ld);
    __syncthreads();
    if (!it.onsite) {
      // W_x = dP_x - [[0, dV_x], [dV_x^T, 0]] C:
      //   rows of A: dP_x[top] - dV_x C[rows of F];  rows of F: dP_x[bottom] - dV_x^T C[rows of A]
      const double* dV = Vdval + 3 * it.vAF;
      const double* dP = Tdval + 3 * it.t;
      // the blocks of the six products (two per x) in one loop over the waves
      const int w = tid >> 6, tn = (K1 + 31) >> 5;
      const int nbA = ((mA + 31) >> 5) * tn, nbF = ((mF + 31) >> 5) * tn;
      for (int blk = w; blk < 3 * (nbA + nbF); blk += kPT / 64) {
        const int x = blk / (nbA + nbF), r = blk % (nbA + nbF);
        const double* dVx = dV + (int64_t)x * mA * mF;
        const double* dPx = dP + (int64_t)x * n * K1;
        double* Wx = X + K1 + (int64_t)x * K1;
        if (r < nbA)
          gemm_block(mA, K1, mF, dVx, mF, 1, X + (int64_t)mA * ld, ld, 1, -1.0, dPx, K1, Wx, ld, 32 * (r / tn),
                     32 * (r % tn));
        else
          gemm_block(mF, K1, mA, dVx, 1, mF, X, ld, 1, -1.0, dPx + (int64_t)mA * K1, K1, Wx + (int64_t)mA * ld, ld,
                     32 * ((r - nbA) / tn), 32 * ((r - nbA) % tn));
      }
      __syncthreads();
      // dC of the key (rows of A): M^-1[rows of A] W_x, straight to the
      // output; the blocks of the three products in one loop
      for (int blk = w; blk < 3 * nbA; blk += kPT / 64) {
        const int x = blk / nbA, r = blk % nbA;
        gemm_block(mA, K1, n, Mi, n, 1, X + K1 + (int64_t)x * K1, ld, 1, 1.0, nullptr, 0,
                   Cdval + 3 * it.c + (int64_t)x * mA * K1, K1, 32 * (r / tn), 32 * (r % tn));
      }
    }
    // the key's block: the rows of A
    for (int64_t e = tid; e < (int64_t)mA * K1; e += kPT) Cval[it.c + e] = X[(e / K1) * ld + e % K1];
    if (it.onsite)
      for (int64_t e = tid; e < (int64_t)3 * mA * K1; e += kPT) Cdval[3 * it.c + e] = 0.0;
    __syncthreads();
  }
}

struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" int lrx_prepare_c(int32_t device, int32_t natom, const int32_t* nao, const int32_t* nabf,
                             const lrx_blocks* V, const lrx_blocks* T, int32_t on_device, double* Cval,
                             double* Cdval, double* flop) {
  if (natom <= 0 || !nao || !nabf || !V || !T || !Cval || !Cdval) return LRX_EINVAL;
  if (T->nblk < 0 || V->nblk <= 0 || !T->first || !T->second || !T->R || !T->off || !V->first || !V->second ||
      !V->R || !V->off || !T->val || !T->dval || !V->val || !V->dval)
    return LRX_EINVAL;
  for (int a = 0; a < natom; ++a)
    if (nao[a] <= 0 || nabf[a] <= 0 || nao[a] > 32 || nabf[a] > 128) return LRX_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LRX_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return LRX_EHIP;
  // V keys -> block
  // the V keys that the C keys use -- V(A,A,0), V(F,F,0), V(A,F,R) -- in a
  // hash, filled in one pass over V's keys (the last of equal keys wins)
  struct Key {
    int f, s, r0, r1, r2;
    bool operator==(const Key& o) const { return f == o.f && s == o.s && r0 == o.r0 && r1 == o.r1 && r2 == o.r2; }
  };
  struct KeyHash {
    size_t operator()(const Key& k) const {   // FNV-1a over the five fields
      uint64_t h = 1469598103934665603ull;
      for (int x : {k.f, k.s, k.r0, k.r1, k.r2}) h = (h ^ (uint32_t)x) * 1099511628211ull;
      return (size_t)h;
    }
  };
  std::unordered_map<Key, int64_t, KeyHash> vk;
  vk.reserve((size_t)(3 * T->nblk + 16));
  for (int64_t b = 0; b < T->nblk; ++b) {
    const int A = T->first[b], F = T->second[b];
    if (A < 0 || A >= natom || F < 0 || F >= natom) return LRX_EINVAL;
    vk.emplace(Key{A, A, 0, 0, 0}, -1);
    vk.emplace(Key{F, F, 0, 0, 0}, -1);
    vk.emplace(Key{A, F, T->R[3 * b], T->R[3 * b + 1], T->R[3 * b + 2]}, -1);
  }
  for (int64_t i = 0; i < V->nblk; ++i) {
    const int f = V->first[i], s = V->second[i];
    if (f < 0 || f >= natom || s < 0 || s >= natom) return LRX_EINVAL;
    const auto q = vk.find(Key{f, s, V->R[3 * i], V->R[3 * i + 1], V->R[3 * i + 2]});
    if (q != vk.end()) q->second = i;
  }
  auto vsize = [&](int64_t i) { return (int64_t)nabf[V->first[i]] * nabf[V->second[i]]; };
  for (int64_t i = 0; i < V->nblk; ++i)
    if (V->off[i] < 0 || V->off[i] + vsize(i) > V->nval) return LRX_EINVAL;
  std::vector<PrepItem> items((size_t)T->nblk);
  int64_t ctot = 0;
  int nmax = 1, ldmax = 1;
  double fl = 0;
  for (int64_t b = 0; b < T->nblk; ++b) {
    PrepItem& it = items[(size_t)b];
    it.A = T->first[b];
    it.F = T->second[b];
    if (it.A < 0 || it.A >= natom || it.F < 0 || it.F >= natom) return LRX_EINVAL;
    const int r0 = T->R[3 * b], r1 = T->R[3 * b + 1], r2 = T->R[3 * b + 2];
    it.onsite = it.A == it.F && r0 == 0 && r1 == 0 && r2 == 0;
    const int mA = nabf[it.A], mF = nabf[it.F], K1 = nao[it.A] * nao[it.F];
    const int n = it.onsite ? mA : mA + mF;
    if (T->off[b] < 0 || T->off[b] + (int64_t)n * K1 > T->nval) return LRX_EINVAL;
    it.t = T->off[b];
    auto find = [&](int f, int s, int a, int c, int d, int64_t* off) {
      const auto q = vk.find(Key{f, s, a, c, d});
      if (q == vk.end() || q->second < 0) return false;
      *off = V->off[q->second];
      return true;
    };
    if (!find(it.A, it.A, 0, 0, 0, &it.vAA)) return LRX_EINVAL;
    it.vFF = it.vAF = it.vAA;
    if (!it.onsite && (!find(it.F, it.F, 0, 0, 0, &it.vFF) || !find(it.A, it.F, r0, r1, r2, &it.vAF)))
      return LRX_EINVAL;
    it.c = ctot;
    ctot += (int64_t)mA * K1;
    nmax = std::max(nmax, n);
    ldmax = std::max(ldmax, it.onsite ? K1 : 4 * K1);
    // Cholesky, the solves, and the products with dV
    fl += (double)n * n * n / 3.0 + 2.0 * n * n * (it.onsite ? K1 : 4 * K1) +
          (it.onsite ? 0.0 : 12.0 * mA * mF * K1);
  }
  if (flop) *flop = fl;
  if (T->nblk == 0) return LRX_OK;
  // the triangle takes a CU's LDS: one workgroup per CU
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu <= 0) ncu = 256;
  const int grid = (int)std::min<int64_t>(T->nblk, ncu);
  const size_t lds = sizeof(double) * kTriLds;
  if (hipFuncSetAttribute((const void*)k_prep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return LRX_EHIP;
  const int64_t wsStride = 3 * (int64_t)nmax * nmax + (int64_t)nmax * ldmax;
  DevMem dItems, dNao, dNabf, dWs, dErr, dTv, dTd, dVv, dVd, dCv, dCd;
  auto alloc = [](DevMem& m, size_t bytes) { return hipMalloc(&m.p, std::max<size_t>(bytes, 8)) == hipSuccess; };
  if (!alloc(dItems, sizeof(PrepItem) * items.size()) || !alloc(dNao, sizeof(int) * natom) ||
      !alloc(dNabf, sizeof(int) * natom) || !alloc(dWs, sizeof(double) * wsStride * grid) ||
      !alloc(dErr, sizeof(int)))
    return LRX_ENOMEM;
  const double *tv = T->val, *td = T->dval, *vv = V->val, *vd = V->dval;
  double *cv = Cval, *cd = Cdval;
  if (!on_device) {
    if (!alloc(dTv, sizeof(double) * T->nval) || !alloc(dTd, sizeof(double) * 3 * T->nval) ||
        !alloc(dVv, sizeof(double) * V->nval) || !alloc(dVd, sizeof(double) * 3 * V->nval) ||
        !alloc(dCv, sizeof(double) * ctot) || !alloc(dCd, sizeof(double) * 3 * ctot))
      return LRX_ENOMEM;
    if (hipMemcpy(dTv.p, T->val, sizeof(double) * T->nval, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dTd.p, T->dval, sizeof(double) * 3 * T->nval, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dVv.p, V->val, sizeof(double) * V->nval, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dVd.p, V->dval, sizeof(double) * 3 * V->nval, hipMemcpyHostToDevice) != hipSuccess)
      return LRX_EHIP;
    tv = (const double*)dTv.p;
    td = (const double*)dTd.p;
    vv = (const double*)dVv.p;
    vd = (const double*)dVd.p;
    cv = (double*)dCv.p;
    cd = (double*)dCd.p;
  }
  if (hipMemcpy(dItems.p, items.data(), sizeof(PrepItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dNao.p, nao, sizeof(int) * natom, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dNabf.p, nabf, sizeof(int) * natom, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(dErr.p, 0, sizeof(int)) != hipSuccess)
    return LRX_EHIP;
  hipLaunchKernelGGL(k_prep, dim3(grid), dim3(kPT), lds, nullptr, (const PrepItem*)dItems.p, (int)T->nblk,
                     (const int*)dNao.p, (const int*)dNabf.p, tv, td, vv, vd, cv, cd, (double*)dWs.p, wsStride, nmax,
                     (int*)dErr.p);
  if (hipGetLastError() != hipSuccess) return LRX_EHIP;
  int herr = 0;
  if (hipMemcpy(&herr, dErr.p, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return LRX_EHIP;
  if (!on_device && (hipMemcpy(Cval, cv, sizeof(double) * ctot, hipMemcpyDeviceToHost) != hipSuccess ||
                     hipMemcpy(Cdval, cd, sizeof(double) * 3 * ctot, hipMemcpyDeviceToHost) != hipSuccess))
    return LRX_EHIP;
  if (herr) return LRX_EINVAL;   // a Coulomb matrix M that is not positive definite
  return LRX_OK;
}
