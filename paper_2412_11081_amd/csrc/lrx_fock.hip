// The exact-exchange Hamiltonian H^X = dE/dD (Eq. Exx2: the term of the
// energy's variation that comes from the density matrix; it equals
// -sum_{kl} (ik|jl) D_kl), from the same folded tensors as the forces.
//
// With Q^{AFB}[beta][a f] = sum_alpha Vf(A,B)[alpha][beta] Cf(A,F)[alpha][a f]
// the energy of the folded form is E = -sum_{A,F,B} <Q^{AFB}, X^{AFB}>, with
//   X^{AFB}[beta][a f] = sum_b D(A,B)[a][b] H(B,F)[b][beta][f]
//                      + sum_b H(B,A)[b][beta][a] D(F,B)[f][b],
//   H(B,X)[b][beta][x] = sum_G sum_g Cf(B,G)[beta][b][g] D(G,X)[g][x].
// Its gradient G = dE/dD over the elements of D then has three parts:
//   G1(A,B)[a][b] = -sum_F sum_{beta,f} Q^{AFB}[beta][a f] H(B,F)[b][beta][f]
//   G2(F,B)[f][b] = -sum_A sum_{beta,a} Q^{AFB}[beta][a f] H(B,A)[b][beta][a]
//   G3(G,X)[g][x] =  sum_B sum_{beta,b} Cf(B,G)[beta][b][g] Hbar(B,X)[b][beta][x]
// with the adjoint of H
//   Hbar(B,X)[b][beta][x] = -sum_{A: F = X} sum_a Q^{AXB}[beta][a x] D(A,B)[a][b]
//                           -sum_{F: A = X} sum_f Q^{XFB}[beta][x f] D(F,B)[f][b].
// The folded form reads D(G,X) where the quartet form reads D(X,G)^T, the same
// numbers for a symmetric D; the symmetric part of G is therefore the
// derivative of the quartet form, and that derivative is symmetric: H^X =
// (G + G^T) / 2.  Screened D pairs are zero in E, so H^X is zero there, and
// E = <H^X, D> / 2 (a quadratic form) is returned beside it.
//
// Kernels (FP64):
//   k_hx_slot   one workgroup per needed H slot (B,X): Hbar(B,X) and the
//               D block (X,B) of G1 + G2.  Q tiles of 16 beta rows on the
//               matrix cores (operands from global memory, result in LDS),
//               the contractions with D and H on the vector units.
//   k_hx_g3     one workgroup per D block (G,X): G3 over the C partners B.
//   k_hx_final  32 x 32 tiles: (G + G^T) / 2 on kept D pairs, and the tile's
//               share of <H^X, D> / 2; k_hx_sum adds the shares in order.
// No atomics: every output element has one writer, so two calls agree bit
// for bit.
#include <hip/hip_runtime.h>

#include "lrx_internal.h"

namespace lrx {

namespace {

constexpr int kHxNT = 256;
constexpr int kGPer = kMaxNao * kMaxNao / kHxNT;         // D-block elements per thread
// Hbar elements of a beta tile per thread, for NAO counts up to NMAX
template <int NMAX>
constexpr int hb_per() { return (16 * NMAX * NMAX + kHxNT - 1) / kHxNT; }

typedef double d4 __attribute__((ext_vector_type(4)));

// position of atom x among the sorted partners list[r0..r1), or -1
__device__ inline int find_partner(const int* __restrict__ list, int r0, int r1, int x) {
  while (r0 < r1) {
    const int m = (r0 + r1) >> 1;
    const int v = list[m];
    if (v == x) return m;
    if (v < x) r0 = m + 1; else r1 = m;
  }
  return -1;
}

// Q[beta][k] (LDS, row stride K1) for the 16 rows beta = 16 t + 0..15 of B:
//   Q[beta][k] = sum_alpha Vf[alpha][16 t + beta] Cf[alpha][k],
// Vf rows ldv apart (B's ABFs padded to 16, zero padding), Cf rows K1 apart.
// f64 16x16x4 MFMA: lane (q, g) gives A[m = q][k = g] = Vf[4 s + g][16 t + q]
// and B[k = g][n = q] = Cf[4 s + g][16 j + q]; result i is row g + 4 i.
__device__ void q_tile(const double* __restrict__ Vf, int ldv, const double* __restrict__ Cf, int mA, int K1, int t,
                       double* Q, int w, int q, int g) {
  const int nj = (K1 + 15) >> 4, ns = (mA + 3) >> 2;
  for (int j = w; j < nj; j += kHxNT / 64) {
    const int c = 16 * j + q;
    d4 acc = {0, 0, 0, 0};
    for (int s = 0; s < ns; ++s) {
      const int al = 4 * s + g;
      const double a = al < mA ? Vf[(int64_t)al * ldv + 16 * t + q] : 0.0;
      const double b = (al < mA && c < K1) ? Cf[(int64_t)al * K1 + c] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (c < K1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Q[(g + 4 * i) * K1 + c] = acc[i];
    }
  }
}

template <int NMAX>
__global__ void __launch_bounds__(kHxNT) k_hx_slot(Dev d, double* __restrict__ Hbar, double* __restrict__ G12) {
  constexpr int kHbPer = hb_per<NMAX>();
  extern __shared__ double Q[];   // [16][K1], K1 <= the largest n_A n_X of the structure
  const int s = blockIdx.x;
  if (!d.need[s]) return;
  const int N = d.N;
  const int64_t nt = d.ntot;
  const int B = d.slotB[s], X = d.slotX[s];
  const int mB = d.nabf[B], nB = d.nao[B], nX = d.nao[X];
  const int ldv = (mB + 15) & ~15, nT = ldv >> 4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  const int nHb = 16 * nB * nX, nG = nX * nB;
  double gacc[kGPer];
#pragma unroll
  for (int k = 0; k < kGPer; ++k) gacc[k] = 0.0;
  // the V pair (X,B), whose C partners F give the second kind of term
  const int vpX = find_partner(d.vpB, d.vpRow[X], d.vpRow[X + 1], B);
  const bool kindB = vpX >= 0 && (d.aliveV[vpX] & 1);
  for (int t = 0; t < nT; ++t) {
    double hb[kHbPer];
#pragma unroll
    for (int k = 0; k < kHbPer; ++k) hb[k] = 0.0;
    // first kind: triples (A, X, B), X a C partner of A
    for (int i = d.cpRow[X]; i < d.cpRow[X + 1]; ++i) {
      const int A = d.cpF[i];
      const int cpA = find_partner(d.cpF, d.cpRow[A], d.cpRow[A + 1], X);
      if (cpA < 0 || !(d.aliveC[cpA] & 1)) continue;
      const int vpA = find_partner(d.vpB, d.vpRow[A], d.vpRow[A + 1], B);
      if (vpA < 0 || !(d.aliveV[vpA] & 1)) continue;
      const int nA = d.nao[A], K1 = nA * nX;
      q_tile(d.Vf + d.vfOff[vpA], ldv, d.Cf + d.cfOff[cpA], d.nabf[A], K1, t, Q, w, q, g);
      __syncthreads();
      if (d.keepD[(int64_t)A * N + B]) {
        // Hbar[b][beta][x] -= sum_a D(A,B)[a][b] Q[beta][a nX + x]
        const double* Dab = d.D + d.ao[A] * nt + d.ao[B];
#pragma unroll
        for (int k = 0; k < kHbPer; ++k) {
          const int e = tid + kHxNT * k;
          if (e < nHb) {
            const int x = e % nX, r = e / nX, be = r & 15, b = r >> 4;
            double acc = 0.0;
            for (int a = 0; a < nA; ++a) acc += Dab[(int64_t)a * nt + b] * Q[be * K1 + a * nX + x];
            hb[k] -= acc;
          }
        }
      }
      // G2(X,B)[x][b] -= sum_{beta,a} Q[beta][a nX + x] H(B,A)[b][beta][a]
      const int sBA = d.hSlotMap[(int64_t)B * N + A];
      const double* Hba = d.H + d.hOff[sBA] + (int64_t)t * nB * 16 * nA;
#pragma unroll
      for (int k = 0; k < kGPer; ++k) {
        const int e = tid + kHxNT * k;
        if (e < nG) {
          const int x = e / nB, b = e % nB;
          double acc = 0.0;
          for (int be = 0; be < 16; ++be) {
            const double* h = Hba + (b * 16 + be) * nA;
            const double* qq = Q + be * K1 + x;
            for (int a = 0; a < nA; ++a) acc += qq[a * nX] * h[a];
          }
          gacc[k] -= acc;
        }
      }
      __syncthreads();
    }
    // second kind: triples (X, F, B) over the C partners F of X
    if (kindB) {
      for (int i = d.cpRow[X]; i < d.cpRow[X + 1]; ++i) {
        if (!(d.aliveC[i] & 1)) continue;
        const int F = d.cpF[i], nF = d.nao[F], K1 = nX * nF;
        q_tile(d.Vf + d.vfOff[vpX], ldv, d.Cf + d.cfOff[i], d.nabf[X], K1, t, Q, w, q, g);
        __syncthreads();
        if (d.keepD[(int64_t)F * N + B]) {
          // Hbar[b][beta][x] -= sum_f Q[beta][x nF + f] D(F,B)[f][b]
          const double* Dfb = d.D + d.ao[F] * nt + d.ao[B];
#pragma unroll
          for (int k = 0; k < kHbPer; ++k) {
            const int e = tid + kHxNT * k;
            if (e < nHb) {
              const int x = e % nX, r = e / nX, be = r & 15, b = r >> 4;
              double acc = 0.0;
              const double* qq = Q + be * K1 + x * nF;
              for (int f = 0; f < nF; ++f) acc += qq[f] * Dfb[(int64_t)f * nt + b];
              hb[k] -= acc;
            }
          }
        }
        // G1(X,B)[x][b] -= sum_{beta,f} Q[beta][x nF + f] H(B,F)[b][beta][f]
        const int sBF = d.hSlotMap[(int64_t)B * N + F];
        const double* Hbf = d.H + d.hOff[sBF] + (int64_t)t * nB * 16 * nF;
#pragma unroll
        for (int k = 0; k < kGPer; ++k) {
          const int e = tid + kHxNT * k;
          if (e < nG) {
            const int x = e / nB, b = e % nB;
            double acc = 0.0;
            for (int be = 0; be < 16; ++be) {
              const double* h = Hbf + (b * 16 + be) * nF;
              const double* qq = Q + be * K1 + x * nF;
              for (int f = 0; f < nF; ++f) acc += qq[f] * h[f];
            }
            gacc[k] -= acc;
          }
        }
        __syncthreads();
      }
    }
    // the beta tile of Hbar(B,X), laid out as the H slot: [b][beta][x]
    double* hout = Hbar + d.hOff[s] + (int64_t)t * nHb;
#pragma unroll
    for (int k = 0; k < kHbPer; ++k) {
      const int e = tid + kHxNT * k;
      if (e < nHb) hout[e] = hb[k];
    }
  }
  // the D block (X,B) of G1 + G2 (this workgroup is its only writer)
#pragma unroll
  for (int k = 0; k < kGPer; ++k) {
    const int e = tid + kHxNT * k;
    if (e < nG) {
      const int x = e / nB, b = e % nB;
      G12[(d.ao[X] + x) * nt + d.ao[B] + b] = gacc[k];
    }
  }
}

// G3(G,X)[g][x] = sum_B sum_{beta,b} Cf(B,G)[beta][b][g] Hbar(B,X)[b][beta][x]
// over the C pairs (B,G) with a value-list block and the needed slots (B,X).
__global__ void __launch_bounds__(kHxNT) k_hx_g3(Dev d, const double* __restrict__ Hbar, double* __restrict__ G3) {
  const int N = d.N;
  const int G = blockIdx.x / N, X = blockIdx.x % N;
  const int64_t nt = d.ntot;
  const int nG = d.nao[G], nX = d.nao[X], n = nG * nX;
  const int tid = threadIdx.x;
  double acc[kGPer];
#pragma unroll
  for (int k = 0; k < kGPer; ++k) acc[k] = 0.0;
  for (int i = d.cpRow[G]; i < d.cpRow[G + 1]; ++i) {
    const int B = d.cpF[i];
    const int sl = d.hSlotMap[(int64_t)B * N + X];
    if (sl < 0 || !d.need[sl]) continue;
    const int cp = find_partner(d.cpF, d.cpRow[B], d.cpRow[B + 1], G);
    if (cp < 0 || !(d.aliveC[cp] & 1)) continue;
    const int mB = d.nabf[B], nB = d.nao[B];
    const double* Cf = d.Cf + d.cfOff[cp];   // [beta][b][g]
    const double* Hb = Hbar + d.hOff[sl];    // [beta / 16][b][beta % 16][x]
#pragma unroll
    for (int k = 0; k < kGPer; ++k) {
      const int e = tid + kHxNT * k;
      if (e < n) {
        const int gg = e / nX, x = e % nX;
        double s = 0.0;
        for (int be = 0; be < mB; ++be) {
          const double* c = Cf + (int64_t)be * nB * nG + gg;
          const double* h = Hb + ((int64_t)(be >> 4) * nB * 16 + (be & 15)) * nX + x;
          for (int b = 0; b < nB; ++b) s += c[b * nG] * h[b * 16 * nX];
        }
        acc[k] += s;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kGPer; ++k) {
    const int e = tid + kHxNT * k;
    if (e < n) G3[(d.ao[G] + e / nX) * nt + d.ao[X] + e % nX] = acc[k];
  }
}

// atom of AO row i (d.ao is sorted)
__device__ inline int atom_of(const Dev& d, int64_t i) {
  int lo = 0, hi = d.N;   // ao[lo] <= i < ao[hi]
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (d.ao[m] <= i) lo = m; else hi = m;
  }
  return lo;
}

constexpr int kFT = 32;   // final tiles: 32 x 32 elements, 256 threads

__global__ void __launch_bounds__(kHxNT) k_hx_final(Dev d, const double* __restrict__ G12,
                                                     const double* __restrict__ G3, double* __restrict__ Hx,
                                                     double* __restrict__ Etile) {
  __shared__ double tr[kFT][kFT + 1];
  __shared__ int ai[kFT], aj[kFT];
  __shared__ double red[kHxNT / 64];
  const int64_t nt = d.ntot;
  const int ntile = (int)((nt + kFT - 1) / kFT);
  const int ti = blockIdx.x / ntile, tj = blockIdx.x % ntile;
  const int64_t i0 = (int64_t)ti * kFT, j0 = (int64_t)tj * kFT;
  const int tid = threadIdx.x;
  if (tid < kFT) ai[tid] = i0 + tid < nt ? atom_of(d, i0 + tid) : -1;
  else if (tid < 2 * kFT) aj[tid - kFT] = j0 + tid - kFT < nt ? atom_of(d, j0 + tid - kFT) : -1;
  // the transposed tile: (G12 + G3)[j0 + r][i0 + c] into tr[c][r]
  for (int e = tid; e < kFT * kFT; e += kHxNT) {
    const int r = e / kFT, c = e % kFT;
    const int64_t j = j0 + r, i = i0 + c;
    tr[c][r] = (j < nt && i < nt) ? G12[j * nt + i] + G3[j * nt + i] : 0.0;
  }
  __syncthreads();
  double es = 0.0;
  for (int e = tid; e < kFT * kFT; e += kHxNT) {
    const int r = e / kFT, c = e % kFT;
    const int64_t i = i0 + r, j = j0 + c;
    if (i >= nt || j >= nt) continue;
    const bool kept = d.keepD[(int64_t)ai[r] * d.N + aj[c]] != 0;
    const double h = kept ? 0.5 * ((G12[i * nt + j] + G3[i * nt + j]) + tr[r][c]) : 0.0;
    Hx[i * nt + j] = h;
    es += h * d.D[i * nt + j];
  }
  // fixed-order sum of the tile's share of <H^X, D> / 2
  for (int o = 32; o > 0; o >>= 1) es += __shfl_down(es, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = es;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < kHxNT / 64; ++k) t += red[k];
    Etile[blockIdx.x] = 0.5 * t;
  }
}

__global__ void __launch_bounds__(1024) k_hx_sum(const double* __restrict__ Etile, int64_t n, double* __restrict__ E) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += Etile[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[k];
    *E = t;
  }
}

__global__ void k_fill_f64(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace

int64_t hx_tiles(int64_t ntot) {
  const int64_t t = (ntot + kFT - 1) / kFT;
  return t * t;
}

void launch_hx(const Dev& d, const HxBufs& b, hipStream_t s, hipEvent_t* ev) {
  const int64_t nt = d.ntot;
  hipLaunchKernelGGL(k_fill_f64, dim3(2048), dim3(256), 0, s, b.G12, nt * nt);
  if (d.nSlot > 0) {
    // the Q tile in LDS: 16 rows of at most kMaxNao^2 doubles (128 KiB)
    const size_t lds = sizeof(double) * 16 * b.kmax;
    auto go = [&](auto kern) {
      if (lds > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(kern, dim3((unsigned)d.nSlot), dim3(kHxNT), lds, s, d, b.Hbar, b.G12);
    };
    if (b.nmax <= 16)
      go(k_hx_slot<16>);
    else if (b.nmax <= 24)
      go(k_hx_slot<24>);
    else
      go(k_hx_slot<kMaxNao>);
  }
  if (ev) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(k_hx_g3, dim3((unsigned)((int64_t)d.N * d.N)), dim3(kHxNT), 0, s, d, (const double*)b.Hbar,
                     b.G3);
  if (ev) (void)hipEventRecord(ev[1], s);
  const int64_t nf = hx_tiles(nt);
  hipLaunchKernelGGL(k_hx_final, dim3((unsigned)nf), dim3(kHxNT), 0, s, d, (const double*)b.G12,
                     (const double*)b.G3, b.Hx, b.Etile);
  hipLaunchKernelGGL(k_hx_sum, dim3(1), dim3(1024), 0, s, (const double*)b.Etile, nf, b.E);
  if (ev) (void)hipEventRecord(ev[2], s);
}

}  // namespace lrx
