// Contraction of the LRI exchange energy and its position derivatives
// (Methods, Eqs. exx_expand, Fexx1 and stress) in the Gamma-point folded form:
//
//   H(B,X)    = sum_G Cf(B,G) D(G,X)                                   k_hbuild
//   X^{AFB}   = D_AB H(B,F) + (D_FB H(B,A)) with (a,f) swapped          k_triple
//   Z(A,B)   += Cf(A,F) X^{AFB T},  Y(A,F) += Vf(A,B) X^{AFB}            k_triple
//   E = -<Vf, Z>;  g_v = -<dV_v, Z(A,B)>;  g_c = -2 <dC_c, Y(A,F)>       k_zgrad, k_cgrad
//   F_first += g, F_second -= g;  sigma = -(1/Omega) sum g (x) r         k_forces, k_final
//
// The dense products run on the gfx950 FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  Operand layout per 64-lane wave, lane l,
// q = l & 15, g = l >> 4:  A[m = q][k = g],  B[k = g][n = q];  element i of
// the result in lane l is D[g + 4 i][q].
#include "lrx_internal.h"

namespace lrx {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kNT = 256;
constexpr int kWaves = kNT / 64;
constexpr int kMaxJW = (kChunkCols / 16 + kWaves - 1) / kWaves;   // column tiles per wave
constexpr int kXS = kChunkCols + 1;                                // odd LDS row stride (doubles)
constexpr int kMaxK = 4096;                                        // concatenated H-build depth

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0;
    for (int i = 0; i < nw; ++i) r += sh[i];
    sh[nw] = r;
  }
  __syncthreads();
  return sh[nw];
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Map consecutive logical work items to the same XCD so the units of
// one atom A (which share H(., A) and Vf(A, .)) meet in one L2.
__device__ inline int xcd_remap(int b, int G) {
  const int x = b & 7, pos = b >> 3;
  const int q = (G + 7) >> 3, r = G & 7;
  if (r == 0) return x * q + pos;
  return x < r ? x * q + pos : r * q + (x - r) * (q - 1) + pos;
}

// ---------------------------------------------------------------------------
// H(B,X)[beta][b][x] = sum_{G alive} sum_g Cf(B,G)[beta][b][g] D(G,X)[g][x]
// rows (beta,b), columns x, depth = the g index of all live C pairs of B.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT) k_hbuild(Dev d) {
  __shared__ int ktab[kMaxK];
  __shared__ int kdepth;
  const int s = blockIdx.x;
  if (!d.need[s]) return;
  const int B = d.slotB[s], X = d.slotX[s];
  const int mB = d.nabf[B], nB = d.nao[B], nX = d.nao[X];
  if (threadIdx.x == 0) {
    int k = 0;
    for (int cp = d.cpRow[B]; cp < d.cpRow[B + 1]; ++cp) {
      if (!d.aliveC[cp]) continue;
      const int nG = d.nao[d.cpF[cp]];
      for (int gg = 0; gg < nG && k < kMaxK; ++gg) ktab[k++] = (cp << 6) | gg;
    }
    const int kp = (k + 3) & ~3;
    for (int i = k; i < kp && i < kMaxK; ++i) ktab[i] = -1;
    kdepth = kp;
  }
  __syncthreads();
  const int K = kdepth;
  const int rows = mB * nB;
  const int RT = (rows + 15) >> 4, XT = (nX + 15) >> 4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane & 15, g = lane >> 4;
  double* Hout = d.H + d.hOff[s];
  for (int t = w; t < RT * XT; t += kWaves) {
    const int rt = t / XT, xt = t % XT;
    const int row = 16 * rt + q, x = 16 * xt + q;
    d4 acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int e = ktab[k0 + g];
      double a = 0, b = 0;
      if (e >= 0) {
        const int cp = e >> 6, gg = e & 63;
        const int G = d.cpF[cp], nG = d.nao[G];
        if (row < rows) a = d.Cf[d.cfOff[cp] + (int64_t)row * nG + gg];
        if (x < nX && d.keepD[(int64_t)G * d.N + X]) b = d.D[(d.ao[G] + gg) * d.ntot + d.ao[X] + x];
      }
      acc = mfma_f64(a, b, acc);
    }
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * rt + g + 4 * i;
      if (r < rows && x < nX) Hout[(int64_t)r * nX + x] = acc[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Triple products.  One workgroup per unit (C pair (A,F), column chunk
// [k0,k1) of the (a,f) index).  For every live V pair (A,B):
//   X[beta][k] (16 rows at a time, in LDS) = sum_b D_AB[a][b] H(B,F)[beta][b][f]
//                                         + sum_b D_FB[f][b] H(B,A)[beta][b][a],
//   Z partial [alpha][beta] = sum_{k in chunk} Cf(A,F)[alpha][k] X[beta][k]  -> Zbuf,
//   Y[alpha][k] += sum_beta Vf(A,B)[alpha][beta] X[beta][k]                 (registers).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT) k_triple(Dev d) {
  __shared__ double Xs[16 * kXS];
  __shared__ double Dab[kMaxNao * kMaxNao];
  __shared__ double Dfb[kMaxNao * kMaxNao];
  const int u = xcd_remap(blockIdx.x, gridDim.x);
  const int cp = d.unitCp[u];
  if (!d.aliveC[cp]) return;
  const int A = d.cpA[cp], F = d.cpF[cp];
  const int mA = d.nabf[A], nA = d.nao[A], nF = d.nao[F], K1 = nA * nF;
  const int k0 = d.unitK0[u], k1 = d.unitK1[u], kc = d.unitKc[u];
  const int Kc = k1 - k0, NTc = (Kc + 15) >> 4, Kcp = NTc * 16;
  const int MT = (mA + 15) >> 4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  const double* Cfp = d.Cf + d.cfOff[cp];
  const int N = d.N;
  const int fpos = cp - d.cpRow[A];
  const int vp0 = d.vpRow[A], nVpA = d.vpRow[A + 1] - vp0;

  d4 yacc[kMaxAlphaTiles][kMaxJW];
#pragma unroll
  for (int i = 0; i < kMaxAlphaTiles; ++i)
#pragma unroll
    for (int j = 0; j < kMaxJW; ++j) yacc[i][j] = d4{0, 0, 0, 0};

  for (int p = vp0; p < vp0 + nVpA; ++p) {
    if (!d.aliveV[p]) continue;
    const int B = d.vpB[p], mB = d.nabf[B], nB = d.nao[B];
    double* Zdst = d.Zbuf + d.zOff[d.tBase[A] + (int64_t)fpos * nVpA + (p - vp0)] + (int64_t)kc * mA * mB;
    const double* Vfp = d.Vf + d.vfOff[p];
    const double* hBF = d.H + d.hOff[d.hSlotMap[(int64_t)B * N + F]];
    const double* hBA = d.H + d.hOff[d.hSlotMap[(int64_t)B * N + A]];
    const bool kAB = d.keepD[(int64_t)A * N + B], kFB = d.keepD[(int64_t)F * N + B];
    __syncthreads();
    for (int e = tid; e < nA * nB; e += kNT)
      Dab[e] = kAB ? d.D[(d.ao[A] + e / nB) * d.ntot + d.ao[B] + e % nB] : 0.0;
    for (int e = tid; e < nF * nB; e += kNT)
      Dfb[e] = kFB ? d.D[(d.ao[F] + e / nB) * d.ntot + d.ao[B] + e % nB] : 0.0;
    __syncthreads();
    for (int b0 = 0; b0 < mB; b0 += 16) {
      for (int e = tid; e < 16 * Kcp; e += kNT) {
        const int r = e / Kcp, c = e - r * Kcp;
        const int be = b0 + r;
        double sacc = 0;
        if (be < mB && c < Kc) {
          const int k = k0 + c;
          const int a = k / nF, f = k - a * nF;
          const double* h1 = hBF + (int64_t)be * nB * nF + f;
          const double* h2 = hBA + (int64_t)be * nB * nA + a;
          for (int b = 0; b < nB; ++b) sacc += Dab[a * nB + b] * h1[b * nF] + Dfb[f * nB + b] * h2[b * nA];
        }
        Xs[r * kXS + c] = sacc;
      }
      __syncthreads();
      // Z partial: alpha tiles w, w + 4, ...
      for (int i = w; i < MT; i += kWaves) {
        d4 acc = {0, 0, 0, 0};
        const int al = 16 * i + q;
        const double* crow = Cfp + (int64_t)al * K1 + k0;
        for (int kk = 0; kk < Kcp; kk += 4) {
          const int c = kk + g;
          const double a = (al < mA && c < Kc) ? crow[c] : 0.0;
          acc = mfma_f64(a, Xs[q * kXS + c], acc);
        }
        for (int r = 0; r < 4; ++r) {
          const int alr = 16 * i + g + 4 * r, be = b0 + q;
          if (alr < mA && be < mB) Zdst[(int64_t)alr * mB + be] = acc[r];
        }
      }
      // Y += Vf[:, b0:b0+16] X
#pragma unroll
      for (int i = 0; i < kMaxAlphaTiles; ++i) {
        if (i < MT) {
          const int al = 16 * i + q;
          double av[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int be = b0 + 4 * s + g;
            av[s] = (al < mA && be < mB) ? Vfp[(int64_t)al * mB + be] : 0.0;
          }
#pragma unroll
          for (int jj = 0; jj < kMaxJW; ++jj) {
            const int j = w + kWaves * jj;
            if (j < NTc) {
#pragma unroll
              for (int s = 0; s < 4; ++s) yacc[i][jj] = mfma_f64(av[s], Xs[(4 * s + g) * kXS + 16 * j + q], yacc[i][jj]);
            }
          }
        }
      }
      __syncthreads();
    }
  }
  double* Y = d.Ybuf + d.yOff[cp];
#pragma unroll
  for (int i = 0; i < kMaxAlphaTiles; ++i)
#pragma unroll
    for (int jj = 0; jj < kMaxJW; ++jj) {
      const int j = w + kWaves * jj;
      if (i < MT && j < NTc) {
        for (int r = 0; r < 4; ++r) {
          const int al = 16 * i + g + 4 * r, c = 16 * j + q;
          if (al < mA && c < Kc) Y[(int64_t)al * K1 + k0 + c] = yacc[i][jj][r];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Z(A,B) = sum over live (A,F) of the Z partials; E and V-block gradients.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT) k_zgrad(Dev d) {
  extern __shared__ double Zs[];
  __shared__ double sh[kWaves + 1];
  const int p = blockIdx.x;
  const int A = d.vpA[p], B = d.vpB[p];
  const int mA = d.nabf[A], mB = d.nabf[B], n = mA * mB;
  if (!d.aliveV[p]) {
    for (int k = d.vpB0[p] + threadIdx.x; k < d.vpB1[p]; k += kNT) {
      const int64_t b = d.vpBlk[k];
      d.gV[3 * b] = d.gV[3 * b + 1] = d.gV[3 * b + 2] = 0.0;
    }
    if (threadIdx.x == 0) d.Ep[p] = 0.0;
    return;
  }
  const int vp0 = d.vpRow[A], nVpA = d.vpRow[A + 1] - vp0, bpos = p - vp0;
  for (int e = threadIdx.x; e < n; e += kNT) {
    double z = 0;
    for (int cp = d.cpRow[A]; cp < d.cpRow[A + 1]; ++cp) {
      if (!d.aliveC[cp]) continue;
      const double* zp = d.Zbuf + d.zOff[d.tBase[A] + (int64_t)(cp - d.cpRow[A]) * nVpA + bpos];
      for (int kc = 0; kc < d.nkc[cp]; ++kc) z += zp[(int64_t)kc * n + e];
    }
    Zs[e] = z;
  }
  __syncthreads();
  const double* vf = d.Vf + d.vfOff[p];
  double s = 0;
  for (int e = threadIdx.x; e < n; e += kNT) s += vf[e] * Zs[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) d.Ep[p] = -s;
  for (int k = d.vpB0[p]; k < d.vpB1[p]; ++k) {
    const int64_t b = d.vpBlk[k];
    if (!d.keepV[b]) {
      if (threadIdx.x == 0) d.gV[3 * b] = d.gV[3 * b + 1] = d.gV[3 * b + 2] = 0.0;
      continue;
    }
    const double* dv = d.Vdval + 3 * d.Voff[b];
    for (int x = 0; x < 3; ++x) {
      double t = 0;
      for (int e = threadIdx.x; e < n; e += kNT) t += dv[(int64_t)x * n + e] * Zs[e];
      t = block_sum(t, sh);
      if (threadIdx.x == 0) d.gV[3 * b + x] = -t;
    }
  }
}

// ---------------------------------------------------------------------------
// C-block gradients: g_c = -2 <dC_c, Y(A,F)>; E from the Y side for checking.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT) k_cgrad(Dev d) {
  __shared__ double sh[kWaves + 1];
  const int cp = blockIdx.x;
  const int A = d.cpA[cp], F = d.cpF[cp];
  const int n = d.nabf[A] * d.nao[A] * d.nao[F];
  if (!d.aliveC[cp]) {
    for (int k = d.cpB0[cp] + threadIdx.x; k < d.cpB1[cp]; k += kNT) {
      const int64_t b = d.cpBlk[k];
      d.gC[3 * b] = d.gC[3 * b + 1] = d.gC[3 * b + 2] = 0.0;
    }
    if (threadIdx.x == 0) d.Ecp[cp] = 0.0;
    return;
  }
  const double* Y = d.Ybuf + d.yOff[cp];
  const double* cf = d.Cf + d.cfOff[cp];
  double s = 0;
  for (int e = threadIdx.x; e < n; e += kNT) s += cf[e] * Y[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) d.Ecp[cp] = -s;
  for (int k = d.cpB0[cp]; k < d.cpB1[cp]; ++k) {
    const int64_t b = d.cpBlk[k];
    if (!d.keepC[b]) {
      if (threadIdx.x == 0) d.gC[3 * b] = d.gC[3 * b + 1] = d.gC[3 * b + 2] = 0.0;
      continue;
    }
    const double* dc = d.Cdval + 3 * d.Coff[b];
    for (int x = 0; x < 3; ++x) {
      double t = 0;
      for (int e = threadIdx.x; e < n; e += kNT) t += dc[(int64_t)x * n + e] * Y[e];
      t = block_sum(t, sh);
      if (threadIdx.x == 0) d.gC[3 * b + x] = -2.0 * t;
    }
  }
}

// ---------------------------------------------------------------------------
// Forces: owner-computes per atom over fixed block lists (no atomics).
// ---------------------------------------------------------------------------
__global__ void k_forces(Dev d) {
  const int M = blockIdx.x * blockDim.x + threadIdx.x;
  if (M >= d.N) return;
  double f[3] = {0, 0, 0};
  for (int k = d.atCfRow[M]; k < d.atCfRow[M + 1]; ++k)
    for (int x = 0; x < 3; ++x) f[x] += d.gC[3 * d.atCf[k] + x];
  for (int k = d.atCsRow[M]; k < d.atCsRow[M + 1]; ++k)
    for (int x = 0; x < 3; ++x) f[x] -= d.gC[3 * d.atCs[k] + x];
  for (int k = d.atVfRow[M]; k < d.atVfRow[M + 1]; ++k)
    for (int x = 0; x < 3; ++x) f[x] += d.gV[3 * d.atVf[k] + x];
  for (int k = d.atVsRow[M]; k < d.atVsRow[M + 1]; ++k)
    for (int x = 0; x < 3; ++x) f[x] -= d.gV[3 * d.atVs[k] + x];
  for (int x = 0; x < 3; ++x) d.out[1 + 3 * M + x] = f[x];
}

// Energy and virial: one workgroup, fixed-order reductions.
constexpr int kFinalNT = 1024;
__global__ void __launch_bounds__(kFinalNT) k_final(Dev d) {
  __shared__ double sh[kFinalNT / 64 + 1];
  double e = 0, ey = 0;
  for (int p = threadIdx.x; p < d.nVp; p += kFinalNT) e += d.Ep[p];
  for (int c = threadIdx.x; c < d.nCp; c += kFinalNT) ey += d.Ecp[c];
  double w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int pass = 0; pass < 2; ++pass) {
    const int64_t nb = pass ? d.nV : d.nC;
    const int* fi = pass ? d.Vfirst : d.Cfirst;
    const int* se = pass ? d.Vsecond : d.Csecond;
    const int* R = pass ? d.VR : d.CR;
    const double* gr = pass ? d.gV : d.gC;
    for (int64_t b = threadIdx.x; b < nb; b += kFinalNT) {
      double r[3];
      for (int x = 0; x < 3; ++x)
        r[x] = d.tau[3 * se[b] + x] - d.tau[3 * fi[b] + x] + R[3 * b] * d.lat[x] + R[3 * b + 1] * d.lat[3 + x] +
               R[3 * b + 2] * d.lat[6 + x];
      for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) w[3 * x + y] += gr[3 * b + x] * r[y];
    }
  }
  e = block_sum(e, sh);
  ey = block_sum(ey, sh);
  for (int i = 0; i < 9; ++i) w[i] = block_sum(w[i], sh);
  if (threadIdx.x == 0) {
    d.out[0] = e;
    for (int i = 0; i < 9; ++i) d.out[1 + 3 * d.N + i] = -w[i] / d.omega;
    d.out[1 + 3 * d.N + 9] = ey;
  }
}

static inline unsigned grid1(int64_t n, int64_t b) { return (unsigned)(n > 0 ? (n + b - 1) / b : 1); }

void launch_contract(const Dev& d, int max_mm, hipStream_t s, hipEvent_t* ev) {
  if (d.nSlot) hipLaunchKernelGGL(k_hbuild, dim3(d.nSlot), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[4], s);
  if (d.nUnit) hipLaunchKernelGGL(k_triple, dim3(d.nUnit), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[5], s);
  if (d.nVp) {
    const size_t lds = (size_t)max_mm * sizeof(double);
    if (lds > 65536) (void)hipFuncSetAttribute((const void*)k_zgrad, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_zgrad, dim3(d.nVp), dim3(kNT), lds, s, d);
  }
  if (ev) (void)hipEventRecord(ev[6], s);
  if (d.nCp) hipLaunchKernelGGL(k_cgrad, dim3(d.nCp), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[7], s);
  hipLaunchKernelGGL(k_forces, dim3(grid1(d.N, kNT)), dim3(kNT), 0, s, d);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kFinalNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[8], s);
}

}  // namespace lrx
