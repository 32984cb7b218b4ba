// Contraction of the LRI exchange energy and its position derivatives
// (Methods, Eqs. exx_expand, Fexx1 and stress) in the Gamma-point folded form:
//
//   H(B,X)    = sum_G Cf(B,G) D(G,X)                                   k_hbuild
//   X^{AFB}   = D_AB H(B,F) + (D_FB H(B,A)) with (a,f) swapped          k_triple
//   Z(A,B)   += Cf(A,F) X^{AFB T},  Y(A,F) += Vf(A,B) X^{AFB}            k_triple
//   E = -<Vf, Z>;  g_v = -<dV_v, Z(A,B)>;  g_c = -2 <dC_c, Y(A,F)>       k_zgrad, k_cgrad
//   F_first += g, F_second -= g;  sigma = -(1/Omega) sum g (x) r         k_forces, k_final
//
// Every kernel of the dense part is a template over the storage type T of
// Cf, Vf, D, H, X, Z and Y (double for the FP64 form, float for the FP32 and
// BF16x3 forms).  The products run on the gfx950 matrix cores with 16x16
// output tiles; per 64-lane wave, lane l, q = l & 15, g = l >> 4:
//   v_mfma_f64_16x16x4f64   A[m=q][k=g], B[k=g][n=q], result element i -> D[g + 4i][q]
//   v_mfma_f32_16x16x4f32   same operands,            result element i -> D[4g + i][q]
//   v_mfma_f32_16x16x16bf16 A[m=q][k=4g+j], B[k=4g+j][n=q] (j<4), result i -> D[4g + i][q]
// The BF16x3 form feeds the two large products (Z and Y) with a bf16 split of
// each FP32 operand, x = hi + lo, and accumulates hi*hi + hi*lo + lo*hi in
// FP32; H and X are built with FP32 products.  The gradient, force, virial
// and energy reductions are FP64 in every form.
#include "lrx_internal.h"

namespace lrx {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int kNT = 256;
constexpr int kWaves = kNT / 64;

// 16x16x4 matrix-core product per storage type
template <class T>
struct M4;
template <>
struct M4<double> {
  using acc = d4;
  __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int g, int i) { return g + 4 * i; }
};
template <>
struct M4<float> {
  using acc = f4;
  __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int g, int i) { return 4 * g + i; }
};

// bf16 with round-to-nearest-even of the FP32 bit pattern (finite inputs)
__device__ inline short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ inline float bf16_value(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }
__device__ inline void split4(const float* x, s4& hi, s4& lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const short h = bf16_bits(x[j]);
    hi[j] = h;
    lo[j] = bf16_bits(x[j] - bf16_value(h));
  }
}
__device__ inline f4 mma_bf16x3(s4 ah, s4 al, s4 bh, s4 bl, f4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
  return c;
}

// buffers of one storage type
template <class T>
struct Buf;
template <>
struct Buf<double> {
  __device__ static const double* Cf(const Dev& d) { return d.Cf; }
  __device__ static const double* Vf(const Dev& d) { return d.Vf; }
  __device__ static const double* D(const Dev& d) { return d.D; }
  __device__ static double* H(const Dev& d) { return d.H; }
  __device__ static double* Z(const Dev& d) { return d.Zbuf; }
  __device__ static double* Y(const Dev& d) { return d.Ybuf; }
};
template <>
struct Buf<float> {
  __device__ static const float* Cf(const Dev& d) { return d.Cf32; }
  __device__ static const float* Vf(const Dev& d) { return d.Vf32; }
  __device__ static const float* D(const Dev& d) { return d.D32; }
  __device__ static float* H(const Dev& d) { return d.H32; }
  __device__ static float* Z(const Dev& d) { return d.Zbuf32; }
  __device__ static float* Y(const Dev& d) { return d.Ybuf32; }
};

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
// Block-wide sums of NV values at once (fixed order; result in every thread).
template <int NV>
__device__ inline void block_sum_n(double* v, double* sh) {
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) sh[w * NV + j] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double r = 0;
    for (int i = 0; i < nw; ++i) r += sh[i * NV + j];
    v[j] = r;
  }
  __syncthreads();
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
// H(B,X)[b][beta][x] = sum_{G alive} sum_g Cf(B,G)[beta][b][g] D(G,X)[g][x].
// One workgroup per (B, 64 rows of (beta,b), 64 columns): the columns are
// the (X, x) pairs of every H slot of B concatenated, so one D tile staged in
// LDS serves four 16-column tiles per wave, and the Cf(B, .) fragments of the
// wave's row tile are requested once per pass.  The depth (every g of every
// live C pair (B,G)) runs in passes of at most kHPass.
// ---------------------------------------------------------------------------
constexpr int kHCols = 64;
template <class T>
__global__ void __launch_bounds__(kNT) k_hbuild(Dev d) {
  using M = M4<T>;
  __shared__ int krow[kHMaxDepth];   // D row (ao[G] + g) of depth index k
  __shared__ int kG[kHMaxDepth];     // atom G, or -1 (padding or screened pair)
  __shared__ int64_t kcf[kHMaxDepth];
  __shared__ int kst[kHMaxDepth];
  __shared__ int cD[kHCols], cAt[kHCols], cSl[kHCols], cX[kHCols];
  __shared__ int kdepth;
  __shared__ T Ds[kHPass * kHCols];
  const T* Cf = Buf<T>::Cf(d);
  const T* Dm = Buf<T>::D(d);
  const int B = d.hbB[blockIdx.x], r0 = d.hbR0[blockIdx.x], c0 = d.hbC0[blockIdx.x];
  const int mB = d.nabf[B], nB = d.nao[B], rows = mB * nB;
  const int ncols = d.hColRow[B + 1] - d.hColRow[B];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  {
    const int h0 = d.hdRow[B], hn = d.hdRow[B + 1] - h0;
    for (int k = tid; k < hn; k += kNT) {
      const int t = d.hdCp[h0 + k];
      const bool live = t >= 0 && d.aliveC[t >> 6];
      krow[k] = d.hdRowD[h0 + k];
      kG[k] = live ? d.hdG[h0 + k] : -1;
      kcf[k] = d.hdCf[h0 + k];
      kst[k] = d.hdStride[h0 + k];
    }
    for (int cl = tid; cl < kHCols; cl += kNT) {
      const int c = c0 + cl;
      const bool in = c < ncols;
      const int s = in ? d.hColSlot[d.hColRow[B] + c] : 0;
      cSl[cl] = in && d.need[s] ? s : -1;
      cD[cl] = in ? d.hColD[d.hColRow[B] + c] : 0;
      cAt[cl] = in ? d.hColAtom[d.hColRow[B] + c] : 0;
      cX[cl] = in ? d.hColX[d.hColRow[B] + c] : 0;
    }
    if (tid == 0) kdepth = hn;
  }
  __syncthreads();
  const int Kall = kdepth;
  const int mBp = (mB + 15) & ~15;
  const int row = r0 + 16 * w + q;    // A-operand row of this lane
  typename M::acc acc[kHCols / 16];
#pragma unroll
  for (int j = 0; j < kHCols / 16; ++j) acc[j] = typename M::acc{0, 0, 0, 0};
  for (int kb = 0; kb < Kall; kb += kHPass) {
    const int K = min(kHPass, Kall - kb);
    T af[kHPass / 4];
#pragma unroll
    for (int s = 0; s < kHPass / 4; ++s) {
      const int k = kb + 4 * s + g;
      af[s] = (4 * s < K && row < rows && kG[k] >= 0) ? Cf[kcf[k] + (int64_t)row * kst[k]] : T(0);
    }
    for (int e = tid; e < K * kHCols; e += kNT) {
      const int k = e / kHCols, cl = e - k * kHCols;
      const int G = kG[kb + k];
      T v = 0;
      if (G >= 0 && cSl[cl] >= 0 && d.keepD[(int64_t)G * d.N + cAt[cl]])
        v = Dm[(int64_t)krow[kb + k] * d.ntot + cD[cl]];
      Ds[k * kHCols + cl] = v;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kHPass / 4; ++s) {
      if (4 * s < K) {
#pragma unroll
        for (int j = 0; j < kHCols / 16; ++j) acc[j] = M::mma(af[s], Ds[(4 * s + g) * kHCols + 16 * j + q], acc[j]);
      }
    }
    __syncthreads();
  }
  T* H = Buf<T>::H(d);
#pragma unroll
  for (int j = 0; j < kHCols / 16; ++j) {
    const int cl = 16 * j + q;
    const int s = cSl[cl];
    if (s < 0) continue;
    const int nX = d.nao[d.slotX[s]], x = cX[cl];
    T* Hout = H + d.hOff[s];
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + 16 * w + M::row(g, i);
      if (r < rows) {
        const int be = r / nB, bb = r - be * nB;
        Hout[((int64_t)bb * mBp + be) * nX + x] = acc[j][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Triple products.  One workgroup of 8 waves per unit (C pair (A,F), column
// chunk [k0,k1) of the (a,f) index, range of V partners), looping over
// "chunks" = (live V pair (A,B), 16 rows beta0..beta0+15 of B's ABFs):
//   X-build (all waves, matrix cores, operands in LDS):
//       X1[beta][a f] = sum_b D_AB[a][b] H(B,F)[b][beta][f]
//       X2[beta][a f] = sum_b D_FB[f][b] H(B,A)[b][beta][a]
//   Z waves 0-3 (K split four ways, Cf(A,F) fragments in registers):
//       Z(A,B)[alpha][beta] partial over (a,f) in the chunk -> Zbuf
//   Y waves 4-7 (accumulators resident for the whole unit):
//       Y(A,F)[alpha][a f] += Vf(A,B)[alpha][beta] X[beta][a f]
// The H slices (and, when B changes, the D blocks) of the next chunk are
// brought into LDS with direct global->LDS loads issued right after the
// X-build of the current chunk, so they arrive while its products run.
// ---------------------------------------------------------------------------
template <int MT, int P>
struct TripleCfg {
  using T = typename std::conditional<P == kP64, double, float>::type;
  static constexpr int kCols = unit_cols(MT);
  static constexpr int kKSW = P == kPB3 ? (kCols / 16 + 3) / 4 : kCols / 16;   // Z k-steps per Z wave
  static constexpr int kJW = (kCols / 16 + 3) / 4;                            // Y column tiles per Y wave
  static constexpr int kXS = kCols + 1;
  static constexpr int kHsBytes = 65280;
  static constexpr int kHs = kHsBytes / sizeof(T);                            // staged H elements per chunk
  static constexpr size_t lds_bytes() {
    return sizeof(T) * (2 * 16 * kXS + 3 * MT * 256 + 2 * kMaxNao * kMaxNao) + kHsBytes;
  }
};

constexpr int kTNT = 512;

struct UnitGeo {
  int cp, A, F, mA, nA, nF, K1, k0, Kc, kc, NTc, KS, XS, T1, T2, fpos, vp0, nVpA, vb, ve, split;
};

struct Chunk {
  int p, B, mB, nB, b0;   // p < 0: no chunk
};

__device__ inline Chunk chunk_at(const Dev& d, const UnitGeo& U, int p, int b0) {
  Chunk c;
  for (; p < U.ve && !d.aliveV[p]; ++p) {
  }
  c.p = p < U.ve ? p : -1;
  c.b0 = b0;
  if (c.p >= 0) {
    c.B = d.vpB[c.p];
    c.mB = d.nabf[c.B];
    c.nB = d.nao[c.B];
  } else {
    c.B = c.mB = c.nB = 0;
  }
  return c;
}
__device__ inline Chunk chunk_next(const Dev& d, const UnitGeo& U, const Chunk& c) {
  if (c.p < 0) return c;
  if (c.b0 + 16 < c.mB) {
    Chunk n = c;
    n.b0 += 16;
    return n;
  }
  return chunk_at(d, U, c.p + 1, 0);
}
__device__ inline int64_t chunk_tri(const Dev& d, const UnitGeo& U, const Chunk& c) {
  return d.tBase[U.A] + (int64_t)U.fpos * U.nVpA + (c.p - U.vp0);
}
// elements of H staged for a chunk: HF[b][16 nF] then HA[b][16 nA]
__device__ inline int chunk_hs(const UnitGeo& U, const Chunk& c) { return c.nB * 16 * (U.nF + U.nA); }

// Direct global->LDS copy of the chunk's H slices (16-byte pieces; H rows
// are 16-element aligned by construction).
template <class T>
__device__ inline void stage_h(const Dev& d, const UnitGeo& U, const Chunk& c, T* Hs, int w, int lane) {
  constexpr int E = 16 / sizeof(T);                 // elements per piece
  const int64_t t = chunk_tri(d, U, c);
  const T* H = Buf<T>::H(d);
  const T* hF = H + d.triHF[t];
  const T* hA = H + d.triHA[t];
  const int mBp = (c.mB + 15) & ~15;
  const int pF = 16 * U.nF / E, pA = 16 * U.nA / E;   // pieces per row
  const int P = c.nB * (pF + pA);
  for (int j = w; j * 64 < P; j += 8) {
    const int pc = j * 64 + lane;
    if (pc < P) {
      const T* src;
      if (pc < c.nB * pF) {
        const int b = pc / pF, m = pc - b * pF;
        src = hF + ((int64_t)b * mBp + c.b0) * U.nF + E * m;
      } else {
        const int pp = pc - c.nB * pF;
        const int b = pp / pA, m = pp - b * pA;
        src = hA + ((int64_t)b * mBp + c.b0) * U.nA + E * m;
      }
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)((char*)Hs + 1024 * j), 16, 0, 0);
    }
  }
}

// Direct global->LDS copy of D(A,B) then D(F,B) (4-byte pieces; rows of the
// dense D are not 16-byte aligned in general).
template <class T>
__device__ inline void stage_d(const Dev& d, const UnitGeo& U, int B, int nB, T* Dab, int w, int lane) {
  constexpr int W = sizeof(T) / 4;                  // dwords per element
  const T* Dm = Buf<T>::D(d);
  const int PA = W * U.nA * nB, PF = W * U.nF * nB;
  for (int j = w; j * 64 < PA + PF; j += 8) {
    const int pc = j * 64 + lane;
    if (pc < PA + PF) {
      const bool ab = pc < PA;
      const int pp = ab ? pc : pc - PA;
      const int e = pp / W, part = pp - e * W;
      const int r = e / nB, b = e - r * nB;
      const T* src = Dm + (d.ao[ab ? U.A : U.F] + r) * d.ntot + d.ao[B] + b;
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)((const char*)src + 4 * part),
                                       (__attribute__((address_space(3))) void*)((char*)Dab + 256 * j), 4, 0, 0);
    }
  }
}

// One X-build tile.  DIRECT: the H slice is read from global memory (chunks
// whose slices exceed the LDS stage).
template <class T, bool DIRECT>
__device__ inline void xbuild_tile(const Dev& d, const UnitGeo& U, const Chunk& ch, int t, int q, int g,
                                   const T* Hs, const T* Dab, const T* Dfb, bool kAB, bool kFB, T* X1, T* X2) {
  using M = M4<T>;
  const bool one = t < U.T1;
  const int tt = one ? t : t - U.T1;
  const int ncol = one ? U.nF : U.nA;
  const int nrow = one ? U.nA : U.nF;
  const int tr = tt / ncol, tc = tt - tr * ncol;
  const T* Ds = one ? Dab : Dfb;
  const bool keep = one ? kAB : kFB;
  const int c = 16 * tc + q;
  const int r = 16 * tr + q;
  const int nB = ch.nB;
  const T* hs;
  int64_t hstride;
  if constexpr (DIRECT) {
    const int64_t tri = chunk_tri(d, U, ch);
    const int mBp = (ch.mB + 15) & ~15;
    hs = Buf<T>::H(d) + (one ? d.triHF[tri] : d.triHA[tri]) + (int64_t)ch.b0 * ncol;
    hstride = (int64_t)mBp * ncol;
  } else {
    hs = one ? Hs : Hs + nB * 16 * U.nF;
    hstride = 16 * ncol;
  }
  typename M::acc acc = {0, 0, 0, 0};
  const int SB = (nB + 3) >> 2;
  for (int s = 0; s < SB; ++s) {
    const int b = 4 * s + g;
    const bool ok = keep && b < nB;
    const T av = (ok && r < nrow) ? Ds[r * nB + b] : T(0);
    const T hv = ok ? hs[b * hstride + c] : T(0);
    acc = M::mma(av, hv, acc);
  }
  const int bl = c / ncol, xo = c - bl * ncol;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rr = 16 * tr + M::row(g, i);
    if (rr < nrow) {
      const int k = one ? rr * U.nF + xo : xo * U.nF + rr;
      const int cl = k - U.k0;
      if (cl >= 0 && cl < U.Kc) (one ? X1 : X2)[bl * U.XS + cl] = acc[i];
    }
  }
}

template <int MT, int P, bool ZROLE>
__device__ void triple_role(const Dev& d, const UnitGeo& U, unsigned char* ldsb, int w, int lane, int q, int g) {
  using Cfg = TripleCfg<MT, P>;
  using T = typename Cfg::T;
  using M = M4<T>;
  using Acc = typename M::acc;           // d4 (FP64) or f4 (FP32, BF16x3)
  using A = typename std::conditional<P == kP64, double, float>::type;
  constexpr bool B3 = P == kPB3;
  T* X1 = (T*)ldsb;
  T* X2 = X1 + 16 * Cfg::kXS;
  A* Zred = (A*)(X2 + 16 * Cfg::kXS);   // partials of Z waves 1-3
  T* Dab = (T*)(Zred + 3 * MT * 256);
  T* Hs = Dab + 2 * kMaxNao * kMaxNao;
  const int ww = w & 3;
  const int N = d.N;
  const int mA = U.mA, XS = U.XS;
  const T* Cf = Buf<T>::Cf(d);
  const T* Vf = Buf<T>::Vf(d);

  // ---- resident operands / accumulators of the role ----------------------
  constexpr int ZI = ZROLE ? MT : 1, ZT = ZROLE ? Cfg::kKSW : 1;
  constexpr int YI = ZROLE ? 1 : MT, YJ = ZROLE ? 1 : Cfg::kJW;
  T cfr[B3 ? 1 : ZI][B3 ? 1 : ZT];
  s4 cfh[B3 ? ZI : 1][B3 ? ZT : 1], cfl[B3 ? ZI : 1][B3 ? ZT : 1];
  Acc yacc[YI][YJ];
  if constexpr (ZROLE) {
    const T* Cfp = Cf + d.cfOff[U.cp];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int t = 0; t < Cfg::kKSW; ++t) {
        const int al = 16 * i + q;
        if constexpr (B3) {
          const int ks = ww + 4 * t;            // 16-wide k-step
          float v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int c = 16 * ks + 4 * g + j;
            v[j] = (ks < U.NTc && c < U.Kc && al < mA) ? Cfp[(int64_t)al * U.K1 + U.k0 + c] : 0.f;
          }
          split4(v, cfh[i][t], cfl[i][t]);
        } else {
          const int ks = ww + 4 * t, c = 4 * ks + g;
          cfr[i][t] = (ks < U.KS && c < U.Kc && al < mA) ? Cfp[(int64_t)al * U.K1 + U.k0 + c] : T(0);
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::kJW; ++j) yacc[i][j] = Acc{0, 0, 0, 0};
  }

  // prologue: stage the first chunk
  Chunk ch = chunk_at(d, U, U.vb, 0);
  if (ch.p >= 0) {
    stage_d<T>(d, U, ch.B, ch.nB, Dab, w, lane);
    if (chunk_hs(U, ch) <= Cfg::kHs) stage_h<T>(d, U, ch, Hs, w, lane);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  while (ch.p >= 0) {
    const Chunk nx = chunk_next(d, U, ch);
    const bool kAB = d.keepD[(int64_t)U.A * N + ch.B], kFB = d.keepD[(int64_t)U.F * N + ch.B];
    const T* Dfb = Dab + U.nA * ch.nB;
    const int64_t tri = chunk_tri(d, U, ch);
    T* Zdst = Buf<T>::Z(d) + d.zOff[tri] + (int64_t)U.kc * mA * ch.mB;
    const T* Vfp = Vf + d.vfOff[ch.p];
    // V fragments of this chunk (Y waves); their latency is covered by the X-build
    T avn[(ZROLE || B3) ? 1 : 4][(ZROLE || B3) ? 1 : MT];
    s4 avh[(!ZROLE && B3) ? MT : 1], avl[(!ZROLE && B3) ? MT : 1];
    if constexpr (!ZROLE) {
      if constexpr (B3) {
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          const int al = 16 * i + q;
          float v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int be = ch.b0 + 4 * g + j;
            v[j] = (al < mA && be < ch.mB) ? Vfp[(int64_t)al * ch.mB + be] : 0.f;
          }
          split4(v, avh[i], avl[i]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int i = 0; i < MT; ++i) {
            const int al = 16 * i + q, be = ch.b0 + 4 * s + g;
            avn[s][i] = (al < mA && be < ch.mB) ? Vfp[(int64_t)al * ch.mB + be] : T(0);
          }
      }
    }
    // ---- X-build of this chunk (all waves) ------------------------------
    const bool staged = chunk_hs(U, ch) <= Cfg::kHs;
    for (int t = w; t < U.T1 + U.T2; t += 8) {
      if (staged)
        xbuild_tile<T, false>(d, U, ch, t, q, g, Hs, Dab, Dfb, kAB, kFB, X1, X2);
      else
        xbuild_tile<T, true>(d, U, ch, t, q, g, Hs, Dab, Dfb, kAB, kFB, X1, X2);
    }
    __syncthreads();
    // ---- stage the next chunk while this one is contracted -------------
    if (nx.p >= 0) {
      if (nx.p != ch.p) stage_d<T>(d, U, nx.B, nx.nB, Dab, w, lane);
      if (chunk_hs(U, nx) <= Cfg::kHs) stage_h<T>(d, U, nx, Hs, w, lane);
    }
    if constexpr (ZROLE) {
      Acc zp[MT];
#pragma unroll
      for (int i = 0; i < MT; ++i) zp[i] = Acc{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < Cfg::kKSW; ++t) {
        if constexpr (B3) {
          const int ks = ww + 4 * t;
          if (ks < U.NTc) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int c = 16 * ks + 4 * g + j;
              v[j] = X1[q * XS + c] + X2[q * XS + c];
            }
            s4 bh, bl;
            split4(v, bh, bl);
#pragma unroll
            for (int i = 0; i < MT; ++i) zp[i] = mma_bf16x3(cfh[i][t], cfl[i][t], bh, bl, zp[i]);
          }
        } else {
          const int ks = ww + 4 * t;
          if (ks < U.KS) {
            const int c = 4 * ks + g;
            const T xb = X1[q * XS + c] + X2[q * XS + c];
#pragma unroll
            for (int i = 0; i < MT; ++i) zp[i] = M::mma(cfr[i][t], xb, zp[i]);
          }
        }
      }
      if (ww > 0) {
#pragma unroll
        for (int i = 0; i < MT; ++i) *(Acc*)&Zred[((ww - 1) * MT + i) * 256 + lane * 4] = zp[i];
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (ww == 0) {
        const int be = ch.b0 + q;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          Acc z = zp[i];
          for (int v = 0; v < 3; ++v) z += *(const Acc*)&Zred[(v * MT + i) * 256 + lane * 4];
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int al = 16 * i + M::row(g, rr);
            if (al < mA && be < ch.mB) Zdst[(int64_t)al * ch.mB + be] = z[rr];
          }
        }
      }
    } else {
      if constexpr (B3) {
#pragma unroll
        for (int jj = 0; jj < Cfg::kJW; ++jj) {
          const int j = ww + 4 * jj;
          if (j < U.NTc) {
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int bl = 4 * g + k;
              v[k] = X1[bl * XS + 16 * j + q] + X2[bl * XS + 16 * j + q];
            }
            s4 bh, blo;
            split4(v, bh, blo);
#pragma unroll
            for (int i = 0; i < MT; ++i) yacc[i][jj] = mma_bf16x3(avh[i], avl[i], bh, blo, yacc[i][jj]);
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int bl = 4 * s + g;
#pragma unroll
          for (int jj = 0; jj < Cfg::kJW; ++jj) {
            const int j = ww + 4 * jj;
            if (j < U.NTc) {
              const T xb = X1[bl * XS + 16 * j + q] + X2[bl * XS + 16 * j + q];
#pragma unroll
              for (int i = 0; i < MT; ++i) yacc[i][jj] = M::mma(avn[s][i], xb, yacc[i][jj]);
            }
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    ch = nx;
  }
  if constexpr (!ZROLE) {
    T* Y = Buf<T>::Y(d) + d.yOff[U.cp] + (int64_t)U.split * mA * U.K1;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int jj = 0; jj < Cfg::kJW; ++jj) {
        const int j = ww + 4 * jj;
        if (j < U.NTc) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int al = 16 * i + M::row(g, rr), c = 16 * j + q;
            if (al < mA && c < U.Kc) Y[(int64_t)al * U.K1 + U.k0 + c] = yacc[i][jj][rr];
          }
        }
      }
  }
}

template <int MT, int P>
__global__ void __launch_bounds__(kTNT, 1) k_triple(Dev d, const int* __restrict__ ulist) {
  using Cfg = TripleCfg<MT, P>;
  using T = typename Cfg::T;
  extern __shared__ __attribute__((aligned(32))) unsigned char ldsb[];
  const int u = ulist[xcd_remap(blockIdx.x, gridDim.x)];
  UnitGeo U;
  U.cp = d.unitCp[u];
  if (!d.aliveC[U.cp]) return;
  U.A = d.cpA[U.cp];
  U.F = d.cpF[U.cp];
  U.mA = d.nabf[U.A];
  U.nA = d.nao[U.A];
  U.nF = d.nao[U.F];
  U.K1 = U.nA * U.nF;
  U.k0 = d.unitK0[u];
  U.Kc = d.unitK1[u] - U.k0;
  U.kc = d.unitKc[u];
  U.NTc = (U.Kc + 15) >> 4;
  U.KS = U.NTc * 4;
  U.XS = U.NTc * 16 + 1;
  U.T1 = ((U.nA + 15) >> 4) * U.nF;
  U.T2 = ((U.nF + 15) >> 4) * U.nA;
  U.fpos = U.cp - d.cpRow[U.A];
  U.vp0 = d.vpRow[U.A];
  U.nVpA = d.vpRow[U.A + 1] - U.vp0;
  U.vb = d.unitV0[u];
  U.ve = d.unitV1[u];
  U.split = d.unitS[u];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  T* X = (T*)ldsb;
  for (int e = tid; e < 32 * Cfg::kXS; e += kTNT) X[e] = T(0);
  __syncthreads();
  if (w < 4)
    triple_role<MT, P, true>(d, U, ldsb, w, lane, q, g);
  else
    triple_role<MT, P, false>(d, U, ldsb, w, lane, q, g);
}

// ---------------------------------------------------------------------------
// Z(A,B) = sum over live (A,F) and column chunks of the Z partials; then, in
// one pass over the pair's blocks, E = -<Vf, Z> and g_v = -<dV_v, Z> (FP64).
// ---------------------------------------------------------------------------
constexpr int kZB = 4;      // V image blocks contracted per pass over Z
constexpr int kZMax = 64;   // Z partials (live C pairs x column chunks) of one V pair

template <class T>
__global__ void __launch_bounds__(kNT) k_zgrad(Dev d) {
  __shared__ double sh[kWaves * (1 + 3 * kZB)];
  __shared__ int64_t zoff[kZMax];
  __shared__ int64_t zb[kZMax];
  __shared__ int zk[kZMax];
  __shared__ int nz;
  const T* Zb = Buf<T>::Z(d);
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
  {
    const int vp0 = d.vpRow[A], nVpA = d.vpRow[A + 1] - vp0, bpos = p - vp0;
    const int c0 = d.cpRow[A], ncp = d.cpRow[A + 1] - c0;
    for (int i = threadIdx.x; i < ncp && i < kZMax; i += kNT) {
      zk[i] = d.aliveC[c0 + i] ? d.nkc[c0 + i] : 0;
      zb[i] = d.zOff[d.tBase[A] + (int64_t)i * nVpA + bpos];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int k = 0;
      for (int i = 0; i < ncp && i < kZMax; ++i)
        for (int kc = 0; kc < zk[i] && k < kZMax; ++kc) zoff[k++] = zb[i] + (int64_t)kc * n;
      nz = k;
    }
    __syncthreads();
  }
  const int NZ = nz;
  const double* vf = d.Vf + d.vfOff[p];
  const int kb0 = d.vpB0[p], kb1 = d.vpB1[p];
  for (int k0 = kb0; k0 < kb1 || k0 == kb0; k0 += kZB) {
    const int nb = max(0, min(kZB, kb1 - k0));
    const double* dv[kZB];
    bool kp[kZB];
#pragma unroll
    for (int j = 0; j < kZB; ++j) {
      const int64_t b = d.vpBlk[j < nb ? k0 + j : kb0];
      kp[j] = j < nb && d.keepV[b];
      dv[j] = d.Vdval + 3 * d.Voff[b];
    }
    double acc[1 + 3 * kZB];
#pragma unroll
    for (int j = 0; j < 1 + 3 * kZB; ++j) acc[j] = 0.0;
    const bool first = k0 == kb0;
    for (int e = threadIdx.x; e < n; e += kNT) {
      double z = 0;
      for (int k = 0; k < NZ; ++k) z += (double)Zb[zoff[k] + e];
      if (first) acc[0] += vf[e] * z;
#pragma unroll
      for (int j = 0; j < kZB; ++j)
        if (kp[j]) {
          acc[1 + 3 * j] += dv[j][e] * z;
          acc[2 + 3 * j] += dv[j][n + e] * z;
          acc[3 + 3 * j] += dv[j][2 * n + e] * z;
        }
    }
    block_sum_n<1 + 3 * kZB>(acc, sh);
    if (threadIdx.x == 0) {
      if (first) d.Ep[p] = -acc[0];
      for (int j = 0; j < nb; ++j) {
        const int64_t b = d.vpBlk[k0 + j];
        for (int x = 0; x < 3; ++x) d.gV[3 * b + x] = kp[j] ? -acc[1 + 3 * j + x] : 0.0;
      }
    }
    if (kb1 <= kb0) break;
  }
}

// ---------------------------------------------------------------------------
// C-block gradients: g_c = -2 <dC_c, Y(A,F)> (FP64); E from the Y side.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(kNT) k_cgrad(Dev d) {
  __shared__ double sh[kWaves * 4];
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
  const T* Y = Buf<T>::Y(d) + d.yOff[cp];
  const int ns = d.nsplit[cp];
  const double* cf = d.Cf + d.cfOff[cp];
  double s[4] = {0, 0, 0, 0};
  for (int e = threadIdx.x; e < n; e += kNT) {
    double y = 0;
    for (int k = 0; k < ns; ++k) y += (double)Y[(int64_t)k * n + e];
    s[0] += cf[e] * y;
  }
  block_sum_n<1>(s, sh);
  if (threadIdx.x == 0) d.Ecp[cp] = -s[0];
  for (int k = d.cpB0[cp]; k < d.cpB1[cp]; ++k) {
    const int64_t b = d.cpBlk[k];
    if (!d.keepC[b]) {
      if (threadIdx.x == 0) d.gC[3 * b] = d.gC[3 * b + 1] = d.gC[3 * b + 2] = 0.0;
      continue;
    }
    const double* dc = d.Cdval + 3 * d.Coff[b];
    double t[3] = {0, 0, 0};
    for (int e = threadIdx.x; e < n; e += kNT) {
      double y = 0;
      for (int kk = 0; kk < ns; ++kk) y += (double)Y[(int64_t)kk * n + e];
      t[0] += dc[e] * y;
      t[1] += dc[n + e] * y;
      t[2] += dc[2 * n + e] * y;
    }
    block_sum_n<3>(t, sh);
    if (threadIdx.x == 0)
      for (int x = 0; x < 3; ++x) d.gC[3 * b + x] = -2.0 * t[x];
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
  __shared__ double sh[(kFinalNT / 64) * 11];
  double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // E, W[9], E from the Y side
  for (int p = threadIdx.x; p < d.nVp; p += kFinalNT) v[0] += d.Ep[p];
  for (int c = threadIdx.x; c < d.nCp; c += kFinalNT) v[10] += d.Ecp[c];
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
        for (int y = 0; y < 3; ++y) v[1 + 3 * x + y] += gr[3 * b + x] * r[y];
    }
  }
  block_sum_n<11>(v, sh);
  if (threadIdx.x == 0) {
    d.out[0] = v[0];
    for (int i = 0; i < 9; ++i) d.out[1 + 3 * d.N + i] = -v[1 + i] / d.omega;
    d.out[1 + 3 * d.N + 9] = v[10];
  }
}

static inline unsigned grid1(int64_t n, int64_t b) { return (unsigned)(n > 0 ? (n + b - 1) / b : 1); }

template <int MT, int P>
static void launch_triple(const Dev& d, hipStream_t s) {
  const int n = d.mtStart[MT + 1] - d.mtStart[MT];
  if (n <= 0) return;
  const size_t lds = TripleCfg<MT, P>::lds_bytes();
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_triple<MT, P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL((k_triple<MT, P>), dim3(n), dim3(kTNT), lds, s, d, d.unitOrder + d.mtStart[MT]);
}

template <int P>
static void launch_triple_mt(const Dev& d, int mt, hipStream_t st) {
  switch (mt) {
    case 1: launch_triple<1, P>(d, st); break;
    case 2: launch_triple<2, P>(d, st); break;
    case 3: launch_triple<3, P>(d, st); break;
    case 4: launch_triple<4, P>(d, st); break;
    case 5: launch_triple<5, P>(d, st); break;
    case 6: launch_triple<6, P>(d, st); break;
    case 7: launch_triple<7, P>(d, st); break;
    default: launch_triple<8, P>(d, st); break;
  }
}

template <int P>
static void launch_contract_p(const Dev& d, hipStream_t s, const hipStream_t* side, const hipEvent_t* fork,
                              hipEvent_t* ev) {
  using T = typename std::conditional<P == kP64, double, float>::type;
  if (d.nHB) hipLaunchKernelGGL(k_hbuild<T>, dim3(d.nHB), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[4], s);
  // The alpha-tile groups are independent: the largest runs on the main
  // stream, the others on side streams that join before the gradients.
  int order[kMaxAlphaTiles];
  int ng = 0;
  for (int mt = 1; mt <= kMaxAlphaTiles; ++mt)
    if (d.mtStart[mt + 1] > d.mtStart[mt]) order[ng++] = mt;
  for (int i = 1; i < ng; ++i)
    for (int j = i; j > 0 && d.mtStart[order[j] + 1] - d.mtStart[order[j]] >
                                 d.mtStart[order[j - 1] + 1] - d.mtStart[order[j - 1]]; --j) {
      const int t = order[j];
      order[j] = order[j - 1];
      order[j - 1] = t;
    }
  (void)hipEventRecord(fork[0], s);
  for (int i = 0; i < ng; ++i) {
    const hipStream_t st = i == 0 ? s : side[(i - 1) % kSideStreams];
    if (i > 0 && i <= kSideStreams) (void)hipStreamWaitEvent(st, fork[0], 0);
    launch_triple_mt<P>(d, order[i], st);
  }
  for (int i = 1; i <= kSideStreams && i < ng; ++i) {
    (void)hipEventRecord(fork[i], side[i - 1]);
    (void)hipStreamWaitEvent(s, fork[i], 0);
  }
  if (ev) (void)hipEventRecord(ev[5], s);
  if (d.nVp) hipLaunchKernelGGL(k_zgrad<T>, dim3(d.nVp), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[6], s);
  if (d.nCp) hipLaunchKernelGGL(k_cgrad<T>, dim3(d.nCp), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[7], s);
  hipLaunchKernelGGL(k_forces, dim3(grid1(d.N, kNT)), dim3(kNT), 0, s, d);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kFinalNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[8], s);
}

void launch_contract(const Dev& d, int prec, hipStream_t s, const hipStream_t* side, const hipEvent_t* fork,
                     hipEvent_t* ev) {
  if (prec == kP64)
    launch_contract_p<kP64>(d, s, side, fork, ev);
  else if (prec == kP32)
    launch_contract_p<kP32>(d, s, side, fork, ev);
  else
    launch_contract_p<kPB3>(d, s, side, fork, ev);
}

}  // namespace lrx
