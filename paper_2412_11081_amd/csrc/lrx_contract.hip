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
// H(B,X)[b][beta][x] = sum_{G alive} sum_g Cf(B,G)[beta][b][g] D(G,X)[g][x].
// One workgroup per (B, 64 rows of (beta,b)): the rows of Cf(B, live G) are
// staged once in LDS (depth = the g index of every live C pair of B) and
// reused for every X of B; wave w owns row tile w.  H is stored with b
// outermost so that the triple kernel reads 16 consecutive (beta,x) per b.
// ---------------------------------------------------------------------------
// One workgroup per (B, 64 rows of (beta,b), 64 columns): the columns are
// the (X, x) pairs of every H slot of B concatenated, so one D tile staged in
// LDS serves four 16-column MFMA tiles per wave, and the Cf(B, .) fragments
// of the wave's row tile stay in registers for the whole tile.  The depth
// (every g of every live C pair (B,G)) runs in passes of at most kHPass.
constexpr int kHCols = 64;
__global__ void __launch_bounds__(kNT) k_hbuild(Dev d) {
  __shared__ int krow[kHMaxDepth];   // D row (ao[G] + g) of depth index k
  __shared__ int kG[kHMaxDepth];     // atom G, or -1 (padding or screened pair)
  __shared__ int64_t kcf[kHMaxDepth];
  __shared__ int kst[kHMaxDepth];
  __shared__ int cD[kHCols], cAt[kHCols], cSl[kHCols], cX[kHCols];
  __shared__ int kdepth;
  __shared__ double Ds[kHPass * kHCols];
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
  d4 acc[kHCols / 16];
#pragma unroll
  for (int j = 0; j < kHCols / 16; ++j) acc[j] = d4{0, 0, 0, 0};
  for (int kb = 0; kb < Kall; kb += kHPass) {
    const int K = min(kHPass, Kall - kb);
    // A fragments of this pass, all requested before any MFMA
    double af[kHPass / 4];
#pragma unroll
    for (int s = 0; s < kHPass / 4; ++s) {
      const int k = kb + 4 * s + g;
      af[s] = (4 * s < K && row < rows && kG[k] >= 0) ? d.Cf[kcf[k] + (int64_t)row * kst[k]] : 0.0;
    }
    // D[(G,g)][column] tile of this pass
    for (int e = tid; e < K * kHCols; e += kNT) {
      const int k = e / kHCols, cl = e - k * kHCols;
      const int G = kG[kb + k];
      double v = 0;
      if (G >= 0 && cSl[cl] >= 0 && d.keepD[(int64_t)G * d.N + cAt[cl]])
        v = d.D[(int64_t)krow[kb + k] * d.ntot + cD[cl]];
      Ds[k * kHCols + cl] = v;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kHPass / 4; ++s) {
      if (4 * s < K) {
#pragma unroll
        for (int j = 0; j < kHCols / 16; ++j) acc[j] = mfma_f64(af[s], Ds[(4 * s + g) * kHCols + 16 * j + q], acc[j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < kHCols / 16; ++j) {
    const int cl = 16 * j + q;
    const int s = cSl[cl];
    if (s < 0) continue;
    const int nX = d.nao[d.slotX[s]], x = cX[cl];
    double* Hout = d.H + d.hOff[s];
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + 16 * w + g + 4 * i;
      if (r < rows) {
        const int be = r / nB, bb = r - be * nB;
        Hout[((int64_t)bb * mBp + be) * nX + x] = acc[j][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Triple products.  One workgroup of 8 waves per unit (C pair (A,F), column
// chunk [k0,k1) of the (a,f) index), looping over "chunks" = (live V pair
// (A,B), 16 rows beta0..beta0+15 of B's ABFs):
//   X-build (all waves, MFMA, operands in LDS):
//       X1[beta][a f] = sum_b D_AB[a][b] H(B,F)[b][beta][f]
//       X2[beta][a f] = sum_b D_FB[f][b] H(B,A)[b][beta][a]
//   Z waves 0-3 (K split four ways, Cf(A,F) fragments in registers):
//       Z(A,B)[alpha][beta] partial over (a,f) in the chunk -> Zbuf
//   Y waves 4-7 (accumulators resident for the whole unit):
//       Y(A,F)[alpha][a f] += Vf(A,B)[alpha][beta] X[beta][a f]
// The H slices (and, when B changes, the D blocks) of the next chunk are
// brought into LDS with direct global->LDS loads issued right after the
// X-build of the current chunk, so they arrive while its MFMAs run.
// ---------------------------------------------------------------------------
template <int MT>
struct TripleCfg {
  static constexpr int kCols = unit_cols(MT);
  static constexpr int kKSW = kCols / 16;           // Z k-steps per Z wave
  static constexpr int kJW = (kCols / 16 + 3) / 4;  // Y column tiles per Y wave
  static constexpr int kXS = kCols + 1;
  static constexpr int kHs = 8160;                  // doubles of staged H per chunk
  static constexpr size_t lds_doubles() { return 2 * 16 * kXS + 3 * MT * 256 + 2 * kMaxNao * kMaxNao + kHs; }
  static constexpr size_t lds_bytes() { return sizeof(double) * lds_doubles(); }
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
// doubles of H staged for a chunk: HF[b][16 nF] then HA[b][16 nA]
__device__ inline int chunk_hs(const UnitGeo& U, const Chunk& c) { return c.nB * 16 * (U.nF + U.nA); }

// Direct global->LDS copy of the chunk's H slices (16-byte pieces).
__device__ inline void stage_h(const Dev& d, const UnitGeo& U, const Chunk& c, double* Hs, int w, int lane) {
  const int64_t t = chunk_tri(d, U, c);
  const double* hF = d.H + d.triHF[t];
  const double* hA = d.H + d.triHA[t];
  const int mBp = (c.mB + 15) & ~15;
  const int pF = 8 * U.nF, pA = 8 * U.nA;            // 16-byte pieces per row
  const int P = c.nB * (pF + pA);
  for (int j = w; j * 64 < P; j += 8) {
    const int pc = j * 64 + lane;
    if (pc < P) {
      const double* src;
      if (pc < c.nB * pF) {
        const int b = pc / pF, m = pc - b * pF;
        src = hF + ((int64_t)b * mBp + c.b0) * U.nF + 2 * m;
      } else {
        const int pp = pc - c.nB * pF;
        const int b = pp / pA, m = pp - b * pA;
        src = hA + ((int64_t)b * mBp + c.b0) * U.nA + 2 * m;
      }
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)(Hs + 128 * j), 16, 0, 0);
    }
  }
}

// Direct global->LDS copy of D(A,B) and D(F,B) (4-byte pieces; rows of the
// dense D are not 16-byte aligned in general).
__device__ inline void stage_d(const Dev& d, const UnitGeo& U, int B, int nB, double* Dab, double* Dfb, int w,
                               int lane) {
  const int PA = 2 * U.nA * nB, PF = 2 * U.nF * nB;
  for (int j = w; j * 64 < PA + PF; j += 8) {
    const int pc = j * 64 + lane;
    // a wave instruction writes 64 consecutive dwords, so the two blocks are
    // staged as one contiguous image: Dab then Dfb
    if (pc < PA + PF) {
      const bool ab = pc < PA;
      const int pp = ab ? pc : pc - PA;
      const int e = pp >> 1, hlf = pp & 1;
      const int r = e / nB, b = e - r * nB;
      const double* src = d.D + (d.ao[ab ? U.A : U.F] + r) * d.ntot + d.ao[B] + b;
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)((const char*)src + 4 * hlf),
                                       (__attribute__((address_space(3))) void*)((char*)Dab + 256 * j), 4, 0, 0);
    }
  }
  (void)Dfb;
}

// One X-build tile from LDS operands.
__device__ inline void xbuild_tile(const UnitGeo& U, int t, int q, int g, int nB, const double* Hs,
                                   const double* Dab, const double* Dfb, bool kAB, bool kFB, double* X1, double* X2) {
  const bool one = t < U.T1;
  const int tt = one ? t : t - U.T1;
  const int ncol = one ? U.nF : U.nA;
  const int nrow = one ? U.nA : U.nF;
  const int tr = tt / ncol, tc = tt - tr * ncol;
  const double* Ds = one ? Dab : Dfb;
  const double* hs = one ? Hs : Hs + nB * 16 * U.nF;
  const bool keep = one ? kAB : kFB;
  const int c = 16 * tc + q;
  const int r = 16 * tr + q;
  d4 acc = {0, 0, 0, 0};
  const int SB = (nB + 3) >> 2;
  for (int s = 0; s < SB; ++s) {
    const int b = 4 * s + g;
    const bool ok = keep && b < nB;
    const double av = (ok && r < nrow) ? Ds[r * nB + b] : 0.0;
    const double hv = ok ? hs[b * 16 * ncol + c] : 0.0;
    acc = mfma_f64(av, hv, acc);
  }
  const int bl = c / ncol, xo = c - bl * ncol;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rr = 16 * tr + g + 4 * i;
    if (rr < nrow) {
      const int k = one ? rr * U.nF + xo : xo * U.nF + rr;
      const int cl = k - U.k0;
      if (cl >= 0 && cl < U.Kc) (one ? X1 : X2)[bl * U.XS + cl] = acc[i];
    }
  }
}

// The H slice of a chunk that does not fit the LDS stage is read directly.
__device__ inline void xbuild_tile_direct(const Dev& d, const UnitGeo& U, const Chunk& ch, int t, int q, int g,
                                          const double* Dab, const double* Dfb, bool kAB, bool kFB, double* X1,
                                          double* X2) {
  const int64_t tri = chunk_tri(d, U, ch);
  const bool one = t < U.T1;
  const int tt = one ? t : t - U.T1;
  const int ncol = one ? U.nF : U.nA;
  const int nrow = one ? U.nA : U.nF;
  const int tr = tt / ncol, tc = tt - tr * ncol;
  const double* Ds = one ? Dab : Dfb;
  const double* hp = d.H + (one ? d.triHF[tri] : d.triHA[tri]);
  const int mBp = (ch.mB + 15) & ~15;
  const bool keep = one ? kAB : kFB;
  const int c = 16 * tc + q;
  const int r = 16 * tr + q;
  const int nB = ch.nB;
  d4 acc = {0, 0, 0, 0};
  const int SB = (nB + 3) >> 2;
  for (int s = 0; s < SB; ++s) {
    const int b = 4 * s + g;
    const bool ok = keep && b < nB;
    const double av = (ok && r < nrow) ? Ds[r * nB + b] : 0.0;
    const double hv = ok ? hp[((int64_t)b * mBp + ch.b0) * ncol + c] : 0.0;
    acc = mfma_f64(av, hv, acc);
  }
  const int bl = c / ncol, xo = c - bl * ncol;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rr = 16 * tr + g + 4 * i;
    if (rr < nrow) {
      const int k = one ? rr * U.nF + xo : xo * U.nF + rr;
      const int cl = k - U.k0;
      if (cl >= 0 && cl < U.Kc) (one ? X1 : X2)[bl * U.XS + cl] = acc[i];
    }
  }
}

template <int MT, bool ZROLE>
__device__ void triple_role(const Dev& d, const UnitGeo& U, double* lds, int w, int lane, int q, int g) {
  using Cfg = TripleCfg<MT>;
  double* X1 = lds;
  double* X2 = lds + 16 * Cfg::kXS;
  double* Zred = lds + 32 * Cfg::kXS;          // partials of Z waves 1-3
  double* Dab = Zred + 3 * MT * 256;
  double* Dfb = Dab;                            // set per B (contiguous after Dab)
  double* Hs = Dab + 2 * kMaxNao * kMaxNao;
  const int ww = w & 3;
  const int N = d.N;
  const int mA = U.mA, XS = U.XS;

  double cfr[ZROLE ? MT : 1][ZROLE ? Cfg::kKSW : 1];
  d4 yacc[ZROLE ? 1 : MT][ZROLE ? 1 : Cfg::kJW];
  if constexpr (ZROLE) {
    const double* Cfp = d.Cf + d.cfOff[U.cp];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int t = 0; t < Cfg::kKSW; ++t) {
        const int ks = ww + 4 * t, c = 4 * ks + g, al = 16 * i + q;
        cfr[i][t] = (ks < U.KS && c < U.Kc && al < mA) ? Cfp[(int64_t)al * U.K1 + U.k0 + c] : 0.0;
      }
  } else {
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::kJW; ++j) yacc[i][j] = d4{0, 0, 0, 0};
  }

  // prologue: stage the first chunk
  Chunk ch = chunk_at(d, U, U.vb, 0);
  if (ch.p >= 0) {
    stage_d(d, U, ch.B, ch.nB, Dab, Dfb, w, lane);
    if (chunk_hs(U, ch) <= Cfg::kHs) stage_h(d, U, ch, Hs, w, lane);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  while (ch.p >= 0) {
    const Chunk nx = chunk_next(d, U, ch);
    const bool kAB = d.keepD[(int64_t)U.A * N + ch.B], kFB = d.keepD[(int64_t)U.F * N + ch.B];
    Dfb = Dab + U.nA * ch.nB;
    const int64_t tri = chunk_tri(d, U, ch);
    double* Zdst = d.Zbuf + d.zOff[tri] + (int64_t)U.kc * mA * ch.mB;
    const double* Vfp = d.Vf + d.vfOff[ch.p];
    // V fragments of this chunk (Y waves); their latency is covered by the X-build
    double avn[ZROLE ? 1 : 4][ZROLE ? 1 : MT];
    if constexpr (!ZROLE) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          const int al = 16 * i + q, be = ch.b0 + 4 * s + g;
          avn[s][i] = (al < mA && be < ch.mB) ? Vfp[(int64_t)al * ch.mB + be] : 0.0;
        }
    }
    // ---- X-build of this chunk (all waves) ------------------------------
    const bool staged = chunk_hs(U, ch) <= Cfg::kHs;
    for (int t = w; t < U.T1 + U.T2; t += 8) {
      if (staged)
        xbuild_tile(U, t, q, g, ch.nB, Hs, Dab, Dfb, kAB, kFB, X1, X2);
      else
        xbuild_tile_direct(d, U, ch, t, q, g, Dab, Dfb, kAB, kFB, X1, X2);
    }
    __syncthreads();
    // ---- stage the next chunk while this one is contracted -------------
    if (nx.p >= 0) {
      if (nx.p != ch.p) stage_d(d, U, nx.B, nx.nB, Dab, Dfb, w, lane);
      if (chunk_hs(U, nx) <= Cfg::kHs) stage_h(d, U, nx, Hs, w, lane);
    }
    if constexpr (ZROLE) {
      d4 zp[MT];
#pragma unroll
      for (int i = 0; i < MT; ++i) zp[i] = d4{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < Cfg::kKSW; ++t) {
        const int ks = ww + 4 * t;
        if (ks < U.KS) {
          const int c = 4 * ks + g;
          const double xb = X1[q * XS + c] + X2[q * XS + c];
#pragma unroll
          for (int i = 0; i < MT; ++i) zp[i] = mfma_f64(cfr[i][t], xb, zp[i]);
        }
      }
      if (ww > 0) {
#pragma unroll
        for (int i = 0; i < MT; ++i) *(d4*)&Zred[((ww - 1) * MT + i) * 256 + lane * 4] = zp[i];
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (ww == 0) {
        const int be = ch.b0 + q;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          d4 z = zp[i];
          for (int v = 0; v < 3; ++v) z += *(const d4*)&Zred[(v * MT + i) * 256 + lane * 4];
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int al = 16 * i + g + 4 * rr;
            if (al < mA && be < ch.mB) Zdst[(int64_t)al * ch.mB + be] = z[rr];
          }
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
            const double xb = X1[bl * XS + 16 * j + q] + X2[bl * XS + 16 * j + q];
#pragma unroll
            for (int i = 0; i < MT; ++i) yacc[i][jj] = mfma_f64(avn[s][i], xb, yacc[i][jj]);
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    ch = nx;
  }
  if constexpr (!ZROLE) {
    double* Y = d.Ybuf + d.yOff[U.cp] + (int64_t)U.split * mA * U.K1;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int jj = 0; jj < Cfg::kJW; ++jj) {
        const int j = ww + 4 * jj;
        if (j < U.NTc) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int al = 16 * i + g + 4 * rr, c = 16 * j + q;
            if (al < mA && c < U.Kc) Y[(int64_t)al * U.K1 + U.k0 + c] = yacc[i][jj][rr];
          }
        }
      }
  }
}

template <int MT>
__global__ void __launch_bounds__(kTNT, 1) k_triple(Dev d, const int* __restrict__ ulist) {
  using Cfg = TripleCfg<MT>;
  extern __shared__ __attribute__((aligned(32))) double lds[];
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
  for (int e = tid; e < 32 * Cfg::kXS; e += kTNT) lds[e] = 0.0;
  __syncthreads();
  if (w < 4)
    triple_role<MT, true>(d, U, lds, w, lane, q, g);
  else
    triple_role<MT, false>(d, U, lds, w, lane, q, g);
}

// ---------------------------------------------------------------------------
// Z(A,B) = sum over live (A,F) and column chunks of the Z partials; then, in
// one pass over the pair's blocks, E = -<Vf, Z> and g_v = -<dV_v, Z>.
// ---------------------------------------------------------------------------
constexpr int kZB = 4;      // V image blocks contracted per pass over Z
constexpr int kZMax = 64;   // Z partials (live C pairs x column chunks) of one V pair

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

__global__ void __launch_bounds__(kNT) k_zgrad(Dev d) {
  __shared__ double sh[kWaves * (1 + 3 * kZB)];
  __shared__ int64_t zoff[kZMax];
  __shared__ int nz;
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
  __shared__ int64_t zb[kZMax];
  __shared__ int zk[kZMax];
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
      for (int k = 0; k < NZ; ++k) z += d.Zbuf[zoff[k] + e];
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
// C-block gradients: g_c = -2 <dC_c, Y(A,F)>; E from the Y side for checking.
// ---------------------------------------------------------------------------
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
  const double* Y = d.Ybuf + d.yOff[cp];
  const int ns = d.nsplit[cp];
  const double* cf = d.Cf + d.cfOff[cp];
  double s[4] = {0, 0, 0, 0};
  for (int e = threadIdx.x; e < n; e += kNT) {
    double y = 0;
    for (int k = 0; k < ns; ++k) y += Y[(int64_t)k * n + e];
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
      for (int kk = 0; kk < ns; ++kk) y += Y[(int64_t)kk * n + e];
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

template <int MT>
static void launch_triple(const Dev& d, hipStream_t s) {
  const int n = d.mtStart[MT + 1] - d.mtStart[MT];
  if (n <= 0) return;
  const size_t lds = TripleCfg<MT>::lds_bytes();
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_triple<MT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL(k_triple<MT>, dim3(n), dim3(kTNT), lds, s, d, d.unitOrder + d.mtStart[MT]);
}

void launch_contract(const Dev& d, int max_mm, int max_depth, hipStream_t s, const hipStream_t* side,
                     const hipEvent_t* fork, hipEvent_t* ev) {
  (void)max_mm;
  (void)max_depth;
  if (d.nHB) hipLaunchKernelGGL(k_hbuild, dim3(d.nHB), dim3(kNT), 0, s, d);
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
    switch (order[i]) {
      case 1: launch_triple<1>(d, st); break;
      case 2: launch_triple<2>(d, st); break;
      case 3: launch_triple<3>(d, st); break;
      case 4: launch_triple<4>(d, st); break;
      case 5: launch_triple<5>(d, st); break;
      case 6: launch_triple<6>(d, st); break;
      case 7: launch_triple<7>(d, st); break;
      default: launch_triple<8>(d, st); break;
    }
  }
  for (int i = 1; i <= kSideStreams && i < ng; ++i) {
    (void)hipEventRecord(fork[i], side[i - 1]);
    (void)hipStreamWaitEvent(s, fork[i], 0);
  }
  if (ev) (void)hipEventRecord(ev[5], s);
  if (d.nVp) hipLaunchKernelGGL(k_zgrad, dim3(d.nVp), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[6], s);
  if (d.nCp) hipLaunchKernelGGL(k_cgrad, dim3(d.nCp), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[7], s);
  hipLaunchKernelGGL(k_forces, dim3(grid1(d.N, kNT)), dim3(kNT), 0, s, d);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kFinalNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[8], s);
}

}  // namespace lrx
