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

// Entry i of a table that the reading kernel does not write, read through the
// constant address space: at a uniform index the compiler can then use a
// scalar load (scalar cache, scalar registers) instead of a vector load.
template <class T>
__device__ __forceinline__ T ldu(const T* p, int64_t i) {
  return ((const __attribute__((address_space(4))) T*)p)[i];
}

// First element of the D block (X,Y) (d_block) through scalar loads; the
// cell term only with k-point sampling (a uniform branch), so that at the
// Gamma point the address costs two independent loads.
__device__ __forceinline__ int64_t d_blk(const Dev& d, int X, int Y) {
  int64_t o = ldu(d.aloc, X) * d.dld + ldu(d.aloc, Y);
  if (d.ncell > 1) o += (int64_t)ldu(d.dsub, ldu(d.acell, X) * d.ncell + ldu(d.acell, Y)) * d.dcellsz;
  return o;
}

// ---------------------------------------------------------------------------
// H(B,X)[b][beta][x] = sum_{G alive} sum_g Cf(B,G)[beta][b][g] D(G,X)[g][x],
// stored in blocks of 16 beta: [beta / 16][b][beta mod 16][x], so the slice
// of one block of 16 beta (what one triple-product chunk reads) is contiguous.
// Per atom B this is one dense product: rows (beta,b), depth (G,g) over the
// live C pairs (B,G), columns (X,x) over the H slots of B concatenated, with
// D(G,X) dropped for screened D pairs.  One workgroup of 8 waves per (B, 128
// rows, kHItemCols columns): each wave keeps the Cf fragments of its 16 rows
// in registers and walks the item's 64-column blocks (4 tiles of 16 per
// wave) and depth passes of at most kHPass; the D tile of the next step is
// loaded into registers while the current one is contracted from LDS
// (double buffer, one barrier per step).  BVK (k-point sampling): a D row or
// column index of the tables packs the atom's cell (bits 21 and up) and the
// AO index within the unit cell, and the element of D(G,X) is read from the
// cell offset's block of D(R) (d_block).
// ---------------------------------------------------------------------------
constexpr int kHT = 512;
constexpr int kHCB = 64;                         // columns of one block: 4 tiles of 16
constexpr int kHPre = kHPass * kHCB / kHT;       // D elements each thread stages per step
static_assert(kHRows == 16 * (kHT / 64), "one 16-row tile per wave");
constexpr int kCellShift = 21;                   // packed D index: cell << 21 | AO index in the cell
template <class T, bool BVK>
__global__ void __launch_bounds__(kHT, 4) k_hbuild(Dev d) {   // 4 waves per SIMD: two workgroups per CU
  using M = M4<T>;
  __shared__ int krow[kHMaxDepth];   // D row (ao[G] + g) of depth index k
  __shared__ int kG[kHMaxDepth];     // atom G, or -1 (padding or screened pair)
  __shared__ int64_t kcf[kHMaxDepth];
  __shared__ int kst[kHMaxDepth];
  __shared__ int cD[kHItemCols], cAt[kHItemCols], cSl[kHItemCols];
  __shared__ int kdepth;
  __shared__ T Ds[2][kHPass * kHCB];
  // D-pair keep flags of the item as a local table [C pair of B][slot],
  // when B has at most 32 C pairs and the item spans at most 64 slots
  __shared__ unsigned char keepL[32 * 64];
  __shared__ signed char kgi[kHMaxDepth], cxi[kHItemCols];
  const T* Cf = Buf<T>::Cf(d);
  const T* Dm = Buf<T>::D(d);
  const int B = d.hbB[blockIdx.x], r0 = d.hbR0[blockIdx.x], c0 = d.hbC0[blockIdx.x];
  const int mB = d.nabf[B], nB = d.nao[B], rows = mB * nB;
  // the item's columns among the needed ones (the grid covers every column
  // of the static table; items past the needed columns have nothing to do)
  const int ncols = min(kHItemCols, d.hcNcol[B] - c0);
  if (ncols <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, q = lane & 15, g = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, uniform
  const int cp0 = d.cpRow[B], ncp = d.cpRow[B + 1] - cp0;
  const int cb = d.hColRow[B];   // first column of B in the (compacted) column table
  const int s0 = d.hcColSlot[cb + c0], nsl = d.hcColSlot[cb + c0 + ncols - 1] - s0 + 1;
  const bool local = ncp <= 32 && nsl <= 64;
  {
    // depth entries of the live C pairs (B,G) only (compacted per evaluation)
    const int h0 = d.hdRow[B], hn = d.hcK[B];
    for (int k = tid; k < hn; k += kHT) {
      const int t = d.hcCp[h0 + k];
      krow[k] = d.hcRowD[h0 + k];
      kG[k] = d.hcG[h0 + k];
      kcf[k] = d.hcCf[h0 + k];
      kst[k] = d.hcStride[h0 + k];
      kgi[k] = (signed char)(t >= 0 && local ? (t >> 6) - cp0 : 0);
    }
    for (int cl = tid; cl < kHItemCols; cl += kHT) {
      const bool in = cl < ncols;
      const int c = cb + c0 + (in ? cl : 0);
      const int sl = d.hcColSlot[c];
      cSl[cl] = in ? sl : -1;
      cD[cl] = d.hcColD[c];          // a valid D column also past the item's end
      cAt[cl] = d.hcColAtom[c];
      cxi[cl] = (signed char)(local ? sl - s0 : 0);
    }
    if (local)
      for (int e = tid; e < ncp * nsl; e += kHT) {
        const int gi = e / nsl, xi = e - gi * nsl;
        keepL[gi * 64 + xi] = d.keepD[(int64_t)d.cpF[cp0 + gi] * d.N + d.slotX[s0 + xi]];
      }
    if (tid == 0) kdepth = hn;
  }
  __syncthreads();
  const int K = kdepth, N = d.N;
  const int npass = (K + kHPass - 1) / kHPass;
  const int nblk = (ncols + kHCB - 1) / kHCB;
  const int steps = nblk * npass;
  const int row = r0 + 16 * w + q;    // A-operand row of this lane
  // output rows of this lane: (b, beta) -> (beta / 16) 16 nB + 16 b + beta mod 16, or -1
  int orow[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + 16 * w + M::row(g, i);
    const int be = r / nB, bb = r - be * nB;
    orow[i] = r < rows ? (be >> 4) * 16 * nB + 16 * bb + (be & 15) : -1;
  }
  // D tile of (column block blk, pass p) into registers: element
  // e = tid + kHT i is (k, cl) = (e / kHCB, e mod kHCB), so a thread keeps
  // one column cl over its kHPre depth indices; screened pairs, dead C pairs
  // and padding give 0
  static_assert(kHT % kHCB == 0, "a thread's column is the same for every i");
  T pv[kHPre];
  auto fetch = [&](int blk, int p) __attribute__((always_inline)) {
    const int kb = p * kHPass, cl = blk * kHCB + (tid & (kHCB - 1));
    constexpr int kLoc = (1 << kCellShift) - 1;
    const T* Dc = Dm + (BVK ? (cD[cl] & kLoc) : cD[cl]);
    const bool cok = cSl[cl] >= 0;
    const int cx = cxi[cl], ca = cAt[cl];
#pragma unroll
    for (int i = 0; i < kHPre; ++i) {
      const int k = kb + (tid >> 6) + (kHT >> 6) * i;
      const int kk = k < K ? k : kb;
      const int G = k < K ? kG[kk] : -1;
      T v;
      if constexpr (BVK) {
        const int kr = krow[kk];
        v = Dc[(int64_t)d.dsub[(kr >> kCellShift) * d.ncell + (cD[cl] >> kCellShift)] * d.dcellsz +
               (int64_t)(kr & kLoc) * d.dld];
      } else {
        v = Dc[(int64_t)krow[kk] * d.ntot];
      }
      const bool keep = G >= 0 && cok &&
                        (local ? keepL[kgi[kk] * 64 + cx] != 0 : d.keepD[(int64_t)G * N + ca] != 0);
      pv[i] = keep ? v : T(0);
    }
  };
  T af[kHPass / 4];
  auto load_a = [&](int p) __attribute__((always_inline)) {
    const int kb = p * kHPass;
#pragma unroll
    for (int t = 0; t < kHPass / 4; ++t) {
      const int k = kb + 4 * t + g;
      af[t] = (k < K && row < rows && kG[k] >= 0) ? Cf[kcf[k] + (int64_t)row * kst[k]] : T(0);
    }
  };
  typename M::acc acc[kHCB / 16];
#pragma unroll
  for (int j = 0; j < kHCB / 16; ++j) acc[j] = typename M::acc{0, 0, 0, 0};
  T* H = Buf<T>::H(d);
  if (steps > 0) fetch(0, 0);
  load_a(0);
  // step st = (column block blk, depth pass p), p fastest
  for (int st = 0, blk = 0, p = 0; st < steps; ++st) {
    T* D2 = Ds[st & 1];
#pragma unroll
    for (int i = 0; i < kHPre; ++i) D2[tid + kHT * i] = pv[i];
    const bool wrap = p + 1 == npass;
    if (st + 1 < steps) fetch(wrap ? blk + 1 : blk, wrap ? 0 : p + 1);
    if (npass > 1 && st > 0) load_a(p);
    __syncthreads();
    const int Kp = min(kHPass, K - p * kHPass);
#pragma unroll
    for (int t = 0; t < kHPass / 4; ++t) {
      if (4 * t < Kp) {
#pragma unroll
        for (int j = 0; j < kHCB / 16; ++j) acc[j] = M::mma(af[t], D2[(4 * t + g) * kHCB + 16 * j + q], acc[j]);
      }
    }
    if (wrap) {
#pragma unroll
      for (int j = 0; j < kHCB / 16; ++j) {
        const int cl = blk * kHCB + 16 * j + q;
        const int sl = cSl[cl];
        if (sl >= 0) {
          // the AO index within atom X: its D column less the atom's first
          // column (BVK: both within the unit cell)
          const int X = cAt[cl], nX = d.nao[X];
          const int x = BVK ? (cD[cl] & ((1 << kCellShift) - 1)) - (int)d.aloc[X] : cD[cl] - (int)d.ao[X];
          T* Hout = H + d.hOff[sl] + x;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (orow[i] >= 0) Hout[(int64_t)orow[i] * nX] = acc[j][i];
        }
        acc[j] = typename M::acc{0, 0, 0, 0};
      }
      ++blk;
      p = 0;
    } else {
      ++p;
    }
  }
}

// ---------------------------------------------------------------------------
// Triple products.  One workgroup of 8 waves per unit (C pair (A,F), column
// chunk [k0,k1) of the (a,f) index, range of V partners), looping over
// "chunks" = (live V pair (A,B), 16 rows beta0..beta0+15 of B's ABFs):
//   X-build (all waves, matrix cores, operands in LDS):
//       X1[beta][a f] = sum_b D_AB[a][b] H(B,F)[b][beta][f]
//           tiles of 16 rows a (from the unit's first a) x 16 columns of the
//           flattened (beta, f) index
//       X2[beta][a f] = sum_b H(B,A)[b][beta][a] D_FB[f][b]
//           tiles of one a: 16 rows beta x 16 columns f
//       Only the tiles that reach the unit's column chunk are formed, one
//       term after the other; a Z wave keeps two tiles in flight (a Y wave
//       one or two, as its registers allow).
//   Z waves 0-3 (K split four ways, Cf(A,F) fragments in registers):
//       Z(A,B)[alpha][beta] over (a,f) in the chunk; the four partial sums
//       of alpha tile i meet in LDS and are added by Z wave (i mod 4), except
//       that a single last tile (MT = 1 mod 4) is added a quarter per wave
//   Y waves 4-7 (accumulators resident for the whole unit):
//       Y(A,F)[alpha][a f] += Vf(A,B)[alpha][beta] X[beta][a f]
// The V slice and the H slices (and, when B changes, the D blocks) of the
// next chunk are brought into LDS with direct global->LDS loads issued
// right after the X-build of the current chunk, so they arrive while its
// products run; the Y waves copy their V fragments out of the stage before
// the X-build of the chunk that uses them.
// ---------------------------------------------------------------------------
template <int MT, int P>
struct TripleCfg {
  using T = typename std::conditional<P == kP64, double, float>::type;
  using A = T;                                                               // Z partial sums
  static constexpr int kCols = unit_cols(MT);
  static constexpr int kKSW = P == kPB3 ? (kCols / 16 + 3) / 4 : kCols / 16;   // Z k-steps per Z wave
  static constexpr int kJW = (kCols / 16 + 3) / 4;                            // Y column tiles per Y wave (4 Y waves)
  static constexpr int kJW8 = (kCols / 16 + 7) / 8;                           // ... when all 8 waves are Y waves
  static constexpr int kXS = kCols + 1;
  // X-build by all eight waves; FP64 with many alpha tiles leaves the Y
  // waves registers for one tile in flight only
  static constexpr int kXW = 8;                                              // waves taking part
  static constexpr int kNUZ = 2;                                             // tiles in flight: Z waves
  static constexpr int kNUY = (P == kP64 && MT >= 5) ? 1 : 2;                 // Y waves (4 Y waves)
  static constexpr int kNUY8 = 2;                                            // ... (8 Y waves)
  // Z reduction: alpha tiles below kMF are owned by Z wave (i mod 4), which
  // adds the three partials the other Z waves park; a single remaining tile
  // (MT = 1 mod 4) is parked by all four and reduced a quarter per wave
  static constexpr int kMF = MT % 4 == 1 ? MT - 1 : MT;
  static constexpr int kZSlots = 3 * kMF + 4 * (MT - kMF);                  // parked 16x16 tiles
  static constexpr int kLds = 163840 - 256;     // X, Z partials and the stage; the rest holds the item slot
  static constexpr int kE = 16 / sizeof(T);
  static constexpr int kStage =
      (kLds - (int)sizeof(T) * 2 * 16 * kXS - (int)sizeof(A) * kZSlots * 256) / (int)sizeof(T) / kE * kE;
  static_assert(2 * kMaxNao * (kMaxNao + 1) + 16 * 16 * MT + kE <= kStage, "stage holds D and V of any chunk");
};

constexpr int kTNT = 512;

// Exact x / d for 0 <= x < 2^16 and 1 <= d < 2^16: with m = ceil(2^32 / d),
// x * m / 2^32 exceeds x / d by less than x / 2^32 < 1 / d.
struct Div {
  unsigned m;
  int one;
  __device__ void init(int d) {
    one = d == 1;
    m = one ? 0u : 0xFFFFFFFFu / (unsigned)d + 1u;
  }
  __device__ int operator()(int x) const { return one ? x : (int)__umulhi((unsigned)x, m); }
};

struct UnitGeo {
  int cp, A, F, mA, nA, nF, K1, k0, Kc, kc, NTc, KS, XS, fpos, vp0, nVpA, vb, ve, split;
  int a0, N1, N2, TF;        // X-build tiles: term 1 rows from a0 (16 per tile), term 2 one a per tile
  int pF, pA;                // 16-byte pieces per b row of the H slices (F and A)
  Div dnF;
};

struct Chunk {
  int p, B, mB, nB, b0;   // p < 0: no chunk
};

// VMASK: the liveness bits of a V pair that give the unit work (3 when it
// forms Z, which is read for any live pair; 1 when it forms Y alone, which
// only V pairs with Vf != 0 change)
template <int VMASK>
__device__ inline Chunk chunk_at(const Dev& d, const UnitGeo& U, int p, int b0) {
  Chunk c;
  for (; p < U.ve && !(ldu(d.aliveV, p) & VMASK); ++p) {
  }
  c.p = p < U.ve ? p : -1;
  c.b0 = b0;
  if (c.p >= 0) {
    c.B = ldu(d.vpB, c.p);
    c.mB = ldu(d.nabf, c.B);
    c.nB = ldu(d.nao, c.B);
  } else {
    c.B = c.mB = c.nB = 0;
  }
  return c;
}
template <int VMASK>
__device__ inline Chunk chunk_next(const Dev& d, const UnitGeo& U, const Chunk& c) {
  if (c.p < 0) return c;
  if (c.b0 + 16 < c.mB) {
    Chunk n = c;
    n.b0 += 16;
    return n;
  }
  return chunk_at<VMASK>(d, U, c.p + 1, 0);
}
__device__ inline int64_t chunk_tri(const Dev& d, const UnitGeo& U, const Chunk& c) {
  return ldu(d.tBase, U.A) + (int64_t)U.fpos * U.nVpA + (c.p - U.vp0);
}

// Chunk stage in LDS (elements of T), with nBp = nB rounded up to 4 (one
// k-step of the X-build) and D rows ldD = nBp + 1 elements apart (an odd
// stride: the 16 rows that 16 lanes read at once fall in distinct banks):
//   [0, nA ldD)             D(A,B)[a][b], b < nBp, zero for nB <= b < nBp
//                           (and everywhere when the block is screened)
//   [nA ldD, (nA+nF) ldD)   D(F,B)[f][b]        (both rewritten only when B changes)
//   [vo, vo + 16 mA)        Vf(A,B)[alpha][beta0 .. beta0+15], 16-byte pieces of a
//                           row stored in XOR-swizzled order (conflict-free reads)
//   [ho, ...)               H(B,F)[b][beta][f] then H(B,A)[b][beta][a], 16 rows
//                           beta, with room for nBp rows of H(B,A)
// vo = (nA+nF) ldD rounded up to 16 bytes, ho = vo + 16 mA.  Everything but
// the zero columns of D is brought in with direct global->LDS loads; H only
// when it fits.  The X-build reads nBp rows b: past nB the D operand is zero
// and the H operand is finite (H(B,A) rows, or stale stage contents, which
// start zeroed), so those k-steps add nothing.
struct StageGeo {
  int nBp, ldD, vo, ho, hend;
};
__device__ inline int d_stride(int nB) { return ((nB + 3) & ~3) + 1; }
template <class T>
__device__ inline StageGeo stage_geo(const UnitGeo& U, int nB) {
  constexpr int E = 16 / sizeof(T);
  StageGeo s;
  s.nBp = (nB + 3) & ~3;
  s.ldD = d_stride(nB);
  s.vo = ((U.nA + U.nF) * s.ldD + E - 1) / E * E;
  s.ho = s.vo + 16 * U.mA;
  s.hend = s.ho + 16 * (nB * U.nF + s.nBp * U.nA);
  return s;
}

// Zero columns nB .. nBp-1 of the staged D rows, and every column of the
// rows of a screened block (kAB: D(A,B) kept, kFB: D(F,B) kept), which the
// direct loads skip (all threads of the workgroup; issued before any of the
// stage's direct loads).
template <class T>
__device__ inline void zero_d_padding(const UnitGeo& U, int nB, bool kAB, bool kFB, T* S) {
  const int nBp = (nB + 3) & ~3, ld = d_stride(nB);
  const int pA = kAB ? nBp - nB : nBp, pF = kFB ? nBp - nB : nBp;   // zeroed columns per row, the last ones
  const int nzA = U.nA * pA, nz = nzA + U.nF * pF;
  for (int e = threadIdx.x; e < nz; e += kTNT) {
    const bool a = e < nzA;
    const int p = a ? pA : pF, e2 = a ? e : e - nzA, r = e2 / p;
    S[(a ? r : U.nA + r) * ld + (nBp - p) + (e2 - r * p)] = T(0);
  }
}

// The direct global->LDS loads that stage one chunk, as a list of 64-lane
// instructions: [D(A,B), D(F,B): 4-byte pieces, only when B changes]
// [V: 16-byte pieces] [H(B,F), H(B,A): 16-byte pieces, only when they fit].
// issue(J) sends instruction J, so the list can be spread over the products
// of the current chunk instead of stalling the waves in one burst.
template <class T>
struct Stager {
  static constexpr int E = 16 / sizeof(T);          // elements per 16-byte piece
  static constexpr int PR = 16 / E;                 // pieces per staged V row (16 elements)
  static constexpr int W = sizeof(T) / 4;           // dwords per element
  int nD, nV, n;                                    // instruction counts: D, D + V, all
  const char* dA;                                   // D rows of A at column ao[B]
  const char* dF;
  unsigned dRow;                                    // bytes per D row
  int nB, ldD, PA, PD;
  Div dB;
  const char* v0;
  unsigned vRow;                                    // bytes per folded V row
  int PV;
  const char* hF;
  const char* hA;
  int PF, PH;
  char* sD;
  char* sV;
  char* sH;

  bool kAB, kFB;                                    // D blocks kept (screened ones stay zero)
  __device__ void init(const Dev& d, const UnitGeo& U, const Chunk& c, const StageGeo& sg, bool with_d, bool with_h,
                       T* S, const T* Dm, const T* Vfg, const T* H) {
    nB = c.nB;
    kAB = with_d && ldu(d.keepD, (int64_t)U.A * d.N + c.B) != 0;
    kFB = with_d && ldu(d.keepD, (int64_t)U.F * d.N + c.B) != 0;
    dRow = (unsigned)(d.dld * sizeof(T));
    dA = (const char*)(Dm + d_blk(d, U.A, c.B));
    dF = (const char*)(Dm + d_blk(d, U.F, c.B));
    ldD = sg.ldD;
    if (with_d) dB.init(ldD);   // a division: only for chunks that stage D
    PA = W * U.nA * ldD;
    PD = with_d ? PA + W * U.nF * ldD : 0;
    const int mBp = (c.mB + 15) & ~15;
    v0 = (const char*)(Vfg + ldu(d.vfOff, c.p) + c.b0);
    vRow = (unsigned)(mBp * sizeof(T));
    PV = PR * U.mA;
    const int64_t t = chunk_tri(d, U, c);
    // the chunk's block of 16 beta in the H slots: contiguous [b][beta][x]
    hF = (const char*)(H + ldu(d.triHF, t) + (int64_t)c.b0 * c.nB * U.nF);
    hA = (const char*)(H + ldu(d.triHA, t) + (int64_t)c.b0 * c.nB * U.nA);
    PF = c.nB * U.pF;
    PH = with_h ? PF + c.nB * U.pA : 0;
    sD = (char*)S;
    sV = (char*)(S + sg.vo);
    sH = (char*)(S + sg.ho);
    nD = (PD + 63) >> 6;
    nV = nD + ((PV + 63) >> 6);
    n = nV + ((PH + 63) >> 6);
  }

  __device__ void issue(int J, int lane, const UnitGeo& U) const {
    // J is uniform: the part is chosen by scalar branches; addresses are
    // 32-bit byte offsets from the part's base (24-bit products)
    if (J < nD) {
      const int pc = J * 64 + lane;
      if (pc < PD) {
        const bool ab = pc < PA;
        const int pp = ab ? pc : pc - PA;
        const int e = W == 2 ? pp >> 1 : pp, part = pp - e * W;
        const int r = dB(e), b = e - r * ldD;
        const unsigned off = __umul24((unsigned)r, dRow) + (unsigned)(b * (int)sizeof(T) + 4 * part);
        // columns b >= nB and screened blocks are zeroed separately (zero_d_padding)
        if (b < nB && (ab ? kAB : kFB))
          __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)((ab ? dA : dF) + off),
                                           (__attribute__((address_space(3))) void*)(sD + 256 * J), 4, 0, 0);
      }
    } else if (J < nV) {
      const int j = J - nD, pc = j * 64 + lane;
      if (pc < PV) {
        const int al = pc / PR, k = pc - al * PR;
        const unsigned off = __umul24((unsigned)al, vRow) + 16u * (unsigned)(k ^ (al & (PR - 1)));
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(v0 + off),
                                         (__attribute__((address_space(3))) void*)(sV + 1024 * j), 16, 0, 0);
      }
    } else {
      const int j = J - nV, pc = j * 64 + lane;
      if (pc < PH) {
        const char* src = pc < PF ? hF + 16u * (unsigned)pc : hA + 16u * (unsigned)(pc - PF);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(sH + 1024 * j), 16, 0, 0);
      }
    }
  }
};

// Element (alpha, beta) of the staged V chunk.
template <class T>
__device__ inline int vs_index(int al, int be) {
  constexpr int E = 16 / sizeof(T), PR = 16 / E;
  return (al * PR + ((be / E) ^ (al & (PR - 1)))) * E + (be & (E - 1));
}

// Barrier for LDS hand-offs only: no wait on outstanding global stores.
__device__ inline void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// X-build of one chunk, one term at a time: this wave's tiles of the term,
// t = first, first + XW, ... below Nt (the two terms continue one round-robin
// over the XW waves that take part), up to NU at a time (independent
// accumulation chains on the matrix core).  The b index runs in k-steps of 4
// up to nBp; past nB the staged D operand is zero, and so is all of a
// screened D block, which makes its term zero.
//   term 1 (TERM2 false): rows a of D(A,B) times H(B,F) columns c = (beta, f),
//     16 rows a and 16 columns c per tile; element (a, c) goes to
//     X1[beta][a nF + f - k0].
//   term 2 (TERM2 true): rows beta of H(B,A) at one a times D(F,B) columns f,
//     16 f per tile; element (beta, f) goes to X2[beta][a nF + f - k0].
// DIRECT: the H slices are read from global memory (chunks whose slices
// exceed the LDS stage); otherwise from the stage.
template <class T, bool DIRECT, int NU, int XW, bool TERM2>
__device__ __forceinline__ void xterm(const UnitGeo& U, int nB, const T* H, int hs, const T* Dm, T* X,
                                      int first, int Nt, int q, int g) {
  const int nBp = (nB + 3) & ~3;   // b extent of the k-steps
  const int ldD = d_stride(nB);    // row stride of the staged D blocks
  const int SB = nBp >> 2;
  // b strides of the A and B operands
  const int as = TERM2 ? hs : 1, bs = TERM2 ? 1 : hs;
  using M = M4<T>;
  // NUx tiles t0, t0 + XW, ... in flight
  auto tiles = [&](auto nu, int t0) __attribute__((always_inline)) {
    constexpr int NUx = decltype(nu)::value;
    const T* ap[NUx];
    const T* bp[NUx];
    T* xb[NUx];
    int kb[NUx], ar[NUx];
#pragma unroll
    for (int u = 0; u < NUx; ++u) {
      const int t = t0 + XW * u;
      if constexpr (!TERM2) {
        const int rt = U.dnF(t), tc = t - rt * U.nF, c = 16 * tc + q, be = U.dnF(c), f = c - be * U.nF;
        ar[u] = U.a0 + 16 * rt;
        ap[u] = Dm + __umul24((unsigned)min(ar[u] + q, U.nA - 1), (unsigned)ldD);
        bp[u] = H + c;
        xb[u] = X + __umul24((unsigned)be, (unsigned)U.XS);
        kb[u] = ar[u] * U.nF + f - U.k0;
      } else {
        const int ai = U.TF == 2 ? t >> 1 : t, tf = t - ai * U.TF, a = U.a0 + ai, f = 16 * tf + q;
        ap[u] = H + __umul24((unsigned)q, (unsigned)U.nA) + a;
        bp[u] = Dm + __umul24((unsigned)min(f, U.nF - 1), (unsigned)ldD);
        xb[u] = X;
        kb[u] = f < U.nF ? a * U.nF + f - U.k0 : -1;   // -1: the lane's column is not stored
        ar[u] = 0;
      }
    }
    typename M::acc acc[NUx];
#pragma unroll
    for (int u = 0; u < NUx; ++u) acc[u] = typename M::acc{0, 0, 0, 0};
    if constexpr (!DIRECT) {
      // every operand is in the stage for b < nBp: plain loads one k-step
      // ahead, addresses advanced by a fixed stride
#pragma unroll
      for (int u = 0; u < NUx; ++u) {
        ap[u] += __umul24((unsigned)g, (unsigned)as);
        bp[u] += __umul24((unsigned)g, (unsigned)bs);
      }
      // two register sets in turn: the loads of step st+1 are in flight
      // while the product of step st is issued
      T a0[NUx], b0[NUx], a1[NUx], b1[NUx];
      auto next = [&](T (&av)[NUx], T (&bv)[NUx]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NUx; ++u) {
          av[u] = *ap[u];
          bv[u] = *bp[u];
          ap[u] += 4 * as;
          bp[u] += 4 * bs;
        }
      };
      next(a0, b0);
      int st = 0;
#pragma unroll 1
      for (; st + 2 < SB; st += 2) {   // steps st, st+1; the loads run one step ahead
        next(a1, b1);
#pragma unroll
        for (int u = 0; u < NUx; ++u) acc[u] = M::mma(a0[u], b0[u], acc[u]);
        next(a0, b0);
#pragma unroll
        for (int u = 0; u < NUx; ++u) acc[u] = M::mma(a1[u], b1[u], acc[u]);
      }
      if (st + 1 < SB) next(a1, b1);   // the last one or two steps
#pragma unroll
      for (int u = 0; u < NUx; ++u) acc[u] = M::mma(a0[u], b0[u], acc[u]);
      if (st + 1 < SB) {
#pragma unroll
        for (int u = 0; u < NUx; ++u) acc[u] = M::mma(a1[u], b1[u], acc[u]);
      }
    } else {
      // the D operand (stage) is read at b < nBp, zero past nB; the H operand
      // (global) at min(b, nB - 1), finite.  The operands of the next pass
      // are requested before the products of the current one.
      T av[NUx][2], bv[NUx][2];
      auto load = [&](int s0, T (&a2)[NUx][2], T (&b2)[NUx][2]) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int b = min(4 * (s0 + s) + g, nBp - 1), bc = min(b, nB - 1);
          const int ba = TERM2 ? bc : b, bb = TERM2 ? b : bc;
#pragma unroll
          for (int u = 0; u < NUx; ++u) {
            a2[u][s] = ap[u][__umul24((unsigned)ba, (unsigned)as)];
            b2[u][s] = bp[u][__umul24((unsigned)bb, (unsigned)bs)];
          }
        }
      };
      load(0, av, bv);
#pragma unroll 1
      for (int s0 = 0; s0 < SB; s0 += 2) {
        T an[NUx][2], bn[NUx][2];
        load(s0 + 2, an, bn);
#pragma unroll
        for (int u = 0; u < NUx; ++u) acc[u] = M::mma(av[u][0], bv[u][0], acc[u]);
        if (s0 + 1 < SB) {   // an odd last pass has one k-step
#pragma unroll
          for (int u = 0; u < NUx; ++u) acc[u] = M::mma(av[u][1], bv[u][1], acc[u]);
        }
#pragma unroll
        for (int u = 0; u < NUx; ++u)
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            av[u][s] = an[u][s];
            bv[u][s] = bn[u][s];
          }
      }
    }
#pragma unroll
    for (int u = 0; u < NUx; ++u) {
      if constexpr (!TERM2) {
        // rows r < rfull lie wholly inside the unit's columns [k0, k0 + Kc)
        // (uniform); other rows are checked per element (rows past nA fall
        // past the unit's columns)
        const int rfull = ar[u] * U.nF >= U.k0 ? min(16, (U.k0 + U.Kc) / U.nF - ar[u]) : 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = kb[u] + M::row(g, i) * U.nF;
          if (M::row(3, i) < rfull)
            xb[u][k] = acc[u][i];
          else if ((unsigned)k < (unsigned)U.Kc)
            xb[u][k] = acc[u][i];
        }
      } else {
        if ((unsigned)kb[u] < (unsigned)U.Kc) {
#pragma unroll
          for (int i = 0; i < 4; ++i) xb[u][(int)__umul24((unsigned)M::row(g, i), (unsigned)U.XS) + kb[u]] = acc[u][i];
        }
      }
    }
  };
  // groups of NU tiles, then the wave's last tile alone when NU does not divide its share
  int t0 = first;
  for (; t0 + XW * (NU - 1) < Nt; t0 += XW * NU) tiles(std::integral_constant<int, NU>{}, t0);
  if constexpr (NU > 1) {
    for (; t0 < Nt; t0 += XW) tiles(std::integral_constant<int, 1>{}, t0);
  }
}

template <class T, bool DIRECT, int NU, int XW>
__device__ __forceinline__ void xbuild(const UnitGeo& U, int nB, const T* HF, int hsF, const T* HA, int hsA,
                                       const T* Dab, const T* Dfb, T* X1, T* X2, int w, int q,
                                       int g) {
  xterm<T, DIRECT, NU, XW, false>(U, nB, HF, hsF, Dab, X1, w, U.N1, q, g);
  xterm<T, DIRECT, NU, XW, true>(U, nB, HA, hsA, Dfb, X2, ((w - U.N1) % XW + XW) % XW, U.N2, q, g);
}

// Roles of a wave in a unit: a Z wave (units whose V pairs form Z, B >= A at
// the Gamma point: Z and Y are both formed), a Y wave beside four Z waves, or
// one of eight Y waves (units whose V pairs do not form Z: Z(A,B) is the
// transpose of the mirror pair's Z, which the units of the mirror's atom
// form, so only Y is formed).
enum Role : int { kRoleZ = 0, kRoleY = 1, kRoleY8 = 2 };

template <int MT, int P, int ROLE>
__device__ __forceinline__ void triple_role(const Dev& d, const UnitGeo& U, typename TripleCfg<MT, P>::T* __restrict__ X1,
                            typename TripleCfg<MT, P>::A* __restrict__ Zred, typename TripleCfg<MT, P>::T* __restrict__ S,
                            const typename TripleCfg<MT, P>::T* __restrict__ Dg,
                            const typename TripleCfg<MT, P>::T* __restrict__ Vg,
                            const typename TripleCfg<MT, P>::T* __restrict__ Hg, int w, int lane, int q, int g) {
  using Cfg = TripleCfg<MT, P>;
  using T = typename Cfg::T;
  using M = M4<T>;
  using Acc = typename M::acc;           // d4 (FP64) or f4 (FP32, BF16x3)
  using A = typename Cfg::A;
  constexpr bool B3 = P == kPB3;
  constexpr bool ZROLE = ROLE == kRoleZ;
  constexpr int NYW = ROLE == kRoleY8 ? 8 : 4;                      // Y waves of the unit
  constexpr int JW = ROLE == kRoleY8 ? Cfg::kJW8 : Cfg::kJW;          // Y column tiles per Y wave
  constexpr int NU = ZROLE ? Cfg::kNUZ : (ROLE == kRoleY8 ? Cfg::kNUY8 : Cfg::kNUY);
  // X1 and X2 (X), Zred (partial Z tiles on their way to the owning wave) and
  // S (the chunk stage) are distinct LDS objects
  T* X2 = X1 + 16 * Cfg::kXS;
  const int ww = ROLE == kRoleY8 ? w : (w & 3);   // index among the waves of the role
  const int N = d.N;
  const int mA = U.mA, XS = U.XS;
  const T* Cf = Buf<T>::Cf(d);

  // ---- resident operands / accumulators of the role ----------------------
  constexpr int ZI = ZROLE ? MT : 1, ZT = ZROLE ? Cfg::kKSW : 1;
  constexpr int YI = ZROLE ? 1 : MT, YJ = ZROLE ? 1 : JW;
  T cfr[B3 ? 1 : ZI][B3 ? 1 : ZT];
  s4 cfh[B3 ? ZI : 1][B3 ? ZT : 1], cfl[B3 ? ZI : 1][B3 ? ZT : 1];
  Acc yacc[YI][YJ];
  if constexpr (ZROLE) {
    const T* Cfp = Cf + ldu(d.cfOff, U.cp);
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
      for (int j = 0; j < JW; ++j) yacc[i][j] = Acc{0, 0, 0, 0};
  }
  // column tiles of this Y wave that reach the chunk's columns
  const int nYJ = min(JW, (U.NTc - ww + NYW - 1) / NYW);

  // prologue: stage the first chunk
  constexpr int VMASK = ROLE == kRoleY8 ? 1 : 3;
  Chunk ch = chunk_at<VMASK>(d, U, U.vb, 0);
  StageGeo sg = stage_geo<T>(U, ch.nB);
  if (ch.p >= 0) {
    Stager<T> st;
    st.init(d, U, ch, sg, true, sg.hend <= Cfg::kStage, S, Dg, Vg, Hg);
    for (int J = w; J < st.n; J += 8) st.issue(J, lane, U);
  }
  __builtin_amdgcn_s_waitcnt(0);
  lds_sync();
  while (ch.p >= 0) {
    const Chunk nx = chunk_next<VMASK>(d, U, ch);
    const int64_t tri = chunk_tri(d, U, ch);
    // V fragments of this chunk (Y waves), read before the stage is reused
    T avn[(ZROLE || B3) ? 1 : 4][(ZROLE || B3) ? 1 : MT];
    s4 avh[(!ZROLE && B3) ? MT : 1], avl[(!ZROLE && B3) ? MT : 1];
    if constexpr (!ZROLE) {
      // element (16 i + q, be) of the staged V is 256 i + vs_index(q, be);
      // rows past mA read other (finite) stage contents and only feed
      // accumulator rows that are never stored
      const T* Vs = S + sg.vo;
      if constexpr (B3) {
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          float v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = Vs[256 * i + vs_index<T>(q, 4 * g + j)];
          split4(v, avh[i], avl[i]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int i = 0; i < MT; ++i) avn[s][i] = Vs[256 * i + vs_index<T>(q, 4 * s + g)];
      }
    }
    // ---- X-build of this chunk (all waves) ------------------------------
    if (!ZROLE && Cfg::kXW == 4) {
    } else if (sg.hend <= Cfg::kStage) {
      xbuild<T, false, NU, Cfg::kXW>(U, ch.nB, S + sg.ho, 16 * U.nF, S + sg.ho + ch.nB * 16 * U.nF, 16 * U.nA, S,
                              S + U.nA * sg.ldD, X1, X2, w, q, g);
    } else {
      xbuild<T, true, NU, Cfg::kXW>(U, ch.nB, Hg + ldu(d.triHF, tri) + (int64_t)ch.b0 * ch.nB * U.nF, 16 * U.nF,
                             Hg + ldu(d.triHA, tri) + (int64_t)ch.b0 * ch.nB * U.nA, 16 * U.nA, S, S + U.nA * sg.ldD,
                             X1, X2, w, q, g);
    }
    lds_sync();
    // ---- stage the next chunk while this one is contracted --------------
    // Each role reads its X operands first and only then issues the loads of
    // the next chunk: an LDS read placed after those loads would wait for
    // them to land (the compiler cannot tell the stage from X).
    const StageGeo sn = stage_geo<T>(U, nx.nB);
    // a new B: zero the padding columns of its D blocks before any wave
    // issues the loads that stage them
    if (nx.p >= 0 && nx.p != ch.p)
      zero_d_padding(U, nx.nB, ldu(d.keepD, (int64_t)U.A * N + nx.B) != 0, ldu(d.keepD, (int64_t)U.F * N + nx.B) != 0, S);
    auto stage_next = [&]() __attribute__((always_inline)) {
      if (nx.p >= 0) {
        Stager<T> st;
        st.init(d, U, nx, sn, nx.p != ch.p, sn.hend <= Cfg::kStage, S, Dg, Vg, Hg);
        for (int J = w; J < st.n; J += 8) st.issue(J, lane, U);
      }
    };
    if constexpr (ZROLE) {
      Acc zp[MT];
#pragma unroll
      for (int i = 0; i < MT; ++i) zp[i] = Acc{0, 0, 0, 0};
      if constexpr (B3) {
        // k-steps past the chunk's columns meet zero Cf fragments; their X
        // reads may leave the row, so the values are dropped as well
        s4 bh[Cfg::kKSW], bl[Cfg::kKSW];
#pragma unroll
        for (int t = 0; t < Cfg::kKSW; ++t) {
          const int ks = ww + 4 * t;
          float v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int c = min(16 * ks + 4 * g + j, XS - 1);
            v[j] = ks < U.NTc ? X1[q * XS + c] + X2[q * XS + c] : 0.f;
          }
          split4(v, bh[t], bl[t]);
        }
        stage_next();
        // k-steps past the chunk's columns are skipped (uniform per wave)
#pragma unroll
        for (int t = 0; t < Cfg::kKSW; ++t) {
          if (ww + 4 * t >= U.NTc) break;
#pragma unroll
          for (int i = 0; i < MT; ++i) zp[i] = mma_bf16x3(cfh[i][t], cfl[i][t], bh[t], bl[t], zp[i]);
        }
      } else {
        // columns 4 ks + g < kCols < XS; past the chunk's columns X and the
        // Cf fragments are zero
        T xb[Cfg::kKSW];
#pragma unroll
        for (int t = 0; t < Cfg::kKSW; ++t) {
          const int c = (int)__umul24((unsigned)q, (unsigned)XS) + 4 * (ww + 4 * t) + g;
          xb[t] = X1[c] + X2[c];
        }
        stage_next();
        // k-steps past the chunk's columns are skipped (uniform per wave)
#pragma unroll
        for (int t = 0; t < Cfg::kKSW; ++t) {
          if (ww + 4 * t >= U.KS) break;
#pragma unroll
          for (int i = 0; i < MT; ++i) zp[i] = M::mma(cfr[i][t], xb[t], zp[i]);
        }
      }
      // tile i < MF is owned by Z wave (i mod 4): the other three park their
      // partials; a remaining tile is parked by all four Z waves, and wave ww
      // adds accumulator component ww of the four
      constexpr int MF = Cfg::kMF;
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        if (i < MF) {
          const int own = i & 3;
          if (own != ww) *(Acc*)&Zred[(((ww - own - 1) & 3) * MF + i) * 256 + lane * 4] = zp[i];
        } else {
          *(Acc*)&Zred[(3 * MF + 4 * (i - MF) + ww) * 256 + lane * 4] = zp[i];
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      lds_sync();
      T* Zdst = Buf<T>::Z(d) + ldu(d.zOff, tri) + (int64_t)U.kc * mA * ch.mB;
      const int be = ch.b0 + q;
      // 32-bit byte offsets from the uniform block base (a Z block is far below 4 GiB)
      auto zstore = [&](int al, T v) __attribute__((always_inline)) {
        if (al < mA && be < ch.mB) *(T*)((char*)Zdst + (unsigned)(al * ch.mB + be) * (unsigned)sizeof(T)) = v;
      };
#pragma unroll
      for (int i = 0; i < MF; ++i) {
        if ((i & 3) != ww) continue;
        Acc z = zp[i];
#pragma unroll
        for (int v = 0; v < 3; ++v) z += *(const Acc*)&Zred[(v * MF + i) * 256 + lane * 4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) zstore(16 * i + M::row(g, rr), z[rr]);
      }
#pragma unroll
      for (int i = MF; i < MT; ++i) {
        const A* zr = Zred + (3 * MF + 4 * (i - MF)) * 256 + lane * 4 + ww;
        T z = zr[0];
#pragma unroll
        for (int v = 1; v < 4; ++v) z += zr[256 * v];
        zstore(16 * i + M::row(g, ww), z);
      }
    } else {
      if constexpr (B3) {
        // column tiles j >= NTc accumulate values that are never stored
        s4 bh[JW], blo[JW];
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
          if (jj == JW - 1 && jj >= nYJ) break;
          const int j = ww + NYW * jj;
          float v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int bl = 4 * g + k, c = min(16 * j + q, XS - 1);
            v[k] = X1[bl * XS + c] + X2[bl * XS + c];
          }
          split4(v, bh[jj], blo[jj]);
        }
        stage_next();
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
          if (jj == JW - 1 && jj >= nYJ) break;
#pragma unroll
          for (int i = 0; i < MT; ++i) yacc[i][jj] = mma_bf16x3(avh[i], avl[i], bh[jj], blo[jj], yacc[i][jj]);
        }
      } else {
        // column tiles j >= NTc accumulate values that are never stored; the
        // last tile of a wave is skipped when it lies past the chunk
        constexpr int JF = JW - 1;
        T xb[4][JW];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int jj = 0; jj < JF; ++jj) {
            const int bl = 4 * s + g, c = min(16 * (ww + NYW * jj) + q, XS - 1);
            const int e = (int)__umul24((unsigned)bl, (unsigned)XS) + c;
            xb[s][jj] = X1[e] + X2[e];
          }
        if (JF < nYJ) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int bl = 4 * s + g, e = (int)__umul24((unsigned)bl, (unsigned)XS) + 16 * (ww + NYW * JF) + q;
            xb[s][JF] = X1[e] + X2[e];
          }
        }
        stage_next();
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int jj = 0; jj < JF; ++jj)
#pragma unroll
            for (int i = 0; i < MT; ++i) yacc[i][jj] = M::mma(avn[s][i], xb[s][jj], yacc[i][jj]);
        if (JF < nYJ) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < MT; ++i) yacc[i][JF] = M::mma(avn[s][i], xb[s][JF], yacc[i][JF]);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      lds_sync();
    }
    ch = nx;
    sg = sn;
  }
  if constexpr (!ZROLE) {
    T* Y = Buf<T>::Y(d) + ldu(d.yOff, U.cp) + (int64_t)U.split * mA * U.K1;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int jj = 0; jj < JW; ++jj) {
        const int j = ww + NYW * jj;
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

// One work unit of structure d: geometry, X cleared, then the two roles.
template <int MT, int P>
__device__ __forceinline__ void triple_unit(const Dev& d, int u, typename TripleCfg<MT, P>::T* X,
                                            typename TripleCfg<MT, P>::A* Zred, typename TripleCfg<MT, P>::T* S) {
  using Cfg = TripleCfg<MT, P>;
  using T = typename Cfg::T;
  UnitGeo U;
  U.cp = ldu(d.unitCp, u);
  if (!ldu(d.aliveC, U.cp)) return;
  U.A = ldu(d.cpA, U.cp);
  U.F = ldu(d.cpF, U.cp);
  U.mA = ldu(d.nabf, U.A);
  U.nA = ldu(d.nao, U.A);
  U.nF = ldu(d.nao, U.F);
  U.K1 = U.nA * U.nF;
  U.k0 = ldu(d.unitK0, u);
  U.Kc = ldu(d.unitK1, u) - U.k0;
  U.kc = ldu(d.unitKc, u);
  U.NTc = (U.Kc + 15) >> 4;
  U.KS = U.NTc * 4;
  U.XS = U.NTc * 16 + 1;
  U.fpos = U.cp - ldu(d.cpRow, U.A);
  U.vp0 = ldu(d.vpRow, U.A);
  U.nVpA = ldu(d.vpRow, U.A + 1) - U.vp0;
  U.vb = ldu(d.unitV0, u);
  U.ve = ldu(d.unitV1, u);
  U.split = ldu(d.unitS, u);
  U.dnF.init(U.nF);
  U.a0 = U.dnF(U.k0);
  const int a1 = U.dnF(U.k0 + U.Kc - 1);
  U.N1 = ((a1 - U.a0) / 16 + 1) * U.nF;
  U.TF = (U.nF + 15) >> 4;
  U.N2 = (a1 - U.a0 + 1) * U.TF;
  U.pF = 16 * U.nF * (int)sizeof(T) / 16;
  U.pA = 16 * U.nA * (int)sizeof(T) / 16;
  const int tid = threadIdx.x, lane = tid & 63, q = lane & 15, g = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, uniform
  for (int e = tid; e < 32 * Cfg::kXS; e += kTNT) X[e] = T(0);
  // the stage starts zeroed: padding rows the X-build reads past nB are finite
  for (int e = tid; e < Cfg::kStage; e += kTNT) S[e] = T(0);
  __syncthreads();
  // Y alone when Z is not formed here (the mirror pairs form it) or Cf(A,F) folds to
  // zero; then nothing when Y(A,F) is not read, else only V pairs with
  // Vf != 0 (the role is read here, not before the geometry: that placement
  // keeps the persistent FP64 kernels free of register spills)
  const int role = ldu(d.unitRole, u);
  if (role == 0) return;
  if (role == 2)
    triple_role<MT, P, kRoleY8>(d, U, X, Zred, S, Buf<T>::D(d), Buf<T>::Vf(d), Buf<T>::H(d), w, lane, q, g);
  else if (w < 4)
    triple_role<MT, P, kRoleZ>(d, U, X, Zred, S, Buf<T>::D(d), Buf<T>::Vf(d), Buf<T>::H(d), w, lane, q, g);
  else
    triple_role<MT, P, kRoleY>(d, U, X, Zred, S, Buf<T>::D(d), Buf<T>::Vf(d), Buf<T>::H(d), w, lane, q, g);
}

// items[i] = (structure index into devs, unit index of that structure).
// PERSIST = false: one workgroup per item.  PERSIST = true: kPersistentGrid
// workgroups; workgroup b first drains segment (b mod 8) of the item list,
// then the other seven, taking items through one counter per segment (the
// counters start at zero).  Every workgroup leaves once all eight segments
// report exhausted.
template <int MT, int P, bool PERSIST>
__global__ void __launch_bounds__(kTNT, 1)
    k_triple(DevBatch devs, const int2* __restrict__ items, int n, int* __restrict__ counters) {
  using Cfg = TripleCfg<MT, P>;
  // LDS: X, the parked Z partials and the chunk stage (the compiler does not
  // tell them apart for the direct global->LDS loads, so every wave reads its
  // X operands before it issues the next chunk's loads), and the item slot
  __shared__ __attribute__((aligned(16))) typename Cfg::T sX[2 * 16 * Cfg::kXS];
  __shared__ __attribute__((aligned(16))) typename Cfg::A sZ[Cfg::kZSlots * 256];
  __shared__ __attribute__((aligned(16))) typename Cfg::T sS[Cfg::kStage];
  __shared__ int s_next;
  if constexpr (!PERSIST) {
    const int2 it = items[xcd_remap(blockIdx.x, gridDim.x)];
    triple_unit<MT, P>(devs.s[it.x], it.y, sX, sZ, sS);
  } else {
    const int q = (n + 7) >> 3;
    for (int k = 0; k < 8; ++k) {
      const int seg = (blockIdx.x + k) & 7;
      const int s0 = seg * q, s1 = min(n, s0 + q);
      for (;;) {
        if (threadIdx.x == 0) s_next = s0 + atomicAdd(&counters[seg], 1);
        __syncthreads();
        // every lane read the same slot: made uniform, so the item, its
        // structure and everything derived from them live in scalar registers
        const int i = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
        if (i >= s1) break;
        const int* it = (const int*)items + 2 * i;
        triple_unit<MT, P>(devs.s[ldu(it, 0)], ldu(it, 1), sX, sZ, sS);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Z(A,B) = sum over live (A,F) and column chunks of the Z partials; then, in
// one pass over the pair's blocks, E = -<Vf, Z> and g_v = -<dV_v, Z> (FP64).
// Only pairs that form Z (A <= B at the Gamma point): the mirror pair (B,A)
// has Z(B,A) = Z(A,B)^T and Vf(B,A) = Vf(A,B)^T, so its energy term is the
// same, and each mirror block (B,A,-R) has dV = -dV(A,B,R)^T, so its
// gradient is -g_v (input checks hold these symmetries to 1e-12 relative).
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
  if (!d.vpZ[p]) return;   // written by the mirror pair, which forms Z
  const int A = d.vpA[p], B = d.vpB[p];
  const int pm = d.vpMir[p];
  const bool mirror = pm != p;   // the mirror's energy term and V gradients are written here too
  const int mA = d.nabf[A], mB = d.nabf[B], n = mA * mB;
  if (!d.aliveV[p]) {
    for (int k = d.vpB0[p] + threadIdx.x; k < d.vpB1[p]; k += kNT) {
      const int64_t b = d.vpBlk[k], bm = d.Vmir[b];
      d.gV[3 * b] = d.gV[3 * b + 1] = d.gV[3 * b + 2] = 0.0;
      if (mirror) d.gV[3 * bm] = d.gV[3 * bm + 1] = d.gV[3 * bm + 2] = 0.0;
    }
    if (threadIdx.x == 0) {
      d.Ep[p] = 0.0;
      if (mirror) d.Ep[pm] = 0.0;
    }
    return;
  }
  {
    const int vp0 = d.vpRow[A], nVpA = d.vpRow[A + 1] - vp0, bpos = p - vp0;
    const int c0 = d.cpRow[A], ncp = d.cpRow[A + 1] - c0;
    for (int i = threadIdx.x; i < ncp && i < kZMax; i += kNT) {
      zk[i] = (d.aliveC[c0 + i] & 1) ? d.nkc[c0 + i] : 0;   // Cf(A,F) = 0 adds nothing
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
  const double* vf = d.Vf + d.vfOff[p];   // rows padded to 16 elements
  const int mBp = (mB + 15) & ~15;
  Div dmB;
  dmB.init(mB);
  const int kb0 = d.vpB0[p], kb1 = d.vpB1[p];
  for (int k0 = kb0; k0 < kb1 || k0 == kb0; k0 += kZB) {
    const int nb = max(0, min(kZB, kb1 - k0));
    const double* dv[kZB];
    bool kp[kZB];
#pragma unroll
    for (int j = 0; j < kZB; ++j) {
      const int64_t b = d.vpBlk[j < nb ? k0 + j : kb0];
      kp[j] = j < nb && (d.keepV[b] & 2);   // in the derivative list
      dv[j] = d.Vdval + 3 * d.Voff[b];
    }
    double acc[1 + 3 * kZB];
#pragma unroll
    for (int j = 0; j < 1 + 3 * kZB; ++j) acc[j] = 0.0;
    const bool first = k0 == kb0;
    for (int e = threadIdx.x; e < n; e += kNT) {
      double z = 0;
      for (int k = 0; k < NZ; ++k) z += (double)Zb[zoff[k] + e];
      if (first) {
        const int al = dmB(e);
        acc[0] += vf[al * mBp + (e - al * mB)] * z;
      }
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
      if (first) {
        d.Ep[p] = -acc[0];
        if (mirror) d.Ep[pm] = -acc[0];
      }
      for (int j = 0; j < nb; ++j) {
        const int64_t b = d.vpBlk[k0 + j];
        for (int x = 0; x < 3; ++x) d.gV[3 * b + x] = kp[j] ? -acc[1 + 3 * j + x] : 0.0;
        if (mirror) {
          const int64_t bm = d.Vmir[b];
          for (int x = 0; x < 3; ++x) d.gV[3 * bm + x] = kp[j] ? acc[1 + 3 * j + x] : 0.0;
        }
      }
    }
    if (kb1 <= kb0) break;
  }
}

// ---------------------------------------------------------------------------
// C-block gradients: g_c = -2 <dC_c, Y(A,F)> (FP64).
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
    return;
  }
  const T* Y = Buf<T>::Y(d) + d.yOff[cp];
  const int ns = d.nsplit[cp];
  for (int k = d.cpB0[cp]; k < d.cpB1[cp]; ++k) {
    const int64_t b = d.cpBlk[k];
    if (!(d.keepC[b] & 2)) {   // not in the derivative list
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
  __shared__ double sh[(kFinalNT / 64) * 10];
  double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // E, W[9]
  for (int p = threadIdx.x; p < d.nVp; p += kFinalNT) v[0] += d.Ep[p];
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
  block_sum_n<10>(v, sh);
  if (threadIdx.x == 0) {
    d.out[0] = v[0];
    for (int i = 0; i < 9; ++i) d.out[1 + 3 * d.N + i] = -v[1 + i] / d.omega;
  }
}

static inline unsigned grid1(int64_t n, int64_t b) { return (unsigned)(n > 0 ? (n + b - 1) / b : 1); }

__global__ void k_fill_i32(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <int MT, int P>
static void launch_triple(const TripleLaunch& tl, hipStream_t s) {
  const int n = tl.n[MT];
  if (n <= 0) return;
  if (tl.mode[MT] == 1) {
    int* cnt = tl.counters + 8 * MT;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, cnt, 8, 0);
    hipLaunchKernelGGL((k_triple<MT, P, true>), dim3(kPersistentGrid), dim3(kTNT), 0, s, tl.devs, tl.items[MT], n,
                       cnt);
  } else {
    hipLaunchKernelGGL((k_triple<MT, P, false>), dim3(n), dim3(kTNT), 0, s, tl.devs, tl.items[MT], n,
                       (int*)nullptr);
  }
}

template <int P>
static void launch_triple_mt(const TripleLaunch& tl, int mt, hipStream_t st) {
  switch (mt) {
    case 1: launch_triple<1, P>(tl, st); break;
    case 2: launch_triple<2, P>(tl, st); break;
    case 3: launch_triple<3, P>(tl, st); break;
    case 4: launch_triple<4, P>(tl, st); break;
    case 5: launch_triple<5, P>(tl, st); break;
    case 6: launch_triple<6, P>(tl, st); break;
    case 7: launch_triple<7, P>(tl, st); break;
    default: launch_triple<8, P>(tl, st); break;
  }
}

void launch_triple_group(const TripleLaunch& tl, int mt, int prec, hipStream_t s) {
  if (prec == kP64)
    launch_triple_mt<kP64>(tl, mt, s);
  else if (prec == kP32)
    launch_triple_mt<kP32>(tl, mt, s);
  else
    launch_triple_mt<kPB3>(tl, mt, s);
}

void launch_hbuild(const Dev& d, int prec, hipStream_t s) {
  if (!d.nHB) return;
  const bool bvk = d.ncell > 1;
  if (prec == kP64) {
    if (bvk)
      hipLaunchKernelGGL((k_hbuild<double, true>), dim3(d.nHB), dim3(kHT), 0, s, d);
    else
      hipLaunchKernelGGL((k_hbuild<double, false>), dim3(d.nHB), dim3(kHT), 0, s, d);
  } else {
    if (bvk)
      hipLaunchKernelGGL((k_hbuild<float, true>), dim3(d.nHB), dim3(kHT), 0, s, d);
    else
      hipLaunchKernelGGL((k_hbuild<float, false>), dim3(d.nHB), dim3(kHT), 0, s, d);
  }
}

void launch_triples(const TripleLaunch& tl, int prec, hipStream_t s, const hipStream_t* side, const hipEvent_t* fork,
                    hipEvent_t* gev) {
  // The alpha-tile groups are independent: the largest runs on the main
  // stream, the others on side streams that join back before the gradients.
  int order[kMaxAlphaTiles];
  int ng = 0;
  for (int mt = 1; mt <= kMaxAlphaTiles; ++mt)
    if (tl.n[mt] > 0) order[ng++] = mt;
  for (int i = 1; i < ng; ++i)
    for (int j = i; j > 0 && tl.n[order[j]] > tl.n[order[j - 1]]; --j) {
      const int t = order[j];
      order[j] = order[j - 1];
      order[j - 1] = t;
    }
  (void)hipEventRecord(fork[0], s);
  for (int i = 0; i < ng; ++i) {
    const hipStream_t st = i == 0 ? s : side[(i - 1) % kSideStreams];
    if (i > 0 && i <= kSideStreams) (void)hipStreamWaitEvent(st, fork[0], 0);
    if (gev) (void)hipEventRecord(gev[2 * order[i]], st);
    launch_triple_group(tl, order[i], prec, st);
    if (gev) (void)hipEventRecord(gev[2 * order[i] + 1], st);
  }
  for (int i = 1; i <= kSideStreams && i < ng; ++i) {
    (void)hipEventRecord(fork[i], side[i - 1]);
    (void)hipStreamWaitEvent(s, fork[i], 0);
  }
}

template <class T>
static void launch_grads_t(const Dev& d, hipStream_t s, hipEvent_t* ev) {
  if (d.nVp) hipLaunchKernelGGL(k_zgrad<T>, dim3(d.nVp), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[6], s);
  if (d.nCp) hipLaunchKernelGGL(k_cgrad<T>, dim3(d.nCp), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[7], s);
  hipLaunchKernelGGL(k_forces, dim3(grid1(d.N, kNT)), dim3(kNT), 0, s, d);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kFinalNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[8], s);
}

void launch_grads(const Dev& d, int prec, hipStream_t s, hipEvent_t* ev) {
  if (prec == kP64)
    launch_grads_t<double>(d, s, ev);
  else
    launch_grads_t<float>(d, s, ev);
}

void launch_contract(const Dev& d, const TripleLaunch& tl, int prec, hipStream_t s, const hipStream_t* side,
                     const hipEvent_t* fork, hipEvent_t* ev, hipEvent_t* gev) {
  launch_hbuild(d, prec, s);
  if (ev) (void)hipEventRecord(ev[4], s);
  launch_triples(tl, prec, s, side, fork, gev);
  if (ev) (void)hipEventRecord(ev[5], s);
  launch_grads(d, prec, s, ev);
}

}  // namespace lrx
