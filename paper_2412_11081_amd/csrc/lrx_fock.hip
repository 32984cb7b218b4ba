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
//               then the contractions with the staged D block and H slice,
//               also on the matrix cores.  Four launches by the 16-wide
//               tile counts of b and x; slots in (X, B) order per XCD.
//   k_hx_g3     one workgroup per D block (G,X) that a C partner B of G
//               reaches through an H slot (B,X): G3 over those B, on the
//               matrix cores.
//   k_hx_final  32 x 32 tiles: (G + G^T) / 2 on kept D pairs, and the tile's
//               share of <H^X, D> / 2; k_hx_sum adds the shares in order.
// No atomics: every output element has one writer, so two calls agree bit
// for bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lrx_internal.h"

namespace lrx {

namespace {

constexpr int kHxNT = 256;
static_assert(kMaxNao <= 32, "two 16-wide tiles per NAO index");

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
// and B[k = g][n = q] = Cf[4 s + g][16 j + q]; result i is row g + 4 i.  Of
// NW waves, a wave keeps up to three column tiles (j, j + NW, j + 2 NW) in
// flight, as many as remain below nj; they share the Vf operand.  Loads are
// unconditional from clamped addresses (no branches in the loop): only the
// A operand of a k past mA is set to zero; columns past K1 within a tile are
// computed from clamped data and not stored.
template <int NTL>
__device__ inline void q_pass(const double* __restrict__ vq, int ldv, const double* __restrict__ Cf, int mA, int K1,
                              int ns, const int (&c)[3], double* Q, int g) {
  int d[NTL];
#pragma unroll
  for (int i = 0; i < NTL; ++i) d[i] = min(c[i], K1 - 1);
  d4 acc[NTL];
#pragma unroll
  for (int i = 0; i < NTL; ++i) acc[i] = d4{0, 0, 0, 0};
  // four k-steps per pass, their loads issued before the products (a step
  // past ns has al >= mA: zero A operand)
  for (int s0 = 0; s0 < ns; s0 += 4) {
    double a[4], b[4][NTL];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int al = 4 * (s0 + u) + g, ac = min(al, mA - 1);
      const double* cr = Cf + (int64_t)ac * K1;
      const double av = vq[(int64_t)ac * ldv];
      a[u] = al < mA ? av : 0.0;
#pragma unroll
      for (int i = 0; i < NTL; ++i) b[u][i] = cr[d[i]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < NTL; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][i], acc[i], 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = (g + 4 * r) * K1;
#pragma unroll
    for (int i = 0; i < NTL; ++i)
      if (c[i] < K1) Q[row + c[i]] = acc[i][r];
  }
}

template <int NW>
__device__ inline void q_tile(const double* __restrict__ Vf, int ldv, const double* __restrict__ Cf, int mA, int K1,
                              int t, double* Q, int w, int q, int g) {
  const int nj = (K1 + 15) >> 4, ns = (mA + 3) >> 2;
  const double* vq = Vf + 16 * t + q;
  for (int j0 = w; j0 < nj; j0 += 3 * NW) {
    const int c[3] = {16 * j0 + q, 16 * (j0 + NW) + q, 16 * (j0 + 2 * NW) + q};
    if (j0 + 2 * NW < nj)
      q_pass<3>(vq, ldv, Cf, mA, K1, ns, c, Q, g);
    else if (j0 + NW < nj)
      q_pass<2>(vq, ldv, Cf, mA, K1, ns, c, Q, g);
    else
      q_pass<1>(vq, ldv, Cf, mA, K1, ns, c, Q, g);
  }
}

// One triple's contractions with its staged D block Ds [nk][nB] (row k of
// the contracted AO index) and H slice Hb (HS: in LDS; else global memory),
// [b][beta][k] with k < nk:
//   Hbar tile of beta:  acc_h[b][x] += sum_k Ds[k][b] Q[beta][qi(x, k)]
//   G tile:             acc_g[x][b] += sum_{beta, k} Q[beta][qi(x, k)] Hb[b][beta][k]
// qi(x, k) = k nX + x for the first kind of triple (k = a), x nF + k for the
// second (k = f); NTB and NTX 16-wide tiles cover b and x; of NW waves, a
// wave takes beta = w + NW j, j < 16 / NW.  The loads of two k-steps are
// issued before their products; as in q_tile, they come from clamped
// addresses; the Ds and Hb operands of a k past nk (and Ds when the D pair
// is screened) are zero, rows and columns past nB, nX are not stored.
template <int NTB, int NTX, int NW>
__device__ inline void contract_triple(const double* __restrict__ Q, int K1, const double* __restrict__ Ds,
                                       const double* __restrict__ Hb, bool with_d, int nk, int nB, int nX,
                                       int qs_x, int qs_k, d4 (&hacc)[16 / NW][NTB][NTX], d4 (&gacc)[NTX][NTB],
                                       int w, int q, int g) {
  const int nsk = (nk + 3) >> 2;
  int xo[NTX], bo[NTB], hb_[NTB];
#pragma unroll
  for (int u = 0; u < NTX; ++u) xo[u] = min(16 * u + q, nX - 1) * qs_x;
#pragma unroll
  for (int u = 0; u < NTB; ++u) {
    bo[u] = min(16 * u + q, nB - 1);
    hb_[u] = bo[u] * 16 * nk;
  }
#pragma unroll
  for (int j = 0; j < 16 / NW; ++j) {
    const int be = w + NW * j;
    const double* Qb = Q + be * K1;
    const double* Hbe = Hb + be * nk;
    for (int s0 = 0; s0 < nsk; s0 += 2) {
      double qv[2][NTX], dv[2][NTB], hv[2][NTB];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = 4 * (s0 + e) + g, kc = min(k, nk - 1);
        const bool kd = k < nk && with_d, kh = k < nk;
#pragma unroll
        for (int u = 0; u < NTX; ++u) qv[e][u] = Qb[xo[u] + kc * qs_k];
#pragma unroll
        for (int u = 0; u < NTB; ++u) {
          const double dd = Ds[kc * nB + bo[u]];
          const double hh = Hbe[hb_[u] + kc];
          dv[e][u] = kd ? dd : 0.0;
          hv[e][u] = kh ? hh : 0.0;
        }
      }
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int ib = 0; ib < NTB; ++ib)
#pragma unroll
          for (int ix = 0; ix < NTX; ++ix) {
            // Hbar: A[m = b][k] = Ds[k][b], B[k][n = x] = Q[beta][x, k]
            hacc[j][ib][ix] = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[e][ib], qv[e][ix], hacc[j][ib][ix], 0, 0, 0);
            // G: A[m = x][k] = Q[beta][x, k], B[k][n = b] = H[b][beta][k]
            gacc[ix][ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(qv[e][ix], hv[e][ib], gacc[ix][ib], 0, 0, 0);
          }
    }
  }
}

// Waves per SIMD that the register allocation of k_hx_slot<NTB, NTX, ., NW>
// is held to (its Hbar accumulators take 64 NTB NTX / NW doubles per lane):
// three for one tile per index, two for the other launches.
constexpr int slot_waves_per_simd(int NTB, int NTX) { return NTB * NTX == 1 ? 3 : 2; }

// NTB, NTX: 16-wide tiles for the b and x indices; the launch takes the slots
// with ceil(nB / 16) = NTB and ceil(nX / 16) = NTX.  HS: the H slice is
// staged in LDS (else read from global memory).  NW: waves per workgroup (4
// or 8).  LDS: Q [16][K1] (or the NW waves' G partials at the end) in qsize
// doubles, Ds [nk][nB] in dsize, Hs [nB][16][nk].
template <int NTB, int NTX, bool HS, int NW>
__global__ void __launch_bounds__(64 * NW, slot_waves_per_simd(NTB, NTX))
    k_hx_slot(Dev d, double* __restrict__ Hbar, double* __restrict__ G12, int qsize, int dsize) {
  constexpr int kNT = 64 * NW, kJ = 16 / NW;
  extern __shared__ double lds[];
  // the slot's triples: C pair, V pair and third atom (A for the first kind,
  // F for the second); an atom has at most kHxMaxCPartners C partners
  // (checked on the host)
  __shared__ int tcp[2 * kHxMaxCPartners], tvp[2 * kHxMaxCPartners], tat[2 * kHxMaxCPartners];
  __shared__ int ntri;
  double* Q = lds;
  double* Ds = lds + qsize;
  double* Hs = Ds + dsize;
  // Workgroups go round-robin to the 8 XCDs, each with its own L2.  XCD i
  // takes the i-th eighth of the slots in (X, B) order: the slots of one X
  // read the same C^Gamma blocks (Cf(A,X) and Cf(X,F)), which then stay in
  // one L2 while its workgroups walk them.  The grid is a multiple of 8.
  const int o = (int)(blockIdx.x & 7) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
  if (o >= d.nSlot) return;
  const int s = d.slotByX[o];
  if (!d.need[s]) return;
  const int N = d.N;
  const int64_t nt = d.ntot;
  const int B = d.slotB[s], X = d.slotX[s];
  const int mB = d.nabf[B], nB = d.nao[B], nX = d.nao[X];
  if ((nB + 15) / 16 != NTB || (nX + 15) / 16 != NTX) return;   // another launch's slot
  const int ldv = (mB + 15) & ~15, nT = ldv >> 4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  d4 gacc[NTX][NTB];
#pragma unroll
  for (int ix = 0; ix < NTX; ++ix)
#pragma unroll
    for (int ib = 0; ib < NTB; ++ib) gacc[ix][ib] = d4{0, 0, 0, 0};
  // the slot's triples, found once (one thread per candidate partner) and
  // listed in a fixed order: first kind (A, X, B) for the C partners A of X
  // with (A,X) and (A,B) in the value lists, then second kind (X, F, B)
  // for the value-list C pairs (X,F) when (X,B) is in the value list
  {
    const int vpX = find_partner(d.vpB, d.vpRow[X], d.vpRow[X + 1], B);
    const bool kindB = vpX >= 0 && (d.aliveV[vpX] & 1);
    const int nA0 = d.cpRow[X + 1] - d.cpRow[X];
    for (int it = tid; it < 2 * nA0; it += kNT) {
      const bool first = it < nA0;
      const int i = d.cpRow[X] + (first ? it : it - nA0);
      int cp = -1, vp = -1, P = d.cpF[i];
      if (first) {
        cp = find_partner(d.cpF, d.cpRow[P], d.cpRow[P + 1], X);
        vp = find_partner(d.vpB, d.vpRow[P], d.vpRow[P + 1], B);
        if (cp < 0 || !(d.aliveC[cp] & 1) || vp < 0 || !(d.aliveV[vp] & 1)) cp = -1;
      } else if (kindB && (d.aliveC[i] & 1)) {
        cp = i;
        vp = vpX;
      }
      tcp[it] = cp;
      tvp[it] = vp;
      tat[it] = P;
    }
    __syncthreads();
    if (tid == 0) {   // compaction in list order
      int n = 0;
      for (int it = 0; it < 2 * nA0; ++it)
        if (tcp[it] >= 0) {
          tcp[n] = tcp[it];
          tvp[n] = tvp[it];
          tat[n] = it < nA0 ? tat[it] : -1 - tat[it];   // second kind: -1 - F
          ++n;
        }
      ntri = n;
    }
    __syncthreads();
  }
  const int nTri = ntri;
  for (int t = 0; t < nT; ++t) {
    d4 hacc[kJ][NTB][NTX];
#pragma unroll
    for (int j = 0; j < kJ; ++j)
#pragma unroll
      for (int ib = 0; ib < NTB; ++ib)
#pragma unroll
        for (int ix = 0; ix < NTX; ++ix) hacc[j][ib][ix] = d4{0, 0, 0, 0};
    for (int it = 0; it < nTri; ++it) {
      const int cp = tcp[it], vp = tvp[it], code = tat[it];
      const bool first = code >= 0;
      const int P = first ? code : -1 - code;   // the atom A (first kind) or F (second)
      const int nk = d.nao[P];
      const int K1 = nk * nX;
      // D(A,B) or D(F,B) [nk][nB] and H(B,A) or H(B,F) [b][beta][k] of tile t
      const bool with_d = d.keepD[(int64_t)P * N + B] != 0;
      const double* Dsrc = d.D + d.ao[P] * nt + d.ao[B];
      if (with_d)
        for (int e = tid; e < nk * nB; e += kNT) Ds[e] = Dsrc[(int64_t)(e / nB) * nt + e % nB];
      const double* Hsrc = d.H + d.hOff[d.hSlotMap[(int64_t)B * N + P]] + (int64_t)t * nB * 16 * nk;
      if constexpr (HS)
        for (int e = tid; e < nB * 16 * nk; e += kNT) Hs[e] = Hsrc[e];
      q_tile<NW>(d.Vf + d.vfOff[vp], ldv, d.Cf + d.cfOff[cp], d.nabf[first ? P : X], K1, t, Q, w, q, g);
      __syncthreads();
      // Q index of (x, k): k nX + x (first kind), x nF + k (second)
      contract_triple<NTB, NTX, NW>(Q, K1, Ds, HS ? Hs : Hsrc, with_d, nk, nB, nX, first ? 1 : nk, first ? nX : 1, hacc,
                          gacc, w, q, g);
      __syncthreads();
    }
    // the beta tile of Hbar(B,X), laid out as the H slot: [b][beta][x]
    double* hout = Hbar + d.hOff[s] + (int64_t)t * 16 * nB * nX;
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
      const int be = w + NW * j;
#pragma unroll
      for (int ib = 0; ib < NTB; ++ib)
#pragma unroll
        for (int ix = 0; ix < NTX; ++ix)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int b = 16 * ib + g + 4 * r, x = 16 * ix + q;
            if (b < nB && x < nX) hout[(b * 16 + be) * nX + x] = -hacc[j][ib][ix][r];
          }
    }
  }
  // the D block (X,B) of G1 + G2: the NW waves' partials (each over its beta
  // rows) added in wave order; this workgroup is the block's only writer
#pragma unroll
  for (int ix = 0; ix < NTX; ++ix)
#pragma unroll
    for (int ib = 0; ib < NTB; ++ib)
#pragma unroll
      for (int r = 0; r < 4; ++r) Q[((w * NTX + ix) * NTB + ib) * 256 + r * 64 + lane] = gacc[ix][ib][r];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int ix = 0; ix < NTX; ++ix)
#pragma unroll
      for (int ib = 0; ib < NTB; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = 0.0;
          for (int ww = 0; ww < NW; ++ww) v += Q[((ww * NTX + ix) * NTB + ib) * 256 + r * 64 + lane];
          const int x = 16 * ix + g + 4 * r, b = 16 * ib + q;
          if (x < nX && b < nB) G12[(d.ao[X] + x) * nt + d.ao[B] + b] = -v;
        }
  }
}

// G3(G,X)[g][x] = sum_B sum_{beta,b} Cf(B,G)[beta][b][g] Hbar(B,X)[b][beta][x]
// over the C pairs (B,G) with a value-list block and the needed slots (B,X),
// on the matrix cores: tiles (g, x) of 16 x 16, the contraction over
// (beta, b) in k-steps of four b, the loads of four k-steps issued before
// their products from clamped addresses (zero operands past nB); wave w
// takes beta = w, w + 4, ...; the four partial tiles are added in wave
// order.  NT: 16-wide tiles for g and
// x; the launch for NT takes the blocks with 16 (NT - 1) < max(nG, nX) <=
// 16 NT.  The launch covers the listed blocks (G,X) that a C partner B of
// G reaches through an H slot (B,X); each is written by one workgroup
// (zeros when nothing reaches it at this screening), the others stay at
// the zeros G3 is filled with.
template <int NT>
__global__ void __launch_bounds__(kHxNT) k_hx_g3(Dev d, const int* __restrict__ blocks, const double* __restrict__ Hbar,
                                                 double* __restrict__ G3) {
  __shared__ double red[4 * NT * NT * 256];
  const int N = d.N;
  const int o = blocks[blockIdx.x];
  const int G = o / N, X = o % N;
  const int64_t nt = d.ntot;
  const int nG = d.nao[G], nX = d.nao[X];
  const int ngx = max(nG, nX);
  if (ngx > 16 * NT || ngx <= 16 * (NT - 1)) return;   // the other launch's block
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  d4 acc[NT][NT];
#pragma unroll
  for (int ig = 0; ig < NT; ++ig)
#pragma unroll
    for (int ix = 0; ix < NT; ++ix) acc[ig][ix] = d4{0, 0, 0, 0};
  for (int i = d.cpRow[G]; i < d.cpRow[G + 1]; ++i) {
    const int B = d.cpF[i];
    const int sl = d.hSlotMap[(int64_t)B * N + X];
    if (sl < 0 || !d.need[sl]) continue;
    const int cp = find_partner(d.cpF, d.cpRow[B], d.cpRow[B + 1], G);
    if (cp < 0 || !(d.aliveC[cp] & 1)) continue;
    const int mB = d.nabf[B], nB = d.nao[B], nsb = (nB + 3) >> 2;
    const double* Cf = d.Cf + d.cfOff[cp];   // [beta][b][g]
    const double* Hb = Hbar + d.hOff[sl];    // [beta / 16][b][beta % 16][x]
    for (int be = w; be < mB; be += 4) {
      const double* cr = Cf + (int64_t)be * nB * nG;
      const double* hr = Hb + ((int64_t)(be >> 4) * nB * 16 + (be & 15)) * nX;
      for (int s0 = 0; s0 < nsb; s0 += 4) {
        double av[4][NT], hv[4][NT];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int b = 4 * (s0 + j) + g, bc = min(b, nB - 1);
          const bool ok = b < nB;
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            const int c = 16 * u + q;
            const double a1 = cr[bc * nG + min(c, nG - 1)], h1 = hr[bc * 16 * nX + min(c, nX - 1)];
            av[j][u] = (ok && c < nG) ? a1 : 0.0;
            hv[j][u] = (ok && c < nX) ? h1 : 0.0;
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int ig = 0; ig < NT; ++ig)
#pragma unroll
            for (int ix = 0; ix < NT; ++ix)
              acc[ig][ix] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j][ig], hv[j][ix], acc[ig][ix], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int ig = 0; ig < NT; ++ig)
#pragma unroll
    for (int ix = 0; ix < NT; ++ix)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[((w * NT + ig) * NT + ix) * 256 + r * 64 + lane] = acc[ig][ix][r];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int ig = 0; ig < NT; ++ig)
#pragma unroll
      for (int ix = 0; ix < NT; ++ix)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = 0.0;
          for (int ww = 0; ww < 4; ++ww) v += red[((ww * NT + ig) * NT + ix) * 256 + r * 64 + lane];
          const int gg = 16 * ig + g + 4 * r, x = 16 * ix + q;
          if (gg < nG && x < nX) G3[(d.ao[G] + gg) * nt + d.ao[X] + x] = v;
        }
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
  hipLaunchKernelGGL(k_fill_f64, dim3(2048), dim3(256), 0, s, b.G3, nt * nt);
  if (d.nSlot > 0) {
    const int nmax = b.nmax;
    // per launch (NTB, NTX): Q tile rows (or the G partials of the NW
    // waves), the D block and the H slice, sized for b < 16 NTB, x < 16 NTX
    // and k <= nmax; the H slice is staged when the workgroups that the
    // registers let a CU hold still fit its 160 KiB of LDS, and at most
    // 80 KiB per workgroup (a larger stage, at one workgroup per CU, was
    // slower than reading the slice from global memory)
    const unsigned grid = 8u * (unsigned)((d.nSlot + 7) / 8);   // see k_hx_slot's slot order
    auto run = [&](auto kern_h, auto kern_g, int NTB, int NTX, int NW) {
      const int bb = std::min(16 * NTB, nmax), bx = std::min(16 * NTX, nmax);
      const int qsize = std::max(16 * nmax * bx, NW * NTB * NTX * 256);
      const int dsize = nmax * bb;
      const size_t base = sizeof(double) * ((size_t)qsize + dsize);
      const size_t with_h = base + sizeof(double) * 16 * (size_t)bb * nmax;
      const size_t per_cu = std::max(1, 4 * slot_waves_per_simd(NTB, NTX) / NW);
      const bool hs = with_h <= std::min((size_t)81920, (size_t)163840 / per_cu);
      const size_t lds = hs ? with_h : base;
      const void* k = hs ? (const void*)kern_h : (const void*)kern_g;
      if (lds > 65536) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (hs)
        hipLaunchKernelGGL(kern_h, dim3(grid), dim3(64 * NW), lds, s, d, b.Hbar, b.G12, qsize, dsize);
      else
        hipLaunchKernelGGL(kern_g, dim3(grid), dim3(64 * NW), lds, s, d, b.Hbar, b.G12, qsize, dsize);
    };
    run(k_hx_slot<1, 1, true, 4>, k_hx_slot<1, 1, false, 4>, 1, 1, 4);
    if (nmax > 16) {
      run(k_hx_slot<1, 2, true, 4>, k_hx_slot<1, 2, false, 4>, 1, 2, 4);
      run(k_hx_slot<2, 1, true, 4>, k_hx_slot<2, 1, false, 4>, 2, 1, 4);
      run(k_hx_slot<2, 2, true, 8>, k_hx_slot<2, 2, false, 8>, 2, 2, 8);
    }
  }
  if (ev) (void)hipEventRecord(ev[0], s);
  if (b.n3[0] > 0)
    hipLaunchKernelGGL(k_hx_g3<1>, dim3((unsigned)b.n3[0]), dim3(kHxNT), 0, s, d, b.g3blk[0], (const double*)b.Hbar,
                       b.G3);
  if (b.n3[1] > 0)
    hipLaunchKernelGGL(k_hx_g3<2>, dim3((unsigned)b.n3[1]), dim3(kHxNT), 0, s, d, b.g3blk[1], (const double*)b.Hbar,
                       b.G3);
  if (ev) (void)hipEventRecord(ev[1], s);
  const int64_t nf = hx_tiles(nt);
  hipLaunchKernelGGL(k_hx_final, dim3((unsigned)nf), dim3(kHxNT), 0, s, d, (const double*)b.G12,
                     (const double*)b.G3, b.Hx, b.Etile);
  hipLaunchKernelGGL(k_hx_sum, dim3(1), dim3(1024), 0, s, (const double*)b.Etile, nf, b.E);
  if (ev) (void)hipEventRecord(ev[2], s);
}

}  // namespace lrx
