// Validation, block norms, two-step screening, image folding and H-slot marking.
//
// Screening follows Sec. "Sparsity exploitation" of the paper: step 1 drops a
// whole atom-pair block when its largest element is at most theta (Table
// thr_default uses one threshold per tensor; here one theta covers C, dC, V,
// dV and D), step 2 bounds what is left with the Cauchy-Schwarz inequality.
// The exact rules are stated in include/lrx.h.
#include "lrx_internal.h"

namespace lrx {

constexpr int kNT = 256;

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Deterministic block reductions: wave butterflies, then wave 0 sums the
// per-wave values in wave order.  `sh` holds at least blockDim/64 + 1 doubles.
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
__device__ inline double block_max(double v, double* sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0;
    for (int i = 0; i < nw; ++i) r = fmax(r, sh[i]);
    sh[nw] = r;
  }
  __syncthreads();
  return sh[nw];
}

// ---------------------------------------------------------------------------
// validation (run once per lrx_set_tensors)
// ---------------------------------------------------------------------------

__device__ inline bool close_rel(double x, double y) {
  return fabs(x - y) <= 1e-12 * (fabs(x) + fabs(y));
}

__global__ void k_val_finite(const double* p, int64_t n, int* err, int code) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(p[i])) atomicOr(err, code);
}

// V(B,A,-R) = V(A,B,R)^T and dV(B,A,-R) = -dV(A,B,R)^T: block b is [mA][mB],
// its mirror [mB][mA].  The mirror is read in 32 x 32 tiles through LDS so
// that both blocks are read along their rows.  Every pair is checked once,
// and as every V block is in a pair, this pass also checks that V and dV
// are finite.
__global__ void __launch_bounds__(kNT) k_val_vmirror(Dev d) {
  constexpr int kT = 32;
  __shared__ double tile[kT][kT + 1];
  const int64_t b = blockIdx.x;
  const int64_t m = d.Vmir[b];
  if (m < b) return;   // the pair (m, b) compares the same elements
  const int mA = d.nabf[d.Vfirst[b]], mB = d.nabf[d.Vsecond[b]];
  const int n = mA * mB;
  int bad = 0;
  for (int x = 0; x < 4; ++x) {   // the value, then the three derivatives
    const double* vb = x == 0 ? d.Vval + d.Voff[b] : d.Vdval + 3 * d.Voff[b] + (int64_t)(x - 1) * n;
    const double* vm = x == 0 ? d.Vval + d.Voff[m] : d.Vdval + 3 * d.Voff[m] + (int64_t)(x - 1) * n;
    const double sgn = x == 0 ? 1.0 : -1.0;
    for (int r0 = 0; r0 < mA; r0 += kT)
      for (int c0 = 0; c0 < mB; c0 += kT) {
        // mirror rows be in [c0, c0+kT), columns al in [r0, r0+kT)
        for (int e = threadIdx.x; e < kT * kT; e += kNT) {
          const int i = e / kT, j = e % kT;
          if (c0 + i < mB && r0 + j < mA) tile[i][j] = vm[(c0 + i) * mA + r0 + j];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kT * kT; e += kNT) {
          const int i = e / kT, j = e % kT;
          if (r0 + i < mA && c0 + j < mB) {
            const double u = vb[(r0 + i) * mB + c0 + j], v = tile[j][i];
            if (!isfinite(u) || !isfinite(v)) bad |= 16;
            if (!close_rel(u, sgn * v)) bad |= 1 << x;
          }
        }
        __syncthreads();
      }
  }
  if (bad & 1) atomicOr(d.err, kErrVMirror);
  if (bad & 14) atomicOr(d.err, kErrDVMirror);
  if (bad & 16) atomicOr(d.err, kErrNonfiniteV);
}

__global__ void k_val_onsite(Dev d) {
  const int64_t b = blockIdx.x;
  if (d.Cfirst[b] != d.Csecond[b] || d.CR[3 * b] || d.CR[3 * b + 1] || d.CR[3 * b + 2]) return;
  const int n = d.nao[d.Cfirst[b]], m = d.nabf[d.Cfirst[b]];
  const double* c = d.Cval + d.Coff[b];
  for (int e = threadIdx.x; e < m * n * n; e += blockDim.x) {
    const int al = e / (n * n), a = (e / n) % n, f = e % n;
    if (!close_rel(c[e], c[al * n * n + f * n + a])) atomicOr(d.err, kErrOnsiteC);
  }
}

// D = D^T (anti: D = -D^T), checked on the 32 x 32 tiles (tr, tc) with
// tr <= tc: tile (tc, tr) is read along its rows into LDS and compared
// transposed.  Workgroup w takes tiles w, w + gridDim.x, ... of the T x T
// tiles and skips those below the diagonal (the skip is uniform over the
// workgroup).
__global__ void __launch_bounds__(kNT) k_val_dsym(const double* D, int64_t nt, double sgn, int* err) {
  constexpr int kT = 32;
  __shared__ double tile[kT][kT + 1];
  const int64_t T = (nt + kT - 1) / kT;
  int bad = 0;
  for (int64_t w = blockIdx.x; w < T * T; w += gridDim.x) {
    const int64_t tr = w / T, tc = w - tr * T;
    if (tr > tc) continue;
    const int64_t r0 = tr * kT, c0 = tc * kT;
    for (int e = threadIdx.x; e < kT * kT; e += kNT) {
      const int i = e / kT, j = e % kT;
      if (c0 + i < nt && r0 + j < nt) tile[i][j] = D[(c0 + i) * nt + r0 + j];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kT * kT; e += kNT) {
      const int i = e / kT, j = e % kT;
      const int64_t r = r0 + i, c = c0 + j;
      if (c > r && c < nt && !close_rel(D[r * nt + c], sgn * tile[j][i])) bad = 1;
    }
    __syncthreads();
  }
  if (bad) atomicOr(err, kErrDSym);
}

void launch_validate_dsym(const double* D, int64_t nt, int anti, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_val_dsym, dim3(2048), dim3(kNT), 0, s, D, nt, anti ? -1.0 : 1.0, err);
}

void launch_validate(const Dev& d, hipStream_t s) {
  const int g = 2048;
  if (d.nV) hipLaunchKernelGGL(k_val_vmirror, dim3((unsigned)d.nV), dim3(kNT), 0, s, d);
  if (d.nC) hipLaunchKernelGGL(k_val_onsite, dim3((unsigned)d.nC), dim3(kNT), 0, s, d);
  hipLaunchKernelGGL(k_val_finite, dim3(g), dim3(kNT), 0, s, d.D, d.dsize, d.err, (int)kErrNonfiniteD);
}

// Finite checks of the block values (sizes known on the host).
void launch_validate_finite(const double* p, int64_t n, int* err, int code, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_val_finite, dim3(2048), dim3(kNT), 0, s, p, n, err, code);
}

// ---------------------------------------------------------------------------
// step 1: block norms (one workgroup per block)
// ---------------------------------------------------------------------------
// max |x| and sum x^2 of this thread's elements i = tid, tid + kNT, ... of
// p[0, n): eight loads in flight per thread, eight partial sums added in a
// fixed order
__device__ inline void block_max_sq(const double* __restrict__ p, int n, double& mx, double& ss) {
  constexpr int U = 8;
  double m[U], s[U];
#pragma unroll
  for (int u = 0; u < U; ++u) m[u] = s[u] = 0.0;
  int i = threadIdx.x;
  for (; i + (U - 1) * kNT < n; i += U * kNT) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = p[i + u * kNT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      m[u] = fmax(m[u], fabs(x[u]));
      s[u] += x[u] * x[u];
    }
  }
  for (; i < n; i += kNT) {
    const double x = p[i];
    m[0] = fmax(m[0], fabs(x));
    s[0] += x * x;
  }
#pragma unroll
  for (int u = 1; u < U; ++u) {
    m[0] = fmax(m[0], m[u]);
    s[0] += s[u];
  }
  mx = m[0];
  ss = s[0];
}

__global__ void __launch_bounds__(kNT) k_block_norms(const double* val, const double* dval, const int64_t* off,
                                                     const int* sz, double* out) {
  __shared__ double sh[kNT / 64 + 1];
  const int64_t b = blockIdx.x;
  const int64_t o = off[b];
  const int n = sz[b];
  double mv = 0, sv = 0, md = 0, sd = 0;
  const double* v = val + o;
  const double* dv = dval + 3 * o;
  block_max_sq(v, n, mv, sv);
  block_max_sq(dv, 3 * n, md, sd);
  mv = block_max(mv, sh);
  md = block_max(md, sh);
  sv = block_sum(sv, sh);
  sd = block_sum(sd, sh);
  if (threadIdx.x == 0) {
    out[4 * b + 0] = mv;
    out[4 * b + 1] = md;
    out[4 * b + 2] = sv;
    out[4 * b + 3] = sd;
  }
}

// D atom-pair blocks: one thread per (X, Y) with X <= Y.
__global__ void k_d_norms(Dev d) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)d.N * d.N) return;
  const int X = (int)(t / d.N), Y = (int)(t % d.N);
  if (Y < X) return;
  const int nX = d.nao[X], nY = d.nao[Y];
  const int64_t o = d_block(d, X, Y);
  const double* p = d.DnRe + o;
  const double* q = d.DnIm ? d.DnIm + o : nullptr;   // a complex D: the modulus
  double mx = 0, ss = 0;
  for (int i = 0; i < nX; ++i)
    for (int j = 0; j < nY; ++j) {
      const double v = p[i * d.dld + j], w = q ? q[i * d.dld + j] : 0.0;
      const double v2 = v * v + w * w;
      mx = fmax(mx, q ? sqrt(v2) : fabs(v));
      ss += v2;
    }
  d.dmax[t] = mx;
  d.dss[t] = ss;
}

// ---------------------------------------------------------------------------
// step 1 decisions for C blocks and D pairs; c(A,F) and d(X,Y) for step 2
// ---------------------------------------------------------------------------
__global__ void k_screen_c(Dev d, Opts o) {
  const int cp = blockIdx.x * blockDim.x + threadIdx.x;
  if (cp >= d.nCp) return;
  double c = 0;
  uint8_t alive = 0;
  for (int k = d.cpB0[cp]; k < d.cpB1[cp]; ++k) {
    const int64_t b = d.cpBlk[k];
    const double* nr = d.nrmC + 4 * b;
    int bits;
    if (o.per_tensor)
      bits = ((!(o.th[0] > 0) || nr[0] > o.th[0]) ? 1 : 0) | ((!(o.th[3] > 0) || nr[1] > o.th[3]) ? 2 : 0);
    else
      bits = (!(o.theta > 0) || nr[0] > o.theta || nr[1] > o.theta) ? 3 : 0;
    d.keepC[b] = (uint8_t)bits;
    if (bits) c += fmax((bits & 1) ? sqrt(nr[2]) : 0.0, (bits & 2) ? sqrt(nr[3]) : 0.0);
    alive |= (uint8_t)bits;
  }
  d.cval[cp] = c;
  d.aliveC[cp] = alive;   // bit 1: Cf(A,F) != 0 may hold; bit 2: Y(A,F) is read
}

__global__ void k_screen_d(Dev d, Opts o) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)d.N * d.N) return;
  const int X = (int)(t / d.N), Y = (int)(t % d.N);
  const int64_t c = X <= Y ? t : (int64_t)Y * d.N + X;
  const double tD = o.per_tensor ? o.th[2] : o.theta;
  const bool keep = !(tD > 0) || d.dmax[c] > tD;
  d.keepD[t] = keep;
  d.dnrm[t] = keep ? sqrt(d.dss[c]) : 0.0;
}

// ---------------------------------------------------------------------------
// step 2: S(A,B) per V pair (evaluated by the pair that forms Z, and mirrored)
// ---------------------------------------------------------------------------
__global__ void k_screen_s(Dev d) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.nVp) return;
  if (!d.vpZ[p]) return;   // S(A,B) = S(B,A): written by the pair that forms Z
  const int A = d.vpA[p], B = d.vpB[p];
  const int N = d.N;
  const double dAB = d.dnrm[(int64_t)A * N + B];
  double s = 0;
  for (int i = d.cpRow[A]; i < d.cpRow[A + 1]; ++i) {
    const double cAF = d.cval[i];
    if (cAF == 0) continue;
    const int F = d.cpF[i];
    const double dFB = d.dnrm[(int64_t)F * N + B];
    for (int j = d.cpRow[B]; j < d.cpRow[B + 1]; ++j) {
      const double cBG = d.cval[j];
      if (cBG == 0) continue;
      const int G = d.cpF[j];
      s += cAF * cBG * (dAB * d.dnrm[(int64_t)F * N + G] + d.dnrm[(int64_t)A * N + G] * dFB);
    }
  }
  d.Svp[p] = s;
  d.Svp[d.vpMir[p]] = s;
}

// V blocks: step 1 with the mirror, then step 2; pair liveness.
__global__ void k_screen_v(Dev d, Opts o) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.nVp) return;
  uint8_t alive = 0;
  const double S = d.Svp[p];
  for (int k = d.vpB0[p]; k < d.vpB1[p]; ++k) {
    const int64_t b = d.vpBlk[k];
    const int64_t m = d.Vmir[b];
    const double* n1 = d.nrmV + 4 * b;
    const double* n2 = d.nrmV + 4 * m;
    const double mv = fmax(n1[0], n2[0]), md = fmax(n1[1], n2[1]);
    int bits;
    if (o.per_tensor)
      bits = ((!(o.th[1] > 0) || mv > o.th[1]) ? 1 : 0) | ((!(o.th[4] > 0) || md > o.th[4]) ? 2 : 0);
    else
      bits = (!(o.theta > 0) || fmax(mv, md) > o.theta) ? 3 : 0;
    const double nv = fmax((bits & 1) ? fmax(sqrt(n1[2]), sqrt(n2[2])) : 0.0,
                           (bits & 2) ? fmax(sqrt(n1[3]), sqrt(n2[3])) : 0.0);
    if (bits && o.theta_cs > 0 && !(nv * S > o.theta_cs)) bits = 0;
    d.keepV[b] = (uint8_t)bits;
    alive |= (uint8_t)bits;
  }
  d.aliveV[p] = alive;    // bit 1: Vf(A,B) != 0 may hold; bit 2: some dV is kept
}

// ---------------------------------------------------------------------------
// image folding: Cf(A,F) = sum of kept C images, Vf(A,B) = sum of kept V images
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT) k_fold_c(Dev d, int prec) {
  const int cp = blockIdx.x;
  if (!d.aliveC[cp]) return;
  const int n = d.nabf[d.cpA[cp]] * d.nao[d.cpA[cp]] * d.nao[d.cpF[cp]];
  double* out = d.Cf + d.cfOff[cp];
  float* out32 = prec != kP64 ? d.Cf32 + d.cfOff[cp] : nullptr;
  const int k0 = d.cpB0[cp], k1 = d.cpB1[cp];
  for (int e = threadIdx.x; e < n; e += kNT) {
    double s = 0;
    for (int k = k0; k < k1; ++k) {
      const int64_t b = d.cpBlk[k];
      if (d.keepC[b] & 1) s += d.Cval[d.Coff[b] + e];
    }
    out[e] = s;
    if (out32) out32[e] = (float)s;
  }
}

__global__ void __launch_bounds__(kNT) k_fold_v(Dev d, int prec) {
  const int p = blockIdx.x;
  if (!d.aliveV[p]) return;
  // folded block [mA][mBp]: rows padded with zeros to 16 elements
  const int mA = d.nabf[d.vpA[p]], mB = d.nabf[d.vpB[p]], mBp = (mB + 15) & ~15;
  double* out = d.Vf + d.vfOff[p];
  float* out32 = prec != kP64 ? d.Vf32 + d.vfOff[p] : nullptr;
  const int k0 = d.vpB0[p], k1 = d.vpB1[p];
  // the kept image blocks, in order (uniform; a pair has few images)
  constexpr int kImg = 4;
  const double* src[kImg];
  int ns = 0, k = k0;
  for (; k < k1 && ns < kImg; ++k) {
    const int64_t b = d.vpBlk[k];
    if (d.keepV[b] & 1) src[ns++] = d.Vval + d.Voff[b];
  }
  // e / mBp exactly for e < 2^16 (mA, mBp <= 128): ceil(2^32 / mBp) times e, high word
  const unsigned mdiv = 0xFFFFFFFFu / (unsigned)mBp + 1u;
  for (int e = threadIdx.x; e < mA * mBp; e += kNT) {
    const int al = (int)__umulhi((unsigned)e, mdiv), be = e - al * mBp;
    double s = 0;
    if (be < mB) {
      const int o = al * mB + be;
#pragma unroll
      for (int j = 0; j < kImg; ++j)
        if (j < ns) s += src[j][o];
      for (int kk = k; kk < k1; ++kk) {   // images past the first kImg kept ones
        const int64_t b = d.vpBlk[kk];
        if (d.keepV[b] & 1) s += d.Vval[d.Voff[b] + o];
      }
    }
    out[e] = s;
    if (out32) out32[e] = (float)s;
  }
}

__global__ void k_to_f32(const double* in, float* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// H slots needed by the live triples (A,F,B): H(B,F) and H(B,A)
// ---------------------------------------------------------------------------
__global__ void k_fill_u8(uint8_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_mark(Dev d) {
  const int cp = blockIdx.x * blockDim.x + threadIdx.x;
  if (cp >= d.nCp) return;
  const int ac = d.aliveC[cp];
  if (!ac) return;
  const int A = d.cpA[cp], F = d.cpF[cp];
  for (int p = d.vpRow[A]; p < d.vpRow[A + 1]; ++p) {
    const int B = d.vpB[p];
    if (!triple_live(ac, d.aliveV[p], !d.vpZ[p])) continue;
    d.need[d.hSlotMap[(int64_t)B * d.N + F]] = 1;
    d.need[d.hSlotMap[(int64_t)B * d.N + A]] = 1;
  }
}

// H slots the Hamiltonian reads: H(B,F) and H(B,A) of every triple (A,F,B)
// whose C pair and V pair have value-list blocks (its energy item).
__global__ void k_mark_hx(Dev d) {
  const int cp = blockIdx.x * blockDim.x + threadIdx.x;
  if (cp >= d.nCp || !(d.aliveC[cp] & 1)) return;
  const int A = d.cpA[cp], F = d.cpF[cp];
  for (int p = d.vpRow[A]; p < d.vpRow[A + 1]; ++p) {
    if (!(d.aliveV[p] & 1)) continue;
    const int B = d.vpB[p];
    d.need[d.hSlotMap[(int64_t)B * d.N + F]] = 1;
    d.need[d.hSlotMap[(int64_t)B * d.N + A]] = 1;
  }
}

// What each triple-product unit forms in this evaluation (triple_live):
// 0 nothing, 1 Z and Y, 2 Y alone.
__global__ void k_unit_role(Dev d) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= d.nUnit) return;
  const int ac = d.aliveC[d.unitCp[u]];
  const bool yonly = unit_y_only(ac, d.unitYonly[u] != 0);
  d.unitRole[u] = (!ac || (yonly && !(ac & 2))) ? 0 : (yonly ? 2 : 1);
}

// Compaction of the H-build tables of atom B (one workgroup per atom):
// depth entries of C pairs (B,G) with a block in the value list (the others
// fold to Cf(B,G) = 0), in table order, padded with entries
// of no atom to a multiple of 4 (at least 4, so a slot whose C pairs are all
// screened is still written, as zeros); columns of the needed slots (B,X),
// in table order.  Ordered prefix sums over the ballots of each 64-lane
// wave: the result does not depend on scheduling.
__device__ inline int block_exclusive_scan(bool flag, int* sh, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const unsigned long long m = __ballot(flag);
  const int within = __popcll(m & ((1ull << lane) - 1ull));
  __syncthreads();
  if (lane == 0) sh[w] = __popcll(m);
  __syncthreads();
  int before = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    before += i < w ? sh[i] : 0;
    all += sh[i];
  }
  *total = all;
  return before + within;
}

__global__ void __launch_bounds__(kNT) k_hcompact(Dev d) {
  __shared__ int sh[kNT / 64];
  const int B = blockIdx.x;
  {
    const int h0 = d.hdRow[B], hn = d.hdRow[B + 1] - h0;
    int n = 0;
    for (int k0 = 0; k0 < hn; k0 += kNT) {
      const int k = k0 + threadIdx.x;
      const int t = k < hn ? d.hdCp[h0 + k] : -1;
      const bool live = t >= 0 && (d.aliveC[t >> 6] & 1);   // Cf(B,G) in the value list
      int tot;
      const int pos = h0 + n + block_exclusive_scan(live, sh, &tot);
      if (live) {
        d.hcRowD[pos] = d.hdRowD[h0 + k];
        d.hcG[pos] = d.hdG[h0 + k];
        d.hcCp[pos] = t;
        d.hcCf[pos] = d.hdCf[h0 + k];
        d.hcStride[pos] = d.hdStride[h0 + k];
      }
      n += tot;
    }
    const int K = max(4, (n + 3) & ~3);   // <= hn: every atom has its on-site pair
    for (int k = n + threadIdx.x; k < K; k += kNT) {
      d.hcRowD[h0 + k] = 0;
      d.hcG[h0 + k] = -1;
      d.hcCp[h0 + k] = -1;
      d.hcCf[h0 + k] = 0;
      d.hcStride[h0 + k] = 0;
    }
    if (threadIdx.x == 0) d.hcK[B] = K;
  }
  {
    const int c0 = d.hColRow[B], cn = d.hColRow[B + 1] - c0;
    int n = 0;
    for (int k0 = 0; k0 < cn; k0 += kNT) {
      const int k = k0 + threadIdx.x;
      const int sl = k < cn ? d.hColSlot[c0 + k] : -1;
      const bool live = sl >= 0 && d.need[sl];
      int tot;
      const int pos = c0 + n + block_exclusive_scan(live, sh, &tot);
      if (live) {
        d.hcColSlot[pos] = sl;
        d.hcColD[pos] = d.hColD[c0 + k];
        d.hcColAtom[pos] = d.hColAtom[c0 + k];
      }
      n += tot;
    }
    if (threadIdx.x == 0) d.hcNcol[B] = n;
  }
}

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)(a > 0 ? (a + b - 1) / b : 1); }

void launch_d_to_f32(const Dev& d, int prec, hipStream_t s) {
  if (prec != kP64) hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(kNT), 0, s, d.D, d.D32, d.dsize);
}

void launch_screen(const Dev& d, const Opts& o, hipStream_t s, hipEvent_t* ev, bool for_hx) {
  const int64_t NN = (int64_t)d.N * d.N;
  if (d.nC) hipLaunchKernelGGL(k_block_norms, dim3((unsigned)d.nC), dim3(kNT), 0, s, d.Cval, d.Cdval, d.Coff, d.Csz, d.nrmC);
  if (d.nV) hipLaunchKernelGGL(k_block_norms, dim3((unsigned)d.nV), dim3(kNT), 0, s, d.Vval, d.Vdval, d.Voff, d.Vsz, d.nrmV);
  hipLaunchKernelGGL(k_d_norms, dim3(cdiv(NN, kNT)), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(k_screen_c, dim3(cdiv(d.nCp, kNT)), dim3(kNT), 0, s, d, o);
  hipLaunchKernelGGL(k_screen_d, dim3(cdiv(NN, kNT)), dim3(kNT), 0, s, d, o);
  hipLaunchKernelGGL(k_screen_s, dim3(cdiv(d.nVp, kNT)), dim3(kNT), 0, s, d);
  hipLaunchKernelGGL(k_screen_v, dim3(cdiv(d.nVp, kNT)), dim3(kNT), 0, s, d, o);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (d.nCp) hipLaunchKernelGGL(k_fold_c, dim3(d.nCp), dim3(kNT), 0, s, d, o.prec);
  if (d.nVp) hipLaunchKernelGGL(k_fold_v, dim3(d.nVp), dim3(kNT), 0, s, d, o.prec);
  if (o.prec != kP64) hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(kNT), 0, s, d.D, d.D32, d.dsize);
  if (ev) (void)hipEventRecord(ev[2], s);
  hipLaunchKernelGGL(k_fill_u8, dim3(cdiv(d.nSlot, kNT)), dim3(kNT), 0, s, d.need,
                     (int64_t)d.nSlot);
  if (for_hx) {
    hipLaunchKernelGGL(k_mark_hx, dim3(cdiv(d.nCp, kNT)), dim3(kNT), 0, s, d);
  } else {
    hipLaunchKernelGGL(k_mark, dim3(cdiv(d.nCp, kNT)), dim3(kNT), 0, s, d);
    hipLaunchKernelGGL(k_unit_role, dim3(cdiv(d.nUnit, kNT)), dim3(kNT), 0, s, d);
  }
  hipLaunchKernelGGL(k_hcompact, dim3((unsigned)d.N), dim3(kNT), 0, s, d);
  if (ev) (void)hipEventRecord(ev[3], s);
}

}  // namespace lrx
