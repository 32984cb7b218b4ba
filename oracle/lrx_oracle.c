/*
 * CPU oracle for the LRI exact-exchange energy, forces and stress.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library, and it is deliberately plain:
 * FP64 throughout, the quartet loop of the paper in the paper's order, no
 * folding over lattice images, no symmetry tricks, no BLAS.
 *
 * What it computes (Gamma point, real tensors, one simulation cell):
 *
 *   E = - sum_{V blocks (A,B,R_B)} sum_{C blocks (A,F,R_F)} sum_{C blocks (B,G,R')}
 *         sum C1[al][a][f] V[al][be] C2[be][b][g]
 *             ( D(A,B)[a][b] D(F,G)[f][g] + D(A,G)[a][g] D(F,B)[f][b] )
 *
 *   This is the ABF-centred form of the LRI exchange energy (Methods, Eq.
 *   exx_expand, from Eqs. Exx-LRI and ABFG_perspective), with the atom A of
 *   the V block in the home cell, every partner an explicit lattice image, the
 *   Gamma-point density matrix the same for every image pair (N_k = 1), and
 *   Re[] dropped because every tensor is real.  Blocks removed by screening
 *   simply do not take part (Sec. Sparsity exploitation).
 *
 *   Every block is a function of its own displacement r = tau_second + R.L -
 *   tau_first, and the caller supplies d(block)/dr.  The force F^{X1} is the
 *   six-term derivative of Eq. Fexx1 with D held fixed (the D-variation part
 *   F^{X2} of Eq. Exx2 is not part of this quantity); here each quartet's
 *   three derivative slots (the C of A, the V, the C of B; Eq.
 *   Exx_energy_variation) are accumulated into a per-block gradient
 *   g_b = dE/dr_b, from which F_first += g, F_second -= g.
 *   The stress follows Eq. stress: sigma = -(1/Omega) sum_b g_b (x) r_b.
 *
 * Screening (Sec. Sparsity exploitation; thresholds as in Table thr_default
 * and Sec. on the Cauchy-Schwarz screening), in the reading used by this
 * project:
 *   S1 (theta > 0): keep a C block iff max|C| > theta or max|dC| > theta;
 *       keep a V block iff the max over the block and its mirror
 *       (B,A,-R) of max|V|, max|dV| exceeds theta; keep the D pair (X,Y) iff
 *       max|D_XY| > theta, taken on the block with X <= Y.
 *   S2 (theta_cs > 0): keep a surviving V block iff
 *       nv * S(A,B) > theta_cs, nv = max of the Frobenius norms of V, dV of
 *       the block and its mirror, and
 *       S(A,B) = sum_F sum_G c(A,F) c(B,G) [d(A,B) d(F,G) + d(A,G) d(F,B)],
 *       c(A,F) = sum over kept C blocks (A,F,R) of max(|C|_F, |dC|_F),
 *       d(X,Y) = |D_XY|_F of a kept D pair (block with X <= Y), else 0.
 *       S is evaluated for A <= B and mirrored.  This is the Cauchy-Schwarz
 *       bound of Sec. Sparsity exploitation summed over the items of one V
 *       pair.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t natom;
  const double* tau;     /* [natom][3] */
  const double* lat;     /* [3][3], rows are lattice vectors */
  const int32_t* nao;    /* [natom] */
  const int32_t* nabf;   /* [natom] */
  int64_t nC;
  const int32_t* C_first; const int32_t* C_second; const int32_t* C_R; const int64_t* C_off;
  const double* C_val; const double* C_dval;
  int64_t nV;
  const int32_t* V_first; const int32_t* V_second; const int32_t* V_R; const int64_t* V_off;
  const double* V_val; const double* V_dval;
  const double* D;       /* dense [n_tot][n_tot] */
} orc_input;

/* ------------------------------------------------------------------------ */
static int64_t ntot_of(const orc_input* in, int64_t* ao_off) {
  int64_t s = 0;
  for (int i = 0; i < in->natom; ++i) { ao_off[i] = s; s += in->nao[i]; }
  ao_off[in->natom] = s;
  return s;
}

static int64_t c_size(const orc_input* in, int64_t b) {
  return (int64_t)in->nabf[in->C_first[b]] * in->nao[in->C_first[b]] * in->nao[in->C_second[b]];
}
static int64_t v_size(const orc_input* in, int64_t b) {
  return (int64_t)in->nabf[in->V_first[b]] * in->nabf[in->V_second[b]];
}

static void block_norms(const double* val, const double* dval, int64_t n, double out[4]) {
  double mv = 0, md = 0, sv = 0, sd = 0;
  for (int64_t i = 0; i < n; ++i) { double x = fabs(val[i]); if (x > mv) mv = x; sv += val[i] * val[i]; }
  for (int64_t i = 0; i < 3 * n; ++i) { double x = fabs(dval[i]); if (x > md) md = x; sd += dval[i] * dval[i]; }
  out[0] = mv; out[1] = md; out[2] = sqrt(sv); out[3] = sqrt(sd);
}

/* V block keys sorted for the mirror lookup (second, first, -R) */
static const orc_input* g_sort_in;
static int key_cmp(const int32_t* a, const int32_t* b) {
  for (int i = 0; i < 5; ++i) if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}
static void v_key(const orc_input* in, int64_t b, int32_t k[5]) {
  k[0] = in->V_first[b]; k[1] = in->V_second[b];
  k[2] = in->V_R[3 * b]; k[3] = in->V_R[3 * b + 1]; k[4] = in->V_R[3 * b + 2];
}
static int idx_cmp(const void* pa, const void* pb) {
  int32_t ka[5], kb[5];
  v_key(g_sort_in, *(const int64_t*)pa, ka);
  v_key(g_sort_in, *(const int64_t*)pb, kb);
  return key_cmp(ka, kb);
}
static int64_t* v_mirrors(const orc_input* in) {
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (in->nV + 1));
  int64_t* mir = (int64_t*)malloc(sizeof(int64_t) * (in->nV + 1));
  for (int64_t b = 0; b < in->nV; ++b) idx[b] = b;
  g_sort_in = in;
  qsort(idx, (size_t)in->nV, sizeof(int64_t), idx_cmp);
  for (int64_t b = 0; b < in->nV; ++b) {
    int32_t want[5] = {in->V_second[b], in->V_first[b], -in->V_R[3 * b], -in->V_R[3 * b + 1], -in->V_R[3 * b + 2]};
    int64_t lo = 0, hi = in->nV - 1, found = -1;
    while (lo <= hi) {
      int64_t mid = (lo + hi) / 2;
      int32_t k[5];
      v_key(in, idx[mid], k);
      int c = key_cmp(k, want);
      if (c == 0) { found = idx[mid]; break; }
      if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    mir[b] = found;
  }
  free(idx);
  return mir;
}

/* S(A,B) = sum_F sum_G c(A,F) c(B,G) [d(A,B) d(F,G) + d(A,G) d(F,B)] for A <= B,
 * with F (and G) running over the partners of nonzero c in ascending order. */
static double s_pair(int N, const double* c, const double* d, const int* prow, const int* plist, int A, int B) {
  double s = 0;
  for (int i = prow[A]; i < prow[A + 1]; ++i) {
    const int F = plist[i];
    const double cAF = c[(int64_t)A * N + F];
    for (int j = prow[B]; j < prow[B + 1]; ++j) {
      const int G = plist[j];
      const double cBG = c[(int64_t)B * N + G];
      s += cAF * cBG * (d[(int64_t)A * N + B] * d[(int64_t)F * N + G] + d[(int64_t)A * N + G] * d[(int64_t)F * N + B]);
    }
  }
  return s;
}

/*
 * Screening decisions (S1 then S2).  keepC[nC], keepV[nV], keepD[natom*natom];
 * S_out (optional) [natom*natom] receives S(A,B) for the atom pairs of V blocks.
 * Returns 0, or -1 if a V block has no mirror.
 */
int orc_screen(const orc_input* in, double theta, double theta_cs,
               uint8_t* keepC, uint8_t* keepV, uint8_t* keepD, double* S_out) {
  const int N = in->natom;
  int64_t* ao = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  const int64_t nt = ntot_of(in, ao);
  double* d = (double*)calloc((size_t)N * N, sizeof(double));
  double* c = (double*)calloc((size_t)N * N, sizeof(double));
  double* S = (double*)calloc((size_t)N * N, sizeof(double));
  uint8_t* have = (uint8_t*)calloc((size_t)N * N, 1);
  /* D pairs, decided on the block with X <= Y and mirrored */
  for (int X = 0; X < N; ++X)
    for (int Y = X; Y < N; ++Y) {
      double mx = 0, ss = 0;
      for (int i = 0; i < in->nao[X]; ++i)
        for (int j = 0; j < in->nao[Y]; ++j) {
          double v = in->D[(ao[X] + i) * nt + ao[Y] + j];
          if (fabs(v) > mx) mx = fabs(v);
          ss += v * v;
        }
      int keep = !(theta > 0) || mx > theta;
      keepD[(int64_t)X * N + Y] = keepD[(int64_t)Y * N + X] = (uint8_t)keep;
      d[(int64_t)X * N + Y] = d[(int64_t)Y * N + X] = keep ? sqrt(ss) : 0.0;
    }
  /* C blocks, and c(A,F) summed over kept images in key order */
  for (int64_t b = 0; b < in->nC; ++b) {
    double nr[4];
    int64_t n = c_size(in, b);
    block_norms(in->C_val + in->C_off[b], in->C_dval + 3 * in->C_off[b], n, nr);
    int keep = !(theta > 0) || nr[0] > theta || nr[1] > theta;
    keepC[b] = (uint8_t)keep;
    if (keep) c[(int64_t)in->C_first[b] * N + in->C_second[b]] += (nr[2] > nr[3] ? nr[2] : nr[3]);
  }
  /* partners F of A with nonzero c(A,F), ascending */
  int* prow = (int*)calloc(N + 1, sizeof(int));
  for (int A = 0; A < N; ++A)
    for (int F = 0; F < N; ++F) if (c[(int64_t)A * N + F] != 0) prow[A + 1]++;
  for (int A = 0; A < N; ++A) prow[A + 1] += prow[A];
  int* plist = (int*)malloc(sizeof(int) * (prow[N] + 1));
  for (int A = 0, k = 0; A < N; ++A)
    for (int F = 0; F < N; ++F) if (c[(int64_t)A * N + F] != 0) plist[k++] = F;
  int64_t* mir = v_mirrors(in);
  int rc = 0;
  for (int64_t b = 0; b < in->nV; ++b) {
    int64_t m = mir[b];
    if (m < 0) { rc = -1; keepV[b] = 0; continue; }
    double n1[4], n2[4];
    int64_t n = v_size(in, b);
    block_norms(in->V_val + in->V_off[b], in->V_dval + 3 * in->V_off[b], n, n1);
    block_norms(in->V_val + in->V_off[m], in->V_dval + 3 * in->V_off[m], n, n2);
    double mx = fmax(fmax(n1[0], n1[1]), fmax(n2[0], n2[1]));
    double nv = fmax(fmax(n1[2], n1[3]), fmax(n2[2], n2[3]));
    const int A = in->V_first[b], B = in->V_second[b];
    const int lo = A < B ? A : B, hi = A < B ? B : A;
    if (!have[(int64_t)lo * N + hi]) {
      double s = s_pair(N, c, d, prow, plist, lo, hi);
      S[(int64_t)lo * N + hi] = S[(int64_t)hi * N + lo] = s;
      have[(int64_t)lo * N + hi] = 1;
    }
    int keep = !(theta > 0) || mx > theta;
    if (keep && theta_cs > 0) keep = nv * S[(int64_t)A * N + B] > theta_cs;
    keepV[b] = (uint8_t)keep;
  }
  if (S_out) memcpy(S_out, S, sizeof(double) * N * N);
  free(ao); free(d); free(c); free(S); free(have); free(prow); free(plist); free(mir);
  return rc;
}

/*
 * Screening with one threshold per tensor (Table thr_default: C, V, D, dC,
 * dV), thr = {theta_C, theta_V, theta_D, theta_dC, theta_dV}; a threshold
 * <= 0 keeps that whole tensor.  keepC / keepV get bit masks: bit 0 when the
 * block's value passes its threshold (max|C| > theta_C; for V the larger of
 * max|V| over the block and its mirror > theta_V), bit 1 when its derivative
 * passes (max|dC| > theta_dC; max|dV| over the block and its mirror >
 * theta_dV); keepD 0/1 (max|D_XY| > theta_D on the block with X <= Y).
 * Step 2 (theta_cs > 0) then drops a V block (both bits) iff
 * nv * S(A,B) <= theta_cs, with c(A,F) summing, over the images with any
 * bit, the larger Frobenius norm of the kept parts, and nv the larger
 * Frobenius norm of the kept parts of the block and its mirror.
 * Returns 0, or -1 if a V block has no mirror.
 */
int orc_screen5(const orc_input* in, const double* thr, double theta_cs,
                uint8_t* keepC, uint8_t* keepV, uint8_t* keepD, double* S_out) {
  const int N = in->natom;
  const double tC = thr[0], tV = thr[1], tD = thr[2], tdC = thr[3], tdV = thr[4];
  int64_t* ao = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  const int64_t nt = ntot_of(in, ao);
  double* d = (double*)calloc((size_t)N * N, sizeof(double));
  double* c = (double*)calloc((size_t)N * N, sizeof(double));
  double* S = (double*)calloc((size_t)N * N, sizeof(double));
  uint8_t* have = (uint8_t*)calloc((size_t)N * N, 1);
  for (int X = 0; X < N; ++X)
    for (int Y = X; Y < N; ++Y) {
      double mx = 0, ss = 0;
      for (int i = 0; i < in->nao[X]; ++i)
        for (int j = 0; j < in->nao[Y]; ++j) {
          double v = in->D[(ao[X] + i) * nt + ao[Y] + j];
          if (fabs(v) > mx) mx = fabs(v);
          ss += v * v;
        }
      int keep = !(tD > 0) || mx > tD;
      keepD[(int64_t)X * N + Y] = keepD[(int64_t)Y * N + X] = (uint8_t)keep;
      d[(int64_t)X * N + Y] = d[(int64_t)Y * N + X] = keep ? sqrt(ss) : 0.0;
    }
  for (int64_t b = 0; b < in->nC; ++b) {
    double nr[4];
    block_norms(in->C_val + in->C_off[b], in->C_dval + 3 * in->C_off[b], c_size(in, b), nr);
    const int bits = ((!(tC > 0) || nr[0] > tC) ? 1 : 0) | ((!(tdC > 0) || nr[1] > tdC) ? 2 : 0);
    keepC[b] = (uint8_t)bits;
    const double a = (bits & 1) ? nr[2] : 0.0, da = (bits & 2) ? nr[3] : 0.0;
    if (bits) c[(int64_t)in->C_first[b] * N + in->C_second[b]] += (a > da ? a : da);
  }
  int* prow = (int*)calloc(N + 1, sizeof(int));
  for (int A = 0; A < N; ++A)
    for (int F = 0; F < N; ++F) if (c[(int64_t)A * N + F] != 0) prow[A + 1]++;
  for (int A = 0; A < N; ++A) prow[A + 1] += prow[A];
  int* plist = (int*)malloc(sizeof(int) * (prow[N] + 1));
  for (int A = 0, k = 0; A < N; ++A)
    for (int F = 0; F < N; ++F) if (c[(int64_t)A * N + F] != 0) plist[k++] = F;
  int64_t* mir = v_mirrors(in);
  int rc = 0;
  for (int64_t b = 0; b < in->nV; ++b) {
    int64_t m = mir[b];
    if (m < 0) { rc = -1; keepV[b] = 0; continue; }
    double n1[4], n2[4];
    int64_t n = v_size(in, b);
    block_norms(in->V_val + in->V_off[b], in->V_dval + 3 * in->V_off[b], n, n1);
    block_norms(in->V_val + in->V_off[m], in->V_dval + 3 * in->V_off[m], n, n2);
    const int bits = ((!(tV > 0) || fmax(n1[0], n2[0]) > tV) ? 1 : 0) |
                     ((!(tdV > 0) || fmax(n1[1], n2[1]) > tdV) ? 2 : 0);
    const double nv = fmax((bits & 1) ? fmax(n1[2], n2[2]) : 0.0, (bits & 2) ? fmax(n1[3], n2[3]) : 0.0);
    const int A = in->V_first[b], B = in->V_second[b];
    const int lo = A < B ? A : B, hi = A < B ? B : A;
    if (!have[(int64_t)lo * N + hi]) {
      double s = s_pair(N, c, d, prow, plist, lo, hi);
      S[(int64_t)lo * N + hi] = S[(int64_t)hi * N + lo] = s;
      have[(int64_t)lo * N + hi] = 1;
    }
    int keep = bits;
    if (keep && theta_cs > 0 && !(nv * S[(int64_t)A * N + B] > theta_cs)) keep = 0;
    keepV[b] = (uint8_t)keep;
  }
  if (S_out) memcpy(S_out, S, sizeof(double) * N * N);
  free(ao); free(d); free(c); free(S); free(have); free(prow); free(plist); free(mir);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* D block (X,Y) as a pointer into the dense matrix (row stride nt), or NULL */
typedef struct { const double* p; int64_t ld; } dblk;

static inline double dget(dblk m, int i, int j) { return m.p ? m.p[i * m.ld + j] : 0.0; }

/*
 * One quartet (C1 = C(A,F,R_F), V = V(A,B,R_B), C2 = C(B,G,R')): the item
 *   sum C1[al][a][f] V[al][be] C2[be][b][g] K[a][f][b][g],
 *   K = D(A,B)[a][b] D(F,G)[f][g] + D(A,G)[a][g] D(F,B)[f][b],
 * and its derivative with respect to each of the three blocks, contracted
 * with that block's d/dr.  E -= item; g -= d(item)/dr per slot.
 */
typedef struct { double* w; } scratch;

static void quartet(int mA, int mB, int nA, int nF, int nB, int nG,
                    const double* C1, const double* dC1, const double* V, const double* dV,
                    const double* C2, const double* dC2,
                    dblk DAB, dblk DFG, dblk DAG, dblk DFB, double* ws, int want,
                    double* E, double g1[3], double gv[3], double g2[3]) {
  /* workspace: What[mB][nA][nF], Wtil[mA][nB][nG], T[nB][nF], U[nG][nF], P[nA][nG], Q[nF][nG] */
  double* What = ws;
  double* Wtil = What + (size_t)mB * nA * nF;
  double* T = Wtil + (size_t)mA * nB * nG;
  double* U = T + nB * nF;
  double* P = U + nG * nF;
  double* Q = P + nA * nG;

  /* What[be][a][f] = sum_{b,g} C2[be][b][g] K[a][f][b][g]
   *               = (D(A,B) C2_be D(F,G)^T)[a][f] + (D(A,G) C2_be^T D(F,B)^T)[a][f] */
  for (int be = 0; be < mB; ++be) {
    const double* c2 = C2 + (size_t)be * nB * nG;
    for (int b = 0; b < nB; ++b)
      for (int f = 0; f < nF; ++f) {
        double s = 0;
        for (int g = 0; g < nG; ++g) s += c2[b * nG + g] * dget(DFG, f, g);
        T[b * nF + f] = s;
      }
    for (int g = 0; g < nG; ++g)
      for (int f = 0; f < nF; ++f) {
        double s = 0;
        for (int b = 0; b < nB; ++b) s += c2[b * nG + g] * dget(DFB, f, b);
        U[g * nF + f] = s;
      }
    double* w = What + (size_t)be * nA * nF;
    for (int a = 0; a < nA; ++a)
      for (int f = 0; f < nF; ++f) {
        double s = 0;
        for (int b = 0; b < nB; ++b) s += dget(DAB, a, b) * T[b * nF + f];
        for (int g = 0; g < nG; ++g) s += dget(DAG, a, g) * U[g * nF + f];
        w[a * nF + f] = s;
      }
  }
  /* S[al][be] = sum_{a,f} C1[al][a][f] What[be][a][f]:  item = <V,S>, V slot = <dV,S>
   * R1[al][af] = sum_be V[al][be] What[be][af]:          C1 slot = <dC1,R1>        */
  const int k1 = nA * nF;
  double item = 0, sv[3] = {0, 0, 0}, s1[3] = {0, 0, 0};
  for (int al = 0; al < mA; ++al)
    for (int be = 0; be < mB; ++be) {
      double s = 0;
      const double* c1 = C1 + (size_t)al * k1;
      const double* w = What + (size_t)be * k1;
      for (int k = 0; k < k1; ++k) s += c1[k] * w[k];
      const int64_t e = (int64_t)al * mB + be;
      item += V[e] * s;
      for (int x = 0; x < 3; ++x) sv[x] += dV[(int64_t)x * mA * mB + e] * s;
    }
  for (int al = 0; al < mA; ++al)
    for (int k = 0; k < k1; ++k) {
      double r = 0;
      for (int be = 0; be < mB; ++be) r += V[(int64_t)al * mB + be] * What[(size_t)be * k1 + k];
      const int64_t e = (int64_t)al * k1 + k;
      for (int x = 0; x < 3; ++x) s1[x] += dC1[(int64_t)x * mA * k1 + e] * r;
    }
  /* Wtil[al][b][g] = sum_{a,f} C1[al][a][f] K[a][f][b][g]
   *               = (D(A,B)^T C1_al D(F,G))[b][g] + (D(F,B)^T C1_al^T D(A,G))[b][g]
   * R2[be][bg] = sum_al V[al][be] Wtil[al][bg]:   C2 slot = <dC2,R2>             */
  for (int al = 0; al < mA; ++al) {
    const double* c1 = C1 + (size_t)al * k1;
    for (int a = 0; a < nA; ++a)
      for (int g = 0; g < nG; ++g) {
        double s = 0;
        for (int f = 0; f < nF; ++f) s += c1[a * nF + f] * dget(DFG, f, g);
        P[a * nG + g] = s;
      }
    for (int f = 0; f < nF; ++f)
      for (int g = 0; g < nG; ++g) {
        double s = 0;
        for (int a = 0; a < nA; ++a) s += c1[a * nF + f] * dget(DAG, a, g);
        Q[f * nG + g] = s;
      }
    double* w = Wtil + (size_t)al * nB * nG;
    for (int b = 0; b < nB; ++b)
      for (int g = 0; g < nG; ++g) {
        double s = 0;
        for (int a = 0; a < nA; ++a) s += dget(DAB, a, b) * P[a * nG + g];
        for (int f = 0; f < nF; ++f) s += dget(DFB, f, b) * Q[f * nG + g];
        w[b * nG + g] = s;
      }
  }
  const int k2 = nB * nG;
  double s2[3] = {0, 0, 0};
  for (int be = 0; be < mB; ++be)
    for (int k = 0; k < k2; ++k) {
      double r = 0;
      for (int al = 0; al < mA; ++al) r += V[(int64_t)al * mB + be] * Wtil[(size_t)al * k2 + k];
      const int64_t e = (int64_t)be * k2 + k;
      for (int x = 0; x < 3; ++x) s2[x] += dC2[(int64_t)x * mB * k2 + e] * r;
    }
  /* want: bit 0 the item (energy), bit 1 the C1 slot, bit 2 the V slot,
   * bit 3 the C2 slot */
  if (want & 1) *E -= item;
  for (int x = 0; x < 3; ++x) {
    if (want & 2) g1[x] -= s1[x];
    if (want & 4) gv[x] -= sv[x];
    if (want & 8) g2[x] -= s2[x];
  }
}

/*
 * Quartet loop over V blocks [v_begin, v_end) in key order; for each, the
 * listed C blocks of A, then the listed C blocks of B (Algorithm 1's loop
 * nest, extended to every term as the text after it describes).
 *
 * keepC / keepV are bit masks per block: bit 0 puts the block in the list of
 * values (C or V), bit 1 in the list of derivatives (dC or dV); keepD 0/1
 * per atom pair.  Each term of a quartet uses its own lists, as the paper's
 * per-tensor thresholds do (Table thr_default): the item (energy) needs C1,
 * V and C2 in the value lists; the C1 slot needs dC1 in the derivative list
 * and V, C2 in the value lists; likewise the V and C2 slots.
 *
 * theta_item > 0: the item-level Cauchy-Schwarz test of Algorithm 1 (Sec.
 * Sparsity exploitation): a term is skipped when the product of the
 * Frobenius norms of its three blocks times |D_AB||D_FG| + |D_AG||D_FB|
 * (Frobenius norms, 0 for a screened D pair) -- a bound on the term --
 * is at most theta_item.  *skipped (optional) receives the sum of the
 * bounds of the skipped energy items, so |E - E(theta_item = 0)| is at most
 * that sum.
 *
 * focus_kind: 0 = all quartets; 1 = only quartets that contain C block
 * focus_idx; 2 = only quartets that contain V block focus_idx.
 * E (scalar), gC[nC][3] and gV[nV][3] are accumulated (caller zeroes them).
 * nthreads > 1 splits the V blocks over OpenMP threads with private
 * accumulators, summed in thread order afterwards.
 */
static double frob(const double* p, int64_t n) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += p[i] * p[i];
  return sqrt(s);
}

int orc_contract2(const orc_input* in, const uint8_t* keepC, const uint8_t* keepV,
                  const uint8_t* keepD, int64_t v_begin, int64_t v_end, int focus_kind,
                  int64_t focus_idx, int nthreads, double theta_item, double* E, double* gC, double* gV,
                  double* skipped) {
  const int N = in->natom;
  int64_t* ao = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  const int64_t nt = ntot_of(in, ao);
  /* kept C blocks grouped by first atom, in key order */
  int64_t* crow = (int64_t*)calloc(N + 1, sizeof(int64_t));
  int64_t* clist = (int64_t*)malloc(sizeof(int64_t) * (in->nC + 1));
  for (int64_t b = 0; b < in->nC; ++b) if (keepC[b] & 3) crow[in->C_first[b] + 1]++;
  for (int i = 0; i < N; ++i) crow[i + 1] += crow[i];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * N);
    for (int i = 0; i < N; ++i) fill[i] = crow[i];
    for (int64_t b = 0; b < in->nC; ++b) if (keepC[b] & 3) clist[fill[in->C_first[b]]++] = b;
    free(fill);
  }
  int mmax = 0, nmax = 0;
  for (int i = 0; i < N; ++i) { if (in->nabf[i] > mmax) mmax = in->nabf[i]; if (in->nao[i] > nmax) nmax = in->nao[i]; }
  const size_t wsz = (size_t)2 * mmax * nmax * nmax + 4 * nmax * nmax + 16;
  if (v_begin < 0) v_begin = 0;
  if (v_end > in->nV) v_end = in->nV;
  int nth = nthreads > 1 ? nthreads : 1;
#ifndef _OPENMP
  nth = 1;
#endif
  double* accE = (double*)calloc(nth, sizeof(double));
  double* accS = (double*)calloc(nth, sizeof(double));
  /* Frobenius norms for the item-level test: [2] per block (value, derivative), D pairs */
  double* nC = NULL; double* nV = NULL; double* nD = NULL;
  if (theta_item > 0) {
    nC = (double*)malloc(sizeof(double) * 2 * (in->nC + 1));
    nV = (double*)malloc(sizeof(double) * 2 * (in->nV + 1));
    nD = (double*)calloc((size_t)N * N, sizeof(double));
    for (int64_t b = 0; b < in->nC; ++b) {
      const int64_t n = c_size(in, b);
      nC[2 * b] = frob(in->C_val + in->C_off[b], n);
      nC[2 * b + 1] = frob(in->C_dval + 3 * in->C_off[b], 3 * n);
    }
    for (int64_t b = 0; b < in->nV; ++b) {
      const int64_t n = v_size(in, b);
      nV[2 * b] = frob(in->V_val + in->V_off[b], n);
      nV[2 * b + 1] = frob(in->V_dval + 3 * in->V_off[b], 3 * n);
    }
    for (int X = 0; X < N; ++X)
      for (int Y = 0; Y < N; ++Y) {
        if (!keepD[X * N + Y]) continue;
        double ss = 0;
        for (int i = 0; i < in->nao[X]; ++i)
          for (int j = 0; j < in->nao[Y]; ++j) {
            const double v = in->D[(ao[X] + i) * nt + ao[Y] + j];
            ss += v * v;
          }
        nD[(int64_t)X * N + Y] = sqrt(ss);
      }
  }
  double* accC = (double*)calloc((size_t)nth * in->nC * 3, sizeof(double));
  double* accV = (double*)calloc((size_t)nth * in->nV * 3, sizeof(double));
  double** wsv = (double**)malloc(sizeof(double*) * nth);
  for (int t = 0; t < nth; ++t) wsv[t] = (double*)malloc(sizeof(double) * wsz);

#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
#endif
  for (int64_t v = v_begin; v < v_end; ++v) {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    if (!(keepV[v] & 3)) continue;
    const int A = in->V_first[v], B = in->V_second[v];
    const int mA = in->nabf[A], mB = in->nabf[B], nA = in->nao[A], nB = in->nao[B];
    const double* V = in->V_val + in->V_off[v];
    const double* dV = in->V_dval + 3 * in->V_off[v];
    dblk DAB = {keepD[A * N + B] ? in->D + ao[A] * nt + ao[B] : NULL, nt};
    for (int64_t i1 = crow[A]; i1 < crow[A + 1]; ++i1) {
      const int64_t c1 = clist[i1];
      const int F = in->C_second[c1], nF = in->nao[F];
      dblk DFB = {keepD[F * N + B] ? in->D + ao[F] * nt + ao[B] : NULL, nt};
      for (int64_t i2 = crow[B]; i2 < crow[B + 1]; ++i2) {
        const int64_t c2 = clist[i2];
        if (focus_kind == 1 && c1 != focus_idx && c2 != focus_idx) continue;
        if (focus_kind == 2 && v != focus_idx) continue;
        const int G = in->C_second[c2], nG = in->nao[G];
        dblk DFG = {keepD[F * N + G] ? in->D + ao[F] * nt + ao[G] : NULL, nt};
        dblk DAG = {keepD[A * N + G] ? in->D + ao[A] * nt + ao[G] : NULL, nt};
        /* the terms this quartet takes: by the lists of its blocks, then by
         * the item-level bound */
        const int e1 = keepC[c1] & 1, d1 = keepC[c1] & 2, ev = keepV[v] & 1, dv = keepV[v] & 2;
        const int e2 = keepC[c2] & 1, d2 = keepC[c2] & 2;
        int want = (e1 && ev && e2 ? 1 : 0) | (d1 && ev && e2 ? 2 : 0) | (e1 && dv && e2 ? 4 : 0) |
                   (e1 && ev && d2 ? 8 : 0);
        if (theta_item > 0 && want) {
          const double kd = nD[(int64_t)A * N + B] * nD[(int64_t)F * N + G] +
                            nD[(int64_t)A * N + G] * nD[(int64_t)F * N + B];
          const double a1 = nC[2 * c1], ad1 = nC[2 * c1 + 1], av = nV[2 * v], adv = nV[2 * v + 1];
          const double a2 = nC[2 * c2], ad2 = nC[2 * c2 + 1];
          if ((want & 1) && a1 * av * a2 * kd <= theta_item) { want &= ~1; accS[t] += a1 * av * a2 * kd; }
          if ((want & 2) && ad1 * av * a2 * kd <= theta_item) want &= ~2;
          if ((want & 4) && a1 * adv * a2 * kd <= theta_item) want &= ~4;
          if ((want & 8) && a1 * av * ad2 * kd <= theta_item) want &= ~8;
        }
        if (!want) continue;
        quartet(mA, mB, nA, nF, nB, nG,
                in->C_val + in->C_off[c1], in->C_dval + 3 * in->C_off[c1], V, dV,
                in->C_val + in->C_off[c2], in->C_dval + 3 * in->C_off[c2],
                DAB, DFG, DAG, DFB, wsv[t], want, &accE[t],
                accC + ((size_t)t * in->nC + c1) * 3, accV + ((size_t)t * in->nV + v) * 3,
                accC + ((size_t)t * in->nC + c2) * 3);
      }
    }
  }
  for (int t = 0; t < nth; ++t) {
    *E += accE[t];
    if (skipped) *skipped += accS[t];
    for (int64_t i = 0; i < 3 * in->nC; ++i) gC[i] += accC[(size_t)t * in->nC * 3 + i];
    for (int64_t i = 0; i < 3 * in->nV; ++i) gV[i] += accV[(size_t)t * in->nV * 3 + i];
    free(wsv[t]);
  }
  free(wsv); free(accE); free(accS); free(accC); free(accV); free(ao); free(crow); free(clist);
  free(nC); free(nV); free(nD);
  return 0;
}

/*
 * The exact-exchange Hamiltonian of Eq. Exx2, H^X = dE/dD (the derivative of
 * Eq. exx_expand with respect to every element of the density matrix, which
 * equals -sum_{kl} (ik|jl) D_kl): the quartet loop above, the energy item of
 * each quartet only (C1, V, C2 in their value lists), with its four D slots.
 * With T[a][f][b][g] = sum_{al,be} C1[al][a][f] V[al][be] C2[be][b][g], a
 * quartet adds
 *   -sum_{fg} T D(F,G)[f][g]  to H(A,B)[a][b],   -sum_{ab} T D(A,B)[a][b]  to H(F,G)[f][g],
 *   -sum_{fb} T D(F,B)[f][b]  to H(A,G)[a][g],   -sum_{ag} T D(A,G)[a][g]  to H(F,B)[f][b],
 * each only where that D pair is kept (a screened pair is zero in E, so E
 * does not depend on it).  H is dense [n_tot][n_tot]; the caller zeroes it.
 * focus_x >= 0: only the quartets with a D slot on the atom pair
 * (focus_x, focus_y), so that block of H is complete and the rest is not.
 * nthreads > 1: private copies over V blocks, summed in thread order.
 */
int orc_hamiltonian(const orc_input* in, const uint8_t* keepC, const uint8_t* keepV, const uint8_t* keepD,
                    int focus_x, int focus_y, int nthreads, double* H) {
  const int N = in->natom;
  int64_t* ao = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  const int64_t nt = ntot_of(in, ao);
  int64_t* crow = (int64_t*)calloc(N + 1, sizeof(int64_t));
  int64_t* clist = (int64_t*)malloc(sizeof(int64_t) * (in->nC + 1));
  for (int64_t b = 0; b < in->nC; ++b) if (keepC[b] & 1) crow[in->C_first[b] + 1]++;
  for (int i = 0; i < N; ++i) crow[i + 1] += crow[i];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * N);
    for (int i = 0; i < N; ++i) fill[i] = crow[i];
    for (int64_t b = 0; b < in->nC; ++b) if (keepC[b] & 1) clist[fill[in->C_first[b]]++] = b;
    free(fill);
  }
  int mmax = 0, nmax = 0;
  for (int i = 0; i < N; ++i) { if (in->nabf[i] > mmax) mmax = in->nabf[i]; if (in->nao[i] > nmax) nmax = in->nao[i]; }
  int nth = nthreads > 1 ? nthreads : 1;
#ifndef _OPENMP
  nth = 1;
#endif
  /* per thread: U[be][a][f], T[a][f][b][g] and a private H */
  const size_t usz = (size_t)mmax * nmax * nmax, tsz = (size_t)nmax * nmax * nmax * nmax;
  double** ws = (double**)malloc(sizeof(double*) * nth);
  double** hp = (double**)malloc(sizeof(double*) * nth);
  for (int t = 0; t < nth; ++t) {
    ws[t] = (double*)malloc(sizeof(double) * (usz + tsz + 1));
    hp[t] = (double*)calloc((size_t)nt * nt, sizeof(double));
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
#endif
  for (int64_t v = 0; v < in->nV; ++v) {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    if (!(keepV[v] & 1)) continue;
    const int A = in->V_first[v], B = in->V_second[v];
    const int mA = in->nabf[A], mB = in->nabf[B], nA = in->nao[A], nB = in->nao[B];
    const double* V = in->V_val + in->V_off[v];
    double* U = ws[t];
    double* T = U + usz;
    double* Hm = hp[t];
    for (int64_t i1 = crow[A]; i1 < crow[A + 1]; ++i1) {
      const int64_t c1 = clist[i1];
      const int F = in->C_second[c1], nF = in->nao[F];
      const double* C1 = in->C_val + in->C_off[c1];
      /* every D slot of a quartet has A or F as its first atom */
      if (focus_x >= 0 && A != focus_x && F != focus_x) continue;
      /* U[be][a f] = sum_al V[al][be] C1[al][a f] */
      const int k1 = nA * nF;
      for (int be = 0; be < mB; ++be)
        for (int k = 0; k < k1; ++k) {
          double s = 0;
          for (int al = 0; al < mA; ++al) s += V[(int64_t)al * mB + be] * C1[(int64_t)al * k1 + k];
          U[(size_t)be * k1 + k] = s;
        }
      for (int64_t i2 = crow[B]; i2 < crow[B + 1]; ++i2) {
        const int64_t c2 = clist[i2];
        const int G = in->C_second[c2], nG = in->nao[G];
        if (focus_x >= 0 && !((A == focus_x && B == focus_y) || (F == focus_x && G == focus_y) ||
                              (A == focus_x && G == focus_y) || (F == focus_x && B == focus_y)))
          continue;
        const double* C2 = in->C_val + in->C_off[c2];
        const int k2 = nB * nG;
        /* T[a f][b g] = sum_be U[be][a f] C2[be][b g] */
        for (int k = 0; k < k1; ++k)
          for (int l = 0; l < k2; ++l) {
            double s = 0;
            for (int be = 0; be < mB; ++be) s += U[(size_t)be * k1 + k] * C2[(int64_t)be * k2 + l];
            T[(size_t)k * k2 + l] = s;
          }
        const int kAB = keepD[A * N + B], kFG = keepD[F * N + G], kAG = keepD[A * N + G], kFB = keepD[F * N + B];
        const double* D = in->D;
        for (int a = 0; a < nA; ++a)
          for (int f = 0; f < nF; ++f)
            for (int b = 0; b < nB; ++b)
              for (int g = 0; g < nG; ++g) {
                const double x = T[(size_t)(a * nF + f) * k2 + b * nG + g];
                const int64_t ia = ao[A] + a, jf = ao[F] + f, kb = ao[B] + b, lg = ao[G] + g;
                const double dAB = kAB ? D[ia * nt + kb] : 0.0, dFG = kFG ? D[jf * nt + lg] : 0.0;
                const double dAG = kAG ? D[ia * nt + lg] : 0.0, dFB = kFB ? D[jf * nt + kb] : 0.0;
                if (kAB) Hm[ia * nt + kb] -= x * dFG;
                if (kFG) Hm[jf * nt + lg] -= x * dAB;
                if (kAG) Hm[ia * nt + lg] -= x * dFB;
                if (kFB) Hm[jf * nt + kb] -= x * dAG;
              }
      }
    }
  }
  for (int t = 0; t < nth; ++t) {
    for (int64_t i = 0; i < nt * nt; ++i) H[i] += hp[t][i];
    free(ws[t]);
    free(hp[t]);
  }
  free(ws); free(hp); free(ao); free(crow); free(clist);
  return 0;
}

/* The joint lists of orc_screen (a kept block in both lists), no item test. */
int orc_contract(const orc_input* in, const uint8_t* keepC, const uint8_t* keepV,
                 const uint8_t* keepD, int64_t v_begin, int64_t v_end, int focus_kind,
                 int64_t focus_idx, int nthreads, double* E, double* gC, double* gV) {
  uint8_t* kc = (uint8_t*)malloc(in->nC + 1);
  uint8_t* kv = (uint8_t*)malloc(in->nV + 1);
  for (int64_t b = 0; b < in->nC; ++b) kc[b] = keepC[b] ? 3 : 0;
  for (int64_t b = 0; b < in->nV; ++b) kv[b] = keepV[b] ? 3 : 0;
  const int rc = orc_contract2(in, kc, kv, keepD, v_begin, v_end, focus_kind, focus_idx, nthreads, 0.0, E, gC, gV,
                               NULL);
  free(kc);
  free(kv);
  return rc;
}

/*
 * Forces and stress from block gradients (Eq. Fexx1 and Eq. stress):
 * block b with displacement r_b = tau_second + R.L - tau_first and
 * g_b = dE/dr_b gives F_first += g_b, F_second -= g_b, W += g_b (x) r_b;
 * sigma = -W / Omega.
 */
void orc_forces_stress(const orc_input* in, const double* gC, const double* gV, double* F, double* sigma) {
  const int N = in->natom;
  double W[9] = {0};
  for (int i = 0; i < 3 * N; ++i) F[i] = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const int64_t nb = pass ? in->nV : in->nC;
    const int32_t* fi = pass ? in->V_first : in->C_first;
    const int32_t* se = pass ? in->V_second : in->C_second;
    const int32_t* R = pass ? in->V_R : in->C_R;
    const double* g = pass ? gV : gC;
    for (int64_t b = 0; b < nb; ++b) {
      double r[3];
      for (int x = 0; x < 3; ++x)
        r[x] = in->tau[3 * se[b] + x] - in->tau[3 * fi[b] + x] + R[3 * b] * in->lat[x] +
               R[3 * b + 1] * in->lat[3 + x] + R[3 * b + 2] * in->lat[6 + x];
      for (int x = 0; x < 3; ++x) {
        F[3 * fi[b] + x] += g[3 * b + x];
        F[3 * se[b] + x] -= g[3 * b + x];
        for (int y = 0; y < 3; ++y) W[3 * x + y] += g[3 * b + x] * r[y];
      }
    }
  }
  const double* L = in->lat;
  double omega = fabs(L[0] * (L[4] * L[8] - L[5] * L[7]) - L[1] * (L[3] * L[8] - L[5] * L[6]) +
                      L[2] * (L[3] * L[7] - L[4] * L[6]));
  for (int i = 0; i < 9; ++i) sigma[i] = -W[i] / omega;
}

int orc_has_openmp(void) {
#ifdef _OPENMP
  return 1;
#else
  return 0;
#endif
}

/* ------------------------------------------------------------------------ */
/*
 * k-point sampling (Methods, Eq. Eexx with the k-sum definition of D, and
 * Eq. exx_expand).  The k mesh of nk[0] x nk[1] x nk[2] points makes the
 * Born-von Karman (BvK) supercell of as many unit cells, and the density
 * matrix of two orbitals depends on the offset of their cells modulo that
 * supercell:
 *   D_{(I,R_I) i, (J,R_J) j} = Dk[r][ao(I) + i][ao(J) + j],
 *   r = r_0 + nk_0 (r_1 + nk_1 r_2),  r_x = (R_J - R_I)_x mod nk_x,
 * complex (Dre, Dim; Dim = NULL for a real D(R)) and Hermitian.  The energy
 * per unit cell is the quartet sum of orc_contract2 with the atom of the V
 * block in the home cell and the weight
 *   Re[ D_AB D*_FG + D_AG D*_FB ],
 *   D_AB at offset R_B, D_FG at R_B + R_G - R_F, D_AG at R_B + R_G, D_FB at R_B - R_F
 * (C1 = C(A,F,R_F), V = V(A,B,R_B), C2 = C(B,G,R_G): F sits at R_F, B at
 * R_B, G at R_B + R_G).  There is no folding: every image keeps its own
 * offset.  Since Re[z w*] = Re z Re w + Im z Im w, a quartet is the real
 * quartet of the real parts plus the real quartet of the imaginary parts,
 * with the same blocks and lists.  With nk = (1,1,1) and Dim = NULL this is
 * exactly orc_contract2 without the item test.
 */
static int kp_offset(const int32_t* nk, int x, int y, int z) {
  int r[3] = {x, y, z};
  for (int k = 0; k < 3; ++k) r[k] = ((r[k] % nk[k]) + nk[k]) % nk[k];
  return r[0] + nk[0] * (r[1] + nk[1] * r[2]);
}

/* D pairs per offset: keepD[(r * N + X) * N + Y] = 1 iff the largest modulus
 * of an element of D(r)_XY exceeds theta_D (theta_D <= 0 keeps every pair).
 * The mirror block D(-r)_YX holds the conjugate transpose, so the decision is
 * the same for both. */
void orc_screen_d_kp(const orc_input* in, const int32_t* nk, const double* Dre, const double* Dim,
                     double theta_D, uint8_t* keepD) {
  const int N = in->natom;
  int64_t* ao = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  const int64_t nt = ntot_of(in, ao);
  const int nr = nk[0] * nk[1] * nk[2];
  for (int r = 0; r < nr; ++r)
    for (int X = 0; X < N; ++X)
      for (int Y = 0; Y < N; ++Y) {
        double mx = 0;
        for (int i = 0; i < in->nao[X]; ++i)
          for (int j = 0; j < in->nao[Y]; ++j) {
            const int64_t e = (int64_t)r * nt * nt + (ao[X] + i) * nt + ao[Y] + j;
            const double re = Dre[e], im = Dim ? Dim[e] : 0.0;
            const double m = sqrt(re * re + im * im);
            if (m > mx) mx = m;
          }
        keepD[((int64_t)r * N + X) * N + Y] = (uint8_t)(!(theta_D > 0) || mx > theta_D);
      }
  free(ao);
}

int orc_contract_kp(const orc_input* in, const int32_t* nk, const double* Dre, const double* Dim,
                    const uint8_t* keepC, const uint8_t* keepV, const uint8_t* keepD, int nthreads, double* E,
                    double* gC, double* gV) {
  const int N = in->natom;
  int64_t* ao = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  const int64_t nt = ntot_of(in, ao);
  const int64_t nn = nt * nt;
  int64_t* crow = (int64_t*)calloc(N + 1, sizeof(int64_t));
  int64_t* clist = (int64_t*)malloc(sizeof(int64_t) * (in->nC + 1));
  for (int64_t b = 0; b < in->nC; ++b) if (keepC[b] & 3) crow[in->C_first[b] + 1]++;
  for (int i = 0; i < N; ++i) crow[i + 1] += crow[i];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * N);
    for (int i = 0; i < N; ++i) fill[i] = crow[i];
    for (int64_t b = 0; b < in->nC; ++b) if (keepC[b] & 3) clist[fill[in->C_first[b]]++] = b;
    free(fill);
  }
  int mmax = 0, nmax = 0;
  for (int i = 0; i < N; ++i) { if (in->nabf[i] > mmax) mmax = in->nabf[i]; if (in->nao[i] > nmax) nmax = in->nao[i]; }
  const size_t wsz = (size_t)2 * mmax * nmax * nmax + 4 * nmax * nmax + 16;
  int nth = nthreads > 1 ? nthreads : 1;
#ifndef _OPENMP
  nth = 1;
#endif
  double* accE = (double*)calloc(nth, sizeof(double));
  double* accC = (double*)calloc((size_t)nth * in->nC * 3, sizeof(double));
  double* accV = (double*)calloc((size_t)nth * in->nV * 3, sizeof(double));
  double** wsv = (double**)malloc(sizeof(double*) * nth);
  for (int t = 0; t < nth; ++t) wsv[t] = (double*)malloc(sizeof(double) * wsz);

#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
#endif
  for (int64_t v = 0; v < in->nV; ++v) {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    if (!(keepV[v] & 3)) continue;
    const int A = in->V_first[v], B = in->V_second[v];
    const int mA = in->nabf[A], mB = in->nabf[B], nA = in->nao[A], nB = in->nao[B];
    const int32_t* RB = in->V_R + 3 * v;
    const double* V = in->V_val + in->V_off[v];
    const double* dV = in->V_dval + 3 * in->V_off[v];
    for (int64_t i1 = crow[A]; i1 < crow[A + 1]; ++i1) {
      const int64_t c1 = clist[i1];
      const int F = in->C_second[c1], nF = in->nao[F];
      const int32_t* RF = in->C_R + 3 * c1;
      for (int64_t i2 = crow[B]; i2 < crow[B + 1]; ++i2) {
        const int64_t c2 = clist[i2];
        const int G = in->C_second[c2], nG = in->nao[G];
        const int32_t* RG = in->C_R + 3 * c2;
        const int rAB = kp_offset(nk, RB[0], RB[1], RB[2]);
        const int rFG = kp_offset(nk, RB[0] + RG[0] - RF[0], RB[1] + RG[1] - RF[1], RB[2] + RG[2] - RF[2]);
        const int rAG = kp_offset(nk, RB[0] + RG[0], RB[1] + RG[1], RB[2] + RG[2]);
        const int rFB = kp_offset(nk, RB[0] - RF[0], RB[1] - RF[1], RB[2] - RF[2]);
        const int kAB = keepD[((int64_t)rAB * N + A) * N + B], kFG = keepD[((int64_t)rFG * N + F) * N + G];
        const int kAG = keepD[((int64_t)rAG * N + A) * N + G], kFB = keepD[((int64_t)rFB * N + F) * N + B];
        const int e1 = keepC[c1] & 1, d1 = keepC[c1] & 2, ev = keepV[v] & 1, dv = keepV[v] & 2;
        const int e2 = keepC[c2] & 1, d2 = keepC[c2] & 2;
        const int want = (e1 && ev && e2 ? 1 : 0) | (d1 && ev && e2 ? 2 : 0) | (e1 && dv && e2 ? 4 : 0) |
                         (e1 && ev && d2 ? 8 : 0);
        if (!want) continue;
        for (int part = 0; part < (Dim ? 2 : 1); ++part) {
          const double* Dp = part ? Dim : Dre;
          dblk DAB = {kAB ? Dp + rAB * nn + ao[A] * nt + ao[B] : NULL, nt};
          dblk DFG = {kFG ? Dp + rFG * nn + ao[F] * nt + ao[G] : NULL, nt};
          dblk DAG = {kAG ? Dp + rAG * nn + ao[A] * nt + ao[G] : NULL, nt};
          dblk DFB = {kFB ? Dp + rFB * nn + ao[F] * nt + ao[B] : NULL, nt};
          quartet(mA, mB, nA, nF, nB, nG,
                  in->C_val + in->C_off[c1], in->C_dval + 3 * in->C_off[c1], V, dV,
                  in->C_val + in->C_off[c2], in->C_dval + 3 * in->C_off[c2],
                  DAB, DFG, DAG, DFB, wsv[t], want, &accE[t],
                  accC + ((size_t)t * in->nC + c1) * 3, accV + ((size_t)t * in->nV + v) * 3,
                  accC + ((size_t)t * in->nC + c2) * 3);
        }
      }
    }
  }
  for (int t = 0; t < nth; ++t) {
    *E += accE[t];
    for (int64_t i = 0; i < 3 * in->nC; ++i) gC[i] += accC[(size_t)t * in->nC * 3 + i];
    for (int64_t i = 0; i < 3 * in->nV; ++i) gV[i] += accV[(size_t)t * in->nV * 3 + i];
    free(wsv[t]);
  }
  free(wsv); free(accE); free(accC); free(accV); free(ao); free(crow); free(clist);
  return 0;
}
