// Internal declarations of the LRI exact-exchange library (gfx950).
//
// Data layout on the device (all row-major, FP64 unless noted):
//   inputs   C/V block values and derivatives exactly as the caller gave them
//            (borrowed or copied), D dense [n_tot][n_tot] (with k-point
//            sampling: D(R) per Born-von Karman cell offset, read through
//            d_block);
//   pairs    the image blocks grouped by (first, second) atom pair: a "C pair"
//            (A,F) and a "V pair" (A,B), each with the sorted list of its
//            image blocks (R lexicographic);
//   folded   Cf(A,F) = sum of kept C images [mA][nA][nF];
//            Vf(A,B) = sum of kept V images [mA][mB rounded up to 16, zero
//            padding]  (Gamma point: the density
//            matrix is the same for every image pair, so the images of a pair
//            meet the same D blocks and can be summed first);
//   H        H(B,X)[b][beta][x] = sum_G Cf(B,G)[beta][b][g] D(G,X)[g][x] for
//            every (B,X) a triple (A,F,B) needs (X = A or X = F); beta runs
//            over the ABFs of B rounded up to 16 (padding rows stay zero);
//   Zbuf     per triple (A,F,B) whose V pair forms Z (vpZ: of a pair and its
//            mirror the one with the lower index; A <= B at the Gamma point)
//            and column chunk: the F-partial of
//            Z(A,B)[alpha][beta] = sum_{F,a,f} Cf(A,F)[alpha][a][f] X^{AFB}[beta][a][f]
//            (Z(B,A) = Z(A,B)^T: D is symmetric and the screening keeps
//            mirror pairs together, so pairs with A > B take the transpose),
//            X^{AFB}[beta][a][f] = sum_b D_AB[a][b] H(B,F)[beta][b][f]
//                                + sum_b D_FB[f][b] H(B,A)[beta][b][a];
//   Ybuf     per C pair and V-pair range s: Y_s(A,F)[alpha][a][f] = sum_{B in range s}
//            sum_beta Vf(A,B)[alpha][beta] X^{AFB}[beta][a][f]  (Y = sum_s Y_s).
// With these, E = -sum_{A,B} <Vf(A,B), Z(A,B)>, dE/dV = -Z and dE/dCf = -2 Y
// (E is a symmetric quadratic form in C), so each image block's gradient is
// a single contraction of its d/dr with Z or Y.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lrx {

constexpr int kMaxNao = 32;
constexpr int kMaxNabf = 128;
constexpr int kMaxAlphaTiles = (kMaxNabf + 15) / 16;

// Columns of the (a,f) index one triple work unit owns, by the number of
// 16-row ABF tiles of its atom A (the unit keeps fragments of Cf(A,F) for
// these columns and the Y tiles of these columns in registers).
__host__ __device__ constexpr int unit_cols(int alpha_tiles) { return alpha_tiles <= 5 ? 176 : 128; }
constexpr int kSideStreams = 3;    // extra streams: alpha-tile groups of the triple kernel run concurrently
constexpr int kHRows = 128;        // rows (beta,b) of H one H-build workgroup owns
constexpr int kHItemCols = 256;    // columns (X,x) of H one H-build workgroup owns
constexpr int kHMaxDepth = 512;    // max sum of NAOs over the C partners of one atom
constexpr int kHPass = 64;         // depth of one H-build pass
constexpr int kHxMaxCPartners = 64;   // C partners of one atom (at most one column chunk each, 64 chunks)

enum Prec : int { kP64 = 0, kP32 = 1, kPB3 = 2 };

// Device memory cache (lrx_mem.hip), per device and process-wide: blocks are
// served from memory the cache has mapped and come back to it on dev_free;
// nullptr when the device is out of memory.  dev_free only after the work
// that uses the block has finished.  dev_trim unmaps idle segments until at
// most `keep` bytes stay mapped (device idle) and returns the bytes mapped.
void* dev_alloc(int device, size_t bytes);
void dev_free(int device, void* p);
size_t dev_trim(int device, size_t keep);
void dev_cache_bytes(int device, size_t* mapped, size_t* used);

// Everything the kernels read or write for one structure.  Passed by value.
struct Dev {
  int N;
  int64_t ntot;
  const double* tau;      // [N][3]
  const double* lat;      // [3][3]
  double omega;
  const int* nao;         // [N]
  const int* nabf;        // [N]
  const int64_t* ao;      // [N+1]

  // input blocks (caller order)
  int64_t nC, nV;
  const int* Cfirst; const int* Csecond; const int* CR; const int64_t* Coff; const int* Csz;
  const double* Cval; const double* Cdval;
  const int* Vfirst; const int* Vsecond; const int* VR; const int64_t* Voff; const int* Vsz;
  const double* Vval; const double* Vdval;
  const int64_t* Vmir;    // mirror block (second, first, -R)
  const double* D;        // [ntot][ntot] at the Gamma point; D(R) [ncell][nt0][nt0] with k-points (d_block)
  // the matrices the D screen measures: DnRe (= D at the Gamma point) and,
  // for a complex density matrix, its imaginary part DnIm (else nullptr); the
  // screen then takes the modulus, so both real passes of a complex D keep
  // the same pairs
  const double* DnRe; const double* DnIm;
  // Addressing of D blocks.  Block (X,Y) starts at element
  //   dsub[acell[X] * ncell + acell[Y]] * dcellsz + aloc[X] * dld + aloc[Y]
  // with rows dld elements apart (d_block).  At the Gamma point: one cell,
  // aloc = ao, dld = ntot, so block (X,Y) is at ao[X] ntot + ao[Y].  With
  // k-point sampling the atoms are those of the Born-von Karman supercell,
  // acell the cell of an atom, aloc its AO offset within the unit cell, and
  // D is the caller's D(R) [ncell][nt0][nt0] (dld = nt0, dcellsz = nt0^2),
  // dsub[t][u] the offset u - t of two cells.  dsize = elements of D.
  const int* acell; const int64_t* aloc; const int* dsub;
  int ncell;
  int64_t dld, dcellsz, dsize;

  // pairs
  int nCp, nVp;
  const int* cpA; const int* cpF; const int* cpB0; const int* cpB1; const int64_t* cpBlk; const int* cpRow;
  const int* vpA; const int* vpB; const int* vpB0; const int* vpB1; const int64_t* vpBlk; const int* vpRow;
  const int* vpMir;
  const uint8_t* vpZ;      // 1: the pair forms Z(A,B) (of a pair and its mirror exactly one; B >= A at the Gamma point)
  const int64_t* cfOff; const int64_t* vfOff;
  double* Cf;             // folded C pair blocks [mA][nA][nF] at cfOff
  double* Vf;             // folded V pair blocks [mA][mB padded to 16] at vfOff (zero padding)
  // FP32 copies used by the reduced-precision forms (allocated on first use)
  float* Cf32; float* Vf32; float* D32; float* H32; float* Zbuf32; float* Ybuf32;

  // screening
  double* nrmC;  // [nC][4]: max|val|, max|dval|, sum val^2, sum dval^2
  double* nrmV;  // [nV][4]
  double* dmax;  // [N][N] (entries with X <= Y)
  double* dss;   // [N][N]
  uint8_t* keepC; uint8_t* keepV; uint8_t* keepD;
  double* cval;  // [nCp]
  double* dnrm;  // [N][N]
  double* Svp;   // [nVp]
  uint8_t* aliveC; uint8_t* aliveV;

  // H slots
  int nSlot;
  const int* slotB; const int* slotX; const int64_t* hOff; const int* hSlotMap; // [N][N] -> slot or -1
  const int* slotRow;      // [N+1] slots of atom B are slotRow[B] .. slotRow[B+1]-1 (sorted by X)
  const int* slotByX;      // [nSlot] the slots in (X, B) order
  int nHB; const int* hbB; const int* hbR0; const int* hbC0;   // H-build work items: (B, first row, first column)
  const int* hColRow;      // [N+1] columns of atom B: the (slot, x) of every H slot of B, concatenated
  const int* hColSlot; const int* hColX; const int* hColD; const int* hColAtom;
  uint8_t* need;
  // per evaluation: the static depth and column tables of every atom B
  // compacted to the live C pairs (B,G) and the needed slots (B,X), in the
  // same regions and order (k_hcompact); hcK[B] depth entries (a multiple of
  // 4, at least 4), hcNcol[B] columns
  int* hcK; int* hcNcol;
  int* hcRowD; int* hcG; int* hcCp; int64_t* hcCf; int* hcStride;
  int* hcColSlot; int* hcColD; int* hcColAtom;
  double* H;

  // triple work units
  int nUnit;
  const int* unitCp; const int* unitK0; const int* unitK1; const int* unitKc;
  const int* unitV0; const int* unitV1; const int* unitS;   // V-pair range and split index of a unit
  const uint8_t* unitYonly; // 1: no V pair of the unit forms Z (only Y is formed; B < A at the Gamma point)
  uint8_t* unitRole;        // per evaluation: 0 no work, 1 Z and Y, 2 Y alone (unit_y_only)
  const int* nsplit;       // [nCp] number of V-pair ranges (Y partials) of a C pair
  const int* unitOrder;    // units grouped by the alpha-tile count of their atom A
  int mtStart[kMaxAlphaTiles + 2];
  const int* nkc;          // [nCp] column chunks of the pair
  const int64_t* tBase;    // [N] first triple index of atom A
  const int64_t* zOff;     // [ntriple] element offset of the triple's Z partials
  const int64_t* triHF;    // [ntriple] offset of H(B,F) in H
  const int64_t* triHA;    // [ntriple] offset of H(B,A) in H
  const int* hdRow;        // [N+1] static H-build depth table of atom B (multiple of 4 entries):
  const int* hdRowD;       //   D row ao[G] + g,
  const int* hdG;          //   atom G (-1: padding),
  const int* hdCp;         //   (C pair << 6) | g,
  const int64_t* hdCf;     //   offset of Cf(B,G)[0][0][g],
  const int* hdStride;     //   n_G (row stride of Cf(B,G) over (beta,b))
  double* Zbuf;
  const int64_t* yOff;     // [nCp]
  double* Ybuf;

  // gradients and outputs
  double* gC;    // [nC][3]
  double* gV;    // [nV][3]
  double* Ep;    // [nVp]
  const int* atCfRow; const int64_t* atCf;   // C blocks by first atom
  const int* atCsRow; const int64_t* atCs;   // ... by second atom
  const int* atVfRow; const int64_t* atVf;
  const int* atVsRow; const int64_t* atVs;
  double* out;   // [1 + 3N + 9]: E, F, sigma
  int* err;      // validation error code (0 = ok)
};

// Screening options of one evaluation.  Joint mode (per_tensor == 0): one
// theta for every tensor, a block kept in both its lists.  Per-tensor mode:
// th = {C, V, D, dC, dV}; keep masks are bits: 1 = value in the value list
// (folded into Cf / Vf), 2 = derivative in the derivative list (its
// gradient is formed); the joint mode stores 3 for a kept block.
struct Opts {
  double theta;
  double theta_cs;
  int prec;
  int per_tensor = 0;
  double th[5] = {0, 0, 0, 0, 0};
};

// Work of the triple (A,F,B) given the liveness bits of C pair (A,F) and V
// pair (A,B) (bit 1: a block in the value list, bit 2: one in the
// derivative list; the joint screening sets both).  Z(A,B) takes
// Cf(A,F) X^{AFB} and is formed by the V pairs that own it (vpZ; the
// mirror's Z is its transpose); it is read when (A,B) is live at all.
// Y(A,F) takes Vf(A,B) X^{AFB} and is read only when (A,F) has a block in
// the derivative list.  A unit whose C pair has no value-list block, or
// whose V pairs do not form Z (z_elsewhere), forms Y alone (y_only) and
// then only over V pairs with a value-list block.
__host__ __device__ inline bool unit_y_only(int aliveC, bool z_elsewhere) { return z_elsewhere || !(aliveC & 1); }
__host__ __device__ inline bool triple_live(int aliveC, int aliveV, bool z_elsewhere) {
  if (!aliveC || !aliveV) return false;
  if (unit_y_only(aliveC, z_elsewhere)) return (aliveC & 2) && (aliveV & 1);
  return true;
}

// kernels (lrx_screen.hip)
// Value checks of the inputs (mirror blocks, on-site symmetry, finiteness of
// V and D); the symmetry of D is checked by launch_validate_dsym.
void launch_validate(const Dev& d, hipStream_t s);
// D[i][j] == D[j][i] (anti = 0) or == -D[j][i] (anti = 1) within rounding,
// for a dense [nt][nt] matrix; a failure sets kErrDSym in *err.
void launch_validate_dsym(const double* D, int64_t nt, int anti, int* err, hipStream_t s);
// Value-check error bits (Dev::err), reported by the set-up.
enum : int {
  kErrNonfiniteC = 1, kErrNonfiniteV = 2, kErrNonfiniteD = 4, kErrVMirror = 8, kErrDVMirror = 16,
  kErrOnsiteC = 32, kErrDSym = 64
};

// First element of the D block (X,Y); rows d.dld elements apart.
__device__ inline int64_t d_block(const Dev& d, int X, int Y) {
  return (int64_t)d.dsub[d.acell[X] * d.ncell + d.acell[Y]] * d.dcellsz + d.aloc[X] * d.dld + d.aloc[Y];
}
// k-point sampling (lrx_kpoint.hip).  D(R) per Born-von Karman cell offset,
// Dk[r][nt][nt] real part and (optionally) imaginary part: D(-r) = D(r)^H
// within rounding, else kErrDSym in *err; non-finite values set
// kErrNonfiniteD.  nk: the mesh; r = r0 + nk0 (r1 + nk1 r2).
void launch_validate_herm(const double* Dre, const double* Dim, const int* nk, int64_t nt, int* err, hipStream_t s);
// x[i] = keep[i] - x[i] for i < n (the second real pass of a complex D).
void launch_sub_from(const double* keep, double* x, int64_t n, hipStream_t s);
// for_hx: the H slots the Hamiltonian reads (every triple whose C pair and V
// pair have value-list blocks) instead of those of the forces
void launch_screen(const Dev& d, const Opts& o, hipStream_t s, hipEvent_t* ev, bool for_hx = false);
// Only the FP32 copy of D that the reduced-precision kernels read (nothing at
// FP64): for a second pass with another D and the same screening decisions.
void launch_d_to_f32(const Dev& d, int prec, hipStream_t s);
// kernels (lrx_contract.hip)

// Work of the triple-product kernels: per alpha-tile group MT, a list of
// (structure, unit) items over an array of structures on the device.  One
// structure for lrx_evaluate; several for lrx_evaluate_batch.
// mode 0: one workgroup per item (block order remapped for XCD locality);
// mode 1: a persistent grid of one workgroup per CU pulling items from eight
//         per-XCD segments (then from the other segments) through counters.
// Up to kBatchDevs structures travel by value in the kernel arguments of
// one triple launch (kernel arguments are limited to 4 KiB).
constexpr int kBatchDevs = 4;
struct DevBatch {
  Dev s[kBatchDevs];
};
struct TripleLaunch {
  DevBatch devs;                             // the structures of the launch
  int* counters = nullptr;                   // device, 8 per group (mode 1)
  const int2* items[kMaxAlphaTiles + 1] = {};
  int n[kMaxAlphaTiles + 1] = {};
  int mode[kMaxAlphaTiles + 1] = {};
};
constexpr int kPersistentGrid = 256;         // workgroups of a mode-1 launch (one per CU)

void launch_hbuild(const Dev& d, int prec, hipStream_t s);
// triple groups of tl: the largest on s, the others on the side streams, joined back into s
// gev (optional): events recorded around each group's launch on its stream,
// gev[2 MT] before and gev[2 MT + 1] after
void launch_triples(const TripleLaunch& tl, int prec, hipStream_t s, const hipStream_t* side, const hipEvent_t* fork,
                    hipEvent_t* gev = nullptr);
// one group on s (the tuner times groups one at a time)
void launch_triple_group(const TripleLaunch& tl, int mt, int prec, hipStream_t s);
void launch_grads(const Dev& d, int prec, hipStream_t s, hipEvent_t* ev);
// the whole contraction of one structure: hbuild, triples, gradients, forces;
// ev (optional) receives stage marks ev[4..8]
void launch_contract(const Dev& d, const TripleLaunch& tl, int prec, hipStream_t s, const hipStream_t* side,
                     const hipEvent_t* fork, hipEvent_t* ev, hipEvent_t* gev = nullptr);
void launch_validate_finite(const double* p, int64_t n, int* err, int code, hipStream_t s);

// kernels (lrx_fock.hip): the exact-exchange Hamiltonian H^X = dE/dD
struct HxBufs {
  double* Hbar;    // adjoint of H, laid out as the H slots (n_h)
  double* G12;     // [ntot][ntot] gradient parts through D(A,B) and D(F,B)
  double* G3;      // [ntot][ntot] gradient part through H
  double* Hx;      // [ntot][ntot] output (device)
  double* Etile;   // [hx_tiles(ntot)]
  double* E;       // [1] <H^X, D> / 2
  int kmax;        // largest n_A n_X over the C pairs (Q tile row length)
  int nmax;        // largest NAO count of an atom
  const int* g3blk[2];   // D blocks G N + X that G3 can reach, by 16-wide tile count of max(nG, nX)
  int n3[2];
};
int64_t hx_tiles(int64_t ntot);
// after launch_screen(..., for_hx = true) and the FP64 H build; ev
// (optional) marks after the slot kernel, after G3 and at the end
void launch_hx(const Dev& d, const HxBufs& b, hipStream_t s, hipEvent_t* ev);

}  // namespace lrx
