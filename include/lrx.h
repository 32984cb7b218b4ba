/*
 * lrx.h -- C-ABI of the MI355X (gfx950) library for the localized-RI (LRI)
 * exact-exchange energy E_X, the analytic forces F^{X1} and the stress
 * sigma^{X1} of a periodic cell at the Gamma point (lrx_set_tensors) or with
 * k-point sampling (lrx_set_kpoint_tensors), the exact-exchange Hamiltonian
 * H^X (lrx_hamiltonian) and the preparation of the LRI coefficients C
 * (lrx_prepare_c).
 *
 * What is computed (Lin, Ji, He, Ren, "Efficient hybrid-functional-based
 * force and stress calculations for periodic systems with thousands of
 * atoms"):
 *
 *   E   = - sum_{V blocks (A,B,R_B)} sum_{C blocks (A,F,R_F)} sum_{C blocks (B,G,R')}
 *           C^{A}_{AF} V_{AB} C^{B}_{BG} [ D_AB D_FG + D_AG D_FB ]
 *         (Methods, Eq. exx_expand, with N_k = 1 and real tensors; the atom of
 *         the V block's first index lies in the home cell, every partner is an
 *         explicit lattice image, and the Gamma-point density matrix is the
 *         same for every image pair),
 *   F   = -dE/dtau with D held fixed: the six terms of Eq. Fexx1 (F^{X1}; the
 *         density-matrix part F^{X2} of Eq. Exx2 belongs to the host DFT code),
 *   sigma = -(1/Omega) sum_b (dE/dr_b) (x) r_b  (Eq. stress), r_b the
 *         displacement of block b.
 *
 * Screening (Sec. Sparsity exploitation; Tables thr_default, thr_cs):
 *   S1 (theta > 0): a C block is kept iff max|C| > theta or max|dC| > theta;
 *       a V block iff the larger of max|V|, max|dV| over the block and its
 *       mirror (B,A,-R) exceeds theta; a D atom pair (X,Y) iff max|D_XY| >
 *       theta (decided on the block with X <= Y, used for both).
 *   S2 (theta_cs > 0): a surviving V block is kept iff
 *       nv * S(A,B) > theta_cs, nv = the largest Frobenius norm of V, dV of
 *       the block and its mirror, S(A,B) = sum_{F,G} c(A,F) c(B,G)
 *       [d(A,B) d(F,G) + d(A,G) d(F,B)] with c(A,F) the sum over kept C
 *       images of max(|C|_F, |dC|_F) and d(X,Y) = |D_XY|_F of a kept D pair.
 *       S bounds |Z(A,B)|_F (Cauchy-Schwarz, Sec. Sparsity exploitation), so
 *       the test drops a V pair only when all of its items together are small.
 *
 * Units: Bohr, Hartree.  All arrays are row-major.  Return codes: 0 on
 * success, a negative LRX_E* code on error; the message is available from
 * lrx_last_error().  No entry point throws or aborts.  One context per host
 * thread; a context is not thread-safe.
 */
#ifndef LRX_H
#define LRX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LRX_OK = 0,
  LRX_EINVAL = -1,     /* invalid argument or inconsistent input            */
  LRX_ENOMEM = -2,     /* device or host allocation failed                  */
  LRX_EHIP = -3,       /* a HIP runtime call failed                         */
  LRX_ESTATE = -4,     /* call out of order (e.g. evaluate before tensors)  */
  LRX_EBUDGET = -5,    /* request exceeds the configured device-memory budget */
  LRX_ENOTFOUND = -6   /* unknown ticket                                    */
};

typedef enum {
  LRX_FP64 = 0,        /* every product in FP64 (MFMA f64)                                   */
  LRX_FP32 = 1,        /* contractions in FP32 on MFMA, FP32 accumulation, FP64 reductions    */
  LRX_BF16X3 = 2       /* contractions as bf16 hi*hi + hi*lo + lo*hi on MFMA with FP32
                          accumulation (operands split into bf16 hi and residual lo), FP64
                          reductions                                                          */
} lrx_precision;

/* lrx_options.flags */
#define LRX_BATCH_EAGER 1     /* lrx_evaluate_batch: launch the kernels one by one; no graph is captured */
#define LRX_BATCH_NO_TUNE 2   /* lrx_evaluate_batch: skip the launch-shape autotuner                     */
#define LRX_SCREEN_PER_TENSOR 4
/* Step 1 with one threshold per tensor (Sec. Sparsity exploitation, Table
 * thr_default): theta_tensor = {C, V, D, dC, dV} replaces theta.  A C block
 * enters the value list (folded into the energy's C) iff max|C| > theta_C and
 * the derivative list (its gradient is formed) iff max|dC| > theta_dC; V
 * blocks likewise over the block and its mirror; D pairs iff max|D| >
 * theta_D.  Every term then uses its own lists: the energy the value lists,
 * the gradient of a block its derivative and the other blocks' values.  A
 * threshold <= 0 keeps that whole list.  Step 2 (theta_cs) drops a V block
 * from both lists, with c(A,F) and nv taken over the kept parts.  Without
 * the flag, theta keeps a block in both lists when its value or its
 * derivative passes. */

typedef struct {
  double theta;        /* S1 threshold; <= 0 disables S1                  */
  double theta_cs;     /* S2 threshold; <= 0 disables S2                  */
  int32_t precision;   /* lrx_precision                                    */
  int32_t timing;      /* nonzero: time every stage with HIP events (lrx_evaluate) */
  int32_t flags;       /* LRX_BATCH_* and LRX_SCREEN_* bits; 0 for the defaults */
  int32_t reserved;    /* set to 0                                         */
  double theta_tensor[5];  /* with LRX_SCREEN_PER_TENSOR: C, V, D, dC, dV thresholds */
} lrx_options;

/*
 * One block-sparse pair tensor (C or V).  Block i couples atom first[i] (the
 * atom carrying the ABF index) with the lattice image R[i] of atom
 * second[i]; its displacement is r_i = tau[second] + R.L - tau[first].
 * Elements: C block [m_first][n_first][n_second] (C^{A alpha}_{A a, F f},
 * Methods, LRI expansion), V block [m_first][m_second] (Eq. V), starting at
 * element off[i] of val.  dval holds d(block)/d r_x for x = 0,1,2 as
 * [3][block] starting at element 3*off[i].  Keys are host arrays; val and
 * dval are host or device pointers (see lrx_set_tensors).
 * Requirements: no duplicate key; every V block has its mirror (second,
 * first, -R) with V_mirror = V^T and dV_mirror = -dV^T (relative 1e-12,
 * Sec. Preparation: V_BA = V_AB^T, grad_B V_AB = -grad_A V_AB); every atom
 * has its on-site C block (A, A, 0), symmetric in (a, f) (swap symmetry of
 * the LRI coefficients).
 */
typedef struct {
  int64_t nblk;
  const int32_t* first;   /* [nblk] */
  const int32_t* second;  /* [nblk] */
  const int32_t* R;       /* [nblk][3] */
  const int64_t* off;     /* [nblk] */
  const double* val;      /* [nval] */
  const double* dval;     /* [3*nval] */
  int64_t nval;
} lrx_blocks;

typedef struct lrx_ctx lrx_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * to run on (e.g. the caller's current stream; it must outlive the
 * context), or NULL for a stream the context owns.  Owned streams, and the
 * context's side streams, come from a per-device pool of non-blocking
 * streams that lrx_destroy refills, so creating and destroying contexts does
 * not create and destroy streams once the pool is warm.  *out is set only on
 * success. */
int lrx_create(lrx_ctx** out, int32_t device, void* hip_stream);

/* Geometry and basis sizes.  tau [natom][3], lattice [3][3] with rows
 * a1, a2, a3; nao/nabf [natom] per-atom NAO and ABF counts (1..32 NAOs,
 * 1..128 ABFs).  Host pointers, copied.  Invalidates earlier tensors. */
int lrx_set_structure(lrx_ctx* ctx, int32_t natom, const double* tau, const double* lattice,
                      const int32_t* nao, const int32_t* nabf);

/* Block tensors and the Gamma-point density matrix D (dense, symmetric,
 * [n_tot][n_tot], n_tot = sum nao, atom blocks in atom order).
 * data_on_device = 0: val/dval/D are host arrays, copied to the device.
 * data_on_device = 1: they are device pointers on the context's device;
 *   they are borrowed, not copied, and must stay valid and unchanged until
 *   the next lrx_set_tensors/lrx_set_structure or lrx_destroy.
 * Keys are always host arrays and are copied.  Validates keys on the host
 * and values on the device (finite, mirror and swap symmetries, D
 * symmetric); returns LRX_EINVAL with a message on the first violation.
 * Per-atom limits (also LRX_EINVAL): the NAOs of an atom's C partners (the
 * atoms it shares a C block with, over all images) sum to at most 508, and
 * its C pairs take at most 64 column chunks of the triple products (a pair
 * of nA nF AO pairs takes ceil(nA nF / w) of them, w = 176 when the atom
 * has at most 80 ABFs, else 128), so an atom has at most 64 C partners.
 * Allocates the lists, folded blocks, norms, masks and gradients for the
 * worst case (nothing screened); the work buffers of a precision (see
 * lrx_stats.work_bytes) are allocated by its first evaluation. */
int lrx_set_tensors(lrx_ctx* ctx, const lrx_blocks* C, const lrx_blocks* V, const double* D,
                    int32_t data_on_device);

/* k-point sampling (Methods: Eq. Eexx with the k-sum definition of the
 * density matrix, and Eq. exx_expand).  A Gamma-centred mesh of
 * nk[0] x nk[1] x nk[2] points (each 1..64) makes the Born-von Karman (BvK)
 * supercell of as many unit cells, and the density matrix of two orbitals
 * depends on the offset of their cells modulo it:
 *   D_{(I,R_I) i, (J,R_J) j} = Dk[r][ao(I) + i][ao(J) + j],
 *   r = r0 + nk0 (r1 + nk1 r2),  r_x = (R_J - R_I)_x mod nk_x,
 * with Dk = Dre + i Dim, each [nk0 nk1 nk2][n_tot][n_tot] of the unit cell
 * set by lrx_set_structure; Dim = NULL for a real D(R) (time-reversal
 * symmetry).  Dk must be Hermitian: Dk[-r] = Dk[r]^H (checked).  C and V
 * are the unit cell's blocks exactly as for lrx_set_tensors (first atom in
 * the home cell, any lattice index R).  lrx_evaluate then returns, per unit
 * cell,
 *   E = - sum C(A,F,R_F) V(A,B,R_B) C(B,G,R_G) Re[D_AB D*_FG + D_AG D*_FB]
 * (D_AB at offset R_B, D_FG at R_B + R_G - R_F, D_AG at R_B + R_G, D_FB at
 * R_B - R_F; no Gamma folding: images fold only modulo the BvK cell), the
 * forces F [natom][3] on the unit cell's atoms (every periodic image moved
 * together, D(R) held fixed) and sigma [3][3] per unit-cell volume.
 * Screening as for lrx_evaluate, with the D pairs decided per cell offset on
 * the modulus |D|; step 2 (theta_cs > 0) is refused.  lrx_keep_masks then
 * reports keepD over the supercell's atoms [natom * cells]^2 (atom (t, i)
 * at t * natom + i).  lrx_evaluate_batch, lrx_evaluate_noalloc, lrx_submit
 * and lrx_hamiltonian refuse such a context.  D(R) is read where it is (the
 * block of two supercell atoms is the block of their cells' offset), so the
 * memory is that of lrx_set_tensors on the supercell's pairs plus D(R)
 * itself.  data_on_device as for lrx_set_tensors: the Dk arrays, like
 * val/dval, are then device pointers, borrowed and not copied, and must stay
 * valid and unchanged until the next set-up or lrx_destroy; host arrays are
 * copied.  Limits: fewer than 1024 k points, at most 16384 atoms in the
 * supercell, fewer than 2^21 NAOs in the unit cell.  A later lrx_set_tensors
 * returns the context to the Gamma point. */
int lrx_set_kpoint_tensors(lrx_ctx* ctx, const int32_t nk[3], const lrx_blocks* C, const lrx_blocks* V,
                           const double* Dre, const double* Dim, int32_t data_on_device);

/* Evaluate E (Ha), F [natom][3] (Ha/Bohr) and sigma [3][3] (Ha/Bohr^3) into
 * host buffers; outputs are written only on success.  Blocks the caller's
 * thread until the result is on the host.  Every step (screening, list
 * masks, image folding, contractions, gradients, force and virial
 * reductions) runs in this library's kernels on the context's stream. */
int lrx_evaluate(lrx_ctx* ctx, const lrx_options* opts, double* E, double* F, double* sigma);

/* Asynchronous form of lrx_evaluate (the same evaluation, Eqs. for E_X, the
 * forces and the stress): queues it on the context's stream and returns at
 * once with *ticket, without waiting for the GPU.  opts->timing must be 0.
 * Several submissions may be outstanding on one context; they run in order,
 * each result going to its own pinned host buffer (owned by the library).
 * Block gradients, masks and stats read after a submission describe the
 * latest submitted evaluation (those calls wait for it).  Errors found while
 * queueing are returned here; the ticket is then not issued. */
int lrx_submit(lrx_ctx* ctx, const lrx_options* opts, int64_t* ticket);

/* Wait for a submitted evaluation and write E, F [natom][3] and sigma [3][3]
 * (host buffers; any may be NULL).  Each ticket is waited for once; an
 * unknown or already-used ticket returns LRX_EINVAL.  Tickets still
 * outstanding at lrx_destroy are waited for and released there. */
int lrx_wait(lrx_ctx* ctx, int64_t ticket, double* E, double* F, double* sigma);

/* Per-block gradients dE/dr_b of the last evaluation, in the caller's block
 * order: gC [C.nblk][3], gV [V.nblk][3] (host buffers; either may be NULL).
 * Screened blocks report 0. */
int lrx_block_gradients(lrx_ctx* ctx, double* gC, double* gV);

/* Screening decisions of the last evaluation (host buffers; keepD
 * [natom][natom] 0/1); any pointer may be NULL.  keepC / keepV: 0/1 per
 * block, or with LRX_SCREEN_PER_TENSOR the bits 1 (value list) and 2
 * (derivative list). */
int lrx_keep_masks(lrx_ctx* ctx, uint8_t* keepC, uint8_t* keepV, uint8_t* keepD);

#define LRX_MAX_ALPHA_TILES 8

typedef struct {
  int64_t kept_c_blocks, kept_v_blocks, alive_c_pairs, alive_v_pairs;
  int64_t alive_triples;        /* (A,F,B) with (A,F) and (A,B) alive      */
  int64_t h_slots;              /* H(B,X) blocks computed                   */
  double flop_alg;              /* algorithmic FLOPs of one evaluation       */
  double flop_triple;           /* ... of the triple-product kernel alone    */
  double flop_triple_group[LRX_MAX_ALPHA_TILES + 1];
                                /* ... of its launch for the atoms A with
                                 * ceil(n_abf(A) / 16) = MT, by MT          */
  double bytes_alg;             /* algorithmic HBM bytes of one evaluation   */
  double device_bytes;          /* device memory held by the context now     */
  double work_bytes[3];         /* device memory of the work buffers of each
                                 * precision (index = lrx_precision): H, Z
                                 * and Y partials, and for FP32/BF16X3 the
                                 * FP32 copies of the folded blocks and D
                                 * (FP32 and BF16X3 share theirs).  Allocated
                                 * by the first evaluation in that precision,
                                 * then held (and counted in device_bytes)
                                 * until new tensors or lrx_destroy.        */
  int32_t work_held[3];         /* 1 if those buffers are allocated          */
  int32_t reserved;
} lrx_stats;

/* Counts of the last evaluation (computed on the host from its masks); before
 * the first evaluation only device_bytes, work_bytes and work_held are set. */
int lrx_get_stats(lrx_ctx* ctx, lrx_stats* out);

/* Stage durations (ms) of the last evaluation run with opts.timing != 0,
 * measured with HIP events on the context's stream.  Writes up to n values
 * into ms and returns the number of stages (LRX_NSTAGES), or a negative code.
 * Stage order: norms, screen, fold, mark, hbuild, triple, zgrad, cgrad,
 * forces. */
#define LRX_NSTAGES 9
int lrx_stage_times(lrx_ctx* ctx, float* ms, int32_t n);
const char* lrx_stage_name(int32_t i);

/* Duration (ms) of each alpha-tile group's triple-product launch in the last
 * timed evaluation, by MT = 0..LRX_MAX_ALPHA_TILES (0 for empty groups),
 * from HIP events recorded around the launch on the stream it runs on (the
 * largest group on the context's stream, the others on side streams, where
 * the time includes waiting for compute units the largest group holds).
 * Writes up to n values; returns LRX_MAX_ALPHA_TILES + 1 or a negative code. */
int lrx_group_times(lrx_ctx* ctx, float* ms, int32_t n);

/* Evaluate several contexts (distinct, all on one device) in one batched
 * pass on the first context's stream.  Per alpha-tile group (the work units
 * of atoms with ceil(n_abf/16) = MT) one triple-product launch serves up to 4
 * structures, their units interleaved as work items; the other kernels run
 * per structure in the same sequence.  The first call for a given list of
 * contexts and options builds a plan; the first plan that meets an alpha
 * group (per precision, per process) times the group's launch shapes (one
 * workgroup per item, or a persistent grid that pulls items through
 * counters) after one eager run, and later plans reuse the choice.  A plan
 * runs eagerly on its first use; its second use captures the whole kernel
 * sequence in a HIP graph, which later calls replay (LRX_BATCH_EAGER keeps
 * it eager).  lrx_evaluate goes through the same plans, with one context.
 * A plan is dropped when one of its contexts gets new tensors, a new
 * structure or is destroyed.
 * Results are written per context: E[i], F + 3*sum_{j<i} natom_j,
 * sigma + 9*i (host buffers); every context's block gradients and masks are
 * then available as after lrx_evaluate.  The contexts must not be used by
 * another thread during the call. */
int lrx_evaluate_batch(lrx_ctx* const* ctxs, int32_t n, const lrx_options* opts, double* E, double* F,
                       double* sigma);

/* Launch shapes of the last plan built with this context first: mode[MT]
 * (0: one workgroup per item, 1: persistent grid) and, for the groups that
 * plan timed, ms[2*MT + m] the best time of shape m (0 if not timed there),
 * for MT = 0..LRX_MAX_ALPHA_TILES (host buffers, either may be NULL).
 * Returns LRX_MAX_ALPHA_TILES + 1. */
int lrx_batch_tuning(const lrx_ctx* ctx, int32_t* mode, float* ms);

/* Image pairs within a cutoff (Methods: the combined index of atom and
 * lattice vector; every two-centre block -- C within the orbital cutoff, V
 * within the Coulomb range -- depends on the displacement
 * r = tau[second] + R.L - tau[first] of its two atoms).  Every key
 * (first, second, R) with |r|^2 < rcut^2 is found on the device, where
 *   R.L = (R_0 a1 + R_1 a2) + R_2 a3,  r = (tau[second] - tau[first]) + R.L,
 *   |r|^2 = (r_x^2 + r_y^2) + r_z^2,
 * each operation rounded to FP64 on its own (no fused multiply-add), so the
 * decision is reproducible; R_i runs over |R_i| <= ceil(rcut / h_i) + 1, h_i
 * the spacing of the lattice planes spanned by the other two vectors.  Keys
 * are written sorted by (first, second, R_0, R_1, R_2); the list is closed
 * under the mirror (second, first, -R) up to the rounding of that formula.
 * tau [natom][3], lattice [3][3] (rows a1..a3), host arrays.  Outputs are
 * host arrays first/second [capacity] and R [capacity][3]; *count receives
 * the number of keys.  Returns LRX_EBUDGET (writing only *count) when
 * capacity is too small, LRX_EINVAL for bad arguments (non-finite
 * positions, a singular lattice, a cutoff more than 62 lattice spacings).
 * Uses device memory of its own for the duration of the call. */
int lrx_enumerate_pairs(int32_t device, int32_t natom, const double* tau, const double* lattice, double rcut,
                        int64_t capacity, int32_t* first, int32_t* second, int32_t* R, int64_t* count);

/* The exact-exchange Hamiltonian (Eq. Exx2): H^X[i][j] = dE/dD[i][j] =
 * -sum_kl (ik|jl) D_kl, the part of the energy's variation that comes from
 * the density matrix, for the tensors of the context and the screening of
 * opts (as lrx_evaluate; a screened D pair is zero in E, so H^X is zero
 * there).  Hx: [n_tot][n_tot] row-major (n_tot = sum of nao), symmetric;
 * a host buffer, or with hx_on_device != 0 a device buffer of the context's
 * device (written on the context's stream; the call returns after it is
 * written).  Hx may be NULL.  *E (optional) receives <H^X, D> / 2, the
 * energy of the same screening (a quadratic form in D).  FP64 only
 * (opts->precision must be LRX_FP64; LRX_EINVAL otherwise).  The first call
 * allocates its work buffers: an adjoint of the H slots and three
 * [n_tot][n_tot] matrices. */
int lrx_hamiltonian(lrx_ctx* ctx, const lrx_options* opts, double* E, double* Hx, int32_t hx_on_device);

/* After lrx_hamiltonian: ms[5] (when that call had opts->timing set; else
 * LRX_ESTATE) the HIP-event times of its stages -- screening with folding,
 * H build, adjoint per H slot, gradient through H, symmetrisation --; flop[4]
 * (optional) the algorithmic FLOPs counted from its lists: total, the slot
 * stage (per triple with value-list C and V pairs: 2 mA mB nA nF once for
 * Vf^T Cf, 2 mB nA nF nB per D-block contraction), the gradient through H,
 * the H build. */
int lrx_hamiltonian_info(lrx_ctx* ctx, float* ms, double* flop);

/* Preparation of C and dC (Eq. C_VA; the gradient after Eq. V_inverse).
 * For every key (A,F,R) of T -- the C keys, A carrying the ABF index of the
 * result -- the LRI coefficients of the AO pair (A a, F f) on the ABFs of A
 * and F solve
 *   M [C^A; C^F] = T,  M = [[V(A,A,0), V(A,F,R)], [V(A,F,R)^T, V(F,F,0)]],
 * and the key's C block is C^A; the on-site key (A,A,0) uses the ABFs of A
 * alone, M = V(A,A,0).  Derivatives with respect to the key's displacement:
 *   M dC = -[[0, dV(A,F,R)], [dV(A,F,R)^T, 0]] [C^A; C^F] + dT,
 * and dC = 0 for the on-site key (its blocks do not move with the atom).
 * T: one block per key, the three-centre integrals (P|phi_A phi_F) with the
 * ABFs of A then those of F, [mA + mF][nA][nF] (on-site [mA][nA][nA]), and
 * d/dr as [3][block] at 3 off, as lrx_blocks.  V: the Coulomb blocks (as for
 * lrx_set_tensors), holding V(A,A,0), V(F,F,0) and V(A,F,R) for every key.
 * Output: Cval [sum over keys of mA nA nF], the keys' blocks in key order,
 * each [mA][nA][nF] (C^{A alpha}_{A a, F f}); Cdval [3][block] per block at
 * 3 x its offset -- the layout lrx_set_tensors takes.  on_device != 0: the
 * values of T and V and both outputs are device pointers of `device` (the
 * keys stay on the host); else host arrays.  *flop (optional): algorithmic
 * FLOPs (n^3 / 3 for the factorisation, 2 n^2 per right-hand side column,
 * 12 mA mF nA nF for the products with dV).  Returns LRX_EINVAL for bad
 * arguments, a missing V block or an M that is not positive definite.  Uses
 * device memory of its own for the duration of the call: a workspace of
 * one slice per CU of the device, 3 n_max^2 + 4 n_max (nA nF)_max doubles
 * each (n_max = the largest mA + mF), and one workgroup per CU that takes
 * the CU's LDS. */
int lrx_prepare_c(int32_t device, int32_t natom, const int32_t* nao, const int32_t* nabf, const lrx_blocks* V,
                  const lrx_blocks* T, int32_t on_device, double* Cval, double* Cdval, double* flop);

/* Size of the fixed device scratch of lrx_evaluate_noalloc (bytes per GPU). */
#define LRX_SCRATCH_BYTES (128ull << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * evaluation as lrx_evaluate (same kernels, same results), but its work
 * buffers (H slots, Z and Y partial sums, and for FP32/BF16X3 the FP32
 * copies of the folded blocks and D) come from a fixed device array of
 * LRX_SCRATCH_BYTES that each GPU holds from the library's load until the
 * process ends, instead of the context's own buffers.  Calls no hipMalloc,
 * hipFree or other allocating routine; kernels run eagerly on the context's
 * stream (no batch plan, no graph).  The context must hold tensors
 * (lrx_set_tensors, which allocates as documented there); inputs and outputs
 * are as for lrx_evaluate; opts->timing must be 0.
 * Returns LRX_EBUDGET, computing nothing, when the structure needs more
 * scratch than LRX_SCRATCH_BYTES (small cells only: lrx_get_stats reports
 * the size as work_bytes).  Every call on one GPU uses that GPU's one array
 * and overwrites what the last call left there, so calls that overlap in
 * time on one GPU (other threads, other contexts or streams) race: the
 * caller must serialise them. */
int lrx_evaluate_noalloc(lrx_ctx* ctx, const lrx_options* opts, double* E, double* F, double* sigma);

/* Message of the last failing call on this context ("" if none). */
const char* lrx_last_error(const lrx_ctx* ctx);

/* Release the context and every device buffer it owns.  NULL is allowed.
 * Device buffers go back to the library's per-device memory cache, which
 * serves later contexts from the memory it has already mapped (memory handed
 * back to the driver has to be cleared before it is mapped again, which
 * holds up the whole device); see lrx_pool_trim. */
void lrx_destroy(lrx_ctx* ctx);

/* Unmap segments of the library's device memory cache that no context uses,
 * largest first, until at most keep_bytes stay mapped, after the device has
 * finished its queued work.  For processes that need the memory for
 * something else (e.g. another allocator).  Returns LRX_OK, or LRX_EINVAL
 * for a device that does not exist. */
int lrx_pool_trim(int32_t device, uint64_t keep_bytes);

#ifdef __cplusplus
}
#endif
#endif /* LRX_H */
