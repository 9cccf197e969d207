/*
 * bsdmrg -- block-sparse two-site DMRG effective-Hamiltonian engine for
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Levy, Solomonik, Clark, "Distributed-Memory DMRG via Sparse and
 * Dense Parallel Tensor Contractions".  The library applies the two-site form
 * of the implicit projected Hamiltonian of Sec. II-C (environments, MPO
 * sites, Fig. 1d) to tensors stored as lists of quantum-number blocks
 * (Sec. II-D; the "list" format of Sec. IV-A), finds its lowest eigenpair
 * with the Davidson routine of Alg. 1, splits the two-site tensor with a
 * truncated per-charge SVD (Sec. II-C, Sec. IV-A) and extends environments.
 *
 * Conventions shared by every call
 * --------------------------------
 * Leg: sectors with integer charge tuples (1 component for U(1), 2 for
 *   U(1)xU(1)), strictly ascending in lexicographic order, each of dimension
 *   >= 1.  The charge of a bond is the total charge to its left.
 * Tensor: one sign per leg; a block (tuple of sector indices) is allowed iff
 *   sum_i sign_i * charge_i == 0 componentwise.  Signs used here:
 *     psi / out / theta (a, s1, s2, c)  (+1, +1, +1, -1)
 *     L environment     (a', w, a)      (-1, +1, +1)   bra, channel, ket
 *     R environment     (c', w, c)      (-1, +1, +1)   bra, channel, ket
 *     MPO site W        (w, s', s, w')  (+1, +1, -1, -1) bra before ket
 *     MPS site          (a, s, b)       (+1, +1, -1)
 * Canonical layout (byte-exact contract): the allowed blocks in
 *   lexicographic order of their sector-index tuples; each block dense and
 *   row-major over its legs; offsets[0] = 0,
 *   offsets[b+1] = offsets[b] + round_up(size_b, 32) elements; padding is 0.
 * Physical legs of bsdmrg_plan and bsdmrg_env_plan must have sectors of
 *   dimension 1 (spin-1/2, electrons); bsdmrg_merge_plan and bsdmrg_truncate
 *   take physical sectors of any dimension up to 64 (e.g. the fused (s', s)
 *   leg of an MPO site compressed as a chain).
 * Memory: every device buffer (operands, outputs, workspace) is allocated and
 *   owned by the caller; the library owns only plan tables, which
 *   bsdmrg_plan_destroy frees.  Device pointers are FP64 in canonical layout.
 * Batches: a plan over n_probs problems addresses concatenated operand
 *   buffers; bsdmrg_plan_offsets gives each problem's element offsets.
 * Errors: every call returns a status; no exception crosses the ABI;
 *   bsdmrg_last_error() gives a thread-local message for the last failure.
 * Streams and threads: work is enqueued on the given stream (0 = default).
 *   Calls are asynchronous unless stated.  A plan or op may be used from
 *   several threads and streams at once if each call has its own workspace
 *   and outputs: its tables are fixed at creation except for the parts built
 *   on first use (the adjoint tables of bsdmrg_heff_backward, bsdmrg_heff_energy
 *   and bsdmrg_env_backward, and the captured graphs of bsdmrg_eigensolve),
 *   which are built, looked up and launched under a lock held by the plan or
 *   op.  bsdmrg_plan_set_tiles and bsdmrg_plan_autotune change the plan and
 *   must not overlap any other call on it; bsdmrg_heff_apply_noalloc shares
 *   one scratch array per GPU (see there).
 */
#ifndef BSDMRG_H
#define BSDMRG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bsdmrg_status;
#define BSDMRG_OK 0
#define BSDMRG_EINVAL 1    /* bad pointer, size, option or shape            */
#define BSDMRG_EQN 2       /* unsorted leg, charge rule violated            */
#define BSDMRG_ENOMEM 3    /* host or device allocation failed              */
#define BSDMRG_EHIP 4      /* HIP runtime error (text in last_error)        */
#define BSDMRG_ESOLVER 5   /* eigensolver or SVD failure                    */
#define BSDMRG_ECAPACITY 6 /* caller buffer too small; required size returned */

#define BSDMRG_F64 0        /* all arithmetic in FP64 (MFMA f64)             */
#define BSDMRG_F32 1        /* block GEMMs in FP32 MFMA, FP32 intermediates  */
#define BSDMRG_F32_REFINE 2 /* eigensolve: FP32 products then FP64 refinement */

#define BSDMRG_PLAN_HOST_ONLY 1 /* plan flag: build tables, no device upload */

typedef struct {
  int32_t n_sectors;
  int32_t n_charges;      /* components per charge (1 or 2)                 */
  const int32_t* charges; /* [n_sectors * n_charges], host memory           */
  const int64_t* dims;    /* [n_sectors], host memory                       */
} bsdmrg_leg;

/* Canonical block table of a tensor (pure host; defined in the header
 * comment).  legs[order], signs[order].  On success *n_blocks is set,
 * block_sectors[n_blocks * order] and offsets[n_blocks + 1] are written.
 * If capacity < n_blocks returns BSDMRG_ECAPACITY with *n_blocks set and the
 * arrays untouched.  Errors: EINVAL (null pointers, order < 1 or > 8),
 * EQN (leg not strictly ascending or a dimension < 1). */
bsdmrg_status bsdmrg_layout(const bsdmrg_leg* legs, int32_t order, const int32_t* signs,
                            int64_t* n_blocks, int32_t* block_sectors, int64_t* offsets,
                            int64_t capacity);

/* One isolated two-site problem (Sec. II-C, Fig. 1c-d):
 *   out(a',s1',s2',c') = sum L(a',w,a) W1(w,s1',s1,w') W2(w',s2',s2,w'')
 *                            R(c',w'',c) psi(a,s1,s2,c)
 * L has legs (a, wl, a), W1 (wl, s1, s1, wm), W2 (wm, s2, s2, wr),
 * R (c, wr, c), psi (a, s1, s2, c).  w1_host / w2_host hold the MPO sites in
 * canonical layout (host memory, read during bsdmrg_plan only): entries that
 * are zero there are structural zeros of the plan, and W blocks that are
 * entirely zero are absent.  Values passed later on the device must keep
 * that pattern. */
typedef struct {
  bsdmrg_leg a, s1, s2, c;
  bsdmrg_leg wl, wm, wr;
  const double* w1_host;
  const double* w2_host;
} bsdmrg_problem;

typedef struct bsdmrg_plan_s* bsdmrg_plan_t;

/* Build the contraction plan (Alg. 2 generalised to the four-operand
 * product): block pairs of every stage, GEMM task and tile tables ordered
 * longest first, MPO-mixing term lists, useful-flop counts, and (unless
 * flags has BSDMRG_PLAN_HOST_ONLY) their device copies.  n_probs >= 1
 * problems are planned as one batch: every stage of all problems runs in one
 * launch.  Errors: EINVAL, EQN, ENOMEM, EHIP. */
bsdmrg_status bsdmrg_plan(const bsdmrg_problem* probs, int32_t n_probs, int32_t flags,
                          bsdmrg_plan_t* out);

typedef struct {
  int64_t n_probs;
  int64_t psi_elems;   /* total elements of the concatenated psi buffers   */
  int64_t L_elems, R_elems, W1_elems, W2_elems;
  int64_t t1_elems, t2_elems;           /* intermediates of one product    */
  int64_t apply_workspace_bytes;        /* workspace of bsdmrg_heff_apply  */
  int64_t backward_workspace_bytes;     /* workspace of bsdmrg_heff_backward once its
                                           tables exist (0 before; see
                                           bsdmrg_heff_backward_workspace) */
  double flops_s1, flops_s2, flops_s3;  /* per product, all problems       */
  int64_t n_s1_tasks, n_s3_tasks, n_s1_tiles, n_s3_tiles;
  int64_t n_mix_terms, n_coefs;
  int64_t s1_big_min, s3_big_min;       /* launch form of the stage: 0 = persistent,
                                           else one workgroup per tile, tasks with
                                           M and N >= this in 128 x 128 tiles, the
                                           others 64 x 64 (2^30: 64 x 64 only) */
  int64_t s3_split_k;                   /* S3 split-K width chosen by the plan: tasks
                                           whose K-list is longer are cut into pieces
                                           of at most this width and summed in a fixed
                                           order (0: no task is split).  The widest of
                                           none, 4096, 2048, 1024 that leaves at least
                                           3072 S3 tiles of 64 x 64, else 512. */
} bsdmrg_plan_info;

bsdmrg_status bsdmrg_plan_query(bsdmrg_plan_t plan, bsdmrg_plan_info* info);

/* Element offsets of problem p inside the concatenated buffers:
 * offs[0..4] = psi, L, R, W1, W2. */
bsdmrg_status bsdmrg_plan_offsets(bsdmrg_plan_t plan, int32_t p, int64_t* offs);

/* Copy the S1 / S3 GEMM task tables of problem-batch order to the host (for
 * tests): per task {M, N, K_total, n_segments}; capacity in tasks. */
bsdmrg_status bsdmrg_plan_tasks(bsdmrg_plan_t plan, int32_t stage, int64_t* tasks4,
                                int64_t capacity, int64_t* n_tasks);

bsdmrg_status bsdmrg_plan_destroy(bsdmrg_plan_t plan);

/* out = H_eff psi for every problem of the plan (Sec. II-C two-site form).
 * precision BSDMRG_F64 or BSDMRG_F32 (GEMM stages in FP32 MFMA with FP32
 * accumulation; psi, out and operands stay FP64 in memory).  Device
 * pointers: L, W1, W2, R, psi [input], out [output, same layout as psi; the
 * padding of out is not written], workspace [apply_workspace_bytes].
 * out must not alias psi.  Errors: EINVAL, EHIP. */
bsdmrg_status bsdmrg_heff_apply(bsdmrg_plan_t plan, int32_t precision, const double* L,
                                const double* W1, const double* W2, const double* R,
                                const double* psi, double* out, void* workspace,
                                int64_t workspace_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (work captured into a
 * graph, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as bsdmrg_heff_apply, same arguments and results (bit for bit),
 * without a workspace argument.  Its workspace is a library-owned array of
 * BSDMRG_NOALLOC_SCRATCH_BYTES in device memory, one per GPU, created when
 * the library's code is loaded on that GPU and held until the process ends;
 * the call itself allocates nothing (no hipMalloc, no host-side library
 * allocation of device memory).  Plans whose product needs more scratch in
 * the requested precision (FP64: T1 and T2 in FP64 plus the split-K pieces;
 * FP32: T1 and T2 in FP32, the pieces and FP32 copies of L and R; at most
 * apply_workspace_bytes) are rejected with EINVAL before any work is
 * enqueued; the m = 1024, k = 14 bond needs 144 MB in FP64.  Every call on a
 * GPU uses that GPU's one array: calls whose work overlaps on one GPU (two
 * streams, two threads, or a captured graph replayed concurrently with
 * another call) race and give wrong results; order them on one stream.
 * Nothing in the array needs to start at zero.  Errors: EINVAL, EHIP. */
#define BSDMRG_NOALLOC_SCRATCH_BYTES (160ll << 20)
bsdmrg_status bsdmrg_heff_apply_noalloc(bsdmrg_plan_t plan, int32_t precision, const double* L,
                                        const double* W1, const double* W2, const double* R,
                                        const double* psi, double* out, hipStream_t stream);

/* Davidson options (Alg. 1; readings of the silent points in the docs of
 * bsdmrg_eigensolve). */
typedef struct {
  int32_t max_iter;        /* products of the first phase (the FP64 phase, or
                              the FP32 phase of BSDMRG_F32_REFINE), 1..4096;
                              without thick restart at most 64 (the basis)   */
  int32_t precision;       /* BSDMRG_F64 or BSDMRG_F32_REFINE               */
  int32_t refine_max_iter; /* FP64 products of the refinement phase (>= 1;
                              it starts with the products of the 1 or 2
                              vectors kept from the FP32 phase)              */
  int32_t fixed_iters;     /* 1: exactly the budgeted products, no host sync */
  int32_t use_graph;       /* 1 with fixed_iters: replay a captured hipGraph */
  int32_t restart_keep;    /* thick restart: 0 = none (a phase ends when its
                              basis is full), 1 = keep the lowest Ritz vector
                              and the previous one (orthogonalised)          */
  uint64_t seed;           /* restart stream seed                            */
  double tol;              /* stop when ||q||_2 <= tol (FP64 phase)          */
  double tol_f32;          /* FP32 phase stops at ||q||_2 <= tol_f32         */
  double restart_rtol;     /* restart if ||t_after|| < rtol * ||t_before||   */
  int32_t basis;           /* basis size with thick restart (3..64; 0: 64)   */
  int32_t precond;         /* 0: none (Alg. 1); 1: Davidson's diagonal
                              preconditioner (see bsdmrg_eigensolve)        */
  int32_t check_every;     /* tol mode: ||q|| is copied back after every
                              check_every-th product (0 or 1: every product)
                              without waiting, and examined at the next such
                              check; when that lagged value is <= tol, the
                              current ||q|| is read (one host sync) and the
                              phase stops if it is <= tol too (so a phase
                              ends at most 2 check_every products after
                              ||q|| first fell to tol); the end of a phase's
                              budget also reads ||q|| synchronously          */
  int32_t reserved;
} bsdmrg_eig_opts;

typedef struct {
  int32_t iters;      /* FP64 products                                      */
  int32_t iters_f32;  /* FP32 products                                      */
  int32_t restarts;   /* random restarts (failed orthogonalisation)         */
  int32_t converged;
  double residual;    /* final ||q||_2                                       */
  int32_t thick_restarts;  /* basis restarts (thick restart and the FP32 -> FP64 switch) */
  int32_t pad;
} bsdmrg_eig_stats;

/* Diagonal of H_eff for every problem of the plan (Davidson's diagonal
 * preconditioner, see bsdmrg_eigensolve):
 * D[e] = <e|H_eff|e> for every allowed element e of psi, i.e.
 *   D(a,s1,s2,c) = sum L(a,w,a) W1(w,s1,s1,w') W2(w',s2,s2,w'') R(c,w'',c)
 * (only flux-0 channels contribute); D has psi's layout, padding written 0.
 * Device pointers, FP64, asynchronous.  Errors: EINVAL, EHIP. */
bsdmrg_status bsdmrg_heff_diagonal(bsdmrg_plan_t plan, const double* L, const double* W1, const double* W2,
                                   const double* R, double* D, hipStream_t stream);

/* Workspace of bsdmrg_eigensolve for these options. */
bsdmrg_status bsdmrg_eig_workspace(bsdmrg_plan_t plan, const bsdmrg_eig_opts* opts,
                                   int64_t* bytes);

/* Lowest eigenpair of H_eff per problem with the Davidson routine of Alg. 1:
 * the start vector and every new basis vector are normalised; at basis size
 * j the j x j projected matrix m_rc = (v^A_c)^T v_r is diagonalised in FP64
 * (Householder tridiagonalisation, Sturm-count multisection for the lowest
 * eigenvalue, inverse iteration for its vector); x = sum s_c v_c,
 * q = sum s_c v^A_c - lambda x; stop when ||q|| <= tol, when the phase's
 * products are spent, or when the basis spans the whole space (its size
 * equals the number of allowed elements of psi: the Ritz pair is then exact;
 * in a batch the smallest problem sets this cap).  The new direction is
 * t = q (Alg. 1) or, with precond = 1, t = q / max(D - lambda, delta) with
 * D the diagonal of H_eff and delta = 1e-3 max(|lambda|, 1) (a positive
 * preconditioner: the plain D - lambda has near-zero denominators while the
 * Ritz value lies above some diagonal entries).  With restart_keep = 1
 * a full basis (basis vectors) is replaced by x and the previous step's Ritz
 * vector orthogonalised against it twice (or, if less than 1e-8 of it
 * remains, the newest basis vector orthogonalised the same way); their
 * products are the same combinations of the stored products, so the restart
 * costs no product.  t is orthogonalised against the basis by classical
 * Gram-Schmidt, with a second pass only when the first removed more than
 * half of ||t||^2 ("twice is enough").  The product is taken of t after the
 * first pass; the second pass and the normalisation are then applied to t
 * and, H_eff being linear, to its product with the same coefficients, the
 * norm after the second pass being ||t||^2 - ||V^T t||^2 (a second pass
 * that would leave less than 1e-4 of ||t||^2 counts as a breakdown).  If
 * ||t|| drops below restart_rtol
 * times its value before orthogonalisation, t is replaced by a seeded
 * Gaussian vector (SplitMix64 + Box-Muller, key from seed, product index,
 * attempt; at most 3 attempts).  All orthogonalisation, Rayleigh quotients
 * and the energy are FP64.  With BSDMRG_F32_REFINE the products of the first
 * phase run in FP32 (FP32 MFMA, FP32 accumulation) and are kept in FP32
 * (every product of the basis is read back and widened to FP64 for the dot
 * products, the Gram matrix and the Ritz vector); when it ends (||q|| <=
 * tol_f32 or max_iter products) its basis is reduced as by a restart to x
 * and the previous Ritz vector, their products are recomputed in FP64, and
 * the solve goes on with FP64 products until ||q|| <= tol.
 * psi_inout: start vectors in, normalised eigenvectors out (device, FP64).
 * energy[n_probs], stats[n_probs]: host arrays.  A batch (n_probs > 1)
 * requires fixed_iters = 1.  The call synchronises the stream before
 * returning.  Errors: EINVAL, EHIP, ESOLVER. */
bsdmrg_status bsdmrg_eigensolve(bsdmrg_plan_t plan, const double* L, const double* W1,
                                const double* W2, const double* R, double* psi_inout,
                                const bsdmrg_eig_opts* opts, double* energy,
                                bsdmrg_eig_stats* stats, void* workspace,
                                int64_t workspace_bytes, hipStream_t stream);

/* Adjoint of the two-site energy E_p = psi_p^T H_eff,p psi_p of every
 * problem p (real tensors; E is linear in each of L, W1, W2, R):
 * writes g_E[p] * dE_p/dX into problem p's part of every non-NULL output
 * (same layout as X): d_psi = g (H_eff + H_eff^T) psi, d_L, d_W1, d_W2,
 * d_R.  g_E: host array of n_probs cotangents.  Outputs are overwritten, not
 * accumulated; padding is written as 0.  d_W1 / d_W2 cover every element of
 * the W blocks that are non-zero in the w1_host / w2_host given to
 * bsdmrg_plan; the other blocks are written as 0 (plan with the sparsity
 * pattern whose gradient is wanted).  The first call builds and uploads the
 * adjoint tables of the plan.  FP64; every sum runs in a fixed order.
 * Device pointers except g_E; outputs may be NULL and must not alias an
 * input.  workspace: bsdmrg_heff_backward_workspace.  Synchronises the stream.
 * Errors: EINVAL, EHIP. */
/* Builds (on the host, once per plan) and checks the adjoint tables of the
 * plan and returns the workspace bytes of bsdmrg_heff_backward and
 * bsdmrg_heff_energy.  Works on host-only plans.  Errors: EINVAL. */
bsdmrg_status bsdmrg_heff_backward_workspace(bsdmrg_plan_t plan, int64_t* bytes);

bsdmrg_status bsdmrg_heff_backward(bsdmrg_plan_t plan, const double* L, const double* W1,
                                   const double* W2, const double* R, const double* psi,
                                   const double* g_E, double* d_psi, double* d_L, double* d_W1,
                                   double* d_W2, double* d_R, void* workspace,
                                   int64_t workspace_bytes, hipStream_t stream);

/* energy[p] = psi_p^T H_eff,p psi_p (host array of n_probs; FP64 product,
 * per-problem reductions in a fixed order).  workspace:
 * bsdmrg_heff_backward_workspace.  Synchronises the stream.  Errors: EINVAL, EHIP. */
bsdmrg_status bsdmrg_heff_energy(bsdmrg_plan_t plan, const double* L, const double* W1,
                                 const double* W2, const double* R, const double* psi,
                                 double* energy, void* workspace, int64_t workspace_bytes,
                                 hipStream_t stream);

/* ------------------------------------------------------------------------
 * Sweep operations (Sec. II-C: split, environment extension, merge).
 * ------------------------------------------------------------------------ */

typedef struct {
  int32_t direction;   /* 0: sweeping right, A = U, B = S V^T;
                          1: sweeping left,  A = U S, B = V^T                */
  int32_t cutoff_mode; /* 0: discard s < cutoff * ||theta|| ("removes all
                          singular values below" the cutoff, Sec. II-C);
                          1: discard the smallest values whose squares sum
                          to at most cutoff * ||theta||^2                   */
  double cutoff;
  int64_t max_m;       /* keep at most max_m values, largest first          */
  double degen_rtol;   /* a kept value v with v - s_first_dropped <=
                          degen_rtol * v is dropped too (multiplets are
                          never split); if that drops all, the plain cut
                          stays                                             */
} bsdmrg_trunc_opts;

/* Workspace bytes of bsdmrg_truncate for a theta with legs theta_legs[4]
 * = (a, s1, s2, c). */
bsdmrg_status bsdmrg_truncate_workspace(const bsdmrg_leg* theta_legs, int64_t* bytes);

/* Truncated SVD split theta(a,s1,s2,c) = A(a,s1,b) B(b,s2,c) (Sec. II-C,
 * Fig. 1e; wrapped per-charge matrices of Sec. IV-A).  theta is wrapped into
 * one matrix per charge q of the new bond (rows (a, s1) with q_a + q_s1 = q,
 * columns (s2, c) with q_c - q_s2 = q, lexicographic), each decomposed in
 * FP64 on the device (QR with column pivoting cut at the numerical rank, then
 * block one-sided Jacobi on R^T; singular values to ~eps ||theta||, those at
 * the rounding level reported as 0); singular values of all charges are
 * pooled (ties by
 * charge index, then index within the charge) and truncated by the options;
 * in every kept pair the entry of u of largest magnitude (first in row order
 * within 1e-10 relative) is made positive.  Outputs: the new bond leg
 * (new_charges[n * n_charges], new_dims[n], ascending), A and B in canonical
 * layout (device, padding zeroed), the kept singular values in descending
 * order (host), their number and the discarded weight (sum of squares of
 * the dropped values).  If leg_capacity, A_capacity, B_capacity or
 * sv_capacity is too small, returns BSDMRG_ECAPACITY with new_n_sectors,
 * A_elems, B_elems and n_kept set.  Synchronises the stream.
 * Errors: EINVAL (also a charge matrix above 4096 columns), EQN, EHIP,
 * ESOLVER (theta not finite, theta == 0, or a sector's block-Jacobi SVD
 * still rotating after its sweep limit of 60). */
bsdmrg_status bsdmrg_truncate(const bsdmrg_leg* theta_legs, const double* theta,
                              const bsdmrg_trunc_opts* opts, int32_t* new_n_sectors,
                              int32_t* new_charges, int64_t* new_dims, int32_t leg_capacity,
                              double* A, int64_t A_capacity, int64_t* A_elems, double* B,
                              int64_t B_capacity, int64_t* B_elems, double* svals,
                              int64_t sv_capacity, int64_t* n_kept, double* discarded,
                              void* workspace, int64_t workspace_bytes, hipStream_t stream);

typedef struct bsdmrg_op_s* bsdmrg_op_t;

/* Environment extension (Sec. II-C; environments are extended from centre to
 * centre while sweeping), FP64:
 *  side 0 (left):  L'(b',w',b) = sum A(a',s',b') L(a',w,a) W(w,s',s,w') A(a,s,b)
 *     env (x, wl, x), mps A (x, s, y), W (wl, s, s, wr) -> env_out (y, wr, y)
 *  side 1 (right): R'(b',w,b) = sum B(b',s',c') W(w,s',s,w') R(c',w',c) B(b,s,c)
 *     env (x, wr, x), mps B (y, s, x), W (wl, s, s, wr) -> env_out (y, wl, y)
 * x is the old bond, y the new one.  w_host: W in canonical layout (host,
 * read at plan time; its zero entries are structural zeros).  The
 * contraction runs as GEMM, MPO mixing with the entries of W, GEMM.  Every
 * plan (also bsdmrg_plan) checks on the host that all its index tables stay
 * inside the operand buffers and fails with EINVAL otherwise. */
typedef struct {
  bsdmrg_leg x, s, y, wl, wr;
  const double* w_host;
} bsdmrg_env_problem;

bsdmrg_status bsdmrg_env_plan(const bsdmrg_env_problem* p, int32_t side, int32_t flags,
                              bsdmrg_op_t* out);

/* Two-site merge theta(a,s1,s2,c) = sum_b A(a,s1,b) B(b,s2,c) (Sec. II-C).
 * legs[5] = (a, s1, b, s2, c).  flags: BSDMRG_PLAN_HOST_ONLY builds and
 * checks the tables without a device copy (as for bsdmrg_env_plan). */
bsdmrg_status bsdmrg_merge_plan(const bsdmrg_leg* legs, int32_t flags, bsdmrg_op_t* out);

/* Workspace bytes, output elements and flops of an op. */
bsdmrg_status bsdmrg_op_query(bsdmrg_op_t op, int64_t* workspace_bytes, int64_t* out_elems,
                              double* flops);
bsdmrg_status bsdmrg_op_destroy(bsdmrg_op_t op);

/* Run an environment op; env_out must not alias the inputs.  Errors:
 * EINVAL, EHIP. */
bsdmrg_status bsdmrg_env_update(bsdmrg_op_t op, const double* env, const double* mps,
                                const double* W, double* env_out, void* workspace,
                                int64_t workspace_bytes, hipStream_t stream);

/* Adjoint of an environment op with respect to W (the extension is linear
 * in W): for the output cotangent d_out (layout of env_out),
 *   d_W[e] = sum over env_out of d_out * d(env_out)/d(W[e])
 * for every element of every symmetry-allowed W block (also the blocks that
 * are zero in the planned W); padding is written as 0.  Left op:
 * d_W(w,s',s,w') = sum A(a',s',b') L(a',w,a) A(a,s,b) d_out(b',w',b); right
 * op: d_W(w,s',s,w') = sum B(b',s',c') R(c',w',c) B(b,s,c) d_out(b',w,b).
 * The cotangent of env itself is the op of the opposite side (x and y
 * swapped, same site tensor and W) applied to d_out; the site tensor's
 * cotangent is not provided (the MPS is held fixed).  The first call builds
 * the adjoint tables of the op.  Device pointers; FP64; fixed summation
 * order.  Errors: EINVAL, EHIP. */
bsdmrg_status bsdmrg_env_backward_workspace(bsdmrg_op_t op, int64_t* bytes);
bsdmrg_status bsdmrg_env_backward(bsdmrg_op_t op, const double* env, const double* mps,
                                  const double* d_out, double* d_W, void* workspace,
                                  int64_t workspace_bytes, hipStream_t stream);

/* Chain rule for a parameter p of the MPO (e.g. J2 of the J1-J2 model,
 * on which every site tensor depends affinely):
 *   dE/dp = sum_s <dE/dW_s, dW_s/dp>,
 * the inner product of each site's energy gradient (bsdmrg_heff_backward,
 * bsdmrg_env_backward; canonical W layout) with that site's derivative
 * tensor dW_s/dp packed in the same layout by the model builder.
 * dE_dW, dW_dp: host arrays of n_sites device pointers (FP64); n_elems: host
 * array of n_sites element counts (0 allowed).  terms: device, n_sites + 1
 * doubles; receives the per-site inner products and, last, their sum taken
 * in site order (each inner product in a fixed order: repeated calls are
 * bit-identical).  *result (host) receives the sum.  Synchronises the
 * stream.  Errors: EINVAL (NULL argument, n_sites < 1, negative count),
 * EHIP. */
bsdmrg_status bsdmrg_param_derivative(int32_t n_sites, const double* const* dE_dW,
                                      const double* const* dW_dp, const int64_t* n_elems,
                                      double* terms, double* result, hipStream_t stream);

/* Run a merge op (no workspace).  Errors: EINVAL, EHIP. */
bsdmrg_status bsdmrg_merge(bsdmrg_op_t op, const double* A, const double* B, double* theta,
                           hipStream_t stream);

/* ------------------------------------------------------------------------
 * Sparse-dense format (Sec. IV-A): the two-site product with every operand
 * one dense array, the blocks that the charge rules forbid stored as zeros
 * and multiplied like any other entry.  It computes the same product as
 * bsdmrg_heff_apply with all the work the block structure avoids, on the
 * same grouped GEMM kernels; its use is to measure that work (ablation).
 * ------------------------------------------------------------------------ */

/* Plan of the dense product for bond dimensions ma (left) and mc (right),
 * k MPO channels and physical dimension d (1..8): three GEMM stages,
 *   T1(a' w, s1 s2 c) = L(a' w, a) psi(a, s1 s2 c),
 *   T2[a'](s1' s2' w'', c) = WW(s1' s2' w'', w s1 s2) T1[a'](w s1 s2, c)
 *     with WW the two sites contracted over their shared channel,
 *   out(a' s1' s2', c') = sum_{w'' c} T2(a' s1' s2', w'' c) R(c', w'', c).
 * bsdmrg_op_query gives the workspace (the larger of the FP64 and FP32
 * needs), out_elems = ma d^2 mc and the flops of the three stages.  flags:
 * BSDMRG_PLAN_HOST_ONLY as for bsdmrg_plan.  Free with bsdmrg_op_destroy.
 * Errors: EINVAL (a dimension out of range, or an operand of 2 GiB or more),
 * EHIP, ENOMEM. */
bsdmrg_status bsdmrg_dense_plan(int64_t ma, int64_t mc, int32_t k, int32_t d, int32_t flags,
                                bsdmrg_op_t* op);

/* out = H_eff psi in the dense format.  Device operands, FP64, dense
 * row-major: L (ma, k, ma) as (bra, channel, ket), W1 and W2 (k, d, d, k) as
 * (w, s', s, w'), R (mc, k, mc), psi and out (ma, d, d, mc).  precision
 * BSDMRG_F64, or BSDMRG_F32 (FP32 MFMA, FP32 intermediates and FP32 copies
 * of L, R, WW in the workspace; out in FP64).  Every output element is
 * summed in a fixed order.  Errors: EINVAL (wrong op kind, NULL operand,
 * out == psi, workspace too small), EHIP. */
bsdmrg_status bsdmrg_dense_apply(bsdmrg_op_t op, int32_t precision, const double* L, const double* W1,
                                 const double* W2, const double* R, const double* psi, double* out,
                                 void* workspace, int64_t workspace_bytes, hipStream_t stream);

/* Measurement helper: runs each stage of one product `reps` times on
 * `stream`, bracketed by HIP events recorded on that stream, and writes the
 * average duration in milliseconds per launch to ms[5] = {WW coefficients,
 * S1 grouped GEMM, S2 MPO mixing, S3 grouped GEMM (split-K pieces), S3
 * fixed-order sum of the split-K pieces}.  Same arguments and results as
 * bsdmrg_heff_apply (out holds the product afterwards); precision may also
 * be BSDMRG_F32_REFINE: the stages as the FP32 phase of a mixed eigensolve
 * runs them (FP32 products: S3 and its sum write FP32 results into out
 * while they are timed), the product afterwards as with BSDMRG_F32 (the
 * padding of out is then zero).
 * Synchronises the stream.  Errors: EINVAL, EHIP. */
bsdmrg_status bsdmrg_stage_timing(bsdmrg_plan_t plan, int32_t precision, const double* L,
                                  const double* W1, const double* W2, const double* R,
                                  const double* psi, double* out, void* workspace,
                                  int64_t workspace_bytes, int32_t reps, float* ms,
                                  hipStream_t stream);

/* Autotuner of the grouped-GEMM tile shapes (batching form of the hot
 * path: one launch per stage over every block pair of every problem).  For
 * each of the two GEMM stages S1 and S3 it tries the shape classes
 * "64 x 64 tiles only" and "128 x 128 tiles for tasks with M and N >= T"
 * (T = 384, 256, 160, 96) and the persistent launch (big_min 0, see
 * bsdmrg_plan_set_tiles), times `reps` launches of each distinct tile
 * schedule with HIP events on `stream` in the given precision (operands as
 * for bsdmrg_heff_apply; out receives one product), and keeps the fastest
 * (a larger tile must win by 2% to replace a smaller one).  The chosen
 * thresholds are returned in big_min[2] (S1, S3) and in
 * bsdmrg_plan_info; the plan's captured eigensolver graph is dropped.
 * Results are unchanged bit for bit by the choice (the K order of every
 * output element is the same).  Synchronises the stream.  Not thread-safe
 * with other calls on the same plan.  Errors: EINVAL, EHIP. */
bsdmrg_status bsdmrg_plan_autotune(bsdmrg_plan_t plan, int32_t precision, const double* L,
                                   const double* W1, const double* W2, const double* R,
                                   const double* psi, double* out, void* workspace,
                                   int64_t workspace_bytes, int32_t reps, int32_t* big_min,
                                   hipStream_t stream);

/* Install the launch form of the two GEMM stages directly (big_min as
 * returned by bsdmrg_plan_autotune): 0 = persistent launch (64 x 64 tiles
 * dealt on the host, XCD-aware longest first, to one workgroup per resident
 * slot, 128 per XCD; each workgroup fetches the first slice of its next tile
 * while it finishes the current one); 2^30 or more: one workgroup per 64 x 64
 * tile; otherwise one workgroup per tile with 128 x 128 tiles for tasks with
 * M and N >= big_min.  Every form gives the same products bit for bit.  Drops
 * the plan's captured graphs.  No work using the plan may be in flight.
 * Errors: EINVAL, EHIP. */
bsdmrg_status bsdmrg_plan_set_tiles(bsdmrg_plan_t plan, int32_t s1_big_min, int32_t s3_big_min);

const char* bsdmrg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BSDMRG_H */
