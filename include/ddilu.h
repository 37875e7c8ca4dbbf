/*
 * ddilu: domain-decomposed ILU0 preconditioning on MI355X (gfx950).
 *
 * C ABI of the GPU library.  It follows the problem statement of
 * "Mapping Sparse Triangular Solves to GPUs via Fine-grained Domain
 * Decomposition" (arXiv 2508.04917):
 *   - Section 3, Algorithm 2: geometric-cut partition of an nx*ny*nz grid;
 *   - Section 3.1, Algorithm 3: row permutation and reorder of the matrix;
 *   - Section 3.2: removal of the inter-subdomain couplings;
 *   - Section 4.2.1 / 4.2.2: per-subdomain level sets (the DAG);
 *   - Section 4.3, Algorithm 5: ILU0 and the ILDU0 post-pass;
 *   - Sections 4.2.2, 4.4: the fused lower solve, diagonal scaling and upper
 *     solve, one workgroup per subdomain with the vector held in LDS;
 *   - Section 2, Algorithm 1: preconditioned BiCGSTAB.
 *
 * Conventions for every entry point:
 *   - Matrices are block sparse row (BSR) with square blocks of size bs
 *     (1 or 3), each block stored row-major: brow_ptr int32[n+1],
 *     bcol int32[nnzb], val double[nnzb*bs*bs].  Blocks of a row may come in
 *     any column order.  Cell (block row) g of the grid is
 *     g = i + nx*(j + ny*k).
 *   - "device" pointers are HIP device allocations owned by the caller; the
 *     library never frees them.  "host" pointers are ordinary memory.
 *   - Every device operation is enqueued on the caller's stream
 *     (hip_stream, a hipStream_t passed as void*; NULL = the null stream).
 *     Calls that must look at a result on the host (setup status,
 *     convergence) synchronise that stream; the others do not.
 *   - Return value: DD_OK (0) or a negative dd_status code; a message is
 *     available from dd_last_error(handle) (or dd_last_error(NULL) for
 *     errors raised before a handle exists).
 *   - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef DDILU_H
#define DDILU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd_ctx *dd_handle;

enum dd_status {
    DD_OK = 0,
    DD_EINVAL = -1,      /* bad argument or unsupported input               */
    DD_ENOTDIV = -2,     /* grid not divisible by the subdomain extents     */
    DD_ELDS = -3,        /* subdomain vector does not fit the LDS budget    */
    DD_EZEROPIVOT = -4,  /* singular or ill-conditioned pivot block         */
    DD_EBREAKDOWN = -5,  /* BiCGSTAB breakdown (zero denominator, NaN/Inf)  */
    DD_ENOCONV = -6,     /* BiCGSTAB reached maxit                          */
    DD_EHIP = -7,        /* a HIP runtime call failed                       */
    DD_ENOMEM = -8,      /* device allocation failed                        */
    DD_ESTATE = -9       /* call out of order (e.g. apply before factor)    */
};

enum dd_precision {
    DD_FP64 = 0,  /* factors, LDS vector and trisolve arithmetic in FP64      */
    DD_FP32 = 1,  /* factors, LDS vector and trisolve arithmetic in FP32     */
    DD_MIXED = 2  /* factors stored in FP32 (half the factor bytes), widened
                     exactly on load; LDS vector and arithmetic in FP64      */
    /* In every precision the apply reads r and writes z in FP64, and the
       FP32 factors are the FP64 factors rounded to nearest even.          */
};

/* Partition request.  sx = sy = sz = 0 selects the automatic rule of
 * dd_auto_subdims(); lds_budget_bytes = 0 uses the device's maximum LDS
 * per workgroup; n_cu = 0 uses the device's compute-unit count. */
typedef struct {
    int32_t nx, ny, nz;        /* grid extents in cells (block rows)     */
    int32_t bs;                /* block size: 1 or 3                     */
    int32_t sx, sy, sz;        /* subdomain extents, or 0,0,0 for auto   */
    int32_t n_cu;              /* compute units, or 0                    */
    int64_t lds_budget_bytes;  /* LDS per workgroup, or 0                */
} dd_partition_desc;

/* A matrix graph without geometry (Section 3: labels from a graph
 * partitioner; Section 5.3: parts balanced to one size). */
typedef struct {
    int64_t n;                 /* block rows (graph vertices)             */
    int32_t bs;                /* 1 or 3                                  */
    int32_t part_rows;         /* rows per subdomain S (n % S == 0), or 0:
                                  among the divisors of n whose vector
                                  (S*bs*8 bytes) fits the LDS budget, the
                                  one that leaves each compute unit the
                                  fewest rows, ceil((n/S)/n_cu)*S (the
                                  apply runs one part per CU at a time),
                                  or the largest within 5% of that        */
    int64_t lds_budget_bytes;  /* LDS per workgroup, or 0 (device's)      */
    int32_t n_cu;              /* compute units, or 0 (device's)          */
    int32_t reserved;          /* 0                                       */
} dd_graph_desc;

/* Sizes of a handle's problem and setup products. */
typedef struct {
    int64_t n;                 /* block rows                              */
    int64_t nnzb;              /* blocks of the full reordered matrix A   */
    int64_t nnzb_dropped;      /* blocks of A~ after the drop (0 before
                                  ilu0_factor)                            */
    int64_t nnzb_lower;        /* strictly lower blocks of A~ (L)         */
    int64_t nnzb_upper;        /* strictly upper blocks of A~ (Uhat)      */
    int32_t bs, S, nsub;       /* block size, rows per subdomain, count   */
    int32_t sx, sy, sz;        /* subdomain extents in use                */
    int32_t level_ptr_len[2];  /* entries of level_ptr for L (0), U (1)   */
    int32_t max_levels[2];     /* most levels of any subdomain, L and U   */
    int32_t factored;          /* 1 after a successful ilu0_factor        */
    int32_t precision;         /* dd_precision of dd_trsv_apply           */
    int64_t apply_bytes;       /* algorithmic bytes one dd_trsv_apply moves
                                  (factor blocks + int32 columns, inv_D,
                                  int32 row pointers of L and Uhat, FP64 r
                                  in and z out)                           */
    int64_t lds_bytes;         /* LDS per workgroup used by the apply     */
    int32_t max_row_blocks;    /* most blocks in a row of A               */
    int32_t spmv_layout;       /* layout dd_spmv and bicgstab_solve read A
                                  in: 1 = a sliced ELL copy built by the
                                  partition step (the k-th blocks of each
                                  wavefront's rows stored together, 7
                                  positions per row; one more copy of A's
                                  blocks), 2 = the same with one width
                                  per wavefront's rows, longest row first
                                  (rows of more than 7 blocks), 3 = as 2
                                  with the slices aligned to the parts of
                                  dd_partition_graph, the SpMV run part
                                  by part with the part's x in LDS (scalar
                                  rows, parts of at least 256 rows), 0 = the
                                  CSR arrays (no memory for the copy)     */
    int32_t apply_layout;      /* streams the automatic apply reads: 1 =
                                  slot layout (rows of at most 3 blocks per
                                  triangle), 2 = segmented slot layout
                                  (longer rows split into segments within
                                  one wavefront), 0 = CSR streams only
                                  (rows too long for 8 segments)          */
    int32_t seg_blocks;        /* segmented layout: blocks per segment (2,
                                  or 3 when a lower-sweep row holds more
                                  than 16 blocks or an upper-sweep row more
                                  than 23; then up to 24 and 31); 0 for the
                                  other layouts                           */
} dd_info;

/* Result of bicgstab_solve. */
typedef struct {
    int32_t iters;             /* BiCGSTAB iterations started             */
    int32_t status;            /* DD_OK, DD_EBREAKDOWN or DD_ENOCONV      */
    double rel_res;            /* recurrence ||r||/||b|| at exit          */
    double rel_res_true;       /* ||b - A x||/||b|| recomputed at exit    */
    double solve_seconds;      /* wall time of the solve on the stream    */
    int32_t applies;           /* preconditioner applies that did work    */
    int32_t restarts;          /* restarts from the current iterate: when
                                  the recurrence residual meets rtol but
                                  ||b - A x|| exceeds 2 rtol ||b||, the
                                  solve restarts (r = r^ = p = b - A x), at
                                  most 4 times within maxit iterations    */
    double apply_seconds;      /* summed duration of those applies (HIP
                                  events recorded at the apply kernel's
                                  start and end, or around the launches of
                                  a multi-kernel apply; 0 unless profiling
                                  was switched on with dd_set_profiling)  */
    int32_t fused;             /* 1 when each apply ran in one launch with
                                  the SpMV after it (dd_set_fusion)       */
    int32_t fallback;          /* 1 when a solve with the learned
                                  correction broke down or missed maxit and
                                  the result comes from the rerun with plain
                                  DD-ILU0 (dd_set_lic_fallback): iters,
                                  rel_res, rel_res_true and status are the
                                  rerun's, solve_seconds, applies and
                                  apply_seconds cover both runs           */
} dd_solve_info;

/* Automatic subdomain extents (host only, no device access).
 * Section 4: a subdomain is sized so that its FP64 vector (S*bs*8 bytes)
 * fits in one workgroup's LDS.  Among divisor triples sx|nx, sy|ny, sz|nz
 * fitting lds_budget_bytes, keep those giving at least n_cu subdomains if
 * any do; then take the largest S, then the smallest surface
 * sx*sy + sy*sz + sz*sx, then the largest sz, then the largest sy.
 * out: host int32[3].  Returns DD_ELDS when no box fits. */
int dd_auto_subdims(int32_t nx, int32_t ny, int32_t nz, int32_t bs,
                    int64_t lds_budget_bytes, int32_t n_cu, int32_t *out);

/* Device limits used by the automatic rule: compute units and maximum LDS
 * bytes per workgroup of the current device.  Host pointers. */
int dd_device_caps(int32_t *n_cu, int64_t *lds_per_workgroup);

/* Section 3 (Algorithm 2) and Section 3.1 (Algorithm 3): label every cell
 * with its subdomain, renumber cells subdomain by subdomain (stable in the
 * old index, i.e. local lexicographic order inside each box), and build the
 * reordered matrix P A P^T with each row's blocks sorted by column.  The
 * full reordered matrix is kept for SpMV (Section 3.2), and a second,
 * sliced ELL copy of it is built for the SpMV (dd_info.spmv_layout), so a
 * handle holds A's blocks twice (the copy pads each wavefront's rows to its
 * longest one).
 * brow_ptr, bcol, val: device, the matrix in grid order, nnzb blocks,
 * at most 64 blocks per row.  The library copies what it needs; the caller
 * may free them after the call returns.
 * out: host, receives a new handle (release with dd_destroy). */
int dd_partition(const dd_partition_desc *desc, const int32_t *brow_ptr,
                 const int32_t *bcol, const double *val, int64_t nnzb,
                 void *hip_stream, dd_handle *out);

/* Like dd_partition for a matrix whose rows carry no grid position: the
 * labels come from a graph partitioner instead of geometric cuts (the paper
 * uses METIS and balances the parts to one size by hand; METIS is not
 * available, so the partitioner here is recursive BFS bisection into parts
 * of exactly S vertices: a segment of k parts splits by a BFS inside it
 * from its smallest vertex, a second BFS from the farthest vertex reached
 * (smallest index on ties), and the order (distance, index), unreached
 * vertices last, giving the first floor(k/2)*S vertices to one half).  The
 * graph is the block pattern (brow_ptr, bcol); it need not be symmetric.
 * The rest (Algorithm 3 renumbering by label, drop, factorisation, apply,
 * solve) is the same as for a geometric partition; dd_get_info reports
 * sx = S, sy = sz = 1.  Arguments, ownership and stream as for
 * dd_partition.  Returns DD_EINVAL (bad arguments, a row of more than 64
 * blocks, a column outside [0, n)), DD_ENOTDIV (n not divisible by
 * part_rows), DD_ELDS, DD_EHIP, DD_ENOMEM. */
int dd_partition_graph(const dd_graph_desc *d, const int32_t *brow_ptr, const int32_t *bcol,
                       const double *val, int64_t nnzb, void *hip_stream, dd_handle *out);

/* Sizes of the handle's products (host struct). */
int dd_get_info(dd_handle h, dd_info *info);

/* Copies of the partition (device int32[n] each, any may be NULL):
 * part_id in grid order, new2old[i] = grid cell of reordered row i,
 * old2new[g] = reordered row of grid cell g. */
int dd_get_partition(dd_handle h, int32_t *part_id, int32_t *new2old,
                     int32_t *old2new, void *hip_stream);

/* Copy of the reordered full matrix (device; ptr int32[n+1], col
 * int32[nnzb], val double[nnzb*bs*bs]; any may be NULL). */
int dd_get_reordered(dd_handle h, int32_t *ptr, int32_t *col, double *val,
                     void *hip_stream);

/* Section 3.2 drop, Section 4.2.1 level sets, Section 4.3 block ILU0
 * (IKJ order, level-scheduled inside each subdomain) and ILDU0 post-pass;
 * then packs the factors in the streaming layout of the apply.
 * precision: dd_precision the apply will use (the FP64 factors are always
 * kept, for dd_get_factors and for switching precision).  Synchronises the stream; returns
 * DD_EZEROPIVOT if a pivot block is singular or has 1-norm condition
 * number above 1e14 (the message names the block row). */
int ilu0_factor(dd_handle h, int32_t precision, void *hip_stream);

/* Numeric refactorisation on the handle's pattern (Section 5.3: the setup
 * is amortised over solves on one sparsity pattern).  val: device
 * double[nnzb*bs*bs], new values of the matrix given to dd_partition (or
 * dd_partition_graph), in that call's block order and pattern.  Reuses the
 * partition, the reorder, the dropped pattern and the level sets; recomputes
 * the reordered values (and the SpMV's sliced ELL copy), block ILU0 and the
 * ILDU0 streams (and their FP32 copies if they exist), giving the factors a
 * fresh dd_partition + ilu0_factor on the new values gives.  The learned
 * correction and the global ILU0 depend on the values: they are switched off
 * and need lic_setup (+ lic_set_params) or dd_global_factor again.
 * Synchronises the stream; DD_ESTATE before a successful ilu0_factor,
 * DD_EZEROPIVOT as for ilu0_factor (the handle then stays unfactored until
 * a later ilu0_refactor or ilu0_factor succeeds). */
int ilu0_refactor(dd_handle h, const double *val, void *hip_stream);

/* Choose the apply precision after factoring (DD_FP32 and DD_MIXED build
 * the FP32 factor copies on first use). */
int dd_set_precision(dd_handle h, int32_t precision, void *hip_stream);

/* Level sets (Section 4.2.2 explicit DAG).  which = 0: lower factor, 1:
 * upper factor.  Device buffers: nlev int32[nsub] levels per subdomain;
 * level_ptr int32[level_ptr_len[which]] holding nlev[s]+1 offsets per
 * subdomain (relative to the subdomain's first row), concatenated over
 * subdomains; level_rows int32[n]: per subdomain, its S local row indices
 * grouped by level, ascending within a level.  Any pointer may be NULL. */
int dd_get_levels(dd_handle h, int32_t which, int32_t *nlev, int32_t *level_ptr,
                  int32_t *level_rows, void *hip_stream);

/* The dropped pattern A~ and its ILDU0 factors in one array (device):
 * ptr int32[n+1], col int32[nnzb_dropped]; f double[nnzb_dropped*bs*bs]
 * holds L in the strictly lower blocks, inv_D = U_II^{-1} in the diagonal
 * blocks and Uhat = inv_D U in the strictly upper blocks.  Any may be NULL. */
int dd_get_factors(dd_handle h, int32_t *ptr, int32_t *col, double *f,
                   void *hip_stream);

/* Sections 4.2.2 and 4.4: z = M_DD^{-1} r with M_DD = L D Uhat of A~, one
 * workgroup per subdomain, the subdomain's vector resident in LDS:
 * forward y_I = r_I - sum_{J<I} L_IJ y_J, then
 * z_I = inv_D_I y_I - sum_{K>I} Uhat_IK z_K (the scaling is fused into the
 * upper sweep).  r, z: device double[n*bs] in REORDERED order; r != z;
 * 8-byte alignment suffices (subdomain slices that start on a 16-byte
 * boundary move as 16-byte pairs, others value by value; the result is the
 * same).  With a learned correction set (lic_set_params), r is first
 * replaced by r + C r, C the per-face interface coupling.  Does not
 * synchronise. */
int dd_trsv_apply(dd_handle h, const double *r, double *z, void *hip_stream);

/* y = A x with the full reordered matrix (device double[n*bs], reordered
 * order, x != y).  Does not synchronise. */
int dd_spmv(dd_handle h, const double *x, double *y, void *hip_stream);

/* Section 2, Algorithm 1 with K1 = I, K2 = M_DD (right preconditioning):
 * solves A x = b to ||r||/||b|| <= rtol on the recurrence residual (an exit
 * after the half step when ||s||/||b|| <= rtol), at most maxit iterations.
 * b, x: device double[n*bs] in GRID order; x holds the initial guess on
 * entry and the solution on exit.  Krylov vectors, dot products and the
 * stopping test are FP64 whatever the apply precision.  A solve whose
 * true residual misses 2*rtol when the recurrence converges restarts from
 * its current iterate (dd_solve_info.restarts); DD_OK therefore implies
 * ||b - A x|| <= 2 rtol ||b||.  Synchronises.
 * info: host, may be NULL.  Returns DD_OK, DD_EBREAKDOWN or DD_ENOCONV (x
 * then holds the last iterate). */
int bicgstab_solve(dd_handle h, const double *b, double *x, double rtol,
                   int32_t maxit, void *hip_stream, dd_solve_info *info);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): bicgstab_solve with the same arguments,
 * kernels and results, whose Krylov workspace (the vectors, the partial
 * sums of the dot products and the device scalars) lives in a fixed array
 * of the library instead of buffers the handle allocates.  The array holds
 * 128 MiB on each device the library is loaded on, until the process ends;
 * it fits 11 * n * bs FP64 values plus the partial sums, about 1.5 million
 * values of n * bs (a 64^3 grid of 3x3 blocks uses 69 MB), and a larger
 * problem returns DD_EINVAL without running.  The call allocates nothing:
 * the handle must already hold what the solve reads (partition, factors in
 * the chosen precision, learned coefficients; apply variant 7 additionally
 * needs one earlier dd_trsv_apply or bicgstab_solve, else DD_ESTATE).
 * Differences from bicgstab_solve: the apply + SpMV fusion (dd_set_fusion)
 * and per-apply profiling are not used (applies and apply_seconds report
 * 0), and solve_seconds is host wall time from the moment the stream is
 * idle to the end of the call.  Every call on one device shares that
 * device's array (its contents are rewritten by each call before they are
 * read): calls that overlap on one device, from several threads or
 * streams, race and give wrong results; serialise them. */
int bicgstab_solve_noalloc(dd_handle h, const double *b, double *x, double rtol,
                           int32_t maxit, void *hip_stream, dd_solve_info *info);

/* Choose the kernel dd_trsv_apply (and bicgstab_solve) uses; all compute the
 * same z up to rounding order.  0 = automatic (3 where the handle's shape
 * allows it, else 1), 1 = plain level loop (a row's blocks loaded four at a
 * time), 2 = level loop in workgroup-pass chunks with the next chunk's
 * blocks prefetched into registers, 3 = fixed per-row block slots so that
 * no load depends on another and later levels' loads are issued while a
 * level computes (rows of at most 3 off-diagonal blocks per sweep, levels no
 * wider than one pass).  A variant the shape does not allow falls back to 1.
 *
 * 4-8 are ablations of the plain level loop (1), each changing one thing,
 * after the kernel variants of Section 5.2 (Tables 3-4): 4 = lower sweep
 * with the diagonal scaling and upper sweep as two kernels (split ILD_U0
 * against fused ILDU0), 5 = the subdomain's vector in global memory instead
 * of LDS, 6 = vertex-centric (one thread per block row), 7 = ILU0 form of
 * the upper sweep (unscaled U, each row's sum multiplied by inv(U_II)),
 * 8 = synchronisation-free sweeps with per-row flags in LDS (Algorithm 4).
 * They run with DD_FP64 and without the learned correction only: the apply
 * and the solve return DD_EINVAL otherwise (also for 8 when the vector and
 * one flag byte per row exceed 160 KB of LDS).  Returns DD_EINVAL for
 * values outside 0..8. */
int dd_set_apply_variant(dd_handle h, int32_t variant);

/* Switch per-apply timing inside bicgstab_solve on (1) or off (0): a HIP
 * event pair times every preconditioner apply (a slot-layout apply records
 * it at its kernel's own start and end through hipExtLaunchKernel; other
 * variants on the solve's stream around their launches) and the summed
 * durations are reported in dd_solve_info.apply_seconds. */
int dd_set_profiling(dd_handle h, int32_t on);

/* Run each preconditioner apply of bicgstab_solve and the SpMV that
 * follows it in Algorithm 1 (v = A M^{-1} p, t = A M^{-1} s, with their dot
 * products) as one launch (on = 1) or as two (on = 0, the default).  The
 * fused launch has one workgroup per subdomain for the apply and one per
 * subdomain for that subdomain's rows of the product; a product workgroup
 * starts once the subdomains its rows read have been applied (per-subdomain
 * completion flags in device memory, waits bounded), so the product fills
 * the compute units the apply's last partial round leaves idle.  It is used
 * where the apply runs the slot kernel (variant 0 or 3 with a shape that
 * allows it), without per-apply profiling and with the DD preconditioner;
 * otherwise the solve uses two launches.  The result is the same up to the
 * order in which the dot products' partial sums are grouped.
 * dd_solve_info.fused reports which was used.  Off by default: every
 * workgroup of the launch reserves the apply's LDS, so the product runs at
 * one workgroup per CU, and at 160^3 (640 subdomains) a fused iteration
 * measured 8% slower than two launches. */
int dd_set_fusion(dd_handle h, int32_t on);

/* Fallback of a learned solve (on = 1, the default; 0 = off).  When the
 * learned interface correction is on (lic_set_params / lic_set_coeffs) and
 * bicgstab_solve with it ends in DD_EBREAKDOWN or DD_ENOCONV, the solve is
 * repeated from the caller's initial guess with the correction off (plain
 * DD-ILU0, which the correction is meant to improve on), and
 * dd_solve_info.fallback is set.  The correction stays on for later calls.
 * The initial guess is kept in the handle's Krylov workspace meanwhile. */
int dd_set_lic_fallback(dd_handle h, int32_t on);

/* Record the residual history of later bicgstab_solve calls on h: entry j
 * of hist (device double[len]) receives ||r_j||/||b|| after iteration j
 * (entry 0 the initial residual; after a half-step exit, ||s||/||b||).
 * Entries past the last iteration are left untouched.  hist = NULL stops
 * recording. */
int dd_set_residual_history(dd_handle h, double *hist, int32_t len);

/* ---------------------------------------------------------------------
 * Global (undecomposed) ILU0 of the full reordered matrix: what the
 * decomposition approximates (Section 4, the rocSPARSE ILU0 the paper
 * compares with, here as our own level-scheduled kernels: one launch per
 * level over the whole matrix, vector in global memory).
 * --------------------------------------------------------------------- */

/* Level sets, block ILU0 and ILDU0 form of the full reordered matrix (no
 * drop).  Synchronises; DD_EZEROPIVOT on a singular pivot block. */
int dd_global_factor(dd_handle h, void *hip_stream);

/* z = M_global^{-1} r for nrhs right-hand sides stored one after another
 * (device double[nrhs*n*bs] each, reordered order, r != z). */
int dd_global_apply(dd_handle h, const double *r, double *z, int32_t nrhs,
                    void *hip_stream);

/* Preconditioner of bicgstab_solve: 0 = the domain-decomposed ILU0 apply
 * (default), 1 = the global ILU0 apply (needs dd_global_factor). */
int dd_set_preconditioner(dd_handle h, int32_t kind);

/* ---------------------------------------------------------------------
 * Learned interface correction (an addition to the paper's method; the
 * paper has no learned component).  Faces are the directed cut pairs
 * (I, J): the blocks A_IJ the drop removes, in CSR order of the reordered
 * matrix.  Per face a 27 -> 64 -> 64 -> 9 ReLU MLP (FP32; parameters
 * W1[64][27] b1[64] W2[64][64] b2[64] W3[9][64] b3[9], 6,537 floats)
 * maps x_f = [A_II, A_IJ, A_JJ] / sigma_f (blocks row-major,
 * sigma_f = sqrt(|tr A_II| |tr A_JJ|) / 3) to C_f (3x3, row-major), and
 * dd_trsv_apply / bicgstab_solve use z = M_DD^{-1} (r + C r) with
 * (C r)_I = sum over faces (I, J) of C_f r_J: a fixed linear operator.
 * Requires 3x3 blocks, rows of at most 3 blocks per triangle and a
 * structurally symmetric pattern (DD_EINVAL otherwise).
 * --------------------------------------------------------------------- */

/* Faces, features and the transposed factor streams of the adjoint apply
 * (after ilu0_factor).  The correction stays off until lic_set_params or
 * lic_set_coeffs. */
int lic_setup(dd_handle h, void *hip_stream);

/* nf: host, number of faces.  fI, fJ (device int32[nf], reordered rows and
 * columns), X (device float[nf*27], features); each may be NULL. */
int lic_get_faces(dd_handle h, int32_t *nf, int32_t *fI, int32_t *fJ, float *X,
                  void *hip_stream);

/* Evaluate the MLP (device float params[6537]) on every face and switch the
 * correction on; params = NULL switches it off (plain DD-ILU0). */
int lic_set_params(dd_handle h, const float *params, void *hip_stream);

/* Set the coefficients directly (device float[nf*9]); NULL switches the
 * correction off. */
int lic_set_coeffs(dd_handle h, const float *C, void *hip_stream);

/* Copy the current coefficients (device float[nf*9]). */
int lic_get_coeffs(dd_handle h, float *C, void *hip_stream);

/* a = M_DD^{-T} g (transposed factors, FP64; device double[n*3],
 * reordered order, g != a).  Needs lic_setup. */
int dd_apply_adjoint(dd_handle h, const double *g, double *a, void *hip_stream);

/* Regression targets for nq probe vectors R (device double[nq*n*3]):
 * Zs = M_global^{-1} r_q and den_q = ||M_DD^{-1} r_q - Zs_q||^2 (device
 * double[nq*n*3] and double[nq]).  Needs dd_global_factor and lic_setup. */
int lic_targets(dd_handle h, int32_t nq, const double *R, double *Zs, double *den,
                void *hip_stream);

/* Loss and gradient of one problem:
 * loss += mean_q ||z_q - Zs_q||^2 / den_q with z_q = M_DD^{-1}(r_q + C r_q),
 * C from params; grad (device float[6537]) = (accumulate ? grad : 0) +
 * d loss / d params, through g_q = 2 (z_q - Zs_q) / (nq den_q),
 * a_q = M_DD^{-T} g_q, dC_f = sum_q a_q[I] r_q[J]^T and backpropagation.
 * loss: device double[1]. */
int lic_loss_grad(dd_handle h, const float *params, int32_t nq, const double *R,
                  const double *Zs, const double *den, double *loss, float *grad,
                  int32_t accumulate, void *hip_stream);

/* One Adam step (Kingma & Ba) on nparam device floats, step number t >= 1. */
int lic_adam(float *params, const float *grad, float *m, float *v, int32_t nparam,
             int32_t t, float lr, float b1, float b2, float eps, void *hip_stream);

/* Training loop: for every epoch, one lic_loss_grad + Adam step (lr,
 * beta = 0.9/0.999, eps = 1e-8) per problem, problems visited in the order
 * order[epoch*nprob + k] (host int32).  hs, R, Zs, den: host arrays of nprob
 * handles / device pointers (each problem's nq probes, targets and
 * denominators).  params, m, v: device float[6537], updated in place.
 * step0: Adam steps already taken with this m, v (0 for a fresh start), so
 * that a run split over several calls keeps its bias correction.
 * loss_hist: host double[epochs] (mean loss per epoch), may be NULL. */
int lic_train(dd_handle *hs, int32_t nprob, const double *const *R,
              const double *const *Zs, const double *const *den, int32_t nq,
              float *params, float *m, float *v, int32_t epochs,
              const int32_t *order, float lr, int32_t step0, double *loss_hist,
              void *hip_stream);

/* Message of the last failed call on h (or of the last failure before a
 * handle existed when h is NULL).  Owned by the library. */
const char *dd_last_error(dd_handle h);

/* Releases every device buffer of the handle. */
void dd_destroy(dd_handle h);

#ifdef __cplusplus
}
#endif

#endif /* DDILU_H */
