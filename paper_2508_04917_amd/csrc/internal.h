// Internal declarations of the ddilu GPU library (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ddilu.h"

namespace ddilu {

constexpr int kMaxRowBlocks = 64;   // blocks per row accepted by the reorder
constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kMaxSlots = 3;        // largest per-row block count of the slot layout

// Streaming layout of one triangular sweep.  Positions are the rows of each
// subdomain in sweep order (level by level, ascending local row inside a
// level); subdomain s owns positions [s*S, (s+1)*S).  Everything a sweep
// reads is laid out in that order so one workgroup streams its factor data
// front to back.
struct Sweep {
    uint16_t *prow = nullptr;   // [n] local row of each position
    int32_t *bptr = nullptr;    // [n+1] first block of each position
    uint16_t *bcol = nullptr;   // [nblk] local column of each block
    double *val64 = nullptr;    // [nblk*bb] L blocks (lower) or Uhat (upper)
    float *val32 = nullptr;     // FP32 copy (built on demand)
    double *d64 = nullptr;      // upper only: inv_D per position [n*bb]
    double *uraw = nullptr;     // upper only, built on demand: U blocks without the inv_D scaling [nblk*bb]
    float *d32 = nullptr;
    int64_t nblk = 0;
    int32_t max_row = 0;        // most blocks of any row in this sweep
    // Slot layout (when every row has at most kMaxSlots blocks): position p
    // owns MB block slots (MB = the handle's slot count; unused slots hold
    // zero blocks) and, in the upper sweep, its inv_D block.  Per position the
    // values are stored as BS runs, run i = row i of every slot block then
    // row i of inv_D, so the BS lanes of a row each read one contiguous run.
    // The address of a block is a function of the position alone, so a sweep
    // can issue its loads without first reading row offsets.
    uint64_t *desc = nullptr;   // [n] local row | column of slot k << 16(k+1); 0xFFFF empty
    double *sval64 = nullptr;   // [n*MB*bb] lower, [n*(MB+1)*bb] upper
    float *sval32 = nullptr;
    int64_t snpos = 0;          // positions of the slot layout (n, or the segmented layout's count)
    // Segmented slot layout (rows of more than kMaxSlots blocks): a row is
    // split into segments at consecutive positions of one wavefront; levels
    // wider than a workgroup pass are cut into chunks.  With MB blocks per
    // segment (dd_ctx::seg): a lower-sweep segment holds MB blocks; in the
    // upper sweep the row's first segment holds MB blocks and inv_D, each
    // continuation MB + 1 blocks, the last one in the inv_D slot.  desc then
    // holds 15-bit fields: local row (a continuation of the upper sweep: the
    // column of its extra block) | continuation flag << 15, columns at
    // 16(k+1) (0x7FFF empty), and, for a row's first segment, its segment
    // count minus one in bits 31, 47 and 63.
    int32_t *gpos = nullptr;    // [nsub+1] first position of each subdomain
    int32_t *gchk = nullptr;    // [nsub+1] first entry of each subdomain's chunk table
    int32_t *chk = nullptr;     // per subdomain: chunk starts (relative; bit 30 = barrier after), end
    int2 *pmap = nullptr;       // [snpos] CSR sweep position (-1 = padding), segment | count << 8
};

constexpr int kSegMax = 8;  // segments of a row in the segmented layout

// Level sets of one factor, per subdomain.
struct Levels {
    int32_t *lev = nullptr;     // [n] level of each row (reordered numbering)
    int32_t *nlev = nullptr;    // [nsub]
    int32_t *off = nullptr;     // [nsub+1] start of each subdomain in ptr
    int32_t *ptr = nullptr;     // [ptr_len] level offsets relative to the subdomain
    int32_t *rows = nullptr;    // [n] local rows grouped by level
    int32_t ptr_len = 0;
    int32_t max_levels = 0;
};

// Learned interface correction state (faces, features, coefficients, and
// the training workspace).
struct Lic {
    int32_t ready = 0, active = 0;
    int32_t nf = 0;               // faces
    int32_t *fptr = nullptr;      // [n+1] faces of each row (CSR order)
    int32_t *fI = nullptr, *fJ = nullptr, *fq = nullptr;  // [nf] row, column, block position in A
    int32_t *diag = nullptr;      // [n] diagonal block position of each row of A
    // the apply's copy of the faces, rank-major per subdomain (first face of
    // every row, then second faces, ...): records, CSR index, coefficients
    int2 *lrec = nullptr;         // [nf] {local row, J}
    int32_t *lperm = nullptr;     // [nf] CSR face index of each rank-major position
    float *Cr = nullptr;          // [nf*9] C in rank-major order
    int32_t *rb = nullptr;        // [nsub*9] faces of ranks < k of subdomain s at rb[9s + k]
    float *X = nullptr;           // [nf*27] features
    float *C = nullptr;           // [nf*9] coefficients
    float *H1 = nullptr, *H2 = nullptr, *G1 = nullptr, *G2 = nullptr, *dC = nullptr;
    double *wpart = nullptr, *rpart = nullptr;
    double *Z = nullptr, *G = nullptr, *A = nullptr;
    int32_t work_q = 0;
    double *adj_val[2] = {nullptr, nullptr};  // transposed slot streams (U^T lower, L^T + inv_D^T upper)
    int32_t adj_ready = 0;                    // adj_val packed from the current factors
};

// Device scalars of one BiCGSTAB run (all FP64 except the control words).
struct KrylovScalars {
    double rho, alpha, omega, beta;
    double bnorm, rnorm, snorm;
    double tol;                  // rtol * ||b||
    int32_t state;               // 0 running, 1 converged, 2 half-step exit pending,
                                 // -5 breakdown, -6 no convergence
    int32_t iters;
    int32_t maxit;
    int32_t half;                // 1 when the solve stopped after a half step
};

}  // namespace ddilu

struct dd_ctx {
    // problem and partition
    int32_t nx = 0, ny = 0, nz = 0, bs = 0;
    int32_t sx = 0, sy = 0, sz = 0;
    int32_t S = 0, nsub = 0;
    int32_t graph = 0;            // labels from the graph partitioner (no geometry: nx = n, sx = S)
    int64_t n = 0, nnzb = 0;
    int32_t *part_id = nullptr, *new2old = nullptr, *old2new = nullptr;
    int32_t *asrc = nullptr;      // [nnzb] input block of each reordered block (for ilu0_refactor)
    int32_t *tsrc = nullptr;      // [nnzt] block of A of each block of the dropped pattern
    // full reordered matrix
    int32_t *aptr = nullptr, *acol = nullptr;
    double *aval = nullptr;
    // dropped pattern and factors
    int64_t nnzt = 0, nlow = 0, nupp = 0;
    int32_t *tptr = nullptr, *tcol = nullptr, *tdiag = nullptr;
    double *lu = nullptr;       // L\U in the dropped pattern
    double *invd = nullptr;     // [n*bb] inv(U_II), reordered row order
    ddilu::Levels lev[2];
    ddilu::Sweep sw[2];
    int32_t factored = 0;
    int32_t patterned = 0;        // drop, levels and streaming layouts built (ilu0_refactor may run)
    int32_t precision = DD_FP64;
    int32_t max_level_width = 0;  // widest level of any subdomain, L or U
    int32_t profile = 0;          // time every apply inside bicgstab_solve
    // events the next apply launch records at its kernel's start and end
    // (set by launch_precond for per-apply timing; tev_used: a slot kernel
    // took them)
    hipEvent_t tev[2] = {nullptr, nullptr};
    int32_t tev_used = 0;
    int32_t slots = 0;            // MB of the slot layout (0: CSR layout only)
    int32_t seg = 0;              // MB of the segmented slot layout (2 or 3; 0: not built)
    int32_t variant = 0;          // apply kernel: 0 auto, 1 simple, 2 pipelined CSR, 3 slots, 4-8 ablations
    double *hist = nullptr;       // optional residual history (device, caller-owned)
    ddilu::Lic lic;
    int32_t pc_kind = 0;          // preconditioner of bicgstab_solve: 0 DD-ILU0, 1 global ILU0
    // global (undecomposed) ILU0 of the full reordered matrix
    int32_t *glev[2] = {nullptr, nullptr};
    int32_t gnlev[2] = {0, 0};
    int32_t *gdiag = nullptr;
    double *glu = nullptr, *ginvd = nullptr, *gf = nullptr;
    int32_t gfactored = 0;
    int32_t hist_len = 0;
    std::vector<hipEvent_t> events;
    // scratch
    int32_t *status = nullptr;  // [4] device status words
    int32_t *scan_tmp = nullptr;
    int64_t scan_tmp_len = 0;
    // Krylov workspace (allocated on first solve)
    double *kv = nullptr;       // kKrylovVectors vectors of n*bs
    double *partials = nullptr; // [8 * spmv_part_stride] per-workgroup partial sums
    int32_t spmv_part_stride = 0;
    int32_t max_row_a = 0;               // most blocks in a row of the full matrix
    int32_t ell_state = 0;               // sliced-ELL copy for the SpMV: 0 not built, 1 ready, -1 not used
    int32_t *ell_col = nullptr;          // [slices][width][rows per wavefront]
    double *ell_val = nullptr;           // the same slots, bs*bs values each
    // per-slice widths (rows of more than kUnroll blocks; null otherwise):
    int32_t *sell_row = nullptr;         // [slices][rows per wavefront] block row, longest first (-1: none)
    int32_t *sell_len = nullptr;         // its length
    int64_t *sell_off = nullptr;         // [slices + 1] first slot run of each slice
    int64_t sell_nslice = 0;             // slices of the copy
    int32_t sell_spp = 0;                // slices per part (part-aligned slices, graphs), 0 otherwise
    int32_t lic_fallback = 1;            // rerun a failed learned solve with plain DD-ILU0
    int32_t fuse = 0;                    // apply + SpMV as one launch inside bicgstab_solve (opt-in)
    int32_t *fdep = nullptr;             // [2 nsub] dependency ranges of the SpMV tiles
    uint32_t *fflag = nullptr;           // [nsub] per-subdomain completion epochs
    unsigned long long *fticket = nullptr;  // workgroup ticket counter
    ddilu::KrylovScalars *ks = nullptr;
    ddilu::KrylovScalars *ks_host = nullptr;  // pinned
    std::vector<void *> allocs;
    std::string err;

    int fail(int code, const char *fmt, ...);
    // hipMalloc of count elements, recorded for dd_destroy
    template <typename T>
    int alloc(T **p, int64_t count) {
        void *q = nullptr;
        const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(DD_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        }
        allocs.push_back(q);
        *p = static_cast<T *>(q);
        return DD_OK;
    }
    ~dd_ctx();
};

namespace ddilu {

// exclusive scan of int32 counts: out[0] = 0, out[i+1] = out[i] + in[i];
// returns the total in *total (synchronises the stream).  tmp: scratch of
// at least scan_tmp_elems(n) int32.
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp,
                          hipStream_t st);

}  // namespace ddilu

// kernel launchers implemented in the .hip files
namespace ddilu {
hipError_t launch_partition(dd_ctx *h, hipStream_t st);
// labels, new2old and old2new of a graph without geometry (recursive BFS
// bisection into parts of h->S vertices); DD_OK or an error code
int graph_partition(dd_ctx *h, const int32_t *ptr, const int32_t *col, hipStream_t st);
hipError_t launch_check_rows(int64_t n, int64_t nnzb, const int32_t *ptr, const int32_t *col, int32_t *status,
                             hipStream_t st);
hipError_t launch_row_len(dd_ctx *h, const int32_t *ptr, int32_t *len, hipStream_t st);
hipError_t launch_reorder_fill(dd_ctx *h, const int32_t *ptr, const int32_t *col,
                               const double *val, int32_t *src, hipStream_t st);
hipError_t launch_drop_count(dd_ctx *h, int32_t *tbeg, int32_t *tlen, hipStream_t st);
hipError_t launch_drop_rows(dd_ctx *h, const int32_t *tbeg, int32_t *tsrc, hipStream_t st);
hipError_t launch_levels(dd_ctx *h, int which, hipStream_t st);
hipError_t launch_plus_one(int64_t m, const int32_t *in, int32_t *out, hipStream_t st);
hipError_t launch_level_lists(dd_ctx *h, int which, hipStream_t st);
hipError_t launch_bilu0(dd_ctx *h, hipStream_t st);
hipError_t launch_pack_count(dd_ctx *h, int which, int32_t *cnt, hipStream_t st);
hipError_t launch_pack_fill(dd_ctx *h, int which, hipStream_t st);
hipError_t launch_pack_unscaled(dd_ctx *h, hipStream_t st);
hipError_t launch_cast32(dd_ctx *h, hipStream_t st);
hipError_t launch_pack_slots(dd_ctx *h, int which, hipStream_t st);
// segmented slot layout: positions and chunk tables (which: 0 lower, 1
// upper; chunk width cw positions, rpw per wavefront), then the values
int build_seg_layout(dd_ctx *h, int which, int mb, int cw, int rpw, hipStream_t st);
hipError_t launch_seg_pack(dd_ctx *h, int which, hipStream_t st);
hipError_t launch_max_count(int64_t n, const int32_t *cnt, int32_t *out, hipStream_t st);
hipError_t launch_export_factors(dd_ctx *h, double *f, hipStream_t st);
// out[k] = val[src[k]] for nblk blocks of bb values
hipError_t launch_gather_blocks(int64_t nblk, int bb, const int32_t *src, const double *val, double *out,
                                hipStream_t st);
// rewrite the sliced ELL copy's values after A's values changed
hipError_t refresh_spmv_layout(dd_ctx *h, hipStream_t st);

hipError_t launch_apply(dd_ctx *h, const double *r, double *z, const int32_t *state,
                        hipStream_t st);
// nrhs applies of right-hand sides stored one after another (n*bs apart):
// one launch (grid.y = right-hand side) where the slot kernel runs, else one
// launch per right-hand side
hipError_t launch_apply_batch(dd_ctx *h, const double *r, double *z, int nrhs, hipStream_t st,
                              const int32_t *state = nullptr);
int apply_lds_bytes(const dd_ctx *h, int precision);
int spin_lds_bytes(const dd_ctx *h);
// 0 if the handle's precision and correction allow apply variant v, else the
// reason (for the ablation variants 4-8: FP64 only, no learned correction)
const char *variant_unsupported(const dd_ctx *h, int v);

// Krylov
hipError_t launch_spmv(dd_ctx *h, const double *x, double *y, hipStream_t st);
// the sliced ELL copy of A for the SpMV (once per handle; synchronises st)
void build_spmv_layout(dd_ctx *h, hipStream_t st);
hipError_t launch_permute(int64_t n, int bs, const int32_t *map, const double *in, double *out,
                          hipStream_t st);
// vectors of n*bs in the Krylov workspace: ten for the recurrence, one to
// keep the initial guess while a learned solve may still fall back
constexpr int kKrylovVectors = 11;
// Device workspace of one solve: the Krylov vectors, the per-workgroup
// partial sums and the device scalars, plus a host copy of the scalars.
// Either the handle's own buffers (allocated on its first solve) or the
// library's fixed array (bicgstab_solve_noalloc).
struct KrylovWork {
    double *kv = nullptr;              // kKrylovVectors vectors of n*bs
    double *partials = nullptr;        // [8 * part_stride] per-workgroup partial sums
    int32_t part_stride = 0;
    KrylovScalars *ks = nullptr;       // device
    KrylovScalars *ks_host = nullptr;  // host (pinned for the handle's workspace)
    // false: create no HIP events (the solve is timed on the host, per-apply
    // profiling is off) and use no buffer outside this workspace (the fused
    // apply + SpMV launch, whose flags the handle allocates, is not used)
    bool handle_owned = true;
};
int bicgstab_run(dd_ctx *h, const KrylovWork &w, const double *b, double *x, double rtol, int32_t maxit,
                 hipStream_t st, dd_solve_info *info);
// the handle's Krylov workspace (allocated on the first call)
int krylov_workspace(dd_ctx *h, KrylovWork *w);
// the workspace in the library's fixed device array: no allocation;
// DD_EINVAL when the problem needs more than that array holds
int noalloc_workspace(dd_ctx *h, KrylovWork *w, KrylovScalars *host);
// bytes of the fixed array (per device)
constexpr int64_t kNoallocBytes = int64_t(128) << 20;

// global ILU0
int global_factor(dd_ctx *h, hipStream_t st);
hipError_t launch_global_apply(dd_ctx *h, const double *r, double *z, int nrhs, hipStream_t st);
hipError_t launch_diag_positions(dd_ctx *h, int32_t *diag, hipStream_t st);

// learned correction
int lic_setup(dd_ctx *h, hipStream_t st);
int lic_coeffs_from_params(dd_ctx *h, const float *params, bool keep_hidden, hipStream_t st);
// refresh the apply's rank-major copy of C after C changed
int lic_publish_coeffs(dd_ctx *h, hipStream_t st);
int lic_loss_grad_run(dd_ctx *h, const float *params, int Q, const double *R, const double *Zs, const double *den,
                      double *loss, float *grad, int accumulate, hipStream_t st);
int lic_targets_run(dd_ctx *h, int Q, const double *R, double *Zs, double *den, hipStream_t st);
hipError_t launch_adam(int np, float *P, const float *G, float *M, float *V, int t, float lr, float b1, float b2,
                       float eps, hipStream_t st);
// nrhs adjoint applies (right-hand sides n*3 apart) in one launch; the
// transposed streams must have been packed (lic_adjoint_streams)
hipError_t launch_apply_adjoint(dd_ctx *h, const double *g, double *a, int nrhs, hipStream_t st);
// pack the transposed factor streams of the adjoint apply (once per factorisation)
int lic_adjoint_streams(dd_ctx *h, hipStream_t st);
// the preconditioner bicgstab_solve uses (DD apply, or the global ILU0 apply)
// ev0/ev1 (optional): timing events around the apply; a slot-layout apply
// records them at its kernel's own start and end (hipExtLaunchKernel), any
// other path on the stream around its launches.
hipError_t launch_precond(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
constexpr int32_t kWaitFailed = -64;  // solve state word after a dependency wait hit its bound
// BiCGSTAB's apply and the SpMV behind it as one launch (mode 0: y = A z with
// the dot w.y; mode 1: the dots y.w and y.y), partials one per subdomain.
// Nonzero when the handle's shape or settings need the separate launches.
int fused_unsupported(const dd_ctx *h);
hipError_t launch_apply_spmv(dd_ctx *h, int mode, const double *r, double *z, double *y, const double *w,
                             double *part, int part_stride, uint32_t epoch, unsigned long long ticket0,
                             int32_t *state, hipStream_t st);
// dep[2k], dep[2k+1]: lowest and highest subdomain read by subdomain k's rows of A
hipError_t launch_dep_range(dd_ctx *h, hipStream_t st);
}  // namespace ddilu
