// C ABI entry points of the ddilu library: handle lifetime, setup
// orchestration and argument checking.  Every numerical step runs in the
// kernels of setup.hip, apply.hip and krylov.hip.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.h"

using namespace ddilu;

static thread_local std::string g_err;

static int set_global_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int dd_ctx::fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    g_err = buf;
    return code;
}

dd_ctx::~dd_ctx() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (void *q : allocs) (void)hipFree(q);
    if (ks_host) (void)hipHostFree(ks_host);
}

static void release(dd_ctx *h, void *q) {
    if (!q) return;
    auto it = std::find(h->allocs.begin(), h->allocs.end(), q);
    if (it != h->allocs.end()) {
        (void)hipFree(q);
        h->allocs.erase(it);
    }
}

#define HCHK(x)                                                                             \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) return h->fail(DD_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)
#define RCHK(x)              \
    do {                     \
        int r_ = (x);        \
        if (r_) return r_;   \
    } while (0)

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- sizing
extern "C" int dd_auto_subdims(int32_t nx, int32_t ny, int32_t nz, int32_t bs, int64_t lds_budget_bytes,
                               int32_t n_cu, int32_t *out) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || (bs != 1 && bs != 3) || !out)
        return set_global_error(DD_EINVAL, "dd_auto_subdims: bad arguments");
    struct Cand {
        int sx, sy, sz;
    };
    std::vector<Cand> all, full;
    for (int sx = 1; sx <= nx; ++sx) {
        if (nx % sx) continue;
        for (int sy = 1; sy <= ny; ++sy) {
            if (ny % sy) continue;
            for (int sz = 1; sz <= nz; ++sz) {
                if (nz % sz) continue;
                const int64_t S = (int64_t)sx * sy * sz;
                if (S * bs * 8 > lds_budget_bytes) continue;
                all.push_back({sx, sy, sz});
                const int64_t nsub = (int64_t)(nx / sx) * (ny / sy) * (nz / sz);
                if (nsub >= n_cu) full.push_back({sx, sy, sz});
            }
        }
    }
    if (all.empty()) return set_global_error(DD_ELDS, "no subdomain box fits %lld bytes of LDS", (long long)lds_budget_bytes);
    const std::vector<Cand> &c = full.empty() ? all : full;
    auto better = [](const Cand &a, const Cand &b) {
        const int64_t Sa = (int64_t)a.sx * a.sy * a.sz, Sb = (int64_t)b.sx * b.sy * b.sz;
        if (Sa != Sb) return Sa > Sb;
        const int64_t fa = (int64_t)a.sx * a.sy + (int64_t)a.sy * a.sz + (int64_t)a.sz * a.sx;
        const int64_t fb = (int64_t)b.sx * b.sy + (int64_t)b.sy * b.sz + (int64_t)b.sz * b.sx;
        if (fa != fb) return fa < fb;
        if (a.sz != b.sz) return a.sz > b.sz;
        return a.sy > b.sy;
    };
    Cand best = c[0];
    for (const Cand &x : c)
        if (better(x, best)) best = x;
    out[0] = best.sx;
    out[1] = best.sy;
    out[2] = best.sz;
    return DD_OK;
}

extern "C" int dd_device_caps(int32_t *n_cu, int64_t *lds_per_workgroup) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_global_error(DD_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    int cu = 0, lds = 0;
    e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return set_global_error(DD_EHIP, "device attribute: %s", hipGetErrorString(e));
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return set_global_error(DD_EHIP, "device attribute: %s", hipGetErrorString(e));
    if (n_cu) *n_cu = cu;
    if (lds_per_workgroup) *lds_per_workgroup = lds;
    return DD_OK;
}

// -------------------------------------------------------------- partition
static int build_handle(dd_ctx *h, const int32_t *brow_ptr, const int32_t *bcol, const double *val,
                        hipStream_t st, dd_handle *out);

extern "C" int dd_partition(const dd_partition_desc *d, const int32_t *brow_ptr, const int32_t *bcol,
                            const double *val, int64_t nnzb, void *hip_stream, dd_handle *out) {
    if (!d || !brow_ptr || !bcol || !val || !out) return set_global_error(DD_EINVAL, "dd_partition: null argument");
    *out = nullptr;
    if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0) return set_global_error(DD_EINVAL, "dd_partition: empty grid");
    if (d->bs != 1 && d->bs != 3) return set_global_error(DD_EINVAL, "dd_partition: bs must be 1 or 3");
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    if (n >= (int64_t)1 << 31) return set_global_error(DD_EINVAL, "dd_partition: too many block rows");
    if (nnzb < n || nnzb >= ((int64_t)1 << 31)) return set_global_error(DD_EINVAL, "dd_partition: bad nnzb %lld", (long long)nnzb);
    int32_t n_cu = d->n_cu;
    int64_t lds = d->lds_budget_bytes;
    if (n_cu <= 0 || lds <= 0) {
        int32_t c;
        int64_t l;
        int rc = dd_device_caps(&c, &l);
        if (rc) return rc;
        if (n_cu <= 0) n_cu = c;
        if (lds <= 0) lds = l;
    }
    int32_t sub[3] = {d->sx, d->sy, d->sz};
    if (sub[0] == 0 && sub[1] == 0 && sub[2] == 0) {
        int rc = dd_auto_subdims(d->nx, d->ny, d->nz, d->bs, lds, n_cu, sub);
        if (rc) return rc;
    }
    if (sub[0] <= 0 || sub[1] <= 0 || sub[2] <= 0) return set_global_error(DD_EINVAL, "dd_partition: bad subdomain extents");
    if (d->nx % sub[0] || d->ny % sub[1] || d->nz % sub[2])
        return set_global_error(DD_ENOTDIV, "grid %dx%dx%d not divisible by subdomain %dx%dx%d", d->nx, d->ny, d->nz,
                                sub[0], sub[1], sub[2]);
    const int64_t S = (int64_t)sub[0] * sub[1] * sub[2];
    if (S * d->bs * 8 > lds)
        return set_global_error(DD_ELDS, "subdomain vector of %lld bytes exceeds the LDS budget %lld",
                                (long long)(S * d->bs * 8), (long long)lds);
    if (S > 65535) return set_global_error(DD_EINVAL, "subdomain of %lld rows exceeds 65535", (long long)S);

    dd_ctx *h = new dd_ctx();
    h->nx = d->nx; h->ny = d->ny; h->nz = d->nz; h->bs = d->bs;
    h->sx = sub[0]; h->sy = sub[1]; h->sz = sub[2];
    h->S = (int32_t)S;
    h->n = n;
    h->nsub = (int32_t)(n / S);
    h->nnzb = nnzb;
    return build_handle(h, brow_ptr, bcol, val, as_stream(hip_stream), out);
}

extern "C" int dd_partition_graph(const dd_graph_desc *d, const int32_t *brow_ptr, const int32_t *bcol,
                                  const double *val, int64_t nnzb, void *hip_stream, dd_handle *out) {
    if (!d || !brow_ptr || !bcol || !val || !out)
        return set_global_error(DD_EINVAL, "dd_partition_graph: null argument");
    *out = nullptr;
    const int64_t n = d->n;
    if (n <= 0 || n >= (int64_t)1 << 31) return set_global_error(DD_EINVAL, "dd_partition_graph: bad n %lld", (long long)n);
    if (d->bs != 1 && d->bs != 3) return set_global_error(DD_EINVAL, "dd_partition_graph: bs must be 1 or 3");
    if (nnzb < n || nnzb >= ((int64_t)1 << 31))
        return set_global_error(DD_EINVAL, "dd_partition_graph: bad nnzb %lld", (long long)nnzb);
    int64_t lds = d->lds_budget_bytes;
    int32_t n_cu = d->n_cu;
    if (lds <= 0 || n_cu <= 0) {
        int32_t c;
        int64_t l;
        int rc = dd_device_caps(&c, &l);
        if (rc) return rc;
        if (lds <= 0) lds = l;
        if (n_cu <= 0) n_cu = c;
    }
    int64_t S = d->part_rows;
    if (S == 0) {
        // Divisors of n whose vector fits the LDS.  The apply runs one part
        // per compute unit at a time, so a CU works through ceil(parts/n_cu)
        // parts of S rows in turn: take the divisor with the fewest rows per
        // CU by that count, and among those within 5% of the fewest the
        // largest (fewer couplings dropped between parts).
        const int64_t cap = std::min<int64_t>(65535, lds / (8 * d->bs));
        auto load = [&](int64_t c) { return (n / c + n_cu - 1) / n_cu * c; };
        int64_t best = 0;
        for (int64_t c = std::min(cap, n); c >= 1; --c)
            if (n % c == 0 && (best == 0 || load(c) < load(best))) best = c;
        S = best;
        for (int64_t c = std::min(cap, n); c > best; --c)
            if (n % c == 0 && load(c) * 100 <= load(best) * 105) {
                S = c;
                break;
            }
    }
    if (S <= 0 || n % S)
        return set_global_error(DD_ENOTDIV, "dd_partition_graph: %lld block rows not divisible by part_rows %lld",
                                (long long)n, (long long)S);
    if (S * d->bs * 8 > lds)
        return set_global_error(DD_ELDS, "subdomain vector of %lld bytes exceeds the LDS budget %lld",
                                (long long)(S * d->bs * 8), (long long)lds);
    if (S > 65535) return set_global_error(DD_EINVAL, "subdomain of %lld rows exceeds 65535", (long long)S);
    dd_ctx *h = new dd_ctx();
    h->nx = (int32_t)n; h->ny = 1; h->nz = 1; h->bs = d->bs;
    h->sx = (int32_t)S; h->sy = 1; h->sz = 1;
    h->graph = 1;
    h->S = (int32_t)S;
    h->n = n;
    h->nsub = (int32_t)(n / S);
    h->nnzb = nnzb;
    return build_handle(h, brow_ptr, bcol, val, as_stream(hip_stream), out);
}

// Everything after the subdomain size is fixed: labels and the permutation
// (geometric cuts, or the graph partitioner when h->graph), then Algorithm 3.
static int build_handle(dd_ctx *h, const int32_t *brow_ptr, const int32_t *bcol, const double *val,
                        hipStream_t st, dd_handle *out) {
    const int64_t n = h->n, nnzb = h->nnzb;
    const int bb = h->bs * h->bs;
    int rc = 0;
    int32_t *len = nullptr, *src = nullptr;
    auto bail = [&](int code) {
        g_err = h->err;
        delete h;
        return code;
    };
    if ((rc = h->alloc(&h->status, 8))) return bail(rc);
    h->scan_tmp_len = scan_tmp_elems(std::max<int64_t>(n, nnzb) + 1);
    if ((rc = h->alloc(&h->scan_tmp, h->scan_tmp_len))) return bail(rc);
    if ((rc = h->alloc(&h->part_id, n)) || (rc = h->alloc(&h->new2old, n)) || (rc = h->alloc(&h->old2new, n)) ||
        (rc = h->alloc(&h->aptr, n + 1)) || (rc = h->alloc(&h->acol, nnzb)) ||
        (rc = h->alloc(&h->aval, nnzb * bb)) || (rc = h->alloc(&len, n)) || (rc = h->alloc(&src, nnzb)))
        return bail(rc);
    int32_t init_status[8] = {0, 0x7fffffff, 0x7fffffff, 0, 0, 0, 0, 0};
    hipError_t e;
#define PCHK(x)                                                                   \
    do {                                                                          \
        e = (x);                                                                  \
        if (e != hipSuccess) {                                                    \
            h->fail(DD_EHIP, "%s: %s", #x, hipGetErrorString(e));                 \
            return bail(DD_EHIP);                                                 \
        }                                                                         \
    } while (0)
    PCHK(hipMemcpyAsync(h->status, init_status, sizeof(init_status), hipMemcpyHostToDevice, st));
    // the caller's pattern is checked before any kernel indexes through it
    PCHK(launch_check_rows(n, nnzb, brow_ptr, bcol, h->status, st));
    {
        int32_t bad = 0;
        PCHK(hipMemcpyAsync(&bad, h->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        PCHK(hipStreamSynchronize(st));
        if (bad & 1) {
            h->fail(DD_EINVAL, "a row holds more than %d blocks (or brow_ptr is not monotone within nnzb)",
                    kMaxRowBlocks);
            return bail(DD_EINVAL);
        }
        if (bad & 2) {
            h->fail(DD_EINVAL, "a column index lies outside [0, %lld)", (long long)n);
            return bail(DD_EINVAL);
        }
    }
    if (h->graph) {
        if ((rc = graph_partition(h, brow_ptr, bcol, st))) return bail(rc);
    } else {
        PCHK(launch_partition(h, st));
    }
    PCHK(launch_row_len(h, brow_ptr, len, st));
    PCHK(launch_max_count(n, len, h->status + 6, st));  // longest row (selects the SpMV layout)
    PCHK(exclusive_scan(len, h->aptr, n, h->scan_tmp, st));
    int32_t total = 0, status[8];
    PCHK(hipMemcpyAsync(&total, h->aptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PCHK(hipMemcpyAsync(status, h->status, sizeof(status), hipMemcpyDeviceToHost, st));
    PCHK(hipStreamSynchronize(st));
    if (status[0]) {
        h->fail(DD_EINVAL, "a row holds more than %d blocks (or brow_ptr is not monotone)", kMaxRowBlocks);
        return bail(DD_EINVAL);
    }
    if (total != nnzb) {
        h->fail(DD_EINVAL, "brow_ptr describes %d blocks, nnzb says %lld", total, (long long)nnzb);
        return bail(DD_EINVAL);
    }
    h->max_row_a = status[6];
    PCHK(launch_reorder_fill(h, brow_ptr, bcol, val, src, st));
    PCHK(hipStreamSynchronize(st));
    release(h, len);
    h->asrc = src;  // kept for ilu0_refactor
    build_spmv_layout(h, st);
    *out = h;
    return DD_OK;
}

extern "C" int dd_get_info(dd_handle h, dd_info *info) {
    if (!h || !info) return set_global_error(DD_EINVAL, "dd_get_info: null argument");
    std::memset(info, 0, sizeof(*info));
    info->n = h->n;
    info->nnzb = h->nnzb;
    info->nnzb_dropped = h->nnzt;
    info->nnzb_lower = h->nlow;
    info->nnzb_upper = h->nupp;
    info->bs = h->bs;
    info->S = h->S;
    info->nsub = h->nsub;
    info->sx = h->sx; info->sy = h->sy; info->sz = h->sz;
    for (int w = 0; w < 2; ++w) {
        info->level_ptr_len[w] = h->lev[w].ptr_len;
        info->max_levels[w] = h->lev[w].max_levels;
    }
    info->factored = h->factored;
    info->precision = h->precision;
    const int64_t wsz = h->precision == DD_FP64 ? 8 : 4;  // factor storage
    const int64_t bb = h->bs * h->bs;
    info->apply_bytes = (h->nlow + h->nupp) * (bb * wsz + 4) + h->n * bb * wsz + 2 * 4 * (h->n + 1) +
                        2 * h->n * h->bs * 8;
    info->lds_bytes = apply_lds_bytes(h, h->precision);
    info->max_row_blocks = h->max_row_a;
    info->spmv_layout = h->ell_state == 1 ? (h->sell_row ? (h->sell_spp ? 3 : 2) : 1) : 0;
    info->apply_layout = h->slots ? 1 : (h->seg ? 2 : 0);
    info->seg_blocks = h->seg;
    return DD_OK;
}

extern "C" int dd_get_partition(dd_handle h, int32_t *part_id, int32_t *new2old, int32_t *old2new,
                                void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_get_partition: null handle");
    hipStream_t st = as_stream(hip_stream);
    const size_t b = h->n * sizeof(int32_t);
    if (part_id) HCHK(hipMemcpyAsync(part_id, h->part_id, b, hipMemcpyDeviceToDevice, st));
    if (new2old) HCHK(hipMemcpyAsync(new2old, h->new2old, b, hipMemcpyDeviceToDevice, st));
    if (old2new) HCHK(hipMemcpyAsync(old2new, h->old2new, b, hipMemcpyDeviceToDevice, st));
    return DD_OK;
}

extern "C" int dd_get_reordered(dd_handle h, int32_t *ptr, int32_t *col, double *val, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_get_reordered: null handle");
    hipStream_t st = as_stream(hip_stream);
    if (ptr) HCHK(hipMemcpyAsync(ptr, h->aptr, (h->n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (col) HCHK(hipMemcpyAsync(col, h->acol, h->nnzb * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (val)
        HCHK(hipMemcpyAsync(val, h->aval, h->nnzb * h->bs * h->bs * sizeof(double), hipMemcpyDeviceToDevice, st));
    return DD_OK;
}

// ----------------------------------------------------------------- factor
static int build_levels(dd_ctx *h, int which, hipStream_t st, int32_t *tmp_i) {
    Levels &L = h->lev[which];
    if (!L.lev) {
        RCHK(h->alloc(&L.lev, h->n));
        RCHK(h->alloc(&L.nlev, h->nsub));
        RCHK(h->alloc(&L.off, h->nsub + 1));
        RCHK(h->alloc(&L.rows, h->n));
    }
    HCHK(launch_levels(h, which, st));
    HCHK(launch_plus_one(h->nsub, L.nlev, tmp_i, st));
    HCHK(exclusive_scan(tmp_i, L.off, h->nsub, h->scan_tmp, st));
    int32_t total = 0;
    HCHK(hipMemcpyAsync(&total, L.off + h->nsub, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    if (L.ptr) release(h, L.ptr);
    RCHK(h->alloc(&L.ptr, total));
    L.ptr_len = total;
    HCHK(launch_level_lists(h, which, st));
    // host copies of the level offsets: largest level count and widest level
    std::vector<int32_t> off(h->nsub + 1), lp(total);
    HCHK(hipMemcpyAsync(off.data(), L.off, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HCHK(hipMemcpyAsync(lp.data(), L.ptr, lp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    int maxl = 0, maxw = 0;
    for (int s = 0; s < h->nsub; ++s) {
        const int nl = off[s + 1] - off[s] - 1;
        maxl = std::max(maxl, nl);
        for (int l = 0; l < nl; ++l) maxw = std::max(maxw, lp[off[s] + l + 1] - lp[off[s] + l]);
    }
    L.max_levels = maxl;
    h->max_level_width = std::max(h->max_level_width, maxw);
    return DD_OK;
}

static int build_sweep(dd_ctx *h, int which, hipStream_t st, int32_t *cnt) {
    Sweep &w = h->sw[which];
    const int bb = h->bs * h->bs;
    if (!w.prow) {
        RCHK(h->alloc(&w.prow, h->n));
        RCHK(h->alloc(&w.bptr, h->n + 1));
    }
    HCHK(launch_pack_count(h, which, cnt, st));
    HCHK(hipMemsetAsync(h->status + 4, 0, sizeof(int32_t), st));
    HCHK(launch_max_count(h->n, cnt, h->status + 4, st));
    HCHK(exclusive_scan(cnt, w.bptr, h->n, h->scan_tmp, st));
    int32_t total = 0, maxrow = 0;
    HCHK(hipMemcpyAsync(&total, w.bptr + h->n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HCHK(hipMemcpyAsync(&maxrow, h->status + 4, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    if (w.bcol) { release(h, w.bcol); release(h, w.val64); w.bcol = nullptr; w.val64 = nullptr; }
    if (w.uraw) { release(h, w.uraw); w.uraw = nullptr; }
    if (w.val32) { release(h, w.val32); w.val32 = nullptr; }
    w.nblk = total;
    w.max_row = maxrow;
    RCHK(h->alloc(&w.bcol, total));
    RCHK(h->alloc(&w.val64, (int64_t)total * bb));
    if (which == 1 && !w.d64) RCHK(h->alloc(&w.d64, h->n * bb));
    HCHK(launch_pack_fill(h, which, st));
    return DD_OK;
}

// Slot layout for both sweeps when no row has more than kMaxSlots blocks.
static int build_slots(dd_ctx *h, hipStream_t st) {
    const int bb = h->bs * h->bs;
    for (int w = 0; w < 2; ++w) {
        Sweep &s = h->sw[w];
        if (s.desc) { release(h, s.desc); release(h, s.sval64); }
        if (s.sval32) release(h, s.sval32);
        s.desc = nullptr; s.sval64 = nullptr; s.sval32 = nullptr;
        s.snpos = 0;
    }
    const int mr = std::max(h->sw[0].max_row, h->sw[1].max_row);
    h->slots = mr <= kMaxSlots ? std::max(mr, 1) : 0;
    h->seg = 0;
    if (!h->slots) {
        // rows of more than three blocks: the segmented layout, for the apply's
        // workgroups of 1,024 lanes, with segments of two blocks (the least
        // zero padding on the row lengths of k-nearest-neighbour graphs:
        // 1.18x the algorithmic bytes against 1.29x with three), or of three
        // when a row would need more than kSegMax segments of two
        const int lo = h->sw[0].max_row, up = h->sw[1].max_row;
        auto fits = [&](int mb) { return lo <= mb * kSegMax && up <= mb + (kSegMax - 1) * (mb + 1); };
        const int mb = fits(2) ? 2 : (fits(3) ? 3 : 0);
        if (!mb) return DD_OK;
        // the walk counts positions in 32-bit integers: a row takes at most
        // kSegMax segments and kSegMax - 1 padding positions, so stay on the
        // plain loop where that bound could pass 2^31
        for (int w = 0; w < 2; ++w)
            if ((int64_t)(h->sw[w].nblk + h->n) * (2 * kSegMax) >= ((int64_t)1 << 31)) return DD_OK;
        const int rpw = kWave / h->bs, cw = rpw * (1024 / kWave);
        h->seg = mb;  // the packing reads it
        for (int w = 0; w < 2; ++w) {
            const int rc = build_seg_layout(h, w, mb, cw, rpw, st);
            if (rc) {
                h->seg = 0;
                return rc;
            }
        }
        return DD_OK;
    }
    for (int w = 0; w < 2; ++w) {
        Sweep &s = h->sw[w];
        s.snpos = h->n;
        RCHK(h->alloc(&s.desc, h->n));
        RCHK(h->alloc(&s.sval64, h->n * (h->slots + w) * bb));  // upper: + inv_D
        HCHK(launch_pack_slots(h, w, st));
    }
    return DD_OK;
}

static int ensure_fp32(dd_ctx *h, hipStream_t st) {
    const int bb = h->bs * h->bs;
    const bool sl = h->slots || h->seg;
    const int mb = h->seg ? h->seg : h->slots;
    if (h->sw[0].val32 && h->sw[1].val32 && h->sw[1].d32 && (!sl || h->sw[0].sval32)) return DD_OK;
    for (int w = 0; w < 2; ++w) {
        if (!h->sw[w].val32) RCHK(h->alloc(&h->sw[w].val32, h->sw[w].nblk * bb));
        if (sl && !h->sw[w].sval32) RCHK(h->alloc(&h->sw[w].sval32, h->sw[w].snpos * (mb + w) * bb));
    }
    if (!h->sw[1].d32) RCHK(h->alloc(&h->sw[1].d32, h->n * bb));
    HCHK(launch_cast32(h, st));
    return DD_OK;
}

extern "C" int ilu0_factor(dd_handle h, int32_t precision, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "ilu0_factor: null handle");
    if (precision != DD_FP64 && precision != DD_FP32 && precision != DD_MIXED)
        return h->fail(DD_EINVAL, "ilu0_factor: bad precision");
    hipStream_t st = as_stream(hip_stream);
    const int bb = h->bs * h->bs;
    h->factored = 0;
    h->patterned = 0;
    h->lic.adj_ready = 0;  // the adjoint apply's streams hold the old factors
    int32_t *tbeg = nullptr, *tlen = nullptr, *tsrc = nullptr;
    RCHK(h->alloc(&tbeg, h->n));
    RCHK(h->alloc(&tlen, h->n + 1));
    int32_t init_status[8] = {0, 0x7fffffff, 0x7fffffff, 0, 0, 0, 0, 0};
    HCHK(hipMemcpyAsync(h->status, init_status, sizeof(init_status), hipMemcpyHostToDevice, st));
    // drop (Section 3.2)
    HCHK(launch_drop_count(h, tbeg, tlen, st));
    if (!h->tptr) RCHK(h->alloc(&h->tptr, h->n + 1));
    HCHK(exclusive_scan(tlen, h->tptr, h->n, h->scan_tmp, st));
    int32_t total = 0, status[8];
    HCHK(hipMemcpyAsync(&total, h->tptr + h->n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HCHK(hipMemcpyAsync(status, h->status, sizeof(status), hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    if (status[1] != 0x7fffffff) {
        release(h, tbeg); release(h, tlen);
        return h->fail(DD_EZEROPIVOT, "block row %d has no diagonal block", status[1]);
    }
    h->nnzt = total;
    h->nlow = h->nupp = (total - h->n) / 2;  // refined below from the sweeps
    if (h->tcol) { release(h, h->tcol); release(h, h->lu); }
    RCHK(h->alloc(&h->tcol, total));
    RCHK(h->alloc(&h->lu, (int64_t)total * bb));
    if (!h->tdiag) RCHK(h->alloc(&h->tdiag, h->n));
    if (!h->invd) RCHK(h->alloc(&h->invd, h->n * bb));
    if (h->tsrc) release(h, h->tsrc);
    h->tsrc = nullptr;
    RCHK(h->alloc(&tsrc, total));
    HCHK(launch_drop_rows(h, tbeg, tsrc, st));
    // level sets (Section 4.2.1) for both factors
    h->max_level_width = 0;
    RCHK(build_levels(h, 0, st, tlen));
    RCHK(build_levels(h, 1, st, tlen));
    // block ILU0 (Algorithm 5), level-scheduled per subdomain
    HCHK(launch_bilu0(h, st));
    HCHK(hipMemcpyAsync(status, h->status, sizeof(status), hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    h->tsrc = tsrc;  // kept for ilu0_refactor
    if (status[2] != 0x7fffffff) {
        release(h, tbeg); release(h, tlen);
        return h->fail(DD_EZEROPIVOT, "singular or ill-conditioned pivot block at reordered block row %d", status[2]);
    }
    // ILDU0 post-pass folded into the packing of the two sweeps
    RCHK(build_sweep(h, 0, st, tlen));
    RCHK(build_sweep(h, 1, st, tlen));
    RCHK(build_slots(h, st));
    h->nlow = h->sw[0].nblk;
    h->nupp = h->sw[1].nblk;
    h->precision = precision;
    if (precision != DD_FP64) RCHK(ensure_fp32(h, st));
    HCHK(hipStreamSynchronize(st));
    release(h, tbeg);
    release(h, tlen);
    h->factored = 1;
    h->patterned = 1;
    return DD_OK;
}

extern "C" int ilu0_refactor(dd_handle h, const double *val, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "ilu0_refactor: null handle");
    if (!val) return h->fail(DD_EINVAL, "ilu0_refactor: null values");
    if (!h->patterned || !h->asrc || !h->tsrc) return h->fail(DD_ESTATE, "ilu0_refactor before ilu0_factor");
    hipStream_t st = as_stream(hip_stream);
    const int bb = h->bs * h->bs;
    h->factored = 0;
    // what depends on A's values and is rebuilt by its own call
    h->lic.adj_ready = 0;
    h->lic.active = 0;
    h->lic.ready = 0;
    h->gfactored = 0;
    if (h->sw[1].uraw) { release(h, h->sw[1].uraw); h->sw[1].uraw = nullptr; }
    // values of the reordered matrix, its sliced ELL copy and the dropped pattern
    HCHK(launch_gather_blocks(h->nnzb, bb, h->asrc, val, h->aval, st));
    HCHK(refresh_spmv_layout(h, st));
    HCHK(launch_gather_blocks(h->nnzt, bb, h->tsrc, h->aval, h->lu, st));
    // block ILU0 on the kept level sets
    int32_t init_status[8] = {0, 0x7fffffff, 0x7fffffff, 0, 0, 0, 0, 0};
    HCHK(hipMemcpyAsync(h->status, init_status, sizeof(init_status), hipMemcpyHostToDevice, st));
    HCHK(launch_bilu0(h, st));
    int32_t status[8];
    HCHK(hipMemcpyAsync(status, h->status, sizeof(status), hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    if (status[2] != 0x7fffffff)
        return h->fail(DD_EZEROPIVOT, "singular or ill-conditioned pivot block at reordered block row %d", status[2]);
    // ILDU0 scaling and the streaming layouts, into the existing arrays
    HCHK(launch_pack_fill(h, 0, st));
    HCHK(launch_pack_fill(h, 1, st));
    if (h->slots) {
        HCHK(launch_pack_slots(h, 0, st));
        HCHK(launch_pack_slots(h, 1, st));
    }
    if (h->seg) {
        HCHK(launch_seg_pack(h, 0, st));
        HCHK(launch_seg_pack(h, 1, st));
    }
    if (h->sw[0].val32) HCHK(launch_cast32(h, st));
    HCHK(hipStreamSynchronize(st));
    h->factored = 1;
    return DD_OK;
}

extern "C" int dd_set_precision(dd_handle h, int32_t precision, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_set_precision: null handle");
    if (!h->factored) return h->fail(DD_ESTATE, "dd_set_precision before ilu0_factor");
    if (precision != DD_FP64 && precision != DD_FP32 && precision != DD_MIXED)
        return h->fail(DD_EINVAL, "bad precision");
    if (precision != DD_FP64) RCHK(ensure_fp32(h, as_stream(hip_stream)));
    h->precision = precision;
    return DD_OK;
}

extern "C" int dd_get_levels(dd_handle h, int32_t which, int32_t *nlev, int32_t *level_ptr, int32_t *level_rows,
                             void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_get_levels: null handle");
    if (which != 0 && which != 1) return h->fail(DD_EINVAL, "dd_get_levels: which must be 0 or 1");
    if (!h->factored) return h->fail(DD_ESTATE, "dd_get_levels before ilu0_factor");
    hipStream_t st = as_stream(hip_stream);
    const Levels &L = h->lev[which];
    if (nlev) HCHK(hipMemcpyAsync(nlev, L.nlev, h->nsub * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (level_ptr) HCHK(hipMemcpyAsync(level_ptr, L.ptr, L.ptr_len * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (level_rows) HCHK(hipMemcpyAsync(level_rows, L.rows, h->n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    return DD_OK;
}

extern "C" int dd_get_factors(dd_handle h, int32_t *ptr, int32_t *col, double *f, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_get_factors: null handle");
    if (!h->factored) return h->fail(DD_ESTATE, "dd_get_factors before ilu0_factor");
    hipStream_t st = as_stream(hip_stream);
    if (ptr) HCHK(hipMemcpyAsync(ptr, h->tptr, (h->n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (col) HCHK(hipMemcpyAsync(col, h->tcol, h->nnzt * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (f) HCHK(launch_export_factors(h, f, st));
    return DD_OK;
}

// ------------------------------------------------------------------ apply
// Checks the apply variant against the handle's state and builds what an
// ablation variant needs beyond the production streams (the unscaled U
// blocks of variant 7, once per factorisation).
static int prepare_variant(dd_ctx *h, const char *who, hipStream_t st) {
    if (const char *why = variant_unsupported(h, h->variant)) return h->fail(DD_EINVAL, "%s: %s", who, why);
    Sweep &U = h->sw[1];
    if (h->variant == 7 && !U.uraw) {
        RCHK(h->alloc(&U.uraw, U.nblk * h->bs * h->bs));
        HCHK(launch_pack_unscaled(h, st));
    }
    return DD_OK;
}

extern "C" int dd_trsv_apply(dd_handle h, const double *r, double *z, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_trsv_apply: null handle");
    if (!h->factored) return h->fail(DD_ESTATE, "dd_trsv_apply before ilu0_factor");
    if (!r || !z || r == z) return h->fail(DD_EINVAL, "dd_trsv_apply: r and z must be distinct device buffers");
    RCHK(prepare_variant(h, "dd_trsv_apply", as_stream(hip_stream)));
    HCHK(launch_apply(h, r, z, nullptr, as_stream(hip_stream)));
    return DD_OK;
}

extern "C" int dd_spmv(dd_handle h, const double *x, double *y, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_spmv: null handle");
    if (!x || !y || x == y) return h->fail(DD_EINVAL, "dd_spmv: x and y must be distinct device buffers");
    HCHK(launch_spmv(h, x, y, as_stream(hip_stream)));
    return DD_OK;
}

static int check_solve_args(dd_ctx *h, const char *who, const double *b, double *x, double rtol, int32_t maxit) {
    if (!h->factored) return h->fail(DD_ESTATE, "%s before ilu0_factor", who);
    if (!b || !x || b == x) return h->fail(DD_EINVAL, "%s: b and x must be distinct device buffers", who);
    if (!(rtol > 0.0) || maxit < 0) return h->fail(DD_EINVAL, "%s: bad rtol or maxit", who);
    return DD_OK;
}

// One solve in workspace w.  A learned solve that breaks down or misses
// maxit is repeated with plain DD-ILU0 from the caller's initial guess, kept
// in the workspace's last vector (the solve overwrites x with its last
// iterate).
static int solve_in(dd_ctx *h, const KrylovWork &w, const double *b, double *x, double rtol, int32_t maxit,
                    hipStream_t st, dd_solve_info *info) {
    const bool learned = h->pc_kind == 0 && h->lic.active;
    if (!learned || !h->lic_fallback) return bicgstab_run(h, w, b, x, rtol, maxit, st, info);
    const int64_t m = h->n * h->bs;
    double *x0 = w.kv + (int64_t)(kKrylovVectors - 1) * m;
    HCHK(hipMemcpyAsync(x0, x, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    dd_solve_info first{};
    const int rc = bicgstab_run(h, w, b, x, rtol, maxit, st, &first);
    if (rc != DD_EBREAKDOWN && rc != DD_ENOCONV) {
        if (info) *info = first;
        return rc;
    }
    HCHK(hipMemcpyAsync(x, x0, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    h->lic.active = 0;
    dd_solve_info second{};
    const int rc2 = bicgstab_run(h, w, b, x, rtol, maxit, st, &second);
    h->lic.active = 1;
    if (info) {
        *info = second;
        info->fallback = 1;
        info->solve_seconds += first.solve_seconds;
        info->applies += first.applies;
        info->apply_seconds += first.apply_seconds;
    }
    return rc2;
}

extern "C" int bicgstab_solve(dd_handle h, const double *b, double *x, double rtol, int32_t maxit, void *hip_stream,
                              dd_solve_info *info) {
    if (!h) return set_global_error(DD_EINVAL, "bicgstab_solve: null handle");
    RCHK(check_solve_args(h, "bicgstab_solve", b, x, rtol, maxit));
    hipStream_t st = as_stream(hip_stream);
    if (h->pc_kind == 0) RCHK(prepare_variant(h, "bicgstab_solve", st));
    KrylovWork w;
    RCHK(krylov_workspace(h, &w));
    return solve_in(h, w, b, x, rtol, maxit, st, info);
}

extern "C" int bicgstab_solve_noalloc(dd_handle h, const double *b, double *x, double rtol, int32_t maxit,
                                      void *hip_stream, dd_solve_info *info) {
    if (!h) return set_global_error(DD_EINVAL, "bicgstab_solve_noalloc: null handle");
    RCHK(check_solve_args(h, "bicgstab_solve_noalloc", b, x, rtol, maxit));
    if (h->pc_kind == 0) {
        if (const char *why = variant_unsupported(h, h->variant))
            return h->fail(DD_EINVAL, "bicgstab_solve_noalloc: %s", why);
        if (h->variant == 7 && !h->sw[1].uraw)
            return h->fail(DD_ESTATE,
                           "bicgstab_solve_noalloc: apply variant 7 needs its unscaled factors, which the first "
                           "dd_trsv_apply or bicgstab_solve with that variant allocates");
    }
    KrylovScalars host{};
    KrylovWork w;
    RCHK(noalloc_workspace(h, &w, &host));
    return solve_in(h, w, b, x, rtol, maxit, as_stream(hip_stream), info);
}

extern "C" int dd_set_lic_fallback(dd_handle h, int32_t on) {
    if (!h) return set_global_error(DD_EINVAL, "dd_set_lic_fallback: null handle");
    h->lic_fallback = on ? 1 : 0;
    return DD_OK;
}

extern "C" int dd_set_apply_variant(dd_handle h, int32_t variant) {
    if (!h) return set_global_error(DD_EINVAL, "dd_set_apply_variant: null handle");
    if (variant < 0 || variant > 8) return h->fail(DD_EINVAL, "dd_set_apply_variant: variant must be 0..8");
    h->variant = variant;
    return DD_OK;
}

extern "C" int dd_set_profiling(dd_handle h, int32_t on) {
    if (!h) return set_global_error(DD_EINVAL, "dd_set_profiling: null handle");
    h->profile = on ? 1 : 0;
    return DD_OK;
}

extern "C" int dd_set_fusion(dd_handle h, int32_t on) {
    if (!h) return set_global_error(DD_EINVAL, "dd_set_fusion: null handle");
    h->fuse = on ? 1 : 0;
    return DD_OK;
}

extern "C" int dd_set_residual_history(dd_handle h, double *hist, int32_t len) {
    if (!h) return set_global_error(DD_EINVAL, "dd_set_residual_history: null handle");
    if (hist && len <= 0) return h->fail(DD_EINVAL, "dd_set_residual_history: len must be positive");
    h->hist = hist;
    h->hist_len = hist ? len : 0;
    return DD_OK;
}

// ------------------------------------------------------------- global ILU0
extern "C" int dd_global_factor(dd_handle h, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_global_factor: null handle");
    return global_factor(h, as_stream(hip_stream));
}

extern "C" int dd_global_apply(dd_handle h, const double *r, double *z, int32_t nrhs, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_global_apply: null handle");
    if (!h->gfactored) return h->fail(DD_ESTATE, "dd_global_apply before dd_global_factor");
    if (!r || !z || r == z || nrhs < 1) return h->fail(DD_EINVAL, "dd_global_apply: bad arguments");
    HCHK(launch_global_apply(h, r, z, nrhs, as_stream(hip_stream)));
    return DD_OK;
}

extern "C" int dd_set_preconditioner(dd_handle h, int32_t kind) {
    if (!h) return set_global_error(DD_EINVAL, "dd_set_preconditioner: null handle");
    if (kind != 0 && kind != 1) return h->fail(DD_EINVAL, "dd_set_preconditioner: kind must be 0 or 1");
    if (kind == 1 && !h->gfactored) return h->fail(DD_ESTATE, "global preconditioner before dd_global_factor");
    h->pc_kind = kind;
    return DD_OK;
}

// ------------------------------------------------------- learned correction
extern "C" int lic_setup(dd_handle h, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "lic_setup: null handle");
    return ddilu::lic_setup(h, as_stream(hip_stream));
}

extern "C" int lic_get_faces(dd_handle h, int32_t *nf, int32_t *fI, int32_t *fJ, float *X, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "lic_get_faces: null handle");
    if (!h->lic.ready) return h->fail(DD_ESTATE, "lic_get_faces before lic_setup");
    hipStream_t st = as_stream(hip_stream);
    const int64_t m = h->lic.nf;
    if (nf) *nf = (int32_t)m;
    if (fI && m) HCHK(hipMemcpyAsync(fI, h->lic.fI, m * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (fJ && m) HCHK(hipMemcpyAsync(fJ, h->lic.fJ, m * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (X && m) HCHK(hipMemcpyAsync(X, h->lic.X, m * 27 * sizeof(float), hipMemcpyDeviceToDevice, st));
    return DD_OK;
}

extern "C" int lic_set_params(dd_handle h, const float *params, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "lic_set_params: null handle");
    if (!params) {
        h->lic.active = 0;
        return DD_OK;
    }
    if (!h->lic.ready) return h->fail(DD_ESTATE, "lic_set_params before lic_setup");
    RCHK(ddilu::lic_coeffs_from_params(h, params, false, as_stream(hip_stream)));
    h->lic.active = 1;
    return DD_OK;
}

extern "C" int lic_set_coeffs(dd_handle h, const float *C, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "lic_set_coeffs: null handle");
    if (!C) {
        h->lic.active = 0;
        return DD_OK;
    }
    if (!h->lic.ready) return h->fail(DD_ESTATE, "lic_set_coeffs before lic_setup");
    if (h->lic.nf)
        HCHK(hipMemcpyAsync(h->lic.C, C, (size_t)h->lic.nf * 9 * sizeof(float), hipMemcpyDeviceToDevice,
                            as_stream(hip_stream)));
    RCHK(ddilu::lic_publish_coeffs(h, as_stream(hip_stream)));
    h->lic.active = 1;
    return DD_OK;
}

extern "C" int lic_get_coeffs(dd_handle h, float *C, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "lic_get_coeffs: null handle");
    if (!h->lic.ready || !C) return h->fail(DD_ESTATE, "lic_get_coeffs before lic_setup");
    if (h->lic.nf)
        HCHK(hipMemcpyAsync(C, h->lic.C, (size_t)h->lic.nf * 9 * sizeof(float), hipMemcpyDeviceToDevice,
                            as_stream(hip_stream)));
    return DD_OK;
}

extern "C" int dd_apply_adjoint(dd_handle h, const double *g, double *a, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "dd_apply_adjoint: null handle");
    if (!h->lic.ready) return h->fail(DD_ESTATE, "dd_apply_adjoint before lic_setup");
    if (!g || !a || g == a) return h->fail(DD_EINVAL, "dd_apply_adjoint: bad arguments");
    RCHK(ddilu::lic_adjoint_streams(h, as_stream(hip_stream)));
    HCHK(launch_apply_adjoint(h, g, a, 1, as_stream(hip_stream)));
    return DD_OK;
}

extern "C" int lic_targets(dd_handle h, int32_t nq, const double *R, double *Zs, double *den, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "lic_targets: null handle");
    if (!h->gfactored || !h->lic.ready) return h->fail(DD_ESTATE, "lic_targets needs dd_global_factor and lic_setup");
    if (nq < 1 || !R || !Zs || !den) return h->fail(DD_EINVAL, "lic_targets: bad arguments");
    return ddilu::lic_targets_run(h, nq, R, Zs, den, as_stream(hip_stream));
}

extern "C" int lic_loss_grad(dd_handle h, const float *params, int32_t nq, const double *R, const double *Zs,
                             const double *den, double *loss, float *grad, int32_t accumulate, void *hip_stream) {
    if (!h) return set_global_error(DD_EINVAL, "lic_loss_grad: null handle");
    if (!h->lic.ready) return h->fail(DD_ESTATE, "lic_loss_grad before lic_setup");
    if (nq < 1 || !params || !R || !Zs || !den || !loss || !grad) return h->fail(DD_EINVAL, "lic_loss_grad: bad arguments");
    return ddilu::lic_loss_grad_run(h, params, nq, R, Zs, den, loss, grad, accumulate, as_stream(hip_stream));
}

extern "C" int lic_adam(float *params, const float *grad, float *m, float *v, int32_t nparam, int32_t t, float lr,
                        float b1, float b2, float eps, void *hip_stream) {
    if (!params || !grad || !m || !v || nparam < 1 || t < 1) return set_global_error(DD_EINVAL, "lic_adam: bad arguments");
    hipError_t e = launch_adam(nparam, params, grad, m, v, t, lr, b1, b2, eps, as_stream(hip_stream));
    if (e != hipSuccess) return set_global_error(DD_EHIP, "lic_adam: %s", hipGetErrorString(e));
    return DD_OK;
}

extern "C" int lic_train(dd_handle *hs, int32_t nprob, const double *const *R, const double *const *Zs,
                         const double *const *den, int32_t nq, float *params, float *m, float *v, int32_t epochs,
                         const int32_t *order, float lr, int32_t step0, double *loss_hist, void *hip_stream) {
    if (!hs || nprob < 1 || !R || !Zs || !den || nq < 1 || !params || !m || !v || epochs < 0 || !order ||
        step0 < 0)
        return set_global_error(DD_EINVAL, "lic_train: bad arguments");
    hipStream_t st = as_stream(hip_stream);
    float *grad = nullptr;
    double *lacc = nullptr;
    hipError_t e = hipMalloc(&grad, 6537 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&lacc, sizeof(double));
    if (e != hipSuccess) return set_global_error(DD_ENOMEM, "lic_train: %s", hipGetErrorString(e));
    int rc = DD_OK, t = step0;
    for (int ep = 0; ep < epochs && rc == DD_OK; ++ep) {
        e = hipMemsetAsync(lacc, 0, sizeof(double), st);
        for (int k = 0; k < nprob && rc == DD_OK && e == hipSuccess; ++k) {
            const int p = order[(int64_t)ep * nprob + k];
            if (p < 0 || p >= nprob) { rc = set_global_error(DD_EINVAL, "lic_train: bad order entry"); break; }
            rc = ddilu::lic_loss_grad_run(hs[p], params, nq, R[p], Zs[p], den[p], lacc, grad, 0, st);
            if (rc) { g_err = hs[p]->err; break; }
            e = launch_adam(6537, params, grad, m, v, ++t, lr, 0.9f, 0.999f, 1e-8f, st);
        }
        double l = 0.0;
        if (e == hipSuccess) e = hipMemcpyAsync(&l, lacc, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess && rc == DD_OK) rc = set_global_error(DD_EHIP, "lic_train: %s", hipGetErrorString(e));
        if (loss_hist) loss_hist[ep] = l / nprob;
    }
    (void)hipFree(grad);
    (void)hipFree(lacc);
    return rc;
}

extern "C" const char *dd_last_error(dd_handle h) { return h ? h->err.c_str() : g_err.c_str(); }

extern "C" void dd_destroy(dd_handle h) { delete h; }
