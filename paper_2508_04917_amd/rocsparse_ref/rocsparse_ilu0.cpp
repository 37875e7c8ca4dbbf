// Vendor-library baseline for the apply comparison of Section 5.2 (Table 4): rocSPARSE's
// block ILU0 (bsrilu0) and its two block triangular solves (bsrsv, lower with
// unit diagonal, then upper), called as a black box on a BSR matrix already
// on the device.  Built as its own library so that the DD-ILU0 library does
// not link rocSPARSE; only the benchmark and the tests load it.
//
// C ABI (all pointers device pointers unless noted; blocks row-major):
//   rsr_create(mb, nnzb, bs, ptr, col, val, stream, &out)
//       copies val, runs the ILU0 analysis, the factorisation and the
//       analyses of both triangular solves on the stream, synchronises, and
//       returns 0, or a negative code (message in rsr_last_error()); a zero
//       pivot is an error.
//   rsr_create_scalar(mb, nnzb, bs, ptr, col, val, stream, &out)
//       the same through rocSPARSE's scalar routines: the BSR matrix is
//       expanded to CSR (bsr2csr), then csrilu0 and two csrsv solves.  On a
//       pattern of dense blocks the scalar ILU0 equals the block ILU0 (the
//       fill stays inside the blocks), so both give the same preconditioner
//       up to rounding.
//   rsr_apply(h, r, z, stream)      z = U^{-1} L^{-1} r (r != z), asynchronous.
//   rsr_destroy(h)
#include <hip/hip_runtime.h>
#include <rocsparse/rocsparse.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

namespace {

thread_local std::string g_err;

int fail(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return -1;
}

struct Rsr {
    rocsparse_handle handle = nullptr;
    rocsparse_mat_descr dM = nullptr, dL = nullptr, dU = nullptr;
    rocsparse_mat_info info = nullptr;
    int32_t mb = 0, nnzb = 0, bs = 0;
    bool scalar = false;  // CSR expansion and the scalar routines
    const int32_t *ptr = nullptr, *col = nullptr;
    int32_t *sptr = nullptr, *scol = nullptr;  // the CSR expansion (scalar)
    double *val = nullptr, *tmp = nullptr;
    void *buf = nullptr;

    ~Rsr() {
        if (buf) (void)hipFree(buf);
        if (sptr) (void)hipFree(sptr);
        if (scol) (void)hipFree(scol);
        if (val) (void)hipFree(val);
        if (tmp) (void)hipFree(tmp);
        if (info) rocsparse_destroy_mat_info(info);
        if (dM) rocsparse_destroy_mat_descr(dM);
        if (dL) rocsparse_destroy_mat_descr(dL);
        if (dU) rocsparse_destroy_mat_descr(dU);
        if (handle) rocsparse_destroy_handle(handle);
    }
};

}  // namespace

#define RS(x)                                                                      \
    do {                                                                           \
        rocsparse_status s_ = (x);                                                 \
        if (s_ != rocsparse_status_success) {                                      \
            delete h;                                                              \
            return fail("%s: rocsparse status %d", #x, (int)s_);                  \
        }                                                                          \
    } while (0)
#define HP(x)                                                                      \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            delete h;                                                              \
            return fail("%s: %s", #x, hipGetErrorString(e_));                     \
        }                                                                          \
    } while (0)

extern "C" {

const char *rsr_last_error() { return g_err.c_str(); }

int rsr_create(int32_t mb, int32_t nnzb, int32_t bs, const int32_t *ptr, const int32_t *col, const double *val,
               void *stream, void **out) {
    if (!out || mb <= 0 || nnzb <= 0 || bs <= 0 || !ptr || !col || !val) return fail("rsr_create: bad arguments");
    *out = nullptr;
    Rsr *h = new Rsr;
    h->mb = mb;
    h->nnzb = nnzb;
    h->bs = bs;
    h->ptr = ptr;
    h->col = col;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t nval = (size_t)nnzb * bs * bs;
    HP(hipMalloc(&h->val, nval * sizeof(double)));
    HP(hipMalloc(&h->tmp, (size_t)mb * bs * sizeof(double)));
    HP(hipMemcpyAsync(h->val, val, nval * sizeof(double), hipMemcpyDeviceToDevice, st));
    RS(rocsparse_create_handle(&h->handle));
    RS(rocsparse_set_stream(h->handle, st));
    RS(rocsparse_create_mat_descr(&h->dM));
    RS(rocsparse_create_mat_descr(&h->dL));
    RS(rocsparse_set_mat_fill_mode(h->dL, rocsparse_fill_mode_lower));
    RS(rocsparse_set_mat_diag_type(h->dL, rocsparse_diag_type_unit));
    RS(rocsparse_create_mat_descr(&h->dU));
    RS(rocsparse_set_mat_fill_mode(h->dU, rocsparse_fill_mode_upper));
    RS(rocsparse_set_mat_diag_type(h->dU, rocsparse_diag_type_non_unit));
    RS(rocsparse_create_mat_info(&h->info));
    const rocsparse_direction dir = rocsparse_direction_row;
    const rocsparse_operation none = rocsparse_operation_none;
    size_t s0 = 0, s1 = 0, s2 = 0;
    RS(rocsparse_dbsrilu0_buffer_size(h->handle, dir, mb, nnzb, h->dM, h->val, ptr, col, bs, h->info, &s0));
    RS(rocsparse_dbsrsv_buffer_size(h->handle, dir, none, mb, nnzb, h->dL, h->val, ptr, col, bs, h->info, &s1));
    RS(rocsparse_dbsrsv_buffer_size(h->handle, dir, none, mb, nnzb, h->dU, h->val, ptr, col, bs, h->info, &s2));
    size_t sz = s0 > s1 ? s0 : s1;
    sz = sz > s2 ? sz : s2;
    HP(hipMalloc(&h->buf, sz > 0 ? sz : 1));
    RS(rocsparse_dbsrilu0_analysis(h->handle, dir, mb, nnzb, h->dM, h->val, ptr, col, bs, h->info,
                                   rocsparse_analysis_policy_reuse, rocsparse_solve_policy_auto, h->buf));
    RS(rocsparse_dbsrsv_analysis(h->handle, dir, none, mb, nnzb, h->dL, h->val, ptr, col, bs, h->info,
                                 rocsparse_analysis_policy_reuse, rocsparse_solve_policy_auto, h->buf));
    RS(rocsparse_dbsrsv_analysis(h->handle, dir, none, mb, nnzb, h->dU, h->val, ptr, col, bs, h->info,
                                 rocsparse_analysis_policy_reuse, rocsparse_solve_policy_auto, h->buf));
    RS(rocsparse_dbsrilu0(h->handle, dir, mb, nnzb, h->dM, h->val, ptr, col, bs, h->info,
                          rocsparse_solve_policy_auto, h->buf));
    rocsparse_int pos = -1;
    const rocsparse_status zp = rocsparse_bsrilu0_zero_pivot(h->handle, h->info, &pos);
    if (zp == rocsparse_status_zero_pivot) {
        delete h;
        return fail("rsr_create: zero pivot in block row %d", (int)pos);
    }
    RS(zp);
    HP(hipStreamSynchronize(st));
    *out = h;
    return 0;
}

int rsr_apply(void *hv, const double *r, double *z, void *stream) {
    Rsr *h = static_cast<Rsr *>(hv);
    if (!h || !r || !z || r == z) return fail("rsr_apply: bad arguments");
    if (rocsparse_set_stream(h->handle, static_cast<hipStream_t>(stream)) != rocsparse_status_success)
        return fail("rsr_apply: rocsparse_set_stream failed");
    const double one = 1.0;
    const rocsparse_direction dir = rocsparse_direction_row;
    const rocsparse_operation none = rocsparse_operation_none;
    if (h->scalar) {
        rocsparse_status s = rocsparse_dcsrsv_solve(h->handle, none, h->mb, h->nnzb, &one, h->dL, h->val, h->ptr,
                                                    h->col, h->info, r, h->tmp, rocsparse_solve_policy_auto, h->buf);
        if (s != rocsparse_status_success) return fail("rsr_apply: lower csrsv status %d", (int)s);
        s = rocsparse_dcsrsv_solve(h->handle, none, h->mb, h->nnzb, &one, h->dU, h->val, h->ptr, h->col, h->info,
                                   h->tmp, z, rocsparse_solve_policy_auto, h->buf);
        if (s != rocsparse_status_success) return fail("rsr_apply: upper csrsv status %d", (int)s);
        return 0;
    }
    rocsparse_status s = rocsparse_dbsrsv_solve(h->handle, dir, none, h->mb, h->nnzb, &one, h->dL, h->val, h->ptr,
                                                h->col, h->bs, h->info, r, h->tmp, rocsparse_solve_policy_auto,
                                                h->buf);
    if (s != rocsparse_status_success) return fail("rsr_apply: lower bsrsv status %d", (int)s);
    s = rocsparse_dbsrsv_solve(h->handle, dir, none, h->mb, h->nnzb, &one, h->dU, h->val, h->ptr, h->col, h->bs,
                               h->info, h->tmp, z, rocsparse_solve_policy_auto, h->buf);
    if (s != rocsparse_status_success) return fail("rsr_apply: upper bsrsv status %d", (int)s);
    return 0;
}

int rsr_create_scalar(int32_t mb, int32_t nnzb, int32_t bs, const int32_t *ptr, const int32_t *col,
                      const double *val, void *stream, void **out) {
    if (!out || mb <= 0 || nnzb <= 0 || bs <= 0 || !ptr || !col || !val) return fail("rsr_create_scalar: bad arguments");
    if ((int64_t)nnzb * bs * bs > INT32_MAX || (int64_t)mb * bs > INT32_MAX)
        return fail("rsr_create_scalar: the CSR expansion exceeds 32-bit indices");
    *out = nullptr;
    Rsr *h = new Rsr;
    h->scalar = true;
    h->mb = mb * bs;           // scalar rows
    h->nnzb = nnzb * bs * bs;  // scalar nonzeros
    h->bs = 1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t m = h->mb, nnz = h->nnzb;
    HP(hipMalloc(&h->val, (size_t)nnz * sizeof(double)));
    HP(hipMalloc(&h->sptr, (size_t)(m + 1) * sizeof(int32_t)));
    HP(hipMalloc(&h->scol, (size_t)nnz * sizeof(int32_t)));
    HP(hipMalloc(&h->tmp, (size_t)m * sizeof(double)));
    h->ptr = h->sptr;
    h->col = h->scol;
    RS(rocsparse_create_handle(&h->handle));
    RS(rocsparse_set_stream(h->handle, st));
    RS(rocsparse_create_mat_descr(&h->dM));
    RS(rocsparse_create_mat_descr(&h->dL));
    RS(rocsparse_set_mat_fill_mode(h->dL, rocsparse_fill_mode_lower));
    RS(rocsparse_set_mat_diag_type(h->dL, rocsparse_diag_type_unit));
    RS(rocsparse_create_mat_descr(&h->dU));
    RS(rocsparse_set_mat_fill_mode(h->dU, rocsparse_fill_mode_upper));
    RS(rocsparse_set_mat_diag_type(h->dU, rocsparse_diag_type_non_unit));
    RS(rocsparse_create_mat_info(&h->info));
    RS(rocsparse_dbsr2csr(h->handle, rocsparse_direction_row, mb, mb, h->dM, val, ptr, col, bs, h->dM, h->val,
                          h->sptr, h->scol));
    const rocsparse_operation none = rocsparse_operation_none;
    size_t s0 = 0, s1 = 0, s2 = 0;
    RS(rocsparse_dcsrilu0_buffer_size(h->handle, m, nnz, h->dM, h->val, h->sptr, h->scol, h->info, &s0));
    RS(rocsparse_dcsrsv_buffer_size(h->handle, none, m, nnz, h->dL, h->val, h->sptr, h->scol, h->info, &s1));
    RS(rocsparse_dcsrsv_buffer_size(h->handle, none, m, nnz, h->dU, h->val, h->sptr, h->scol, h->info, &s2));
    size_t sz = s0 > s1 ? s0 : s1;
    sz = sz > s2 ? sz : s2;
    HP(hipMalloc(&h->buf, sz > 0 ? sz : 1));
    RS(rocsparse_dcsrilu0_analysis(h->handle, m, nnz, h->dM, h->val, h->sptr, h->scol, h->info,
                                   rocsparse_analysis_policy_reuse, rocsparse_solve_policy_auto, h->buf));
    RS(rocsparse_dcsrsv_analysis(h->handle, none, m, nnz, h->dL, h->val, h->sptr, h->scol, h->info,
                                 rocsparse_analysis_policy_reuse, rocsparse_solve_policy_auto, h->buf));
    RS(rocsparse_dcsrsv_analysis(h->handle, none, m, nnz, h->dU, h->val, h->sptr, h->scol, h->info,
                                 rocsparse_analysis_policy_reuse, rocsparse_solve_policy_auto, h->buf));
    RS(rocsparse_dcsrilu0(h->handle, m, nnz, h->dM, h->val, h->sptr, h->scol, h->info, rocsparse_solve_policy_auto,
                          h->buf));
    rocsparse_int pos = -1;
    const rocsparse_status zp = rocsparse_csrilu0_zero_pivot(h->handle, h->info, &pos);
    if (zp == rocsparse_status_zero_pivot) {
        delete h;
        return fail("rsr_create_scalar: zero pivot in row %d", (int)pos);
    }
    RS(zp);
    HP(hipStreamSynchronize(st));
    *out = h;
    return 0;
}

void rsr_destroy(void *hv) { delete static_cast<Rsr *>(hv); }

}  // extern "C"
