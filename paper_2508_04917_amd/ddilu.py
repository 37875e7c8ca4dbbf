"""Python binding of the ddilu C ABI (include/ddilu.h).

Argument marshalling only: every function here forwards torch tensors'
device pointers and the current HIP stream to the library of the same name;
all computation runs in the library's kernels.  torch provides device
memory and streams.  There is no fallback: if libddilu.so is missing or fails
to load, every call raises.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddilu.so")

DD_OK, DD_EINVAL, DD_ENOTDIV, DD_ELDS, DD_EZEROPIVOT = 0, -1, -2, -3, -4
DD_EBREAKDOWN, DD_ENOCONV, DD_EHIP, DD_ENOMEM, DD_ESTATE = -5, -6, -7, -8, -9
DD_FP64, DD_FP32, DD_MIXED = 0, 1, 2

STATUS_NAMES = {0: "DD_OK", -1: "DD_EINVAL", -2: "DD_ENOTDIV", -3: "DD_ELDS", -4: "DD_EZEROPIVOT",
                -5: "DD_EBREAKDOWN", -6: "DD_ENOCONV", -7: "DD_EHIP", -8: "DD_ENOMEM", -9: "DD_ESTATE"}

# every symbol include/ddilu.h declares
EXPORTS = ("dd_auto_subdims", "dd_device_caps", "dd_partition", "dd_partition_graph", "dd_get_info", "dd_get_partition",
           "dd_get_reordered", "ilu0_factor", "ilu0_refactor", "dd_set_precision", "dd_get_levels", "dd_get_factors",
           "dd_trsv_apply", "dd_spmv", "bicgstab_solve", "bicgstab_solve_noalloc", "dd_set_apply_variant", "dd_set_fusion", "dd_set_lic_fallback",
           "dd_set_profiling",
           "dd_set_residual_history", "dd_global_factor", "dd_global_apply", "dd_set_preconditioner",
           "lic_setup", "lic_get_faces", "lic_set_params", "lic_set_coeffs", "lic_get_coeffs",
           "dd_apply_adjoint", "lic_targets", "lic_loss_grad", "lic_adam", "lic_train",
           "dd_last_error", "dd_destroy")

LIC_NPARAM = 6537


class PartitionDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bs", C.c_int32),
                ("sx", C.c_int32), ("sy", C.c_int32), ("sz", C.c_int32), ("n_cu", C.c_int32),
                ("lds_budget_bytes", C.c_int64)]


class GraphDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("bs", C.c_int32), ("part_rows", C.c_int32),
                ("lds_budget_bytes", C.c_int64), ("n_cu", C.c_int32), ("reserved", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnzb", C.c_int64), ("nnzb_dropped", C.c_int64),
                ("nnzb_lower", C.c_int64), ("nnzb_upper", C.c_int64),
                ("bs", C.c_int32), ("S", C.c_int32), ("nsub", C.c_int32),
                ("sx", C.c_int32), ("sy", C.c_int32), ("sz", C.c_int32),
                ("level_ptr_len", C.c_int32 * 2), ("max_levels", C.c_int32 * 2),
                ("factored", C.c_int32), ("precision", C.c_int32),
                ("apply_bytes", C.c_int64), ("lds_bytes", C.c_int64),
                ("max_row_blocks", C.c_int32), ("spmv_layout", C.c_int32), ("apply_layout", C.c_int32),
                ("seg_blocks", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double),
                ("rel_res_true", C.c_double), ("solve_seconds", C.c_double),
                ("applies", C.c_int32), ("restarts", C.c_int32), ("apply_seconds", C.c_double),
                ("fused", C.c_int32), ("fallback", C.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (run python -m paper_2508_04917_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "dd_auto_subdims": (C.c_int, [i32, i32, i32, i32, i64, i32, vp]),
            "dd_device_caps": (C.c_int, [vp, vp]),
            "dd_partition": (C.c_int, [C.POINTER(PartitionDesc), vp, vp, vp, i64, vp, C.POINTER(vp)]),
            "dd_partition_graph": (C.c_int, [C.POINTER(GraphDesc), vp, vp, vp, i64, vp, C.POINTER(vp)]),
            "dd_get_info": (C.c_int, [vp, C.POINTER(Info)]),
            "dd_get_partition": (C.c_int, [vp, vp, vp, vp, vp]),
            "dd_get_reordered": (C.c_int, [vp, vp, vp, vp, vp]),
            "ilu0_factor": (C.c_int, [vp, i32, vp]),
            "ilu0_refactor": (C.c_int, [vp, vp, vp]),
            "dd_set_precision": (C.c_int, [vp, i32, vp]),
            "dd_get_levels": (C.c_int, [vp, i32, vp, vp, vp, vp]),
            "dd_get_factors": (C.c_int, [vp, vp, vp, vp, vp]),
            "dd_trsv_apply": (C.c_int, [vp, vp, vp, vp]),
            "dd_spmv": (C.c_int, [vp, vp, vp, vp]),
            "bicgstab_solve": (C.c_int, [vp, vp, vp, C.c_double, i32, vp, C.POINTER(SolveInfo)]),
            "bicgstab_solve_noalloc": (C.c_int, [vp, vp, vp, C.c_double, i32, vp, C.POINTER(SolveInfo)]),
            "dd_set_apply_variant": (C.c_int, [vp, i32]),
            "dd_set_fusion": (C.c_int, [vp, i32]),
            "dd_set_lic_fallback": (C.c_int, [vp, i32]),
            "dd_set_profiling": (C.c_int, [vp, i32]),
            "dd_set_residual_history": (C.c_int, [vp, vp, i32]),
            "dd_global_factor": (C.c_int, [vp, vp]),
            "dd_global_apply": (C.c_int, [vp, vp, vp, i32, vp]),
            "dd_set_preconditioner": (C.c_int, [vp, i32]),
            "lic_setup": (C.c_int, [vp, vp]),
            "lic_get_faces": (C.c_int, [vp, vp, vp, vp, vp, vp]),
            "lic_set_params": (C.c_int, [vp, vp, vp]),
            "lic_set_coeffs": (C.c_int, [vp, vp, vp]),
            "lic_get_coeffs": (C.c_int, [vp, vp, vp]),
            "dd_apply_adjoint": (C.c_int, [vp, vp, vp, vp]),
            "lic_targets": (C.c_int, [vp, i32, vp, vp, vp, vp]),
            "lic_loss_grad": (C.c_int, [vp, vp, i32, vp, vp, vp, vp, vp, i32, vp]),
            "lic_adam": (C.c_int, [vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp]),
            "lic_train": (C.c_int, [vp, i32, vp, vp, vp, i32, vp, vp, vp, i32, vp, C.c_float, i32, vp, vp]),
            "dd_last_error": (C.c_char_p, [vp]),
            "dd_destroy": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int, h=None):
    if rc != DD_OK:
        raise DDError(rc, dd_last_error(h))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_check(t, dtype, numel, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == numel):
        raise ValueError(f"{name}: expected a contiguous {dtype} CUDA tensor of {numel} elements")


def _vecs(h, count, **named):
    """FP64 device vectors of count * n * bs values each (the library reads
    and writes exactly that many through the raw pointers)."""
    for name, t in named.items():
        _dev_check(t, torch.float64, count * h.m, name)


class Handle:
    """Owns a dd_handle; released by close() or garbage collection."""

    def __init__(self, ptr: int):
        self.ptr = C.c_void_p(ptr)

    def close(self):
        if self.ptr:
            lib().dd_destroy(self.ptr)
            self.ptr = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        return dd_get_info(self)

    @property
    def m(self) -> int:
        """Length n*bs of the handle's vectors (cached)."""
        if getattr(self, "_m", None) is None:
            i = dd_get_info(self)
            self._m = int(i["n"]) * int(i["bs"])
        return self._m


def dd_last_error(h=None) -> str:
    s = lib().dd_last_error(h.ptr if h is not None else None)
    return s.decode() if s else ""


def dd_auto_subdims(nx, ny, nz, bs, lds_budget_bytes, n_cu):
    out = (C.c_int32 * 3)()
    _check(lib().dd_auto_subdims(nx, ny, nz, bs, lds_budget_bytes, n_cu, out))
    return tuple(out)


def dd_device_caps():
    cu = C.c_int32(0)
    lds = C.c_int64(0)
    _check(lib().dd_device_caps(C.byref(cu), C.byref(lds)))
    return cu.value, lds.value


def dd_partition(nx, ny, nz, bs, brow_ptr, bcol, val, sub=(0, 0, 0), n_cu=0, lds_budget_bytes=0,
                 stream=None) -> Handle:
    n = nx * ny * nz
    nnzb = bcol.numel()
    _dev_check(brow_ptr, torch.int32, n + 1, "brow_ptr")
    _dev_check(bcol, torch.int32, nnzb, "bcol")
    _dev_check(val, torch.float64, nnzb * bs * bs, "val")
    d = PartitionDesc(nx, ny, nz, bs, sub[0], sub[1], sub[2], n_cu, lds_budget_bytes)
    out = C.c_void_p(None)
    _check(lib().dd_partition(C.byref(d), _ptr(brow_ptr), _ptr(bcol), _ptr(val), nnzb, _stream(stream),
                              C.byref(out)))
    return Handle(out.value)


def dd_partition_graph(n, bs, brow_ptr, bcol, val, part_rows=0, lds_budget_bytes=0, n_cu=0,
                       stream=None) -> Handle:
    """Partition a matrix graph without geometry (recursive BFS bisection
    into parts of part_rows vertices; 0 = the divisor of n that fits the LDS
    and leaves each compute unit the fewest rows to apply), then reorder as
    dd_partition does."""
    nnzb = bcol.numel()
    _dev_check(brow_ptr, torch.int32, n + 1, "brow_ptr")
    _dev_check(bcol, torch.int32, nnzb, "bcol")
    _dev_check(val, torch.float64, nnzb * bs * bs, "val")
    d = GraphDesc(n, bs, part_rows, lds_budget_bytes, n_cu, 0)
    out = C.c_void_p(None)
    _check(lib().dd_partition_graph(C.byref(d), _ptr(brow_ptr), _ptr(bcol), _ptr(val), nnzb, _stream(stream),
                                    C.byref(out)))
    return Handle(out.value)


def dd_get_info(h: Handle) -> dict:
    inf = Info()
    _check(lib().dd_get_info(h.ptr, C.byref(inf)), h)
    d = {k: getattr(inf, k) for k, _ in Info._fields_}
    d["level_ptr_len"] = tuple(inf.level_ptr_len)
    d["max_levels"] = tuple(inf.max_levels)
    return d


def _i32(n, device="cuda"):
    return torch.empty(n, dtype=torch.int32, device=device)


def dd_get_partition(h: Handle, stream=None):
    n = dd_get_info(h)["n"]
    pid, n2o, o2n = _i32(n), _i32(n), _i32(n)
    _check(lib().dd_get_partition(h.ptr, _ptr(pid), _ptr(n2o), _ptr(o2n), _stream(stream)), h)
    return pid, n2o, o2n


def dd_get_reordered(h: Handle, stream=None):
    inf = dd_get_info(h)
    n, nnzb, bs = inf["n"], inf["nnzb"], inf["bs"]
    ptr, col = _i32(n + 1), _i32(nnzb)
    val = torch.empty(nnzb * bs * bs, dtype=torch.float64, device="cuda")
    _check(lib().dd_get_reordered(h.ptr, _ptr(ptr), _ptr(col), _ptr(val), _stream(stream)), h)
    return ptr, col, val


def ilu0_factor(h: Handle, precision=DD_FP64, stream=None):
    _check(lib().ilu0_factor(h.ptr, precision, _stream(stream)), h)


def ilu0_refactor(h: Handle, val, stream=None):
    """New values (CUDA float64, the partitioned matrix's blocks in the order
    given to dd_partition) on the handle's pattern."""
    info = dd_get_info(h)
    _dev_check(val, torch.float64, int(info["nnzb"]) * int(info["bs"]) ** 2, "val")
    _check(lib().ilu0_refactor(h.ptr, _ptr(val), _stream(stream)), h)


def dd_set_precision(h: Handle, precision, stream=None):
    _check(lib().dd_set_precision(h.ptr, precision, _stream(stream)), h)


def dd_get_levels(h: Handle, which: int, stream=None):
    inf = dd_get_info(h)
    nlev = _i32(inf["nsub"])
    lptr = _i32(inf["level_ptr_len"][which])
    rows = _i32(inf["n"])
    _check(lib().dd_get_levels(h.ptr, which, _ptr(nlev), _ptr(lptr), _ptr(rows), _stream(stream)), h)
    return nlev, lptr, rows


def dd_get_factors(h: Handle, stream=None):
    inf = dd_get_info(h)
    n, m, bs = inf["n"], inf["nnzb_dropped"], inf["bs"]
    ptr, col = _i32(n + 1), _i32(m)
    f = torch.empty(m * bs * bs, dtype=torch.float64, device="cuda")
    _check(lib().dd_get_factors(h.ptr, _ptr(ptr), _ptr(col), _ptr(f), _stream(stream)), h)
    return ptr, col, f


def dd_trsv_apply(h: Handle, r, z=None, stream=None):
    if z is None:
        z = torch.empty_like(r)
    _vecs(h, 1, r=r, z=z)
    _check(lib().dd_trsv_apply(h.ptr, _ptr(r), _ptr(z), _stream(stream)), h)
    return z


def dd_spmv(h: Handle, x, y=None, stream=None):
    if y is None:
        y = torch.empty_like(x)
    _vecs(h, 1, x=x, y=y)
    _check(lib().dd_spmv(h.ptr, _ptr(x), _ptr(y), _stream(stream)), h)
    return y


def bicgstab_solve(h: Handle, b, x=None, rtol=1e-8, maxit=10000, stream=None):
    """Returns (x, info).  info['status'] is DD_OK, DD_EBREAKDOWN or DD_ENOCONV;
    other failures raise."""
    if x is None:
        x = torch.zeros_like(b)
    _vecs(h, 1, b=b, x=x)
    si = SolveInfo()
    rc = lib().bicgstab_solve(h.ptr, _ptr(b), _ptr(x), rtol, maxit, _stream(stream), C.byref(si))
    if rc not in (DD_OK, DD_EBREAKDOWN, DD_ENOCONV):
        raise DDError(rc, dd_last_error(h))
    return x, {k: getattr(si, k) for k, _ in SolveInfo._fields_}


def bicgstab_solve_noalloc(h: Handle, b, x, rtol=1e-8, maxit=10000, stream=None):
    """bicgstab_solve with the library's fixed workspace (no device
    allocation in the call; x must be given).  Returns (x, info)."""
    _vecs(h, 1, b=b, x=x)
    si = SolveInfo()
    rc = lib().bicgstab_solve_noalloc(h.ptr, _ptr(b), _ptr(x), rtol, maxit, _stream(stream), C.byref(si))
    if rc not in (DD_OK, DD_EBREAKDOWN, DD_ENOCONV):
        raise DDError(rc, dd_last_error(h))
    return x, {k: getattr(si, k) for k, _ in SolveInfo._fields_}


def dd_set_apply_variant(h: Handle, variant: int):
    _check(lib().dd_set_apply_variant(h.ptr, variant), h)


def dd_set_fusion(h: Handle, on: bool):
    _check(lib().dd_set_fusion(h.ptr, 1 if on else 0), h)


def dd_set_lic_fallback(h: Handle, on: bool):
    _check(lib().dd_set_lic_fallback(h.ptr, 1 if on else 0), h)


def dd_set_profiling(h: Handle, on: bool):
    _check(lib().dd_set_profiling(h.ptr, 1 if on else 0), h)


def dd_set_residual_history(h: Handle, hist):
    """hist: CUDA float64 tensor (or None to stop recording)."""
    if hist is None:
        _check(lib().dd_set_residual_history(h.ptr, None, 0), h)
    else:
        _dev_check(hist, torch.float64, hist.numel(), "hist")
        _check(lib().dd_set_residual_history(h.ptr, _ptr(hist), hist.numel()), h)


def dd_destroy(h: Handle):
    h.close()


# ------------------------------------------------------------- global ILU0
def dd_global_factor(h: Handle, stream=None):
    _check(lib().dd_global_factor(h.ptr, _stream(stream)), h)


def dd_global_apply(h: Handle, r, z=None, nrhs=1, stream=None):
    if z is None:
        z = torch.empty_like(r)
    _vecs(h, nrhs, r=r, z=z)
    _check(lib().dd_global_apply(h.ptr, _ptr(r), _ptr(z), nrhs, _stream(stream)), h)
    return z


def dd_set_preconditioner(h: Handle, kind: int):
    """0: the domain-decomposed ILU0 apply; 1: the global ILU0 apply."""
    _check(lib().dd_set_preconditioner(h.ptr, kind), h)


# ------------------------------------------------------ learned correction
def lic_setup(h: Handle, stream=None):
    _check(lib().lic_setup(h.ptr, _stream(stream)), h)


def lic_get_faces(h: Handle, stream=None):
    nf = C.c_int32(0)
    _check(lib().lic_get_faces(h.ptr, C.byref(nf), None, None, None, _stream(stream)), h)
    m = nf.value
    fI, fJ = _i32(m), _i32(m)
    X = torch.empty(m * 27, dtype=torch.float32, device="cuda")
    _check(lib().lic_get_faces(h.ptr, C.byref(nf), _ptr(fI), _ptr(fJ), _ptr(X), _stream(stream)), h)
    return fI, fJ, X.view(m, 27)


def lic_set_params(h: Handle, params, stream=None):
    """params: CUDA float32 tensor of 6537 values, or None for the plain apply."""
    if params is not None:
        _dev_check(params, torch.float32, LIC_NPARAM, "params")
    _check(lib().lic_set_params(h.ptr, _ptr(params), _stream(stream)), h)


def lic_set_coeffs(h: Handle, coeffs, stream=None):
    if coeffs is not None and not (coeffs.is_cuda and coeffs.dtype == torch.float32 and coeffs.is_contiguous()):
        raise ValueError("coeffs: contiguous CUDA float32 tensor [nf, 3, 3]")
    _check(lib().lic_set_coeffs(h.ptr, _ptr(coeffs), _stream(stream)), h)


def lic_get_coeffs(h: Handle, nf: int, stream=None):
    out = torch.empty(nf * 9, dtype=torch.float32, device="cuda")
    _check(lib().lic_get_coeffs(h.ptr, _ptr(out), _stream(stream)), h)
    return out.view(nf, 3, 3)


def dd_apply_adjoint(h: Handle, g, a=None, stream=None):
    if a is None:
        a = torch.empty_like(g)
    _vecs(h, 1, g=g, a=a)
    _check(lib().dd_apply_adjoint(h.ptr, _ptr(g), _ptr(a), _stream(stream)), h)
    return a


def lic_targets(h: Handle, R, stream=None):
    """R: CUDA float64 [nq, 3n] probes.  Returns (Zs, den): global ILU0 applies
    and den_q = ||M_DD^{-1} r_q - Zs_q||^2."""
    nq = R.shape[0]
    _vecs(h, nq, R=R)
    Zs = torch.empty_like(R)
    den = torch.empty(nq, dtype=torch.float64, device="cuda")
    _check(lib().lic_targets(h.ptr, nq, _ptr(R), _ptr(Zs), _ptr(den), _stream(stream)), h)
    return Zs, den


def lic_loss_grad(h: Handle, params, R, Zs, den, loss=None, grad=None, accumulate=False, stream=None):
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    if grad is None:
        grad = torch.zeros(LIC_NPARAM, dtype=torch.float32, device="cuda")
    nq = R.shape[0]
    _vecs(h, nq, R=R, Zs=Zs)
    _dev_check(den, torch.float64, nq, "den")
    _dev_check(params, torch.float32, LIC_NPARAM, "params")
    _dev_check(grad, torch.float32, LIC_NPARAM, "grad")
    _dev_check(loss, torch.float64, 1, "loss")
    _check(lib().lic_loss_grad(h.ptr, _ptr(params), R.shape[0], _ptr(R), _ptr(Zs), _ptr(den), _ptr(loss),
                               _ptr(grad), 1 if accumulate else 0, _stream(stream)), h)
    return loss, grad


def lic_adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    _check(lib().lic_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), t, lr, b1, b2, eps,
                          _stream(stream)))


def lic_train(handles, Rs, Zss, dens, params, m, v, epochs, order, lr=1e-3, step0=0, stream=None):
    """One Adam step per problem, problems visited in order[epoch] (host
    int array epochs x nprob); step0 = Adam steps already taken with m, v.
    Returns the mean loss of every epoch."""
    import numpy as np
    nprob = len(handles)
    hs = (C.c_void_p * nprob)(*[h.ptr.value for h in handles])
    R = (C.c_void_p * nprob)(*[t.data_ptr() for t in Rs])
    Z = (C.c_void_p * nprob)(*[t.data_ptr() for t in Zss])
    D = (C.c_void_p * nprob)(*[t.data_ptr() for t in dens])
    order = np.ascontiguousarray(order, dtype=np.int32)
    hist = np.zeros(epochs)
    _check(lib().lic_train(hs, nprob, R, Z, D, Rs[0].shape[0], _ptr(params), _ptr(m), _ptr(v), epochs,
                           order.ctypes.data_as(C.c_void_p), lr, step0, hist.ctypes.data_as(C.c_void_p),
                           _stream(stream)))
    return hist
