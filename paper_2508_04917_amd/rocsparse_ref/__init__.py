"""ctypes binding of the rocSPARSE baseline (``librocsparse_ref.so``, built
by ``paper_2508_04917_amd.build``): rocSPARSE's block ILU0 and its two block
triangular solves on a BSR matrix already on the device, as the vendor
reference the paper compares its apply against (Section 5.2, Table 4).  Used by
``bench.py --mode rocsparse`` and its parity test only."""

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librocsparse_ref.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2508_04917_amd.build first")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.rsr_create.restype = C.c_int
        L.rsr_create.argtypes = [i32, i32, i32, vp, vp, vp, vp, C.POINTER(vp)]
        L.rsr_create_scalar.restype = C.c_int
        L.rsr_create_scalar.argtypes = [i32, i32, i32, vp, vp, vp, vp, C.POINTER(vp)]
        L.rsr_apply.restype = C.c_int
        L.rsr_apply.argtypes = [vp, vp, vp, vp]
        L.rsr_destroy.restype = None
        L.rsr_destroy.argtypes = [vp]
        L.rsr_last_error.restype = C.c_char_p
        L.rsr_last_error.argtypes = []
        _lib = L
    return _lib


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class RocsparseILU0:
    """rocSPARSE block ILU0 of the BSR matrix (ptr, col, val: int32, int32,
    float64 device tensors, blocks row-major).  The factorisation works on a
    copy of val; ptr and col are referenced, so this object keeps them.
    scalar=True expands the matrix to CSR and uses rocSPARSE's scalar ILU0
    and triangular solves instead (the same preconditioner on a pattern of
    dense blocks)."""

    def __init__(self, mb, bs, ptr, col, val, stream=None, scalar=False):
        import torch
        self._torch = torch
        self.mb, self.bs = int(mb), int(bs)
        self.ptr = ptr.to(torch.int32).contiguous()
        self.col = col.to(torch.int32).contiguous()
        val = val.to(torch.float64).contiguous()
        self.nnzb = int(self.col.numel())
        h = C.c_void_p()
        create = lib().rsr_create_scalar if scalar else lib().rsr_create
        rc = create(self.mb, self.nnzb, self.bs, self.ptr.data_ptr(), self.col.data_ptr(),
                    val.data_ptr(), _stream(torch, stream), C.byref(h))
        if rc != 0:
            raise RuntimeError(lib().rsr_last_error().decode())
        self.h = h

    def apply(self, r, z=None, stream=None):
        if z is None:
            z = self._torch.empty_like(r)
        rc = lib().rsr_apply(self.h, r.data_ptr(), z.data_ptr(), _stream(self._torch, stream))
        if rc != 0:
            raise RuntimeError(lib().rsr_last_error().decode())
        return z

    def close(self):
        if self.h:
            lib().rsr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dropped_matrix(ptr, col, val, S, bs):
    """The blocks (I, J) of a reordered BSR matrix with I and J in the same
    subdomain of S consecutive block rows (Section 3.2), as (ptr, col, val)
    device tensors; the order inside each row is kept."""
    import torch
    n = ptr.numel() - 1
    counts = (ptr[1:] - ptr[:-1]).long()
    rows = torch.repeat_interleave(torch.arange(n, device=ptr.device, dtype=torch.int64), counts)
    keep = (rows // S) == (col.long() // S)
    kept = torch.zeros(n, dtype=torch.int64, device=ptr.device).index_add_(0, rows[keep], torch.ones_like(rows[keep]))
    ptr_t = torch.zeros(n + 1, dtype=torch.int32, device=ptr.device)
    ptr_t[1:] = torch.cumsum(kept, 0).to(torch.int32)
    return ptr_t, col[keep].contiguous(), val.view(-1, bs * bs)[keep].reshape(-1).contiguous()


def level_order(ptr, col):
    """A renumbering (new -> old, int64 device tensor) that sorts the block
    rows by their level in the lower triangle (a row's level is one more than
    the largest level among the rows it couples to with a smaller number;
    ties keep the old order).  Every coupled pair keeps its relative order,
    so the ILU0 factors of the renumbered matrix are those of the original,
    renumbered (equal up to the order of rounding); only the order in which a
    triangular solve meets the rows changes."""
    import torch
    n = ptr.numel() - 1
    counts = (ptr[1:] - ptr[:-1]).long()
    rows = torch.repeat_interleave(torch.arange(n, device=ptr.device, dtype=torch.int64), counts)
    cols = col.long()
    low = cols < rows
    rows, cols = rows[low], cols[low]
    lev = torch.zeros(n, dtype=torch.int64, device=ptr.device)
    while True:  # longest path from the rows without lower couplings: one sweep per level
        nxt = lev.scatter_reduce(0, rows, lev[cols] + 1, reduce="amax", include_self=True)
        if torch.equal(nxt, lev):
            break
        lev = nxt
    return torch.sort(lev, stable=True).indices


def permuted_matrix(ptr, col, val, new2old, bs):
    """P A P^T of a BSR matrix for the renumbering new2old (block row i of
    the result is block row new2old[i] of A), columns sorted in every row."""
    import torch
    n = ptr.numel() - 1
    old2new = torch.empty_like(new2old)
    old2new[new2old] = torch.arange(n, device=ptr.device, dtype=new2old.dtype)
    counts = (ptr[1:] - ptr[:-1]).long()
    rows = torch.repeat_interleave(torch.arange(n, device=ptr.device, dtype=torch.int64), counts)
    nr, nc = old2new[rows], old2new[col.long()]
    order = torch.sort(nr * n + nc).indices
    ptr_p = torch.zeros(n + 1, dtype=torch.int32, device=ptr.device)
    ptr_p[1:] = torch.cumsum(counts[new2old], 0).to(torch.int32)
    return ptr_p, nc[order].to(torch.int32), val.view(-1, bs * bs)[order].reshape(-1).contiguous()
