"""CPU FP64 oracle (test infrastructure only).

A plain, slow, obviously correct statement of what the domain-decomposed
ILU0 path computes, used to check the GPU library.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package; the
GPU library never does, and this package never imports the GPU library.

The numerics live in ``oracle.c`` (plain sequential C loops, FP64), loaded
through ctypes; the thin wrappers here only allocate numpy arrays.  Each
function cites the part of arXiv 2508.04917 it follows.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB lets the mutation tests load a deliberately broken copy of the
# oracle (built from a mutated oracle.c) in a child process.
_LIB = os.environ.get("ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))

O_OK, O_EINVAL, O_ENOTDIV, O_EZEROPIVOT, O_EBREAKDOWN, O_ENOCONV = 0, -1, -2, -4, -5, -6


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
        )
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        i64, i32, vp = C.c_int64, C.c_int32, C.c_void_p
        sig = {
            "o_block_inverse": (C.c_int, [C.c_int, vp, vp]),
            "o_partition": (C.c_int, [C.c_int] * 6 + [vp]),
            "o_permutation": (C.c_int, [i64, i32, vp, vp, vp]),
            "o_graph_partition": (C.c_int, [i64, vp, vp, i32, vp]),
            "o_reorder": (C.c_int, [i64, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp]),
            "o_drop": (i64, [i64, C.c_int, i64, vp, vp, vp, vp, vp, vp]),
            "o_levels": (C.c_int, [i64, vp, vp, C.c_int, vp]),
            "o_level_lists": (i64, [i64, i64, vp, vp, vp, vp]),
            "o_bilu0": (C.c_int, [i64, C.c_int, vp, vp, vp, vp]),
            "o_ildu0": (C.c_int, [i64, C.c_int, vp, vp, vp, vp]),
            "o_apply": (None, [i64, C.c_int, vp, vp, vp, vp, vp]),
            "o_apply_ilu0": (C.c_int, [i64, C.c_int, vp, vp, vp, vp, vp]),
            "o_apply_transpose": (None, [i64, C.c_int, vp, vp, vp, vp, vp]),
            "o_spmv": (None, [i64, C.c_int, vp, vp, vp, vp, vp]),
            "o_bicgstab": (C.c_int, [i64, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp,
                                     C.c_double, i32, vp, vp, vp]),
            "o_lic_nparam": (i64, []),
            "o_cut_faces": (i64, [i64, i64, vp, vp, vp, vp, vp]),
            "o_lic_features": (None, [i64, vp, vp, vp, vp, vp, vp, vp]),
            "o_mlp_forward": (None, [i64, vp, vp, vp, vp, vp]),
            "o_mlp_backward": (None, [i64, vp, vp, vp, vp, vp, vp]),
            "o_lic_correct": (None, [i64, i64, vp, vp, vp, vp, vp]),
            "o_lic_dC": (None, [i64, i64, vp, vp, C.c_int, vp, vp, vp]),
            "o_adam": (None, [i64, vp, vp, vp, vp, C.c_int, C.c_double, C.c_double, C.c_double,
                              C.c_double]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


# ---------------------------------------------------------------- partition
def subdomain_count(nx, ny, nz, sx, sy, sz):
    return (nx // sx) * (ny // sy) * (nz // sz)


def auto_subdims(nx, ny, nz, bs, lds_budget_bytes, n_cu):
    """Automatic subdomain extents: the largest box whose FP64 vector
    (S*bs*8 bytes) fits one workgroup's LDS budget (Section 4: the subdomain
    is sized so that its vector data fits in shared memory).

    Candidates are divisor triples (sx|nx, sy|ny, sz|nz).  If some candidate
    gives at least n_cu subdomains, only those are kept (every compute unit
    gets work).  Then: largest S, then smallest surface sx*sy+sy*sz+sz*sx
    (fewest dropped couplings), then largest sz, then largest sy.
    Returns None when nothing fits.
    """
    def divs(m):
        return [d for d in range(1, m + 1) if m % d == 0]

    cands = []
    for sx in divs(nx):
        for sy in divs(ny):
            for sz in divs(nz):
                S = sx * sy * sz
                if S * bs * 8 <= lds_budget_bytes:
                    cands.append((sx, sy, sz))
    if not cands:
        return None
    full = [c for c in cands if subdomain_count(nx, ny, nz, *c) >= n_cu]
    if full:
        cands = full

    def key(c):
        sx, sy, sz = c
        return (-(sx * sy * sz), sx * sy + sy * sz + sz * sx, -sz, -sy)

    return min(cands, key=key)


def partition(nx, ny, nz, sx, sy, sz):
    """Section 3, Algorithm 2: part_id for every cell g = i + nx*(j + ny*k)."""
    out = np.empty(nx * ny * nz, dtype=np.int32)
    rc = lib().o_partition(nx, ny, nz, sx, sy, sz, _p(out))
    if rc:
        raise OracleError(rc, "partition")
    return out


def graph_partition(n, ptr, col, S):
    """Parts of exactly S vertices of the matrix graph, by recursive BFS
    bisection (no geometry; METIS stand-in, see o_graph_partition)."""
    ptr, col = _i32(ptr), _i32(col)
    pid = np.empty(n, dtype=np.int32)
    rc = lib().o_graph_partition(n, _p(ptr), _p(col), S, _p(pid))
    if rc:
        raise OracleError(rc, f"graph partition of {n} vertices into parts of {S}")
    return pid


def permutation(part_id, nsub):
    """Section 3.1: group rows by label, stable in the old index.
    Returns (new2old, old2new)."""
    part_id = _i32(part_id)
    n = part_id.shape[0]
    n2o = np.empty(n, dtype=np.int32)
    o2n = np.empty(n, dtype=np.int32)
    rc = lib().o_permutation(n, nsub, _p(part_id), _p(n2o), _p(o2n))
    if rc:
        raise OracleError(rc, "permutation")
    return n2o, o2n


def reorder(n, bs, ptr, col, val, new2old, old2new):
    """Section 3.1, Algorithm 3 in block form; val may be None (pattern only)."""
    ptr, col = _i32(ptr), _i32(col)
    nnzb = col.shape[0]
    optr = np.empty(n + 1, dtype=np.int32)
    ocol = np.empty(nnzb, dtype=np.int32)
    oval = None
    if val is not None:
        val = _f64(val)
        oval = np.empty_like(val)
    lib().o_reorder(n, bs, _p(ptr), _p(col), _p(val), _p(_i32(new2old)), _p(_i32(old2new)),
                    _p(optr), _p(ocol), _p(oval))
    return optr, ocol, oval


def drop(n, bs, S, ptr, col, val=None):
    """Section 3.2: keep block (I,J) iff I and J lie in the same S-row window."""
    ptr, col = _i32(ptr), _i32(col)
    if val is not None:
        val = _f64(val).reshape(-1, bs, bs)  # blocks row-major, whatever shape they came in
    m = lib().o_drop(n, bs, S, _p(ptr), _p(col), None, None, None, None)
    tptr = np.empty(n + 1, dtype=np.int32)
    tcol = np.empty(m, dtype=np.int32)
    tval = None if val is None else np.empty((m, bs, bs), dtype=np.float64)
    lib().o_drop(n, bs, S, _p(ptr), _p(col), _p(val), _p(tptr), _p(tcol), _p(tval))
    return tptr, tcol, tval


def count_after_drop(n, S, ptr, col):
    ptr, col = _i32(ptr), _i32(col)
    return int(lib().o_drop(n, 1, S, _p(ptr), _p(col), None, None, None, None))


# ------------------------------------------------------------------- levels
def levels(ptr, col, which):
    """Section 4.2.1: per-row longest-path level (which=0 lower, 1 upper)."""
    ptr, col = _i32(ptr), _i32(col)
    n = ptr.shape[0] - 1
    lev = np.empty(n, dtype=np.int32)
    rc = lib().o_levels(n, _p(ptr), _p(col), which, _p(lev))
    if rc:
        raise OracleError(rc, "levels")
    return lev


def level_lists(lev, S):
    """Section 4.2.2 explicit per-subdomain DAG: (nlev[nsub], level_ptr, level_rows)."""
    lev = _i32(lev)
    n = lev.shape[0]
    nsub = n // S
    nlev = np.empty(nsub, dtype=np.int32)
    lptr = np.empty(n + nsub, dtype=np.int32)
    rows = np.empty(n, dtype=np.int32)
    w = lib().o_level_lists(n, S, _p(lev), _p(nlev), _p(lptr), _p(rows))
    if w < 0:
        raise OracleError(int(w), "level_lists")
    return nlev, lptr[:w].copy(), rows


# ---------------------------------------------------------------- factorise
def bilu0(n, bs, ptr, col, val):
    """Section 4.3, Algorithm 5 (block IKJ ILU0); returns L\\U in val's pattern."""
    f = _f64(val).copy()
    bad = C.c_int64(-1)
    rc = lib().o_bilu0(n, bs, _p(_i32(ptr)), _p(_i32(col)), _p(f), C.byref(bad))
    if rc:
        raise OracleError(rc, f"zero pivot at block row {bad.value}")
    return f


def ildu0(n, bs, ptr, col, lu):
    """Section 4.3 ILDU0 post-pass: diagonal slot <- U_II^{-1}, upper <- inv_D U."""
    f = _f64(lu).copy()
    bad = C.c_int64(-1)
    rc = lib().o_ildu0(n, bs, _p(_i32(ptr)), _p(_i32(col)), _p(f), C.byref(bad))
    if rc:
        raise OracleError(rc, f"zero pivot at block row {bad.value}")
    return f


def block_inverse(A):
    A = _f64(A)
    bs = A.shape[0]
    out = np.empty_like(A)
    rc = lib().o_block_inverse(bs, _p(A), _p(out))
    if rc:
        raise OracleError(rc, "singular block")
    return out


# -------------------------------------------------------------------- apply
def apply(n, bs, ptr, col, f, r):
    """Sections 4.2.2 and 4.4: z = (L D Uhat)^{-1} r (forward, scale, backward)."""
    r = _f64(r)
    z = np.empty_like(r)
    lib().o_apply(n, bs, _p(_i32(ptr)), _p(_i32(col)), _p(_f64(f)), _p(r), _p(z))
    return z


def apply_ilu0(n, bs, ptr, col, lu, r):
    """Algorithm 7 form: division by U_II inside the backward row."""
    r = _f64(r)
    z = np.empty_like(r)
    rc = lib().o_apply_ilu0(n, bs, _p(_i32(ptr)), _p(_i32(col)), _p(_f64(lu)), _p(r), _p(z))
    if rc:
        raise OracleError(rc, "apply_ilu0")
    return z


def apply_transpose(n, bs, ptr, col, f, r):
    """z = M^{-T} r for M = L D Uhat."""
    r = _f64(r)
    z = np.empty_like(r)
    lib().o_apply_transpose(n, bs, _p(_i32(ptr)), _p(_i32(col)), _p(_f64(f)), _p(r), _p(z))
    return z


def spmv(n, bs, ptr, col, val, x):
    x = _f64(x)
    y = np.empty_like(x)
    lib().o_spmv(n, bs, _p(_i32(ptr)), _p(_i32(col)), _p(_f64(val)), _p(x), _p(y))
    return y


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    relres: float
    status: int
    history: np.ndarray


def bicgstab(n, bs, aptr, acol, aval, fptr, fcol, fval, b, rtol=1e-8, maxit=10000, x0=None):
    """Section 2, Algorithm 1 with K1 = I, K2 = M (right preconditioning)."""
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    hist = np.full(maxit + 1, np.nan)
    rc = lib().o_bicgstab(n, bs, _p(_i32(aptr)), _p(_i32(acol)), _p(_f64(aval)),
                          _p(_i32(fptr)), _p(_i32(fcol)), _p(_f64(fval)),
                          _p(b), _p(x), rtol, maxit, C.byref(it), C.byref(rr), _p(hist))
    return SolveResult(x, it.value, rr.value, rc, hist[: it.value + 1])


# --------------------------------------------------------- whole-path setup
@dataclass
class OracleSetup:
    n: int
    bs: int
    sub: tuple
    S: int
    nsub: int
    part_id: np.ndarray
    new2old: np.ndarray
    old2new: np.ndarray
    aptr: np.ndarray   # full reordered A
    acol: np.ndarray
    aval: np.ndarray
    tptr: np.ndarray   # dropped pattern A~
    tcol: np.ndarray
    tval: np.ndarray
    lu: np.ndarray     # L\U on A~
    f: np.ndarray      # L\inv_D\Uhat on A~ (ILDU0)

    def apply(self, r):
        return apply(self.n, self.bs, self.tptr, self.tcol, self.f, r)

    def apply_fp32_factors(self, r, round_input=True):
        """FP32-factor variants (an addition to the method; not in the paper): the FP64
        apply run with L, inv_D and Uhat rounded to FP32 (round to nearest
        even) and, when round_input, with r rounded to FP32 as well."""
        f32 = np.asarray(self.f, dtype=np.float64).astype(np.float32).astype(np.float64)
        r = np.asarray(r, dtype=np.float64)
        if round_input:
            r = r.astype(np.float32).astype(np.float64)
        return apply(self.n, self.bs, self.tptr, self.tcol, f32, r)

    def spmv(self, x):
        return spmv(self.n, self.bs, self.aptr, self.acol, self.aval, x)

    def levels(self, which):
        return level_lists(levels(self.tptr, self.tcol, which), self.S)

    def permute(self, v):
        """original order -> reordered (block rows)."""
        return np.asarray(v).reshape(self.n, self.bs)[self.new2old].reshape(-1)

    def unpermute(self, v):
        return np.asarray(v).reshape(self.n, self.bs)[self.old2new].reshape(-1)

    def bicgstab(self, b_orig, rtol=1e-8, maxit=10000):
        res = bicgstab(self.n, self.bs, self.aptr, self.acol, self.aval,
                       self.tptr, self.tcol, self.f, self.permute(b_orig), rtol, maxit)
        res.x = self.unpermute(res.x)
        return res


def setup(problem, sub):
    """Partition, reorder, drop, BILU0 and ILDU0 for a problem (problems.Problem)."""
    nx, ny, nz, bs = problem.nx, problem.ny, problem.nz, problem.bs
    sx, sy, sz = sub
    n = nx * ny * nz
    S = sx * sy * sz
    pid = partition(nx, ny, nz, sx, sy, sz)
    return _setup_from_labels(problem, n, bs, S, tuple(sub), pid)


def setup_graph(problem, S):
    """As setup, with the labels of graph_partition (parts of S vertices)."""
    n = problem.brow_ptr.shape[0] - 1
    pid = graph_partition(n, problem.brow_ptr, problem.bcol, S)
    return _setup_from_labels(problem, n, problem.bs, S, (S, 1, 1), pid)


def _setup_from_labels(problem, n, bs, S, sub, pid):
    nsub = n // S
    n2o, o2n = permutation(pid, nsub)
    aptr, acol, aval = reorder(n, bs, problem.brow_ptr, problem.bcol, problem.val, n2o, o2n)
    tptr, tcol, tval = drop(n, bs, S, aptr, acol, aval)
    lu = bilu0(n, bs, tptr, tcol, tval)
    f = ildu0(n, bs, tptr, tcol, lu)
    return OracleSetup(n, bs, tuple(sub), S, nsub, pid, n2o, o2n, aptr, acol, aval,
                       tptr, tcol, tval, lu, f)


# ------------------------------------------ learned interface correction
# An addition to the paper's method (the paper has no learned component):
# a per-face MLP 27 -> 64 -> 64 -> 9 maps scale-normalised local blocks
# [A_II, A_IJ, A_JJ] of each cut face (I, J) to a 3x3 C_f, and the
# preconditioner becomes z = M_DD^{-1} (r + C r).  It is trained by
# regression onto the global ILU0 apply (the same reordered matrix without
# the drop) on probe vectors.
LIC_NPARAM = 6537


def cut_faces(n, S, ptr, col):
    """Directed cut pairs (I, J) = the dropped blocks, CSR order: (fI, fJ, fq)."""
    ptr, col = _i32(ptr), _i32(col)
    m = lib().o_cut_faces(n, S, _p(ptr), _p(col), None, None, None)
    fI, fJ, fq = (np.empty(m, dtype=np.int32) for _ in range(3))
    lib().o_cut_faces(n, S, _p(ptr), _p(col), _p(fI), _p(fJ), _p(fq))
    return fI, fJ, fq


def lic_features(ptr, col, val, faces):
    fI, fJ, fq = faces
    X = np.empty((fI.shape[0], 27))
    lib().o_lic_features(fI.shape[0], _p(_i32(ptr)), _p(_i32(col)), _p(_f64(val)), _p(fI), _p(fJ),
                         _p(fq), _p(X))
    return X


def mlp_forward(P, X):
    P, X = _f64(P), _f64(X)
    nf = X.shape[0]
    H1, H2, OUT = np.empty((nf, 64)), np.empty((nf, 64)), np.empty((nf, 9))
    lib().o_mlp_forward(nf, _p(P), _p(X), _p(H1), _p(H2), _p(OUT))
    return H1, H2, OUT


def mlp_backward(P, X, H1, H2, dOUT):
    dP = np.zeros(LIC_NPARAM)
    lib().o_mlp_backward(X.shape[0], _p(_f64(P)), _p(_f64(X)), _p(_f64(H1)), _p(_f64(H2)),
                         _p(_f64(dOUT)), _p(dP))
    return dP


def lic_correct(n, faces, C, r):
    fI, fJ, _ = faces
    r = _f64(r)
    rt = np.empty_like(r)
    lib().o_lic_correct(n, fI.shape[0], _p(fI), _p(fJ), _p(_f64(C)), _p(r), _p(rt))
    return rt


def lic_dC(n, faces, A, R):
    fI, fJ, _ = faces
    A, R = _f64(A), _f64(R)
    dC = np.empty((fI.shape[0], 3, 3))
    lib().o_lic_dC(n, fI.shape[0], _p(fI), _p(fJ), A.shape[0], _p(A), _p(R), _p(dC))
    return dC


def adam(P, G, M, V, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on P, M, V (float64 arrays)."""
    lib().o_adam(P.shape[0], _p(P), _p(_f64(G)), _p(M), _p(V), t, lr, b1, b2, eps)


class LicOracle:
    """Learned-correction pieces on one problem's oracle setup."""

    def __init__(self, st: "OracleSetup"):
        if st.bs != 3:
            raise ValueError("the learned correction is defined for 3x3 blocks")
        self.st = st
        self.faces = cut_faces(st.n, st.S, st.aptr, st.acol)
        self.X = lic_features(st.aptr, st.acol, st.aval, self.faces)
        self._glob = None

    @property
    def nf(self):
        return self.faces[0].shape[0]

    def coeffs(self, P):
        return mlp_forward(P, self.X)[2].reshape(-1, 3, 3)

    def apply(self, C, r):
        """z = M_DD^{-1} (r + C r)."""
        return self.st.apply(lic_correct(self.st.n, self.faces, C, r))

    def global_factors(self):
        """ILU0 + ILDU0 of the full reordered matrix (no drop), same ordering."""
        if self._glob is None:
            st = self.st
            lu = bilu0(st.n, 3, st.aptr, st.acol, st.aval)
            self._glob = ildu0(st.n, 3, st.aptr, st.acol, lu)
        return self._glob

    def apply_global(self, r):
        return apply(self.st.n, 3, self.st.aptr, self.st.acol, self.global_factors(), r)

    def loss_and_grad(self, P, R, Zstar, den, want_grad=True):
        """Loss = mean over probes q of ||z_q - z*_q||^2 / den_q with
        z_q = M_DD^{-1}(r_q + C r_q), den_q = ||z_DD,q - z*_q||^2; and its
        gradient with respect to the MLP parameters:
        g_q = 2 (z_q - z*_q) / (Q den_q), a_q = M_DD^{-T} g_q,
        dL/dC_f = sum_q a_q[I] r_q[J]^T, then backpropagation."""
        st = self.st
        H1, H2, OUT = mlp_forward(P, self.X)
        C = OUT.reshape(-1, 3, 3)
        Q = R.shape[0]
        loss = 0.0
        A = np.empty_like(R)
        for q in range(Q):
            z = self.apply(C, R[q])
            e = z - Zstar[q]
            loss += (e @ e) / den[q] / Q
            if want_grad:
                A[q] = apply_transpose(st.n, 3, st.tptr, st.tcol, st.f, 2.0 * e / (Q * den[q]))
        if not want_grad:
            return loss, None
        dC = lic_dC(st.n, self.faces, A, R)
        return loss, mlp_backward(P, self.X, H1, H2, dC.reshape(-1, 9))
