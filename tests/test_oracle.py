"""Pins for the CPU oracle: each test checks the oracle against something other
than itself -- a value the paper prints, a closed form, a textbook or library
routine, or brute force on a tiny input -- so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails at least one test.
"""

import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from problems import (laplacian_scalar, lognormal_problem, random_blocks, stencil_pattern)
from problems.generators import Problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- helpers
def dense_bsr(n, bs, ptr, col, val):
    A = np.zeros((n * bs, n * bs))
    for I in range(n):
        for p in range(ptr[I], ptr[I + 1]):
            J = col[p]
            A[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = val[p].reshape(bs, bs)
    return A


def scipy_bsr(n, bs, ptr, col, val):
    return sp.bsr_matrix((np.asarray(val).reshape(-1, bs, bs), col, ptr), shape=(n * bs, n * bs))


def split_factors(n, bs, ptr, col, f):
    """Dense L (unit), D (inverse of the stored inv_D), Uhat (unit) from the ILDU0 storage."""
    L = np.eye(n * bs)
    Uh = np.eye(n * bs)
    D = np.zeros((n * bs, n * bs))
    for I in range(n):
        for p in range(ptr[I], ptr[I + 1]):
            J = col[p]
            blk = f[p].reshape(bs, bs)
            sl = (slice(I * bs, (I + 1) * bs), slice(J * bs, (J + 1) * bs))
            if J < I:
                L[sl] = blk
            elif J > I:
                Uh[sl] = blk
            else:
                D[sl] = np.linalg.inv(blk)
    return L, D, Uh


def split_lu(n, bs, ptr, col, lu):
    L = np.eye(n * bs)
    U = np.zeros((n * bs, n * bs))
    for I in range(n):
        for p in range(ptr[I], ptr[I + 1]):
            J = col[p]
            sl = (slice(I * bs, (I + 1) * bs), slice(J * bs, (J + 1) * bs))
            if J < I:
                L[sl] = lu[p].reshape(bs, bs)
            else:
                U[sl] = lu[p].reshape(bs, bs)
    return L, U


def small_setup(kind="rand", dims=(6, 4, 4), sub=(3, 2, 2), seed=11):
    nx, ny, nz = dims
    if kind == "rand":
        p = random_blocks(nx, ny, nz, seed=seed)
    elif kind == "lap":
        p = laplacian_scalar(nx, ny, nz, seed=seed)
    else:
        p = lognormal_problem(nx, ny, nz, seed=seed, sigma=1.5, corr_len=2.0)
    return p, O.setup(p, sub)


# ------------------------------------------------------------- partitioning
@pytest.mark.parametrize("dims,sub", [((8, 6, 4), (4, 3, 2)), ((16, 16, 16), (8, 8, 8)),
                                      ((10, 20, 5), (5, 4, 5)), ((7, 3, 2), (7, 1, 1))])
def test_partition_boxes(dims, sub):
    """Algorithm 2: every label covers exactly one sx x sy x sz box of cells."""
    nx, ny, nz = dims
    sx, sy, sz = sub
    pid = O.partition(nx, ny, nz, sx, sy, sz)
    g = np.arange(nx * ny * nz)
    i, j, k = g % nx, (g // nx) % ny, g // (nx * ny)
    nsub = O.subdomain_count(nx, ny, nz, sx, sy, sz)
    assert sorted(np.unique(pid)) == list(range(nsub))
    for s in range(nsub):
        m = pid == s
        assert m.sum() == sx * sy * sz
        for ax, ext in ((i, sx), (j, sy), (k, sz)):
            lo, hi = ax[m].min(), ax[m].max()
            assert hi - lo + 1 == ext and lo % ext == 0
    # labels grow along x fastest, as block indices (bx, by, bz) of the box
    assert pid[0] == 0
    if nx // sx > 1:
        assert pid[sx] == 1


def test_partition_not_divisible():
    with pytest.raises(O.OracleError) as e:
        O.partition(10, 10, 10, 3, 5, 5)
    assert e.value.code == O.O_ENOTDIV


def test_permutation_stable_sort():
    """Section 3.1 renumbering == stable argsort of the labels == the box closed form."""
    nx, ny, nz, sx, sy, sz = 12, 8, 6, 4, 4, 3
    pid = O.partition(nx, ny, nz, sx, sy, sz)
    nsub = O.subdomain_count(nx, ny, nz, sx, sy, sz)
    n2o, o2n = O.permutation(pid, nsub)
    assert np.array_equal(n2o, np.argsort(pid, kind="stable"))
    assert np.array_equal(o2n[n2o], np.arange(pid.size))
    g = np.arange(nx * ny * nz)
    i, j, k = g % nx, (g // nx) % ny, g // (nx * ny)
    closed = pid * (sx * sy * sz) + (i % sx) + sx * ((j % sy) + sy * (k % sz))
    assert np.array_equal(o2n, closed)


def test_reorder_is_symmetric_permutation():
    """Algorithm 3 result equals P A P^T (scipy), rows sorted by column."""
    p = random_blocks(6, 4, 4, seed=3)
    nsub = O.subdomain_count(6, 4, 4, 3, 2, 2)
    pid = O.partition(6, 4, 4, 3, 2, 2)
    n2o, o2n = O.permutation(pid, nsub)
    optr, ocol, oval = O.reorder(p.n, 3, p.brow_ptr, p.bcol, p.val, n2o, o2n)
    A = scipy_bsr(p.n, 3, p.brow_ptr, p.bcol, p.val).toarray()
    idx = (3 * n2o[:, None] + np.arange(3)[None, :]).reshape(-1)
    PAPt = A[np.ix_(idx, idx)]
    assert np.array_equal(dense_bsr(p.n, 3, optr, ocol, oval), PAPt)
    for I in range(p.n):
        assert np.all(np.diff(ocol[optr[I]:optr[I + 1]]) > 0)


def test_drop_keeps_diagonal_windows():
    p = random_blocks(6, 4, 4, seed=3)
    st = O.setup(p, (3, 2, 2))
    A = dense_bsr(p.n, 3, st.aptr, st.acol, st.aval)
    At = dense_bsr(p.n, 3, st.tptr, st.tcol, st.tval)
    blk = np.arange(p.n * 3) // (3 * st.S)
    mask = blk[:, None] == blk[None, :]
    assert np.array_equal(At, np.where(mask, A, 0.0))


def test_drop_count_closed_form():
    """7-point stencil: nnzb(A~) = n_sub (7S - 2(sx sy + sy sz + sx sz))."""
    for dims, sub in (((16, 16, 16), (8, 8, 8)), ((64, 64, 64), (8, 8, 16)),
                      ((24, 12, 18), (6, 4, 9))):
        ptr, col, _ = stencil_pattern(*dims)
        n = int(np.prod(dims))
        pid = O.partition(*dims, *sub)
        nsub = O.subdomain_count(*dims, *sub)
        n2o, o2n = O.permutation(pid, nsub)
        optr, ocol, _ = O.reorder(n, 1, ptr, col, None, n2o, o2n)
        sx, sy, sz = sub
        S = sx * sy * sz
        assert O.count_after_drop(n, S, optr, ocol) == nsub * (7 * S - 2 * (sx * sy + sy * sz + sx * sz))


def _golden_table5():
    rows = []
    with open(os.path.join(GOLDEN, "table5_partition.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                rows.append((t[0],) + tuple(int(v) for v in t[1:]))
    return rows


@pytest.mark.parametrize("row", _golden_table5(), ids=lambda r: r[0])
def test_table5_nonzeros_after_drop(row):
    """Paper Table 5: nonzeros before and after the inter-subdomain drop."""
    name, nx, ny, nz, sx, sy, sz, nsub_expect, nnz_full, nnz_drop = row
    ptr, col, _ = stencil_pattern(nx, ny, nz)
    n = nx * ny * nz
    assert 9 * col.shape[0] == nnz_full
    pid = O.partition(nx, ny, nz, sx, sy, sz)
    nsub = O.subdomain_count(nx, ny, nz, sx, sy, sz)
    assert nsub == nsub_expect
    n2o, o2n = O.permutation(pid, nsub)
    optr, ocol, _ = O.reorder(n, 1, ptr, col, None, n2o, o2n)
    assert 9 * O.count_after_drop(n, sx * sy * sz, optr, ocol) == nnz_drop


def test_auto_subdims_rule():
    """The automatic rule picks the largest fitting box (FP64 vector in LDS)."""
    kb160 = 160 * 1024
    assert O.auto_subdims(160, 160, 160, 3, kb160, 256) == (16, 20, 20)
    assert O.auto_subdims(64, 64, 64, 3, kb160, 256) == (8, 8, 16)
    assert O.auto_subdims(128, 128, 128, 3, kb160, 256) == (16, 16, 16)
    # the paper's MI210 sizing: 64 KB LDS holds 8192 FP64 scalars (Section 4)
    sx, sy, sz = O.auto_subdims(128, 128, 128, 1, 64 * 1024, 104)
    assert sx * sy * sz == 8192
    assert O.auto_subdims(4, 4, 4, 3, 8, 1) is None


# ---------------------------------------------------------------- levels
def test_levels_structured_closed_form():
    """Lexicographic box: levL = li+lj+lk, levU = the mirror; sx+sy+sz-2 levels."""
    p = laplacian_scalar(8, 6, 10)
    sub = (4, 3, 5)
    st = O.setup(p, sub)
    sx, sy, sz = sub
    li = np.arange(st.S) % sx
    lj = (np.arange(st.S) // sx) % sy
    lk = np.arange(st.S) // (sx * sy)
    levL = O.levels(st.tptr, st.tcol, 0).reshape(st.nsub, st.S)
    levU = O.levels(st.tptr, st.tcol, 1).reshape(st.nsub, st.S)
    for s in range(st.nsub):
        assert np.array_equal(levL[s], li + lj + lk)
        assert np.array_equal(levU[s], (sx - 1 - li) + (sy - 1 - lj) + (sz - 1 - lk))
    nlev, lptr, rows = st.levels(0)
    assert np.all(nlev == sx + sy + sz - 2)


def _trinomial_widths(sx, sy, sz):
    w = np.convolve(np.convolve(np.ones(sx), np.ones(sy)), np.ones(sz))
    return w.astype(int)


@pytest.mark.parametrize("sub,nlev,wmax", [((8, 8, 8), 22, 48), ((16, 16, 16), 46, 192),
                                           ((16, 20, 20), 54, 256)])
def test_level_widths_trinomial(sub, nlev, wmax):
    ptr, col, _ = stencil_pattern(*sub)
    lev = O.levels(ptr, col, 0)
    nl, lptr, rows = O.level_lists(lev, int(np.prod(sub)))
    widths = np.diff(lptr)
    assert nl[0] == nlev and widths.max() == wmax
    assert np.array_equal(widths, _trinomial_widths(*sub))
    # rows ascend within each level, and each level lists exactly its rows
    for l in range(nl[0]):
        r = rows[lptr[l]:lptr[l + 1]]
        assert np.all(np.diff(r) > 0) and np.all(lev[r] == l)


def test_levels_brute_force_random_dag():
    """Longest path by memoised recursion on random lower/upper patterns."""
    rng = np.random.default_rng(5)
    n = 60
    for trial in range(5):
        dense = rng.random((n, n)) < 0.06
        np.fill_diagonal(dense, True)
        A = sp.csr_matrix(dense.astype(float))
        ptr, col = A.indptr.astype(np.int32), A.indices.astype(np.int32)
        memo = {}

        def lvl(i, lower):
            key = (i, lower)
            if key not in memo:
                deps = [j for j in col[ptr[i]:ptr[i + 1]] if (j < i if lower else j > i)]
                memo[key] = 0 if not deps else 1 + max(lvl(j, lower) for j in deps)
            return memo[key]

        assert list(O.levels(ptr, col, 0)) == [lvl(i, True) for i in range(n)]
        assert list(O.levels(ptr, col, 1)) == [lvl(i, False) for i in range(n)]


# ------------------------------------------------------------ factorisation
@pytest.mark.parametrize("kind", ["rand", "lap", "logn"])
def test_bilu0_matches_A_on_pattern(kind):
    """Defining property of ILU0: (L U)_IJ = A~_IJ wherever A~ has a block."""
    p, st = small_setup(kind)
    bs = p.bs
    L, U = split_lu(st.n, bs, st.tptr, st.tcol, st.lu)
    LU = L @ U
    At = dense_bsr(st.n, bs, st.tptr, st.tcol, st.tval)
    mask = np.zeros_like(At, dtype=bool)
    for I in range(st.n):
        for q in range(st.tptr[I], st.tptr[I + 1]):
            J = st.tcol[q]
            mask[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = True
    err = np.abs(LU - At)[mask].max() / np.abs(At).max()
    assert err < 1e-14
    # and L is strictly block-lower, U block-upper
    assert np.allclose(np.tril(U, -bs), 0.0)


@pytest.mark.parametrize("bs", [1, 3])
def test_bilu0_tridiagonal_is_exact_lu(bs):
    """No fill on a (block) tridiagonal matrix: ILU0 = exact LU over the whole matrix,
    and for bs=1 it equals scipy's LU (which pivots nowhere on this matrix)."""
    n = 40
    p = random_blocks(n, 1, 1, seed=4) if bs == 3 else laplacian_scalar(n, 1, 1)
    st = O.setup(p, (n, 1, 1))
    L, U = split_lu(n, bs, st.tptr, st.tcol, st.lu)
    A = dense_bsr(n, bs, st.aptr, st.acol, st.aval)
    assert np.abs(L @ U - A).max() < 1e-14 * np.abs(A).max()
    if bs == 1:
        P, Ls, Us = scipy.linalg.lu(A)
        assert np.array_equal(P, np.eye(n))
        assert np.allclose(Ls, L, rtol=0, atol=1e-15)
        assert np.allclose(Us, U, rtol=0, atol=1e-14)


def test_bilu0_scalar_laplacian_pivots():
    """Constant-coefficient scalar 7-point: d_g = 6 - sum over lower neighbours 1/d_h,
    L_gh = -1/d_h, Uhat_gh = -1/d_g; pivots tend to 3 + sqrt(6)."""
    p = laplacian_scalar(8, 8, 8)
    st = O.setup(p, (8, 8, 8))
    n = st.n
    diag = {}
    for I in range(n):
        for q in range(st.tptr[I], st.tptr[I + 1]):
            if st.tcol[q] == I:
                diag[I] = st.lu[q, 0, 0]
    g = lambda i, j, k: int(st.old2new[i + 8 * (j + 8 * k)])
    assert diag[g(0, 0, 0)] == 6.0
    assert abs(diag[g(1, 0, 0)] - 35.0 / 6.0) < 1e-15
    assert abs(diag[g(1, 1, 0)] - 198.0 / 35.0) < 1e-14
    assert abs(diag[g(1, 1, 1)] - (6.0 - 3.0 * 35.0 / 198.0)) < 1e-14
    assert abs(diag[g(7, 7, 7)] - 5.449489742828569) < 1e-12
    assert abs(diag[g(7, 7, 7)] - (3 + np.sqrt(6))) < 1e-9
    for I in range(n):
        for q in range(st.tptr[I], st.tptr[I + 1]):
            J = st.tcol[q]
            if J < I:
                assert abs(st.f[q, 0, 0] + 1.0 / diag[J]) < 1e-15
            elif J > I:
                assert abs(st.f[q, 0, 0] + 1.0 / diag[I]) < 1e-15


def test_symmetric_gives_uhat_equal_lT():
    """Symmetric A: ILU0 = IC0, so Uhat = L^T."""
    p, st = small_setup("lap", dims=(6, 6, 4), sub=(3, 3, 4))
    L, D, Uh = split_factors(st.n, 1, st.tptr, st.tcol, st.f)
    assert np.abs(Uh - L.T).max() < 1e-15


def test_ildu0_reproduces_lu():
    """ILDU0 post-pass: L D Uhat = L U, and inv_D is the inverse diagonal."""
    p, st = small_setup("rand")
    L, U = split_lu(st.n, 3, st.tptr, st.tcol, st.lu)
    L2, D, Uh = split_factors(st.n, 3, st.tptr, st.tcol, st.f)
    assert np.array_equal(L, L2)
    assert np.abs(D @ Uh - U).max() < 1e-13 * np.abs(U).max()
    assert np.allclose(np.diag(Uh), 1.0)


def test_zero_pivot_detected():
    p = random_blocks(4, 2, 2, seed=1)
    val = p.val.copy()
    for I in range(p.n):
        for q in range(p.brow_ptr[I], p.brow_ptr[I + 1]):
            if p.bcol[q] == I and I == 0:
                val[q] = 0.0  # cell 0 starts its subdomain: U_00 = A_00 = 0
    p.val = val
    with pytest.raises(O.OracleError) as e:
        O.setup(p, (2, 2, 2))
    assert e.value.code == O.O_EZEROPIVOT


def test_block_inverse():
    rng = np.random.default_rng(1)
    for _ in range(20):
        A = rng.standard_normal((3, 3)) + 3 * np.eye(3)
        assert np.abs(O.block_inverse(A) @ A - np.eye(3)).max() < 1e-14
    with pytest.raises(O.OracleError):
        O.block_inverse(np.array([[1.0, 2, 3], [2, 4, 6], [0, 0, 1]]))


# ------------------------------------------------------------------- apply
@pytest.mark.parametrize("kind", ["rand", "lap", "logn"])
def test_apply_inverts_factors(kind):
    """L D Uhat z = r to ~1e-13: the apply solves with the factors it was given."""
    p, st = small_setup(kind)
    r = np.random.default_rng(2).standard_normal(st.n * p.bs)
    z = st.apply(r)
    L, D, Uh = split_factors(st.n, p.bs, st.tptr, st.tcol, st.f)
    assert np.linalg.norm(L @ D @ Uh @ z - r) / np.linalg.norm(r) < 1e-13


def test_apply_ilu0_equals_ildu0():
    """Algorithm 7 (divide inside the row) and the ILDU0 form give the same z."""
    p, st = small_setup("logn")
    r = np.random.default_rng(3).standard_normal(st.n * 3)
    z1 = st.apply(r)
    z2 = O.apply_ilu0(st.n, 3, st.tptr, st.tcol, st.lu, r)
    assert np.linalg.norm(z1 - z2) / np.linalg.norm(z1) < 1e-13


def test_apply_single_cell_subdomains_is_block_jacobi():
    p = random_blocks(4, 3, 2, seed=9)
    st = O.setup(p, (1, 1, 1))
    r = np.random.default_rng(4).standard_normal(st.n * 3)
    z = st.apply(r)
    for I in range(st.n):
        q = st.aptr[I] + int(np.where(st.acol[st.aptr[I]:st.aptr[I + 1]] == I)[0][0])
        zi = np.linalg.solve(st.aval[q], r[3 * I:3 * I + 3])
        assert np.allclose(z[3 * I:3 * I + 3], zi, rtol=1e-13, atol=0)


def test_apply_line_subdomains_exact_solve():
    """Subdomains that are x-lines: A~ is block tridiagonal per line, ILU0 is exact,
    so the apply is the exact line solve (line Jacobi)."""
    p = lognormal_problem(10, 3, 2, seed=6, sigma=1.0, corr_len=2.0)
    st = O.setup(p, (10, 1, 1))
    r = np.random.default_rng(5).standard_normal(st.n * 3)
    z = st.apply(r)
    At = dense_bsr(st.n, 3, st.tptr, st.tcol, st.tval)
    assert np.linalg.norm(z - np.linalg.solve(At, r)) / np.linalg.norm(z) < 1e-13


def test_single_subdomain_is_global_ilu0():
    """One subdomain spanning the grid: nothing is dropped, M is the global ILU0."""
    p = random_blocks(4, 4, 3, seed=8)
    st = O.setup(p, (4, 4, 3))
    assert np.array_equal(st.tcol, st.acol)
    L, U = split_lu(st.n, 3, st.tptr, st.tcol, st.lu)
    A = dense_bsr(st.n, 3, st.aptr, st.acol, st.aval)
    r = np.random.default_rng(6).standard_normal(st.n * 3)
    z = st.apply(r)
    assert np.linalg.norm(L @ U @ z - r) / np.linalg.norm(r) < 1e-13
    # ILU0 differs from A only off the pattern (fill-in positions)
    assert np.abs(L @ U - A)[np.abs(A) > 0].max() < 1e-13


def test_apply_transpose_adjoint():
    """<M^{-1} a, b> = <a, M^{-T} b>, and M^{-T} matches the dense inverse transpose."""
    p, st = small_setup("rand")
    rng = np.random.default_rng(7)
    a = rng.standard_normal(st.n * 3)
    b = rng.standard_normal(st.n * 3)
    za = st.apply(a)
    zb = O.apply_transpose(st.n, 3, st.tptr, st.tcol, st.f, b)
    assert abs(za @ b - a @ zb) < 1e-13 * np.linalg.norm(za) * np.linalg.norm(b)
    L, D, Uh = split_factors(st.n, 3, st.tptr, st.tcol, st.f)
    Minv_T = np.linalg.inv(L @ D @ Uh).T
    assert np.linalg.norm(zb - Minv_T @ b) / np.linalg.norm(zb) < 1e-12


# -------------------------------------------------------------------- spmv
def test_spmv_matches_scipy():
    p, st = small_setup("logn", dims=(8, 6, 4), sub=(4, 3, 2))
    x = np.random.default_rng(8).standard_normal(st.n * 3)
    y = st.spmv(x)
    ref = scipy_bsr(st.n, 3, st.aptr, st.acol, st.aval) @ x
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-14


# ---------------------------------------------------------------- bicgstab
def test_bicgstab_exact_preconditioner_half_step():
    """M = A (tridiagonal, one subdomain): p^ = A^{-1} b, alpha = 1, s = 0 -> stop
    after the half step of the first trip."""
    p = random_blocks(50, 1, 1, seed=3)
    st = O.setup(p, (50, 1, 1))
    res = st.bicgstab(p.b, rtol=1e-8)
    assert res.status == 0 and res.iters == 1
    A = scipy_bsr(p.n, 3, p.brow_ptr, p.bcol, p.val)
    assert np.linalg.norm(A @ res.x - p.b) / np.linalg.norm(p.b) < 1e-12


def test_bicgstab_scalar_laplacian_true_residual():
    p = laplacian_scalar(16, 16, 16, seed=1)
    st = O.setup(p, (8, 8, 8))
    res = st.bicgstab(p.b, rtol=1e-8)
    assert res.status == 0 and res.relres <= 1e-8
    A = scipy_bsr(p.n, 1, p.brow_ptr, p.bcol, p.val)
    assert np.linalg.norm(p.b - A @ res.x) / np.linalg.norm(p.b) <= 2e-8
    # residual history is the recurrence ||r_j||/||b||, starting at 1
    assert res.history[0] == 1.0 and res.history[-1] <= 1e-8


def test_bicgstab_cross_check_scipy():
    """Same operator and preconditioner through scipy's BiCGSTAB (right-preconditioned):
    iteration counts within +-2 and both solutions within tolerance."""
    p = random_blocks(12, 12, 12, seed=21)
    st = O.setup(p, (6, 6, 6))
    res = st.bicgstab(p.b, rtol=1e-8)
    A = scipy_bsr(p.n, 3, st.aptr, st.acol, st.aval).tocsr()
    bp = st.permute(p.b)
    M = spla.LinearOperator(A.shape, matvec=lambda v: st.apply(np.asarray(v).ravel()))
    count = [0]

    def cb(xk):
        count[0] += 1

    xs, info = spla.bicgstab(A, bp, rtol=1e-8, atol=0.0, M=M, callback=cb, maxiter=1000)
    assert info == 0
    assert abs(count[0] - res.iters) <= 2
    xr = st.permute(res.x)
    assert np.linalg.norm(xs - xr) / np.linalg.norm(xs) < 1e-6
    assert np.linalg.norm(bp - A @ xr) / np.linalg.norm(bp) <= 2e-8


def test_bicgstab_dd_costs_iterations():
    """Dropping couplings weakens the preconditioner: more subdomains, more iterations
    than the global ILU0 (Section 5.3 reports about 1.6x)."""
    p = random_blocks(16, 16, 8, seed=22)
    glob = O.setup(p, (16, 16, 8)).bicgstab(p.b, rtol=1e-8)
    dd = O.setup(p, (4, 4, 4)).bicgstab(p.b, rtol=1e-8)
    assert glob.status == 0 and dd.status == 0
    assert dd.iters > glob.iters


def test_bicgstab_maxit_and_breakdown():
    p = random_blocks(8, 8, 8, seed=2)
    st = O.setup(p, (4, 4, 4))
    res = st.bicgstab(p.b, rtol=1e-30, maxit=3)
    assert res.status == O.O_ENOCONV and res.iters == 3
    b = p.b.copy()
    b[0] = np.nan
    res = st.bicgstab(b, rtol=1e-8, maxit=10)
    assert res.status == O.O_EBREAKDOWN


def test_block_values_in_any_shape():
    """The oracle takes a matrix's blocks as (nnzb, bs, bs) or flat; both give
    the same dropped pattern and factors (a flat array once made the drop
    allocate one value per block instead of bs*bs)."""
    p = random_blocks(6, 5, 4, seed=31)
    flat = Problem(**{**p.__dict__, "val": p.val.reshape(-1)})
    a, b = O.setup(p, (3, 5, 2)), O.setup(flat, (3, 5, 2))
    assert np.array_equal(a.tptr, b.tptr) and np.array_equal(a.tcol, b.tcol)
    assert np.array_equal(a.tval.reshape(-1), b.tval.reshape(-1))
    assert np.array_equal(a.f.reshape(-1), b.f.reshape(-1))
