"""Shape sweeps of the oracle's definitions (hypothesis, CPU).

Random grid extents, subdomain extents, block sizes, problem families and
seeds; on each draw the oracle's setup must satisfy what the paper's
definitions fix, checked by independent means:

- Algorithm 2: every label covers exactly one sx x sy x sz box;
- Algorithm 3: the renumbering is a permutation that keeps subdomains
  contiguous and each subdomain's cells in their old order, and the
  reordered matrix is P A P^T;
- Section 3.2: the kept blocks are exactly the blocks of A~ whose row and
  column share a subdomain;
- Algorithm 6: every row's level is one more than the largest level of the
  rows it depends on inside the sweep (a recursion written here);
- Algorithm 5: (L U)_IJ = A~_IJ wherever A~ has a block, L strictly
  block-lower;
- the apply: L D Uhat z = r.

Draws are derandomised (the same cases every run) and small enough for
dense checks."""

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st_

import oracle as O
from problems import laplacian_scalar, lognormal_problem, random_blocks

SETTINGS = settings(max_examples=80, deadline=None, derandomize=True, database=None)


@st_.composite
def shapes(draw):
    sub = tuple(draw(st_.integers(1, 5)) for _ in range(3))
    mult = [draw(st_.integers(1, 3)) for _ in range(3)]
    kind = draw(st_.sampled_from(["rand", "lap", "logn"]))
    bs = 1 if kind == "lap" else 3
    while np.prod([s * m for s, m in zip(sub, mult)]) * bs > 900 and max(mult) > 1:
        mult[int(np.argmax(mult))] -= 1  # keep the dense checks small
    dims = tuple(s * m for s, m in zip(sub, mult))
    if kind == "logn" and np.prod(dims) == 1:
        kind = "rand"  # a lone cell has no faces, so its diffusion block is zero
    seed = draw(st_.integers(0, 10_000))
    return dims, sub, kind, seed


def make(dims, kind, seed):
    nx, ny, nz = dims
    if kind == "rand":
        return random_blocks(nx, ny, nz, seed=seed)
    if kind == "lap":
        return laplacian_scalar(nx, ny, nz, seed=seed)
    return lognormal_problem(nx, ny, nz, seed=seed, sigma=1.5, corr_len=2.0)


def dense(n, bs, ptr, col, val):
    A = np.zeros((n * bs, n * bs))
    for I in range(n):
        for q in range(ptr[I], ptr[I + 1]):
            J = col[q]
            A[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = np.asarray(val[q]).reshape(bs, bs)
    return A


@SETTINGS
@given(shapes())
def test_setup_definitions(case):
    dims, sub, kind, seed = case
    p = make(dims, kind, seed)
    nx, ny, nz = dims
    sx, sy, sz = sub
    n, bs, S = nx * ny * nz, p.bs, sx * sy * sz
    st = O.setup(p, sub)

    # Algorithm 2: boxes
    g = np.arange(n)
    i, j, k = g % nx, (g // nx) % ny, g // (nx * ny)
    nsub = n // S
    assert sorted(set(st.part_id.tolist())) == list(range(nsub))
    for s in range(nsub):
        m = st.part_id == s
        assert m.sum() == S
        for ax, ext in ((i, sx), (j, sy), (k, sz)):
            assert ax[m].max() - ax[m].min() + 1 == ext and ax[m].min() % ext == 0

    # Algorithm 3: a stable, subdomain-contiguous permutation; A~ = P A P^T
    n2o, o2n = st.new2old, st.old2new
    assert np.array_equal(np.sort(n2o), g) and np.array_equal(o2n[n2o], g)
    assert np.array_equal(st.part_id[n2o], np.repeat(np.arange(nsub), S))
    for s in range(nsub):
        assert np.all(np.diff(n2o[s * S:(s + 1) * S]) > 0)
    A = dense(n, bs, p.brow_ptr, p.bcol, p.val.reshape(-1, bs * bs))
    At = dense(n, bs, st.aptr, st.acol, st.aval.reshape(-1, bs * bs))
    perm = (n2o[:, None] * bs + np.arange(bs)).reshape(-1)
    assert np.array_equal(At, A[np.ix_(perm, perm)])

    # Section 3.2: the kept blocks are those inside one subdomain
    kept = {(I, int(J)) for I in range(n) for J in st.tcol[st.tptr[I]:st.tptr[I + 1]]}
    want = {(I, int(J)) for I in range(n) for J in st.acol[st.aptr[I]:st.aptr[I + 1]] if I // S == J // S}
    assert kept == want

    # Algorithm 6: levels by the recursion over the kept pattern
    for which in (0, 1):
        lev = O.levels(st.tptr, st.tcol, which)
        order = range(n) if which == 0 else range(n - 1, -1, -1)
        ref = np.zeros(n, dtype=np.int64)
        for I in order:
            deps = [int(J) for J in st.tcol[st.tptr[I]:st.tptr[I + 1]] if (J < I if which == 0 else J > I)]
            ref[I] = 1 + max((ref[J] for J in deps), default=-1)
        assert np.array_equal(np.asarray(lev), ref)

    # Algorithm 5: ILU0 reproduces A~ on its kept pattern
    L = np.eye(n * bs)
    U = np.zeros((n * bs, n * bs))
    for I in range(n):
        for q in range(st.tptr[I], st.tptr[I + 1]):
            J = st.tcol[q]
            sl = (slice(I * bs, (I + 1) * bs), slice(J * bs, (J + 1) * bs))
            (L if J < I else U)[sl] = st.lu[q].reshape(bs, bs)
    Ak = dense(n, bs, st.tptr, st.tcol, st.tval.reshape(-1, bs * bs))
    mask = dense(n, bs, st.tptr, st.tcol, np.ones((st.tcol.size, bs * bs))) > 0
    LU = L @ U
    assert np.abs(LU - Ak)[mask].max() <= 1e-13 * np.abs(Ak).max()

    # the apply inverts the factors
    # (triangular substitution is backward stable: the residual is bounded by
    # rounding on |L| |U| |z|, whatever the conditioning)
    r = np.random.default_rng(seed + 1).standard_normal(n * bs)
    z = st.apply(r)
    bound = np.abs(L) @ (np.abs(U) @ np.abs(z))
    assert np.all(np.abs(LU @ z - r) <= 1e-13 * bound + 1e-300)


@SETTINGS
@given(shapes())
def test_single_subdomain_drops_nothing(case):
    """With the whole grid as one subdomain nothing is dropped and the apply
    is the global ILU0 solve."""
    dims, _, kind, seed = case
    p = make(dims, kind, seed)
    st = O.setup(p, dims)
    assert np.array_equal(st.tcol, st.acol) and np.array_equal(st.tptr, st.aptr)


if __name__ == "__main__":  # pragma: no cover
    pytest.main([__file__, "-q"])
