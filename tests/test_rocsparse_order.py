"""Host checks of the renumbering helpers the rocSPARSE comparison uses
(torch on the CPU): the level order of a 7-point grid sorts the rows by
their diagonal plane x + y + z (the closed form of the longest lower path),
and the renumbered matrix is P A P^T with sorted columns in every row."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2508_04917_amd.rocsparse_ref import level_order, permuted_matrix  # noqa: E402


def grid_matrix(nx, ny, nz, bs, seed):
    rows, cols = [], []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = x + nx * (y + ny * z)
                for dx, dy, dz in ((0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    X, Y, Z = x + dx, y + dy, z + dz
                    if 0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz:
                        rows.append(i)
                        cols.append(X + nx * (Y + ny * Z))
    n = nx * ny * nz
    rows, cols = np.array(rows), np.array(cols)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    ptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))])
    val = np.random.default_rng(seed).standard_normal(len(cols) * bs * bs)
    return (torch.tensor(ptr, dtype=torch.int32), torch.tensor(cols, dtype=torch.int32),
            torch.tensor(val, dtype=torch.float64))


def dense(ptr, col, val, bs):
    n = ptr.numel() - 1
    A = np.zeros((n * bs, n * bs))
    v = val.numpy().reshape(-1, bs, bs)
    p, c = ptr.numpy(), col.numpy()
    for i in range(n):
        for q in range(p[i], p[i + 1]):
            A[i * bs:(i + 1) * bs, c[q] * bs:(c[q] + 1) * bs] = v[q]
    return A


@pytest.mark.parametrize("shape,bs", [((4, 3, 5), 3), ((6, 1, 2), 1)])
def test_level_order_is_the_diagonal_planes(shape, bs):
    nx, ny, nz = shape
    ptr, col, val = grid_matrix(nx, ny, nz, bs, seed=1)
    n2o = level_order(ptr, col).numpy()
    i = np.arange(nx * ny * nz)
    plane = i % nx + (i // nx) % ny + i // (nx * ny)
    # sorted by plane, ties in the old order
    assert np.array_equal(n2o, np.lexsort((i, plane)))


@pytest.mark.parametrize("bs", [1, 3])
def test_permuted_matrix_is_pap(bs):
    ptr, col, val = grid_matrix(3, 4, 2, bs, seed=2)
    n = ptr.numel() - 1
    n2o = torch.tensor(np.random.default_rng(3).permutation(n), dtype=torch.int64)
    pp, pc, pv = permuted_matrix(ptr, col, val, n2o, bs)
    A, Ap = dense(ptr, col, val, bs), dense(pp, pc, pv, bs)
    perm = (n2o.numpy()[:, None] * bs + np.arange(bs)).reshape(-1)
    assert np.array_equal(Ap, A[np.ix_(perm, perm)])
    for r in range(n):
        assert np.all(np.diff(pc.numpy()[pp[r]:pp[r + 1]]) > 0)
