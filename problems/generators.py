"""Seeded generators for structured 3D 7-point operators in BSR form.

Conventions shared by every consumer:
  * cell index g = i + nx*(j + ny*k), x fastest (the grid numbering of the
    geometric-cut partitioner, Section 3, Algorithm 2);
  * BSR arrays ``brow_ptr`` (int32, n+1), ``bcol`` (int32, nnzb) and ``val``
    (float64, nnzb x bs x bs), each block row-major, blocks of a row sorted by
    ascending column;
  * right-hand sides have length n*bs, block-row major.

The stand-in workloads follow the shapes of the paper's structured 3x3 BSR
Laplacians (Section 5, Table 2: 128^3 grid; Table 1: 4M block rows and 28M
nonzero blocks = 160^3).  Their coefficient recipes are synthetic: a scalar
Laplacian, a random-block operator, and log-normal permeability fields that
stand in for the reservoir matrices (spe10-like variation) the paper uses.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Offsets of the 7-point stencil in ascending column order for g = i + nx*(j + ny*k):
# -z, -y, -x, self, +x, +y, +z.   kind codes 0..6 follow this order.
KIND_NAMES = ("-z", "-y", "-x", "self", "+x", "+y", "+z")
KIND_AXIS = np.array([2, 1, 0, -1, 0, 1, 2], dtype=np.int8)  # 0=x 1=y 2=z, -1 = diagonal


@dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    bs: int
    brow_ptr: np.ndarray
    bcol: np.ndarray
    val: np.ndarray
    b: np.ndarray
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nnzb(self) -> int:
        return int(self.bcol.shape[0])


def stencil_pattern(nx: int, ny: int, nz: int):
    """7-point pattern: returns (brow_ptr int32[n+1], bcol int32[nnzb], kind int8[nnzb])."""
    n = nx * ny * nz
    g = np.arange(n, dtype=np.int64)
    i = g % nx
    j = (g // nx) % ny
    k = g // (nx * ny)
    offs = np.array([-nx * ny, -nx, -1, 0, 1, nx, nx * ny], dtype=np.int64)
    valid = np.stack(
        [k > 0, j > 0, i > 0, np.ones(n, dtype=bool), i < nx - 1, j < ny - 1, k < nz - 1],
        axis=1,
    )
    cand = g[:, None] + offs[None, :]
    counts = valid.sum(axis=1)
    brow_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=brow_ptr[1:])
    bcol = cand[valid].astype(np.int32)
    kind = np.broadcast_to(np.arange(7, dtype=np.int8), (n, 7))[valid]
    if brow_ptr[-1] >= 2**31:
        raise ValueError("pattern too large for int32 offsets")
    return brow_ptr.astype(np.int32), bcol, np.ascontiguousarray(kind)


def laplacian_scalar(nx: int = 16, ny: int = 16, nz: int = 16, seed: int = 1) -> Problem:
    """Scalar (1x1) 7-point Laplacian with eliminated Dirichlet boundary.

    A_gg = 6, A_gh = -1 for every existing neighbour (no h^2 scaling);
    b ~ uniform[-1, 1] from ``default_rng(seed)``.
    """
    ptr, col, kind = stencil_pattern(nx, ny, nz)
    val = np.where(kind == 3, 6.0, -1.0).reshape(-1, 1, 1).astype(np.float64)
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1.0, 1.0, nx * ny * nz)
    return Problem("laplacian_scalar", nx, ny, nz, 1, ptr, col, val, b, seed)


def random_blocks(nx: int = 64, ny: int = 64, nz: int = 64, seed: int = 2) -> Problem:
    """3x3 BSR 7-point operator with random blocks.

    Draw order from ``default_rng(seed)``: G (n,3,3), then H (nnzb-n,3,3) in CSR
    order of the off-diagonal blocks, then b (3n).  A_II = 6I + 0.1*(G+G^T)/2,
    A_IJ = -I + 0.05*H_IJ.  (I,J) and (J,I) draw independently, so A is
    nonsymmetric.
    """
    ptr, col, kind = stencil_pattern(nx, ny, nz)
    n = nx * ny * nz
    nnzb = col.shape[0]
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, 3, 3))
    H = rng.standard_normal((nnzb - n, 3, 3))
    b = rng.standard_normal(3 * n)
    eye = np.eye(3)
    val = np.empty((nnzb, 3, 3), dtype=np.float64)
    diag = kind == 3
    val[diag] = 6.0 * eye + 0.1 * 0.5 * (G + G.transpose(0, 2, 1))
    val[~diag] = -eye + 0.05 * H
    return Problem("random_blocks", nx, ny, nz, 3, ptr, col, val, b, seed)


def laplacian_blocks(nx: int, ny: int, nz: int, seed: int = 0) -> Problem:
    """3x3 block 7-point Laplacian (Dirichlet boundary eliminated): diagonal
    blocks 6 I, coupling blocks -I, i.e. the scalar operator of
    laplacian_scalar times I_3; the paper's structured test matrices are 3x3
    BSR Laplacians of this pattern (it does not print their values).  b is
    N(0,1) from default_rng(seed)."""
    ptr, col, kind = stencil_pattern(nx, ny, nz)
    n = nx * ny * nz
    val = np.where((kind == 3)[:, None, None], 6.0 * np.eye(3), -np.eye(3))
    b = np.random.default_rng(seed).standard_normal(3 * n)
    return Problem("laplacian_blocks", nx, ny, nz, 3, ptr, col, np.ascontiguousarray(val), b, seed)


def grid_graph(nx: int, ny: int, nz: int):
    """Pattern (brow_ptr, bcol) of the 7-point grid operator (5-point in 2D,
    a path in 1D), diagonal included: a graph with known geometry."""
    ptr, col, _ = stencil_pattern(nx, ny, nz)
    return ptr, col


def unstructured_problem(n: int, seed: int, bs: int = 3, k: int = 6) -> Problem:
    """Stand-in for the paper's unstructured matrices (graph-partitioned
    there with METIS): n random points in the unit cube, each coupled to its
    k nearest neighbours (pattern symmetrised, diagonal added), numbered in
    the random order the points were drawn, so the numbering carries no
    locality.  Draw order from ``default_rng(seed)``: points (n,3), G
    (n,bs,bs), H (off-diagonal blocks in CSR order, bs,bs), b (n*bs).
    A_II = (deg_I + 0.5) I + 0.1 (G+G^T)/2, A_IJ = -I + 0.05 H_IJ; returned
    with nx = n, ny = nz = 1."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    _, nb = cKDTree(pts).query(pts, k=k + 1)
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = nb[:, 1:].reshape(-1).astype(np.int64)
    pairs = np.unique(np.concatenate([rows * n + cols, cols * n + rows, np.arange(n, dtype=np.int64) * (n + 1)]))
    r, c = pairs // n, pairs % n
    counts = np.bincount(r, minlength=n)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    nnzb = c.shape[0]
    G = rng.standard_normal((n, bs, bs))
    H = rng.standard_normal((nnzb - n, bs, bs))
    b = rng.standard_normal(n * bs)
    eye = np.eye(bs)
    diag = r == c
    deg = counts - 1
    val = np.empty((nnzb, bs, bs), dtype=np.float64)
    val[diag] = (deg + 0.5)[:, None, None] * eye + 0.1 * 0.5 * (G + G.transpose(0, 2, 1))
    val[~diag] = -eye + 0.05 * H
    return Problem("unstructured", n, 1, 1, bs, ptr.astype(np.int32), c.astype(np.int32), val, b, seed,
                   meta=dict(k=k, max_row_blocks=int(counts.max())))


def lognormal_field(rng: np.random.Generator, nx: int, ny: int, nz: int,
                    sigma: float, corr_len: float = 8.0) -> np.ndarray:
    """Log-normal permeability k = exp(sigma * g), g a unit-variance Gaussian field.

    White noise (nz,ny,nx) is filtered periodically (FFT) by a Gaussian kernel of
    standard deviation corr_len/sqrt(2) cells, so that the covariance is
    exp(-r^2 / (2 corr_len^2)); the result is normalised to sample mean 0, std 1.
    Returned array is flattened in g order (x fastest).
    """
    w = rng.standard_normal((nz, ny, nx))
    s = corr_len / np.sqrt(2.0)
    fz = np.fft.fftfreq(nz)[:, None, None]
    fy = np.fft.fftfreq(ny)[None, :, None]
    fx = np.fft.rfftfreq(nx)[None, None, :]
    kern = np.exp(-2.0 * np.pi ** 2 * s ** 2 * (fx ** 2 + fy ** 2 + fz ** 2))
    gfield = np.fft.irfftn(np.fft.rfftn(w) * kern, s=(nz, ny, nx), axes=(0, 1, 2))
    gfield -= gfield.mean()
    gfield /= gfield.std()
    return np.exp(sigma * gfield).reshape(-1)


def lognormal_problem(nx: int, ny: int, nz: int, seed: int, sigma: float = 2.0,
                      corr_len: float = 8.0, aniso=(1.0, 1.0, 1.0), noise: float = 0.05,
                      name: str = "lognormal", draw_sigma: tuple | None = None) -> Problem:
    """3x3 BSR two-point-flux operator on a log-normal permeability field.

    Draw order from ``default_rng(seed)``: [sigma ~ U(draw_sigma) if given], the
    white noise of the field, H (nnzb-n,3,3) in CSR order of the off-diagonal
    blocks, then b ~ N(0,1) (3n).

    Face value k_f = 2 k_a k_b / (k_a + k_b) times the axis multiplier aniso[axis].
    Coupling block B_IJ = k_f (I - noise * H_IJ) (noise relative to k_f, drawn
    independently for (I,J) and (J,I), so A is nonsymmetric); A_IJ = -B_IJ.
    Diagonal block A_II = sum_J B_IJ + (sum over boundary faces of 2 k_I
    aniso[axis]) I: every interior block row sums to zero (flux conservation),
    and the Dirichlet boundary at the half cell makes the operator nonsingular.
    """
    ptr, col, kind = stencil_pattern(nx, ny, nz)
    n = nx * ny * nz
    nnzb = col.shape[0]
    rng = np.random.default_rng(seed)
    if draw_sigma is not None:
        sigma = float(rng.uniform(draw_sigma[0], draw_sigma[1]))
    kcell = lognormal_field(rng, nx, ny, nz, sigma, corr_len)
    H = rng.standard_normal((nnzb - n, 3, 3))
    b = rng.standard_normal(3 * n)

    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(ptr.astype(np.int64)))
    off = kind != 3
    ka = kcell[rows[off]]
    kb = kcell[col[off]]
    mult = np.asarray(aniso, dtype=np.float64)[KIND_AXIS[kind[off]]]
    kf = mult * 2.0 * ka * kb / (ka + kb)
    eye = np.eye(3)
    B = kf[:, None, None] * (eye - noise * H)

    # boundary faces: each missing neighbour of a cell contributes 2 k_I aniso[axis]
    g = np.arange(n, dtype=np.int64)
    i = g % nx
    j = (g // nx) % ny
    k = g // (nx * ny)
    ax = np.asarray(aniso, dtype=np.float64)
    nb_missing = ((i == 0).astype(np.float64) + (i == nx - 1)) * ax[0] \
        + ((j == 0).astype(np.float64) + (j == ny - 1)) * ax[1] \
        + ((k == 0).astype(np.float64) + (k == nz - 1)) * ax[2]
    diag = np.zeros((n, 3, 3))
    for e in range(9):
        diag.reshape(n, 9)[:, e] = np.bincount(rows[off], weights=B.reshape(-1, 9)[:, e], minlength=n)
    diag += (2.0 * kcell * nb_missing)[:, None, None] * eye

    val = np.empty((nnzb, 3, 3), dtype=np.float64)
    val[off] = -B
    val[~off] = diag
    meta = {"sigma": sigma, "corr_len": corr_len, "aniso": tuple(aniso), "noise": noise}
    return Problem(name, nx, ny, nz, 3, ptr, col, val, b, seed, meta)


def training_problem(seed: int, n: int = 48) -> Problem:
    """One problem of the learned-correction training set: n^3 log-normal, sigma ~ U[1,3]."""
    return lognormal_problem(n, n, n, seed, draw_sigma=(1.0, 3.0), name="lognormal_train")


def probe_vectors(seed: int, n_probes: int, size: int) -> np.ndarray:
    """Probe q of problem ``seed`` is N(0,1) from default_rng([seed, 7, q])."""
    out = np.empty((n_probes, size), dtype=np.float64)
    for q in range(n_probes):
        out[q] = np.random.default_rng([seed, 7, q]).standard_normal(size)
    return out


def lic_init_params(seed: int = 0) -> np.ndarray:
    """Initial parameters of the 27 -> 64 -> 64 -> 9 interface MLP (6,537 values,
    layout W1[64][27] b1[64] W2[64][64] b2[64] W3[9][64] b3[9]): He-normal
    W1 and W2 from default_rng(seed), zero biases, and W3 = b3 = 0 so that the
    untrained correction is exactly zero."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((64, 27)) * np.sqrt(2.0 / 27)
    W2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), np.zeros(9 * 64),
                           np.zeros(9)])


def training_order(seed: int, epochs: int, nprob: int) -> np.ndarray:
    """Order in which the training problems are visited: a fresh permutation of
    range(nprob) per epoch from default_rng(seed), shape (epochs, nprob)."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(nprob) for _ in range(epochs)]).astype(np.int32)


# Named workloads: (generator, kwargs, default subdomain dims or None = automatic rule)
WORKLOADS = {
    # scalar 7-point Laplacian, 16^3, eight 8^3 subdomains
    "laplacian16_scalar": (laplacian_scalar, dict(nx=16, ny=16, nz=16, seed=1), (8, 8, 8)),
    # random 3x3 blocks on a 64^3 grid
    "random64_bsr3": (random_blocks, dict(nx=64, ny=64, nz=64, seed=2), None),
    # log-normal permeability (sigma 2, correlation 8 cells) on a 160^3 grid
    "lognormal160_bsr3": (lognormal_problem, dict(nx=160, ny=160, nz=160, seed=3), None),
    # anisotropic x:y:z = 1:1:100 on top of the log-normal field, 160^3
    "aniso160_bsr3": (lognormal_problem,
                      dict(nx=160, ny=160, nz=160, seed=5, aniso=(1.0, 1.0, 100.0),
                           name="aniso"), None),
    # unstructured stand-in (random points, 6 nearest neighbours, random numbering), 2,048,000 block rows
    "unstructured2m_bsr3": (unstructured_problem, dict(n=2_048_000, seed=21, bs=3), None),
    # the scalar (1x1) counterpart: the CSR path on an unstructured graph, 4,096,000 rows
    "unstructured4m_scalar": (unstructured_problem, dict(n=4_096_000, seed=22, bs=1), None),
    # unseen evaluation problems for the learned correction, 128^3
    "lognormal128_eval": (lognormal_problem, dict(nx=128, ny=128, nz=128, seed=2000), None),
    # the shapes of the paper's laplacian1 / laplacian2 (Table 5): 3x3 block
    # Laplacians cut into 8x16x16 boxes of 2,048 block rows
    "laplacian1_bsr3": (laplacian_blocks, dict(nx=128, ny=128, nz=128, seed=31), (8, 16, 16)),
    "laplacian2_bsr3": (laplacian_blocks, dict(nx=128, ny=128, nz=256, seed=32), (8, 16, 16)),
}


def make_workload(name: str, **override) -> Problem:
    gen, kw, _ = WORKLOADS[name]
    kw = dict(kw)
    kw.update(override)
    return gen(**kw)
