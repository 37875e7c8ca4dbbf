"""Element-wise bounds for the floating-point parity tests.

A single global 2-norm ratio hides a wrong entry whose magnitude is small
next to the largest ones (on the log-normal cases the block rows of z span
more than five orders of magnitude).  So every floating-point comparison of
a GPU result with the oracle is made per unit (a block row of a vector, a
block of a factor, a face's features or coefficients) as well as in norm:

    ||got_u - ref_u|| <= tol * (||ref_u|| + FLOOR * max_v ||ref_v||)

FLOOR = 1e-6 keeps a unit that is exactly zero, or cancels to near zero, from
turning rounding noise into an infinite relative error; it is far below the
smallest nonzero unit of any parity case, so in practice the bound is
relative per unit.  The tolerances themselves are set where they are used.
Measured spread that motivates them (CPU, same factors, a second apply
written independently with a different summation order): worst block row
4e-15 relative (FP64), factor blocks from a second inverse formula 6e-16;
FP32 arithmetic through the sweeps against the FP64 apply of the rounded
factors: up to 9e-5 on rows that cancel (1.2e-5 with a floor of 1e-3), which
is why the FP32-arithmetic tests use a wider floor.
"""

import numpy as np

import oracle as O

FLOOR = 1e-6


def unit_ratio(got, ref, unit, floor=FLOOR):
    """Largest per-unit error ||got_u - ref_u|| / (||ref_u|| + floor * max ||ref_v||)."""
    g = np.asarray(got, dtype=np.float64).reshape(-1, unit)
    r = np.asarray(ref, dtype=np.float64).reshape(-1, unit)
    assert g.shape == r.shape, (g.shape, r.shape)
    if g.shape[0] == 0:
        return 0.0
    d = np.linalg.norm(g - r, axis=1)
    rn = np.linalg.norm(r, axis=1)
    scale = rn + floor * rn.max()
    if rn.max() == 0.0:
        return 0.0 if d.max() == 0.0 else np.inf
    return float((d / scale).max())


def check_close(got, ref, unit, tol, floor=FLOOR, what="", norm_tol=None, scale=None):
    """Assert per-unit and norm agreement; print the measured values.

    unit: entries per unit (bs for a vector's block rows, bs*bs for factor
    blocks, 27 for a face's features, 9 for a face's coefficients).
    norm_tol: bound on ||got - ref|| / ||ref|| (default tol).
    scale: per-unit magnitudes to measure the error against instead of
    ||ref_u|| + floor * max ||ref_v|| (see apply_scale).  Returns (norm
    error, worst unit ratio)."""
    g = np.asarray(got, dtype=np.float64).reshape(-1)
    r = np.asarray(ref, dtype=np.float64).reshape(-1)
    assert np.isfinite(g).all(), f"{what}: non-finite entries"
    rn = np.linalg.norm(r)
    nerr = float(np.linalg.norm(g - r) / rn) if rn > 0 else float(np.linalg.norm(g))
    if scale is None:
        uerr = unit_ratio(g, r, unit, floor)
        how = f"floor {floor:g}"
    else:
        d = np.linalg.norm((g - r).reshape(-1, unit), axis=1)
        sc = np.asarray(scale, dtype=np.float64)
        assert sc.shape == d.shape and (sc > 0).all()
        uerr = float((d / sc).max()) if d.size else 0.0
        how = "against the magnitude recursion"
    print(f"[parity] {what}: norm {nerr:.2e}, worst unit {uerr:.2e} "
          f"(tol {tol:g}, {how})", flush=True)
    assert nerr <= (tol if norm_tol is None else norm_tol), f"{what}: norm error {nerr:.3e}"
    assert uerr <= tol, f"{what}: worst unit error {uerr:.3e}"
    return nerr, uerr


def magnitude_factors(ptr, col, f, bs):
    """ILDU0 factors with every off-diagonal block replaced by -|block| and
    every diagonal (inv_D) block by |block| (entrywise): the oracle's apply,
    which subtracts the off-diagonal products, then runs the magnitude
    recursion  y'_I = |r_I| + sum_J |L_IJ| y'_J,
    z'_I = |inv_D_I| y'_I + sum_K |Uhat_IK| z'_K  on |r|."""
    n = len(ptr) - 1
    rowid = np.repeat(np.arange(n), np.diff(ptr))
    F = np.abs(np.asarray(f, dtype=np.float64).reshape(-1, bs * bs)).copy()
    F[np.asarray(col) != rowid] *= -1.0
    return F


def apply_scale(n, bs, ptr, col, f, r, transpose=False):
    """Per block row, ||z'_I|| of the magnitude recursion for z = M^{-1} r
    (or M^{-T} r).  Rounding-error analysis of substitution bounds the
    forward error of each computed row by a small multiple of the unit
    roundoff (depth of the recursion times terms per row) times this
    magnitude: rows whose value cancels to near zero are measured against
    the size of the terms that cancelled, not against their own value."""
    F = magnitude_factors(ptr, col, f, bs)
    ra = np.abs(np.asarray(r, dtype=np.float64))
    za = (O.apply_transpose if transpose else O.apply)(n, bs, ptr, col, F, ra)
    return np.linalg.norm(za.reshape(-1, bs), axis=1)


def dd_scale(st, r):
    """apply_scale of the DD-ILU0 apply of an oracle setup."""
    return apply_scale(st.n, st.bs, st.tptr, st.tcol, st.f, r)


# Layer boundaries of the 27 -> 64 -> 64 -> 9 network's flat parameter
# vector: W1[64][27] b1[64] W2[64][64] b2[64] W3[9][64] b3[9].
LAYERS = (("W1", 0, 1728), ("b1", 1728, 1792), ("W2", 1792, 5888), ("b2", 5888, 5952),
          ("W3", 5952, 6528), ("b3", 6528, 6537))


def check_layers(got, ref, tol, what=""):
    """Relative error per parameter group (a wrong layer's gradient cannot
    hide behind the norm of the others)."""
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    worst = 0.0
    for name, a, b in LAYERS:
        rn = np.linalg.norm(r[a:b])
        e = np.linalg.norm(g[a:b] - r[a:b]) / rn if rn > 0 else np.linalg.norm(g[a:b])
        print(f"[parity] {what} {name}: rel {e:.2e}", flush=True)
        assert e <= tol, f"{what} {name}: rel error {e:.3e}"
        worst = max(worst, e)
    return worst


def check_spmv(st, x, y_g, y_o, what=""):
    """SpMV parity: in norm to 1e-14, and per block row against the forward
    error bound of a sum of products, |y_I - fl(y_I)| <= gamma_k (|A||x|)_I
    with gamma_k = k u / (1 - k u) for the row's k = bs x (blocks in the row)
    terms and u = 2^-53.  Both sides obey it, so per row they differ by at
    most 2 gamma_k (|A||x|)_I."""
    u = 2.0 ** -53
    k = st.bs * np.diff(st.aptr).astype(np.float64)
    bound = 2 * k * u / (1 - k * u)
    absAx = O.spmv(st.n, st.bs, st.aptr, st.acol, np.abs(st.aval), np.abs(x))
    scale = np.linalg.norm(absAx.reshape(-1, st.bs), axis=1)
    d = np.linalg.norm((np.asarray(y_g) - y_o).reshape(-1, st.bs), axis=1)
    ratio = d / np.where(scale > 0, scale * bound, 1.0)
    nerr = np.linalg.norm(y_g - y_o) / np.linalg.norm(y_o)
    print(f"[parity] {what} spmv: norm {nerr:.2e}, worst row error / (2 gamma_k (|A||x|)_I) "
          f"{ratio.max():.2e}", flush=True)
    assert np.isfinite(y_g).all()
    assert nerr < 1e-14
    assert ratio.max() <= 1.0
