"""Graph partitions (no geometry): the library's recursive BFS bisection
against the oracle's, bit for bit, then the whole path on those labels —
reordered matrix, levels, factors, apply and BiCGSTAB — against the oracle's
graph-based setup; and the input checks of the partition calls."""

import numpy as np
import pytest

import oracle as O
from parity import check_close, check_spmv, dd_scale
from problems import grid_graph, laplacian_scalar, unstructured_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402

CASES = {
    # name: (problem factory, rows per part)
    "unstructured_bs3": (lambda: unstructured_problem(6000, seed=11, bs=3), 500),
    "unstructured_bs1": (lambda: unstructured_problem(4096, seed=12, bs=1), 256),
    "laplacian16_scalar": (lambda: laplacian_scalar(16, 16, 16, seed=1), 512),
    "unstructured_one_part": (lambda: unstructured_problem(900, seed=13, bs=3), 900),
    "unstructured_odd_parts": (lambda: unstructured_problem(7 * 300, seed=14, bs=3), 300),
    "unstructured_jacobi": (lambda: unstructured_problem(240, seed=17, bs=3), 1),
    # levels wider than one workgroup pass (the shape of the 2M-row graph
    # workload's parts: 6,400 rows of up to 17 blocks; a pass of the level
    # loops holds 336 block rows of 3x3, 1,024 scalar rows)
    "unstructured_wide_bs3": (lambda: unstructured_problem(12800, seed=18, bs=3), 6400),
    "unstructured_wide_bs1": (lambda: unstructured_problem(20480, seed=19, bs=1), 10240),
}

# rows one pass of the level loops covers: 1,024 threads, BS lanes per row,
# whole rows per 64-lane wavefront
PASS_ROWS = {3: (1024 // 64) * (64 // 3), 1: 1024}

_cache = {}


def case(name):
    if name not in _cache:
        make, S = CASES[name]
        p = make()
        print(f"[graph {name}] n {p.n} nnzb {p.nnzb} bs {p.bs} S {S}", flush=True)
        s = DDSolver.from_problem(p, graph_part_rows=S)
        st = O.setup_graph(p, S)
        _cache[name] = (p, s, st)
    return _cache[name]


def np_(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_spmv_layouts(name):
    """SpMV against the oracle on graph-partitioned matrices: for scalar rows,
    part by part with the part's x in LDS (slices aligned to the parts) where
    a part holds at least four wavefronts' rows and its x fits the LDS;
    otherwise the fixed-width sliced ELL copy where rows hold at most 7
    blocks, the copy with one width per wavefront's rows where rows are
    longer."""
    p, s, st = case(name)
    x = np.random.default_rng(6).standard_normal(st.n * st.bs)
    y_o = st.spmv(x)
    y_g = np_(s.spmv(torch.as_tensor(x, device="cuda")))
    check_spmv(st, x, y_g, y_o, f"graph {name}")
    inf = dd.dd_get_info(s.h)
    longest = int(np.diff(st.aptr).max())
    print(f"[graph {name}] longest row {longest} blocks, layout {inf['spmv_layout']}", flush=True)
    assert inf["max_row_blocks"] == longest
    S, bs = CASES[name][1], p.bs
    part_local = bs == 1 and S >= 4 * 64 and S * 8 <= 163840 - 1024
    assert inf["spmv_layout"] == (3 if part_local else (1 if longest <= 7 else 2))


def test_worked_example_matches_oracle():
    ptr, col = grid_graph(4, 4, 1)
    val = np.where(col == np.repeat(np.arange(16), np.diff(ptr)), 4.0, -1.0)
    s = DDSolver(16, 1, 1, 1, ptr, col, val, graph_part_rows=4)
    try:
        pid, _, _ = dd.dd_get_partition(s.h)
        assert np.array_equal(np_(pid), O.graph_partition(16, ptr, col, 4))
    finally:
        s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_partition_bitexact(name):
    p, s, st = case(name)
    pid, n2o, o2n = dd.dd_get_partition(s.h)
    assert np.array_equal(np_(pid), st.part_id)
    assert np.array_equal(np_(n2o), st.new2old)
    assert np.array_equal(np_(o2n), st.old2new)
    inf = s.info
    assert (inf["S"], inf["sx"], inf["sy"], inf["sz"]) == (CASES[name][1], CASES[name][1], 1, 1)


@pytest.mark.parametrize("name", list(CASES))
def test_reorder_levels_factors(name):
    p, s, st = case(name)
    ptr, col, val = dd.dd_get_reordered(s.h)
    assert np.array_equal(np_(ptr), st.aptr) and np.array_equal(np_(col), st.acol)
    assert np.array_equal(np_(val), st.aval.reshape(-1))
    for which in (0, 1):
        nlev, lptr, rows = dd.dd_get_levels(s.h, which)
        onl, optr, orows = st.levels(which)
        assert np.array_equal(np_(nlev), onl) and np.array_equal(np_(lptr), optr)
        assert np.array_equal(np_(rows), orows)
    fptr, fcol, f = dd.dd_get_factors(s.h)
    assert np.array_equal(np_(fptr), st.tptr) and np.array_equal(np_(fcol), st.tcol)
    check_close(np_(f), st.f, st.bs * st.bs, 1e-12, what=f"graph {name} factor blocks")


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 8])
@pytest.mark.parametrize("name", list(CASES))
def test_apply(name, variant):
    p, s, st = case(name)
    dd.dd_set_apply_variant(s.h, variant)
    try:
        r = np.random.default_rng(7).standard_normal(p.n * p.bs)
        z_o = st.apply(r)
        z_g = np_(s.apply(torch.as_tensor(r, device="cuda")))
        check_close(z_g, z_o, p.bs, 1e-12, what=f"graph {name} apply v{variant}", scale=dd_scale(st, r))
    finally:
        dd.dd_set_apply_variant(s.h, 0)


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
@pytest.mark.parametrize("name", ["unstructured_bs3", "unstructured_bs1", "unstructured_wide_bs3",
                                  "unstructured_wide_bs1"])
def test_apply_reduced_precision(name, prec):
    """FP32 factors on the graph cases (rows of more than three blocks run the
    segmented slot layout): against the oracle with the factors rounded to
    FP32 (and, for DD_FP32, the input and arithmetic in FP32: a bound from
    FP32 rounding, not from the FP64 tolerance)."""
    p, s, st = case(name)
    s.set_precision(dd.DD_MIXED if prec == "mixed" else dd.DD_FP32)
    try:
        r = np.random.default_rng(8).standard_normal(p.n * p.bs)
        z_o = st.apply_fp32_factors(r, round_input=(prec == "fp32"))
        z_g = np_(s.apply(torch.as_tensor(r, device="cuda")))
    finally:
        s.set_precision(dd.DD_FP64)
    if prec == "mixed":
        check_close(z_g, z_o, p.bs, 1e-10, what=f"graph {name} apply mixed", scale=dd_scale(st, r))
    else:  # the FP32 bounds of the structured parity cases
        check_close(z_g, z_o, p.bs, 2e-4, floor=1e-3, norm_tol=2e-5, what=f"graph {name} apply fp32")


@pytest.mark.parametrize("name", ["unstructured_bs3", "unstructured_bs1", "unstructured_wide_bs3"])
def test_segmented_layout_in_use(name):
    """Rows of more than three blocks per sweep: the handle builds the
    segmented slot layout, which the automatic apply then runs."""
    p, s, st = case(name)
    ptr, col = np.asarray(st.tptr), np.asarray(st.tcol)
    rows = np.repeat(np.arange(p.n), np.diff(ptr))
    longest = max(np.bincount(rows[col < rows], minlength=p.n).max(),
                  np.bincount(rows[col > rows], minlength=p.n).max())
    assert longest > 3
    assert dd.dd_get_info(s.h)["apply_layout"] == 2


@pytest.mark.parametrize("name", ["unstructured_wide_bs3", "unstructured_wide_bs1"])
def test_wide_levels_span_several_passes(name):
    """The wide cases really exercise the multi-pass branches: some level of
    some part holds more rows than one workgroup pass."""
    p, s, st = case(name)
    widest = 0
    for which in (0, 1):
        nlev, lptr, rows = st.levels(which)
        off = 0
        for k in range(st.nsub):
            w = np.diff(lptr[off:off + nlev[k] + 1])
            widest = max(widest, int(w.max()))
            off += nlev[k] + 1
    print(f"[graph {name}] widest level {widest} rows, one pass {PASS_ROWS[p.bs]}", flush=True)
    assert widest > PASS_ROWS[p.bs]


@pytest.mark.parametrize("name", ["unstructured_bs3", "unstructured_bs1", "laplacian16_scalar",
                                  "unstructured_wide_bs3"])
def test_bicgstab(name):
    p, s, st = case(name)
    ref = st.bicgstab(p.b)
    x, info = s.solve(torch.as_tensor(p.b, device="cuda"), rtol=1e-8)
    print(f"[graph {name}] iterations GPU {info['iters']}, oracle {ref.iters}", flush=True)
    assert info["status"] == 0 and info["rel_res_true"] <= 2e-8
    assert abs(info["iters"] - ref.iters) <= max(3, ref.iters // 7)


def chain_with_hub(n, extra, bs=3, seed=21):
    """A chain of n block rows (tridiagonal pattern) whose row 10 is also
    coupled, both ways, to `extra` far rows: row 10 then holds 3 + extra
    blocks, the largest in the matrix."""
    rng = np.random.default_rng(seed)
    far = [20, 30, 40, 50, 60][:extra]
    far += [j for j in range(n) if abs(j - 10) > 1 and j not in far][:extra - len(far)]
    nb = [{i} | {j for j in (i - 1, i + 1) if 0 <= j < n} for i in range(n)]
    for j in far:
        nb[10].add(j)
        nb[j].add(10)
    ptr = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for i in range(n):
        c = sorted(nb[i])
        cols += c
        ptr[i + 1] = ptr[i] + len(c)
    col = np.array(cols, dtype=np.int32)
    val = rng.standard_normal((col.size, bs, bs))
    for i in range(n):
        k = ptr[i] + list(col[ptr[i]:ptr[i + 1]]).index(i)
        val[k] += 8.0 * np.eye(bs)
    from problems.generators import Problem
    return Problem(name="chain_hub", nx=n, ny=1, nz=1, bs=bs, brow_ptr=ptr, bcol=col, val=val.reshape(-1),
                   b=rng.standard_normal(n * bs), seed=seed)


def chain_with_links(n, links, bs=3, seed=23):
    """A chain of n block rows plus the given couplings (i, j), both ways;
    diagonal blocks N(0,1) + 8 I, the rest N(0,1)."""
    rng = np.random.default_rng(seed)
    nb = [{i} | {j for j in (i - 1, i + 1) if 0 <= j < n} for i in range(n)]
    for i, j in links:
        nb[i].add(j)
        nb[j].add(i)
    ptr = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for i in range(n):
        cols += sorted(nb[i])
        ptr[i + 1] = len(cols)
    col = np.array(cols, dtype=np.int32)
    val = rng.standard_normal((col.size, bs, bs))
    val[col == np.repeat(np.arange(n), np.diff(ptr))] += 8.0 * np.eye(bs)
    from problems.generators import Problem
    return Problem(name="chain_links", nx=n, ny=1, nz=1, bs=bs, brow_ptr=ptr, bcol=col, val=val.reshape(-1),
                   b=rng.standard_normal(n * bs), seed=seed)


@pytest.mark.parametrize("lower_far,width", [(12, 2), (20, 3)])
def test_segment_width(lower_far, width):
    """The segmented apply cuts rows into segments of two blocks, or of three
    when a lower-sweep row holds more than 16 blocks.  Row 60 of a 64-row
    chain couples to lower_far rows below it (lower sweep: lower_far + 1
    blocks), row 3 to 21 rows above it (upper sweep: 22 blocks, several
    continuations that carry an extra block each).  One part, so nothing is
    dropped; the apply (every precision) against the oracle."""
    links = [(60, 58 - 2 * k) for k in range(lower_far)] + [(3, 6 + 2 * k) for k in range(21)]
    p = chain_with_links(64, links)
    s = DDSolver(p.n, 1, 1, p.bs, p.brow_ptr, p.bcol, p.val, graph_part_rows=64)
    try:
        inf = dd.dd_get_info(s.h)
        print(f"[segments] lower rows up to {lower_far + 1} blocks: apply layout {inf['apply_layout']}, "
              f"segments of {inf['seg_blocks']}", flush=True)
        assert inf["apply_layout"] == 2 and inf["seg_blocks"] == width
        st = O.setup_graph(p, 64)
        r = np.random.default_rng(4).standard_normal(p.n * p.bs)
        rd = torch.as_tensor(r, device="cuda")
        check_close(np_(s.apply(rd)), st.apply(r), 3, 1e-12, what=f"segments of {width}", scale=dd_scale(st, r))
        s.set_precision(dd.DD_MIXED)
        check_close(np_(s.apply(rd)), st.apply_fp32_factors(r, round_input=False), 3, 1e-10,
                    what=f"segments of {width}, FP32 factors")
        s.set_precision(dd.DD_FP64)
    finally:
        s.close()


@pytest.mark.parametrize("extra,layout", [(4, 1), (5, 2), (40, 2)])
def test_spmv_layout_threshold(extra, layout):
    """A longest row of 7 blocks takes the fixed-width sliced ELL copy, 8
    blocks (and a hub of 43, several chunks of 8) the copy with one width
    per wavefront's rows; both agree with the oracle's product on the
    reordered matrix."""
    p = chain_with_hub(64, extra)
    S = 16
    s = DDSolver(p.n, 1, 1, p.bs, p.brow_ptr, p.bcol, p.val, graph_part_rows=S)
    try:
        st = O.setup_graph(p, S)
        x = np.random.default_rng(3).standard_normal(p.n * p.bs)
        y_o = st.spmv(x)
        y_g = np_(s.spmv(torch.as_tensor(x, device="cuda")))
        check_spmv(st, x, y_g, y_o, f"hub chain, {3 + extra} blocks")
        inf = dd.dd_get_info(s.h)
        assert inf["max_row_blocks"] == 3 + extra
        assert inf["spmv_layout"] == layout
        xs, info = s.solve(torch.as_tensor(p.b, device="cuda"), rtol=1e-10)
        assert info["status"] == 0 and info["rel_res_true"] <= 2e-10
    finally:
        s.close()


def test_spmv_long_rows_and_empty_rows():
    """Per-slice-width layout with rows of 0 to 18 blocks: a hub chain with
    four rows emptied (no blocks, no references), ragged final slice
    (n = 70 is not a multiple of one wavefront's 21 rows).  Only the
    partition and the SpMV run (empty rows have no pivot); the oracle's
    partition, renumbering and product give the reference."""
    from types import SimpleNamespace
    p = chain_with_hub(70, 16)
    empty = {30, 31, 32, 33}
    ptr, cols, vals = [0], [], []
    blocks = p.val.reshape(-1, p.bs, p.bs)
    for i in range(p.n):
        for q in range(p.brow_ptr[i], p.brow_ptr[i + 1]):
            j = int(p.bcol[q])
            if i not in empty and j not in empty:
                cols.append(j)
                vals.append(blocks[q])
        ptr.append(len(cols))
    ptr = np.array(ptr, dtype=np.int32)
    col = np.array(cols, dtype=np.int32)
    val = np.array(vals).reshape(-1)
    S = 14
    h = dd.dd_partition_graph(p.n, p.bs, torch.as_tensor(ptr, device="cuda"), torch.as_tensor(col, device="cuda"),
                              torch.as_tensor(val, device="cuda"), part_rows=S)
    try:
        pid = O.graph_partition(p.n, ptr, col, S)
        assert np.array_equal(np_(dd.dd_get_partition(h)[0]), pid)
        n2o, o2n = O.permutation(pid, p.n // S)
        aptr, acol, aval = O.reorder(p.n, p.bs, ptr, col, val, n2o, o2n)
        st = SimpleNamespace(n=p.n, bs=p.bs, aptr=aptr, acol=acol, aval=aval)
        x = np.random.default_rng(8).standard_normal(p.n * p.bs)
        y_o = O.spmv(p.n, p.bs, aptr, acol, aval, x)
        y_g = np_(dd.dd_spmv(h, torch.as_tensor(x, device="cuda")))
        check_spmv(st, x, y_g, y_o, "hub chain with empty rows")
        inf = dd.dd_get_info(h)
        assert inf["spmv_layout"] == 2 and inf["max_row_blocks"] == int(np.diff(ptr).max()) > 8
        assert np.all(y_g.reshape(-1, p.bs)[o2n[sorted(empty)]] == 0.0)
    finally:
        h.close()


def test_isolated_vertices_match_oracle():
    n, S = 48, 4
    ptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    val = np.full(n, 2.0)
    s = DDSolver(n, 1, 1, 1, ptr, col, val, graph_part_rows=S)
    try:
        pid, _, _ = dd.dd_get_partition(s.h)
        assert np.array_equal(np_(pid), O.graph_partition(n, ptr, col, S))
        r = torch.as_tensor(np.arange(n, dtype=np.float64), device="cuda")
        assert np.allclose(np_(s.apply(r)), np.arange(n) / 2.0, rtol=0, atol=1e-15)
    finally:
        s.close()


def test_rejects_indivisible_and_bad_columns():
    p = unstructured_problem(1000, seed=15, bs=3)
    ptr = torch.as_tensor(p.brow_ptr, device="cuda")
    col = torch.as_tensor(p.bcol, device="cuda")
    val = torch.as_tensor(p.val.reshape(-1), device="cuda")
    with pytest.raises(dd.DDError, match="not divisible"):
        dd.dd_partition_graph(p.n, 3, ptr, col, val, part_rows=300)
    bad = col.clone()
    bad[17] = p.n + 5
    with pytest.raises(dd.DDError, match="column index"):
        dd.dd_partition_graph(p.n, 3, ptr, bad, val, part_rows=250)
    q = laplacian_scalar(8, 8, 8, seed=1)
    qcol = torch.as_tensor(q.bcol, device="cuda").clone()
    qcol[3] = -1
    with pytest.raises(dd.DDError, match="column index"):
        dd.dd_partition(8, 8, 8, 1, torch.as_tensor(q.brow_ptr, device="cuda"), qcol,
                        torch.as_tensor(q.val.reshape(-1), device="cuda"), sub=(4, 4, 4))


def test_learned_correction_on_graph_partition():
    """The learned correction needs no geometry: faces, features and the
    corrected apply on a graph partition match the oracle's (a 7-point
    log-normal operator, whose rows fit the slot layout the correction
    requires, partitioned as a graph)."""
    from problems import lic_init_params, lognormal_problem
    p = lognormal_problem(16, 12, 8, seed=41, sigma=1.5, corr_len=3.0)
    s = DDSolver.from_problem(p, graph_part_rows=192)
    st = O.setup_graph(p, 192)
    L = O.LicOracle(st)
    dd.lic_setup(s.h)
    fI, fJ, X = dd.lic_get_faces(s.h)
    assert np.array_equal(np_(fI), L.faces[0]) and np.array_equal(np_(fJ), L.faces[1])
    assert np.allclose(np_(X), L.X, rtol=1e-6, atol=1e-7)
    P = lic_init_params(3)
    P[5952:] = np.random.default_rng(3).standard_normal(585) * 0.05
    Co = L.coeffs(P).astype(np.float32)
    dd.lic_set_coeffs(s.h, torch.as_tensor(Co, device="cuda"))
    try:
        r = np.random.default_rng(8).standard_normal(p.n * 3)
        zg = np_(s.apply(torch.as_tensor(r, device="cuda")))
    finally:
        dd.lic_set_coeffs(s.h, None)
        s.close()
    zo = L.apply(Co.astype(np.float64), r)
    sc = dd_scale(st, O.lic_correct(st.n, L.faces, np.abs(Co.astype(np.float64)), np.abs(r)))
    check_close(zg, zo, 3, 1e-12, what="graph corrected apply", scale=sc)


def test_automatic_part_size():
    """part_rows = 0: among the divisors of n whose vector fits the LDS, the
    one that leaves each compute unit the fewest rows, ceil(parts/n_cu)*S,
    or the largest within 5% of that.  64,000 rows: with 8 CUs, 8,000 (one
    part each; 16,000 would leave 16,000 rows on four CUs); with 2 CUs and
    room for 20,480 rows, 16,000 (two parts each, 32,000 rows: the fewest
    possible); with 3 CUs, 3,200 (20 parts, 7 per CU, 22,400 rows: parts of
    1 or 2 rows would leave 21,334, and 3,200 is the largest divisor within
    5% of that); with 1,000 CUs, 64 (one part each)."""
    p = unstructured_problem(64000, seed=16, bs=1)
    ptr = torch.as_tensor(p.brow_ptr, device="cuda")
    col = torch.as_tensor(p.bcol, device="cuda")
    val = torch.as_tensor(p.val.reshape(-1), device="cuda")
    for n_cu, lds, S in ((8, 163840, 8000), (2, 163840, 16000), (4, 80000, 8000), (1000, 163840, 64),
                         (3, 163840, 3200)):
        h = dd.dd_partition_graph(p.n, 1, ptr, col, val, part_rows=0, lds_budget_bytes=lds, n_cu=n_cu)
        try:
            assert dd.dd_get_info(h)["S"] == S, (n_cu, lds)
        finally:
            h.close()
