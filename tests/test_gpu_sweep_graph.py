"""Shape sweep of the graph path against the oracle (hypothesis).

Random matrices without geometry (k-nearest-neighbour graphs of random
points, k from 3 to 12, 1x1 or 3x3 blocks), random part sizes and seeds:
partition labels, renumbering, levels and dropped pattern bit for bit; the
apply in its automatic layout (slots, or segments of two or three blocks),
FP64 per block row to 1e-12 and with FP32 factors to 1e-10; the SpMV in its
automatic layout (fixed-width or per-slice-width ELL copy).  Derandomised:
every run tests the same cases; each prints its shape before it runs."""

import numpy as np
import pytest
from hypothesis import example, given, settings, strategies as st_

import oracle as O
from parity import check_close, check_spmv, dd_scale
from problems import unstructured_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402

SETTINGS = settings(max_examples=30, deadline=None, derandomize=True, database=None)


@st_.composite
def graphs(draw):
    bs = draw(st_.sampled_from([1, 3]))
    parts = draw(st_.integers(1, 12))
    S = draw(st_.integers(16, 2400 if bs == 3 else 6000))
    k = draw(st_.integers(3, 12))
    return parts * S, S, bs, k, draw(st_.integers(0, 10_000))


def np_(t):
    return t.detach().cpu().numpy()


@SETTINGS
@given(graphs())
# wide levels (several chunks per level), long rows (segments of three, or
# the plain loop past 24 lower blocks), scalar rows
@example((12 * 2400, 2400, 3, 12, 1))
@example((4 * 2400, 2400, 3, 20, 2))
@example((6 * 6000, 6000, 1, 10, 3))
def test_graph_sweep_against_oracle(case):
    n, S, bs, k, seed = case
    print(f"[graph sweep] n {n} S {S} bs {bs} k {k} seed {seed}", flush=True)
    p = unstructured_problem(n, seed=seed, bs=bs, k=min(k, n - 1))
    st = O.setup_graph(p, S)
    s = DDSolver.from_problem(p, graph_part_rows=S)
    try:
        inf = dd.dd_get_info(s.h)
        what = f"graph sweep n {n} S {S} bs {bs} k {k} (apply layout {inf['apply_layout']}/{inf['seg_blocks']}, " \
               f"SpMV layout {inf['spmv_layout']})"
        pid, n2o, _ = dd.dd_get_partition(s.h)
        assert np.array_equal(np_(pid), st.part_id) and np.array_equal(np_(n2o), st.new2old)
        for which in (0, 1):
            nlev, lptr, rows = dd.dd_get_levels(s.h, which)
            onl, optr, orows = st.levels(which)
            assert np.array_equal(np_(nlev), onl) and np.array_equal(np_(lptr), optr)
            assert np.array_equal(np_(rows), orows)
        fptr, fcol, _ = dd.dd_get_factors(s.h)
        assert np.array_equal(np_(fptr), st.tptr) and np.array_equal(np_(fcol), st.tcol)
        r = np.random.default_rng(seed + 3).standard_normal(n * bs)
        rd = torch.as_tensor(r, device="cuda")
        check_close(np_(s.apply(rd)), st.apply(r), bs, 1e-12, what=what, scale=dd_scale(st, r))
        s.set_precision(dd.DD_MIXED)
        check_close(np_(s.apply(rd)), st.apply_fp32_factors(r, round_input=False), bs, 1e-10,
                    what=what + " FP32 factors", scale=dd_scale(st, r))
        s.set_precision(dd.DD_FP64)
        check_spmv(st, r, np_(s.spmv(rd)), st.spmv(r), what)
    finally:
        s.close()
