"""ilu0_refactor: new values on a kept pattern (the setup is amortised over
solves on one sparsity pattern, Section 5.3).  The refactored handle must
hold exactly what a fresh dd_partition + ilu0_factor on the new values
holds: the same kernels run on the same numbers, so the reordered matrix,
the factors, applies in every precision and a BiCGSTAB solve agree bit for
bit; the fresh path itself is pinned to the oracle by the parity tests, and
one apply is checked against the oracle here too."""

import numpy as np
import pytest

import oracle as O
from parity import check_close, dd_scale
from problems import lognormal_problem, random_blocks, unstructured_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402


def cu(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda").to(dt).reshape(-1)


def factors(h):
    inf = dd.dd_get_info(h)
    bb = inf["bs"] ** 2
    ptr = torch.empty(inf["n"] + 1, dtype=torch.int32, device="cuda")
    col = torch.empty(inf["nnzb_dropped"], dtype=torch.int32, device="cuda")
    f = torch.empty(inf["nnzb_dropped"] * bb, dtype=torch.float64, device="cuda")
    lib = dd.lib()
    dd._check(lib.dd_get_factors(h.ptr, dd._ptr(ptr), dd._ptr(col), dd._ptr(f), dd._stream(None)), h)
    val = torch.empty(inf["nnzb"] * bb, dtype=torch.float64, device="cuda")
    dd._check(lib.dd_get_reordered(h.ptr, None, None, dd._ptr(val), dd._stream(None)), h)
    torch.cuda.synchronize()
    return ptr, col, f, val


CASES = {
    # name: (problem on the first values, problem with the same pattern and new values, subdomains)
    "lognormal_24x32x40": (lambda: lognormal_problem(24, 32, 40, seed=7, sigma=2.0),
                           lambda: lognormal_problem(24, 32, 40, seed=8, sigma=1.0), (12, 16, 20)),
    "random_ragged": (lambda: random_blocks(12, 10, 6, seed=5), lambda: random_blocks(12, 10, 6, seed=6), (4, 5, 3)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_refactor_equals_fresh_factorisation(name):
    make1, make2, sub = CASES[name]
    p1, p2 = make1(), make2()
    assert np.array_equal(p1.brow_ptr, p2.brow_ptr) and np.array_equal(p1.bcol, p2.bcol)
    print(f"[refactor] {name}: grid {p1.nx}x{p1.ny}x{p1.nz}, subdomains {sub}", flush=True)
    s = DDSolver.from_problem(p1, sub=sub)
    b2 = cu(p2.b)
    x1, i1 = s.solve(b2, rtol=1e-8)  # a solve on the old values first (workspace, ELL copy in use)
    s.set_precision(dd.DD_MIXED)      # FP32 copies exist before the refactorisation
    dd.ilu0_refactor(s.h, cu(p2.val))
    fresh = DDSolver.from_problem(p2, sub=sub)
    fresh.set_precision(dd.DD_MIXED)
    for a, b_, what in zip(factors(s.h), factors(fresh.h), ("ptr", "col", "factors", "reordered values")):
        assert torch.equal(a, b_), f"{name}: {what} differ after ilu0_refactor"
    r = cu(np.random.default_rng(3).standard_normal(p2.n * p2.bs))
    for prec in (dd.DD_MIXED, dd.DD_FP32, dd.DD_FP64):
        s.set_precision(prec)
        fresh.set_precision(prec)
        assert torch.equal(s.apply(r), fresh.apply(r)), f"{name}: apply differs (precision {prec})"
        assert torch.equal(s.spmv(r), fresh.spmv(r)), f"{name}: SpMV differs"
    x, info = s.solve(b2, rtol=1e-8)
    xf, inff = fresh.solve(b2, rtol=1e-8)
    print(f"[refactor] {name}: {info['iters']} it after refactor, {inff['iters']} fresh "
          f"({i1['iters']} on the old values)", flush=True)
    assert info["status"] == dd.DD_OK and info["iters"] == inff["iters"] and torch.equal(x, xf)
    # and the oracle on the new values
    st = O.setup(p2, sub)
    z = s.apply(r).cpu().numpy()
    zo = st.apply(r.cpu().numpy())
    check_close(z, zo, p2.bs, 1e-12, what=f"{name} apply after refactor", scale=dd_scale(st, r.cpu().numpy()))
    s.close()
    fresh.close()


def test_refactor_state_and_errors():
    p = random_blocks(12, 10, 6, seed=5)
    s = DDSolver.from_problem(p, sub=(4, 5, 3))
    dd.lic_setup(s.h)
    dd.lic_set_params(s.h, torch.zeros(dd.LIC_NPARAM, dtype=torch.float32, device="cuda"))
    # a zero pivot block in the new values: reported, the handle left unfactored.
    # Cell 0 is the first row of its subdomain (no lower neighbour inside it),
    # so its pivot block is its diagonal block of A.
    val = p.val.copy().reshape(-1, 3, 3)
    bad = val.copy()
    bad[p.brow_ptr[0] + np.searchsorted(p.bcol[p.brow_ptr[0]:p.brow_ptr[1]], 0)] = 0.0
    with pytest.raises(dd.DDError) as e:
        dd.ilu0_refactor(s.h, cu(bad))
    assert e.value.code == dd.DD_EZEROPIVOT
    r = cu(np.ones(p.n * 3))
    with pytest.raises(dd.DDError) as e:
        dd.dd_trsv_apply(s.h, r)
    assert e.value.code == dd.DD_ESTATE
    # good values again: factored, and the learned correction needs its setup again
    dd.ilu0_refactor(s.h, cu(val))
    assert dd.dd_get_info(s.h)["factored"] == 1
    with pytest.raises(dd.DDError) as e:
        dd.lic_set_params(s.h, torch.zeros(dd.LIC_NPARAM, dtype=torch.float32, device="cuda"))
    assert e.value.code == dd.DD_ESTATE
    s.close()
    # before ilu0_factor
    q = random_blocks(12, 10, 6, seed=5)
    h = dd.dd_partition(q.nx, q.ny, q.nz, q.bs, cu(q.brow_ptr, torch.int32), cu(q.bcol, torch.int32), cu(q.val),
                        sub=(4, 5, 3))
    with pytest.raises(dd.DDError) as e:
        dd.ilu0_refactor(h, cu(q.val))
    assert e.value.code == dd.DD_ESTATE
    h.close()


@pytest.mark.parametrize("bs,spmv_layout", [(3, 2), (1, 3)])
def test_refactor_graph_partition(bs, spmv_layout):
    """The same on a matrix without geometry (rows of up to 15 blocks): the
    apply's segmented slot layout and the SpMV's per-slice-width copy are
    rewritten in place (for scalar rows the copy aligned to the parts), and
    everything again equals a fresh setup."""
    import dataclasses
    p1 = unstructured_problem(6000, seed=31, bs=bs)
    blocks = p1.val.reshape(-1, bs, bs)
    off = (p1.bcol != np.repeat(np.arange(p1.n), np.diff(p1.brow_ptr)))[:, None, None]
    scale = 1.0 - 0.2 * np.random.default_rng(32).random((blocks.shape[0], 1, 1))
    p2 = dataclasses.replace(p1, val=np.where(off, blocks * scale, blocks))
    S = 600
    s = DDSolver.from_problem(p1, graph_part_rows=S)
    inf = dd.dd_get_info(s.h)
    print(f"[refactor] graph: n {p1.n}, longest row {inf['max_row_blocks']} blocks, "
          f"apply layout {inf['apply_layout']}, SpMV layout {inf['spmv_layout']}", flush=True)
    assert inf["apply_layout"] == 2 and inf["spmv_layout"] == spmv_layout
    b2 = cu(p2.b)
    s.solve(b2, rtol=1e-8)
    s.set_precision(dd.DD_MIXED)
    dd.ilu0_refactor(s.h, cu(p2.val))
    fresh = DDSolver.from_problem(p2, graph_part_rows=S)
    fresh.set_precision(dd.DD_MIXED)
    for a, b_, what in zip(factors(s.h), factors(fresh.h), ("ptr", "col", "factors", "reordered values")):
        assert torch.equal(a, b_), f"graph: {what} differ after ilu0_refactor"
    r = cu(np.random.default_rng(3).standard_normal(p2.n * p2.bs))
    for prec in (dd.DD_MIXED, dd.DD_FP32, dd.DD_FP64):
        s.set_precision(prec)
        fresh.set_precision(prec)
        assert torch.equal(s.apply(r), fresh.apply(r)), f"graph: apply differs (precision {prec})"
        assert torch.equal(s.spmv(r), fresh.spmv(r)), "graph: SpMV differs"
    x, info = s.solve(b2, rtol=1e-8)
    xf, inff = fresh.solve(b2, rtol=1e-8)
    assert info["status"] == dd.DD_OK and info["iters"] == inff["iters"] and torch.equal(x, xf)
    st = O.setup_graph(p2, S)
    rn = r.cpu().numpy()
    check_close(s.apply(r).cpu().numpy(), st.apply(rn), p2.bs, 1e-12, what="graph apply after refactor",
                scale=dd_scale(st, rn))
    s.close()
    fresh.close()
