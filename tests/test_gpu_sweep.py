"""Shape sweep of the GPU path against the oracle (hypothesis).

Random grid and subdomain extents (the grid a multiple of the box in each
axis), problem families (3x3 random blocks, scalar Laplacian, 3x3
log-normal diffusion) and seeds.  On every draw: partition, permutation,
reordered matrix, dropped pattern and level sets bit for bit; factors per
block and the apply (every kernel variant, FP64) per block row to 1e-12;
the FP32-factor apply (FP64 arithmetic) to 1e-10 against the oracle's
apply of the rounded factors; the SpMV.  Draws are derandomised, so every
run tests the same cases; each case prints its shape before it runs."""

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st_

import oracle as O
from parity import check_close, check_spmv, dd_scale
from problems import laplacian_scalar, lognormal_problem, random_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_04917_amd as P  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True, database=None)


@st_.composite
def shapes(draw):
    sub = [draw(st_.integers(1, 12)) for _ in range(3)]
    mult = [draw(st_.integers(1, 4)) for _ in range(3)]
    while np.prod([s * m for s, m in zip(sub, mult)]) > 24_000 and max(mult) > 1:
        mult[int(np.argmax(mult))] -= 1  # keep the oracle's share to seconds
    dims = tuple(s * m for s, m in zip(sub, mult))
    kind = draw(st_.sampled_from(["rand", "lap", "logn"]))
    if kind == "logn" and np.prod(dims) == 1:
        kind = "rand"  # a lone cell has no faces, so its diffusion block is zero
    return dims, tuple(sub), kind, draw(st_.integers(0, 10_000))


def make(dims, kind, seed):
    nx, ny, nz = dims
    if kind == "rand":
        return random_blocks(nx, ny, nz, seed=seed)
    if kind == "lap":
        return laplacian_scalar(nx, ny, nz, seed=seed)
    return lognormal_problem(nx, ny, nz, seed=seed, sigma=2.0, corr_len=3.0)


def np_(t):
    return t.detach().cpu().numpy()


@SETTINGS
@given(shapes())
def test_sweep_against_oracle(case):
    dims, sub, kind, seed = case
    print(f"[sweep] grid {dims} sub {sub} {kind} seed {seed}", flush=True)
    p = make(dims, kind, seed)
    st = O.setup(p, sub)
    s = DDSolver.from_problem(p, sub=sub)
    try:
        pid, n2o, o2n = P.dd_get_partition(s.h)
        assert np.array_equal(np_(pid), st.part_id)
        assert np.array_equal(np_(n2o), st.new2old) and np.array_equal(np_(o2n), st.old2new)
        ptr, col, val = P.dd_get_reordered(s.h)
        assert np.array_equal(np_(ptr), st.aptr) and np.array_equal(np_(col), st.acol)
        assert np.array_equal(np_(val), st.aval.reshape(-1))
        for which in (0, 1):
            nlev, lptr, rows = P.dd_get_levels(s.h, which)
            onl, optr, orows = st.levels(which)
            assert np.array_equal(np_(nlev), onl) and np.array_equal(np_(lptr), optr)
            assert np.array_equal(np_(rows), orows)
        fptr, fcol, f = P.dd_get_factors(s.h)
        assert np.array_equal(np_(fptr), st.tptr) and np.array_equal(np_(fcol), st.tcol)
        check_close(np_(f), st.f, st.bs * st.bs, 1e-12, what=f"sweep {dims}/{sub} factors")
        rng = np.random.default_rng(seed + 7)
        r = rng.standard_normal(st.n * st.bs)
        rd = torch.as_tensor(r, device="cuda")
        z_o = st.apply(r)
        for variant in (0, 1, 2, 3):
            P.ddilu.dd_set_apply_variant(s.h, variant)
            check_close(np_(s.apply(rd)), z_o, st.bs, 1e-12, what=f"sweep {dims}/{sub} apply v{variant}",
                        scale=dd_scale(st, r))
        P.ddilu.dd_set_apply_variant(s.h, 0)
        s.set_precision(P.DD_MIXED)
        check_close(np_(s.apply(rd)), st.apply_fp32_factors(r, round_input=False), st.bs, 1e-10,
                    what=f"sweep {dims}/{sub} mixed apply")
        s.set_precision(P.DD_FP64)
        check_spmv(st, r, np_(s.spmv(rd)), st.spmv(r), f"sweep {dims}/{sub}")
    finally:
        s.close()
