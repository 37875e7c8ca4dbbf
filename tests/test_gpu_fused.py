"""BiCGSTAB with each preconditioner apply and the SpMV after it in one launch
(dd_set_fusion, opt-in).  The launch computes the same M^{-1} x and
A M^{-1} x as the two separate launches; only the grouping of the dot
products' partial sums differs (one partial per subdomain instead of one per
SpMV workgroup).  So, on every parity shape: the solve reports the fused
launch, its residual history agrees with the two-launch solve's to rounding
over the first iterations (a product workgroup that read a stale z would
differ at once), both converge to the same solution, fused solves are
bit-reproducible, and the solve falls back to two launches where the
settings need them."""

import numpy as np
import pytest

import oracle as O
from problems import laplacian_scalar, lognormal_problem, make_workload, random_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines, skipped by marker
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402

CASES = {
    "lap16_8cube": (lambda: laplacian_scalar(16, 16, 16, seed=1), (8, 8, 8)),
    "rand64_auto": (lambda: random_blocks(64, 64, 64, seed=2), (0, 0, 0)),
    "rand_ragged": (lambda: random_blocks(12, 10, 6, seed=5), (4, 5, 3)),
    "logn_lds_max": (lambda: lognormal_problem(32, 40, 40, seed=8, sigma=2.0), (16, 20, 20)),
    "rand_jacobi": (lambda: random_blocks(6, 5, 4, seed=9), (1, 1, 1)),
    "lap_one_sub": (lambda: laplacian_scalar(12, 10, 8, seed=3), (12, 10, 8)),
}

_cache = {}


def case(name):
    if name not in _cache:
        make, sub = CASES[name]
        p = make()
        print(f"[fused {name}] grid {p.nx}x{p.ny}x{p.nz} bs {p.bs} sub {sub}", flush=True)
        s = DDSolver.from_problem(p, sub=sub)
        dd.dd_set_fusion(s.h, True)
        _cache[name] = (p, s)
    return _cache[name]


def solve_with_history(s, b, fuse, k=None, rtol=1e-8):
    maxit = k if k is not None else 10000
    hist = torch.full((maxit + 1 if k is not None else 20001,), float("nan"), dtype=torch.float64, device="cuda")
    dd.dd_set_fusion(s.h, fuse)
    dd.dd_set_residual_history(s.h, hist)
    try:
        x, info = s.solve(b, rtol=rtol, maxit=maxit)
    finally:
        dd.dd_set_residual_history(s.h, None)
        dd.dd_set_fusion(s.h, True)
    return x, info, hist[: info["iters"] + 1].cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_fused_matches_two_launches(name):
    p, s = case(name)
    b = torch.as_tensor(p.b, device="cuda")
    xf, inf_f, hf = solve_with_history(s, b, True)
    xu, inf_u, hu = solve_with_history(s, b, False)
    print(f"[fused {name}] iters fused {inf_f['iters']} two-launch {inf_u['iters']}", flush=True)
    assert inf_f["fused"] == 1 and inf_u["fused"] == 0
    for inf in (inf_f, inf_u):
        assert inf["status"] == dd.DD_OK and inf["rel_res_true"] <= 2e-8
    # same recurrence up to the summation order of the dots: the early
    # residuals agree to rounding, the exits within a few iterations
    m = min(8, len(hf), len(hu))
    assert np.allclose(hf[:m], hu[:m], rtol=1e-9, atol=0), (hf[:m], hu[:m])
    assert abs(inf_f["iters"] - inf_u["iters"]) <= max(2, inf_u["iters"] // 10)
    assert float(torch.linalg.norm(xf - xu) / torch.linalg.norm(xu)) < 1e-5


@pytest.mark.parametrize("name", ["lap16_8cube", "logn_lds_max"])
def test_fused_against_oracle(name):
    """The fused solve's solution and iteration count against the oracle's
    BiCGSTAB (iterations in the oracle's band over unit-roundoff
    perturbations of b, widened by 2, as for the two-launch solve)."""
    p, s = case(name)
    inf = s.info
    st = O.setup(p, (inf["sx"], inf["sy"], inf["sz"]))
    ref = st.bicgstab(p.b, rtol=1e-8)
    its = [ref.iters]
    rng = np.random.default_rng(99)
    for _ in range(4):
        its.append(st.bicgstab(p.b * (1 + 1e-15 * rng.standard_normal(p.b.size)), rtol=1e-8).iters)
    x, info = s.solve(torch.as_tensor(p.b, device="cuda"), rtol=1e-8)
    assert info["fused"] == 1 and info["status"] == dd.DD_OK
    assert min(its) - 2 <= info["iters"] <= max(its) + 2, (info["iters"], its)
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x) < 1e-5


@pytest.mark.parametrize("prec", [dd.DD_MIXED, dd.DD_FP32], ids=["mixed", "fp32"])
def test_fused_reduced_precision(prec):
    p, s = case("logn_lds_max")
    b = torch.as_tensor(p.b, device="cuda")
    s.set_precision(prec)
    try:
        xf, inf_f, hf = solve_with_history(s, b, True)
        xu, inf_u, hu = solve_with_history(s, b, False)
    finally:
        s.set_precision(dd.DD_FP64)
    assert inf_f["fused"] == 1 and inf_u["fused"] == 0
    assert inf_f["status"] == dd.DD_OK and inf_f["rel_res_true"] <= 2e-8
    # FP32 factors are the same, so the early residuals still agree to the
    # apply's own rounding (FP32 arithmetic for DD_FP32)
    m = min(6, len(hf), len(hu))
    tol = 1e-9 if prec == dd.DD_MIXED else 1e-4
    assert np.allclose(hf[:m], hu[:m], rtol=tol, atol=0), (hf[:m], hu[:m])
    assert float(torch.linalg.norm(xf - xu) / torch.linalg.norm(xu)) < 1e-5


def test_fused_bit_reproducible():
    p, s = case("rand64_auto")
    b = torch.as_tensor(p.b, device="cuda")
    x1, i1 = s.solve(b, rtol=1e-8)
    for _ in range(3):
        x2, i2 = s.solve(b, rtol=1e-8)
        assert i2["fused"] == 1 and i2["iters"] == i1["iters"] and torch.equal(x2, x1)


def test_fused_steps_aside():
    """Per-apply profiling, another apply variant or the global ILU0
    preconditioner take the two-launch path; so does a new handle, on which
    fusion is off by default."""
    p, s = case("rand_ragged")
    b = torch.as_tensor(p.b, device="cuda")
    dd.dd_set_profiling(s.h, True)
    try:
        _, info = s.solve(b, rtol=1e-8)
    finally:
        dd.dd_set_profiling(s.h, False)
    assert info["fused"] == 0 and info["status"] == dd.DD_OK and info["apply_seconds"] > 0
    dd.dd_set_apply_variant(s.h, 1)
    try:
        _, info = s.solve(b, rtol=1e-8)
    finally:
        dd.dd_set_apply_variant(s.h, 0)
    assert info["fused"] == 0 and info["status"] == dd.DD_OK
    dd.dd_global_factor(s.h)
    dd.dd_set_preconditioner(s.h, 1)
    try:
        _, info = s.solve(b, rtol=1e-8)
    finally:
        dd.dd_set_preconditioner(s.h, 0)
    assert info["fused"] == 0 and info["status"] == dd.DD_OK
    _, info = s.solve(b, rtol=1e-8)
    assert info["fused"] == 1
    s2 = DDSolver.from_problem(p, sub=CASES["rand_ragged"][1])
    _, info = s2.solve(b, rtol=1e-8)
    assert info["fused"] == 0 and info["status"] == dd.DD_OK


def test_fused_converged_and_maxit():
    """Solves that stop early (by maxit, or at once by a loose rtol) leave the
    flags and the ticket counter consistent for the next solve."""
    p, s = case("rand_ragged")
    b = torch.as_tensor(p.b, device="cuda")
    _, info = s.solve(b, rtol=1e-30, maxit=1)
    assert info["status"] == dd.DD_ENOCONV and info["fused"] == 1
    _, info = s.solve(b, rtol=1.0, maxit=5)
    assert info["status"] == dd.DD_OK
    x, info = s.solve(b, rtol=1e-8)
    dd.dd_set_fusion(s.h, False)
    try:
        xu, infou = s.solve(b, rtol=1e-8)
    finally:
        dd.dd_set_fusion(s.h, True)
    assert info["status"] == dd.DD_OK and info["fused"] == 1
    assert float(torch.linalg.norm(x - xu) / torch.linalg.norm(xu)) < 1e-5


def test_fused_fullsize():
    """The benchmark's 160^3 workload: the fused solve's first iterations
    agree with the two-launch solve's to rounding, the full solve converges
    to the same solution, and two fused solves are bit-identical."""
    print("[fused fullsize] generating lognormal160_bsr3", flush=True)
    p = make_workload("lognormal160_bsr3")
    s = DDSolver.from_problem(p)
    dd.dd_set_fusion(s.h, True)
    b = torch.as_tensor(p.b, device="cuda")
    _, i_f, hf = solve_with_history(s, b, True, k=8, rtol=1e-30)
    _, i_u, hu = solve_with_history(s, b, False, k=8, rtol=1e-30)
    print(f"[fused fullsize] history fused {hf}\n[fused fullsize] history two  {hu}", flush=True)
    assert i_f["fused"] == 1 and i_u["fused"] == 0
    assert np.allclose(hf, hu, rtol=1e-9, atol=0)
    x1, i1 = s.solve(b, rtol=1e-8)
    x2, i2 = s.solve(b, rtol=1e-8)
    dd.dd_set_fusion(s.h, False)
    try:
        xu, iu = s.solve(b, rtol=1e-8)
    finally:
        dd.dd_set_fusion(s.h, True)
    print(f"[fused fullsize] iters fused {i1['iters']} two-launch {iu['iters']} "
          f"solve s {i1['solve_seconds']:.3f} / {iu['solve_seconds']:.3f}", flush=True)
    assert i1["status"] == dd.DD_OK and i1["rel_res_true"] <= 2e-8 and i1["fused"] == 1
    assert i2["iters"] == i1["iters"] and torch.equal(x1, x2)
    assert abs(i1["iters"] - iu["iters"]) <= max(3, iu["iters"] // 10)
    assert float(torch.linalg.norm(x1 - xu) / torch.linalg.norm(xu)) < 1e-5
