"""bicgstab_solve_noalloc: the BiCGSTAB solve with its Krylov workspace in
the library's fixed device array instead of buffers the handle allocates.

It runs the same kernels in the same launch configuration as bicgstab_solve
(the fused apply + SpMV launch is off by default, and the solve's dot
products are reduced in a fixed order), so on the same handle and inputs the
two give the same iterations and bit-identical iterates; every check below
is that equality, through the C ABI.  The fixed array keeps the previous
call's contents, so the calls come in a row on different problems, the
second smaller than the first, then a learned solve that falls back to the
plain one (the initial guess is kept in the fixed array meanwhile)."""

import numpy as np
import pytest

from problems import laplacian_scalar, lic_init_params, random_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402

# 128 MiB: 11 vectors of n*bs FP64 values, the partial sums and the scalars
FIXED_BYTES = 128 << 20


def _solve_pair(s, b, x0, rtol=1e-8, maxit=2000):
    """(x, info) of bicgstab_solve and of bicgstab_solve_noalloc from x0."""
    xa, ia = dd.bicgstab_solve(s.h, b, x0.clone(), rtol=rtol, maxit=maxit)
    xb, ib = dd.bicgstab_solve_noalloc(s.h, b, x0.clone(), rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    return (xa, ia), (xb, ib)


def _same(a, b, what):
    (xa, ia), (xb, ib) = a, b
    print(f"[noalloc] {what}: bicgstab_solve {ia['iters']} it status {ia['status']}, "
          f"noalloc {ib['iters']} it status {ib['status']}", flush=True)
    for k in ("iters", "status", "restarts", "fallback"):
        assert ia[k] == ib[k], (what, k, ia[k], ib[k])
    assert ia["rel_res"] == ib["rel_res"] and ia["rel_res_true"] == ib["rel_res_true"], what
    assert torch.equal(xa, xb), f"{what}: iterates differ"
    assert ib["solve_seconds"] > 0.0 and ib["applies"] == 0 and ib["fused"] == 0


def test_noalloc_matches_bicgstab_solve_two_calls():
    # call 1: 3x3 blocks, 32^3 grid, 64 subdomains (98,304 unknowns)
    print("[noalloc] case 1: random 3x3 blocks 32^3, subdomains 8x8x16", flush=True)
    p1 = random_blocks(32, 32, 32, seed=21)
    s1 = DDSolver.from_problem(p1, sub=(8, 8, 16))
    b1 = torch.as_tensor(p1.b, device="cuda")
    x01 = torch.zeros_like(b1)
    r1 = _solve_pair(s1, b1, x01)
    _same(*r1, "call 1 (32^3, 3x3)")
    assert r1[0][1]["status"] == dd.DD_OK and r1[0][1]["rel_res_true"] <= 2e-8

    # call 2, smaller: scalar 16^3 Laplacian, 8 subdomains (4,096 unknowns),
    # with a nonzero initial guess; the fixed array still holds call 1's data
    print("[noalloc] case 2: scalar Laplacian 16^3, subdomains 8^3", flush=True)
    p2 = laplacian_scalar(16, 16, 16, seed=1)
    s2 = DDSolver.from_problem(p2, sub=(8, 8, 8))
    b2 = torch.as_tensor(p2.b, device="cuda")
    x02 = torch.as_tensor(np.random.default_rng(4).standard_normal(p2.n) * 1e-2, device="cuda")
    r2 = _solve_pair(s2, b2, x02)
    _same(*r2, "call 2 (16^3, scalar)")
    assert r2[0][1]["status"] == dd.DD_OK

    # call 3, back on the first handle: a stopped solve (maxit) agrees too
    r3 = _solve_pair(s1, b1, x01, rtol=1e-30, maxit=5)
    _same(*r3, "call 3 (32^3, maxit 5)")
    assert r3[0][1]["status"] == dd.DD_ENOCONV and r3[0][1]["iters"] == 5
    s1.close()
    s2.close()


def test_noalloc_takes_no_device_memory():
    """On a fresh handle the regular solve takes its workspace (11 vectors)
    on its first call; the noalloc solve takes none.  Checked only when the
    free-memory reading does see the regular solve's workspace."""
    print("[noalloc] case 3: random 3x3 blocks 32x32x48, subdomains 16^3, fresh handle", flush=True)
    p = random_blocks(32, 32, 48, seed=22)
    s = DDSolver.from_problem(p, sub=(16, 16, 16))
    b = torch.as_tensor(p.b, device="cuda")
    x0 = torch.zeros_like(b)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    xb, ib = dd.bicgstab_solve_noalloc(s.h, b, x0.clone(), rtol=1e-8, maxit=2000)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    xa, ia = dd.bicgstab_solve(s.h, b, x0.clone(), rtol=1e-8, maxit=2000)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    work = 11 * p.n * 3 * 8
    print(f"[noalloc] free memory: -{free0 - free1} B across the noalloc call, "
          f"-{free1 - free2} B across the first regular call (workspace {work} B)", flush=True)
    _same((xa, ia), (xb, ib), "fresh handle (32x32x48, 3x3)")
    if free1 - free2 >= work:  # the reading sees the regular solve's workspace
        assert free0 - free1 < work // 2, "bicgstab_solve_noalloc took device memory"
    s.close()


def test_noalloc_learned_fallback_and_precisions():
    """Mixed-precision factors, the learned correction and its fallback to
    plain DD-ILU0 (poisoned network output) through the fixed workspace."""
    print("[noalloc] case 4: random 3x3 blocks 24x16x16, subdomains 8^3, learned", flush=True)
    p = random_blocks(24, 16, 16, seed=17)
    s = DDSolver.from_problem(p, sub=(8, 8, 8))
    b = torch.as_tensor(p.b, device="cuda")
    x0 = torch.as_tensor(np.random.default_rng(5).standard_normal(p.n * 3) * 1e-3, device="cuda")
    s.set_precision(dd.DD_MIXED)
    _same(*_solve_pair(s, b, x0), "mixed precision")
    dd.lic_setup(s.h)
    P = lic_init_params(5)
    P[5952:] = 0.01 * np.random.default_rng(6).standard_normal(P.size - 5952)  # small nonzero output layer
    dd.lic_set_params(s.h, torch.as_tensor(P, dtype=torch.float32, device="cuda"))
    r = _solve_pair(s, b, x0)
    _same(*r, "learned, mixed precision")
    assert r[0][1]["fallback"] == 0
    P[5952:] = np.nan
    dd.lic_set_params(s.h, torch.as_tensor(P, dtype=torch.float32, device="cuda"))
    r = _solve_pair(s, b, x0)
    _same(*r, "poisoned learned -> plain fallback")
    assert r[0][1]["fallback"] == 1 and r[0][1]["status"] == dd.DD_OK
    dd.lic_set_params(s.h, None)
    plain = _solve_pair(s, b, x0)
    assert torch.equal(plain[1][0], r[1][0]), "the fallback's result must be the plain solve from x0"
    s.close()


def test_noalloc_rejects_problems_beyond_the_fixed_array():
    """A problem whose workspace exceeds the fixed array is refused before
    anything runs, and x is left untouched."""
    print("[noalloc] case 5: random 3x3 blocks 128x64x64 (too large for the fixed array)", flush=True)
    p = random_blocks(128, 64, 64, seed=23)
    assert 11 * p.n * 3 * 8 > FIXED_BYTES
    s = DDSolver.from_problem(p, sub=(16, 16, 16))
    b = torch.as_tensor(p.b, device="cuda")
    x = torch.full_like(b, 0.5)
    with pytest.raises(dd.DDError) as e:
        dd.bicgstab_solve_noalloc(s.h, b, x, rtol=1e-8, maxit=10)
    assert e.value.code == dd.DD_EINVAL and "fixed array" in str(e.value)
    torch.cuda.synchronize()
    assert bool((x == 0.5).all())
    s.close()
