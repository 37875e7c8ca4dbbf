"""The learned correction's fallback to plain DD-ILU0, inside the library
(dd_set_lic_fallback): a learned solve that breaks down or misses maxit is
repeated from the caller's initial guess with the correction off, and the
solve reports it.  Poisoned network parameters (non-finite output layer)
force the breakdown; the plain rerun must then be exactly the plain solve."""

import numpy as np
import pytest

from problems import lic_init_params, lognormal_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.lic import load_params  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402


@pytest.fixture(scope="module")
def prob():
    print("[fallback] lognormal 24x32x40, subdomains 12x16x20", flush=True)
    p = lognormal_problem(24, 32, 40, seed=7, sigma=2.0)
    s = DDSolver.from_problem(p, sub=(12, 16, 20))
    dd.lic_setup(s.h)
    return p, s


def poisoned_params():
    P = lic_init_params(5)
    P[5952:] = np.nan  # output layer: every coefficient C_f is NaN
    return torch.as_tensor(P, dtype=torch.float32, device="cuda")


def test_poisoned_learned_solve_falls_back(prob):
    p, s = prob
    b = torch.as_tensor(p.b, device="cuda")
    x0 = torch.as_tensor(np.random.default_rng(3).standard_normal(p.n * 3) * 1e-3, device="cuda")
    xp, ip = s.solve(b, x=x0.clone(), rtol=1e-8)
    assert ip["status"] == dd.DD_OK and ip["fallback"] == 0
    dd.lic_set_params(s.h, poisoned_params())
    try:
        # fallback off: the learned solve breaks down and says so
        dd.dd_set_lic_fallback(s.h, False)
        _, ib = s.solve(b, x=x0.clone(), rtol=1e-8)
        print(f"[fallback] poisoned, fallback off: {ib}", flush=True)
        assert ib["status"] == dd.DD_EBREAKDOWN and ib["fallback"] == 0
        # fallback on (the default): plain DD-ILU0 from the same initial guess
        dd.dd_set_lic_fallback(s.h, True)
        xf, inf = s.solve(b, x=x0.clone(), rtol=1e-8)
        print(f"[fallback] poisoned, fallback on: {inf}", flush=True)
        assert inf["status"] == dd.DD_OK and inf["fallback"] == 1
        assert inf["iters"] == ip["iters"] and inf["rel_res_true"] <= 2e-8
        assert torch.equal(xf, xp), "the rerun must be the plain solve from the caller's x0"
        assert inf["solve_seconds"] > 0.0
        # the correction stays on for later calls: the apply still reads NaN coefficients
        z = s.apply(b)
        assert not torch.isfinite(z).all()
    finally:
        dd.lic_set_params(s.h, None)
        dd.dd_set_lic_fallback(s.h, True)


def test_maxit_learned_solve_falls_back(prob):
    """A learned solve cut off by maxit is also repeated plainly (with the
    same maxit, which the plain solve may or may not meet)."""
    p, s = prob
    b = torch.as_tensor(p.b, device="cuda")
    P = torch.as_tensor(load_params()[0], device="cuda")
    dd.lic_set_params(s.h, P)
    try:
        _, i1 = s.solve(b, rtol=1e-30, maxit=3)
    finally:
        dd.lic_set_params(s.h, None)
    _, i0 = s.solve(b, rtol=1e-30, maxit=3)
    assert i1["fallback"] == 1 and i1["status"] == dd.DD_ENOCONV and i1["iters"] == 3
    assert i0["fallback"] == 0 and i0["status"] == dd.DD_ENOCONV
    assert i1["rel_res"] == i0["rel_res"]


def test_successful_learned_solve_keeps_its_result(prob):
    p, s = prob
    b = torch.as_tensor(p.b, device="cuda")
    P = torch.as_tensor(load_params()[0], device="cuda")
    dd.lic_set_params(s.h, P)
    try:
        x1, i1 = s.solve(b, rtol=1e-8)
        dd.dd_set_lic_fallback(s.h, False)
        x2, i2 = s.solve(b, rtol=1e-8)
    finally:
        dd.dd_set_lic_fallback(s.h, True)
        dd.lic_set_params(s.h, None)
    _, ip = s.solve(b, rtol=1e-8)
    print(f"[fallback] learned {i1['iters']} it, plain {ip['iters']} it", flush=True)
    assert i1["status"] == dd.DD_OK and i1["fallback"] == 0
    assert i1["iters"] == i2["iters"] and torch.equal(x1, x2)
    assert i1["iters"] < ip["iters"]
