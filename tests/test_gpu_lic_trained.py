"""The committed, trained interface-correction network on unseen problems:
its held-out loss is well below 1 (the plain DD-ILU0 apply) and the learned
preconditioner needs fewer BiCGSTAB iterations than plain DD-ILU0, in FP64
and with FP32 factors.  Problems: 64^3 log-normal fields (sigma = 2, seeds
outside the training and validation ranges), 16^3 subdomains as in
training."""

import os

import numpy as np
import pytest

from problems import lognormal_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd import lic  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402

SUB = (16, 16, 16)
SEEDS = (2100, 2101)


@pytest.fixture(scope="module")
def params():
    assert os.path.exists(lic.DEFAULT_PARAMS), "trained parameters are part of the package"
    P, meta = lic.load_params()
    assert P.shape == (dd.LIC_NPARAM,) and np.isfinite(P).all()
    return P


@pytest.mark.parametrize("seed", SEEDS)
def test_heldout_loss_below_one(params, seed):
    print(f"[lic-trained] held-out loss, 64^3 seed {seed}", flush=True)
    p = lognormal_problem(64, 64, 64, seed=seed, sigma=2.0)
    loss = lic.heldout_loss(params, p, SUB, nq=8, probe_seed=seed)
    assert loss < 0.5, loss


@pytest.mark.parametrize("prec", [dd.DD_FP64, dd.DD_MIXED], ids=["fp64", "mixed"])
def test_learned_needs_fewer_iterations(params, prec):
    plain, learned = 0, 0
    for seed in SEEDS:
        print(f"[lic-trained] solves, 64^3 seed {seed}, precision {prec}", flush=True)
        p = lognormal_problem(64, 64, 64, seed=seed, sigma=2.0)
        s = DDSolver.from_problem(p, sub=SUB)
        try:
            s.set_precision(prec)
            b = torch.as_tensor(p.b, device="cuda")
            _, i0 = s.solve(b, rtol=1e-8)
            dd.lic_setup(s.h)
            dd.lic_set_params(s.h, torch.as_tensor(params, device="cuda"))
            _, i1 = s.solve(b, rtol=1e-8)
        finally:
            s.close()
        assert i0["status"] == 0 and i1["status"] == 0
        assert i1["rel_res_true"] <= 2e-8
        plain += i0["iters"]
        learned += i1["iters"]
    assert learned <= 0.95 * plain, (plain, learned)
