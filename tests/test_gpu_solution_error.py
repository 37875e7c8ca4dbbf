"""Errors of the reduced-precision and learned solves against the FP64
oracle.  The FP32-factor variants and the learned interface correction are
additions to the paper's method (its solves are FP64 throughout); each
result's error is stated against the oracle's FP64 BiCGSTAB solution on the
same system:

- the oracle recomputes the GPU solution's residual ||b - A x|| / ||b|| with
  its own FP64 SpMV: it must meet the solver's guarantee, 2 rtol;
- ||x - x_oracle|| / ||x_oracle||, where both solutions satisfy the stopping
  test, is bounded by cond(A) (res_gpu + res_oracle); the bound used, 1e-5,
  allows cond(A) up to about 300 at these residuals, and the measured values
  (printed) are far below it.

Workloads: the 64^3 3x3 random-block operator with the automatic partition
(8x8x16), and a 64^3 log-normal field (sigma = 2) with 16^3 subdomains, the
shape the learned correction is trained on."""

import numpy as np
import pytest

import oracle as O
from problems import lognormal_problem, random_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.lic import load_params  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402

RTOL = 1e-8
XERR_BOUND = 1e-5

CASES = {
    "rand64_auto": (lambda: random_blocks(64, 64, 64, seed=2), (0, 0, 0)),
    "logn64_sub16": (lambda: lognormal_problem(64, 64, 64, seed=2102, sigma=2.0), (16, 16, 16)),
}
_cache = {}


def case(name):
    if name not in _cache:
        make, sub = CASES[name]
        p = make()
        s = DDSolver.from_problem(p, sub=sub)
        inf = s.info
        print(f"[solution error {name}] oracle setup and FP64 solve, subdomain "
              f"{inf['sx']}x{inf['sy']}x{inf['sz']}", flush=True)
        st = O.setup(p, (inf["sx"], inf["sy"], inf["sz"]))
        ref = st.bicgstab(p.b, rtol=RTOL)
        assert ref.status == 0
        print(f"[solution error {name}] oracle {ref.iters} iterations", flush=True)
        _cache[name] = (p, s, st, ref)
    return _cache[name]


VARIANTS = [("fp64", dd.DD_FP64, False), ("mixed", dd.DD_MIXED, False), ("fp32", dd.DD_FP32, False),
            ("learned_mixed", dd.DD_MIXED, True), ("learned_fp32", dd.DD_FP32, True)]


@pytest.mark.parametrize("variant", VARIANTS, ids=[v[0] for v in VARIANTS])
@pytest.mark.parametrize("name", list(CASES))
def test_solution_against_oracle(name, variant):
    label, prec, learned = variant
    p, s, st, ref = case(name)
    b = torch.as_tensor(p.b, device="cuda")
    s.set_precision(prec)
    if learned:
        dd.lic_setup(s.h)
        dd.lic_set_params(s.h, torch.as_tensor(load_params()[0], device="cuda"))
    try:
        x, info = s.solve(b, rtol=RTOL)
    finally:
        dd.lic_set_params(s.h, None)
        s.set_precision(dd.DD_FP64)
    xg = x.cpu().numpy()
    res_o = np.linalg.norm(st.unpermute(st.spmv(st.permute(xg))) - p.b) / np.linalg.norm(p.b)
    xerr = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
    print(f"[solution error {name} {label}] {info['iters']} it (oracle FP64 {ref.iters}), "
          f"status {info['status']}, fallback {info['fallback']}, restarts {info['restarts']}; "
          f"oracle residual {res_o:.2e}, x vs oracle x {xerr:.2e}", flush=True)
    assert info["status"] == dd.DD_OK
    assert res_o <= 2 * RTOL
    assert xerr <= XERR_BOUND
