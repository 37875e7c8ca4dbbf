"""GPU parity at the benchmark's full size and launch configuration: the
160^3 log-normal 3x3 BSR workload (4,096,000 block rows, 28,518,400 blocks)
with the automatic partition, checked against the oracle on the same
matrix."""

import numpy as np
import pytest

import oracle as O
from parity import check_close, check_spmv, dd_scale
from problems import make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402


@pytest.fixture(scope="module")
def full():
    print("[fullsize] generating lognormal160_bsr3", flush=True)
    p = make_workload("lognormal160_bsr3")
    s = DDSolver.from_problem(p)
    inf = s.info
    print(f"[fullsize] GPU setup done, subdomain {inf['sx']}x{inf['sy']}x{inf['sz']}", flush=True)
    st = O.setup(p, (inf["sx"], inf["sy"], inf["sz"]))
    print("[fullsize] oracle setup done", flush=True)
    return p, s, st


def np_(t):
    return t.detach().cpu().numpy()


def test_fullsize_partition_and_levels(full):
    p, s, st = full
    pid, n2o, o2n = dd.dd_get_partition(s.h)
    assert np.array_equal(np_(n2o), st.new2old)
    assert s.info["nnzb_dropped"] == st.tcol.shape[0]
    for which in (0, 1):
        nlev, lptr, rows = dd.dd_get_levels(s.h, which)
        onl, optr, orows = st.levels(which)
        assert np.array_equal(np_(nlev), onl)
        assert np.array_equal(np_(lptr), optr)
        assert np.array_equal(np_(rows), orows)


def test_fullsize_apply_fp64(full):
    p, s, st = full
    r = np.random.default_rng(31).standard_normal(st.n * 3)
    zo = st.apply(r)
    zg = np_(s.apply(torch.as_tensor(r, device="cuda")))
    check_close(zg, zo, 3, 1e-12, what="fullsize apply", scale=dd_scale(st, r))
    # per-subdomain check: no subdomain is off (a wrong workgroup would hide in the norm)
    e_sub = np.linalg.norm((zg - zo).reshape(st.nsub, -1), axis=1) / np.linalg.norm(zo.reshape(st.nsub, -1), axis=1)
    assert e_sub.max() < 1e-11


def test_fullsize_spmv(full):
    p, s, st = full
    x = np.random.default_rng(32).standard_normal(st.n * 3)
    yo = st.spmv(x)
    yg = np_(s.spmv(torch.as_tensor(x, device="cuda")))
    check_spmv(st, x, yg, yo, "fullsize")


def test_fullsize_bicgstab_first_iterations(full):
    """The first iterations' residual history matches the oracle's."""
    p, s, st = full
    k = 6
    ref = st.bicgstab(p.b, rtol=1e-30, maxit=k)
    hist = torch.full((k + 1,), float("nan"), dtype=torch.float64, device="cuda")
    dd.dd_set_residual_history(s.h, hist)
    x, info = s.solve(torch.as_tensor(p.b, device="cuda"), rtol=1e-30, maxit=k)
    dd.dd_set_residual_history(s.h, None)
    hg = np_(hist)
    print(f"[fullsize] history gpu {hg}\n[fullsize] history ora {ref.history}", flush=True)
    assert info["iters"] == k
    assert np.allclose(hg, ref.history, rtol=1e-8, atol=0)


@pytest.mark.parametrize("prec", [dd.DD_FP64, dd.DD_MIXED, dd.DD_FP32], ids=["fp64", "mixed", "fp32"])
def test_fullsize_solve_true_residual(full, prec):
    """Full solves in each precision: DD_OK implies a true residual within
    2 rtol (an FP32 trisolve drifts, the solver restarts from its iterate),
    and the solution agrees with the FP64 one to the conditioning of the
    stopping test."""
    p, s, st = full
    b = torch.as_tensor(p.b, device="cuda")
    s.set_precision(dd.DD_FP64)
    x64, i64 = s.solve(b, rtol=1e-8)
    s.set_precision(prec)
    try:
        x, info = s.solve(b, rtol=1e-8)
    finally:
        s.set_precision(dd.DD_FP64)
    print(f"[fullsize] precision {prec}: {info}", flush=True)
    assert i64["status"] == dd.DD_OK and i64["rel_res_true"] <= 2e-8
    assert info["status"] in (dd.DD_OK, dd.DD_ENOCONV)
    if info["status"] == dd.DD_OK:
        assert info["rel_res_true"] <= 2e-8
        assert float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64)) < 1e-5
    else:
        assert info["restarts"] == 4 or info["iters"] >= 10000


def test_fullsize_learned_correction(full):
    """The learned interface correction at full size with the shipped
    parameters: faces bit-exact, features and MLP coefficients on sampled
    faces, and the corrected apply (with the GPU's coefficients) against the
    oracle's corrected apply."""
    from paper_2508_04917_amd.lic import load_params
    p, s, st = full
    L = O.LicOracle(st)
    print(f"[fullsize] oracle faces: {L.nf}", flush=True)
    P = load_params()[0]
    dd.lic_setup(s.h)
    dd.lic_set_params(s.h, torch.as_tensor(P, device="cuda"))
    try:
        fI, fJ, X = dd.lic_get_faces(s.h)
        assert np.array_equal(np_(fI), L.faces[0]) and np.array_equal(np_(fJ), L.faces[1])
        idx = np.random.default_rng(33).choice(L.nf, 4096, replace=False)
        Xg = np_(X)[idx].astype(np.float64)
        assert np.allclose(Xg, L.X[idx], rtol=1e-6, atol=1e-7)
        Cg = dd.lic_get_coeffs(s.h, L.nf)
        Co = O.mlp_forward(P.astype(np.float64), L.X[idx])[2].reshape(-1, 3, 3)
        check_close(np_(Cg)[idx], Co, 9, 1e-5, what="fullsize sampled MLP coefficients")
        dd.lic_set_coeffs(s.h, Cg)
        r = np.random.default_rng(34).standard_normal(st.n * 3)
        zg = np_(s.apply(torch.as_tensor(r, device="cuda")))
        C64 = np_(Cg).astype(np.float64)
        zo = L.apply(C64, r)
        sc = dd_scale(st, O.lic_correct(st.n, L.faces, np.abs(C64), np.abs(r)))
        check_close(zg, zo, 3, 1e-12, what="fullsize corrected apply", scale=sc)
    finally:
        dd.lic_set_params(s.h, None)
