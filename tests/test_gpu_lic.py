"""GPU parity of the global ILU0 path and of the learned interface correction
(faces, features, MLP, corrected apply, adjoint apply, targets, loss and
gradient, Adam) against the CPU oracle on the same seeded inputs."""

import numpy as np
import pytest

import oracle as O
from parity import apply_scale, check_close, check_layers, dd_scale
from problems import lic_init_params, lognormal_problem, probe_vectors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_04917_amd import ddilu as dd  # noqa: E402
from paper_2508_04917_amd.solver import DDSolver  # noqa: E402


@pytest.fixture(scope="module")
def prob():
    print("[lic] problem 16x12x8, subdomains 8x6x4", flush=True)
    p = lognormal_problem(16, 12, 8, seed=41, sigma=1.5, corr_len=3.0)
    s = DDSolver.from_problem(p, sub=(8, 6, 4))
    st = O.setup(p, (8, 6, 4))
    L = O.LicOracle(st)
    dd.lic_setup(s.h)
    dd.dd_global_factor(s.h)
    return p, s, st, L


def np_(t):
    return t.detach().cpu().numpy()


def cu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def trained_like_params(seed=7):
    P = lic_init_params(seed)
    P[5952:] = np.random.default_rng(seed).standard_normal(585) * 0.05
    return P


def test_faces_and_features(prob):
    p, s, st, L = prob
    fI, fJ, X = dd.lic_get_faces(s.h)
    assert np.array_equal(np_(fI), L.faces[0])
    assert np.array_equal(np_(fJ), L.faces[1])
    assert np.allclose(np_(X), L.X, rtol=1e-6, atol=1e-7)


def test_global_apply_parity(prob):
    p, s, st, L = prob
    R = probe_vectors(3, 2, st.n * 3)
    Z = np_(dd.dd_global_apply(s.h, cu(R.reshape(-1)), nrhs=2)).reshape(2, -1)
    for q in range(2):
        zo = L.apply_global(R[q])
        sc = apply_scale(st.n, 3, st.aptr, st.acol, L.global_factors(), R[q])
        check_close(Z[q], zo, 3, 1e-12, what=f"global apply probe {q}", scale=sc)


def test_global_preconditioned_bicgstab(prob):
    p, s, st, L = prob
    dd.dd_set_preconditioner(s.h, 1)
    try:
        x, info = s.solve(cu(p.b), rtol=1e-8)
    finally:
        dd.dd_set_preconditioner(s.h, 0)
    assert info["status"] == 0 and info["rel_res_true"] <= 2e-8
    xdd, idd = s.solve(cu(p.b), rtol=1e-8)
    assert info["iters"] <= idd["iters"]


def test_adjoint_apply_parity(prob):
    p, s, st, L = prob
    g = np.random.default_rng(4).standard_normal(st.n * 3)
    a = np_(dd.dd_apply_adjoint(s.h, cu(g)))
    ao = O.apply_transpose(st.n, 3, st.tptr, st.tcol, st.f, g)
    sc = apply_scale(st.n, 3, st.tptr, st.tcol, st.f, g, transpose=True)
    check_close(a, ao, 3, 1e-12, what="adjoint apply", scale=sc)


def test_zero_output_is_plain_apply(prob):
    p, s, st, L = prob
    r = cu(np.random.default_rng(5).standard_normal(st.n * 3))
    z0 = s.apply(r).clone()
    dd.lic_set_params(s.h, cu(lic_init_params(2), torch.float32))
    try:
        z1 = s.apply(r)
        assert torch.equal(z0, z1)
    finally:
        dd.lic_set_params(s.h, None)


def test_mlp_coefficients(prob):
    p, s, st, L = prob
    P = trained_like_params()
    dd.lic_set_params(s.h, cu(P, torch.float32))
    try:
        Cg = np_(dd.lic_get_coeffs(s.h, L.nf))
    finally:
        dd.lic_set_params(s.h, None)
    Co = L.coeffs(P)
    check_close(Cg, Co, 9, 1e-5, what="MLP coefficients per face")


@pytest.mark.parametrize("variant", [1, 3])
def test_corrected_apply_parity(prob, variant):
    p, s, st, L = prob
    Co = L.coeffs(trained_like_params()).astype(np.float32)
    dd.lic_set_coeffs(s.h, cu(Co, torch.float32))
    dd.dd_set_apply_variant(s.h, variant)
    try:
        r = np.random.default_rng(6).standard_normal(st.n * 3)
        zg = np_(s.apply(cu(r)))
    finally:
        dd.lic_set_coeffs(s.h, None)
        dd.dd_set_apply_variant(s.h, 0)
    zo = L.apply(Co.astype(np.float64), r)
    sc = dd_scale(st, O.lic_correct(st.n, L.faces, np.abs(Co.astype(np.float64)), np.abs(r)))
    check_close(zg, zo, 3, 1e-12, what=f"corrected apply v{variant}", scale=sc)


@pytest.mark.parametrize("variant", [1, 3])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_corrected_apply_several_passes(variant, prec):
    """Thin subdomains (4x4x12: levels of at most 16 rows, so one wavefront
    per workgroup) with 224 cut faces each: the correction's 672 items take
    two passes of the workgroup's lanes, and corner rows have three faces."""
    print("[lic] problem 16x16x24, subdomains 4x4x12 (several correction passes)", flush=True)
    p = lognormal_problem(16, 16, 24, seed=45, sigma=1.5, corr_len=3.0)
    s = DDSolver.from_problem(p, sub=(4, 4, 12))
    st = O.setup(p, (4, 4, 12))
    L = O.LicOracle(st)
    dd.lic_setup(s.h)
    Co = L.coeffs(trained_like_params()).astype(np.float32)
    dd.lic_set_coeffs(s.h, cu(Co, torch.float32))
    dd.dd_set_apply_variant(s.h, variant)
    r = np.random.default_rng(7).standard_normal(st.n * 3)
    if prec == "mixed":
        s.set_precision(dd.DD_MIXED)
        zo = st.apply_fp32_factors(O.lic_correct(st.n, L.faces, Co.astype(np.float64), r), round_input=False)
        tol = 1e-10
    else:
        zo = L.apply(Co.astype(np.float64), r)
        tol = 1e-12
    zg = np_(s.apply(cu(r)))
    s.close()
    sc = dd_scale(st, O.lic_correct(st.n, L.faces, np.abs(Co.astype(np.float64)), np.abs(r)))
    check_close(zg, zo, 3, tol, what=f"corrected apply, several passes, v{variant} {prec}", scale=sc)


def test_targets_loss_and_gradient(prob):
    """GPU FP32 network + FP64 applies vs the FP64 oracle: loss to 1e-5,
    gradient to 1e-3 (relative, in norm)."""
    p, s, st, L = prob
    Q = 4
    R = probe_vectors(41, Q, st.n * 3)
    Zs_g, den_g = dd.lic_targets(s.h, cu(R))
    Zs_o = np.stack([L.apply_global(r) for r in R])
    den_o = np.array([((st.apply(r) - z) ** 2).sum() for r, z in zip(R, Zs_o)])
    sc = np.concatenate([apply_scale(st.n, 3, st.aptr, st.acol, L.global_factors(), r) for r in R])
    check_close(np_(Zs_g), Zs_o, 3, 1e-12, what="global ILU0 targets", scale=sc)
    assert np.allclose(np_(den_g), den_o, rtol=1e-10)
    P = trained_like_params()
    loss_g, grad_g = dd.lic_loss_grad(s.h, cu(P, torch.float32), cu(R), Zs_g, den_g)
    P32 = P.astype(np.float32).astype(np.float64)
    loss_o, grad_o = L.loss_and_grad(P32, R, Zs_o, den_o)
    assert abs(float(loss_g.item()) - loss_o) / loss_o < 1e-5
    gg = np_(grad_g).astype(np.float64)
    assert np.linalg.norm(gg - grad_o) / np.linalg.norm(grad_o) < 1e-3
    check_layers(gg, grad_o, 1e-3, what="gradient")


def test_adam_step():
    rng = np.random.default_rng(3)
    P = rng.standard_normal(6537)
    G = rng.standard_normal(6537)
    Pg, Gg = cu(P, torch.float32), cu(G, torch.float32)
    M = torch.zeros_like(Pg)
    V = torch.zeros_like(Pg)
    Mo, Vo = np.zeros(6537), np.zeros(6537)
    Po = P.astype(np.float32).astype(np.float64)
    for t in (1, 2):
        dd.lic_adam(Pg, Gg, M, V, t, lr=1e-2)
        O.adam(Po, G.astype(np.float32).astype(np.float64), Mo, Vo, t, lr=1e-2)
    assert np.allclose(np_(Pg), Po, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss(prob):
    p, s, st, L = prob
    Q = 4
    R = cu(probe_vectors(41, Q, st.n * 3))
    Zs, den = dd.lic_targets(s.h, R)
    params = cu(lic_init_params(1), torch.float32)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    order = np.zeros((30, 1), dtype=np.int32)
    hist = dd.lic_train([s.h], [R], [Zs], [den], params, m, v, 30, order, lr=1e-3)
    assert abs(hist[0] - 1.0) < 1e-6  # untrained correction is zero: loss 1
    assert hist[-1] < hist[0]


@pytest.fixture(scope="module")
def prob16():
    """The training shape: 16^3 subdomains (here 32x32x16 cells, two by two
    by one subdomains), where lic_train runs."""
    print("[lic] problem 32x32x16, subdomains 16x16x16", flush=True)
    p = lognormal_problem(32, 32, 16, seed=43, sigma=2.0, corr_len=4.0)
    s = DDSolver.from_problem(p, sub=(16, 16, 16))
    st = O.setup(p, (16, 16, 16))
    L = O.LicOracle(st)
    dd.lic_setup(s.h)
    dd.dd_global_factor(s.h)
    return p, s, st, L


def test_adjoint_apply_parity_training_shape(prob16):
    p, s, st, L = prob16
    for seed in (4, 5):
        g = np.random.default_rng(seed).standard_normal(st.n * 3)
        a = np_(dd.dd_apply_adjoint(s.h, cu(g)))
        ao = O.apply_transpose(st.n, 3, st.tptr, st.tcol, st.f, g)
        sc = apply_scale(st.n, 3, st.tptr, st.tcol, st.f, g, transpose=True)
        check_close(a, ao, 3, 1e-12, what=f"adjoint apply 16^3 seed {seed}", scale=sc)


def test_loss_and_gradient_training_shape(prob16):
    """lic_loss_grad at the shape lic_train runs on, against the oracle:
    targets per block row to 1e-12, loss to 1e-5, gradient to 1e-3 in norm
    and per layer."""
    p, s, st, L = prob16
    Q = 4
    R = probe_vectors(43, Q, st.n * 3)
    Zs_g, den_g = dd.lic_targets(s.h, cu(R))
    Zs_o = np.stack([L.apply_global(r) for r in R])
    den_o = np.array([((st.apply(r) - z) ** 2).sum() for r, z in zip(R, Zs_o)])
    sc = np.concatenate([apply_scale(st.n, 3, st.aptr, st.acol, L.global_factors(), r) for r in R])
    check_close(np_(Zs_g), Zs_o, 3, 1e-12, what="16^3 targets", scale=sc)
    assert np.allclose(np_(den_g), den_o, rtol=1e-10)
    P = trained_like_params(11)
    loss_g, grad_g = dd.lic_loss_grad(s.h, cu(P, torch.float32), cu(R), Zs_g, den_g)
    P32 = P.astype(np.float32).astype(np.float64)
    loss_o, grad_o = L.loss_and_grad(P32, R, Zs_o, den_o)
    lerr = abs(float(loss_g.item()) - loss_o) / loss_o
    gg = np_(grad_g).astype(np.float64)
    gerr = np.linalg.norm(gg - grad_o) / np.linalg.norm(grad_o)
    print(f"[lic 16^3] loss {loss_o:.6f} rel err {lerr:.2e}, gradient rel err {gerr:.2e}", flush=True)
    assert lerr < 1e-5
    assert gerr < 1e-3
    check_layers(gg, grad_o, 1e-3, what="16^3 gradient")
