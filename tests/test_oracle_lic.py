"""Pins for the oracle's learned interface correction (an addition to the
paper's method): zero output reproduces the plain apply exactly, features
are scale invariant, forward/backward/Adam agree with independent library
implementations, the analytic gradient agrees with central differences, and
the free per-face least-squares fit bounds what any network can reach."""

import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as O
from problems import Problem, lic_init_params, lognormal_problem, probe_vectors

GOLDEN_FEATURES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lic_features_3cell.txt")


@pytest.fixture(scope="module")
def small():
    p = lognormal_problem(8, 8, 4, seed=5, sigma=1.0, corr_len=2.0)
    st = O.setup(p, (4, 4, 4))
    L = O.LicOracle(st)
    R = probe_vectors(5, 4, st.n * 3)
    Zs = np.stack([L.apply_global(r) for r in R])
    Zdd = np.stack([st.apply(r) for r in R])
    den = ((Zdd - Zs) ** 2).sum(axis=1)
    return p, st, L, R, Zs, den


def test_faces_are_the_dropped_blocks(small):
    p, st, L, *_ = small
    assert L.nf == st.acol.size - st.tcol.size
    fI, fJ, fq = L.faces
    assert np.all(fI // st.S != fJ // st.S)
    assert np.array_equal(st.acol[fq], fJ)


def test_zero_output_layer_is_plain_apply(small):
    """W3 = b3 = 0 at initialisation: C = 0 and the corrected apply equals the
    plain DD apply bit for bit."""
    p, st, L, R, *_ = small
    P = lic_init_params(3)
    C = L.coeffs(P)
    assert np.all(C == 0.0)
    assert np.array_equal(L.apply(C, R[0]), st.apply(R[0]))


def test_features_scale_invariant(small):
    p, st, L, *_ = small
    X2 = O.lic_features(st.aptr, st.acol, st.aval * 1234.5, L.faces)
    assert np.allclose(X2, L.X, rtol=1e-14, atol=1e-15)
    # the diagonal blocks of an interior cell: trace part 3, coupling about -1/6 each
    assert np.all(np.abs(L.X[:, 0] + L.X[:, 4] + L.X[:, 8]) > 0)


def _golden_features():
    blocks, faces = {}, []
    with open(GOLDEN_FEATURES) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "block":
                blocks[(int(w[1]), int(w[2]))] = np.array([float(v) for v in w[3:12]]).reshape(3, 3)
            elif w[0] == "face":
                faces.append((int(w[1]), int(w[2]), int(w[3]), [float(Fraction(v)) for v in w[4:]]))
    return blocks, faces


def test_features_hand_worked():
    """Faces and features of a three-cell chain cut into single cells,
    against values worked by hand (golden/lic_features_3cell.txt).  Every
    sigma is an exact integer (sqrt(324)/3, sqrt(81)/3), so each feature is
    one correctly rounded division and must equal the fraction exactly."""
    blocks, faces = _golden_features()
    n = 3
    ptr = [0]
    col, val = [], []
    for I in range(n):
        for J in range(n):
            if (I, J) in blocks:
                col.append(J)
                val.append(blocks[(I, J)])
        ptr.append(len(col))
    p = Problem(name="chain3", nx=3, ny=1, nz=1, bs=3, brow_ptr=np.array(ptr, dtype=np.int32),
                bcol=np.array(col, dtype=np.int32), val=np.array(val).reshape(-1), b=np.zeros(9), seed=0)
    st = O.setup(p, (1, 1, 1))
    L = O.LicOracle(st)
    fI, fJ, fq = L.faces
    assert list(zip(fI.tolist(), fJ.tolist())) == [(f[0], f[1]) for f in faces]
    assert np.array_equal(st.acol[fq], fJ)
    for k, (I, J, sigma, x) in enumerate(faces):
        assert np.array_equal(L.X[k], np.array(x)), (I, J, L.X[k], x)
    # the same features through the plain wrapper on the unreordered matrix
    X = O.lic_features(p.brow_ptr, p.bcol, p.val, L.faces)
    assert np.array_equal(X, L.X)


def test_mlp_forward_backward_against_torch(small):
    p, st, L, *_ = small
    rng = np.random.default_rng(0)
    P = rng.standard_normal(O.LIC_NPARAM) * 0.3
    X = L.X[:50]
    H1, H2, OUT = O.mlp_forward(P, X)
    t = torch.tensor(P, dtype=torch.float64, requires_grad=True)
    W1 = t[0:1728].view(64, 27); b1 = t[1728:1792]
    W2 = t[1792:5888].view(64, 64); b2 = t[5888:5952]
    W3 = t[5952:6528].view(9, 64); b3 = t[6528:6537]
    xt = torch.tensor(X)
    out = torch.nn.functional.linear(torch.relu(torch.nn.functional.linear(
        torch.relu(torch.nn.functional.linear(xt, W1, b1)), W2, b2)), W3, b3)
    assert np.allclose(OUT, out.detach().numpy(), rtol=1e-13, atol=1e-13)
    dOUT = rng.standard_normal(OUT.shape)
    (out * torch.tensor(dOUT)).sum().backward()
    dP = O.mlp_backward(P, X, H1, H2, dOUT)
    assert np.allclose(dP, t.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_adam_against_torch():
    rng = np.random.default_rng(1)
    P = rng.standard_normal(40)
    M, V = np.zeros(40), np.zeros(40)
    t = torch.tensor(P.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        G = rng.standard_normal(40)
        O.adam(P, G, M, V, step, lr=1e-2)
        opt.zero_grad()
        t.grad = torch.tensor(G)
        opt.step()
    assert np.allclose(P, t.detach().numpy(), rtol=1e-12, atol=1e-13)


def test_loss_gradient_central_differences(small):
    """Analytic gradient (adjoint apply + backprop) vs central differences."""
    p, st, L, R, Zs, den = small
    rng = np.random.default_rng(2)
    P = lic_init_params(4)
    P[5952:] = rng.standard_normal(585) * 0.05  # nonzero output layer
    loss, g = L.loss_and_grad(P, R, Zs, den)
    idx = np.concatenate([rng.integers(0, 1728, 4), rng.integers(1792, 5888, 4), rng.integers(5952, 6537, 6)])
    for i in idx:
        h = 1e-6 * max(1.0, abs(P[i]))
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (L.loss_and_grad(Pp, R, Zs, den, want_grad=False)[0]
              - L.loss_and_grad(Pm, R, Zs, den, want_grad=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (i, fd, g[i])


def test_least_squares_bound(small):
    """z is linear in the per-face coefficients: a least-squares fit of free
    C_f on the probes bounds the loss any network can reach.  The bound is
    below 1 (a correction can help) and the untrained network sits at 1."""
    p, st, L, R, Zs, den = small
    n, nf = st.n, L.nf
    fI, fJ, _ = L.faces
    Q = R.shape[0]
    # column (f, a, b): M^{-1} e_{I_f,a} r_q[J_f, b], scaled by 1/sqrt(den_q)
    basis = {}
    for I in np.unique(fI):
        for a in range(3):
            e = np.zeros(3 * n)
            e[3 * I + a] = 1.0
            basis[(I, a)] = st.apply(e)
    cols = []
    for f in range(nf):
        for a in range(3):
            for b in range(3):
                cols.append(np.concatenate([basis[(fI[f], a)] * R[q][3 * fJ[f] + b] / np.sqrt(den[q])
                                            for q in range(Q)]))
    D = np.stack(cols, axis=1)
    Zdd = np.stack([st.apply(r) for r in R])
    rhs = np.concatenate([(Zs[q] - Zdd[q]) / np.sqrt(den[q]) for q in range(Q)])
    coef, *_ = np.linalg.lstsq(D, rhs, rcond=None)
    ls_loss = ((D @ coef - rhs) ** 2).sum() / Q
    assert ls_loss < 0.9
    # the same loss through the correction + apply path, and a zero gradient
    # (adjoint apply + dC) at the minimiser
    C_ls = coef.reshape(nf, 3, 3)

    def loss_and_dC(C):
        A = np.empty_like(R)
        loss = 0.0
        for q in range(Q):
            e = L.apply(C, R[q]) - Zs[q]
            loss += (e @ e) / den[q] / Q
            A[q] = O.apply_transpose(n, 3, st.tptr, st.tcol, st.f, 2.0 * e / (Q * den[q]))
        return loss, O.lic_dC(n, L.faces, A, R)

    loss_ls2, g_ls = loss_and_dC(C_ls)
    loss_zero, g_zero = loss_and_dC(np.zeros_like(C_ls))
    assert abs(loss_ls2 - ls_loss) <= 1e-10 * ls_loss
    assert abs(loss_zero - 1.0) < 1e-12
    assert np.linalg.norm(g_ls) <= 1e-7 * np.linalg.norm(g_zero)
    P = lic_init_params(0)
    loss0, _ = L.loss_and_grad(P, R, Zs, den, want_grad=False)
    assert abs(loss0 - 1.0) < 1e-12
    # a few Adam steps reduce the loss but never below the bound
    M, V = np.zeros_like(P), np.zeros_like(P)
    for t in range(1, 31):
        loss, g = L.loss_and_grad(P, R, Zs, den)
        O.adam(P, g, M, V, t, lr=1e-3)
    loss_end, _ = L.loss_and_grad(P, R, Zs, den, want_grad=False)
    assert ls_loss - 1e-9 <= loss_end < loss0


def test_global_ilu0_defining_property(small):
    """Global factors of the full reordered matrix: (L U)_IJ = A_IJ on A's pattern."""
    p, st, L, *_ = small
    f = L.global_factors()
    n = st.n
    Ld = np.eye(3 * n)
    Ud = np.zeros((3 * n, 3 * n))
    A = np.zeros((3 * n, 3 * n))
    mask = np.zeros((3 * n, 3 * n), dtype=bool)
    for I in range(n):
        for q in range(st.aptr[I], st.aptr[I + 1]):
            J = st.acol[q]
            sl = (slice(3 * I, 3 * I + 3), slice(3 * J, 3 * J + 3))
            A[sl] = st.aval[q]
            mask[sl] = True
            if J < I:
                Ld[sl] = f[q]
            elif J == I:
                Ud[sl] = np.linalg.inv(f[q])
            else:
                Ud[sl] = np.linalg.inv(f[st.aptr[I] + int(np.where(st.acol[st.aptr[I]:st.aptr[I + 1]] == I)[0][0])]) @ f[q]
    assert np.abs((Ld @ Ud - A)[mask]).max() < 1e-12 * np.abs(A).max()
