"""Pins of the oracle's full consistency step (paper Sec. 3.1, Eq. 1-8).

The screened-Poisson energy, its gradient and the momentum iteration are tied
to finite differences of the discrete energy, a direct sparse solve of the
Euler-Lagrange equation, exact conservation laws, and closed-form special
cases of the weights (Eq. 2-7).  CPU only.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import tcflow_oracle as O

RNG = np.random.default_rng(77)


def laplace_brute(X):
    C, H, W = X.shape
    out = np.zeros_like(X)
    for c in range(C):
        for y in range(H):
            for x in range(W):
                s = 0.0
                for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                    yy, xx = y + dy, x + dx
                    if 0 <= yy < H and 0 <= xx < W:
                        s += X[c, yy, xx] - X[c, y, x]
                out[c, y, x] = s
    return out


def forward_diff_matrix(H, W):
    """Sparse D stacking horizontal and vertical forward differences."""
    idx = np.arange(H * W).reshape(H, W)
    rows, cols, vals = [], [], []
    r = 0
    for y in range(H):
        for x in range(W - 1):
            rows += [r, r]; cols += [idx[y, x + 1], idx[y, x]]; vals += [1.0, -1.0]; r += 1
    for y in range(H - 1):
        for x in range(W):
            rows += [r, r]; cols += [idx[y + 1, x], idx[y, x]]; vals += [1.0, -1.0]; r += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(r, H * W))


def test_laplacian_brute_force_and_matrix():
    X = RNG.standard_normal((2, 7, 9))
    L = O.laplacian(X)
    assert np.allclose(L, laplace_brute(X), atol=1e-13)
    D = forward_diff_matrix(7, 9)
    for c in range(2):
        assert np.allclose(L[c].ravel(), -(D.T @ (D @ X[c].ravel())), atol=1e-12)
    assert np.allclose(L.sum(axis=(1, 2)), 0.0, atol=1e-12)
    assert np.all(O.laplacian(np.full((1, 4, 5), 3.0)) == 0)


def energy(Ov, P, A, w_c):
    D = forward_diff_matrix(*P.shape[1:])
    e = 0.0
    for c in range(P.shape[0]):
        g = D @ (Ov[c] - P[c]).ravel()
        e += 0.5 * (g ** 2).sum() + 0.5 * (w_c.ravel() * (Ov[c] - A[c]).ravel() ** 2).sum()
    return e


def test_energy_gradient_is_finite_difference_of_energy():
    P, A, Ov = (RNG.random((3, 5, 6)) for _ in range(3))
    w_c = RNG.random((5, 6)) * 2
    g = O.energy_gradient(Ov, P, A, w_c)
    h = 1e-6
    for (c, y, x) in [(0, 0, 0), (1, 2, 3), (2, 4, 5), (0, 3, 0)]:
        Op, Om = Ov.copy(), Ov.copy()
        Op[c, y, x] += h
        Om[c, y, x] -= h
        num = (energy(Op, P, A, w_c) - energy(Om, P, A, w_c)) / (2 * h)
        assert abs(num - g[c, y, x]) < 1e-7


def test_momentum_iteration_converges_to_direct_solve():
    """Fixed point of Eq. 8 = solution of (-Lap + W_c) O = -Lap P + W_c A."""
    H, W = 10, 13
    P, A = RNG.random((3, H, W)), RNG.random((3, H, W))
    w_c = 0.2 + RNG.random((H, W))
    prm = dict(O.PAPER_DEFAULTS, iters=4000)
    Osol = O.poisson_solve(P, A, w_c, prm)
    D = forward_diff_matrix(H, W)
    M = (D.T @ D + sp.diags(w_c.ravel())).tocsc()
    for c in range(3):
        rhs = D.T @ (D @ P[c].ravel()) + w_c.ravel() * A[c].ravel()
        ref = spla.spsolve(M, rhs).reshape(H, W)
        assert np.allclose(Osol[c], ref, atol=1e-9)


def test_one_iteration_closed_form():
    P, A, Oc = (RNG.random((3, 6, 7)) for _ in range(3))
    w_c = RNG.random((6, 7))
    prm = dict(O.PAPER_DEFAULTS, iters=1)
    got = O.poisson_solve(P, A, w_c, prm, O0=Oc)
    # first step: no momentum (O^{-1} = O^0)
    exp = Oc - 0.15 * (-laplace_brute(Oc - P) + w_c[None] * (Oc - A))
    assert np.allclose(got, exp, atol=1e-14)
    prm2 = dict(O.PAPER_DEFAULTS, iters=2)
    got2 = O.poisson_solve(P, A, w_c, prm2, O0=Oc)
    exp2 = exp - 0.15 * (-laplace_brute(exp - P) + w_c[None] * (exp - A)) + 0.2 * (exp - Oc)
    assert np.allclose(got2, exp2, atol=1e-14)


def test_lambda_zero_preserves_mean():
    P, A = RNG.random((3, 8, 9)), RNG.random((3, 8, 9))
    Osol = O.poisson_solve(P, A, np.zeros((8, 9)), dict(O.PAPER_DEFAULTS, lam=0.0))
    assert np.allclose(Osol.mean(axis=(1, 2)), A.mean(axis=(1, 2)), atol=1e-12)


def test_consistent_inputs_are_a_fixed_point():
    """P = A: the gradient vanishes and O stays A exactly."""
    P = RNG.random((3, 8, 9))
    Osol = O.poisson_solve(P, P.copy(), RNG.random((8, 9)), O.PAPER_DEFAULTS)
    assert np.array_equal(Osol, P)


def _frames(h=9, w=11):
    return [RNG.random((3, h, w)) for _ in range(7)]


def test_weights_identical_frames_zero_flow():
    """I_{t-1} = I_t = I_{t+1}, zero flows: exp(0) = 1 is clamped to k1, k2;
    A^I = I so w_c = lambda; A = k1 G + (1 - k1) L with the closed-form L."""
    I, Pp, P, Pn, Op, *_ = _frames()
    z = np.zeros((2,) + I.shape[1:])
    prm = O.PAPER_DEFAULTS
    A, w_c, w_p, w_n = O.paper_reference(I, I, I, Pp, P, Pn, Op, z, z, prm)
    k1, k2 = prm["k1"], prm["k2"]
    assert np.all(w_p == k1) and np.all(w_n == k2)
    assert np.allclose(w_c, prm["lam"])
    L = (1 - k1 - k2) * P + k1 * Pp + k2 * Pn
    assert np.allclose(A, k1 * Op + (1 - k1) * L, atol=1e-14)


def test_weights_zero_clamps_return_stylized():
    """k1 = k2 = 0: L = A = P and O = P exactly (per-frame result kept)."""
    I0, I1, I2, Pp, P, Pn, Op = _frames()
    f = RNG.standard_normal((2,) + P.shape[1:])
    prm = dict(O.PAPER_DEFAULTS, k1=0.0, k2=0.0)
    Ot, A, w_c = O.paper_consistency(I0, I1, I2, Pp, P, Pn, Op, f, -f, prm)
    assert np.array_equal(A, P) and np.array_equal(Ot, P)


def test_photometric_weight_and_warp_shift():
    """Integer shift: Gamma(I_{t-1}) reproduces I_t away from the border, so
    w_p = k1 there; elsewhere the photometric weight decays as exp(-a d^2)."""
    H, W = 10, 12
    I_prev = RNG.random((3, H, W))
    I_cur = np.roll(I_prev, shift=(0, 2), axis=(1, 2))     # content moved 2 px right
    f_tp = np.zeros((2, H, W)); f_tp[0] = -2.0            # t -> t-1
    z = np.zeros((2, H, W))
    P = RNG.random((3, H, W))
    A, w_c, w_p, w_n = O.paper_reference(I_prev, I_cur, I_cur, P, P, P, P, f_tp, z,
                                         O.PAPER_DEFAULTS)
    assert np.all(w_p[:, 2:] == O.PAPER_DEFAULTS["k1"])
    d = np.array([[0.1, 0.0, 0.0]]).T
    assert np.isclose(O.photometric_weight(np.zeros((3, 1)), d, 100.0)[0], np.exp(-1.0))
