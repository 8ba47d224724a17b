"""Pins of the fast-factorization oracle (Section 1.3 "A fast factorization",
Theorem 1): each function is checked against something other than itself,
namely closed forms, numpy's FFT, dense eigendecomposition, and the error
and rank bounds the paper proves."""

import math

import numpy as np
import pytest

from oracle import factorization as fz
from oracle import slepian_oracle as so


def test_kf_is_nearest_odd_integer():
    # 2NW = 128 (even): tie between 127 and 129, the upper one is taken
    assert fz.kf_count(1024, 1 / 16) == 129
    # 2NW = 409.6: 409 is nearest
    assert fz.kf_count(1024, 0.2) == 409
    # 2NW = 410.4: 411 is nearest
    assert fz.kf_count(1026, 0.2) == 411
    for N, W in [(100, 0.13), (4096, 0.031), (777, 0.45)]:
        k = fz.kf_count(N, W)
        assert k % 2 == 1 and abs(k - 2 * N * W) <= 1


@pytest.mark.parametrize("N,W", [(64, 0.1), (256, 1 / 8), (300, 0.21)])
def test_fr_is_orthonormal_and_spans_the_dirichlet_projection(N, W):
    """F_r^T F_r = I and F_r F_r^T equals F F^*, whose entries are the
    Dirichlet kernel sin(pi kf (m-n)/N) / (N sin(pi (m-n)/N)) (Section 1.2)."""
    kf = fz.kf_count(N, W)
    F = fz.fr_matrix(N, kf)
    np.testing.assert_allclose(F.T @ F, np.eye(kf), atol=1e-12)
    m = np.arange(N)
    dd = (m[:, None] - m[None, :]).astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        D = np.sin(math.pi * kf * dd / N) / (N * np.sin(math.pi * dd / N))
    D[dd == 0] = kf / N
    np.testing.assert_allclose(F @ F.T, D, atol=1e-12)
    # the complex partial DFT matrix of Theorem 1 gives the same projection
    k = np.arange(-(kf - 1) // 2, (kf - 1) // 2 + 1)
    Fc = np.exp(2j * math.pi * np.outer(m, k) / N) / math.sqrt(N)
    np.testing.assert_allclose((Fc @ Fc.conj().T).real, F @ F.T, atol=1e-12)
    assert np.abs((Fc @ Fc.conj().T).imag).max() < 1e-12


@pytest.mark.parametrize("N,W", [(64, 0.1), (257, 0.2), (1024, 1 / 16)])
def test_fr_fft_routes_match_the_explicit_matrix(N, W):
    kf = fz.kf_count(N, W)
    F = fz.fr_matrix(N, kf)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((N, 3))
    c = rng.standard_normal((kf, 3))
    np.testing.assert_allclose(fz.fr_adjoint(x, kf), F.T @ x, atol=1e-12 * np.abs(x).sum(0).max())
    np.testing.assert_allclose(fz.fr_apply(c, N), F @ c, atol=1e-12 * np.abs(c).sum(0).max())


def test_difference_column_is_b_minus_ffstar():
    N, W = 200, 0.17
    kf = fz.kf_count(N, W)
    F = fz.fr_matrix(N, kf)
    D = so.prolate_matrix(N, W) - F @ F.T
    np.testing.assert_allclose(fz.difference_column(N, W, kf), D[:, 0], atol=1e-14)


@pytest.mark.parametrize("N,W,eps", [(256, 1 / 8, 1e-6), (1024, 1 / 16, 1e-6), (1024, 0.2, 1e-3),
                                     (512, 0.05, 1e-9)])
def test_theorem1_factor_error_and_rank(N, W, eps):
    """||B - F F^* - L1 L2^T|| <= eps with r1 within Theorem 1's bound; one
    factor fewer breaks the bound (the truncation is tight)."""
    kf = fz.kf_count(N, W)
    V, mu = fz.difference_factor(N, W, eps, kf)
    F = fz.fr_matrix(N, kf)
    D = so.prolate_matrix(N, W) - F @ F.T
    E1 = D - (V * mu) @ V.T
    assert np.linalg.norm(E1, 2) <= eps
    assert len(mu) <= fz.theorem1_rank_bound(N, eps)
    E1m = D - (V[:, :-1] * mu[:-1]) @ V[:, :-1].T
    assert np.linalg.norm(E1m, 2) > eps
    np.testing.assert_allclose(V.T @ V, np.eye(len(mu)), atol=1e-10)


@pytest.mark.parametrize("N,W,eps", [(256, 1 / 8, 1e-6), (1024, 1 / 16, 1e-6), (1024, 0.2, 1e-3)])
def test_t1t2_is_within_two_eps_of_the_projection(N, W, eps):
    """||S_K S_K^T - T1 T2^T|| <= 2 eps (Section 1.3), with T1 T2^T formed by
    recovering the compression of every unit vector; the compressed length
    K' meets Section 1.3's bound."""
    fac = fz.fast_factorization(N, W, eps)
    T = fz.recover(fac, fz.compress(fac, np.eye(N)))
    lam, S = np.linalg.eigh(so.prolate_matrix(N, W))
    K = so.choose_K(N, W)
    P = S[:, -K:] @ S[:, -K:].T
    assert np.linalg.norm(P - T, 2) <= 2 * eps
    kp = fac["kf"] + fac["r1"] + fac["U"].shape[1]
    assert kp <= fz.kprime_bound(N, W, eps)
    # the factor is not the projection itself: without L1 L2^T the error is O(1)
    c = fz.compress(fac, np.eye(N))
    c[fac["kf"]:fac["kf"] + fac["r1"]] = 0
    assert np.linalg.norm(P - fz.recover(fac, c), 2) > 0.1


def test_lanczos_route_matches_dense_route():
    """At N just above the dense limit the Lanczos route's V diag(mu) V^T
    agrees with the dense eigendecomposition of the same Toeplitz matrix."""
    N, W, eps = fz.DENSE_MAX * 2, 1 / 8, 1e-6
    kf = fz.kf_count(N, W)
    V, mu = fz.difference_factor(N, W, eps, kf)
    t = fz.difference_column(N, W, kf)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((N, 2))
    # dense reference on the same matrix (eigh of an 8192 x 8192 Toeplitz)
    idx = np.arange(N)
    T = t[np.abs(idx[:, None] - idx[None, :])]
    mud, Vd = np.linalg.eigh(T)
    keep = np.abs(mud) > eps
    ref = (Vd[:, keep] * mud[keep]) @ (Vd[:, keep].T @ x)
    got = (V * mu) @ (V.T @ x)
    assert len(mu) == int(keep.sum())
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(x)
    # and it reproduces T x up to eps
    assert np.linalg.norm(T @ x - got) <= eps * np.linalg.norm(x)
