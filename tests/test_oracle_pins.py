"""Pins for the CPU FP64 oracle.

Each test fixes part of the oracle against something other than the oracle
itself: the operator definition evaluated by quadrature, closed forms at tiny
N, brute force, invariants the paper states (trace, eigenvalue range,
orthonormality, the W <-> 1/2 - W symmetry, the error structure of Lemmas 4-6,
the bounds of Corollaries 1-4), and scipy's independent DPSS routine.  The
"planted mistake" tests at the end show that a plausible slip in the oracle
(a dropped term, a wrong sign, an off-by-one index) fails at least one pin.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial.legendre import leggauss
from scipy.signal.windows import dpss as scipy_dpss

from oracle import slepian_oracle as o


# ---------------------------------------------------------------------------
# B and B x
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,W", [(7, 0.1), (16, 0.25), (33, 0.03)])
def test_prolate_matrix_is_bandlimit_of_timelimit(N, W):
    """B is the N x N section of B_W T_N (Definition 1 / Section 1.2):
    B[m, n] = integral over |f| <= W of exp(j 2 pi f (m - n)) df, evaluated
    here by Gauss-Legendre quadrature, independent of the sinc formula."""
    t, w = leggauss(200)
    f = W * t
    wt = W * w
    k = np.arange(-(N - 1), N)
    vals = (wt[None, :] * np.cos(2 * np.pi * f[None, :] * k[:, None])).sum(axis=1)
    idx = np.arange(N)
    Bq = vals[(idx[:, None] - idx[None, :]) + N - 1]
    np.testing.assert_allclose(o.prolate_matrix(N, W), Bq, atol=1e-13)


def test_closed_form_N2():
    """N = 2: B = [[2W, s], [s, 2W]] with s = sin(2 pi W)/pi; eigenvalues
    2W + s, 2W - s; eigenvectors (1, 1)/sqrt2 and (1, -1)/sqrt2."""
    for W in (0.05, 0.2, 0.37):
        s = math.sin(2 * math.pi * W) / math.pi
        lam, S = o.dense_eig(2, W)
        np.testing.assert_allclose(lam, [2 * W + s, 2 * W - s], atol=1e-15)
        np.testing.assert_allclose(np.abs(S), np.full((2, 2), 1 / math.sqrt(2)), atol=1e-15)
        lt, St = o.slepian_vectors(2, W, 0, 1)
        np.testing.assert_allclose(lt, lam, atol=1e-15)
        np.testing.assert_allclose(St[:, 1], [1 / math.sqrt(2), -1 / math.sqrt(2)], atol=1e-15)


def test_closed_form_N3_antisymmetric():
    """N = 3: (1, 0, -1)/sqrt2 is an eigenvector with eigenvalue 2W - c2,
    c2 = sin(4 pi W)/(2 pi); it is the l = 1 Slepian vector (odd parity)."""
    W = 0.15
    c2 = math.sin(4 * math.pi * W) / (2 * math.pi)
    lam, S = o.slepian_vectors(3, W, 0, 2)
    np.testing.assert_allclose(lam[1], 2 * W - c2, atol=1e-15)
    np.testing.assert_allclose(S[:, 1], [1 / math.sqrt(2), 0, -1 / math.sqrt(2)], atol=1e-15)


@pytest.mark.parametrize("N,W", [(5, 0.2), (64, 0.1), (100, 0.23), (257, 1 / 16)])
def test_fft_product_matches_dense(N, W):
    """B x by FFT (Section 4.1) equals the dense product; any length L >= 2N-1
    gives the same result (the circulant embedding is exact)."""
    rng = np.random.default_rng(N)
    x = rng.standard_normal((N, 3))
    ref = o.apply_prolate_dense(N, W, x)
    for L in (o.fft_length(N), 2 * N - 1, 2 * N + 7):
        np.testing.assert_allclose(o.apply_prolate(N, W, x, L), ref, atol=1e-13)


def test_kernel_spectrum_real_even():
    N, W = 300, 0.07
    L = o.fft_length(N)
    ch = o.kernel_spectrum(N, W)
    assert L == 1024 and ch.shape == (L,)
    np.testing.assert_allclose(ch[1:], ch[1:][::-1], atol=1e-13)
    # sum of the spectrum / L is the embedded sequence at 0, i.e. B's diagonal
    assert abs(ch.sum() / L - 2 * W) < 1e-13


def test_sizes():
    assert [o.fft_length(n) for n in (1, 2, 3, 1024, 1025, 65536)] == [2, 4, 8, 2048, 4096, 131072]
    assert o.choose_K(1024, 1 / 16) == 128
    assert o.choose_K(65536, 1 / 8) == 16384
    assert o.choose_K(262144, 0.05) == 26214
    assert o.choose_K(10, 0.125) == 3     # 2.5 rounds away from zero
    assert o.choose_K(1048576, 0.02) == 41943


# ---------------------------------------------------------------------------
# Eigenpairs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,W", [(64, 0.1), (128, 1 / 16), (100, 0.23)])
def test_eigen_invariants(N, W):
    """Eigenvalues in (0, 1), strictly decreasing, summing to trace(B) = 2NW;
    the Slepian basis is orthonormal (Definition 2 with eq. dpssnorm,
    eq. dpssorth)."""
    lam, S = o.dense_eig(N, W)
    B = o.prolate_matrix(N, W)
    assert abs(np.trace(B) - 2 * N * W) < 1e-12
    assert abs(lam.sum() - 2 * N * W) < 1e-11
    assert np.all(lam > -1e-14) and np.all(lam < 1 + 1e-14)
    # distinct where resolvable in float64 (the eigenvalues near 1 and 0 cluster
    # tighter than float64 spacing, so only the transition part is checked)
    mid = (lam > 1e-10) & (lam < 1 - 1e-10)
    assert np.all(np.diff(lam[mid]) < 0)
    np.testing.assert_allclose(S.T @ S, np.eye(N), atol=1e-12)
    assert np.linalg.norm(B, 2) <= 1 + 1e-14


@pytest.mark.parametrize("N,W", [(64, 0.1), (128, 1 / 16), (100, 0.23), (97, 0.31)])
def test_tridiagonal_commutes_and_shares_eigenvectors(N, W):
    """The tridiagonal matrix commutes with B, and its eigenvectors (taken in
    descending order) are eigenvectors of B with the eigenvalues of dense B in
    the same order."""
    d, e = o.slepian_tridiagonal(N, W)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    B = o.prolate_matrix(N, W)
    comm = B @ T - T @ B
    assert np.linalg.norm(comm) <= 1e-12 * np.linalg.norm(T)
    lam_t, S_t = o.slepian_vectors(N, W, 0, N - 1)
    lam_d, _ = o.dense_eig(N, W)
    np.testing.assert_allclose(lam_t, lam_d, atol=1e-14)
    resid = B @ S_t - S_t * lam_t[None, :]
    assert np.max(np.linalg.norm(resid, axis=0)) < 1e-12


@pytest.mark.parametrize("N,W,eps", [(256, 1 / 8, 1e-6), (1024, 1 / 16, 1e-6)])
def test_transition_vectors_match_dense(N, W, eps):
    """In the transition region the eigenvalues are well separated, so the
    tridiagonal route and dense eig give the same vectors up to sign."""
    tp = o.transition_plan(N, W, eps, 1 - eps)
    lam_d, S_d = o.dense_eig(N, W)
    sl = slice(tp["lo"] + tp["j0"], tp["lo"] + tp["j1"])
    S_t = tp["S"][:, tp["j0"]:tp["j1"]]
    ov = np.abs(np.einsum("nj,nj->j", S_t, S_d[:, sl]))
    assert np.all(ov > 1 - 1e-10)
    np.testing.assert_allclose(tp["lam"][tp["j0"]:tp["j1"]], lam_d[sl], atol=1e-14)


@pytest.mark.parametrize("N,W", [(64, 0.1), (128, 0.2), (100, 0.23)])
def test_half_band_symmetry(N, W):
    """lambda_{N,1/2-W}^(l) = 1 - lambda_{N,W}^(N-1-l) (Section 1.2, quoting
    Slepian 1978 eq. 13)."""
    a, _ = o.dense_eig(N, W)
    b, _ = o.dense_eig(N, 0.5 - W)
    np.testing.assert_allclose(b, 1 - a[::-1], atol=1e-14)


def test_parity_of_slepian_vectors():
    """Even-l vectors are symmetric about (N-1)/2, odd-l antisymmetric."""
    N, W = 200, 0.1
    lam, S = o.slepian_vectors(N, W, 0, N - 1)
    for l in range(N):
        sgn = 1 if l % 2 == 0 else -1
        assert np.max(np.abs(S[::-1, l] - sgn * S[:, l])) < 1e-11


@pytest.mark.parametrize("N,W", [(128, 1 / 16), (255, 0.1)])
def test_scipy_dpss_agrees(N, W):
    """scipy's independent DPSS routine (concentration ratios and tapers)."""
    K = o.choose_K(N, W) + 10
    tapers, ratios = scipy_dpss(N, N * W, Kmax=K, return_ratios=True)
    lam, S = o.slepian_vectors(N, W, 0, K - 1)
    np.testing.assert_allclose(lam, ratios, atol=1e-12)
    ov = np.abs(np.einsum("jn,nj->j", tapers / np.linalg.norm(tapers, axis=1, keepdims=True), S))
    # vectors inside the lambda ~ 1 cluster are only defined up to the
    # cluster; in the transition region and just below it they must agree
    mid = lam < 1 - 1e-8
    assert np.all(ov[mid] > 1 - 1e-9)


def test_sign_convention():
    S = np.array([[0.0, -1e-9, 0.5], [-2.0, 3.0, -0.1], [1.0, 1.0, 0.2]]).T
    F = o.sign_fix(S)
    for j in range(3):
        col = F[:, j]
        first = np.nonzero(np.abs(col) >= 1e-3 * np.max(np.abs(col)))[0][0]
        assert col[first] > 0
        np.testing.assert_allclose(np.abs(col), np.abs(S[:, j]))


# ---------------------------------------------------------------------------
# Projection, pinv, Tikhonov: exact operators and their fast forms
# ---------------------------------------------------------------------------

def _dense_operator(fn, N):
    return fn(np.eye(N))


@pytest.mark.parametrize("N,W", [(128, 1 / 16), (150, 0.2)])
def test_exact_projection_invariants(N, W):
    """P = S_K S_K^T is symmetric, idempotent, of trace and rank K."""
    K = o.choose_K(N, W)
    P = _dense_operator(lambda X: o.project_exact(N, W, X), N)
    np.testing.assert_allclose(P, P.T, atol=1e-13)
    np.testing.assert_allclose(P @ P, P, atol=1e-12)
    assert abs(np.trace(P) - K) < 1e-10
    assert np.linalg.matrix_rank(P, tol=1e-8) == K


@pytest.mark.parametrize("N,W,eps", [(256, 1 / 8, 1e-6), (200, 0.05, 1e-3), (300, 0.3, 1e-9)])
def test_fast_projection_error_closed_form(N, W, eps):
    """Lemma 4: S_K S_K^T - (B + U1 U2^T) = V1 (I - Lambda1) V1^T - V4 Lambda4 V4^T,
    whose 2-norm is max(max over I1 of 1 - lambda, max over I4 of lambda) <= eps."""
    K = o.choose_K(N, W)
    lam, _ = o.dense_eig(N, W)
    assert lam[K - 1] > eps and lam[K] < 1 - eps      # K satisfies Corollary 2
    tp = o.transition_plan(N, W, eps, 1 - eps)
    Pe = _dense_operator(lambda X: o.project_exact(N, W, X), N)
    Pf = _dense_operator(lambda X: o.project_fast(N, W, eps, X, tp=tp), N)
    err = np.linalg.norm(Pe - Pf, 2)
    i1 = lam >= 1 - eps
    i4 = lam <= eps
    expect = max(np.max(1 - lam[i1], initial=0), np.max(lam[i4], initial=0))
    assert err <= eps * (1 + 1e-9)
    assert abs(err - expect) < 1e-11


@pytest.mark.parametrize("N,W,eps", [(256, 1 / 8, 1e-6), (200, 0.1, 1e-4)])
def test_fast_pinv_error(N, W, eps):
    """Lemma 5: the error is V1 (Lambda1^-1 - Lambda1) V1^T - V4 Lambda4 V4^T,
    of norm <= 3 eps."""
    lam, _ = o.dense_eig(N, W)
    tp = o.transition_plan(N, W, eps, 1 - eps)
    Ae = _dense_operator(lambda X: o.pinv_exact(N, W, X), N)
    Af = _dense_operator(lambda X: o.pinv_fast(N, W, eps, X, tp=tp), N)
    err = np.linalg.norm(Ae - Af, 2)
    i1 = lam >= 1 - eps
    i4 = lam <= eps
    expect = max(np.max(1 / lam[i1] - lam[i1], initial=0), np.max(lam[i4], initial=0))
    assert err <= 3 * eps
    assert abs(err - expect) < 1e-10
    # B_K^+ B restricted to span(S_K) is the identity: B_K^+ B S_K = S_K
    K = o.choose_K(N, W)
    _, S = o.dense_eig(N, W)
    np.testing.assert_allclose(Ae @ (o.prolate_matrix(N, W) @ S[:, :K]), S[:, :K], atol=1e-9)


@pytest.mark.parametrize("N,W,eps,alpha", [(256, 1 / 8, 1e-6, 1e-3), (200, 0.1, 1e-4, 0.05)])
def test_fast_tikhonov_error(N, W, eps, alpha):
    """Lemma 6: (B^2 + alpha I)^-1 B - (B/(1+alpha) + U5 U5^T) has norm <= eps,
    and the exact operator solves min ||y - B x||^2 + alpha ||x||^2 (checked by
    least squares on the stacked system [B; sqrt(alpha) I] x = [y; 0])."""
    B = o.prolate_matrix(N, W)
    rng = np.random.default_rng(3)
    y = rng.standard_normal((N, 2))
    xe = o.tikhonov_exact(N, W, alpha, y)
    A = np.vstack([B, math.sqrt(alpha) * np.eye(N)])
    xl = np.linalg.lstsq(A, np.vstack([y, np.zeros((N, 2))]), rcond=None)[0]
    np.testing.assert_allclose(xe, xl, atol=1e-9)
    tp = o.transition_plan(N, W, alpha * (1 + alpha) * eps, 1 - eps / 3)
    Te = _dense_operator(lambda X: o.tikhonov_exact(N, W, alpha, X), N)
    Tf = _dense_operator(lambda X: o.tikhonov_fast(N, W, eps, alpha, X, tp=tp), N)
    assert np.linalg.norm(Te - Tf, 2) <= eps


def test_tikhonov_g_outside_set_bounded():
    """Lemma 6's bound: outside the selected set, 0 <= lambda(1-lambda^2) /
    ((1+alpha)(lambda^2+alpha)) <= eps."""
    alpha, eps = 1e-3, 1e-6
    lam = np.concatenate([np.linspace(0, alpha * (1 + alpha) * eps, 50),
                          np.linspace(1 - eps / 3, 1, 50)])
    v = lam * (1 - lam ** 2) / ((1 + alpha) * (lam ** 2 + alpha))
    assert np.all(v >= 0) and np.all(v <= eps)
    g, sel = o.tikhonov_g(lam, alpha, eps)
    assert not sel.any() and np.all(g == 0)


def test_tikhonov_cg_matches_dense():
    N, W, alpha = 300, 0.1, 1e-3
    y = np.random.default_rng(5).standard_normal((N, 2))
    np.testing.assert_allclose(o.tikhonov_cg(N, W, alpha, y), o.tikhonov_exact(N, W, alpha, y),
                               atol=1e-9)


def test_coeffs_reconstruct_projection():
    N, W = 128, 1 / 16
    x = np.random.default_rng(1).standard_normal((N, 2))
    K = o.choose_K(N, W)
    _, S = o.slepian_vectors(N, W, 0, K - 1)
    c = o.coeffs_exact(N, W, x)
    assert c.shape == (K, 2)
    # the tridiagonal vectors span the same subspace as dense eig's first K
    np.testing.assert_allclose(S @ c, o.project_exact(N, W, x), atol=1e-11)
    np.testing.assert_allclose(S.T @ S, np.eye(K), atol=1e-12)
    # energy in the band: ||c|| = ||P x|| <= ||x||
    assert np.all(np.linalg.norm(c, axis=0) <= np.linalg.norm(x, axis=0))


# ---------------------------------------------------------------------------
# Transition-region size (Corollary 1, eq. asymptotic, the earlier bound)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,W,eps", [(1024, 1 / 16, 1e-6), (1024, 0.25, 1e-3),
                                     (4096, 0.25, 1e-9), (2048, 0.1, 1e-12)])
def test_transition_count_bounds(N, W, eps):
    tp = o.transition_plan(N, W, eps, 1 - eps)
    r = tp["j1"] - tp["j0"]
    assert r <= o.cor1_bound(N, eps)
    a = o.asymptotic_count(N, eps)
    assert 0.5 * a <= r <= 1.5 * a + 2
    # the set is exactly {eps < lambda < 1-eps} over the whole spectrum
    lam_all, _ = o.slepian_vectors(N, W, tp["lo"], tp["hi"])
    assert lam_all[0] >= 1 - eps or tp["lo"] == 0
    assert lam_all[-1] <= eps or tp["hi"] == N - 1


def test_transition_count_dense_brute_force():
    """Counting {eps < lambda < 1-eps} on the full dense spectrum gives the
    same set as the windowed tridiagonal solve."""
    N, W, eps = 512, 0.2, 1e-6
    lam, _ = o.dense_eig(N, W)
    idx = np.nonzero((lam > eps) & (lam < 1 - eps))[0]
    tp = o.transition_plan(N, W, eps, 1 - eps)
    assert idx[0] == tp["lo"] + tp["j0"] and idx[-1] == tp["lo"] + tp["j1"] - 1


# ---------------------------------------------------------------------------
# Planted mistakes: each plausible slip in the oracle must fail a pin above.
# The mistake is planted in a copy of the oracle's arithmetic, on the CPU.
# ---------------------------------------------------------------------------

def test_planted_wrong_sign_in_d_is_caught(monkeypatch):
    N, W, eps = 256, 1 / 8, 1e-6
    good = o.projection_d

    def bad(lam, ells, K, e):
        d, sel = good(lam, ells, K, e)
        _, i2, i3, _ = o.partition(lam, ells, K, e)
        d[i3] = +lam[i3]          # sign slip on I3
        return d, sel

    monkeypatch.setattr(o, "projection_d", bad)
    with pytest.raises(AssertionError):
        test_fast_projection_error_closed_form(N, W, eps)


def test_planted_diagonal_mistake_is_caught(monkeypatch):
    good = o._sinc_values

    def bad(k, W):
        v = good(k, W)
        return np.where(np.asarray(k) == 0, W, v)    # W instead of 2W

    monkeypatch.setattr(o, "_sinc_values", bad)
    with pytest.raises(AssertionError):
        test_prolate_matrix_is_bandlimit_of_timelimit(16, 0.25)


def test_planted_tridiagonal_index_shift_is_caught(monkeypatch):
    good = o.slepian_tridiagonal

    def bad(N, W):
        d, e = good(N, W)
        m = np.arange(0, N - 1, dtype=np.float64)     # n (N - n)/2 shifted by one
        return d, m * (N - m) / 2.0 + 0.5 * (m == 0)

    monkeypatch.setattr(o, "slepian_tridiagonal", bad)
    with pytest.raises(AssertionError):
        test_tridiagonal_commutes_and_shares_eigenvectors(64, 0.1)


def test_planted_missing_tikhonov_scale_is_caught(monkeypatch):
    good = o.tikhonov_fast

    def bad(N, W, eps, alpha, y, tp=None):
        return good(N, W, eps, alpha, y, tp) * (1 + alpha) ** 0 + o.apply_prolate(N, W, y) * alpha / (1 + alpha)

    monkeypatch.setattr(o, "tikhonov_fast", bad)
    with pytest.raises(AssertionError):
        test_fast_tikhonov_error(200, 0.1, 1e-4, 0.05)
