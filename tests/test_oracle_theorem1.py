"""Pins of the oracle's construction of Theorem 1's factor (Section 2, the
proof of Theorem 1, with Lemma 2 and its proof in the appendix) and of the
bound functions the paper states (Theorem 1, Corollary 1, eq. asymptotic,
the bound on K' in Section 1.3).

Each piece is checked against something other than its own formula: the
identities eq. (BA0) and eq. (A0A1) on dense matrices built from the
entrywise definitions, the CF-ADI error identity of the appendix, mpmath's
elliptic functions, the alternating series of the zeta coefficients, the
per-piece error bounds of the proof, the relations between the paper's
bounds (Lemma 3 in the proof of Corollary 1 gives count <= 2 rank; the bound
on K' adds Theorem 1's and Corollary 2's ranks), and transition counts of
the oracle's dense-pinned eigensolver.  The planted-constant tests at the end
show that a changed constant in any bound function fails one of these.
"""

import math

import mpmath
import numpy as np
import pytest

from oracle import factorization as fz
from oracle import slepian_oracle as so


def _dense_pieces(N, W):
    kf = fz.kf_count(N, W)
    Wp = kf / (2.0 * N)
    m = np.arange(N, dtype=np.float64)
    d = m[:, None] - m[None, :]
    off = d != 0
    A0 = np.zeros((N, N))
    A0[off] = 1.0 / (math.pi * d[off]) - 1.0 / (N * np.sin(math.pi * d[off] / N))
    B0 = np.full((N, N), 2.0 * (W - Wp))
    B0[off] = 2.0 * np.sin(math.pi * (W - Wp) * d[off]) / (math.pi * d[off])
    A1 = np.zeros((N, N))
    A1[off] = A0[off] - 1.0 / (math.pi * (d[off] + N)) - 1.0 / (math.pi * (d[off] - N))
    H = 1.0 / (m[:, None] + m[None, :] + 1.0)
    J = np.eye(N)[::-1]
    DA = np.diag(np.exp(2j * math.pi * Wp * m))
    DB = np.diag(np.exp(1j * math.pi * (W + Wp) * m))
    return kf, Wp, A0, B0, A1, H, J, DA, DB


# ---------------------------------------------------------------------------
# eq. (BA0), eq. (A0A1): the splitting of B - F F^*
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,W", [(64, 0.1), (127, 0.23), (200, 1 / 8)])
def test_ba0_and_a0a1_identities(N, W):
    kf, Wp, A0, B0, A1, H, J, DA, DB = _dense_pieces(N, W)
    F = fz.fr_matrix(N, kf)
    D = so.prolate_matrix(N, W) - F @ F.T
    rhs = (DA @ A0 @ DA.conj().T - DA.conj().T @ A0 @ DA) / 2j + (DB @ B0 @ DB.conj().T + DB.conj().T @ B0 @ DB) / 2
    np.testing.assert_allclose(rhs.real, D, atol=1e-13)
    assert np.abs(rhs.imag).max() < 1e-13
    np.testing.assert_allclose(A0, (H @ J - J @ H) / math.pi + A1, atol=1e-13)


def test_db_reading_without_pi_fails():
    """The printed D_B = diag(e^{j (W + W') n}) does not reproduce B - F F^*;
    with the factor pi it does (the reading the oracle takes)."""
    N, W = 64, 0.1
    kf, Wp, A0, B0, A1, H, J, DA, DB = _dense_pieces(N, W)
    F = fz.fr_matrix(N, kf)
    D = so.prolate_matrix(N, W) - F @ F.T
    m = np.arange(N)
    DBp = np.diag(np.exp(1j * (W + Wp) * m))
    rhs = (DA @ A0 @ DA.conj().T - DA.conj().T @ A0 @ DA) / 2j + (DBp @ B0 @ DBp.conj().T + DBp.conj().T @ B0 @ DBp) / 2
    assert np.abs(rhs.real - D).max() > 1e-3


# ---------------------------------------------------------------------------
# The Hilbert factor (Lemma 2, CF-ADI of the appendix)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kappa", [3.0, 15.0, 1e3, 131071.0, 2097151.0])
def test_elliptic_functions_match_mpmath(kappa):
    mpmath.mp.dps = 40
    try:
        kc = 1.0 / kappa
        m = 1 - mpmath.mpf(kc) ** 2
        K = fz.elliptic_k(kc)
        assert abs(K - float(mpmath.ellipk(m))) <= 1e-14 * K
        for f in (0.01, 0.25, 0.5, 0.75, 0.99):
            u = f * K
            ref = float(mpmath.ellipfun("dn", u, m=m))
            assert abs(fz.jacobi_dn(u, kc) - ref) <= 2e-14
    finally:
        mpmath.mp.dps = 15


@pytest.mark.parametrize("N,eps", [(64, 1e-6), (200, 1e-3), (256, 1e-12)])
def test_cfadi_error_identity_and_bound(N, eps):
    """H - Z Z^T = phi(A) H phi(A) for A = diag(n + 1/2) (the appendix), and
    with r_H columns the error is within delta_H (Schur: ||H|| <= pi, and
    max |phi|^2 <= delta_H / pi on the spectrum by Lemma 2)."""
    dH, _, _ = fz.theorem1_tolerances(eps)
    r = fz.hilbert_rank(N, dH)
    Z, p = fz.hilbert_factor(N, r)
    m = np.arange(N, dtype=np.float64)
    H = 1.0 / (m[:, None] + m[None, :] + 1.0)
    ph = fz.adi_rational(m + 0.5, p)
    np.testing.assert_allclose(H - Z @ Z.T, ph[:, None] * H * ph[None, :], atol=1e-14)
    assert np.max(ph ** 2) <= dH / math.pi
    # the lemma's bound holds on the whole interval [a, b], not only at the
    # eigenvalues of A
    xs = np.geomspace(0.5, N - 0.5, 20001)
    assert np.max(fz.adi_rational(xs, p) ** 2) <= dH / math.pi
    assert np.linalg.norm(H, 2) <= math.pi
    assert np.linalg.norm(H - Z @ Z.T, 2) <= dH
    # shifts inside [a, b]
    assert p.min() >= 0.5 and p.max() <= N - 0.5


def test_cfadi_with_one_shift_fewer_misses_the_bound():
    """The shift count of Lemma 2 is close to necessary: one fewer shift
    leaves max |phi|^2 above delta on [a, b]."""
    N, eps = 4096, 1e-6
    dH, _, _ = fz.theorem1_tolerances(eps)
    r = fz.hilbert_rank(N, dH)
    p = fz.adi_shifts(0.5, N - 0.5, r - 1)
    xs = np.geomspace(0.5, N - 0.5, 20001)
    assert np.max(fz.adi_rational(xs, p) ** 2) > dH / math.pi * 0.3


# ---------------------------------------------------------------------------
# The polynomial factors of A1 (zeta series) and B0 (sine series)
# ---------------------------------------------------------------------------

def test_zeta_coefficients_against_alternating_series():
    """c_k = 1 - (1 - 2^{-(2k-1)}) zeta(2k) = sum_{n>=2} (-1)^n n^{-2k}
    (the eta-function identity of the proof), and 0 <= c_k <= 2^{-2k}."""
    c = fz.zeta_coefficients(20)
    mpmath.mp.dps = 30
    try:
        for k in range(1, 21):
            ref = float(mpmath.nsum(lambda n: (-1) ** n / mpmath.mpf(n) ** (2 * k), [2, mpmath.inf]))
            assert abs(c[k - 1] - ref) <= 4e-16
            assert 0.0 <= c[k - 1] <= 2.0 ** (-2 * k)
    finally:
        mpmath.mp.dps = 15
    # k = 1 in closed form: 1 - pi^2/12
    assert abs(c[0] - (1 - math.pi ** 2 / 12)) < 1e-15


@pytest.mark.parametrize("N,W,eps", [(64, 0.1, 1e-6), (300, 0.21, 1e-9), (256, 1 / 8, 1e-3)])
def test_polynomial_factors_meet_their_bounds(N, W, eps):
    kf, Wp, A0, B0, A1, H, J, DA, DB = _dense_pieces(N, W)
    _, dA, dB = fz.theorem1_tolerances(eps)
    rA, rB = fz.a1_terms(dA), fz.b0_terms(dB)
    VA, CA = fz.a1_factor(N, rA)
    VB, CB = fz.b0_factor(N, W, Wp, rB)
    # the factored form equals the truncated series entry by entry
    m = np.arange(N, dtype=np.float64)
    x = (m[:, None] - m[None, :]) / N
    c = fz.zeta_coefficients(rA)
    A1t = sum(2.0 / (N * math.pi) * c[k - 1] * x ** (2 * k - 1) for k in range(1, rA + 1))
    th = math.pi * (W - Wp) * N
    B0t = sum(2.0 / (N * math.pi) * (-1) ** k * th ** (2 * k + 1) / math.factorial(2 * k + 1) * x ** (2 * k)
              for k in range(rB))
    np.testing.assert_allclose(VA @ CA @ VA.T, A1t, atol=1e-15)
    np.testing.assert_allclose(VB @ CB @ VB.T, B0t, atol=1e-15)
    assert VA.shape[1] == 2 * rA and VB.shape[1] == 2 * rB - 1
    # truncation errors within the proof's bounds, which are within delta
    eA = np.linalg.norm(A1 - A1t, 2)
    eB = np.linalg.norm(B0 - B0t, 2)
    assert eA <= 2.0 / (3 * math.pi) * 0.5 ** (2 * rA) <= dA
    assert eB <= 1.5 * (math.pi / 6) ** (2 * rB) <= dB
    # entries of the scaled-monomial factors stay bounded
    assert np.abs(VA).max() <= 1.0 and np.abs(CA).max() * N <= 1.0 and np.abs(VB).max() <= 1.0


# ---------------------------------------------------------------------------
# The assembled factor (Putting it all together)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,W,eps", [(64, 0.1, 1e-6), (256, 1 / 8, 1e-6), (512, 0.05, 1e-9),
                                     (1024, 0.2, 1e-3), (1000, 0.31, 1e-12), (333, 0.45, 1e-6)])
def test_constructed_factor_error_and_rank(N, W, eps):
    kf = fz.kf_count(N, W)
    F = fz.fr_matrix(N, kf)
    D = so.prolate_matrix(N, W) - F @ F.T
    L1, L2 = fz.theorem1_factor_complex(N, W, eps)
    L = L1 @ L2.conj().T
    assert np.abs(L.imag).max() < 1e-15
    E1 = D - L.real
    assert np.linalg.norm(E1, 2) <= eps
    # the error splits into the three pieces' errors (triangle inequality)
    _, Wp, A0, B0, A1, H, J, DA, DB = _dense_pieces(N, W)
    dH, dA, dB = fz.theorem1_tolerances(eps)
    Z, _ = fz.hilbert_factor(N, fz.hilbert_rank(N, dH))
    VA, CA = fz.a1_factor(N, fz.a1_terms(dA))
    VB, CB = fz.b0_factor(N, W, Wp, fz.b0_terms(dB))
    eH = np.linalg.norm(H - Z @ Z.T, 2)
    eA = np.linalg.norm(A1 - VA @ CA @ VA.T, 2)
    eB = np.linalg.norm(B0 - VB @ CB @ VB.T, 2)
    assert np.linalg.norm(E1, 2) <= 2 / math.pi * eH + eA + eB + 1e-15
    assert 2 / math.pi * dH + dA + dB == pytest.approx(eps, rel=1e-12)
    # rank: the column count of "Putting it all together", within Theorem 1's bound
    r1 = fz.theorem1_rank(N, eps)
    assert L1.shape == L2.shape == (N, r1)
    assert r1 <= fz.theorem1_rank_bound(N, eps)
    # the real form has the same product
    L1r, L2r = fz.theorem1_factor(N, W, eps)
    assert L1r.shape == L2r.shape == (N, r1)
    np.testing.assert_allclose(L1r @ L2r.T, L.real, atol=1e-14)


@pytest.mark.parametrize("method", ["theorem1", "eig"])
@pytest.mark.parametrize("N,W,eps", [(256, 1 / 8, 1e-6), (1024, 0.2, 1e-3)])
def test_t1t2_within_two_eps_both_factors(method, N, W, eps):
    fac = fz.fast_factorization(N, W, eps, method=method)
    T = fz.recover(fac, fz.compress(fac, np.eye(N)))
    lam, S = np.linalg.eigh(so.prolate_matrix(N, W))
    K = so.choose_K(N, W)
    P = S[:, -K:] @ S[:, -K:].T
    assert np.linalg.norm(P - T, 2) <= 2 * eps
    kp = fac["kf"] + fac["r1"] + fac["U"].shape[1]
    assert kp <= fz.kprime_bound(N, W, eps)


# ---------------------------------------------------------------------------
# The paper's bound functions, pinned by the relations between them, by the
# construction and by dense-pinned counts
# ---------------------------------------------------------------------------

GRID_N = [16, 256, 4096, 65536, 1 << 20]
GRID_EPS = [0.4, 1e-3, 1e-6, 1e-9, 1e-12]


def check_cor1_vs_theorem1(cor1, thm1):
    """Lemma 3 (proof of Corollary 1): #transition <= 2 rank(L), applied to
    Theorem 1's factor, gives Corollary 1's bound as twice Theorem 1's."""
    return all(abs(cor1(N, e) - 2 * thm1(N, e)) <= 1e-9 * cor1(N, e) for N in GRID_N for e in GRID_EPS)


def check_kprime_vs_theorem1(kprime, thm1):
    """K' = 2NW' + r1 + r2 with r1 bounded by Theorem 1 and r2 by Corollary 2
    (twice Theorem 1's bound): the K' bound less ceil(2NW) is three times
    Theorem 1's."""
    for N in GRID_N:
        for W in (0.01, 0.125, 0.3):
            for e in GRID_EPS:
                if abs(kprime(N, W, e) - math.ceil(2 * N * W) - 3 * thm1(N, e)) > 1e-9 * kprime(N, W, e):
                    return False
    return True


def check_theorem1_vs_construction(thm1):
    """The bound holds for the construction's column count and exceeds it by
    no more than the ceilings and the proof's final rounding of constants
    allow (four ceilings of at most 1 each, weights 4; 0.71 + 0.03 log(15/eps)
    from replacing 2/log 2 + 2/log(6/pi) by 6 and 8N - 4 by 8N)."""
    for N in GRID_N:
        for e in GRID_EPS:
            r1 = fz.theorem1_rank(N, e)
            b = thm1(N, e)
            if not (r1 <= b <= r1 + 12 + 0.72 + 0.03 * math.log(15 / e)):
                return False
    return True


def test_cor1_bound_is_twice_theorem1():
    assert check_cor1_vs_theorem1(so.cor1_bound, fz.theorem1_rank_bound)


def test_kprime_bound_is_theorem1_plus_corollary2():
    assert check_kprime_vs_theorem1(fz.kprime_bound, fz.theorem1_rank_bound)


def test_theorem1_bound_is_tight_for_the_construction():
    assert check_theorem1_vs_construction(fz.theorem1_rank_bound)


_COUNTS = {}


def _count(N, eps):
    key = (N, eps)
    if key not in _COUNTS:
        tp = so.transition_plan(N, 0.25, eps, 1 - eps)
        _COUNTS[key] = tp["j1"] - tp["j0"]
    return _COUNTS[key]


def check_asymptotic(asym):
    """Figure 1's setting (W = 1/4): the count's growth from N = 2^8 to 2^14
    matches the asymptotic one within 2.5, and for N >= 1024 the count lies
    within 0.1 a + 3 of the asymptotic value a."""
    for e in (1e-3, 1e-6, 1e-9, 1e-12):
        d_count = _count(1 << 14, e) - _count(1 << 8, e)
        d_asym = asym(1 << 14, e) - asym(1 << 8, e)
        if abs(d_count - d_asym) > 2.5:
            return False
        for lg in (10, 12, 14):
            a = asym(1 << lg, e)
            if abs(_count(1 << lg, e) - a) > 0.1 * a + 3:
                return False
    return True


def test_asymptotic_count_matches_counts():
    assert check_asymptotic(so.asymptotic_count)


def test_counts_within_corollary1():
    for e in (1e-3, 1e-6, 1e-9, 1e-12):
        for lg in (8, 10, 12, 14):
            assert _count(1 << lg, e) <= so.cor1_bound(1 << lg, e)


# planted constants: each changed constant must fail a check above

def test_planted_constants_in_cor1_bound_are_caught():
    for bad in (lambda N, e: (8 / math.pi ** 2 * math.log(8 * N) + 13) * math.log(15 / e),
                lambda N, e: (9 / math.pi ** 2 * math.log(8 * N) + 12) * math.log(15 / e),
                lambda N, e: (8 / math.pi ** 2 * math.log(4 * N) + 12) * math.log(15 / e),
                lambda N, e: (8 / math.pi ** 2 * math.log(8 * N) + 12) * math.log(16 / e)):
        assert not check_cor1_vs_theorem1(bad, fz.theorem1_rank_bound)


def test_planted_constants_in_kprime_bound_are_caught():
    for bad in (lambda N, W, e: math.ceil(2 * N * W) + (12 / math.pi ** 2 * math.log(8 * N) + 19) * math.log(15 / e),
                lambda N, W, e: math.ceil(2 * N * W) + (13 / math.pi ** 2 * math.log(8 * N) + 18) * math.log(15 / e),
                lambda N, W, e: math.floor(2 * N * W) + (12 / math.pi ** 2 * math.log(8 * N) + 18) * math.log(15 / e),
                lambda N, W, e: math.ceil(2 * N * W) + (12 / math.pi ** 2 * math.log(8 * N) + 18) * math.log(14 / e)):
        assert not check_kprime_vs_theorem1(bad, fz.theorem1_rank_bound)


def test_planted_constants_in_theorem1_bound_are_caught():
    for bad in (lambda N, e: (4 / math.pi ** 2 * math.log(8 * N) + 7) * math.log(15 / e),
                lambda N, e: (4 / math.pi ** 2 * math.log(8 * N) + 5) * math.log(15 / e),
                lambda N, e: (5 / math.pi ** 2 * math.log(8 * N) + 6) * math.log(15 / e),
                lambda N, e: (3 / math.pi ** 2 * math.log(8 * N) + 6) * math.log(15 / e),
                lambda N, e: (4 / math.pi ** 2 * math.log(16 * N) + 6) * math.log(15 / e),
                lambda N, e: (4 / math.pi ** 2 * math.log(8 * N) + 6) * math.log(30 / e)):
        assert not check_theorem1_vs_construction(bad)


def test_planted_constants_in_asymptotic_count_are_caught():
    for bad in (lambda N, e: 4 / math.pi ** 2 * math.log(N) * math.log(1 / e - 1),
                lambda N, e: 1 / math.pi ** 2 * math.log(N) * math.log(1 / e - 1),
                lambda N, e: 2 / math.pi ** 2 * math.log2(N) * math.log(1 / e - 1),
                lambda N, e: 2 / math.pi * math.log(N) * math.log(1 / e - 1),
                lambda N, e: 2 / math.pi ** 2 * math.log(N) * math.log10(1 / e - 1)):
        assert not check_asymptotic(bad)
