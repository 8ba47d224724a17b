"""Plain CPU FP64 oracle for the fast factorization S_K S_K^T ~= T1 T2^T of
Section 1.3 ("A fast factorization"), built on Theorem 1.

THIS MODULE IS TEST INFRASTRUCTURE, like the rest of this package: only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it, and it shares no code with the GPU library.

The factorization combines three pieces:
  * F, the partial DFT matrix of Theorem 1: the 2NW' lowest-frequency
    length-N DFT vectors, scaled by 1/sqrt(N), where 2NW' is the odd integer
    nearest to 2NW;
  * L1 L2^T, a rank-r1 approximation of B - F F^* within eps (Theorem 1),
    by default the explicit construction in the proof of Theorem 1
    (Section 2): eq. (BA0) and eq. (A0A1) split B - F F^* into modulated
    copies of the Hilbert matrix H, a remainder A1 and a matrix B0; H gets
    a CF-ADI factor (Lemma 2, proved in the appendix), A1 and B0 truncated
    power series ("Putting it all together" sets the three tolerances);
  * U1 U2^T = U_T diag(d) U_T^T over the transition set (Corollary 2,
    Lemma 4).
Then T1 = [F, L1, U1], T2 = [F, L2, U2], the compression is T2^T x (K' =
2NW' + r1 + r numbers) and the recovery T1 c; the two errors add, so
||S_K S_K^T - T1 T2^T|| <= 2 eps.

Readings of points the paper leaves open:
  * 2NW' is read as the odd integer nearest to 2NW (the printed definition
    names W itself, which is not an integer); when 2NW is an even integer
    the two candidates tie and the upper one, 2NW + 1, is taken.
  * For real signals F is replaced by the real matrix F_r whose columns are
    1/sqrt(N), then sqrt(2/N) cos(2 pi k n / N) and -sqrt(2/N) sin(2 pi k n / N)
    for k = 1 .. (2NW' - 1)/2, interleaved in that order.  F_r F_r^T = F F^*
    (both are the projection onto the same real span), so T1 T2^T is
    unchanged and the compressed vector has 2NW' real entries for the F part.
  * The construction's complex L1, L2 have columns in conjugate pairs, so
    for real signals they are replaced by real matrices with the same
    product (theorem1_factor); r1 is unchanged.
  * The second modulation of the construction, D_B, is read as
    diag(exp(j pi (W + W') n)): the exponent as printed lacks the factor
    pi, which the derivation of eq. (BA0) (a cosine of pi (W + W')(m - n))
    fixes.  The expanded four-term line for L carries a sign slip in its
    last term; the bracketed form and the printed L1, L2 agree, and are
    followed.
  * The polynomial factors of A1 and B0 use monomials of the centred,
    scaled index (m - (N-1)/2)/N instead of m itself (same span, same
    product V C V^T in exact arithmetic, bounded entries).
  * The alternative factor (method "eig") takes the eigenpairs of the
    symmetric matrix B - F F^* with |mu| > eps: its error is the largest
    discarded |mu| <= eps and its rank is the least possible for that
    error.  L1 = V diag(mu), L2 = V.

Parity status: every function is pinned by tests/test_oracle_factorization.py
against closed forms (the Dirichlet kernel of F F^*, the CF-ADI error
identity H - Z Z^T = phi(A) H phi(A), the zeta coefficients' alternating
series), independent library routines (numpy's FFT, dense eigh, mpmath's
elliptic functions), the error and rank bounds of Theorem 1 and of each
piece of its proof, and the relations between the paper's bounds (the
proof of Corollary 1, the bound on K'); none is "parity unpinned".
"""

from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft
import scipy.sparse.linalg as ssl

from . import slepian_oracle as so

DENSE_MAX = 4096


def kf_count(N: int, W: float) -> int:
    """2NW': the odd integer nearest to 2NW (Theorem 1's partial Fourier
    matrix); ties (2NW an even integer) go to 2NW + 1."""
    v = 2.0 * N * W
    lo = math.floor(v)
    if lo % 2 == 0:
        lo -= 1
    hi = lo + 2
    return lo if (v - lo) < (hi - v) else hi


def theorem1_rank_bound(N: int, eps: float) -> float:
    """Theorem 1's bound on r1: (4/pi^2 log(8N) + 6) log(15/eps)."""
    return (4.0 / math.pi ** 2 * math.log(8 * N) + 6.0) * math.log(15.0 / eps)


def kprime_bound(N: int, W: float, eps: float) -> float:
    """Section 1.3's bound on the compressed length:
    K' <= ceil(2NW) + (12/pi^2 log(8N) + 18) log(15/eps)."""
    return math.ceil(2 * N * W) + (12.0 / math.pi ** 2 * math.log(8 * N) + 18.0) * math.log(15.0 / eps)


def fr_matrix(N: int, kf: int) -> np.ndarray:
    """F_r explicitly (N x kf), columns [1, cos_1, -sin_1, cos_2, -sin_2, ...]
    scaled to unit norm (small N only; the tests use it as the definition)."""
    n = np.arange(N)
    cols = [np.full(N, 1.0 / math.sqrt(N))]
    for k in range(1, (kf - 1) // 2 + 1):
        cols.append(math.sqrt(2.0 / N) * np.cos(2 * math.pi * k * n / N))
        cols.append(-math.sqrt(2.0 / N) * np.sin(2 * math.pi * k * n / N))
    return np.stack(cols, axis=1)


def fr_adjoint(x: np.ndarray, kf: int) -> np.ndarray:
    """F_r^T x by a length-N FFT: with X(k) = sum_n x[n] e^{-j 2 pi k n / N},
    entry 0 is X(0)/sqrt(N) and entries 2k-1, 2k are sqrt(2/N) Re X(k) and
    sqrt(2/N) Im X(k)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    M = (kf - 1) // 2
    X = sfft.fft(x, axis=0)
    out = np.empty((kf,) + x.shape[1:])
    out[0] = X[0].real / math.sqrt(N)
    s = math.sqrt(2.0 / N)
    out[1::2] = s * X[1:M + 1].real
    out[2::2] = s * X[1:M + 1].imag
    return out


def fr_apply(c: np.ndarray, N: int) -> np.ndarray:
    """F_r c by a length-N inverse FFT of the conjugate-symmetric spectrum
    Y(0) = sqrt(N) c0, Y(k) = sqrt(N/2) (c_{2k-1} + j c_{2k}), Y(-k) = conj Y(k)."""
    c = np.asarray(c, dtype=np.float64)
    kf = c.shape[0]
    M = (kf - 1) // 2
    Y = np.zeros((N,) + c.shape[1:], dtype=np.complex128)
    Y[0] = math.sqrt(N) * c[0]
    Yk = math.sqrt(N / 2.0) * (c[1::2] + 1j * c[2::2])
    Y[1:M + 1] = Yk
    if M:
        Y[N - M:] = np.conj(Yk[::-1])
    return sfft.ifft(Y, axis=0).real


def difference_column(N: int, W: float, kf: int) -> np.ndarray:
    """First column of the symmetric Toeplitz matrix B - F F^*:
    sin(2 pi W m)/(pi m) - sin(pi kf m / N)/(N sin(pi m / N)), and 2W - kf/N at m = 0."""
    m = np.arange(1, N, dtype=np.float64)
    t = np.empty(N)
    t[0] = 2.0 * W - kf / N
    t[1:] = np.sin(2 * math.pi * W * m) / (math.pi * m) - np.sin(math.pi * kf * m / N) / (N * np.sin(math.pi * m / N))
    return t


def _toeplitz_apply(t: np.ndarray):
    """x -> T x for the symmetric Toeplitz T with first column t, by a
    circulant embedding of length L = smallest power of two >= 2N."""
    N = t.shape[0]
    L = so.fft_length(N)
    c = np.zeros(L)
    c[:N] = t
    c[L - N + 1:] = t[1:][::-1]
    ch = sfft.rfft(c)

    def mv(x):
        x = np.asarray(x, dtype=np.float64)
        X = sfft.rfft(x.reshape(N, -1), n=L, axis=0)
        return sfft.irfft(X * ch[:, None], n=L, axis=0)[:N].reshape(x.shape)

    return mv


def difference_factor(N: int, W: float, eps: float, kf: int | None = None):
    """V, mu with B - F F^* ~= V diag(mu) V^T: all eigenpairs with |mu| > eps,
    sorted by decreasing |mu| (Theorem 1; the reading in the module header).
    Dense eigh of the explicit Toeplitz matrix for N <= DENSE_MAX, otherwise
    Lanczos (scipy eigsh) on the FFT-applied matrix, widened until the
    smallest |mu| it returns is <= eps.  Each V column is signed so that its
    first entry of magnitude >= 1e-3 max |V| is positive."""
    if kf is None:
        kf = kf_count(N, W)
    t = difference_column(N, W, kf)
    if N <= DENSE_MAX:
        idx = np.arange(N)
        T = t[np.abs(idx[:, None] - idx[None, :])]
        mu, V = np.linalg.eigh(T)
    else:
        mv = _toeplitz_apply(t)
        A = ssl.LinearOperator((N, N), matvec=mv, matmat=mv, dtype=np.float64)
        k = 64
        while True:
            mu, V = ssl.eigsh(A, k=min(k, N - 2), which="LM", tol=1e-14)
            if np.abs(mu).min() <= eps or k >= N - 2:
                break
            k *= 2
    keep = np.abs(mu) > eps
    mu, V = mu[keep], V[:, keep]
    order = np.argsort(-np.abs(mu), kind="stable")
    return so.sign_fix(V[:, order]), mu[order]


def fast_factorization(N: int, W: float, eps: float, K: int | None = None, method: str = "theorem1") -> dict:
    """All pieces of T1 = [F_r, L1, U diag(d)], T2 = [F_r, L2, U].

    method "theorem1": L1, L2 from the construction in the proof of
    Theorem 1 (theorem1_factor).  method "eig": L1 = V diag(mu), L2 = V from
    the eigenpairs of B - F F^* with |mu| > eps (difference_factor), the
    least-rank factor within the same error."""
    kf = kf_count(N, W)
    extra = {}
    if method == "theorem1":
        L1, L2 = theorem1_factor(N, W, eps)
    elif method == "eig":
        V, mu = difference_factor(N, W, eps, kf)
        L1, L2 = V * mu, V
        extra = {"V": V, "mu": mu}
    else:
        raise ValueError(f"unknown factor method {method!r}")
    tp = so.transition_plan(N, W, eps, 1 - eps, K)
    ells = np.arange(tp["lo"], tp["hi"] + 1)
    d, sel = so.projection_d(tp["lam"], ells, tp["K"], eps)
    return {"N": N, "W": W, "eps": eps, "kf": kf, "L1": L1, "L2": L2, "r1": L1.shape[1], "method": method,
            "U": tp["S"][:, sel], "d": d[sel], "K": tp["K"], **extra}


def compress(fac: dict, x: np.ndarray) -> np.ndarray:
    """T2^T x = [F_r^T x; L2^T x; U^T x] (Section 1.3), K' rows."""
    x = np.asarray(x, dtype=np.float64)
    return np.concatenate([fr_adjoint(x, fac["kf"]), fac["L2"].T @ x, fac["U"].T @ x], axis=0)


def recover(fac: dict, c: np.ndarray) -> np.ndarray:
    """T1 c = F_r c_F + L1 c_L + U (d . c_U) (Section 1.3)."""
    c = np.asarray(c, dtype=np.float64)
    kf, r1 = fac["kf"], fac["r1"]
    cf, cl, cu = c[:kf], c[kf:kf + r1], c[kf + r1:]
    d = fac["d"] if c.ndim == 1 else fac["d"][:, None]
    return fr_apply(cf, fac["N"]) + fac["L1"] @ cl + fac["U"] @ (d * cu)


# ---------------------------------------------------------------------------
# Theorem 1's explicit construction of L1, L2 (Section 2, the proof of
# Theorem 1; the Hilbert factor by Lemma 2 and the appendix's CF-ADI proof)
# ---------------------------------------------------------------------------
#
# B - F F^* is written through eq. (BA0) as four modulated copies of two
# Toeplitz matrices A0 and B0, and A0 through eq. (A0A1) as the Hilbert
# matrix H flipped by the exchange matrix J plus a remainder A1.  H gets a
# factor Z Z^T from the CF-ADI iteration for the Lyapunov equation
# A X + X A = 1 1^T with A = diag(n + 1/2); A1 and B0 get polynomial
# factors from truncated series (coefficients from the zeta function for
# A1, the sine series for B0).  The tolerances are delta_H = 4 pi eps / 15
# and delta_A = delta_B = 7 eps / 30, so the three errors add to eps.
#
# Readings: the modulation D_B is diag(exp(j pi (W + W') n)) (the printed
# exponent lacks the factor pi; the derivation's cos(pi (W + W')(m - n))
# fixes it); the polynomial factors use the monomials of the centred,
# scaled index u = (m - (N-1)/2) / N rather than of m itself: the span and
# the product V C V^T are the same matrices in exact arithmetic, and the
# scaled monomials keep every entry of V and C below 1 in magnitude.


def theorem1_tolerances(eps: float):
    """delta_H, delta_A, delta_B of "Putting it all together"."""
    return 4.0 * math.pi * eps / 15.0, 7.0 * eps / 30.0, 7.0 * eps / 30.0


def hilbert_rank(N: int, delta_H: float) -> int:
    """r_H = ceil((1/pi^2) log(8N - 4) log(4 pi / delta_H)): Lemma 2 with
    kappa = 2N - 1 and delta = delta_H / pi."""
    return int(math.ceil(math.log(8 * N - 4) * math.log(4 * math.pi / delta_H) / math.pi ** 2))


def a1_terms(delta_A: float) -> int:
    """r_A = ceil(log(2 / (3 pi delta_A)) / (2 log 2)) series terms."""
    return int(math.ceil(math.log(2.0 / (3.0 * math.pi * delta_A)) / (2.0 * math.log(2.0))))


def b0_terms(delta_B: float) -> int:
    """r_B = ceil(log(3 / (2 delta_B)) / (2 log(6/pi))) series terms."""
    return int(math.ceil(math.log(3.0 / (2.0 * delta_B)) / (2.0 * math.log(6.0 / math.pi))))


def theorem1_rank(N: int, eps: float) -> int:
    """r1 = 4 r_H + 2 (2 r_A) + 2 (2 r_B - 1), the number of columns of the
    constructed L1 and L2."""
    dH, dA, dB = theorem1_tolerances(eps)
    return 4 * hilbert_rank(N, dH) + 4 * a1_terms(dA) + 2 * (2 * b0_terms(dB) - 1)


def _agm_sequence(kc: float):
    """Arithmetic-geometric mean of 1 and kc with the half-differences c_n
    (c_0 = sqrt(1 - kc^2)); a fixed cap of 64 halvings, far more than FP64
    convergence needs."""
    a, b, c = [1.0], [kc], [math.sqrt((1.0 - kc) * (1.0 + kc))]
    for _ in range(64):
        if c[-1] <= 4e-16 * a[-1]:
            break
        an, bn = a[-1], b[-1]
        a.append(0.5 * (an + bn))
        b.append(math.sqrt(an * bn))
        c.append(0.5 * (an - bn))
    return a, b, c


def elliptic_k(kc: float) -> float:
    """Complete elliptic integral of the first kind I(tau) for the modulus
    tau = sqrt(1 - kc^2), given the complementary modulus kc (which avoids
    forming 1 - tau^2 when tau is close to 1): pi / (2 AGM(1, kc))."""
    a, _, _ = _agm_sequence(kc)
    return math.pi / (2.0 * a[-1])


def jacobi_dn(u: float, kc: float) -> float:
    """Jacobi elliptic function dn(u, tau), tau = sqrt(1 - kc^2), by the
    descending Landen (AGM) scheme: phi_n = 2^n a_n u, then
    phi_{k-1} = (phi_k + asin(c_k sin(phi_k) / a_k)) / 2, and
    dn = cos(phi_0) / cos(phi_1 - phi_0)."""
    a, _, c = _agm_sequence(kc)
    n = len(a) - 1
    if n == 0:
        return 1.0
    phi = (2.0 ** n) * a[n] * u
    prev = phi
    for k in range(n, 0, -1):
        prev = phi
        phi = 0.5 * (phi + math.asin(c[k] * math.sin(phi) / a[k]))
    return math.cos(phi) / math.cos(prev - phi)


def adi_shifts(a: float, b: float, r: int) -> np.ndarray:
    """The r shifts of the appendix's second remark that minimise
    max over [a, b] of |phi(x)|, phi(x) = prod_j (x - p_j)/(x + p_j):
    p_j = b dn((2j - 1)/(2r) I(tau), tau) with tau = sqrt(1 - (a/b)^2)."""
    kc = a / b
    K = elliptic_k(kc)
    return np.array([b * jacobi_dn((2 * j - 1) / (2.0 * r) * K, kc) for j in range(1, r + 1)])


def adi_rational(x: np.ndarray, p: np.ndarray) -> np.ndarray:
    """phi(x) = prod_j (x - p_j) / (x + p_j)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    for pj in p:
        out = out * (x - pj) / (x + pj)
    return out


def hilbert_factor(N: int, r: int) -> tuple[np.ndarray, np.ndarray]:
    """Z (N x r) with Z Z^T ~= H, H[m, n] = 1/(m + n + 1): the CF-ADI
    iteration of the appendix for A = diag(n + 1/2) (so that H solves
    A X + X A = 1 1^T) and B = the all-ones vector, with the shifts above
    on [1/2, N - 1/2]:  Z_1 = sqrt(2 p_1) (A + p_1 I)^{-1} 1,
    Z_k = sqrt(p_k / p_{k-1}) (I - (p_k + p_{k-1})(A + p_k I)^{-1}) Z_{k-1}.
    Returns (Z, shifts)."""
    alpha = np.arange(N, dtype=np.float64) + 0.5
    p = adi_shifts(0.5, N - 0.5, r)
    Z = np.empty((N, r))
    Z[:, 0] = math.sqrt(2.0 * p[0]) / (alpha + p[0])
    for k in range(1, r):
        Z[:, k] = math.sqrt(p[k] / p[k - 1]) * (1.0 - (p[k] + p[k - 1]) / (alpha + p[k])) * Z[:, k - 1]
    return Z, p


def zeta_coefficients(rA: int) -> np.ndarray:
    """c_k = 1 - (1 - 2^{-(2k-1)}) zeta(2k), k = 1..rA: the coefficients of
    the odd series of A1 (Section 2, "Low rank approximation of A1")."""
    from scipy.special import zeta
    k = np.arange(1, rA + 1)
    return 1.0 - (1.0 - 2.0 ** (-(2 * k - 1))) * zeta(2 * k)


def centred_index(N: int) -> np.ndarray:
    """u_m = (m - (N-1)/2) / N, so that u_m - u_n = (m - n)/N."""
    return (np.arange(N, dtype=np.float64) - 0.5 * (N - 1)) / N


def a1_factor(N: int, rA: int) -> tuple[np.ndarray, np.ndarray]:
    """V_A (N x 2 rA) and C_A with V_A C_A V_A^T = A1~, where
    A1~[m, n] = (2/(N pi)) sum_{k=1}^{rA} c_k ((m - n)/N)^{2k-1}: with
    (m - n)/N = u_m - u_n, the binomial expansion gives
    C_A[i, l] = (2/(N pi)) c_k binom(2k-1, i) (-1)^l for i + l = 2k - 1."""
    from scipy.special import comb
    u = centred_index(N)
    V = u[:, None] ** np.arange(2 * rA)[None, :]
    ck = zeta_coefficients(rA)
    C = np.zeros((2 * rA, 2 * rA))
    for k in range(1, rA + 1):
        p = 2 * k - 1
        for i in range(p + 1):
            C[i, p - i] = 2.0 / (N * math.pi) * ck[k - 1] * comb(p, i, exact=True) * (-1.0) ** (p - i)
    return V, C


def b0_factor(N: int, W: float, Wp: float, rB: int) -> tuple[np.ndarray, np.ndarray]:
    """V_B (N x (2 rB - 1)) and C_B with V_B C_B V_B^T = B0~, where
    B0~[m, n] = (2/(N pi)) sum_{k=0}^{rB-1} (-1)^k theta^{2k+1} / (2k+1)!
    ((m - n)/N)^{2k}, theta = pi (W - W') N (the sine series of B0)."""
    from scipy.special import comb
    u = centred_index(N)
    V = u[:, None] ** np.arange(2 * rB - 1)[None, :]
    theta = math.pi * (W - Wp) * N
    C = np.zeros((2 * rB - 1, 2 * rB - 1))
    for k in range(rB):
        p = 2 * k
        coef = 2.0 / (N * math.pi) * (-1.0) ** k * theta ** (2 * k + 1) / math.factorial(2 * k + 1)
        for i in range(p + 1):
            C[i, p - i] = coef * comb(p, i, exact=True) * (-1.0) ** (p - i)
    return V, C


def theorem1_factor_complex(N: int, W: float, eps: float):
    """L1, L2 (complex, N x r1) of "Putting it all together":
    L1 = [D_A Z/(2 pi j), -D_A J Z/(2 pi j), -D_A^* Z/(2 pi j), D_A^* J Z/(2 pi j),
          D_A V_A/(2j), -D_A^* V_A/(2j), D_B V_B/2, D_B^* V_B/2],
    L2 = [D_A J Z, D_A Z, D_A^* J Z, D_A^* Z, D_A V_A C_A^T, D_A^* V_A C_A^T,
          D_B V_B C_B^T, D_B^* V_B C_B^T],
    with D_A = diag(e^{j 2 pi W' n}), D_B = diag(e^{j pi (W + W') n}),
    2NW' = kf_count(N, W).  L1 L2^* approximates B - F F^* within eps."""
    dH, dA, dB = theorem1_tolerances(eps)
    rH, rA, rB = hilbert_rank(N, dH), a1_terms(dA), b0_terms(dB)
    Wp = kf_count(N, W) / (2.0 * N)
    n = np.arange(N, dtype=np.float64)
    DA = np.exp(2j * math.pi * Wp * n)[:, None]
    DB = np.exp(1j * math.pi * (W + Wp) * n)[:, None]
    Z, _ = hilbert_factor(N, rH)
    JZ = Z[::-1]
    VA, CA = a1_factor(N, rA)
    VB, CB = b0_factor(N, W, Wp, rB)
    s = 1.0 / (2j * math.pi)
    L1 = np.hstack([s * DA * Z, -s * DA * JZ, -s * DA.conj() * Z, s * DA.conj() * JZ,
                    DA * VA / 2j, -DA.conj() * VA / 2j, DB * VB / 2, DB.conj() * VB / 2])
    L2 = np.hstack([DA * JZ, DA * Z, DA.conj() * JZ, DA.conj() * Z,
                    DA * (VA @ CA.T), DA.conj() * (VA @ CA.T), DB * (VB @ CB.T), DB.conj() * (VB @ CB.T)])
    return L1, L2


def theorem1_factor(N: int, W: float, eps: float) -> tuple[np.ndarray, np.ndarray]:
    """Real N x r1 matrices L1_r, L2_r with L1_r L2_r^T = L1 L2^* for the
    constructed factor.  Its columns come in conjugate pairs (the first and
    third groups, the second and fourth, the fifth and sixth, the seventh
    and eighth), so for real x a pair contributes 2 Re(l1 (l2^* x)) =
    2 Re(l1) (Re(l2)^T x) + 2 Im(l1) (Im(l2)^T x): L2_r holds Re and Im of
    the first member of each pair, L1_r twice Re and Im of the matching L1
    column, in the order [Re of groups 1, 2, 5, 7 | Im of groups 1, 2, 5, 7]."""
    dH, dA, dB = theorem1_tolerances(eps)
    rH, rA, rB = hilbert_rank(N, dH), a1_terms(dA), b0_terms(dB)
    Wp = kf_count(N, W) / (2.0 * N)
    n = np.arange(N, dtype=np.float64)
    DA = np.exp(2j * math.pi * Wp * n)[:, None]
    DB = np.exp(1j * math.pi * (W + Wp) * n)[:, None]
    Z, _ = hilbert_factor(N, rH)
    JZ = Z[::-1]
    VA, CA = a1_factor(N, rA)
    VB, CB = b0_factor(N, W, Wp, rB)
    s = 1.0 / (2j * math.pi)
    A1 = np.hstack([s * DA * Z, -s * DA * JZ, DA * VA / 2j, DB * VB / 2])
    A2 = np.hstack([DA * JZ, DA * Z, DA * (VA @ CA.T), DB * (VB @ CB.T)])
    L1r = np.hstack([2.0 * A1.real, 2.0 * A1.imag])
    L2r = np.hstack([A2.real, A2.imag])
    return L1r, L2r
