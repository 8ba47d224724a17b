"""Plain CPU FP64 oracle for the fast factorization S_K S_K^T ~= T1 T2^T of
Section 2.3 ("A fast factorization"), built on Theorem 1.

THIS MODULE IS TEST INFRASTRUCTURE, like the rest of this package: only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it, and it shares no code with the GPU library.

The factorization combines three pieces:
  * F, the partial DFT matrix of Theorem 1: the 2NW' lowest-frequency
    length-N DFT vectors, scaled by 1/sqrt(N), where 2NW' is the odd integer
    nearest to 2NW;
  * L1 L2^T, a rank-r1 approximation of B - F F^* within eps (Theorem 1);
  * U1 U2^T = U_T diag(d) U_T^T over the transition set (Corollary 2,
    Lemma 5).
Then T1 = [F, L1, U1], T2 = [F, L2, U2], the compression is T2^T x (K' =
2NW' + r1 + r numbers) and the recovery T1 c; the two errors add, so
||S_K S_K^T - T1 T2^T|| <= 2 eps.

Readings of points the paper leaves open:
  * 2NW' is the odd integer nearest to 2NW (the printed definition says "to
    W"); when 2NW is an even integer the two candidates tie and the upper one,
    2NW + 1, is taken.
  * For real signals F is replaced by the real matrix F_r whose columns are
    1/sqrt(N), then sqrt(2/N) cos(2 pi k n / N) and -sqrt(2/N) sin(2 pi k n / N)
    for k = 1 .. (2NW' - 1)/2, interleaved in that order.  F_r F_r^T = F F^*
    (both are the projection onto the same real span), so T1 T2^T is
    unchanged and the compressed vector has 2NW' real entries for the F part.
  * L1 L2^T is taken as V diag(mu) V^T, the eigenpairs of the symmetric
    matrix B - F F^* whose |mu| exceeds eps.  Its error is the largest
    discarded |mu| <= eps, and its rank is the least possible for that error,
    so it is at most the r1 of the explicit construction in the proof of
    Theorem 1 (which meets the same error bound).  L1 = V diag(mu), L2 = V.

Parity status: every function is pinned by tests/test_oracle_factorization.py
against closed forms (the Dirichlet kernel of F F^*, orthonormality),
independent library routines (numpy's FFT, dense eigh), and the error bounds
of Theorem 1 and of the factorization (<= eps and <= 2 eps); none is
"parity unpinned".
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
    """Section 2.3's bound on the compressed length:
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


def fast_factorization(N: int, W: float, eps: float, K: int | None = None) -> dict:
    """All pieces of T1 = [F_r, V diag(mu), U diag(d)], T2 = [F_r, V, U]."""
    kf = kf_count(N, W)
    V, mu = difference_factor(N, W, eps, kf)
    tp = so.transition_plan(N, W, eps, 1 - eps, K)
    ells = np.arange(tp["lo"], tp["hi"] + 1)
    d, sel = so.projection_d(tp["lam"], ells, tp["K"], eps)
    return {"N": N, "W": W, "eps": eps, "kf": kf, "V": V, "mu": mu, "U": tp["S"][:, sel], "d": d[sel],
            "K": tp["K"]}


def compress(fac: dict, x: np.ndarray) -> np.ndarray:
    """T2^T x = [F_r^T x; V^T x; U^T x] (Section 2.3), K' rows."""
    x = np.asarray(x, dtype=np.float64)
    return np.concatenate([fr_adjoint(x, fac["kf"]), fac["V"].T @ x, fac["U"].T @ x], axis=0)


def recover(fac: dict, c: np.ndarray) -> np.ndarray:
    """T1 c = F_r c_F + V (mu . c_V) + U (d . c_U) (Section 2.3)."""
    c = np.asarray(c, dtype=np.float64)
    kf, r1 = fac["kf"], fac["mu"].shape[0]
    cf, cv, cu = c[:kf], c[kf:kf + r1], c[kf + r1:]
    mu = fac["mu"] if c.ndim == 1 else fac["mu"][:, None]
    d = fac["d"] if c.ndim == 1 else fac["d"][:, None]
    return fr_apply(cf, fac["N"]) + fac["V"] @ (mu * cv) + fac["U"] @ (d * cu)
