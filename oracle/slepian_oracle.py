"""Plain CPU FP64 oracle for the fast Slepian transform (Karnik, Zhu, Wakin,
Romberg, Davenport, "The Fast Slepian Transform", arXiv:1611.04950).

THIS MODULE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  It shares no code with
the GPU library: nothing here is used to build, run or feed the HIP kernels,
and it does not import the GPU package.

Everything is float64 numpy/scipy, written for readability rather than speed.
Each function names the passage of the paper it follows.  Notation follows the
paper: N (signal length), W (half bandwidth, in cycles/sample), eps (the
tolerance of the fast approximations), K (number of leading Slepian vectors),
B (the N x N prolate matrix), lambda (its eigenvalues, sorted descending),
S (its eigenvectors, the Slepian basis).

Readings of points the paper leaves open:
  * B's diagonal is 2W, the limit of sin(2 pi W k)/(pi k) as k -> 0.
  * K = round(2NW) rounds halves away from zero (Section 4.1 uses "round").
  * The FFT length for B x is the smallest power of two >= 2N (Section 4.1).
  * Individual Slepian vectors are signed so that the first entry whose
    magnitude is >= 1e-3 of the vector's largest magnitude is positive.
  * The fast Tikhonov operator is (1/(1+alpha)) B + U5 U5^T (Corollary 4 and
    Lemma 6); the short restatement in Section 1.3 drops the 1/(1+alpha).
  * The Slepian vectors of large N are computed from the symmetric
    tridiagonal matrix that commutes with B (Slepian 1978, cited by the paper
    as its source for the DPSS); the paper does not print that matrix.  At
    small N the tests pin it against the dense eigendecomposition of B.
  * The projection onto a multiband (modulated Slepian) dictionary, which
    Section 1.4 names without an algorithm, is the orthogonal projection
    onto the span of the modulated bases E_f S_K over the bands' centres
    +-f_i.  It is computed by conjugate gradients on the sum of the bands'
    fast projections (multiband_projection), stopped per signal once the
    residual falls to eps; the plain sum of the bands' projections
    (multiband_fast) is a separate operator, which differs from the
    projection by the subspaces' overlap.

Parity status: every public function below is pinned by tests in
tests/test_oracle_pins.py against closed forms, brute force, invariants the
paper states, or an independent library routine; none is "parity unpinned".
"""

from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

__all__ = [
    "fft_length", "choose_K", "prolate_matrix", "sinc_column",
    "kernel_spectrum", "apply_prolate", "apply_prolate_dense",
    "dense_eig", "slepian_tridiagonal", "slepian_vectors",
    "transition_plan", "partition", "projection_d", "pinv_d", "tikhonov_g",
    "project_exact", "project_fast", "pinv_exact", "pinv_threshold", "pinv_fast",
    "tikhonov_exact", "tikhonov_fast", "tikhonov_cg", "coeffs_exact", "multiband_fast", "multiband_exact",
    "multiband_sum_exact", "multiband_projection",
    "cor1_bound", "asymptotic_count", "sign_fix",
]


# ---------------------------------------------------------------------------
# Sizes (Section 4.1)
# ---------------------------------------------------------------------------

def fft_length(N: int) -> int:
    """Smallest power of two that is at least 2N (Section 4.1)."""
    L = 1
    while L < 2 * N:
        L *= 2
    return L


def choose_K(N: int, W: float) -> int:
    """K = round(2NW) with halves rounded away from zero (Section 4.1)."""
    v = 2.0 * N * W
    return int(math.floor(v + 0.5))


# ---------------------------------------------------------------------------
# The prolate matrix and its product with a vector (Section 1.2, eq. Prolate
# matrix; Section 1.3 and Section 4.1 for the FFT product)
# ---------------------------------------------------------------------------

def _sinc_values(k: np.ndarray, W: float) -> np.ndarray:
    """sin(2 pi W k) / (pi k), with the k = 0 limit 2W."""
    k = np.asarray(k, dtype=np.float64)
    out = np.empty_like(k)
    z = k == 0
    out[z] = 2.0 * W
    kk = k[~z]
    out[~z] = np.sin(2.0 * np.pi * W * kk) / (np.pi * kk)
    return out


def prolate_matrix(N: int, W: float) -> np.ndarray:
    """Dense B[m, n] = sin(2 pi W (m - n)) / (pi (m - n)), diagonal 2W
    (Section 1.2, eq. Prolate matrix)."""
    idx = np.arange(N)
    return _sinc_values(idx[:, None] - idx[None, :], W)


def sinc_column(N: int, W: float) -> np.ndarray:
    """First column of B: c[k] = B[k, 0], k = 0..N-1."""
    return _sinc_values(np.arange(N), W)


def kernel_spectrum(N: int, W: float, L: int | None = None) -> np.ndarray:
    """DFT of the length-L circulant embedding of B's first column.

    The embedding puts c[k] at index k and at index L - k (1 <= k <= N-1) and
    zero elsewhere, so the length-L circular convolution restricted to the
    first N outputs equals the Toeplitz product B x (Section 4.1: B is applied
    with an FFT of length the smallest power of two >= 2N).  The sequence is
    real and even, so its DFT is real; the real part is returned.
    """
    if L is None:
        L = fft_length(N)
    if L < 2 * N - 1:
        raise ValueError("L must be at least 2N-1")
    c = sinc_column(N, W)
    e = np.zeros(L)
    e[:N] = c
    e[L - N + 1:] = c[1:][::-1]
    return sfft.fft(e).real


def apply_prolate(N: int, W: float, x: np.ndarray, L: int | None = None) -> np.ndarray:
    """B x by zero padding to length L, FFT, multiply, inverse FFT, keep the
    first N outputs (Section 1.3 "Fast projections", Section 4.1)."""
    x = np.asarray(x, dtype=np.float64)
    if L is None:
        L = fft_length(N)
    ch = kernel_spectrum(N, W, L)
    X = sfft.fft(x, n=L, axis=0)
    if X.ndim == 2:
        X = X * ch[:, None]
    else:
        X = X * ch
    return sfft.ifft(X, axis=0)[:N].real


def apply_prolate_dense(N: int, W: float, x: np.ndarray) -> np.ndarray:
    """B x by the dense matrix (brute force, small N only)."""
    return prolate_matrix(N, W) @ np.asarray(x, dtype=np.float64)


# ---------------------------------------------------------------------------
# Slepian basis (Definitions 1 and 2; Section 1.2: B = S Lambda S^*)
# ---------------------------------------------------------------------------

def sign_fix(S: np.ndarray) -> np.ndarray:
    """Sign each column so its first entry of magnitude >= 1e-3 * max|.| is
    positive (a convention; the paper leaves the sign free)."""
    S = np.array(S, dtype=np.float64, copy=True)
    if S.ndim == 1:
        S = S[:, None]
        squeeze = True
    else:
        squeeze = False
    for j in range(S.shape[1]):
        col = S[:, j]
        m = np.max(np.abs(col))
        if m == 0:
            continue
        first = np.nonzero(np.abs(col) >= 1e-3 * m)[0][0]
        if col[first] < 0:
            S[:, j] = -col
    return S[:, 0] if squeeze else S


def dense_eig(N: int, W: float):
    """Eigen-decomposition of dense B with eigenvalues sorted descending
    (Section 1.2).  Returns (lam, S) with S[:, l] the l-th Slepian vector."""
    lam, V = np.linalg.eigh(prolate_matrix(N, W))
    order = np.argsort(lam)[::-1]
    return lam[order], sign_fix(V[:, order])


def slepian_tridiagonal(N: int, W: float):
    """Symmetric tridiagonal matrix that commutes with B (Slepian 1978, the
    paper's reference for the DPSS).  Diagonal ((N-1)/2 - n)^2 cos(2 pi W),
    off-diagonal n (N - n) / 2 for n = 1..N-1.  Its eigenvectors are the
    Slepian vectors; its largest eigenvalue belongs to l = 0."""
    n = np.arange(N, dtype=np.float64)
    diag = ((N - 1) / 2.0 - n) ** 2 * np.cos(2.0 * np.pi * W)
    m = np.arange(1, N, dtype=np.float64)
    off = m * (N - m) / 2.0
    return diag, off


def slepian_vectors(N: int, W: float, lo: int, hi: int, L: int | None = None):
    """Slepian vectors l = lo..hi (inclusive) and their eigenvalues.

    The vectors come from the tridiagonal matrix above (bisection plus inverse
    iteration, LAPACK via scipy); each eigenvalue of B is then the Rayleigh
    quotient lambda_l = s_l^T B s_l with B applied by the FFT product.
    Returns (lam[lo..hi], S[:, lo..hi]) with unit-norm, sign-fixed columns.
    """
    if not (0 <= lo <= hi <= N - 1):
        raise ValueError("bad index range")
    d, e = slepian_tridiagonal(N, W)
    # ascending index i = N-1-l
    i_lo, i_hi = N - 1 - hi, N - 1 - lo
    if N == 1:
        S = np.ones((1, 1))
    else:
        _, V = sla.eigh_tridiagonal(d, e, select="i", select_range=(i_lo, i_hi))
        S = V[:, ::-1]  # descending theta == ascending l
    S = S / np.linalg.norm(S, axis=0, keepdims=True)
    S = sign_fix(S)
    BS = apply_prolate(N, W, S, L)
    lam = np.einsum("nj,nj->j", S, BS)
    return lam, S


def asymptotic_count(N: int, eps: float) -> float:
    """(2/pi^2) log N log(1/eps - 1), the asymptotic number of eigenvalues in
    [eps, 1-eps] (Section 1.2, eq. asymptotic)."""
    return 2.0 / np.pi ** 2 * math.log(N) * math.log(1.0 / eps - 1.0)


def cor1_bound(N: int, eps: float) -> float:
    """Corollary 1: #{eps < lambda < 1-eps} <= (8/pi^2 log 8N + 12) log(15/eps)."""
    return (8.0 / np.pi ** 2 * math.log(8 * N) + 12.0) * math.log(15.0 / eps)


def transition_plan(N: int, W: float, thr_lo: float, thr_hi: float,
                    K: int | None = None, L: int | None = None):
    """Slepian vectors whose eigenvalues lie strictly between thr_lo and thr_hi.

    Because lambda is strictly decreasing in l, the set {thr_lo < lambda <
    thr_hi} is a contiguous range of indices.  A window of indices around K
    is solved and grown until its first eigenvalue is >= thr_hi (or the
    window reaches l = 0) and its last is <= thr_lo (or reaches l = N-1).
    Returns dict with the window (lo, hi), its eigenvalues and vectors, and
    the index range [j0, j1) of the selected columns within the window.
    """
    if K is None:
        K = choose_K(N, W)
    h = int(2 * asymptotic_count(max(N, 2), min(thr_lo, 1 - thr_hi)) + 30)
    lo = max(0, K - h)
    hi = min(N - 1, K + h)
    while True:
        lam, S = slepian_vectors(N, W, lo, hi, L)
        ok_lo = lo == 0 or lam[0] >= thr_hi
        ok_hi = hi == N - 1 or lam[-1] <= thr_lo
        if ok_lo and ok_hi:
            break
        h *= 2
        lo = max(0, K - h) if not ok_lo else lo
        hi = min(N - 1, K + h) if not ok_hi else hi
    sel = np.nonzero((lam > thr_lo) & (lam < thr_hi))[0]
    if sel.size:
        j0, j1 = int(sel[0]), int(sel[-1]) + 1
    else:
        j0 = j1 = int(np.searchsorted(-lam, -0.5))
    return {"lo": lo, "hi": hi, "lam": lam, "S": S, "j0": j0, "j1": j1, "K": K}


# ---------------------------------------------------------------------------
# Eigenvalue partition and the diagonal weights of the low-rank corrections
# (Lemma 4, Lemma 5, Lemma 6 in Section 3, the proofs of Corollaries 2-4)
# ---------------------------------------------------------------------------

def partition(lam: np.ndarray, ells: np.ndarray, K: int, eps: float):
    """The sets I1..I4 of Lemma 4: I1 = {lambda >= 1-eps},
    I2 = {l < K, eps < lambda < 1-eps}, I3 = {l >= K, eps < lambda < 1-eps},
    I4 = {lambda <= eps}.  Returns four boolean masks over `ells`."""
    lam = np.asarray(lam)
    ells = np.asarray(ells)
    mid = (lam > eps) & (lam < 1 - eps)
    return (lam >= 1 - eps, mid & (ells < K), mid & (ells >= K), lam <= eps)


def projection_d(lam, ells, K, eps):
    """d for S_K S_K^T ~= B + U diag(d) U^T over I2 u I3 (Lemma 4):
    d = 1 - lambda on I2, d = -lambda on I3 (U1 U2^* written as U diag(d) U^T)."""
    _, i2, i3, _ = partition(lam, ells, K, eps)
    d = np.zeros_like(np.asarray(lam, dtype=np.float64))
    d[i2] = 1.0 - lam[i2]
    d[i3] = -lam[i3]
    return d, (i2 | i3)


def pinv_d(lam, ells, K, eps):
    """d for B_K^+ ~= B + U diag(d) U^T over I2 u I3 (Lemma 5):
    d = 1/lambda - lambda on I2, d = -lambda on I3."""
    _, i2, i3, _ = partition(lam, ells, K, eps)
    d = np.zeros_like(np.asarray(lam, dtype=np.float64))
    d[i2] = 1.0 / lam[i2] - lam[i2]
    d[i3] = -lam[i3]
    return d, (i2 | i3)


def tikhonov_g(lam, alpha, eps):
    """g for (B^2 + alpha I)^-1 B ~= B/(1+alpha) + U diag(g) U^T (Lemma 6):
    g = lambda/(lambda^2 + alpha) - lambda/(1+alpha) on the set
    {alpha(1+alpha) eps < lambda < 1 - eps/3}."""
    lam = np.asarray(lam, dtype=np.float64)
    sel = (lam > alpha * (1 + alpha) * eps) & (lam < 1 - eps / 3.0)
    g = np.zeros_like(lam)
    g[sel] = lam[sel] / (lam[sel] ** 2 + alpha) - lam[sel] / (1 + alpha)
    return g, sel


# ---------------------------------------------------------------------------
# Exact operators (dense; Section 1.3 problem statements)
# ---------------------------------------------------------------------------

def project_exact(N: int, W: float, x: np.ndarray, K: int | None = None) -> np.ndarray:
    """S_K S_K^T x from the dense eigendecomposition (Section 1.3)."""
    if K is None:
        K = choose_K(N, W)
    _, S = dense_eig(N, W)
    SK = S[:, :K]
    return SK @ (SK.T @ np.asarray(x, dtype=np.float64))


def coeffs_exact(N: int, W: float, x: np.ndarray, K: int | None = None) -> np.ndarray:
    """S_K^T x, the K Slepian coefficients (Section 1.3, "A fast factorization"),
    with the oracle's sign convention on each Slepian vector.

    The vectors come from the tridiagonal route: inside the clusters of
    eigenvalues numerically equal to 1, a dense eigensolver of B returns an
    arbitrary orthonormal basis of the cluster, while the individual Slepian
    vectors are defined uniquely (the eigenvalues are distinct, Definition 1)
    and are resolved by the tridiagonal matrix's well separated eigenvalues."""
    if K is None:
        K = choose_K(N, W)
    _, S = slepian_vectors(N, W, 0, K - 1)
    return S.T @ np.asarray(x, dtype=np.float64)


def pinv_exact(N: int, W: float, y: np.ndarray, K: int | None = None) -> np.ndarray:
    """Rank-K truncated pseudoinverse B_K^+ y = S_K Lambda_K^-1 S_K^T y (Lemma 5)."""
    if K is None:
        K = choose_K(N, W)
    lam, S = dense_eig(N, W)
    SK = S[:, :K]
    C = SK.T @ np.asarray(y, dtype=np.float64)
    C = C / lam[:K, None] if C.ndim == 2 else C / lam[:K]
    return SK @ C


def pinv_threshold(N: int, W: float, y: np.ndarray, thr: float) -> tuple[np.ndarray, int]:
    """The truncated pseudoinverse that drops the eigenvalues below thr (the
    Fourier-extension experiment of Section 4.2): rank K = #{lambda >= thr},
    B_K^+ y = S_K Lambda_K^-1 S_K^T y.  Returns (B_K^+ y, K)."""
    lam, _ = dense_eig(N, W)
    K = int((lam >= thr).sum())
    return pinv_exact(N, W, y, K), K


def tikhonov_exact(N: int, W: float, alpha: float, y: np.ndarray) -> np.ndarray:
    """(B^2 + alpha I)^-1 B y by a dense solve (Section 1.3, Tikhonov)."""
    B = prolate_matrix(N, W)
    G = B @ B + alpha * np.eye(N)
    return np.linalg.solve(G, B @ np.asarray(y, dtype=np.float64))


def tikhonov_cg(N: int, W: float, alpha: float, y: np.ndarray, tol: float = 1e-13,
                maxiter: int = 2000) -> np.ndarray:
    """(B^2 + alpha I)^-1 B y by conjugate gradients on the symmetric positive
    definite B^2 + alpha I, with B applied by the FFT product (large N)."""
    y = np.asarray(y, dtype=np.float64)
    cols = y if y.ndim == 2 else y[:, None]
    out = np.empty_like(cols)
    for s in range(cols.shape[1]):
        rhs = apply_prolate(N, W, cols[:, s])
        x = np.zeros(N)
        r = rhs.copy()
        p = r.copy()
        rr = r @ r
        nb = math.sqrt(rhs @ rhs)
        for _ in range(maxiter):
            if math.sqrt(rr) <= tol * nb:
                break
            Ap = apply_prolate(N, W, apply_prolate(N, W, p)) + alpha * p
            a = rr / (p @ Ap)
            x += a * p
            r -= a * Ap
            rr_new = r @ r
            p = r + (rr_new / rr) * p
            rr = rr_new
        out[:, s] = x
    return out if y.ndim == 2 else out[:, 0]


# ---------------------------------------------------------------------------
# Fast operators (Corollaries 2, 3, 4; Section 1.3)
# ---------------------------------------------------------------------------

def _lowrank(S, d, x):
    x = np.asarray(x, dtype=np.float64)
    C = S.T @ x
    return S @ (d[:, None] * C if C.ndim == 2 else d * C)


def project_fast(N: int, W: float, eps: float, x: np.ndarray, K: int | None = None,
                 tp: dict | None = None) -> np.ndarray:
    """B x + U1 U2^T x, the fast projection onto the span of S_K (Corollary 2,
    Lemma 4): U1 U2^T = U_T diag(d) U_T^T over the eigenvalues in (eps, 1-eps)."""
    if tp is None:
        tp = transition_plan(N, W, eps, 1 - eps, K)
    K = tp["K"]
    ells = np.arange(tp["lo"], tp["hi"] + 1)
    d, sel = projection_d(tp["lam"], ells, K, eps)
    return apply_prolate(N, W, x) + _lowrank(tp["S"][:, sel], d[sel], x)


def pinv_fast(N: int, W: float, eps: float, y: np.ndarray, K: int | None = None,
              tp: dict | None = None) -> np.ndarray:
    """B y + U3 U4^T y, the fast truncated pseudoinverse (Corollary 3, Lemma 5)."""
    if tp is None:
        tp = transition_plan(N, W, eps, 1 - eps, K)
    K = tp["K"]
    ells = np.arange(tp["lo"], tp["hi"] + 1)
    d, sel = pinv_d(tp["lam"], ells, K, eps)
    return apply_prolate(N, W, y) + _lowrank(tp["S"][:, sel], d[sel], y)


def tikhonov_fast(N: int, W: float, eps: float, alpha: float, y: np.ndarray,
                  tp: dict | None = None) -> np.ndarray:
    """B y / (1+alpha) + U5 U5^T y, the fast Tikhonov operator (Corollary 4,
    Lemma 6), with U5 = V diag(sqrt(g))."""
    if tp is None:
        tp = transition_plan(N, W, alpha * (1 + alpha) * eps, 1 - eps / 3.0)
    g, sel = tikhonov_g(tp["lam"], alpha, eps)
    return apply_prolate(N, W, y) / (1 + alpha) + _lowrank(tp["S"][:, sel], g[sel], y)


# ---------------------------------------------------------------------------
# Multiband (modulated Slepian) dictionaries (Section 1.4)
# ---------------------------------------------------------------------------

def _band_weight(f: float) -> float:
    return 2.0 if f > 0 else 1.0


def multiband_fast(N: int, W: float, eps: float, freqs, x: np.ndarray, tp: dict | None = None) -> np.ndarray:
    """Sum over bands of the modulated fast projections for a real signal x:
    y = sum_i w_i Re(E_i P~ E_i^* x), E_i = diag(exp(2 pi i f_i n)), w_i = 2
    for f_i > 0 (the pair +-f_i) and 1 for f_i = 0, P~ = B + U diag(d) U^T
    (Corollary 2) applied to the real and imaginary parts (B is real)."""
    if tp is None:
        tp = transition_plan(N, W, eps, 1 - eps)
    x = np.asarray(x, dtype=np.float64)
    n = np.arange(N)
    y = np.zeros_like(x)
    for f in freqs:
        e = np.exp(2j * np.pi * f * n)
        z = (np.conj(e)[:, None] * x) if x.ndim == 2 else np.conj(e) * x
        pz = project_fast(N, W, eps, z.real, tp=tp) + 1j * project_fast(N, W, eps, z.imag, tp=tp)
        y += _band_weight(f) * ((e[:, None] * pz).real if x.ndim == 2 else (e * pz).real)
    return y


def multiband_exact(N: int, W: float, freqs, x: np.ndarray, K: int | None = None) -> np.ndarray:
    """Orthogonal projection of a real x onto the span of the modulated
    Slepian bases E_f S_K, f in {+-f_i} (dense; Section 1.4's merged
    dictionary)."""
    if K is None:
        K = choose_K(N, W)
    _, S = dense_eig(N, W)
    SK = S[:, :K]
    n = np.arange(N)
    cols = []
    for f in freqs:
        e = np.exp(2j * np.pi * f * n)
        cols.append(e[:, None] * SK)
        if f > 0:
            cols.append(np.conj(e)[:, None] * SK)
    Q, _ = np.linalg.qr(np.hstack(cols))
    x = np.asarray(x, dtype=np.float64)
    return (Q @ (Q.conj().T @ x)).real


def multiband_sum_exact(N: int, W: float, freqs, x: np.ndarray, K: int | None = None) -> np.ndarray:
    """sum_i w_i Re(E_i S_K S_K^T E_i^* x) with the dense S_K: what the fast
    sum approximates band by band (Corollary 2 per band)."""
    if K is None:
        K = choose_K(N, W)
    _, S = dense_eig(N, W)
    SK = S[:, :K]
    n = np.arange(N)
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    for f in freqs:
        e = np.exp(2j * np.pi * f * n)[:, None]
        y += _band_weight(f) * (e * (SK @ (SK.T @ (np.conj(e) * x)))).real
    return y


def multiband_projection(N: int, W: float, eps: float, freqs, x: np.ndarray, tol: float | None = None,
                         max_iter: int = 50, tp: dict | None = None, operator=None):
    """Orthogonal projection of a real x onto the span of the modulated
    Slepian dictionary {E_f S_K : f in +-f_i} (Section 1.4, application i),
    by conjugate gradients on the band-sum operator
    A = sum_i w_i Re(E_i P~ E_i^* .) (multiband_fast; P~ the fast projection
    of Corollary 2).

    With exact projections P_f, A is the sum of the orthogonal projections
    onto the dictionary's subspaces: symmetric, positive semidefinite, with
    range equal to their span.  CG on A z = A x from z = 0 keeps its iterates
    in the Krylov space of A x, inside that range, and its solution there is
    the orthogonal projection of x onto the span.  With the fast P~ the
    complement of the span carries eigenvalues of A of size at most about
    eps rather than 0, so the iteration stops per signal at the first step
    whose residual ||A x - A z|| is at most tol ||A x|| (default tol = eps),
    before it starts to resolve them.  `operator` replaces A (for tests).
    Returns (z, iterations per signal)."""
    if tol is None:
        tol = eps
    x = np.asarray(x, dtype=np.float64)
    X = x if x.ndim == 2 else x[:, None]
    if operator is None:
        if tp is None:
            tp = transition_plan(N, W, eps, 1 - eps)

        def operator(v):
            return multiband_fast(N, W, eps, freqs, v, tp=tp)
    b = operator(X)
    z = np.zeros_like(X)
    r = b.copy()
    p = r.copy()
    rr = np.einsum("ns,ns->s", r, r)
    nb = np.sqrt(rr)
    active = np.sqrt(rr) > tol * nb
    iters = np.zeros(X.shape[1], dtype=np.int64)
    for _ in range(max_iter):
        if not active.any():
            break
        Ap = operator(p)
        pAp = np.einsum("ns,ns->s", p, Ap)
        a = np.where(active, rr / np.where(active, pAp, 1.0), 0.0)
        z += a * p
        r -= a * Ap
        rr_new = np.einsum("ns,ns->s", r, r)
        beta = np.where(active, rr_new / np.where(active, rr, 1.0), 0.0)
        p = np.where(active, r + beta * p, p)
        rr = np.where(active, rr_new, rr)
        iters += active
        active = active & (np.sqrt(rr) > tol * nb)
    return (z if x.ndim == 2 else z[:, 0]), iters

