"""Oracle pins for the multiband (modulated Slepian) dictionaries (Section
1.4, application i): the orthogonal projection onto the dictionary's span by
conjugate gradients on the band-sum operator (against the dense union
projection, with exact and with fast per-band projections); the band-by-band fast sum reduces to the fast projection for the
baseband band alone and matches the dense per-band sum within the bands'
eps; the dense union projection is an orthogonal projector that keeps the
dictionary's span; the sum differs from the union projection by the
subspaces' mutual coherence, measured and bounded here.  Also the host
checks of the C entry point's band validation, and the two identities the
prepared band sets compute with (dense, in FP64): the bands' B parts add up
to one Toeplitz product, and the bands' corrections to one correction with
modulated columns."""

import ctypes as C

import numpy as np
import pytest

from oracle import slepian_oracle as o

N, W, EPS = 512, 1 / 32, 1e-6
BANDS = [0.0, 0.125, 0.25, 0.375]


def _x(seed=2, b=3):
    return np.random.default_rng(seed).standard_normal((N, b))


def test_baseband_alone_is_the_fast_projection():
    x = _x()
    np.testing.assert_allclose(o.multiband_fast(N, W, EPS, [0.0], x), o.project_fast(N, W, EPS, x),
                               rtol=0, atol=1e-12)


def test_fast_sum_matches_dense_sum():
    x = _x()
    yf = o.multiband_fast(N, W, EPS, BANDS, x)
    yd = o.multiband_sum_exact(N, W, BANDS, x)
    # each band's fast projection is within eps of S_K S_K^T (Corollary 2);
    # weights sum to 1 + 2 + 2 + 2
    assert np.linalg.norm(yf - yd, axis=0).max() <= 7 * EPS * np.linalg.norm(x, axis=0).max()


def test_union_projection_is_an_orthogonal_projector():
    x, z = _x(3), _x(4)
    px = o.multiband_exact(N, W, BANDS, x)
    np.testing.assert_allclose(o.multiband_exact(N, W, BANDS, px), px, rtol=0, atol=1e-10)
    pz = o.multiband_exact(N, W, BANDS, z)
    np.testing.assert_allclose(px.T @ z, x.T @ pz, rtol=1e-10, atol=1e-10)
    # a real combination of the modulated Slepian vectors is kept
    _, S = o.dense_eig(N, W)
    SK = S[:, :o.choose_K(N, W)]
    n = np.arange(N)
    c = np.random.default_rng(5).standard_normal(SK.shape[1])
    v = SK @ c + 2 * (np.exp(2j * np.pi * 0.25 * n) * (SK @ c)).real
    np.testing.assert_allclose(o.multiband_exact(N, W, BANDS, v), v, rtol=0, atol=1e-9 * np.abs(v).max())


def test_sum_versus_union_projection_coherence():
    x = _x(6)
    yf = o.multiband_fast(N, W, EPS, BANDS, x)
    ye = o.multiband_exact(N, W, BANDS, x)
    dev = np.linalg.norm(yf - ye) / np.linalg.norm(ye)
    assert 1e-4 < dev < 3e-2


# ---------------------------------------------------------------------------
# The projection onto the span by conjugate gradients on the band-sum operator
# ---------------------------------------------------------------------------

SPAN_CASES = [
    (512, 1 / 32, [0.0, 0.125, 0.25, 0.375], 1e-6),
    (512, 1 / 32, [0.0, 1 / 16, 2 / 16, 3 / 16], 1e-6),      # adjacent bands
    (1024, 1 / 64, [1 / 64, 3 / 64, 5 / 64, 7 / 64, 9 / 64], 1e-3),
    (1000, 1 / 40, [0.1, 0.2, 0.3, 0.4, 0.475], 1e-9),
    (768, 1 / 16, [1 / 16, 3 / 16], 1e-6),
]


@pytest.mark.parametrize("n,w,freqs", [(c[0], c[1], c[2]) for c in SPAN_CASES[:4]])
def test_span_cg_with_exact_projections_reaches_the_union_projection(n, w, freqs):
    """With the band sum of the dense projections S_K S_K^T as the operator,
    CG from z = 0 converges to the orthogonal projection onto the span (the
    QR route of multiband_exact), to rounding."""
    x = np.random.default_rng(11).standard_normal((n, 3))
    z, it = o.multiband_projection(n, w, 1e-6, freqs, x, tol=1e-12, max_iter=80,
                                   operator=lambda v: o.multiband_sum_exact(n, w, freqs, v))
    ref = o.multiband_exact(n, w, freqs, x)
    assert np.linalg.norm(z - ref, axis=0).max() <= 1e-9 * np.linalg.norm(x, axis=0).max()
    assert it.max() < 80


@pytest.mark.parametrize("n,w,freqs,eps", SPAN_CASES)
def test_span_cg_with_fast_projections_within_eps(n, w, freqs, eps):
    """With the fast operator and tol = eps the result lies within a few eps
    (relative to ||x||) of the orthogonal projection onto the span, its
    residual x - z is orthogonal to every modulated Slepian vector to the
    same level, and it stops within 25 steps."""
    x = np.random.default_rng(12).standard_normal((n, 3))
    z, it = o.multiband_projection(n, w, eps, freqs, x)
    ref = o.multiband_exact(n, w, freqs, x)
    xn = np.linalg.norm(x, axis=0)
    J = sum(2 if f > 0 else 1 for f in freqs)
    assert (np.linalg.norm(z - ref, axis=0) / xn).max() <= 2 * J * eps
    assert it.max() <= 25 and it.min() >= 1
    _, S = o.dense_eig(n, w)
    SK = S[:, :o.choose_K(n, w)]
    t = np.arange(n)
    for f in freqs:
        e = np.exp(2j * np.pi * f * t)[:, None]
        g = SK.T @ (np.conj(e) * (x - z))
        assert (np.linalg.norm(g, axis=0) / xn).max() <= 2 * J * eps
    # the band sum alone is much farther from the projection
    yb = o.multiband_fast(n, w, eps, freqs, x)
    assert (np.linalg.norm(yb - ref, axis=0) / xn).max() > 10 * (np.linalg.norm(z - ref, axis=0) / xn).max()


def test_span_cg_of_a_dictionary_vector_is_itself():
    n, w, freqs = 512, 1 / 32, [0.0, 0.25]
    _, S = o.dense_eig(n, w)
    SK = S[:, :o.choose_K(n, w)]
    t = np.arange(n)
    c = np.random.default_rng(5).standard_normal(SK.shape[1])
    v = SK @ c + 2 * (np.exp(2j * np.pi * 0.25 * t) * (SK @ c)).real
    z, _ = o.multiband_projection(n, w, 1e-6, freqs, v)
    assert np.linalg.norm(z - v) <= 1e-5 * np.linalg.norm(v)


def test_planted_cg_mistakes_are_caught(monkeypatch):
    """A wrong sign in the direction update, or a start at z = x, fails the
    exact-projection pin above."""
    n, w, freqs = 512, 1 / 32, [0.0, 1 / 16, 2 / 16]
    x = np.random.default_rng(11).standard_normal((n, 2))
    ref = o.multiband_exact(n, w, freqs, x)
    opx = lambda v: o.multiband_sum_exact(n, w, freqs, v)  # noqa: E731
    src = o.multiband_projection.__code__
    import types
    for old, new in (("p = np.where(active, r + beta * p, p)", "p = np.where(active, r - beta * p, p)"),
                     ("z = np.zeros_like(X)", "z = X.copy()")):
        import inspect
        code = inspect.getsource(o.multiband_projection)
        assert old in code
        ns = {}
        exec(compile(code.replace(old, new), "<planted>", "exec"), o.__dict__.copy(), ns)
        z, _ = ns["multiband_projection"](n, w, 1e-6, freqs, x, tol=1e-12, max_iter=80, operator=opx)
        assert np.linalg.norm(z - ref, axis=0).max() > 1e-6 * np.linalg.norm(x, axis=0).max()
    assert src is o.multiband_projection.__code__


def test_bad_bands_rejected_before_device_work():
    pytest.importorskip("torch")
    from paper_1611_04950_amd import slepian as S
    lib = S._lib
    for freqs in ([0.01], [0.49], [0.1, 0.12], [-0.1], [0.5]):
        f = (C.c_double * len(freqs))(*freqs)
        # a null plan is rejected first; the band checks need a plan, so
        # check the count and pointer rules here and the band rules on the GPU
        assert lib.slepian_project_multiband(None, len(freqs), f, None, 0, None, 0, 1, None, 0, None) == \
            S.SLEPIAN_EINVAL
    assert lib.slepian_project_multiband(None, 0, None, None, 0, None, 0, 0, None, 0, None) == S.SLEPIAN_EINVAL


def test_band_sum_of_B_is_one_toeplitz_product():
    """sum_i w_i Re(E_i B E_i^* x) = T x for real x, T the symmetric Toeplitz
    matrix of k(m) = b(m) sum_i w_i cos(2 pi f_i m), b(m) = sin(2 pi W m)/(pi m)
    (b(0) = 2W).  It holds band by band, whatever the weights; a sine in place
    of the cosine, or a phase of f m instead of 2 pi f m, breaks it."""
    n = 200
    x = np.random.default_rng(4).standard_normal((n, 3))
    B = o.prolate_matrix(n, W)
    t = np.arange(n)
    lhs = np.zeros_like(x)
    for f in BANDS:
        e = np.exp(2j * np.pi * f * t)
        lhs += (2.0 if f > 0 else 1.0) * (e[:, None] * (B @ (np.conj(e)[:, None] * x))).real
    m = np.abs(t[:, None] - t[None, :])
    bm = np.where(m == 0, 2 * W, np.sin(2 * np.pi * W * m) / (np.pi * np.maximum(m, 1)))
    k = bm * sum((2.0 if f > 0 else 1.0) * np.cos(2 * np.pi * f * m) for f in BANDS)
    np.testing.assert_allclose(k @ x, lhs, rtol=0, atol=1e-12 * np.abs(lhs).max())


def test_band_sum_of_corrections_is_one_modulated_correction():
    """sum_i w_i Re(E_i U D U^T E_i^* x) = sum_(i,c) w_i V_ic D V_ic^T x with
    V_i0 = cos(2 pi f_i n) U and V_i1 = -sin(2 pi f_i n) U (rows scaled), for
    real U, diagonal D and real x."""
    n, r = 150, 7
    rng = np.random.default_rng(6)
    U = rng.standard_normal((n, r))
    D = np.diag(rng.standard_normal(r))
    x = rng.standard_normal((n, 2))
    t = np.arange(n)
    lhs = np.zeros_like(x)
    rhs = np.zeros_like(x)
    for f in BANDS:
        w = 2.0 if f > 0 else 1.0
        e = np.exp(2j * np.pi * f * t)
        lhs += w * (e[:, None] * (U @ D @ U.T @ (np.conj(e)[:, None] * x))).real
        for m in (np.cos(2 * np.pi * f * t), -np.sin(2 * np.pi * f * t)):
            V = m[:, None] * U
            rhs += w * (V @ D @ V.T @ x)
    np.testing.assert_allclose(rhs, lhs, rtol=0, atol=1e-12 * np.abs(lhs).max())
