"""Multiband (modulated Slepian) dictionaries on the GPU (Section 1.4,
application i): the projection onto the span of the modulated dictionary
(conjugate gradients on the band sum, slepian_project_bands_span) against
the FP64 oracle's same iteration (1e-5 relative per signal, FP32 and mixed
plans, N = 512..4096 with 2 to 8 bands, and sampled signals at N = 2^16) and
against the dense projection onto the span; the band sum
y = sum_i w_i Re(E_i P~ E_i^* x) band by band against the oracle's; in
place, the iteration's failure return, and the band validation of the C
entry point."""

import numpy as np
import pytest
import torch

from oracle import slepian_oracle as o
from paper_1611_04950_amd import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1611_04950_amd import slepian as S

CASES = [(512, 1 / 32, 1e-6, [0.0, 0.125, 0.25, 0.375]), (4096, 1 / 64, 1e-6, [0.05, 0.2, 0.41]),
         (3001, 0.02, 1e-3, [0.0, 0.3])]


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


@pytest.mark.parametrize("N,W,eps,bands", CASES)
@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_multiband_matches_oracle(N, W, eps, bands, prec):
    P = S.slepian_plan(N, W, eps, precision=S.SLEPIAN_MIXED if prec == "mixed" else S.SLEPIAN_FP32)
    x = synth.gaussian(N, 5, 91, device="cuda")
    y = S.slepian_project_multiband(P, bands, x)
    torch.cuda.synchronize()
    ref = o.multiband_fast(N, W, eps, bands, x.double().cpu().numpy().T).T
    e = _rel(y.cpu().numpy(), ref)
    assert e.max() <= 1e-5, e
    # in place
    z = x.clone()
    S.slepian_project_multiband(P, bands, z, z)
    torch.cuda.synchronize()
    assert torch.equal(z, y)


SPAN_CASES = [(512, 1 / 32, 1e-6, [0.0, 0.125, 0.25, 0.375]),
              (1024, 1 / 64, 1e-6, [1 / 64, 3 / 64, 5 / 64, 7 / 64, 9 / 64]),
              (2048, 1 / 128, 1e-6, [1 / 32 + k / 16 for k in range(8)]),
              (4096, 1 / 64, 1e-3, [0.05, 0.2, 0.41]),
              (3001, 0.02, 1e-6, [0.0, 0.3])]


@pytest.mark.parametrize("N,W,eps,bands", SPAN_CASES)
@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_span_projection_matches_oracle(N, W, eps, bands, prec):
    print(f"span projection N={N} W={W} eps={eps} bands={len(bands)} {prec}", flush=True)
    P = S.slepian_plan(N, W, eps, precision=S.SLEPIAN_MIXED if prec == "mixed" else S.SLEPIAN_FP32)
    B = S.slepian_bands_create(P, bands)
    x = synth.gaussian(N, 4, 93, device="cuda")
    y, it = S.slepian_project_bands_span(B, x)
    torch.cuda.synchronize()
    xh = x.double().cpu().numpy().T
    tol = max(eps, 1e-6)
    ref, it_o = o.multiband_projection(N, W, eps, bands, xh, tol=tol)
    e = _rel(y.double().cpu().numpy(), ref.T)
    print(f"  steps GPU {it}, oracle {list(it_o)}; max rel diff {e.max():.2e}", flush=True)
    assert e.max() <= 1e-5, e
    assert all(abs(a - b) <= 1 for a, b in zip(it, it_o))
    if N <= 2048:
        ex = o.multiband_exact(N, W, bands, xh).T
        J = sum(2 if f > 0 else 1 for f in bands)
        d = np.linalg.norm(y.double().cpu().numpy() - ex, axis=1) / np.linalg.norm(xh.T, axis=1)
        assert d.max() <= 2 * J * eps + 1e-5


def test_span_projection_sampled_at_2p16():
    """N = 2^16, W = 1/64, four bands, 6 signals on the GPU; signals 0 and 5
    against the oracle's iteration."""
    N, W, eps = 1 << 16, 1 / 64, 1e-6
    bands = [0.0, 0.1, 0.25, 0.4]
    P = S.slepian_plan(N, W, eps, precision=S.SLEPIAN_MIXED)
    B = S.slepian_bands_create(P, bands)
    x = synth.gaussian(N, 6, 95, device="cuda")
    y, it = S.slepian_project_bands_span(B, x)
    torch.cuda.synchronize()
    pick = [0, 5]
    xh = x[pick].double().cpu().numpy().T
    ref, it_o = o.multiband_projection(N, W, eps, bands, xh, tol=eps)
    e = _rel(y[pick].double().cpu().numpy(), ref.T)
    print(f"  N=2^16 steps GPU {it}, oracle {list(it_o)}; max rel diff {e.max():.2e}", flush=True)
    assert e.max() <= 1e-5, e


def test_span_projection_in_place_workspace_and_failure():
    N, W, eps = 2048, 1 / 64, 1e-6
    P = S.slepian_plan(N, W, eps)
    B = S.slepian_bands_create(P, [0.0, 0.25])
    x = synth.gaussian(N, 3, 7, device="cuda")
    y, it = S.slepian_project_bands_span(B, x)
    z = x.clone()
    nbytes = S.slepian_bands_span_workspace_size(B, 3)
    assert nbytes >= 3 * 3 * N * 4
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    z2, it2 = S.slepian_project_bands_span(B, z, z, work=work)
    torch.cuda.synchronize()
    assert torch.equal(z, y) and it2 == it
    # one step cannot meet the tolerance: ENOCONV, the first iterate kept
    y1, it1, st = S.slepian_project_bands_span(B, x, max_iter=1, check=False)
    assert st == S.SLEPIAN_ENOCONV and it1 == [1, 1, 1]
    # bad tolerances and step counts
    for tol, mi in ((1e-8, 10), (0.5, 10), (1e-3, 0), (1e-3, 1001)):
        with pytest.raises(S.SlepianError) as ei:
            S.slepian_project_bands_span(B, x, tol=tol, max_iter=mi)
        assert ei.value.status == S.SLEPIAN_EINVAL
    # a zero signal stops at once with a zero projection
    y0, it0 = S.slepian_project_bands_span(B, torch.zeros((2, N), device="cuda"))
    torch.cuda.synchronize()
    assert it0 == [0, 0] and bool((y0 == 0).all())


def test_bad_bands_rejected():
    P = S.slepian_plan(1024, 1 / 32, 1e-6)
    x = synth.gaussian(1024, 2, 3, device="cuda")
    for bands in ([0.01], [0.49], [0.1, 0.12], [-0.1], [0.5], [0.2] * 65):
        with pytest.raises(S.SlepianError):
            S.slepian_project_multiband(P, bands, x)


@pytest.mark.parametrize("f", [0.0, 0.3125, 0.4921875])
def test_single_band_full_size_composition(f):
    """At N = 2^20 (phases f n up to 5e5 turns): the one-band sum equals
    w Re(E P~ E^* x) assembled from the plain projection of the real and
    imaginary parts, with the modulation done in FP64 by torch."""
    N, W, eps = 1 << 20, 1 / 256, 1e-6
    P = S.slepian_plan(N, W, eps)
    x = synth.gaussian(N, 2, 17, device="cuda")
    y = S.slepian_project_multiband(P, [f], x)
    n = torch.arange(N, dtype=torch.float64, device="cuda")
    ph = torch.remainder(f * n, 1.0) * (2 * np.pi)
    c, s = torch.cos(ph), torch.sin(ph)
    xd = x.double()
    zr, zi = (xd * c).float(), (-xd * s).float()
    pr = S.slepian_project(P, zr)
    pi_ = S.slepian_project(P, zi)
    w = 1.0 if f == 0.0 else 2.0
    ref = w * (c * pr.double() - s * pi_.double())
    torch.cuda.synchronize()
    e = (torch.linalg.vector_norm(y.double() - ref, dim=1) / torch.linalg.vector_norm(ref, dim=1)).max().item()
    assert e <= 1e-5, e


def test_workspace_size_and_explicit_workspace():
    P = S.slepian_plan(2048, 1 / 32, 1e-6)
    x = synth.gaussian(2048, 3, 5, device="cuda")
    nbytes = S.slepian_workspace_size(P, S.SLEPIAN_OP_MULTIBAND, 2 * 3)
    assert nbytes >= 2 * 2 * 2 * 3 * 2048 * 4
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y1 = S.slepian_project_multiband(P, [0.0, 0.25], x, work=work)
    y2 = S.slepian_project_multiband(P, [0.0, 0.25], x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    with pytest.raises(S.SlepianError):
        S.slepian_project_multiband(P, [0.0, 0.25], x, work=work[: nbytes // 2])


# Prepared band sets: one FFT product with the band-sum kernel and a modulated
# correction of rank 2 J r.  Batches and band counts below cover every column
# packing of the correction (G = 1, 4, 8, 16 and 32 signals per 32-column
# block, one and several column groups), a rank above one 32-row block
# (N = 4096, W = 1/8, eps = 1e-12: r = 46), unaligned rows (odd N) and a
# plan whose product runs in three passes (N = 5000).
BAND_CASES = [
    (512, 1 / 32, 1e-6, [0.0, 0.125, 0.25, 0.375], 5),
    (4096, 1 / 64, 1e-6, [0.05, 0.2, 0.41], 16),
    (3001, 0.02, 1e-3, [0.0, 0.3], 1),
    (2048, 1 / 128, 1e-6, [0.0] + [k / 40 for k in range(1, 20)], 16),
    (4096, 1 / 8, 1e-12, [0.0, 0.25], 70),
    (777, 0.01, 1e-6, [0.03], 3),
    (5000, 1 / 40, 1e-6, [0.0, 0.2, 0.35], 7),  # L = 16384: the three-pass product
]


@pytest.mark.parametrize("N,W,eps,bands,b", BAND_CASES)
@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_prepared_bands_match_oracle(N, W, eps, bands, b, prec):
    P = S.slepian_plan(N, W, eps, precision=S.SLEPIAN_MIXED if prec == "mixed" else S.SLEPIAN_FP32)
    B = S.slepian_bands_create(P, bands)
    x = synth.gaussian(N, b, 123, device="cuda")
    y = S.slepian_project_bands(B, x)
    torch.cuda.synchronize()
    ref = o.multiband_fast(N, W, eps, bands, x.double().cpu().numpy().T).T
    e = _rel(y.cpu().numpy(), ref)
    print(f"N={N} bands={len(bands)} b={b} {prec}: max rel err {e.max():.2e}")
    assert e.max() <= 1e-5, e
    # in place, and with a caller-owned workspace: the same bits
    z = x.clone()
    S.slepian_project_bands(B, z, z)
    work = torch.empty(S.slepian_bands_workspace_size(B, b), dtype=torch.uint8, device="cuda")
    w = S.slepian_project_bands(B, x, work=work)
    torch.cuda.synchronize()
    assert torch.equal(z, y)
    assert torch.equal(w, y)


def test_prepared_bands_full_size_against_per_band_path():
    """N = 2^20, W = 1/256, eight bands (2k+1)/32, 16 signals: the prepared
    set against the band-by-band path (two independent GPU computations of
    the same operator), in both precisions."""
    N, W, eps = 1 << 20, 1 / 256, 1e-6
    freqs = [(2 * k + 1) / 32 for k in range(8)]
    x = synth.gaussian(N, 16, 4242, device="cuda")
    for prec in (S.SLEPIAN_FP32, S.SLEPIAN_MIXED):
        P = S.slepian_plan(N, W, eps, precision=prec)
        B = S.slepian_bands_create(P, freqs)
        y = S.slepian_project_bands(B, x)
        ref = S.slepian_project_multiband(P, freqs, x)
        torch.cuda.synchronize()
        e = (torch.linalg.vector_norm((y - ref).double(), dim=1) / torch.linalg.vector_norm(ref.double(), dim=1))
        print(f"precision {prec}: max rel diff {e.max().item():.2e}")
        assert e.max().item() <= 1e-5


def test_prepared_bands_errors():
    P = S.slepian_plan(1024, 1 / 32, 1e-6)
    for bands in ([0.01], [0.49], [0.1, 0.12], [], [0.2] * 65):
        with pytest.raises(S.SlepianError):
            S.slepian_bands_create(P, bands)
    B = S.slepian_bands_create(P, [0.0, 0.25])
    x = synth.gaussian(1024, 4, 9, device="cuda")
    need = S.slepian_bands_workspace_size(B, 4)
    with pytest.raises(S.SlepianError):
        S.slepian_project_bands(B, x, work=torch.empty(need // 2, dtype=torch.uint8, device="cuda"))
    with pytest.raises(S.SlepianError):  # partial overlap of x and y
        buf = torch.zeros(5 * 1024, device="cuda")
        S.slepian_project_bands(B, buf[:4096].view(4, 1024), buf[1024:].view(4, 1024))
    y0 = S.slepian_project_bands(B, x[:0])
    assert y0.shape == (0, 1024)
