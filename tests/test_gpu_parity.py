"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Tolerances: the FP32 fast projection must match the FP64 fast oracle to a
relative l2 error of 1e-5 per signal, and the exact projection S_K S_K^T x to
(eps + 1e-6) ||x|| (Corollary 2's bound plus FP32 rounding).  FP64 results
(plan eigenpairs, the FP64 product B x) are held to near machine precision.
"""

import functools
import math
import os
import sys

import numpy as np
import pytest
import torch

from oracle import slepian_oracle as o
from paper_1611_04950_amd import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1611_04950_amd import slepian as S


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def otp(N, W, lo, hi):
    """Oracle transition plan, cached across tests (setup dominates at large N)."""
    return o.transition_plan(N, W, lo, hi)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


# (N, W, eps, batch): single-pass (L <= 8192) and three-pass shapes, ragged
# and odd sizes, W near both ends, tiny N
CASES = [
    (1024, 1 / 16, 1e-6, 8),      # the small workload
    (1000, 0.1, 1e-3, 5),
    (37, 0.2, 1e-6, 3),
    (4096, 0.25, 1e-9, 4),
    (5000, 0.03, 1e-6, 3),        # three-pass FP32 (L = 16384), FP64 three-pass
    (20000, 0.45, 1e-6, 2),
    (65536, 1 / 8, 1e-6, 2),      # the paper-scale workload's shape
    (3, 0.3, 1e-3, 1),
]


@pytest.fixture(scope="module")
def plans():
    cache = {}

    def get(N, W, eps, alpha=0.0):
        key = (N, W, eps, alpha)
        if key not in cache:
            _log(f"plan N={N} W={W} eps={eps} alpha={alpha}")
            cache[key] = S.slepian_plan(N, W, eps, alpha=alpha)
        return cache[key]

    return get


@pytest.mark.parametrize("N,W,eps,b", CASES)
def test_plan_matches_oracle(plans, N, W, eps, b):
    P = plans(N, W, eps)
    info = P.info
    tp = otp(N, W, eps, 1 - eps)
    assert info["K"] == o.choose_K(N, W)
    assert info["L"] == o.fft_length(N)
    r_or = tp["j1"] - tp["j0"]
    assert info["r"] == r_or
    if r_or:
        assert info["l_first"] == tp["lo"] + tp["j0"]
    l0, lam, V = S.slepian_plan_eigenpairs(P)
    lam = lam.numpy()
    V = V.cpu().numpy()
    ell = np.arange(l0, l0 + lam.size)
    # oracle eigenpairs for the same indices
    lo_, hi_ = tp["lo"], tp["hi"]
    assert lo_ <= ell[0] and ell[-1] <= hi_ if lam.size else True
    lam_o = tp["lam"][ell - lo_]
    S_o = tp["S"][:, ell - lo_]
    np.testing.assert_allclose(lam, lam_o, atol=1e-12)
    ov = np.einsum("jn,nj->j", V, S_o)
    assert np.all(ov > 1 - 1e-9), ov.min()
    assert abs(info["lam_Km1"] - tp["lam"][info["K"] - 1 - lo_]) < 1e-12
    assert abs(info["lam_K"] - tp["lam"][info["K"] - lo_]) < 1e-12


@pytest.mark.parametrize("N,W,eps,b", CASES)
def test_project_matches_oracle(plans, N, W, eps, b):
    P = plans(N, W, eps)
    x = synth.gaussian(N, b, 100 + N, device="cuda")
    _log(f"project N={N} b={b}")
    y = S.slepian_project(P, x)
    torch.cuda.synchronize()
    xh = x.double().cpu().numpy()
    yf = o.project_fast(N, W, eps, xh.T, tp=otp(N, W, eps, 1 - eps)).T
    e = rel_err(y.cpu().numpy(), yf)
    assert e.max() <= 1e-5, e
    if N <= 4096:
        ye = o.project_exact(N, W, xh.T).T
        dev = np.linalg.norm(y.double().cpu().numpy() - ye, axis=1) / np.linalg.norm(xh, axis=1)
        assert dev.max() <= eps + 1e-6, dev


def test_project_in_place_and_strided(plans):
    N, W, eps = 1500, 0.07, 1e-6
    P = plans(N, W, eps)
    base = synth.gaussian(N + 13, 5, 7, device="cuda")
    x = base[:, :N]                     # leading dimension N + 13
    ref = S.slepian_project(P, x.contiguous())
    y = torch.zeros((5, N + 13), dtype=torch.float32, device="cuda")[:, :N]
    S.slepian_project(P, x, y)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)
    xc = x.contiguous()
    S.slepian_project(P, xc, xc)       # in place
    torch.cuda.synchronize()
    assert torch.equal(xc, ref)


def test_project_batch_edge_cases(plans):
    N, W, eps = 6000, 0.1, 1e-6
    P = plans(N, W, eps)
    x = synth.gaussian(N, 9, 55, device="cuda")
    full = S.slepian_project(P, x)
    one = S.slepian_project(P, x[3:4])
    torch.cuda.synchronize()
    # a signal's result does not depend on its batch or partner in the pair
    assert torch.allclose(one[0], full[3], rtol=0, atol=1e-6 * float(full[3].abs().max()))
    empty = torch.empty((0, N), dtype=torch.float32, device="cuda")
    assert S.slepian_project(P, empty).shape == (0, N)
    z = torch.zeros((3, N), dtype=torch.float32, device="cuda")
    assert torch.count_nonzero(S.slepian_project(P, z)) == 0


def test_project_deterministic(plans):
    N, W, eps = 65536, 1 / 8, 1e-6
    P = plans(N, W, eps)
    x = synth.gaussian(N, 6, 9, device="cuda")
    a = S.slepian_project(P, x)
    b = S.slepian_project(P, x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("N,W", [(1024, 1 / 16), (3000, 0.2), (70000, 0.05)])
def test_apply_b64_matches_oracle(plans, N, W):
    P = plans(N, W, 1e-6)
    x = synth.gaussian(N, 3, 5, device="cuda").double()
    y = S.slepian_apply_b64(P, x)
    torch.cuda.synchronize()
    ref = o.apply_prolate(N, W, x.cpu().numpy().T).T
    e = rel_err(y.cpu().numpy(), ref)
    assert e.max() < 1e-13, e


@pytest.mark.parametrize("N,W,eps", [(1024, 1 / 16, 1e-6), (9000, 0.1, 1e-4)])
def test_pinv_matches_oracle(plans, N, W, eps):
    P = plans(N, W, eps)
    y = synth.gaussian(N, 3, 21, device="cuda")
    x, rep = S.slepian_lsq(P, y, mode=S.SLEPIAN_PINV, tol=0.0, max_iter=0)
    torch.cuda.synchronize()
    ref = o.pinv_fast(N, W, eps, y.double().cpu().numpy().T, tp=otp(N, W, eps, 1 - eps)).T
    e = rel_err(x.cpu().numpy(), ref)
    assert e.max() <= 1e-5, e
    if N <= 2048:
        ex = o.pinv_exact(N, W, y.double().cpu().numpy().T).T
        dev = np.linalg.norm(x.cpu().numpy() - ex, axis=1) / np.linalg.norm(y.double().cpu().numpy(), axis=1)
        assert dev.max() <= 3 * eps + 1e-5


def test_tikhonov_residual_over_several_sweeps(plans):
    """The refinement keeps B x and B^2 x of the iterate in FP64 and updates
    them with FP32 products of each correction; after several sweeps (an
    unreachable tolerance, so every sweep runs) the residual it reports must
    still be the residual of the x it returns, recomputed from scratch on
    the CPU in FP64 (Corollary 4's normal equations, residual definition)."""
    import ctypes as C
    N, W, eps, alpha, b = 2000, 0.1, 1e-6, 1e-2, 3
    P = plans(N, W, eps, alpha)
    y = synth.sinusoids(N, b, W, 20, 10.0, 77, device="cuda")
    yh = y.double().cpu().numpy().T
    By = o.apply_prolate(N, W, yh)
    for sweeps in (1, 2, 3):
        xd = torch.empty(y.shape, dtype=torch.float64, device="cuda")
        rep = S.LsqReport()
        st = S._lib.slepian_lsq(P.handle, S.SLEPIAN_TIKHONOV, alpha, S._ptr(y), N, S._ptr(xd), N, b, 0.0, sweeps,
                                None, 0, None, C.byref(rep))
        assert st == S.SLEPIAN_ENOCONV and rep.iterations == sweeps, (st, rep.iterations)
        # the report describes the returned x (the residual after the last
        # correction, computed from the incrementally updated B x, B^2 x)
        xh = xd.cpu().numpy().T
        res = By - o.apply_prolate(N, W, o.apply_prolate(N, W, xh)) - alpha * xh
        cpu = float((np.linalg.norm(res, axis=0) / np.linalg.norm(By, axis=0)).max())
        _log(f"sweeps {sweeps}: reported {rep.rel_residual:.3e}, CPU FP64 {cpu:.3e}")
        assert abs(rep.rel_residual - cpu) <= 1e-12 + 1e-3 * cpu, (sweeps, rep.rel_residual, cpu)
    exact = o.tikhonov_exact(N, W, alpha, yh).T
    assert rel_err(xd.cpu().numpy(), exact).max() <= 1e-8


@pytest.mark.parametrize("N,W,eps,alpha", [(1024, 1 / 16, 1e-6, 1e-3), (2000, 0.1, 1e-6, 1e-2)])
def test_tikhonov_fast_and_refined(plans, N, W, eps, alpha):
    P = plans(N, W, eps, alpha)
    assert P.info["r_tik"] > 0
    y = synth.sinusoids(N, 3, W, 20, 10.0, 31, device="cuda")
    yh = y.double().cpu().numpy()
    x0, rep0 = S.slepian_lsq(P, y, mode=S.SLEPIAN_TIKHONOV, alpha=alpha, tol=0.0, max_iter=0)
    torch.cuda.synchronize()
    fast = o.tikhonov_fast(N, W, eps, alpha, yh.T).T
    e = rel_err(x0.cpu().numpy(), fast)
    assert e.max() <= 1e-5, e
    x1, rep = S.slepian_lsq(P, y, mode=S.SLEPIAN_TIKHONOV, alpha=alpha, tol=1e-10, max_iter=20)
    torch.cuda.synchronize()
    assert rep["converged"] == 1 and rep["rel_residual"] <= 1e-10, rep
    exact = o.tikhonov_exact(N, W, alpha, yh.T).T
    e1 = rel_err(x1.cpu().numpy(), exact)
    assert e1.max() <= 1e-8, e1
    # the definition of the residual, checked on the CPU in FP64
    xh = x1.cpu().numpy().T
    By = o.apply_prolate(N, W, yh.T)
    res = By - o.apply_prolate(N, W, o.apply_prolate(N, W, xh)) - alpha * xh
    assert (np.linalg.norm(res, axis=0) / np.linalg.norm(By, axis=0)).max() <= 2e-10


@pytest.mark.parametrize("N,W", [(256, 1 / 8), (1024, 1 / 16), (777, 0.21)])
@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_coeffs_match_oracle(plans, N, W, prec):
    P = plans(N, W, 1e-6) if prec == "fp32" else S.slepian_plan(N, W, 1e-6, precision=S.SLEPIAN_MIXED)
    x = synth.gaussian(N, 5, 3, device="cuda")
    c = S.slepian_coeffs(P, x)
    torch.cuda.synchronize()
    ref = o.coeffs_exact(N, W, x.double().cpu().numpy().T).T
    e = rel_err(c.cpu().numpy(), ref)
    assert e.max() <= 1e-5, e
    # rows of x that are slices with an odd leading dimension, and a strided c
    xb = torch.zeros((5, N + 3), device="cuda")
    xb[:, :N] = x
    cb = torch.full((5, P.K + 5), float("nan"), device="cuda")
    S.slepian_coeffs(P, xb[:, :N], cb[:, :P.K])
    torch.cuda.synchronize()
    assert torch.equal(cb[:, :P.K], c)
    assert torch.isnan(cb[:, P.K:]).all()


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_coeffs_tiles_and_splits(prec):
    """The coefficient GEMM across its tiling: K = 820 Slepian indices (seven
    128-row FP32 tiles or four 256-row mixed tiles, the last one partial),
    300 signals (a full and a partial 256-signal tile), N = 2050 (65 steps
    of 32 samples, 130 substeps of 16, the last ones partial) cut into two
    reduction splits of 33 and 32 steps; against the oracle's S_K^T x, and
    deterministic."""
    N, W, b = 2050, 0.2, 300
    pr = S.SLEPIAN_FP32 if prec == "fp32" else S.SLEPIAN_MIXED
    P = S.slepian_plan(N, W, 1e-6, precision=pr)
    x = synth.gaussian(N, b, 13, device="cuda")
    c = S.slepian_coeffs(P, x)
    torch.cuda.synchronize()
    ref = o.coeffs_exact(N, W, x.double().cpu().numpy().T).T
    e = rel_err(c.cpu().numpy(), ref)
    assert e.max() <= 1e-5, e.max()
    assert torch.equal(S.slepian_coeffs(P, x), c)


def test_save_load_roundtrip(plans, tmp_path):
    N, W, eps = 3000, 0.15, 1e-6
    P = plans(N, W, eps)
    path = str(tmp_path / "p.plan")
    S.slepian_plan_save(P, path)
    Q = S.slepian_plan_load(path)
    assert Q.info == P.info
    x = synth.gaussian(N, 4, 77, device="cuda")
    a = S.slepian_project(P, x)
    b = S.slepian_project(Q, x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_group_matches_single_plans(plans):
    specs = [(1024, 0.05, 1e-3, 4), (5000, 0.2, 1e-6, 3), (20000, 0.11, 1e-6, 2), (2048, 0.25, 1e-3, 7)]
    ps = [plans(N, W, e) for N, W, e, _ in specs]
    xs = [synth.gaussian(N, b, 500 + i, device="cuda") for i, (N, _, _, b) in enumerate(specs)]
    ys = [torch.empty_like(x) for x in xs]
    G = S.slepian_group_create(ps, [b for *_, b in specs])
    for rep in range(3):
        for y in ys:
            y.zero_()
        S.slepian_group_project(G, xs, ys)
        torch.cuda.synchronize()
        for p, x, y in zip(ps, xs, ys):
            ref = S.slepian_project(p, x)
            torch.cuda.synchronize()
            assert torch.equal(y, ref), rep


@pytest.mark.parametrize("prec,rows", [("fp32", 13), ("mixed", 13), ("mixed", 12)])
def test_group_paths_match_single_plans(prec, rows, tmp_path):
    """Every grouped path: single pass with and without the in-kernel
    correction, three passes with the update fused into the inverse column
    pass (L1 <= 16) or applied separately (L1 = 32), odd and unaligned
    lengths, and (rows = 12) three-pass plans tuned to rows of 4096 points
    through a tuning-cache entry (L1 = 64 runs plan by plan); the grouped call
    reproduces the single-plan calls bit for bit, on two calls in a row with
    different buffers."""
    pr = S.SLEPIAN_FP32 if prec == "fp32" else S.SLEPIAN_MIXED
    specs = [(1024, 0.05, 1e-3, 20), (3001, 0.2, 1e-6, 33), (700, 0.3, 1e-6, 3), (20000, 0.11, 1e-6, 9),
             (70001, 0.05, 1e-6, 5), (5000, 0.03, 1e-6, 64), (100, 0.1, 1e-3, 6)]
    if rows == 12:
        cache = str(tmp_path / "rows.txt")
        with open(cache, "w") as f:
            for N, W, e, b in specs:
                f.write(f"slepian-tune-v1 {N} {W!r} {e!r} {pr} {b} 12 4 0 1.0\n")
        ps = [S.slepian_plan(N, W, e, precision=pr, tune=True, tune_batch=b, tune_cache=cache)
              for N, W, e, b in specs]
        assert sum(p.info["row_log2"] == 12 and p.info["col_log2"] > 0 for p in ps) >= 3
    else:
        ps = [S.slepian_plan(N, W, e, precision=pr) for N, W, e, _ in specs]
    G = S.slepian_group_create(ps, [b for *_, b in specs])
    for rep in range(2):
        xs = [synth.gaussian(N, b, 700 + 10 * rep + i, device="cuda") for i, (N, _, _, b) in enumerate(specs)]
        ys = [torch.full_like(x, float("nan")) for x in xs]
        S.slepian_group_project(G, xs, ys)
        torch.cuda.synchronize()
        for p, x, y in zip(ps, xs, ys):
            ref = S.slepian_project(p, x, precision=pr)
            torch.cuda.synchronize()
            assert torch.equal(y, ref), (rep, p.info["N"])


@pytest.mark.parametrize("N,W,eps,b", [(1024, 1 / 16, 1e-6, 8), (65536, 1 / 8, 1e-6, 6), (3000, 0.2, 1e-6, 70)])
def test_project_precision_modes(plans, N, W, eps, b):
    """MIXED (BF16 hi/lo matrix-core correction) meets the FP32 gate of 1e-5;
    BF16 operands alone (no lo terms) meet the 3e-3 gate for an unrefined
    BF16 correction."""
    P = plans(N, W, eps)
    x = synth.gaussian(N, b, 900 + N, device="cuda")
    xh = x.double().cpu().numpy()
    yf = o.project_fast(N, W, eps, xh.T, tp=otp(N, W, eps, 1 - eps)).T
    errs = {}
    for prec in (S.SLEPIAN_FP32, S.SLEPIAN_MIXED, S.SLEPIAN_BF16_RAW):
        y = S.slepian_project(P, x, precision=prec)
        torch.cuda.synchronize()
        errs[prec] = rel_err(y.cpu().numpy(), yf).max()
    _log(f"precision errors N={N}: {errs}")
    assert errs[S.SLEPIAN_FP32] <= 1e-5
    assert errs[S.SLEPIAN_MIXED] <= 1e-5
    assert errs[S.SLEPIAN_BF16_RAW] <= 3e-3
