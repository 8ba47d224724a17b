"""Fast factorization S_K S_K^T ~= T1 T2^T on the GPU (Section 1.3 "A fast
factorization", Theorem 1) against the FP64 oracle in oracle/factorization.py,
for both ways of getting the factor L1 L2^* of B - F F^*.

Theorem 1's construction (Section 2, the library's default): r1 and the
construction's rH, rA, rB equal the oracle's; the rows of T2 and the columns
of T1 (compression of unit vectors, recovery of unit coefficients) equal the
oracle's L2 and L1 entry by entry (1e-5 of each column's norm); the
compressed L2^T x and the round trip match the oracle's (1e-5), and, where
the dense projection is affordable, the round trip lies within
(2 eps + 1e-6) ||x|| of S_K S_K^T x.

The eigenpair factor (SLEPIAN_FACTOR_EIG), compared element by element on
the same seeded FP32 inputs:
  * kf, r and the factor's eigenvalues mu (the setup's subspace iteration
    against dense eigh / Lanczos on the same Toeplitz matrix, 1e-9 absolute);
  * the compressed F_r^T x (unique; 1e-5 of the signal's coefficient norm);
  * U^T x (sign convention shared) and V^T x for the columns with |mu| >=
    1e-3 (well separated, so unique up to the shared sign convention);
  * the recovery T1 T2^T x (a rotation inside V or a Ritz value at eps does
    not move it beyond eps; 1e-5 relative, the FP32 gate);
  * F_r c alone for random coefficients (the inverse path by itself);
and, where the dense projection is affordable, ||T1 T2^T x - S_K S_K^T x||
<= (2 eps + 1e-6) ||x|| (the factorization's bound plus the FP32 floor).
r1 may differ from the oracle's by one only when the boundary |mu| lies
within 1% of eps (either choice then meets the bound).
"""

import numpy as np
import pytest
import torch

from oracle import factorization as fz
from oracle import slepian_oracle as so
from paper_1611_04950_amd import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1611_04950_amd import slepian as S

# N, W, eps, batch, precision: single pass (L <= 8192) and three passes (L1 = 4, 16 with the
# update fused into the inverse column pass, L1 = 32 without)
CASES = [
    (256, 1 / 8, 1e-6, 5, "fp32"),
    (1024, 1 / 16, 1e-6, 8, "mixed"),
    (4096, 0.2, 1e-3, 3, "fp32"),
    (16384, 1 / 8, 1e-6, 6, "mixed"),
    (16384, 0.05, 1e-4, 7, "fp32"),
    (65536, 1 / 8, 1e-6, 4, "mixed"),
    (131072, 1 / 16, 1e-6, 3, "fp32"),  # L1 = 32: update after the inverse column pass
    (262144, 0.05, 1e-4, 2, "mixed"),  # L1 = 64: column passes through LDS
]
_FAC = {}


def _prec(name):
    return {"fp32": S.SLEPIAN_FP32, "mixed": S.SLEPIAN_MIXED}[name]


def _oracle(N, W, eps, method="eig"):
    key = (N, W, eps, method)
    if key not in _FAC:
        if len(_FAC) > 4:
            _FAC.clear()
        _FAC[key] = fz.fast_factorization(N, W, eps, method=method)
    return _FAC[key]


def _x(N, b, seed):
    return synth.gaussian(N, b, seed).numpy().T  # N x b FP32


def _setup(N, W, eps, prec, method=None):
    P = S.slepian_plan(N, W, eps, precision=_prec(prec))
    F = S.slepian_factor_create(P, S.SLEPIAN_FACTOR_EIG if method == "eig" else S.SLEPIAN_FACTOR_THEOREM1)
    return P, F


def _check_r1(F, fac, eps):
    mu_o = np.abs(fac["mu"])
    if F.info["r1"] != len(mu_o):
        # the boundary value must be within 1% of eps for either choice to stand
        t = fz.difference_factor(fac["N"], fac["W"], eps * 0.5, fac["kf"])[1]
        near = np.abs(np.abs(t) - eps) <= 0.01 * eps
        assert abs(F.info["r1"] - len(mu_o)) == 1 and near.any()


@pytest.mark.parametrize("N,W,eps,b,prec", CASES)
def test_theorem1_factorization_matches_oracle(N, W, eps, b, prec):
    print(f"theorem1 factorization N={N} W={W} eps={eps} b={b} {prec}", flush=True)
    P, F = _setup(N, W, eps, prec)
    fac = _oracle(N, W, eps, "theorem1")
    kf, r, r1 = fac["kf"], fac["U"].shape[1], fac["r1"]
    dH, dA, dB = fz.theorem1_tolerances(eps)
    assert F.info["method"] == S.SLEPIAN_FACTOR_THEOREM1 and F.mu is None
    assert (F.info["r_h"], F.info["r_a"], F.info["r_b"]) == (fz.hilbert_rank(N, dH), fz.a1_terms(dA), fz.b0_terms(dB))
    assert F.info["kf"] == kf and F.info["r"] == r and F.info["r1"] == r1 == fz.theorem1_rank(N, eps)
    assert F.info["kprime"] == kf + r1 + r
    x = _x(N, b, 11)
    xd = torch.from_numpy(x.T.copy()).cuda()
    c = S.slepian_factor_compress(F, xd)
    y = S.slepian_factor_recover(F, c)
    torch.cuda.synchronize()
    c = c.cpu().numpy().astype(np.float64).T
    y = y.cpu().numpy().astype(np.float64).T
    x64 = x.astype(np.float64)
    cf = fz.fr_adjoint(x64, kf)
    for s in range(b):
        assert np.abs(c[:kf, s] - cf[:, s]).max() <= 1e-5 * np.linalg.norm(cf[:, s])
    cl = fac["L2"].T @ x64
    tol = (1e-5 * np.linalg.norm(fac["L2"], axis=0)[:, None] + 1e-30) * np.linalg.norm(x64, axis=0)[None, :]
    assert np.all(np.abs(c[kf:kf + r1] - cl) <= tol)
    cu = fac["U"].T @ x64
    assert np.abs(c[kf + r1:, :] - cu).max() <= 1e-5 * np.linalg.norm(x64, axis=0).max()
    ref = fz.recover(fac, fz.compress(fac, x64))
    err = max(np.linalg.norm(y[:, s] - ref[:, s]) / np.linalg.norm(ref[:, s]) for s in range(b))
    print(f"  r1={r1} (rH {F.info['r_h']}, rA {F.info['r_a']}, rB {F.info['r_b']}) round trip vs oracle {err:.2e}",
          flush=True)
    assert err <= 1e-5
    if N <= 4096:
        Pk = so.project_exact(N, W, x64)
        for s in range(b):
            assert np.linalg.norm(y[:, s] - Pk[:, s]) <= (2 * eps + 1e-6) * np.linalg.norm(x64[:, s])


@pytest.mark.parametrize("N,W,eps,prec", [(256, 1 / 8, 1e-6, "fp32"), (1024, 0.2, 1e-9, "fp32"),
                                          (1024, 1 / 16, 1e-6, "mixed"), (4096, 0.05, 1e-3, "fp32")])
def test_theorem1_factor_columns_match_oracle(N, W, eps, prec):
    """The setup's L2 (rows of T2 from compressing unit vectors) and L1
    (columns of T1 from recovering unit coefficients of the L part) equal
    the oracle's construction column by column."""
    P, F = _setup(N, W, eps, prec)
    L1, L2 = fz.theorem1_factor(N, W, eps)
    kf, r1, kp = F.info["kf"], F.info["r1"], F.info["kprime"]
    eye = torch.eye(N, device="cuda")
    T2 = S.slepian_factor_compress(F, eye).double().cpu().numpy()  # row n = T2^T e_n, i.e. row n of T2
    g2 = T2[:, kf:kf + r1]
    cu = torch.zeros((r1, kp), device="cuda")
    cu[:, kf:kf + r1] = torch.eye(r1, device="cuda")
    T1 = S.slepian_factor_recover(F, cu).double().cpu().numpy().T  # column j = L1[:, j]
    # column j enters T1 T2^T as L1[:, j] L2[:, j]^T, so each column is held to
    # 1e-5 of that term's norm; the highest sine-series columns of L2 fall
    # below the FP32 range (norms down to 1e-43 at eps = 1e-9) while their
    # terms are below 1e-40, hence the absolute floor
    cn1, cn2 = np.linalg.norm(L1, axis=0), np.linalg.norm(L2, axis=0)
    assert np.all(np.linalg.norm(g2 - L2, axis=0) * cn1 <= 1e-5 * cn1 * cn2 + 1e-20)
    assert np.all(np.linalg.norm(T1 - L1, axis=0) * cn2 <= 1e-5 * cn1 * cn2 + 1e-20)
    # the terms that matter are resolved to 1e-5 of their own size
    big = cn1 * cn2 > 1e-12
    assert np.all(np.linalg.norm(g2 - L2, axis=0)[big] <= 1e-5 * cn2[big])
    assert np.all(np.linalg.norm(T1 - L1, axis=0)[big] <= 1e-5 * cn1[big])


@pytest.mark.parametrize("N,W,eps,b,prec", CASES)
def test_eig_factorization_matches_oracle(N, W, eps, b, prec):
    print(f"eig factorization N={N} W={W} eps={eps} b={b} {prec}", flush=True)
    P, F = _setup(N, W, eps, prec, "eig")
    fac = _oracle(N, W, eps)
    kf, r = fac["kf"], fac["U"].shape[1]
    assert F.info["kf"] == kf and F.info["r"] == r
    _check_r1(F, fac, eps)
    r1 = F.info["r1"]
    assert F.info["kprime"] == kf + r1 + r
    assert F.info["mu_dropped"] <= eps
    assert F.info["ritz_residual"] <= 0.25 * eps
    # no eigenvalue above eps left outside the kept pairs' span
    assert 0 < F.info["deflated_norm"] <= eps
    print(f"  r1={F.info['r1']} subspace={F.info['subspace']} ritz residual {F.info['ritz_residual']:.2e} "
          f"deflated norm {F.info['deflated_norm']:.2e}", flush=True)
    n = min(r1, len(fac["mu"]))
    np.testing.assert_allclose(np.array(F.mu[:n]), fac["mu"][:n], rtol=0, atol=1e-9)

    x = _x(N, b, 11)
    xd = torch.from_numpy(x.T.copy()).cuda()
    c = S.slepian_factor_compress(F, xd)
    y = S.slepian_factor_recover(F, c)
    torch.cuda.synchronize()
    c = c.cpu().numpy().astype(np.float64).T
    y = y.cpu().numpy().astype(np.float64).T
    x64 = x.astype(np.float64)

    cf = fz.fr_adjoint(x64, kf)
    for s in range(b):
        assert np.abs(c[:kf, s] - cf[:, s]).max() <= 1e-5 * np.linalg.norm(cf[:, s])
    cu = fac["U"].T @ x64
    assert np.abs(c[kf + r1:, :] - cu).max() <= 1e-5 * np.linalg.norm(x64, axis=0).max()
    big = np.abs(fac["mu"][:n]) >= 1e-3
    cv = fac["V"][:, :n].T @ x64
    assert np.abs(c[kf:kf + n][big] - cv[big]).max() <= 1e-5 * np.linalg.norm(x64, axis=0).max()

    ref = fz.recover(fac, fz.compress(fac, x64))
    for s in range(b):
        assert np.linalg.norm(y[:, s] - ref[:, s]) <= 1e-5 * np.linalg.norm(ref[:, s])
    if N <= 4096:
        Pk = so.project_exact(N, W, x64)
        for s in range(b):
            assert np.linalg.norm(y[:, s] - Pk[:, s]) <= (2 * eps + 1e-6) * np.linalg.norm(x64[:, s])


@pytest.mark.parametrize("N,W,eps,prec", [(1024, 1 / 16, 1e-6, "fp32"), (16384, 1 / 8, 1e-6, "mixed")])
def test_recover_f_part_alone(N, W, eps, prec):
    """T1 on coefficients with only the F part set is F_r c_F (inverse bins path)."""
    P, F = _setup(N, W, eps, prec)
    kf, kp, b = F.info["kf"], F.info["kprime"], 5
    rng = np.random.default_rng(3)
    c = np.zeros((kp, b), dtype=np.float32)
    c[:kf] = rng.standard_normal((kf, b)).astype(np.float32)
    y = S.slepian_factor_recover(F, torch.from_numpy(c.T.copy()).cuda()).cpu().numpy().astype(np.float64).T
    ref = fz.fr_apply(c[:kf].astype(np.float64), N)
    for s in range(b):
        assert np.linalg.norm(y[:, s] - ref[:, s]) <= 1e-5 * np.linalg.norm(ref[:, s])


def test_strided_ragged_and_empty():
    """Leading dimensions above N and kprime, an odd batch (a lone signal in
    the last pair), batch 1, and batch 0 (no-op) agree with contiguous calls."""
    N, W, eps = 16384, 1 / 8, 1e-6
    P, F = _setup(N, W, eps, "mixed")
    kp = F.info["kprime"]
    x = torch.from_numpy(_x(N, 5, 4).T.copy()).cuda()
    c_ref = S.slepian_factor_compress(F, x)
    y_ref = S.slepian_factor_recover(F, c_ref)
    xs = torch.zeros((5, N + 40), device="cuda")
    xs[:, :N] = x
    cs = torch.full((5, kp + 24), 7.0, device="cuda")
    S.slepian_factor_compress(F, xs[:, :N], cs[:, :kp])
    ys = torch.full((5, N + 8), 3.0, device="cuda")
    S.slepian_factor_recover(F, cs[:, :kp], ys[:, :N])
    torch.cuda.synchronize()
    assert torch.equal(cs[:, :kp], c_ref) and torch.equal(ys[:, :N], y_ref)
    assert bool((cs[:, kp:] == 7.0).all()) and bool((ys[:, N:] == 3.0).all())
    c1 = S.slepian_factor_compress(F, x[4:5].contiguous())
    y1 = S.slepian_factor_recover(F, c1)
    torch.cuda.synchronize()
    assert torch.equal(c1[0], c_ref[4])
    assert torch.allclose(y1[0], y_ref[4], rtol=0, atol=1e-6 * float(y_ref[4].abs().max()))
    e = torch.empty((0, N), device="cuda")
    assert S.slepian_factor_compress(F, e).shape == (0, kp)


def test_factorization_errors():
    P = S.slepian_plan(1000, 1 / 16, 1e-6)  # N not a power of two
    with pytest.raises(S.SlepianError) as ei:
        S.slepian_factor_create(P)
    assert ei.value.status == S.SLEPIAN_ENOTSUP
    P2 = S.slepian_plan(128, 1 / 8, 1e-6)  # below the smallest row transform
    with pytest.raises(S.SlepianError) as ei:
        S.slepian_factor_create(P2)
    assert ei.value.status == S.SLEPIAN_ENOTSUP
    P3, F = _setup(1024, 1 / 16, 1e-6, "fp32")
    import ctypes as C
    h = C.c_void_p()
    assert S._lib.slepian_factor_create_ex(P3.handle, 7, C.byref(h)) == S.SLEPIAN_EINVAL
    mu = (C.c_double * 4)()
    assert S._lib.slepian_factor_mu(F.handle, mu, 4) == S.SLEPIAN_ENOTSUP
    x = torch.zeros((2, 1024), device="cuda")
    c = torch.zeros((2, F.info["kprime"]), device="cuda")
    lib = S._lib
    import ctypes as C
    # ldc below kprime, and c overlapping x
    assert lib.slepian_factor_compress(F.handle, S._ptr(x), 1024, S._ptr(c), F.info["kprime"] - 1, 2, None, 0,
                                       None) == S.SLEPIAN_EINVAL
    assert lib.slepian_factor_compress(F.handle, S._ptr(x), 1024, S._ptr(x), 1024, 1, None, 0,
                                       None) == S.SLEPIAN_EINVAL
    ws = C.c_size_t()
    assert lib.slepian_factor_workspace_size(F.handle, 4, C.byref(ws)) == S.SLEPIAN_OK and ws.value > 0


@pytest.mark.parametrize("method", ["theorem1", "eig"])
def test_factorization_random_configs(method):
    """Seeded random plans (N = 2^8 .. 2^14, W in [0.01, 0.45], eps in {1e-3,
    1e-6, 1e-9}, 1..9 signals, FP32 or mixed): kf and r1 equal the oracle's
    and the round trip matches the oracle's within 1e-5 per signal."""
    rng = np.random.default_rng(1611)
    for i in range(8):
        N = int(2 ** rng.integers(8, 15))
        W = float(rng.uniform(0.01, 0.45))
        eps = float(rng.choice([1e-3, 1e-6, 1e-9]))
        b = int(rng.integers(1, 10))
        prec = str(rng.choice(["fp32", "mixed"]))
        print(f"random factorization case {i} ({method}): N={N} W={W:.4f} eps={eps:g} b={b} {prec}", flush=True)
        P, F = _setup(N, W, eps, prec, method)
        fac = fz.fast_factorization(N, W, eps, method=method)
        assert F.info["kf"] == fac["kf"]
        if method == "eig":
            _check_r1(F, fac, eps)
        else:
            assert F.info["r1"] == fac["r1"]
        x = _x(N, b, 500 + i)
        y = S.slepian_factor_recover(F, S.slepian_factor_compress(F, torch.from_numpy(x.T.copy()).cuda()))
        y = y.cpu().numpy().astype(np.float64).T
        ref = fz.recover(fac, fz.compress(fac, x.astype(np.float64)))
        for s in range(b):
            assert np.linalg.norm(y[:, s] - ref[:, s]) <= 1e-5 * np.linalg.norm(ref[:, s])


def test_factorization_batch_slices():
    """A batch whose pair intermediate exceeds one 256 MiB slice (N = 2^18:
    64 pairs per slice; 130 signals = 65 pairs, so two slices, the second
    with one pair): signals on both sides of the slice boundary match the
    oracle's round trip, and the F part of the compression matches F_r^T x."""
    N, W, eps, b = 262144, 0.05, 1e-4, 130
    P, F = _setup(N, W, eps, "mixed")
    fac = _oracle(N, W, eps, "theorem1")
    x = synth.gaussian(N, b, 77)
    xd = x.cuda()
    c = S.slepian_factor_compress(F, xd)
    y = S.slepian_factor_recover(F, c)
    torch.cuda.synchronize()
    pick = [0, 1, 126, 127, 128, 129]
    xs = x[pick].double().numpy().T
    ref = fz.recover(fac, fz.compress(fac, xs))
    ys = y[pick].double().cpu().numpy().T
    cf = fz.fr_adjoint(xs, fac["kf"])
    cs = c[pick, :fac["kf"]].double().cpu().numpy().T
    for q in range(len(pick)):
        assert np.linalg.norm(ys[:, q] - ref[:, q]) <= 1e-5 * np.linalg.norm(ref[:, q])
        assert np.abs(cs[:, q] - cf[:, q]).max() <= 1e-5 * np.linalg.norm(cf[:, q])
