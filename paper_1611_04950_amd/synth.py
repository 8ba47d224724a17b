"""Seeded synthetic signals for tests and benchmarks.

This module only draws inputs; it holds none of the transform's arithmetic and
is shared by the GPU tests, the benchmark and the oracle-side checks, which all
receive the same arrays.  Signals are generated in float64 and rounded to
float32 once, so both sides see identical float32 samples.

Layout: a batch of b signals of length N is a (b, N) tensor, each signal
contiguous (column-major N x b with leading dimension N in BLAS terms).

Recipes (the paper uses random vectors of unstated distribution, Section 4.1):
  gaussian   i.i.d. N(0, 1) samples, signal s drawn from seed base + s.
  sinusoids  x[n] = sum_k a_k cos(2 pi f_k n + phi_k), a_k ~ N(0, 1),
             f_k ~ U[-W, W], phi_k ~ U[0, 2 pi), plus white Gaussian noise
             with variance mean(x^2) / 10^(snr_db / 10) (per signal).
"""

from __future__ import annotations

import math

import numpy as np
import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def gaussian(N: int, b: int, seed_base: int, device="cpu", dtype=torch.float32) -> torch.Tensor:
    out = torch.empty((b, N), dtype=dtype, device=device)
    for s in range(b):
        g = _gen(seed_base + s, device)
        out[s] = torch.randn(N, generator=g, dtype=torch.float64, device=device).to(dtype)
    return out


def sinusoids(N: int, b: int, W: float, n_tones: int, snr_db: float, seed_base: int,
              device="cpu", dtype=torch.float32, chunk: int = 1 << 16) -> torch.Tensor:
    out = torch.empty((b, N), dtype=dtype, device=device)
    for s in range(b):
        gp = _gen(seed_base + s, "cpu")
        a = torch.randn(n_tones, generator=gp, dtype=torch.float64)
        f = (torch.rand(n_tones, generator=gp, dtype=torch.float64) * 2.0 - 1.0) * W
        ph = torch.rand(n_tones, generator=gp, dtype=torch.float64) * (2.0 * math.pi)
        a, f, ph = a.to(device), f.to(device), ph.to(device)
        sig = torch.empty(N, dtype=torch.float64, device=device)
        for n0 in range(0, N, chunk):
            n = torch.arange(n0, min(N, n0 + chunk), dtype=torch.float64, device=device)
            sig[n0:n0 + n.numel()] = torch.cos(2.0 * math.pi * f[None, :] * n[:, None] + ph[None, :]) @ a
        p = float((sig * sig).mean())
        sigma = math.sqrt(p / 10.0 ** (snr_db / 10.0))
        gn = _gen(seed_base + s + 7919, device)
        sig += sigma * torch.randn(N, generator=gn, dtype=torch.float64, device=device)
        out[s] = sig.to(dtype)
    return out


def config_signals(cfg: int, N: int, b: int, W: float, device="cpu") -> torch.Tensor:
    """Signals for the five workloads: 1 and 4 Gaussian; 2 and 3 sixty-four
    tones at 20 dB SNR; 5 two hundred tones at 10 dB SNR."""
    base = 1000 * cfg
    if cfg in (1, 4):
        return gaussian(N, b, base, device)
    if cfg in (2, 3):
        return sinusoids(N, b, W, 64, 20.0, base, device)
    if cfg == 5:
        return sinusoids(N, b, W, 200, 10.0, base, device)
    raise ValueError(cfg)


def batching_plans(n_plans: int = 512, seed: int = 4000):
    """Plan parameters of the many-plans workload: N log-uniform over
    2^10..2^17 (rounded to an integer), W uniform in [0.01, 0.25], eps drawn
    from {1e-3, 1e-6}, 4..64 signals per plan (uniform).  Returns a list of
    (N, W, eps, b) tuples; the signals of plan i are gaussian(N, b, seed *
    1000 + 100 * i)."""
    g = _gen(seed, "cpu")
    logn = torch.rand(n_plans, generator=g, dtype=torch.float64) * 7.0 + 10.0
    w = torch.rand(n_plans, generator=g, dtype=torch.float64) * 0.24 + 0.01
    e = torch.randint(0, 2, (n_plans,), generator=g)
    nb = torch.randint(4, 65, (n_plans,), generator=g)
    out = []
    for i in range(n_plans):
        N = int(round(2.0 ** float(logn[i])))
        out.append((N, float(w[i]), 1e-3 if int(e[i]) == 0 else 1e-6, int(nb[i])))
    return out


# ---------------------------------------------------------------------------
# Fourier extension (the least-squares application of Section 1.4 and its
# experiment in Section 4.2): a function on [-1, 1], the right-hand side
# F y of the normal equations F F^* g = F y (F F^* = B with N = 2M + 1 and
# W = 1/(2T)), and the evaluation of a coefficient vector as a 2T-periodic
# series.  Input preparation and error measurement on the host in FP64; the
# solve itself is the library's (slepian_lsq).
# ---------------------------------------------------------------------------

def fe_function(n_terms: int = 500, a0: float = 5.0, seed: int = 7000) -> dict:
    """f(t) = a0 t + sum_l a_l exp(-|t - mu_l| / sigma_l): continuous, not
    smooth, f(-1) != f(1).  The paper draws a_l, mu_l, sigma_l "in a random
    manner"; here a_l ~ U[-1, 1], mu_l ~ U[-1, 1], sigma_l ~ U[0.01, 0.2]."""
    g = np.random.default_rng(seed)
    return {"a0": a0, "a": g.uniform(-1.0, 1.0, n_terms), "mu": g.uniform(-1.0, 1.0, n_terms),
            "sigma": g.uniform(0.01, 0.2, n_terms)}


def fe_eval(fp: dict, t: np.ndarray, device="cpu", chunk: int = 1 << 15) -> np.ndarray:
    """f at the points t (FP64; the sum over the terms runs in torch on
    `device`, chunked)."""
    t = np.asarray(t, dtype=np.float64)
    a = torch.as_tensor(fp["a"], dtype=torch.float64, device=device)
    mu = torch.as_tensor(fp["mu"], dtype=torch.float64, device=device)
    sg = torch.as_tensor(fp["sigma"], dtype=torch.float64, device=device)
    out = np.empty_like(t)
    for i in range(0, t.size, chunk):
        tt = torch.as_tensor(t[i:i + chunk], dtype=torch.float64, device=device)
        v = fp["a0"] * tt + torch.exp(-torch.abs(tt[:, None] - mu[None, :]) / sg[None, :]) @ a
        out[i:i + chunk] = v.cpu().numpy()
    return out


def fe_grid(M: int) -> int:
    """Quadrature length 2^(13 + floor(log2 M)) (the experiment's choice)."""
    return 1 << (13 + int(math.floor(math.log2(max(M, 1)))))


def _fe_samples(fp, T: float, Q: int, device="cpu"):
    t = -T + 2.0 * T * np.arange(Q) / Q
    inside = np.abs(t) <= 1.0
    f = np.zeros(Q)
    f[inside] = fp(t[inside]) if callable(fp) else fe_eval(fp, t[inside], device)
    return t, inside, f


def fe_coefficients(fp, M: int, T: float, Q: int | None = None, device="cpu") -> np.ndarray:
    """c_n = (1/sqrt(2T)) int_{-1}^{1} f(t) exp(-i n pi t / T) dt, n = -M..M
    (f: fe_function's parameters, or any real function of a numpy array),
    by the Q-point rectangle rule on the grid t_k = -T + 2Tk/Q of [-T, T)
    (f set to zero outside [-1, 1]), i.e. one length-Q FFT."""
    Q = fe_grid(M) if Q is None else Q
    _, _, f = _fe_samples(fp, T, Q, device)
    F = np.fft.fft(f)
    n = np.arange(-M, M + 1)
    return (2.0 * T / Q) / math.sqrt(2.0 * T) * ((-1.0) ** np.abs(n)) * F[n % Q]


def fe_series(c: np.ndarray, T: float, Q: int) -> np.ndarray:
    """g(t_k) = (1/sqrt(2T)) sum_n c_n exp(i n pi t_k / T) on the grid
    t_k = -T + 2Tk/Q, by one length-Q inverse FFT."""
    M = (len(c) - 1) // 2
    n = np.arange(-M, M + 1)
    A = np.zeros(Q, dtype=np.complex128)
    A[n % Q] = c * ((-1.0) ** np.abs(n))
    return Q * np.fft.ifft(A) / math.sqrt(2.0 * T)


def fe_rel_rms(fp, c: np.ndarray, T: float, Q: int | None = None, device="cpu") -> float:
    """||f - g||_{L2[-1,1]} / ||f||_{L2[-1,1]} on the uniform grid of [-T, T)
    restricted to [-1, 1]."""
    M = (len(c) - 1) // 2
    Q = fe_grid(M) if Q is None else Q
    _, inside, f = _fe_samples(fp, T, Q, device)
    g = fe_series(c, T, Q)
    return float(np.linalg.norm(f[inside] - g[inside]) / np.linalg.norm(f[inside]))
