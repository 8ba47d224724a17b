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
