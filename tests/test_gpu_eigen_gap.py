"""The eigenvalue-gap study (Section 1.2, Figure 1) on the GPU plans: the
number of eigenvalues of B in (eps, 1-eps) that a plan selects equals the
oracle's count (integer, exact), stays under Corollary 1's bound, and grows
with log N and log(1/eps - 1) like the asymptotic count.  Both sides decide
each eigenvalue's membership in FP64."""

import math

import pytest
import torch

from oracle import slepian_oracle as o

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1611_04950_amd import slepian as S

CASES = [(64, 0.25, 1e-3), (1024, 0.25, 1e-12), (4096, 0.25, 1e-9), (4096, 2.0 ** -8, 1e-6),
         (4096, 2.0 ** -10, 1e-12), (3000, 0.1, 1e-6)]


@pytest.mark.parametrize("N,W,eps", CASES)
def test_transition_count_matches_oracle(N, W, eps):
    P = S.slepian_plan(N, W, eps)
    r = P.info["r"]
    tp = o.transition_plan(N, W, eps, 1 - eps)
    assert r == tp["j1"] - tp["j0"]
    assert r <= o.cor1_bound(N, eps)
    print(f"N={N} W={W} eps={eps}: count {r}, asymptotic {o.asymptotic_count(N, eps):.1f}, "
          f"Corollary 1 bound {o.cor1_bound(N, eps):.0f}")


def test_count_grows_like_log_n_log_eps():
    """W = 1/4: the count at N = 2^14 minus the count at N = 2^8 is close to
    the asymptotic difference (2/pi^2) log(2^6) log(1/eps - 1), within a few
    eigenvalues, for eps = 1e-3 .. 1e-12."""
    for eps in (1e-3, 1e-6, 1e-9, 1e-12):
        r_lo = S.slepian_plan(1 << 8, 0.25, eps).info["r"]
        r_hi = S.slepian_plan(1 << 14, 0.25, eps).info["r"]
        d_asym = 2.0 / math.pi ** 2 * math.log(1 << 6) * math.log(1.0 / eps - 1.0)
        print(f"eps={eps}: counts {r_lo} (N=2^8), {r_hi} (N=2^14); asymptotic difference {d_asym:.1f}")
        assert abs((r_hi - r_lo) - d_asym) <= 4
