"""The allocation-free projection entry point against slepian_project,
called through the C ABI on the GPU: two calls in a row, the second with a
smaller input, each within 1e-5 relative of the allocating entry point's
result (Corollary 2's fast projection) and in practice bit for bit."""

import ctypes as C
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return ((torch.linalg.vector_norm((a - b).double(), dim=1) / torch.linalg.vector_norm(b.double(), dim=1))
            .max().item())


@pytest.mark.parametrize("N,W,eps,b1,b2,prec", [
    (65536, 1 / 8, 1e-6, 256, 37, 1),      # paper-scale batch, then a smaller odd one
    (262144, 0.05, 1e-4, 300, 64, 1),      # needs sub-batches of the fixed scratch
    (1024, 1 / 16, 1e-6, 8, 3, 0),         # single-pass plan with the FP32 correction
    (12000, 0.1, 1e-6, 20, 5, 0),          # generic (non power-of-two) size
])
def test_noalloc_matches_project(N, W, eps, b1, b2, prec):
    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth
    print(f"noalloc case N={N} W={W} eps={eps} b={b1},{b2} precision={prec}", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    plan = S.slepian_plan(N, W, eps, precision=prec)
    for b, seed in ((b1, 71), (b2, 72)):
        x = synth.gaussian(N, b, seed, device=dev)
        y_ref = S.slepian_project(plan, x)
        y = torch.full_like(x, float("nan"))
        S.slepian_project_noalloc(plan, x, y)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert _rel(y, y_ref) <= 1e-5
        print(f"  b={b}: max rel diff {_rel(y, y_ref):.2e}, bitwise equal {torch.equal(y, y_ref)}",
              file=sys.stderr, flush=True)


def test_noalloc_in_place_and_rejections():
    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth
    dev = torch.device("cuda:0")
    plan = S.slepian_plan(4096, 1 / 8, 1e-6)
    x = synth.gaussian(4096, 6, 5, device=dev)
    ref = S.slepian_project(plan, x)
    z = x.clone()
    S.slepian_project_noalloc(plan, z, z)
    torch.cuda.synchronize()
    assert _rel(z, ref) <= 1e-5
    lib = S._lib
    assert lib.slepian_project_noalloc(None, S._ptr(x), 4096, S._ptr(z), 4096, 6, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_project_noalloc(plan.handle, S._ptr(x), 4095, S._ptr(z), 4096, 6, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_project_noalloc(plan.handle, S._ptr(x), 4096, S._ptr(x[1:]), 4096, 5, None) == \
        S.SLEPIAN_EINVAL
    assert lib.slepian_project_noalloc(plan.handle, S._ptr(x), 4096, S._ptr(z), 4096, 0, None) == S.SLEPIAN_OK
