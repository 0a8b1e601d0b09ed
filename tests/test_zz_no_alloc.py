"""The no-allocation NDF tensor build (library-held scratch) against the
workspace build, through the C ABI, on two calls in a row (the second on a
smaller map), and the size limit refused on the host.  The direct build sums
each block with LDS atomics, so two builds agree to rounding, not bit for bit:
the bar is that of the tensor parity tests (1e-12 of the largest entry for
FP64, 1e-6 for FP32), with every entry written."""
import numpy as np
import pytest
import torch

import gen

pytestmark = pytest.mark.gpu

import paper_2109_14807_amd as G  # noqa: E402
from paper_2109_14807_amd import _lib as L  # noqa: E402


def _pair(nu, nv, nl, N, sigma, dtype, seed):
    nxy = torch.tensor(gen.flake_map(nu, nv, max(4, nu * nv // 40), 0.2, seed), device="cuda")
    d = G.desc_of(nu, nv, nl, N, sigma)
    want = torch.empty((nu, nv, nl, N, N), dtype=dtype, device="cuda")
    ws = torch.empty(L.glint_build_tensor_workspace(d), dtype=torch.uint8, device="cuda")
    L.glint_build_tensor(d, nxy, want, 0, ws)
    got = torch.full_like(want, float("nan"))
    L.glint_build_tensor_noalloc(d, nxy, got, 0)
    torch.cuda.synchronize()
    return got, want


def test_noalloc_build_equals_workspace_build_twice():
    cases = [(96, 80, 5, 32, 0.01, torch.float32, 1), (24, 40, 3, 16, 0.03, torch.float64, 2)]
    for nu, nv, nl, N, sigma, dtype, seed in cases:
        print(f"noalloc build {nu}x{nv} levels={nl} N={N} {dtype}", flush=True)
        got, want = _pair(nu, nv, nl, N, sigma, dtype, seed)
        assert not torch.isnan(got).any()
        tol = 1e-12 if dtype == torch.float64 else 1e-6
        err = float((got - want).abs().max()) / float(want.abs().max())
        assert err <= tol, err


def test_noalloc_build_refuses_maps_beyond_its_scratch():
    # 2048^2 texels need 2048^2 * (8 + 16 * 7) bytes of bin windows, above the limit
    d = G.desc_of(2048, 2048, 4, 64, 0.005)
    assert L.glint_build_tensor_workspace(d) > L.NOALLOC_SCRATCH_BYTES
    T = torch.empty(16, dtype=torch.float32, device="cuda")
    nxy = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(G.GlintError, match="scratch"):
        L.glint_build_tensor_noalloc(d, nxy, T, 0)
