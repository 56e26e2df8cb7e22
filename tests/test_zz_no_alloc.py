"""mlbm_moments_noalloc (the entry point for callers that cannot allocate) against mlbm_moments.

Both run the same moment kernel and the same fixed-order reduction, so the per-cell outputs must be
equal bit for bit and the sums, divided by N as mlbm_moments divides them on the host, must equal
mlbm_moments' global averages bit for bit; the population counts must agree.  Two calls in a row, the
second on a smaller lattice (the library's buffer keeps the first call's contents), and replays of
the call captured in a HIP graph.
"""
import numpy as np
import pytest
import torch

from helpers import fields, gpu_init, make_handle
from paper_1309_1656_amd import mlbm

pytestmark = pytest.mark.gpu


def _perturbed_state(shape, seed, storage=mlbm.MLBM_STORE_F64):
    """A field with some negative-eigenvalue populations, so that every output is exercised."""
    h = make_handle(shape, storage=storage)
    W = gpu_init(h, fields(shape, seed))
    gen = torch.Generator(device="cuda").manual_seed(seed)
    # FP16 deviation storage holds (a - R_ki) / s_i: the same relative push needs a larger step there
    amp = 2.0 if storage == mlbm.MLBM_STORE_F16DEV else 0.02
    W.add_(amp * torch.randn(W.shape, dtype=torch.float64, device="cuda", generator=gen).to(W.dtype))
    return h, W


def _outputs(h, W, noalloc):
    d, grid = h.info["d"], tuple(h.grid)
    rho4 = torch.full((4,) + grid, float("nan"), dtype=torch.float64, device="cuda")
    u = torch.full((d,) + grid, float("nan"), dtype=torch.float64, device="cuda")
    eps = torch.full(grid, float("nan"), dtype=torch.float64, device="cuda")
    if noalloc:
        sums = torch.full((10,), float("nan"), dtype=torch.float64, device="cuda")
        mlbm.mlbm_moments_noalloc(h, W, rho4, u, eps, sums)
        torch.cuda.synchronize()
        s = sums.cpu().numpy()
        g8 = s[:8] * (1.0 / h.info["ncell"])
        return rho4, u, eps, g8, int(s[8]), int(s[9])
    g8, nneg = mlbm.mlbm_moments(h, W, rho4, u, eps)
    return rho4, u, eps, g8, nneg, 0


@pytest.mark.parametrize("storage", [mlbm.MLBM_STORE_F64, mlbm.MLBM_STORE_F32, mlbm.MLBM_STORE_F16DEV])
def test_noalloc_equals_moments_twice(storage):
    for shape, seed in (((13, 9, 130), 3), ((5, 6, 7), 4)):       # the second call on a smaller lattice
        print(f"noalloc moments {shape} storage={storage}", flush=True)
        h, W = _perturbed_state(shape, seed, storage)
        a = _outputs(h, W, noalloc=True)
        b = _outputs(h, W, noalloc=False)
        for x, y in zip(a[:3], b[:3]):
            assert torch.equal(x, y)
        assert np.array_equal(a[3], b[3])
        assert a[4] == b[4]
        assert a[4] > 0 or storage == mlbm.MLBM_STORE_F16DEV
        assert a[5] == 0


def test_noalloc_in_graph_replays():
    """Captured once, replayed three times on a changing field with eager work in between: every
    replay equals an eager call."""
    shape = (37, 70)
    h, W = _perturbed_state(shape, 5)
    sums = torch.zeros(10, dtype=torch.float64, device="cuda")
    rho4 = torch.zeros((4,) + shape, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mlbm.mlbm_moments_noalloc(h, W, rho4, None, None, sums)      # first call on the device: address lookup
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mlbm.mlbm_moments_noalloc(h, W, rho4, None, None, sums)
    scratch = h.empty_field()
    for rep in range(3):
        mlbm.mlbm_step(h, W, scratch, 2)                              # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got_rho, got_sums = rho4.clone(), sums.clone()
        ref_rho = torch.empty_like(rho4)
        ref_sums = torch.empty_like(sums)
        mlbm.mlbm_moments_noalloc(h, W, ref_rho, None, None, ref_sums)
        torch.cuda.synchronize()
        assert torch.equal(got_rho, ref_rho), rep
        assert torch.equal(got_sums, ref_sums), rep
