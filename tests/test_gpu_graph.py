"""mlbm_step under HIP graph capture (torch.cuda.CUDAGraph).

The step enqueues kernel launches only (no allocation, no memset, no host
synchronisation), so it can be captured once and replayed.  Every replay is
compared bit for bit with the same number of eager steps; replays are
separated by eager work of the program and synchronisations.
"""
import numpy as np
import pytest
import torch

from helpers import fields, gpu_init, make_handle
from paper_1309_1656_amd import mlbm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,storage,field", [((37, 70), mlbm.MLBM_STORE_F64, False),
                                                 ((13, 9, 11), mlbm.MLBM_STORE_F32, True),
                                                 ((2, 2048), mlbm.MLBM_STORE_F64, False)])
def test_captured_steps_replay_bitwise(shape, storage, field):
    print(f"graph {shape} storage={storage} field={field}", flush=True)
    h = make_handle(shape, tau=0.9, storage=storage)
    bmap = None
    if field:
        rng = np.random.default_rng(1)
        bmap = torch.from_numpy(rng.normal(0, 0.2, size=(3,) + shape)).cuda()
        mlbm.mlbm_set_magnetic_field_map(h, bmap)
    W0 = gpu_init(h, fields(shape, 12))
    k = 7
    Wg, tg = W0.clone(), h.empty_field()
    We, te = W0.clone(), h.empty_field()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                         # warm-up outside the capture
        tmp = W0.clone()
        mlbm.mlbm_step(h, tmp, h.empty_field(), 2)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mlbm.mlbm_step(h, Wg, tg, k)
    for rep in range(3):
        g.replay()
        mlbm.mlbm_step(h, We, te, k)                   # eager reference, same kernels
        junk = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(Wg, We), f"replay {rep}"
        assert torch.isfinite(junk)
