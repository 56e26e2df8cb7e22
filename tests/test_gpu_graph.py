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


@pytest.mark.parametrize("shape,n", [((37, 70), 5), ((13, 9, 11), 4)])
def test_captured_checkpoint_segment_replay_bitwise(shape, n):
    """A checkpointed segment as the rollout runs it, captured once: mlbm_step_states keeping the
    states, then mlbm_adjoint_sweep over them (odd n adds its final device copy).  Every replay
    matches the eager calls bit for bit, dL/domega included."""
    print(f"graph segment {shape} n={n}", flush=True)
    h = make_handle(shape, tau=0.9, storage=mlbm.MLBM_STORE_F64)
    W0 = gpu_init(h, fields(shape, 14))
    rng = np.random.default_rng(3)
    lamN = torch.from_numpy(rng.standard_normal(tuple(W0.shape))).cuda()
    bufs = {}
    for tag in ("g", "e"):
        bufs[tag] = dict(out=h.empty_field(), lam=h.empty_field(), tmp=h.empty_field(),
                         states=torch.empty((n,) + tuple(W0.shape), dtype=W0.dtype, device="cuda"),
                         dom=torch.zeros(1, dtype=torch.float64, device="cuda"))

    def segment(b):
        b["lam"].copy_(lamN)
        b["dom"].zero_()
        mlbm.mlbm_step_states(h, W0, b["out"], b["states"], n, nstates=n)
        mlbm.mlbm_adjoint_sweep(h, W0, b["states"], n, b["lam"], b["tmp"], b["dom"])

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                         # warm-up (sizes the library's reduction buffer)
        segment(bufs["g"])
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        segment(bufs["g"])
    for rep in range(3):
        g.replay()
        segment(bufs["e"])
        torch.cuda.synchronize()
        for key in ("out", "lam", "states", "dom"):
            assert torch.equal(bufs["g"][key], bufs["e"][key]), (rep, key)


_FRESH_CAPTURE = r"""
import sys
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import torch
from helpers import fields, gpu_init, make_handle
from paper_1309_1656_amd import mlbm
shape = (13, 9, 130)
h = make_handle(shape, tau=0.9, storage=mlbm.MLBM_STORE_F64)
W0 = gpu_init(h, fields(shape, 12))
Wg, tg, We, te = W0.clone(), h.empty_field(), W0.clone(), h.empty_field()
torch.cuda.synchronize()
g = torch.cuda.CUDAGraph()
with torch.cuda.graph(g):              # the first step launch of this process happens under capture
    mlbm.mlbm_step(h, Wg, tg, 5)
for rep in range(3):
    g.replay()
    mlbm.mlbm_step(h, We, te, 5)
    torch.cuda.synchronize()
    assert torch.equal(Wg, We), rep
print("fresh capture ok")
"""


def test_first_launch_under_capture():
    """In a new process the first mlbm_step call may come inside a capture: the launch-shape set-up
    (occupancy queries for the LDS cap) enqueues nothing, so capture and replays still work."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, "-c", _FRESH_CAPTURE, root], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "fresh capture ok" in res.stdout
