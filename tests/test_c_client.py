"""The C ABI used from plain C (tests/c_abi_demo.c, built by build()): no
Python in the loop.  CPU: the client is built and linked against the in-tree
libmlbm.so.  GPU: its global averages equal the binding's on the same inputs
(to the rounding of the host sine), match the oracle's initial state, and are
conserved by the steps.
"""
import os
import subprocess

import numpy as np
import pytest

from paper_1309_1656_amd import build, mlbm

DIMS = (24, 20, 16)
STEPS = 5


def test_client_is_built_against_the_package_library():
    assert os.path.exists(build.C_DEMO), "run build() first"
    out = subprocess.run(["ldd", build.C_DEMO], capture_output=True, text=True).stdout
    line = [ln for ln in out.splitlines() if "libmlbm.so" in ln]
    assert line and os.path.dirname(build.LIB) in line[0]


def _inputs(xi):
    """The client's input fields, in the same order (rho4, u, T) and cell order."""
    nx, ny, nz = DIMS
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sx, sy, sz = 2 * np.pi * x / nx, 2 * np.pi * y / ny, 2 * np.pi * z / nz
    rho4 = np.stack([1.0 + 0.05 * np.sin(sx) * np.cos(sy), 0.1 * np.sin(sz), np.full(x.shape, 0.05),
                     0.1 * np.cos(sx)])
    u = xi * 0.02 * np.stack([np.sin(sy), np.cos(sz), np.sin(sx)])
    T = 1.0 + 0.02 * np.cos(sx + sy + sz)
    return rho4, u, T


@pytest.mark.gpu
def test_client_matches_binding_and_oracle():
    import torch
    from oracle import qlbm
    print("c client", flush=True)
    res = subprocess.run([build.C_DEMO, *map(str, DIMS), str(STEPS)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    lines = {ln.split()[0]: ln.split()[1:] for ln in res.stdout.splitlines()}
    g0 = np.array([float(v) for v in lines["global0"]])
    g1 = np.array([float(v) for v in lines["global1"]])
    assert int(lines["nneg"][0]) == 0
    # the binding on the same inputs
    h = mlbm.mlbm_create(19, DIMS, 0.8, 1.0, mlbm.MLBM_STORE_F64)
    rho4, u, T = _inputs(h.info["xi"])
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, to(rho4), to(u), to(T))
    b0, _ = mlbm.mlbm_moments(h, W)
    mlbm.mlbm_step(h, W, h.empty_field(), STEPS)
    b1, _ = mlbm.mlbm_moments(h, W)
    # the inputs agree to the last bit of the host sine (libm against NumPy)
    scale = np.max(np.abs(b0))
    assert np.max(np.abs(g0 - b0)) < 1e-15 * scale and np.max(np.abs(g1 - b1)) < 1e-15 * scale
    # the oracle's initial state, and conservation
    lat = qlbm.Lattice(3)
    Wo = qlbm.init_equilibrium(lat, rho4[0], rho4[1:], u, T)
    go = qlbm.global_means(lat, Wo)
    assert np.max(np.abs(g0 - go)) < 1e-13 * np.max(np.abs(go))
    assert np.max(np.abs(g1 - g0)) < 1e-13 * np.max(np.abs(g0))
