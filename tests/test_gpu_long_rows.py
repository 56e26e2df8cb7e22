"""Rows whose byte offsets pass 2^31.

The kernels address a cell within one row segment by a 32-bit unsigned byte
offset from a scalar segment start (x * sizeof(T), rows of at most 2^29
cells).  With FP64 storage a row longer than 2^28 cells puts offsets at and
above 2^31, where a signed reading of the offset would go wrong.  A D2Q9 grid
of one row of 2^28 + 2^16 + 3 cells (77.3 GB per FP64 field) is stepped by the
collide-only pass (out of place), then by the fused pull + collide pass, and
each is checked at sampled cells against the oracle; the sample holds the
cells on both sides of the 2^31 boundary, the ragged end and the periodic
wrap.  With room for a third field the adjoint step is checked the same way.
Inputs are smooth closed-form fields of the generic family (trace 1 +- 0.1,
|s| <= 0.3, |u| <= 0.05, T 1 +- 0.05), built on the device.
"""
import math

import numpy as np
import pytest
import torch

from helpers import make_handle, normwise_rel_err
from oracle import adjoint, pauli, qlbm
from paper_1309_1656_amd import mlbm

pytestmark = pytest.mark.gpu

NX = (1 << 28) + (1 << 16) + 3
SHAPE = (1, NX)
TAU = 0.8


def _log(msg):
    print(msg, flush=True)


def _inputs(h):
    x = torch.arange(NX, dtype=torch.float64, device="cuda") * (2.0 * math.pi / NX)
    tr = 1.0 + 0.1 * torch.sin(3.0 * x + 0.4)
    s = torch.stack([torch.sin(5.0 * x), torch.cos(7.0 * x + 0.3), torch.sin(2.0 * x + 1.1)])
    s = s * (0.3 / s.norm(dim=0).max())
    rho4 = torch.cat([tr[None], tr[None] * s]).reshape(4, *SHAPE).contiguous()
    u = torch.stack([0.05 * torch.cos(4.0 * x), 0.03 * torch.sin(6.0 * x + 0.2)]) * h.info["xi"]
    T = 1.0 + 0.05 * torch.cos(2.0 * x + 0.7)
    return rho4, u.reshape(2, *SHAPE).contiguous(), T.reshape(SHAPE).contiguous()


def _sample_x(n_random=256, seed=0):
    rng = np.random.default_rng(seed)
    b = 1 << 28                     # x * 8 = 2^31
    edges = np.concatenate([np.arange(0, 4), np.arange(b - 4, b + 4), np.arange(NX - 4, NX)])
    above = rng.integers(b, NX, 128)
    rand = rng.integers(0, NX, n_random)
    return np.unique(np.concatenate([edges, above, rand]))


def _gather(h, W, xs, ys=None):
    ys = np.zeros_like(xs) if ys is None else ys
    sel = h.pauli_view(W)[:, :, torch.from_numpy(ys).cuda(), torch.from_numpy(xs).cuda()]
    return sel.to(torch.float64).cpu().numpy()                                   # [4, Q, M]


def _collide_oracle(lat, a):
    return pauli.pauli_from_matrix(qlbm.collide(lat, pauli.matrix_from_pauli(a), TAU))


@pytest.fixture(scope="module")
def lattice():
    return qlbm.Lattice(2, 1.0)


def test_long_row_step_f64(lattice):
    torch.cuda.empty_cache()
    fb = 4 * 9 * NX * 8
    if torch.cuda.mem_get_info()[0] < 2 * fb + 16 * NX * 8:
        pytest.skip("needs two 77 GB fields")
    _log(f"long row D2Q9 F64 nx={NX}: init")
    h = make_handle(SHAPE, tau=TAU, storage=mlbm.MLBM_STORE_F64)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *_inputs(h))
    torch.cuda.empty_cache()
    g0, _ = mlbm.mlbm_moments(h, W)
    xs = _sample_x()
    before = _gather(h, W, xs)
    S = h.empty_field()
    _log("  collide-only pass, out of place")
    mlbm.mlbm_collide(h, W, S)
    err_c = normwise_rel_err(_gather(h, S, xs), _collide_oracle(lattice, before))
    # fused pass from the post-collision state: W(x) = collide(pull(S)(x)), pull(S)(x)_i = S(x - c_i)_i
    Q = lattice.Q
    nb = ((xs[:, None] - lattice.c[None, :, 0]) % NX).reshape(-1)
    pulled_all = _gather(h, S, nb).reshape(4, Q, xs.size, Q)
    pulled = np.diagonal(pulled_all, axis1=1, axis2=3).transpose(0, 2, 1)          # [4, Q, M]
    _log("  fused pull + collide pass")
    mlbm.mlbm_step_post(h, S, 1, dst=W, src_post=True)
    err_f = normwise_rel_err(_gather(h, W, xs), _collide_oracle(lattice, pulled))
    g1, nneg = mlbm.mlbm_moments(h, W)
    drift = float(np.abs(g1 - g0).max() / np.abs(g0).max())
    _log(f"  collide {err_c:.2e}, fused {err_f:.2e}, drift {drift:.2e}, n_neg {nneg}")
    assert err_c < 1e-13 and err_f < 1e-13
    assert drift < 1e-12 and nneg == 0
    del W, S, h
    torch.cuda.empty_cache()


def test_long_row_adjoint_f64(lattice):
    torch.cuda.empty_cache()
    fb = 4 * 9 * NX * 8
    if torch.cuda.mem_get_info()[0] < 3 * fb + 16 * NX * 8:
        pytest.skip("needs three 77 GB fields")
    _log(f"long row D2Q9 F64 adjoint nx={NX}")
    h = make_handle(SHAPE, tau=TAU, storage=mlbm.MLBM_STORE_F64)
    W = h.empty_field()
    mlbm.mlbm_init_equilibrium(h, W, *_inputs(h))
    torch.cuda.empty_cache()
    gen = torch.Generator(device="cuda").manual_seed(29)
    lam1 = torch.randn(h.field_shape, dtype=torch.float64, device="cuda", generator=gen)
    lam0 = h.empty_field()
    mlbm.mlbm_adjoint_step(h, W, lam1, lam0, None)
    xs = _sample_x(seed=1)
    Q = lattice.Q
    w_cells = _gather(h, W, xs)
    nb = ((xs[:, None] + lattice.c[None, :, 0]) % NX).reshape(-1)                  # lam_{n+1} at x + c_i
    g_all = _gather(h, lam1, nb).reshape(4, Q, xs.size, Q)
    g_cells = np.diagonal(g_all, axis1=1, axis2=3).transpose(0, 2, 1)
    Lc, _ = adjoint.collision_vjp(lattice, pauli.matrix_from_pauli(w_cells), pauli.matrix_from_pauli(2.0 * g_cells), TAU)
    err = normwise_rel_err(_gather(h, lam0, xs), pauli.pauli_from_matrix(Lc) / 2.0)
    _log(f"  lam_n at sampled cells {err:.2e}")
    assert err < 1e-12
    del W, lam1, lam0, h
    torch.cuda.empty_cache()
