"""Shared helpers of the GPU tests: input marshalling and error metrics.

No arithmetic of the method lives here: inputs come from
paper_1309_1656_amd.synthetic, expected values from the oracle.
"""
import numpy as np
import torch

from oracle import pauli, qlbm
from paper_1309_1656_amd import mlbm, synthetic


def dims_of(shape):
    """Grid shape (y, x) or (z, y, x) -> library dims (nx, ny, nz)."""
    if len(shape) == 2:
        return (shape[1], shape[0], 1)
    return (shape[2], shape[1], shape[0])


def lattice_of(shape):
    return 9 if len(shape) == 2 else 19


def make_handle(shape, tau=0.8, beta0=1.0, storage=mlbm.MLBM_STORE_F64):
    return mlbm.mlbm_create(lattice_of(shape), dims_of(shape), tau, beta0, storage)


def device_inputs(h, fields):
    """(rho4, u, T) device tensors for mlbm_init_equilibrium; u = xi * u_lat with the library's xi."""
    rho4 = np.concatenate([fields["trrho"][None], fields["r"]])
    u = h.info["xi"] * fields["u_lat"]
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    return to(rho4), to(u), to(fields["T"])


def gpu_init(h, fields):
    W = h.empty_field()
    rho4, u, T = device_inputs(h, fields)
    mlbm.mlbm_init_equilibrium(h, W, rho4, u, T)
    return W


def oracle_init(shape, fields, beta0=1.0):
    lat = qlbm.Lattice(len(shape), beta0)
    W = qlbm.init_equilibrium(lat, fields["trrho"], fields["r"], lat.xi * fields["u_lat"], fields["T"])
    return lat, W


def to_pauli_np(h, t):
    """Library field -> float64 NumPy array [4, Q, *grid]."""
    return h.pauli_view(t.detach()).to(torch.float64).cpu().numpy()


def from_pauli(h, a):
    """[4, Q, *grid] values -> device field in the library layout and storage type."""
    return h.field_from_pauli(np.ascontiguousarray(a))


def oracle_pauli(W):
    """Oracle matrix field [Q, *grid, 2, 2] -> Pauli coefficients [4, Q, *grid]."""
    return pauli.pauli_from_matrix(W)


def normwise_rel_err(got, ref):
    """max over Pauli components k of max|got_k - ref_k| / max|ref_k|."""
    errs = []
    whole = np.abs(ref).max()
    for k in range(4):
        scale = np.abs(ref[k]).max()
        # a component that is zero throughout (e.g. no spin along x) is measured on the whole field's scale
        errs.append(np.abs(got[k] - ref[k]).max() / (scale if scale > 0 else whole))
    return max(errs)


def fields(shape, seed):
    return synthetic.macroscopic_fields(shape, seed)
