"""The validation runs of Sec. 4 on the GPU, through the C ABI.

Each function sets up a handle and the initial state from the inputs in
`synthetic`, steps the field with mlbm_step and records observables with
mlbm_moments / mlbm_relaxation; all arithmetic runs in the library.

  riemann       D2Q9 2048 x 2, tau 10, 385 steps from two Fermi-Dirac halves
                (mlbm_init_chemical); returns tr rho, u, eps per cell.
  interference  D2Q9 128^2, tau 10, two colliding spin-polarised packets;
                records the energy split every step and keeps snapshots.
  convergence   D3Q19 32^3, tau 10, opposite spin domains; records the
                distances from the uniform equilibrium every `every` steps.
"""
import numpy as np

from . import mlbm, synthetic


def _dims(shape):
    return (shape[1], shape[0], 1) if len(shape) == 2 else (shape[2], shape[1], shape[0])


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _handle(wl, storage, tau=None):
    return mlbm.mlbm_create(wl["Q"], _dims(wl["shape"]), wl["tau"] if tau is None else tau, 1.0, storage)


def _init_from_fields(h, f):
    W = h.empty_field()
    rho4 = np.concatenate([f["trrho"][None], f["r"]])
    mlbm.mlbm_init_equilibrium(h, W, _dev(rho4), _dev(h.info["xi"] * f["u_lat"]), _dev(f["T"]))
    return W


def cell_moments(h, W):
    """(rho4 [4, *grid], u [d, *grid], eps [*grid]) as NumPy arrays."""
    import torch
    grid = h.grid
    rho4 = torch.empty((4,) + grid, dtype=torch.float64, device=W.device)
    u = torch.empty((h.info["d"],) + grid, dtype=torch.float64, device=W.device)
    eps = torch.empty(grid, dtype=torch.float64, device=W.device)
    mlbm.mlbm_moments(h, W, rho4, u, eps)
    return rho4.cpu().numpy(), u.cpu().numpy(), eps.cpu().numpy()


def riemann(storage=mlbm.MLBM_STORE_F64, steps=None):
    wl = synthetic.WORKLOADS["d2q9_riemann"]
    f = synthetic.riemann_fields(wl["shape"])
    h = _handle(wl, storage)
    W = h.empty_field()
    mlbm.mlbm_init_chemical(h, W, _dev(f["nu"]), _dev(h.info["xi"] * f["u_lat"]), _dev(f["T"]))
    mlbm.mlbm_step(h, W, h.empty_field(), wl["steps"] if steps is None else steps)
    rho4, u, eps = cell_moments(h, W)
    return {"handle": h, "W": W, "trrho": rho4[0], "u": u, "eps": eps}


def interference(storage=mlbm.MLBM_STORE_F64, steps=None, snapshots=(32, 54)):
    wl = synthetic.WORKLOADS["d2q9_interference"]
    h = _handle(wl, storage)
    W = _init_from_fields(h, synthetic.interference_fields(wl["shape"]))
    tmp = h.empty_field()
    steps = wl["steps"] if steps is None else steps
    hist = [mlbm.mlbm_relaxation(h, W)]
    snaps = {}
    for n in range(1, steps + 1):
        mlbm.mlbm_step(h, W, tmp, 1)
        hist.append(mlbm.mlbm_relaxation(h, W))
        if n in snapshots:
            snaps[n] = cell_moments(h, W)
    keys = mlbm.RELAXATION_KEYS
    return {"handle": h, "W": W, "history": {k: np.array([r[k] for r in hist]) for k in keys}, "snapshots": snaps}


def convergence(storage=mlbm.MLBM_STORE_F64, steps=None, every=10):
    wl = synthetic.WORKLOADS["d3q19_convergence"]
    h = _handle(wl, storage)
    W = _init_from_fields(h, synthetic.dichotomic_fields(wl["shape"]))
    tmp = h.empty_field()
    steps = wl["steps"] if steps is None else steps
    t, hist = [0], [mlbm.mlbm_relaxation(h, W)]
    n = 0
    while n < steps:
        k = min(every, steps - n)
        mlbm.mlbm_step(h, W, tmp, k)
        n += k
        t.append(n)
        hist.append(mlbm.mlbm_relaxation(h, W))
    keys = mlbm.RELAXATION_KEYS
    return {"handle": h, "W": W, "t": np.array(t), "history": {k: np.array([r[k] for r in hist]) for k in keys}}
