"""Seeded synthetic initial conditions shaped like the paper's 2D/3D runs.

This module only draws random macroscopic fields; it contains none of the
lattice Boltzmann arithmetic.  Both the library's callers and the CPU test
oracle take their inputs from here.

Smooth field recipe (one scalar field f on a periodic grid of shape n):
    f(x) = sum_{k in K} A_k cos(2 pi k.x / n + phi_k),
    K = { k in Z^d : 1 <= max|k_a| <= 3 }, one representative per +-k pair
        (first nonzero component positive), in lexicographic order of
        (k_x, k_y[, k_z]);
    A_k ~ N(0, 1) / |k|^2, phi_k ~ U[0, 2 pi), drawn as one vector of A's then
    one vector of phi's; then f <- f / max|f|.
The sum is evaluated exactly (up to rounding) through an inverse FFT.

Macroscopic fields (eight smooth fields f1..f8 drawn in this order):
    tr rho = 1 + 0.1 f1
    s      = 0.3 (f2, f3, f4) / max_x |(f2, f3, f4)|   (spin polarisation)
    r      = tr rho * s                                 (Bloch vector of rho)
    u_lat  = 0.05 (f5, f6[, f7]) / max_x |(...)|        (fraction of the
             lattice speed xi; multiply by the lattice constant xi to get the
             velocity in momentum units)
    T      = 1 + 0.05 f8                                (temperature, 1/beta)
"""
import itertools

import numpy as np

BASE_SEED = 13091656


def _modes(d):
    out = []
    for k in itertools.product(range(-3, 4), repeat=d):
        if max(abs(v) for v in k) < 1:
            continue
        first = next(v for v in k if v != 0)
        if first > 0:
            out.append(k)
    return out


def _spectrum(rng, shape):
    """Fourier coefficients {array index: complex} of one smooth field."""
    d = len(shape)
    ks = _modes(d)
    amp = rng.standard_normal(len(ks)) / np.array([float(sum(v * v for v in k)) for k in ks])
    phase = rng.uniform(0.0, 2.0 * np.pi, len(ks))
    ncell = int(np.prod(shape))
    coef = {}
    for k, A, ph in zip(ks, amp, phase):
        # k is (k_x, k_y[, k_z]); array axes are reversed (x fastest)
        idx = tuple(k[d - 1 - ax] % shape[ax] for ax in range(d))
        coef[idx] = coef.get(idx, 0.0) + ncell * A * np.exp(1j * ph)
    return coef


def smooth_field(rng, shape, device=None):
    """One normalised smooth periodic field on grid ``shape`` = (y, x) or (z, y, x).

    With ``device`` (a torch device) the inverse FFT runs there and a torch
    tensor is returned; the values equal the NumPy ones up to rounding.
    """
    coef = _spectrum(rng, shape)
    if device is None:
        spec = np.zeros(shape, dtype=np.complex128)
        for idx, c in coef.items():
            spec[idx] = c
        f = np.real(np.fft.ifftn(spec))
        return f / np.abs(f).max()
    import torch
    spec = torch.zeros(shape, dtype=torch.complex128, device=device)
    for idx, c in coef.items():
        spec[idx] = complex(c)
    f = torch.fft.ifftn(spec).real.contiguous()
    del spec
    return f / f.abs().max()


def _normalise_vec(v, amp):
    norm = (v ** 2).sum(axis=0).max() ** 0.5
    return v * (amp / norm)


def macroscopic_fields(shape, seed, device=None):
    """dict(trrho [*shape], r [3, *shape], u_lat [d, *shape], T [*shape], s [3, *shape]).

    float64 NumPy arrays, or torch tensors on ``device`` when given.
    """
    d = len(shape)
    rng = np.random.default_rng(np.random.PCG64(seed))
    f = [smooth_field(rng, shape, device) for _ in range(8)]
    stack = np.stack if device is None else __import__("torch").stack
    trrho = 1.0 + 0.1 * f[0]
    s = _normalise_vec(stack(f[1:4]), 0.3)
    u_lat = _normalise_vec(stack(f[4:4 + d]), 0.05)
    T = 1.0 + 0.05 * f[7]
    return {"trrho": trrho, "r": trrho[None] * s, "u_lat": u_lat, "T": T, "s": s}


def shear_band_fields(shape, seed):
    """2D smooth fields plus a periodic double shear band with a rotating spin.

    With n = ny, L = n/32 and the signed distance t = y - n/4 for y < n/2 and
    3n/4 - y otherwise (periodic, no jump at the wrap), the band profile is
    q(y) = tanh(t/L).  The x velocity gains 0.05 q(y) (lattice units) and the
    spin polarisation becomes the average of the generic field and a band
    spin 0.3 (0, sin th, cos th), th = (pi/4)(1 + q(y)), which turns from the
    z to the y direction across each band; |s| <= 0.3 still holds.
    """
    if len(shape) != 2:
        raise ValueError("the shear band is defined on 2D grids")
    base = macroscopic_fields(shape, seed)
    ny = shape[0]
    y = np.arange(ny, dtype=np.float64)
    t = np.where(y < ny / 2, y - ny / 4, 3 * ny / 4 - y)
    q = np.tanh(t / (ny / 32.0))[:, None] * np.ones(shape)
    th = 0.25 * np.pi * (1.0 + q)
    band = 0.3 * np.stack([np.zeros(shape), np.sin(th), np.cos(th)])
    s = 0.5 * (base["s"] + band)
    u_lat = base["u_lat"].copy()
    u_lat[0] += 0.05 * q
    trrho = base["trrho"]
    return {"trrho": trrho, "r": trrho[None] * s, "u_lat": u_lat, "T": base["T"], "s": s}


def target_bloch_field(shape, seed, amplitude=0.3):
    """Smooth target Bloch-vector field r_target [3, *shape] with max |r_target| = amplitude."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return _normalise_vec(np.stack([smooth_field(rng, shape) for _ in range(3)]), amplitude)


# Workloads: (lattice Q, grid shape, tau, steps).  The grid shape is (y, x) or (z, y, x).
def riemann_fields(shape=(2, 2048)):
    """Initial data of the Riemann problem of Sec. 4 on a quasi-1D periodic grid.

    Two equilibrated halves, separated at the middle of the x range (the
    membrane at x = 0; the periodic wrap is a second, mirrored membrane):
    left nu_up = -3/2, nu_dn = -5/2, right nu_up = -2, nu_dn = -3, with
    beta = 1, u = 0 and the spin axis +z on both sides.  Returns nu [2, *grid]
    (beta mu of the up and down channel), u_lat [2, *grid] and T [*grid].
    """
    nx = shape[-1]
    left = np.arange(nx) < nx // 2
    nu = np.empty((2,) + tuple(shape))
    nu[0] = np.where(left, -1.5, -2.0)
    nu[1] = np.where(left, -2.5, -3.0)
    return {"nu": nu, "u_lat": np.zeros((2,) + tuple(shape)), "T": np.ones(shape)}


def interference_fields(shape=(128, 128), sigma=6.0, amp=0.1, offset=18):
    """Two wavelet-shaped packets that collide (Sec. 4, interference).

    Packet 1 sits at (y, x) = (c - offset, c - offset), packet 2 at
    (c + offset, c - offset), c the grid centre.  Each carries a Ricker
    wavelet psi = (1 - r^2/sigma^2) exp(-r^2 / 2 sigma^2) of amplitude amp on
    tr rho = 1; packet 1 is spin-polarised along +z, packet 2 along +y (Bloch
    vector 0.3 tr rho times the Gaussian envelope); the velocity of a simple
    acoustic wave, u_lat = 0.8 (delta rho / rho) along (1, 1)/sqrt 2 for
    packet 1 and (1, -1)/sqrt 2 for packet 2, sends them toward each other.
    T = 1.  Deterministic: no seed.
    """
    ny, nx = shape
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    cy, cx = ny / 2.0, nx / 2.0
    packets = [((cy - offset, cx - offset), (1.0, 1.0), 2), ((cy + offset, cx - offset), (-1.0, 1.0), 1)]
    trrho = np.ones(shape)
    r = np.zeros((3,) + shape)
    u_lat = np.zeros((2,) + shape)
    bumps = []
    for (py, px), _, _ in packets:
        r2 = (y - py) ** 2 + (x - px) ** 2
        env = np.exp(-r2 / (2 * sigma ** 2))
        bumps.append((amp * (1 - r2 / sigma ** 2) * env, env))
        trrho += bumps[-1][0]
    for ((py, px), (dy, dx), comp), (dpsi, env) in zip(packets, bumps):
        r[comp] += 0.3 * trrho * env
        norm = np.hypot(dy, dx)
        u_lat[0] += 0.8 * dpsi / trrho * dx / norm      # x component
        u_lat[1] += 0.8 * dpsi / trrho * dy / norm      # y component
    return {"trrho": trrho, "r": r, "u_lat": u_lat, "T": np.ones(shape)}


def dichotomic_fields(shape=(32, 32, 32), amp=0.3):
    """Uniform tr rho with spin domains of opposite z polarisation (Sec. 4,
    convergence to equilibrium): r_z = amp tanh(4 sin(2 pi x/n) sin(2 pi y/n)
    sin(2 pi z/n)), a smooth two-valued outline; u_lat along x proportional to
    r_z with 0.05 at r_z = amp; T = 1.  Deterministic: no seed."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64) for n in shape), indexing="ij")
    s = np.sin(2 * np.pi * x / nx) * np.sin(2 * np.pi * y / ny) * np.sin(2 * np.pi * z / nz)
    rz = amp * np.tanh(4.0 * s)
    r = np.zeros((3,) + shape)
    r[2] = rz
    u_lat = np.zeros((3,) + shape)
    u_lat[0] = 0.05 * rz / amp
    return {"trrho": np.ones(shape), "r": r, "u_lat": u_lat, "T": np.ones(shape)}


WORKLOADS = {
    "d2q9_64": dict(Q=9, shape=(64, 64), tau=0.8, steps=100, seed=BASE_SEED + 1),
    "d2q9_1024_shear": dict(Q=9, shape=(1024, 1024), tau=0.6, steps=1000, seed=BASE_SEED + 2),
    "d3q19_128": dict(Q=19, shape=(128, 128, 128), tau=0.8, steps=500, seed=BASE_SEED + 3),
    "d3q19_384": dict(Q=19, shape=(384, 384, 384), tau=0.8, steps=200, seed=BASE_SEED + 4),
    "d3q19_64": dict(Q=19, shape=(64, 64, 64), tau=0.8, steps=200, seed=BASE_SEED + 4),
    "d2q9_512_adjoint": dict(Q=9, shape=(512, 512), tau=0.8, steps=200, seed=BASE_SEED + 5),
    "d2q9_16_adjoint": dict(Q=9, shape=(16, 16), tau=0.8, steps=10, seed=BASE_SEED + 5),
    # Sec. 4 validation workloads
    "d2q9_riemann": dict(Q=9, shape=(2, 2048), tau=10.0, steps=385, seed=None),
    "d2q9_interference": dict(Q=9, shape=(128, 128), tau=10.0, steps=54, seed=None),
    "d3q19_convergence": dict(Q=19, shape=(32, 32, 32), tau=10.0, steps=300, seed=None),
}
