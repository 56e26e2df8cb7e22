"""The quantum lattice Boltzmann step in matrix form, FP64, written from Sec. 3.3.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A field W has shape [Q, *grid, 2, 2] (complex128, Hermitian 2x2 per
population), grid axes (y, x) in 2D and (z, y, x) in 3D.  Time step Delta t = 1,
so the lattice spacing is Delta x = xi (Sec. 3.3, first paragraph) and a
population moving with e_i = xi c_i advances by c_i cells per step.

Per time step (Sec. 3.3, the three items):
  1. moments rho, u, eps of every cell by the cubature (Eq. DiscrAvr), with the
     weights already absorbed into W_i;
  2. W_eq_i = w_i rho P_i(u, eps) (Eq. WeqAlgo), P_i the quadratic polynomial
     with the Appendix coefficients and eps_FD := eps;
  3. BGK collision W_coll = W + (Delta t / tau)(W_eq - W) (Eq. CollisionStep);
  4. streaming W_i(x + Delta t e_i, t + Delta t) = W_coll_i(x, t)
     (Eq. TransportStep) on a periodic grid (Sec. 3, periodic conditions).
"""
import numpy as np

from . import constants, fermi, lattice
from .pauli import SIGMA, pauli_from_matrix


class Lattice:
    """Velocities e_i = xi c_i, weights w_i and polynomial coefficients.

    beta0 is the reference inverse temperature of the cubature; mu0 = 0
    (Sec. 3.1, paragraph after Eq. QuadSolution3Dmu0).
    """

    def __init__(self, d, beta0=1.0):
        if d not in (2, 3):
            raise ValueError("d must be 2 or 3")
        self.d = d
        self.beta0 = float(beta0)
        k = constants.as_float(d, beta0)
        self.c = lattice.velocities(d)
        self.Q = len(self.c)
        self.xi = k["xi"]
        self.e = self.xi * self.c.astype(np.float64)
        cls = lattice.velocity_class(self.c)
        self.w = np.array([k["class_w"][m] for m in cls], dtype=np.float64)
        self.coef = {n: k[n] for n in ("a1_0", "a1_b", "a2_0", "a2_b", "a3", "a4", "a5")}

    def grid_axis(self, comp):
        """Array axis of a field W (leading Q axis included) for velocity component comp."""
        return 1 + (self.d - 1 - comp)


def _bshape(v, ndim_after):
    return v.reshape(v.shape + (1,) * ndim_after)


def trace_real(W):
    """Re tr W_i for every population and cell: shape W.shape[:-2]."""
    return np.real(W[..., 0, 0] + W[..., 1, 1])


def moments(lat, W):
    """(rho, T, u, eps) of every cell, Eq. DiscrAvr.

    rho = sum_i W_i (2x2 per cell), T = tr rho,
    tr(rho) u = sum_i e_i tr W_i,
    tr(rho) eps = sum_i |e_i - u|^2 / 2 tr W_i.
    Shapes: rho [*grid, 2, 2], T [*grid], u [d, *grid], eps [*grid].
    """
    g = W.ndim - 3
    rho = W.sum(axis=0)
    trW = trace_real(W)
    T = trW.sum(axis=0)
    u = np.stack([(_bshape(lat.e[:, a], g) * trW).sum(axis=0) / T for a in range(lat.d)])
    dev2 = np.zeros_like(trW)
    for a in range(lat.d):
        dev2 += (_bshape(lat.e[:, a], g) - u[a][None]) ** 2
    eps = (0.5 * dev2 * trW).sum(axis=0) / T
    return rho, T, u, eps


def poly_factor(lat, u, eps):
    """P_i(u, eps), the scalar last factor of Eq. WeqAlgo; shape [Q, *grid].

    P_i = alpha1 + alpha2 beta0 |e_i|^2/2 + alpha3 beta0 (e_i.u)
          + alpha4 (beta0 e_i.u)^2 + alpha5 beta0 |u|^2/2,
    alpha1 = a1_0 + a1_b b, alpha2 = a2_0 + a2_b b, b = beta0 eps (Appendix).
    """
    g = u.ndim - 1
    k = lat.coef
    b0 = lat.beta0
    b = b0 * eps
    al1 = k["a1_0"] + k["a1_b"] * b
    al2 = k["a2_0"] + k["a2_b"] * b
    e2 = (lat.e ** 2).sum(axis=1)
    eu = sum(_bshape(lat.e[:, a], g) * u[a][None] for a in range(lat.d))
    u2 = (u ** 2).sum(axis=0)
    return (al1[None] + al2[None] * b0 * 0.5 * _bshape(e2, g) + k["a3"] * b0 * eu
            + k["a4"] * (b0 * eu) ** 2 + k["a5"] * b0 * 0.5 * u2[None])


def equilibrium(lat, rho, u, eps):
    """W_eq_i = w_i rho P_i (Eq. WeqAlgo); shape [Q, *grid, 2, 2]."""
    P = poly_factor(lat, u, eps)
    g = u.ndim - 1
    return _bshape(lat.w, g + 2) * P[..., None, None] * rho[None]


def collide(lat, W, tau, dt=1.0):
    """W_coll = W + (dt / tau)(W_eq - W), Eq. CollisionStep."""
    rho, T, u, eps = moments(lat, W)
    Weq = equilibrium(lat, rho, u, eps)
    return W + (dt / tau) * (Weq - W)


def stream(lat, W, sign=1):
    """Periodic transport by sign * c_i cells (Eq. TransportStep for sign = +1)."""
    out = np.empty_like(W)
    axes = tuple(lat.grid_axis(a) - 1 for a in range(lat.d))
    for i in range(lat.Q):
        shift = tuple(int(sign * lat.c[i, a]) for a in range(lat.d))
        out[i] = np.roll(W[i], shift=shift, axis=axes)
    return out


def step(lat, W, tau):
    """One time step: collision followed by streaming (Sec. 3.3)."""
    return stream(lat, collide(lat, W, tau))


def run(lat, W, tau, nsteps):
    for _ in range(nsteps):
        W = step(lat, W, tau)
    return W


def density_matrix(trrho, r):
    """rho = (tr(rho) I + r . sigma) / 2 from trace and Bloch vector r_k = tr(rho s_k)."""
    m = 0.5 * trrho[..., None, None] * SIGMA[0]
    for k in range(3):
        m = m + 0.5 * r[k][..., None, None] * SIGMA[k + 1]
    return m


def fd_parameters(d, trrho, r, T):
    """(beta, nu_up, nu_dn, eps) of the Fermi-Dirac state with density matrix rho.

    The eigenvalues of rho are n_up/dn = (tr rho +- |r|)/2 (the unitary U of
    Eq. WeqFD diagonalises rho); nu_s = beta mu_s solves
    n_s = (2 pi / beta)^(d/2) F_{d/2-1}(nu_s) (Eq. nFDstdOmega), and eps is
    Eq. energyFDstdOmega.
    """
    beta = 1.0 / T
    absr = np.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)
    n_up = 0.5 * (trrho + absr)
    n_dn = 0.5 * (trrho - absr)
    nu_up = fermi.chemical_potential_scaled(d, beta, n_up)
    nu_dn = fermi.chemical_potential_scaled(d, beta, n_dn)
    eps = fermi.internal_energy(d, beta, nu_up, nu_dn)
    return beta, nu_up, nu_dn, eps


def init_equilibrium(lat, trrho, r, u, T):
    """Discrete Fermi-Dirac equilibrium W_i = w_i rho P_i(u, eps_FD) per cell.

    Inputs per cell: tr rho > 0, Bloch vector r (|r| < tr rho), velocity u in
    the paper's momentum units, temperature T = 1 / beta > 0.  This is
    Eq. WeqDiscr with U diag(n_up, n_dn) U* = rho.
    """
    trrho = np.asarray(trrho, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    if np.any(~(trrho > 0)) or np.any(~(T > 0)):
        raise ValueError("tr rho and T must be positive")
    if np.any(~(np.sqrt((r ** 2).sum(axis=0)) < trrho)):
        raise ValueError("|r| must be below tr rho")
    _, _, _, eps = fd_parameters(lat.d, trrho, r, T)
    return equilibrium(lat, density_matrix(trrho, r), u, eps)


def init_chemical(lat, nu_up, nu_dn, u, T, axis=None):
    """Fermi-Dirac equilibrium named by the channels' chemical potentials.

    nu_s = beta mu_s per cell; the up channel is polarised along the unit
    vector `axis` ([3, *grid], default +z).  The channel densities are
    Eq. nFDstdOmega, rho = U diag(n_up, n_dn) U* with U turning z onto the axis,
    and eps is Eq. energyFDstdOmega (the Riemann problem of Sec. 4 starts from
    such states with u = 0 and beta = 1).
    """
    nu_up = np.asarray(nu_up, dtype=np.float64)
    nu_dn = np.asarray(nu_dn, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    if np.any(~(T > 0)):
        raise ValueError("T must be positive")
    beta = 1.0 / T
    n_up = fermi.channel_density(lat.d, beta, nu_up)
    n_dn = fermi.channel_density(lat.d, beta, nu_dn)
    if axis is None:
        axis = np.zeros((3,) + nu_up.shape)
        axis[2] = 1.0
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.sqrt((axis ** 2).sum(axis=0))
    # U diag(n_up, n_dn) U* = ((n_up + n_dn) I + (n_up - n_dn) axis . sigma) / 2
    rho = density_matrix(n_up + n_dn, (n_up - n_dn) * axis)
    eps = fermi.internal_energy(lat.d, beta, nu_up, nu_dn)
    return equilibrium(lat, rho, np.asarray(u, dtype=np.float64), eps)


def bloch(rho):
    """Bloch vector r_k = tr(rho s_k), k = 1..3 (Sec. 4, interference example)."""
    return pauli_from_matrix(rho)[1:]


def global_means(lat, W):
    """Global averages of Eqs. GlobalDensity, GlobalVelocity, GlobalTotalEnergy.

    Returns an 8-vector: Pauli coefficients of the mean density matrix (4),
    mean of tr(rho) u (3; zero third entry in 2D), mean of tr(rho) eps_tot.
    """
    ncell = W[0, ..., 0, 0].size
    g = W.ndim - 3
    trW = trace_real(W)
    rho_mean = pauli_from_matrix(W.sum(axis=0)).reshape(4, -1).sum(axis=1) / ncell
    mom = np.zeros(3)
    for a in range(lat.d):
        mom[a] = (_bshape(lat.e[:, a], g) * trW).sum() / ncell
    e2 = (lat.e ** 2).sum(axis=1)
    etot = (0.5 * _bshape(e2, g) * trW).sum() / ncell
    return np.concatenate([rho_mean, mom, [etot]])


def relaxation(lat, W):
    """Distances of every cell from the uniform state of the global averages
    (Eqs. GlobalDensity, GlobalVelocity, GlobalTotalEnergy; Sec. 4, convergence
    to equilibrium) and the global internal and kinetic energy (Sec. 4,
    interference).  Returns the 8 numbers: max over cells of the spectral norm
    of rho(x) - rho_bar, of |u(x) - u_bar| and of |eps_tot(x) - eps_tot_bar|;
    mean of tr rho eps and of tr rho |u|^2 / 2; root mean squares of the three
    distances.  rho_bar is the mean density matrix, u_bar = mean(tr rho u) /
    mean(tr rho), eps_tot_bar = mean(tr rho eps_tot) / mean(tr rho).
    """
    rho, T, u, eps = moments(lat, W)
    g = tuple(range(1, rho.ndim - 2 + 1))
    axes = tuple(range(rho.ndim - 2))
    rho_bar = rho.mean(axis=axes)
    Tm = T.mean()
    u_bar = (T[None] * u).mean(axis=tuple(range(1, u.ndim))) / Tm
    uu = (u ** 2).sum(axis=0)
    etot = eps + 0.5 * uu
    etot_bar = (T * etot).mean() / Tm
    drho = np.abs(np.linalg.eigvalsh(rho - rho_bar)).max(axis=-1)
    du = np.sqrt(((u - u_bar.reshape((-1,) + (1,) * (u.ndim - 1))) ** 2).sum(axis=0))
    de = np.abs(etot - etot_bar)
    return np.array([drho.max(), du.max(), de.max(), (T * eps).mean(), (0.5 * T * uu).mean(),
                     np.sqrt((drho ** 2).mean()), np.sqrt((du ** 2).mean()), np.sqrt((de ** 2).mean())])


def count_negative_eigenvalues(W):
    """Number of populations W_i(x) with a negative eigenvalue (Sec. 3.2, last paragraph)."""
    ev = np.linalg.eigvalsh(W)
    return int((ev[..., 0] < 0).sum())
