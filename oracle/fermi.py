"""Complete Fermi-Dirac integrals and the density -> chemical-potential inversion.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2 defines F_k(x) = Gamma(k+1)^-1 int_0^inf y^k / (e^(y-x) + 1) dy,
states F_k(x) = -Li_{k+1}(-e^x), dF_k/dx = F_{k-1}, and the per-spin-channel
density n_{d,beta,mu} = (2 pi / beta)^(d/2) F_{d/2-1}(beta mu)
(Eq. nFDstdOmega) and internal energy
eps_FD = (d/2) beta^-1 sum_s F_{d/2}(nu_s) / sum_s F_{d/2-1}(nu_s)
(Eq. energyFDstdOmega), with nu_s = beta mu_s.

For x < 0 the polylogarithm series gives
    F_k(x) = sum_{j>=1} (-1)^(j+1) e^(j x) / j^(k+1),
which this module sums with 120 terms where x <= -1/2 (the tail is below
e^-60).  Elsewhere it falls back to mpmath's polylogarithm, element by element.
"""
import math

import mpmath as mp
import numpy as np

_NTERMS = 120
_SERIES_XMAX = -0.5


def _series(k, x):
    # sum_j (-1)^(j+1) e^(j x) / j^(k+1), accumulated from the smallest term up
    acc = np.zeros_like(x)
    for j in range(_NTERMS, 0, -1):
        sign = 1.0 if j % 2 == 1 else -1.0
        acc += (sign / float(j) ** (k + 1.0)) * np.exp(j * x)
    return acc


def fd(k, x):
    """F_k(x) elementwise, float64 (k may be an integer or a half-integer)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lo = x <= _SERIES_XMAX
    if lo.any():
        out[lo] = _series(k, x[lo])
    if (~lo).any():
        hi_vals = [float(mp.re(-mp.polylog(k + 1, -mp.exp(mp.mpf(float(v))))))
                   for v in x[~lo].ravel()]
        out[~lo] = np.array(hi_vals, dtype=np.float64).reshape(x[~lo].shape)
    return out


def invert_density(k, c, tol=1e-15, maxit=60):
    """Solve F_k(nu) = c for nu elementwise (c > 0) by Newton's method.

    F_k is increasing and convex in nu (its derivatives are F_{k-1} > 0 and
    F_{k-2} > 0), so Newton converges from either side of the root.  The start
    is the classical (non-degenerate) limit F_k(nu) ~ e^nu, i.e. nu0 = log c,
    or the degenerate limit F_k(nu) ~ nu^(k+1) / Gamma(k+2) when c > 1.
    """
    c = np.asarray(c, dtype=np.float64)
    if np.any(~(c > 0)):
        raise ValueError("density must be positive")
    g = math.gamma(k + 2.0)
    nu = np.where(c < 1.0, np.log(c), (c * g) ** (1.0 / (k + 1.0)))
    for _ in range(maxit):
        step = (fd(k, nu) - c) / fd(k - 1, nu)
        nu = nu - step
        if np.all(np.abs(step) <= tol * np.maximum(1.0, np.abs(nu))):
            return nu
    raise RuntimeError("Fermi-Dirac inversion did not converge")


def channel_density(d, beta, nu):
    """n_{d,beta,mu} = (2 pi / beta)^(d/2) F_{d/2-1}(nu), nu = beta mu (Eq. nFDstdOmega)."""
    return (2.0 * np.pi / beta) ** (d / 2.0) * fd(d / 2.0 - 1.0, nu)


def internal_energy(d, beta, nu_up, nu_dn):
    """eps_FD of Eq. energyFDstdOmega for the two spin channels."""
    num = fd(d / 2.0, nu_up) + fd(d / 2.0, nu_dn)
    den = fd(d / 2.0 - 1.0, nu_up) + fd(d / 2.0 - 1.0, nu_dn)
    return (d / 2.0) / beta * num / den


def chemical_potential_scaled(d, beta, n):
    """nu = beta mu such that n_{d,beta,mu} = n (inverse of Eq. nFDstdOmega)."""
    return invert_density(d / 2.0 - 1.0, n * (beta / (2.0 * np.pi)) ** (d / 2.0))
