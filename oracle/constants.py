"""Closed-form constants of the lattice rules and of the polynomial equilibrium.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is evaluated with mpmath at 40 significant digits and rounded to
float64 only where the step uses it.

* Cubature weight parameter ``a`` and lattice length ``xi`` at mu0 = 0:
  Sec. 3.1, Eq. QuadSolution2Dmu0 (d = 2) and Eq. QuadSolution3Dmu0 (d = 3).
  The general-mu forms, Eqs. QuadSolution2D / QuadSolution3D, are provided
  too, so that a test can check that they reduce to the mu = 0 forms.
* Weights per velocity class: Eq. QuadSolution2D gives w00 = 1 - 5a,
  w01 = a, w11 = a/4; Eq. QuadSolution3D gives w000 = 1 - 12a, w001 = a,
  w011 = a/2.  The class of a velocity is its number of nonzero components.
* Polynomial-equilibrium coefficients alpha_1..alpha_5: Appendix, d = 2 and
  d = 3.  alpha_3, alpha_4, alpha_5 are constants; alpha_1 and alpha_2 are
  affine in b = beta0 * eps_FD.
"""
import mpmath as mp

mp.mp.dps = 40


def fd_integral_mp(k, x):
    """Complete Fermi-Dirac integral F_k(x) = -Li_{k+1}(-e^x) (Sec. 2.2), mpmath."""
    return mp.re(-mp.polylog(mp.mpf(k) + 1, -mp.exp(mp.mpf(x))))


def cubature_mu0(d, beta0=1):
    """(a, xi) of the Fermi-Dirac weighted cubature at mu0 = 0.

    d = 2: a = pi^4 / (972 zeta(3) log 2),  xi = (3/pi) sqrt(3 zeta(3)/beta0)
           (Eq. QuadSolution2Dmu0).
    d = 3: a = (41 + 9 sqrt2) zeta(5/2)^2 / (558 zeta(3/2) zeta(7/2)),
           xi = sqrt((3/beta0) (15 + 2 sqrt2) zeta(7/2) / (14 zeta(5/2)))
           (Eq. QuadSolution3Dmu0).
    """
    beta0 = mp.mpf(beta0)
    if d == 2:
        a = mp.pi ** 4 / (972 * mp.zeta(3) * mp.log(2))
        xi = (3 / mp.pi) * mp.sqrt(3 * mp.zeta(3) / beta0)
    elif d == 3:
        s2 = mp.sqrt(2)
        a = (41 + 9 * s2) * mp.zeta(mp.mpf(5) / 2) ** 2 / (
            558 * mp.zeta(mp.mpf(3) / 2) * mp.zeta(mp.mpf(7) / 2))
        xi = mp.sqrt((3 / beta0) * (15 + 2 * s2) * mp.zeta(mp.mpf(7) / 2)
                     / (14 * mp.zeta(mp.mpf(5) / 2)))
    else:
        raise ValueError("d must be 2 or 3")
    return a, xi


def cubature_general(d, beta, mu):
    """(a, xi) for a general chemical potential mu (Eqs. QuadSolution2D/3D)."""
    x = mp.mpf(beta) * mp.mpf(mu)
    F = lambda k: fd_integral_mp(k, x)
    if d == 2:
        a = F(1) ** 2 / (9 * F(0) * F(2))
        xi = mp.sqrt((3 / mp.mpf(beta)) * F(2) / F(1))
    elif d == 3:
        h = mp.mpf(1) / 2
        a = F(3 * h) ** 2 / (18 * F(h) * F(5 * h))
        xi = mp.sqrt((3 / mp.mpf(beta)) * F(5 * h) / F(3 * h))
    else:
        raise ValueError("d must be 2 or 3")
    return a, xi


def class_weights(d, a):
    """Weight of a velocity with 0, 1, 2 nonzero components (Eqs. QuadSolution2D/3D)."""
    if d == 2:
        return (1 - 5 * a, a, a / 4)
    if d == 3:
        return (1 - 12 * a, a, a / 2)
    raise ValueError("d must be 2 or 3")


def alpha_coefficients(d):
    """Appendix coefficients as a dict of mpf.

    Keys: 'fac' (alpha_fac), 'a1_0', 'a1_b' (alpha_1 = a1_0 + a1_b * b),
    'a2_0', 'a2_b' (alpha_2 = a2_0 + a2_b * b), 'a3', 'a4', 'a5',
    where b = beta0 * eps_FD.
    """
    if d == 2:
        z3 = mp.zeta(3)
        l2 = mp.log(2)
        p6 = mp.pi ** 2 / 6
        fac = 72 * l2 / (216 * l2 * z3 - mp.pi ** 4)
        return {
            "fac": fac,
            "a1_0": fac * 3 * z3, "a1_b": -fac * p6,
            "a2_0": -fac * p6, "a2_b": fac * 2 * l2,
            "a3": 12 * l2 / mp.pi ** 2,
            "a4": fac * l2,
            "a5": -fac * p6,
        }
    if d == 3:
        s2 = mp.sqrt(2)
        z32 = mp.zeta(mp.mpf(3) / 2)
        z52 = mp.zeta(mp.mpf(5) / 2)
        z72 = mp.zeta(mp.mpf(7) / 2)
        fac = 4 * z32 / (5 * (9 - 5 * s2) * z32 * z72 - 3 * (9 - 4 * s2) * z52 ** 2)
        return {
            "fac": fac,
            "a1_0": fac * mp.mpf(5) / 4 * (9 - 5 * s2) * z72,
            "a1_b": -fac * (5 - 3 * s2) * z52,
            "a2_0": -fac * (5 - 3 * s2) * z52,
            "a2_b": fac * (6 - 4 * s2) * z32 * mp.mpf(2) / 3,
            "a3": 2 * z32 / ((3 + s2) * z52),
            "a4": fac * (3 - 2 * s2) * z32,
            "a5": -fac * (5 - 3 * s2) * z52,
        }
    raise ValueError("d must be 2 or 3")


def as_float(d, beta0=1.0):
    """float64 copy of everything the step needs, for lattice dimension d."""
    a, xi = cubature_mu0(d, beta0)
    al = alpha_coefficients(d)
    out = {"a": float(a), "xi": float(xi),
           "class_w": tuple(float(w) for w in class_weights(d, a))}
    out.update({k: float(v) for k, v in al.items()})
    return out
