"""Exact solution of the Riemann problem for the Euler equations of Eq. Euler.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2 shows that near equilibrium the moments obey the classical Euler
equations with mass density tr rho, velocity u and pressure
P = (2/d) tr rho eps, i.e. an ideal polytropic gas with gamma = 1 + 2/d.
Sec. 4 validates the scheme on a Riemann problem against the analytic solution
of these equations (a textbook result the paper cites), which is a function
of x / t only.  It is computed here in one space dimension:

* the star-region pressure p* solves f_L(p) + f_R(p) + u_R - u_L = 0, where
  f_K is the velocity jump across the wave facing state K: the Hugoniot
  (shock) branch for p > p_K, the isentropic (rarefaction) branch for
  p <= p_K; f is increasing and concave, so Newton's method from below
  converges;
* u* = (u_L + u_R + f_R(p*) - f_L(p*)) / 2, the contact speed;
* the density on each side of the contact follows from the Hugoniot relation
  or the isentrope, shock speeds from mass conservation, rarefaction fans
  from the characteristic u -/+ c = x / t with a constant Riemann invariant.
"""
import numpy as np


def sound_speed(gamma, rho, p):
    return np.sqrt(gamma * p / rho)


def _wave_jump(gamma, p, rho_k, p_k):
    """f_K(p) and its derivative for the wave facing state K."""
    c_k = sound_speed(gamma, rho_k, p_k)
    if p > p_k:
        a = 2.0 / ((gamma + 1.0) * rho_k)
        b = (gamma - 1.0) / (gamma + 1.0) * p_k
        root = np.sqrt(a / (p + b))
        return (p - p_k) * root, root * (1.0 - 0.5 * (p - p_k) / (p + b))
    e = (gamma - 1.0) / (2.0 * gamma)
    f = 2.0 * c_k / (gamma - 1.0) * ((p / p_k) ** e - 1.0)
    df = (p / p_k) ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho_k * c_k)
    return f, df


def star_state(gamma, left, right, tol=1e-15, maxit=100):
    """(p*, u*) between the two waves; left and right are (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = sound_speed(gamma, rl, pl), sound_speed(gamma, rr, pr)
    if 2.0 * (cl + cr) / (gamma - 1.0) <= ur - ul:
        raise ValueError("the initial data create a vacuum")
    e = (gamma - 1.0) / (2.0 * gamma)
    p = min(pl, pr)
    if _wave_jump(gamma, p, rl, pl)[0] + _wave_jump(gamma, p, rr, pr)[0] + ur - ul >= 0.0:
        # p* <= min(p_L, p_R): two rarefactions, closed form
        p = ((cl + cr - 0.5 * (gamma - 1.0) * (ur - ul)) / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    else:
        # f is increasing and concave: Newton from below stays below and rises monotonically
        for _ in range(maxit):
            fl, dl = _wave_jump(gamma, p, rl, pl)
            fr, dr = _wave_jump(gamma, p, rr, pr)
            step = (fl + fr + ur - ul) / (dl + dr)
            p -= step
            if abs(step) <= tol * p:
                break
        else:
            raise RuntimeError("star pressure did not converge")
    fl, _ = _wave_jump(gamma, p, rl, pl)
    fr, _ = _wave_jump(gamma, p, rr, pr)
    return p, 0.5 * (ul + ur + fr - fl)


def _side(gamma, s, p_star, u_star, rho_k, u_k, p_k, sign):
    """State at x / t = s on the side of state K (sign = -1 left, +1 right)."""
    c_k = sound_speed(gamma, rho_k, p_k)
    g1, g2 = (gamma - 1.0) / (gamma + 1.0), (gamma - 1.0) / (2.0 * gamma)
    if p_star > p_k:                       # shock
        rho_star = rho_k * (p_star / p_k + g1) / (g1 * p_star / p_k + 1.0)
        speed = u_k + sign * c_k * np.sqrt((gamma + 1.0) / (2.0 * gamma) * p_star / p_k + g2)
        outside = (s > speed) if sign > 0 else (s < speed)
        return np.where(outside, rho_k, rho_star), np.where(outside, u_k, u_star), np.where(outside, p_k, p_star)
    rho_star = rho_k * (p_star / p_k) ** (1.0 / gamma)   # isentrope
    c_star = c_k * (p_star / p_k) ** g2
    head = u_k + sign * c_k
    tail = u_star + sign * c_star
    # inside the fan x / t = u + sign c, and the Riemann invariant
    # u - sign 2 c / (gamma - 1) keeps its value of state K
    u_fan = 2.0 / (gamma + 1.0) * (-sign * c_k + 0.5 * (gamma - 1.0) * u_k + s)
    c_fan = np.maximum(sign * (s - u_fan), 0.0)     # used only inside the fan, where it is positive
    rho_fan = rho_k * (c_fan / c_k) ** (2.0 / (gamma - 1.0))
    p_fan = p_k * (c_fan / c_k) ** (2.0 * gamma / (gamma - 1.0))
    if sign > 0:
        outside, inside = s > head, s > tail
    else:
        outside, inside = s < head, s < tail
    rho = np.where(outside, rho_k, np.where(inside, rho_fan, rho_star))
    u = np.where(outside, u_k, np.where(inside, u_fan, u_star))
    p = np.where(outside, p_k, np.where(inside, p_fan, p_star))
    return rho, u, p


def sample(gamma, left, right, s):
    """(rho, u, p) of the exact solution at the similarity coordinates s = x / t."""
    s = np.asarray(s, dtype=np.float64)
    p_star, u_star = star_state(gamma, left, right)
    rl, ul, pl = _side(gamma, s, p_star, u_star, *left, -1)
    rr, ur, pr = _side(gamma, s, p_star, u_star, *right, +1)
    on_left = s < u_star
    return np.where(on_left, rl, rr), np.where(on_left, ul, ur), np.where(on_left, pl, pr)


def waves(gamma, left, right):
    """Speeds of the wave edges: dict with the star state and, per side, the shock
    speed or the rarefaction head and tail speeds."""
    p_star, u_star = star_state(gamma, left, right)
    out = {"p_star": p_star, "u_star": u_star}
    for name, (rho_k, u_k, p_k), sign in (("left", left, -1), ("right", right, +1)):
        c_k = sound_speed(gamma, rho_k, p_k)
        if p_star > p_k:
            g1, g2 = (gamma - 1.0) / (gamma + 1.0), (gamma - 1.0) / (2.0 * gamma)
            out[name] = {"kind": "shock",
                         "speed": u_k + sign * c_k * np.sqrt((gamma + 1.0) / (2.0 * gamma) * p_star / p_k + g2),
                         "rho_star": rho_k * (p_star / p_k + g1) / (g1 * p_star / p_k + 1.0)}
        else:
            c_star = c_k * (p_star / p_k) ** ((gamma - 1.0) / (2.0 * gamma))
            out[name] = {"kind": "rarefaction", "head": u_k + sign * c_k, "tail": u_star + sign * c_star,
                         "rho_star": rho_k * (p_star / p_k) ** (1.0 / gamma)}
    return out
