"""Pins of the two collision variants (oracle.variants).

Isothermal model (Sec. 3.1, paragraph on beta0 and mu0):
* mass and momentum conserved exactly; energy changes unless T = 1/beta0;
* a Fermi-Dirac state at T = 1/beta0 collides exactly as in the thermal model
  (its moment eps equals eps_FD(beta0)), also at beta0 != 1;
* the equilibrium energy matches the 2D closed form (nu = log(expm1(beta0 n /
  2 pi)), F_1 from mpmath's polylogarithm), computed here independently;
* on a spatially uniform field the repeated collision has the closed form
  W(n) = W_eq + (1 - omega)^n (W(0) - W_eq) with W_eq of the beta0 state.
Positivity-limited relaxation (Sec. 3.3, paragraph after the algorithm):
* where the plain collision keeps every population positive semidefinite the
  variant is the plain collision, bit for bit;
* on nearly pure states with over-relaxation every output population is
  positive semidefinite up to rounding, conservation holds, and the rate is
  maximal: in every limited cell some population sits on the boundary, and a
  slightly larger rate breaks positivity (brute force).
"""
import mpmath
import numpy as np
import pytest

from oracle import pauli, qlbm, variants
from paper_1309_1656_amd import synthetic


def _cons(lat, W):
    g = qlbm.global_means(lat, W)
    return g


def _state(d, shape, seed, T=None):
    lat = qlbm.Lattice(d)
    f = synthetic.macroscopic_fields(shape, seed)
    W = qlbm.init_equilibrium(lat, f["trrho"], f["r"], lat.xi * f["u_lat"], f["T"] if T is None else T)
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 0.01, size=(4,) + W.shape[:-2]) * lat.w.reshape((1, -1) + (1,) * d)
    return lat, W + pauli.matrix_from_pauli(a)


@pytest.mark.parametrize("d,shape", [(2, (6, 7)), (3, (3, 4, 5))])
def test_isothermal_conserves_mass_and_momentum_not_energy(d, shape):
    lat, W = _state(d, shape, 1)
    Wc = variants.collide_isothermal(lat, W, 0.8)
    r0, T0, u0, e0 = qlbm.moments(lat, W)
    r1, T1, u1, e1 = qlbm.moments(lat, Wc)
    assert np.max(np.abs(r1 - r0)) < 1e-14 and np.max(np.abs(T1[None] * u1 - T0[None] * u0)) < 1e-14
    g0, g1 = qlbm.global_means(lat, W), qlbm.global_means(lat, Wc)
    assert abs(g1[7] - g0[7]) > 1e-4 * g0[7]          # T varies around 1 = 1/beta0: energy moves


@pytest.mark.parametrize("d,beta0", [(2, 1.0), (2, 0.8), (3, 1.25)])
def test_isothermal_equals_thermal_at_beta0(d, beta0):
    shape = (5, 6) if d == 2 else (3, 4, 5)
    lat = qlbm.Lattice(d, beta0)
    f = synthetic.macroscopic_fields(shape, 4)
    W = qlbm.init_equilibrium(lat, f["trrho"], f["r"], lat.xi * f["u_lat"], np.full(shape, 1.0 / beta0))
    a = variants.collide_isothermal(lat, W, 0.7)
    b = qlbm.collide(lat, W, 0.7)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))


def test_isothermal_energy_closed_form_2d():
    lat = qlbm.Lattice(2, 0.9)
    rho = qlbm.density_matrix(np.array([1.3, 0.7]), np.array([[0.2, 0.0], [0.1, -0.3], [0.4, 0.1]]))
    got = variants.isothermal_energy(2, 0.9, rho)
    F1 = lambda x: float(mpmath.re(-mpmath.polylog(2, -mpmath.exp(x))))
    for j in range(2):
        tr = [1.3, 0.7][j]
        rv = np.linalg.norm([[0.2, 0.1, 0.4], [0.0, -0.3, 0.1]][j])
        nus = [np.log(np.expm1(0.9 * n / (2 * np.pi))) for n in (0.5 * (tr + rv), 0.5 * (tr - rv))]
        F0 = [np.log1p(np.exp(v)) for v in nus]
        expect = (F1(nus[0]) + F1(nus[1])) / (0.9 * (F0[0] + F0[1]))
        assert abs(got[j] / expect - 1) < 1e-13


def test_isothermal_homogeneous_closed_form():
    lat = qlbm.Lattice(3)
    shape = (2, 2, 2)
    f = synthetic.macroscopic_fields((4, 4, 4), 6)
    one = {k: v[(slice(None),) * (v.ndim - 3) + (0, 0, 0)] for k, v in f.items()}
    trrho = np.full(shape, one["trrho"])
    r = np.broadcast_to(one["r"].reshape(3, 1, 1, 1), (3,) + shape)
    u = np.broadcast_to(lat.xi * one["u_lat"].reshape(3, 1, 1, 1), (3,) + shape)
    W0 = qlbm.init_equilibrium(lat, trrho, r, u, np.full(shape, 1.4))      # hotter than 1/beta0
    rho, T, uu, eps = qlbm.moments(lat, W0)
    Weq = qlbm.equilibrium(lat, rho, uu, variants.isothermal_energy(3, 1.0, rho))
    om = 1 / 0.8
    W = W0
    for n in range(1, 6):
        W = variants.collide_isothermal(lat, W, 0.8)
        W = qlbm.stream(lat, W)                    # a uniform field is unchanged by streaming
        expect = Weq + (1 - om) ** n * (W0 - Weq)
        assert np.max(np.abs(W - expect)) < 1e-13 * np.max(np.abs(Weq))


def _nearly_pure(d, shape, seed, frac=0.97):
    lat, W = _state(d, shape, seed)
    a = pauli.pauli_from_matrix(W)
    rng = np.random.default_rng(seed + 1)
    dirs = rng.normal(size=(3,) + a.shape[1:])
    dirs /= np.linalg.norm(dirs, axis=0)
    a[1:] = frac * a[0][None] * dirs
    return lat, pauli.matrix_from_pauli(a)


@pytest.mark.parametrize("d,shape", [(2, (6, 7)), (3, (3, 4, 5))])
def test_positive_is_plain_where_plain_stays_positive(d, shape):
    lat, W = _state(d, shape, 2)
    assert qlbm.count_negative_eigenvalues(qlbm.collide(lat, W, 0.8)) == 0
    assert np.array_equal(variants.collide_positive(lat, W, 0.8), qlbm.collide(lat, W, 0.8))


@pytest.mark.parametrize("d,shape", [(2, (6, 7)), (3, (3, 4, 5))])
@pytest.mark.parametrize("isothermal", [False, True])
def test_positive_keeps_semidefinite_and_is_maximal(d, shape, isothermal):
    lat, W = _nearly_pure(d, shape, 3)
    tau = 0.55
    plain = variants.collide_isothermal(lat, W, tau) if isothermal else qlbm.collide(lat, W, tau)
    assert qlbm.count_negative_eigenvalues(plain) > 10                # the plain collision breaks positivity
    Wp = variants.collide_positive(lat, W, tau, isothermal=isothermal)
    scale = np.max(np.abs(W))
    ev = np.linalg.eigvalsh(Wp)[..., 0]
    assert ev.min() > -1e-15 * scale
    r0, T0, u0, _ = qlbm.moments(lat, W)
    r1, T1, u1, _ = qlbm.moments(lat, Wp)
    assert np.max(np.abs(r1 - r0)) < 1e-14 and np.max(np.abs(T1[None] * u1 - T0[None] * u0)) < 1e-14
    if not isothermal:
        assert abs(qlbm.global_means(lat, Wp)[7] - qlbm.global_means(lat, W)[7]) < 1e-14
    # maximality, by brute force on the limited cells
    rho, T, u, eps = qlbm.moments(lat, W)
    e = variants.isothermal_energy(lat.d, lat.beta0, rho) if isothermal else eps
    Weq = qlbm.equilibrium(lat, rho, u, e)
    om = variants.positive_omega(lat, W, Weq, 1 / tau)
    limited = om < 1 / tau
    assert limited.sum() > 3
    assert np.all(ev.min(axis=0)[limited] < 1e-12 * scale)            # a population sits on the boundary
    bump = np.minimum(om + 1e-7, 1 / tau)[None, ..., None, None]
    worse = np.linalg.eigvalsh(W + bump * (Weq - W))[..., 0].min(axis=0)
    assert np.all(worse[limited] < 0)
