"""Pins of the oracle's magnetic-field collision (Sec. 5, Eq. sigmaB_comm).

* The precession equals direct numerical integration (scipy solve_ivp) of
  dW/dt = -i [mu sigma.B, W] over one time step.
* Without collision (tau -> infinity is not allowed; a uniform equilibrium
  state is used instead, where the BGK term vanishes) the Bloch vector of
  every population turns about B by 2 mu |B| per step: after n steps the
  angle is 2 n mu |B|, checked against the rotation formula of a vector about
  an axis.
* Traces, hence momentum and energy, and the length of every Bloch vector are
  unchanged by the precession; the step with B = 0 is the plain step.
* Rotating W and B by the same SU(2) matrix commutes with the step.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import magnetic, pauli, qlbm
from paper_1309_1656_amd import synthetic


def _state(d, shape, seed=3):
    lat = qlbm.Lattice(d)
    f = synthetic.macroscopic_fields(shape, seed)
    W = qlbm.init_equilibrium(lat, f["trrho"], f["r"], lat.xi * f["u_lat"], f["T"])
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 0.02, size=(4,) + W.shape[:-2]) * lat.w.reshape((1, -1) + (1,) * d)
    return lat, W + pauli.matrix_from_pauli(a)


def test_precession_matches_ode_integration():
    rng = np.random.default_rng(0)
    mu_b = rng.normal(0, 0.4, size=(3, 4))
    W0 = pauli.matrix_from_pauli(rng.normal(0, 1, size=(4, 4)))       # 4 cells, one population
    got = magnetic.precess(W0[None], mu_b)[0]
    for c in range(4):
        H = sum(mu_b[k, c] * pauli.SIGMA[k + 1] for k in range(3))

        def rhs(t, y):
            Wm = y.reshape(2, 2)
            return (-1j * (H @ Wm - Wm @ H)).ravel()

        sol = solve_ivp(rhs, (0.0, 1.0), W0[c].ravel().astype(np.complex128), rtol=1e-12, atol=1e-14,
                        method="DOP853")
        assert np.max(np.abs(sol.y[:, -1].reshape(2, 2) - got[c])) < 1e-10


def _rotate(v, axis, angle):
    """Vector v turned about the unit axis by angle (right-hand rule)."""
    return (v * np.cos(angle) + np.cross(axis, v) * np.sin(angle)
            + axis * np.dot(axis, v) * (1 - np.cos(angle)))


def test_pure_precession_angle():
    """On a uniform equilibrium state the BGK term vanishes; only the field acts."""
    lat = qlbm.Lattice(2)
    shape = (3, 4)
    trrho = np.full(shape, 1.0)
    r = np.zeros((3,) + shape)
    r[0] = 0.2
    r[2] = 0.1
    W = qlbm.init_equilibrium(lat, trrho, r, np.zeros((2,) + shape), np.ones(shape))
    B = np.array([0.3, -0.2, 0.5])
    mu_b = np.broadcast_to(B[:, None, None], (3,) + shape).copy()
    n = 7
    Wn = magnetic.run_with_field(lat, W, 0.8, mu_b, n)
    axis = B / np.linalg.norm(B)
    angle = 2 * n * np.linalg.norm(B)
    a0 = pauli.pauli_from_matrix(W)[:, :, 0, 0]
    an = pauli.pauli_from_matrix(Wn)[:, :, 0, 0]
    for i in range(lat.Q):
        # sign: U = exp(-i t sigma.B) turns the Bloch vector about +B by +2|B|t
        assert np.allclose(an[1:, i], _rotate(a0[1:, i], axis, angle), atol=1e-14)
        assert abs(an[0, i] - a0[0, i]) < 1e-14


@pytest.mark.parametrize("d,shape", [(2, (6, 7)), (3, (4, 5, 6))])
def test_precession_conserves_traces_and_bloch_length(d, shape):
    lat, W = _state(d, shape)
    rng = np.random.default_rng(1)
    mu_b = rng.normal(0, 0.3, size=(3,) + shape)
    Wp = magnetic.precess(W, mu_b)
    a, b = pauli.pauli_from_matrix(W), pauli.pauli_from_matrix(Wp)
    assert np.max(np.abs(a[0] - b[0])) < 1e-15
    assert np.max(np.abs(np.linalg.norm(a[1:], axis=0) - np.linalg.norm(b[1:], axis=0))) < 1e-14
    # with the collision: momentum and energy of every cell unchanged
    Wc = magnetic.collide_with_field(lat, W, 0.7, mu_b)
    r0, T0, u0, e0 = qlbm.moments(lat, W)
    r1, T1, u1, e1 = qlbm.moments(lat, Wc)
    assert np.max(np.abs(T1 - T0)) < 1e-14 and np.max(np.abs(u1 - u0)) < 1e-14 and np.max(np.abs(e1 - e0)) < 1e-13


@pytest.mark.parametrize("d,shape", [(2, (6, 7)), (3, (4, 5, 6))])
def test_zero_field_is_plain_step(d, shape):
    lat, W = _state(d, shape)
    a = magnetic.run_with_field(lat, W, 0.8, np.zeros((3,) + shape), 3)
    b = qlbm.run(lat, W, 0.8, 3)
    assert np.max(np.abs(a - b)) < 1e-16


@pytest.mark.parametrize("d,shape", [(2, (6, 7)), (3, (4, 5, 6))])
def test_joint_su2_covariance(d, shape):
    lat, W = _state(d, shape)
    rng = np.random.default_rng(4)
    mu_b = rng.normal(0, 0.3, size=(3,) + shape)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    U = np.array([[q[0] + 1j * q[1], q[2] + 1j * q[3]], [-q[2] + 1j * q[3], q[0] - 1j * q[1]]])
    rot = lambda X: U @ X @ U.conj().T
    # B transforms like a Bloch vector: sigma.B -> U (sigma.B) U*
    H = sum(mu_b[k][..., None, None] * pauli.SIGMA[k + 1] for k in range(3))
    mu_b_rot = pauli.pauli_from_matrix(rot(H))[1:] / 2.0      # H = sigma.B carries no 1/2
    lhs = magnetic.run_with_field(lat, rot(W), 0.75, mu_b_rot, 3)
    rhs = rot(magnetic.run_with_field(lat, W, 0.75, mu_b, 3))
    assert np.max(np.abs(lhs - rhs)) < 1e-14


@pytest.mark.parametrize("d,shape", [(2, (5, 6)), (3, (3, 4, 5))])
def test_field_step_vjp_matches_finite_differences(d, shape):
    lat, W = _state(d, shape, seed=9)
    rng = np.random.default_rng(5)
    mu_b = rng.normal(0, 0.3, size=(3,) + shape)
    tau = 0.7
    Lam_next = pauli.matrix_from_pauli(rng.normal(0, 1, size=(4, lat.Q) + shape))
    Lam, dom = magnetic.step_vjp_with_field(lat, W, Lam_next, tau, mu_b)
    pair = lambda A, B: float(np.real((A * np.swapaxes(B, -1, -2)).sum()))
    for seed in (1, 2):
        dW = pauli.matrix_from_pauli(np.random.default_rng(seed).normal(0, 1e-2, size=(4, lat.Q) + shape))
        h = 1e-5
        fd = (pair(Lam_next, magnetic.step_with_field(lat, W + h * dW, tau, mu_b))
              - pair(Lam_next, magnetic.step_with_field(lat, W - h * dW, tau, mu_b))) / (2 * h)
        assert abs(pair(Lam, dW) - fd) <= 1e-8 * max(1.0, abs(fd))
    h = 1e-6
    om = 1.0 / tau
    fd = (pair(Lam_next, magnetic.step_with_field(lat, W, 1.0 / (om + h), mu_b))
          - pair(Lam_next, magnetic.step_with_field(lat, W, 1.0 / (om - h), mu_b))) / (2 * h)
    assert abs(dom - fd) <= 1e-7 * max(1.0, abs(fd))
    # with no field the adjoint is the plain one
    from oracle import adjoint
    L0, d0 = magnetic.step_vjp_with_field(lat, W, Lam_next, tau, np.zeros((3,) + shape))
    L1, d1 = adjoint.step_vjp(lat, W, Lam_next, tau)
    assert np.max(np.abs(L0 - L1)) < 1e-15 * np.max(np.abs(L1)) + 1e-300 and abs(d0 - d1) < 1e-13 * abs(d1)
