"""Conversion between the oracle's matrix form and real Pauli coefficients.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A Hermitian 2x2 matrix W is written W = (a0 I + a1 sx + a2 sy + a3 sz) / 2,
so that a0 = tr W and ak = tr(W sk) are the Bloch components of Sec. 4
(interference example), r_k = tr(rho s_k).  Explicitly
    W = 1/2 [[a0 + a3, a1 - i a2], [a1 + i a2, a0 - a3]].
The Pauli axis is the leading axis of the coefficient array: shape [4, ...].
"""
import numpy as np

SIGMA = np.array([
    [[1, 0], [0, 1]],
    [[0, 1], [1, 0]],
    [[0, -1j], [1j, 0]],
    [[1, 0], [0, -1]],
], dtype=np.complex128)


def matrix_from_pauli(a):
    """[4, ...] real coefficients -> [..., 2, 2] complex Hermitian matrices."""
    a = np.asarray(a, dtype=np.float64)
    m = np.empty(a.shape[1:] + (2, 2), dtype=np.complex128)
    m[..., 0, 0] = 0.5 * (a[0] + a[3])
    m[..., 1, 1] = 0.5 * (a[0] - a[3])
    m[..., 0, 1] = 0.5 * (a[1] - 1j * a[2])
    m[..., 1, 0] = 0.5 * (a[1] + 1j * a[2])
    return m


def pauli_from_matrix(m):
    """[..., 2, 2] Hermitian matrices -> [4, ...] coefficients a_k = Re tr(W s_k)."""
    m = np.asarray(m)
    a0 = np.real(m[..., 0, 0] + m[..., 1, 1])
    a1 = np.real(m[..., 0, 1] + m[..., 1, 0])
    a2 = np.imag(m[..., 1, 0] - m[..., 0, 1])
    a3 = np.real(m[..., 0, 0] - m[..., 1, 1])
    return np.stack([a0, a1, a2, a3])
