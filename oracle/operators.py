"""Probing operator A of the per-pixel problem, FP64 (test infrastructure only).

Paper: Sec. 2.2, Eq. (optTMsmall2IQ) and Eq. (probingmatrix). The probing
matrix stacks K blocks Q_m = F diag(e^{j psi_m}) where F is the 2-D Fourier
matrix of an n1 x n2 grid; the incident fields are the rows of A
(transposed, not conjugated). Each row t of the TM maps to KN intensities
|A t|^2 (Eq. forwardmodel / optTMsmall2).

Readings (paper silent or ambiguous):
  * F is the unnormalised DFT with kernel exp(-2 pi j k i / n): the paper
    needs a pure-phase Q (unit-modulus entries) and uses the forward FFT for
    Q and the inverse for Q^H.
  * The grid is row-major: input index i = i1*n2 + i2, F = F_n1 (x) F_n2.
  * Measurements are mask-major: a row's KN intensities are ordered
    [m][k1][k2].
Consequence: A^H A = K N I_N, since each block is sqrt(N) times a unitary.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(n: int) -> np.ndarray:
    """F_n[k, i] = exp(-2 pi j k i / n), unnormalised. The product k*i is
    reduced mod n in integers first so that the angle is exact to one
    rounding."""
    k = np.arange(n, dtype=np.int64)
    e = np.outer(k, k) % n
    return np.exp(-2j * np.pi * e / n)


def dft2_matrix(n1: int, n2: int) -> np.ndarray:
    """2-D DFT of a row-major n1 x n2 grid as an N x N matrix: kron(F_n1, F_n2)."""
    return np.kron(dft_matrix(n1), dft_matrix(n2))


def probing_matrix(masks: np.ndarray, n1: int, n2: int) -> np.ndarray:
    """Dense A = [F diag(psi_1); ...; F diag(psi_K)], shape [K*N, N] (Eq. probingmatrix)."""
    F = dft2_matrix(n1, n2)
    return np.concatenate([F * m[None, :] for m in masks], axis=0)


class DenseOp:
    """A and A^H by explicit dense products. Rows of `t` are TM rows."""

    def __init__(self, masks: np.ndarray, n1: int, n2: int):
        self.masks = np.asarray(masks, dtype=np.complex128)
        self.K, self.N = self.masks.shape
        self.n1, self.n2 = n1, n2
        assert n1 * n2 == self.N
        self.A = probing_matrix(self.masks, n1, n2)

    def forward(self, t: np.ndarray) -> np.ndarray:
        """y = A t for each row; returns [P, K, N] (mask-major measurement order)."""
        t = np.atleast_2d(t)
        return (t @ self.A.T).reshape(t.shape[0], self.K, self.N)

    def adjoint(self, y: np.ndarray) -> np.ndarray:
        """x = A^H y for each row; y is [P, K, N]."""
        y = y.reshape(y.shape[0], self.K * self.N)
        return y @ self.A.conj()


class FFTOp:
    """A and A^H evaluated with library FFTs (numpy.fft), as the paper
    proposes (Sec. 2.2: the products with Q and Q^H are FFTs and inverse
    FFTs). F x = fft2(x); F^H y = N * ifft2(y)."""

    def __init__(self, masks: np.ndarray, n1: int, n2: int):
        self.masks = np.asarray(masks, dtype=np.complex128)
        self.K, self.N = self.masks.shape
        self.n1, self.n2 = n1, n2
        assert n1 * n2 == self.N

    def forward(self, t: np.ndarray) -> np.ndarray:
        t = np.atleast_2d(t)
        P = t.shape[0]
        x = (self.masks[None, :, :] * t[:, None, :]).reshape(P, self.K, self.n1, self.n2)
        return np.fft.fft2(x).reshape(P, self.K, self.N)

    def adjoint(self, y: np.ndarray) -> np.ndarray:
        P = y.shape[0]
        x = np.fft.ifft2(y.reshape(P, self.K, self.n1, self.n2)).reshape(P, self.K, self.N) * self.N
        return np.einsum("pkn,kn->pn", x, self.masks.conj())


def intensities(op, t: np.ndarray) -> np.ndarray:
    """I = |A t|^2 per row, [P, K, N] (Eq. forwardmodel, per pixel as Eq. optTMsmall2)."""
    return np.abs(op.forward(t)) ** 2


class MatrixOp:
    """y = Q t and x = Q^H y for an explicit dense probing matrix Q [M][N]
    (the random-phase probing of the prior art the paper compares with,
    whose products cost Theta(M N) without FFTs, Sec. 2.2 and Table time)."""

    def __init__(self, Q: np.ndarray):
        self.Q = np.asarray(Q, dtype=np.complex128)
        self.M, self.N = self.Q.shape

    def forward(self, t: np.ndarray) -> np.ndarray:
        return np.atleast_2d(t) @ self.Q.T

    def adjoint(self, y: np.ndarray) -> np.ndarray:
        return y @ self.Q.conj()
