"""Phase-offset correction from defocus intensities, FP64 (test infrastructure only).

Paper: Sec. 2.3. The retrieved rows carry one unknown phase each,
TM_true = diag(e^{j phi}) TM_est (Eq. phaseoffset). With the field
c_n = TM_est e^{j theta_n} predicted at the fiber end for a defocus input
e^{j theta_n}, the defocus image is
    I_n = | K2^H P diag(h) K1 diag(c_n) e^{j phi} |^2
(Eq. forwarddefocusImage) with K1 the 2-D Fourier matrix of the field grid,
h the angular-spectrum kernel with pupil (Eq. angularspectrum and the pupil
definition after it), P zero padding to twice the size in frequency, K2^H
the inverse 2-D Fourier matrix of the image grid. phi minimises
g(phi) = sum_n || I_n - |A_n e^{j phi}|^2 ||^2 (Eq. optphase) with the
gradient of Eq. phasederive (App. B), by L-BFGS.

Readings:
  * c_n excludes phi (the paper's c_n already contains e^{j phi} but A_n
    applies it again; the second application is the one kept).
  * The P rows are pixels of the nf1 x nf2 field grid (raster indices
    `pix`); other pixels carry zero field.
  * K1 and K2^H are unitary ("ortho"); the pupil includes its boundary
    (lambda sqrt(u^2+v^2) <= NA); h uses +j; spatial frequencies are
    u_k = k / (n ps) for k < n/2 and (k - n) / (n ps) otherwise.
  * Zero padding keeps each signed frequency at the same signed frequency
    of the doubled grid; the Nyquist bin is zero under the pupil whenever
    NA < lambda / (2 ps), so its split is moot.
  * L-BFGS over phi in R^P from phi = 0 (the commented-out Algorithm 2),
    memory m, first direction -sqrt(P) g/||g|| (a = 1 changes the offsets by
    1 rad RMS; the same after a reset of the history), pairs with s^T y <= 0
    skipped; line search from a = 1 that doubles the step while a trial
    satisfies Armijo (c = 1e-4) but not the curvature condition (c2 = 0.9)
    and takes the last such trial, or halves it while no trial satisfies
    Armijo.
  * phi is defined up to a constant; comparisons remove the circular mean
    of the difference.
"""
from __future__ import annotations

import numpy as np

from .operators import dft_matrix


def freqs(n: int, ps: float) -> np.ndarray:
    k = np.arange(n)
    return np.where(k < (n + 1) // 2, k, k - n) / (n * ps)


def pupil_kernel(nf1: int, nf2: int, ps: float, lam: float, NA: float, z: float):
    """h(u, v, z) = exp(j 2pi/lambda sqrt(1 - (lambda u)^2 - (lambda v)^2) z) p(u, v)
    on the field grid's frequency raster (Eq. angularspectrum). Returns
    (h [nf1, nf2] complex128, pupil [nf1, nf2] bool)."""
    u = freqs(nf1, ps)[:, None]
    v = freqs(nf2, ps)[None, :]
    rho2 = (lam * u) ** 2 + (lam * v) ** 2
    pupil = np.sqrt(rho2) <= NA
    arg = np.sqrt(np.where(pupil, 1.0 - rho2, 0.0))
    h = np.where(pupil, np.exp(1j * 2 * np.pi / lam * arg * z), 0.0)
    return h, pupil


def pad_index(n: int) -> np.ndarray:
    """Position in the 2n-point spectrum of each bin of the n-point spectrum
    (same signed frequency)."""
    k = np.arange(n)
    signed = np.where(k < (n + 1) // 2, k, k - n)
    return np.mod(signed, 2 * n)


def padding_matrix(nf1: int, nf2: int) -> np.ndarray:
    """P: [4 nf1 nf2, nf1 nf2] 0/1 matrix placing the field spectrum into the
    doubled spectrum."""
    i1 = pad_index(nf1)
    i2 = pad_index(nf2)
    Pm = np.zeros((4 * nf1 * nf2, nf1 * nf2))
    for a in range(nf1):
        for b in range(nf2):
            Pm[i1[a] * (2 * nf2) + i2[b], a * nf2 + b] = 1.0
    return Pm


def dense_propagator(nf1: int, nf2: int, h: np.ndarray) -> np.ndarray:
    """K2^H P diag(h) K1 as a dense [4 nf1 nf2, nf1 nf2] matrix (unitary K's)."""
    K1 = np.kron(dft_matrix(nf1), dft_matrix(nf2)) / np.sqrt(nf1 * nf2)
    K2 = np.kron(dft_matrix(2 * nf1), dft_matrix(2 * nf2)) / np.sqrt(4 * nf1 * nf2)
    return K2.conj().T @ padding_matrix(nf1, nf2) @ (h.ravel()[:, None] * K1)


class DefocusModel:
    """A_n u = K2^H P diag(h) K1 S diag(c_n) u for the P pixels `pix`
    (S scatters pixel values into the nf1 x nf2 field grid)."""

    def __init__(self, tm_est, theta, pix, nf1, nf2, lam, ps, NA, z, dense=False):
        self.c = np.asarray(theta) @ np.asarray(tm_est).T          # [Nd, P]  c_n = TM_est e^{j theta_n}
        self.pix = np.asarray(pix, dtype=np.int64)
        self.nf1, self.nf2 = nf1, nf2
        self.h, self.pupil = pupil_kernel(nf1, nf2, ps, lam, NA, z)
        self.i1, self.i2 = pad_index(nf1), pad_index(nf2)
        self.dense = dense
        if dense:
            G = dense_propagator(nf1, nf2, self.h)
            self.G = G[:, self.pix]                                   # [4 nf1 nf2, P]

    def forward(self, u: np.ndarray) -> np.ndarray:
        """[Nd, 2nf1, 2nf2] complex fields at the defocus plane for pixel phasors u [P]."""
        Nd = self.c.shape[0]
        x = self.c * u[None, :]
        if self.dense:
            return (x @ self.G.T).reshape(Nd, 2 * self.nf1, 2 * self.nf2)
        fld = np.zeros((Nd, self.nf1 * self.nf2), dtype=np.complex128)
        fld[:, self.pix] = x
        S = np.fft.fft2(fld.reshape(Nd, self.nf1, self.nf2), norm="ortho") * self.h[None]
        S2 = np.zeros((Nd, 2 * self.nf1, 2 * self.nf2), dtype=np.complex128)
        S2[:, self.i1[:, None], self.i2[None, :]] = S
        return np.fft.ifft2(S2, norm="ortho")

    def adjoint(self, v: np.ndarray) -> np.ndarray:
        """sum_n A_n^H v_n for v [Nd, 2nf1, 2nf2]; returns [P]."""
        Nd = self.c.shape[0]
        if self.dense:
            back = v.reshape(Nd, -1) @ self.G.conj()
        else:
            S2 = np.fft.fft2(v, norm="ortho")
            S = S2[:, self.i1[:, None], self.i2[None, :]] * np.conj(self.h)[None]
            fld = np.fft.ifft2(S, norm="ortho").reshape(Nd, -1)
            back = fld[:, self.pix]
        return np.sum(np.conj(self.c) * back, axis=0)

    def objective(self, Id: np.ndarray, phi: np.ndarray):
        """g(phi) (Eq. optphase) and dg/dphi = -4 Im(conj(u) w),
        w = sum_n A_n^H ((A_n u) r_n), r_n = I_n - |A_n u|^2; this equals the
        real expression of Eq. phasederive."""
        u = np.exp(1j * phi)
        a = self.forward(u)
        r = Id - np.abs(a) ** 2
        g = float(np.sum(r * r))
        w = self.adjoint(a * r)
        return g, -4.0 * np.imag(np.conj(u) * w)

    def images(self, phi: np.ndarray) -> np.ndarray:
        return np.abs(self.forward(np.exp(1j * phi))) ** 2


def lbfgs_phase(model: DefocusModel, Id: np.ndarray, phi0: np.ndarray, iters: int, m: int = 5,
                c_armijo: float = 1e-4, max_halvings: int = 40, c_curv: float = 0.9, max_doublings: int = 20,
                trace: list | None = None):
    """L-BFGS over phi (real R^P). Line search from a = 1: a trial that lowers
    g enough (Armijo, c_armijo) while g still falls steeply along d (the
    curvature condition d^T grad(trial) >= c_curv d^T grad fails) is kept and
    the step doubled, at most max_doublings times; the iteration takes the last
    kept trial once a doubled trial is no better, or a trial that meets both
    conditions. Before any trial is kept, failing trials halve the step (at
    most max_halvings times). Returns (phi, history of g); `trace` (a list)
    receives (a, f_trial, slope_trial, kept) per trial."""
    x = np.array(phi0, dtype=np.float64)
    f, g = model.objective(Id, x)
    S, Y = [], []
    hist = [f]
    for _ in range(iters):
        q = g.copy()
        al = []
        for s_, y_ in zip(reversed(S), reversed(Y)):
            a = np.dot(s_, q) / np.dot(y_, s_)
            q -= a * y_
            al.append(a)
        if S:
            q *= np.dot(S[-1], Y[-1]) / np.dot(Y[-1], Y[-1])
        else:
            gn = np.linalg.norm(g)
            q *= np.sqrt(x.size) / gn if gn > 0 else 0.0  # a = 1 moves the offsets by 1 rad RMS
        for (s_, y_), a in zip(zip(S, Y), reversed(al)):
            b = np.dot(y_, q) / np.dot(y_, s_)
            q += (a - b) * s_
        d = -q
        slope = float(np.dot(g, d))
        if not slope < 0:
            S, Y = [], []
            gn = np.linalg.norm(g)
            if gn == 0:
                break
            d = -np.sqrt(x.size) * g / gn
            slope = float(np.dot(g, d))
        a = 1.0
        best = None
        halvings = doublings = 0
        while True:
            fn, gn_ = model.objective(Id, x + a * d)
            ok = fn <= f + c_armijo * a * slope and (best is None or fn < best[1])
            slope_n = float(np.dot(gn_, d))
            if trace is not None:
                trace.append((a, fn, slope_n, ok))
            if ok:
                best = (a, fn, gn_)
                if halvings > 0 or slope_n >= c_curv * slope or doublings >= max_doublings:
                    break
                a *= 2.0
                doublings += 1
            elif best is not None:
                break
            else:
                halvings += 1
                if halvings >= max_halvings:
                    break
                a *= 0.5
        if best is None:
            break
        a, fn, gn_ = best
        s_vec = a * d
        y_vec = gn_ - g
        if np.dot(s_vec, y_vec) > 0:
            S.append(s_vec)
            Y.append(y_vec)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        x, f, g = x + s_vec, fn, gn_
        hist.append(f)
    return x, np.array(hist)


def circular_offset_error(phi_hat: np.ndarray, phi_true: np.ndarray) -> np.ndarray:
    """Per-row phase error after removing the circular-mean difference, in (-pi, pi]."""
    d = np.angle(np.exp(1j * (phi_hat - phi_true)))
    c = np.angle(np.mean(np.exp(1j * d)))
    return np.angle(np.exp(1j * (d - c)))
