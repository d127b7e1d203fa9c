"""Spectral discretizations of the Green operators (paper Sec. 3): Moulinec-Suquet
(Fourier polynomials) and Willot's rotated scheme (willot_frequencies).

Fields are real arrays [3, 3, n3, n2, n1] (tensor indices i, J first, then z, y, x
with x fastest).  The discrete Fourier transform is numpy's FFT over the three
grid axes; naive_dft3 is a plain O(n^2) DFT used by the tests to pin it.

Frequencies: xi_d(k) = 2 pi k / l_d with k in FFT order
{0, 1, ..., ceil(n/2)-1, -floor(n/2), ..., -1}.

Green operator (eq. Gamma0, Gamma^0 = Grad G^0 Div) for the reference medium
C^0 = mu0 (identity on 2-tensors) + kappa0 I (x) I, whose acoustic tensor is
K(xi) = mu0 |xi|^2 I + kappa0 xi (x) xi:
    (Gamma^0_hat tau_hat)_iJ = xi_J [K(xi)^{-1} (tau_hat xi)]_i .
The plain projector G (mu0 = 1, kappa0 = 0) is
    (G_hat tau_hat)_iJ = xi_J (tau_hat xi)_i / |xi|^2 .

Reading where the paper is silent: both operators vanish at xi = 0 and on every
Nyquist plane k_d = -n_d/2 of an even axis.  There the multiplier xi_J xi_L is
not Hermitian-consistent (the mode has no sign), so keeping it would make the
operators non-real; zeroing it keeps them exact real orthogonal projectors.
"""
import numpy as np


def fftn(x):
    return np.fft.fftn(x, axes=(-3, -2, -1))


def ifftn(x):
    return np.fft.ifftn(x, axes=(-3, -2, -1))


def naive_dft1(x, axis, inverse=False):
    """Plain DFT along one axis: X_k = sum_j x_j exp(-+ 2 pi i j k / n)."""
    n = x.shape[axis]
    j = np.arange(n)
    sgn = 1.0 if inverse else -1.0
    W = np.exp(sgn * 2j * np.pi * np.outer(j, j) / n)
    out = np.moveaxis(np.tensordot(W, np.moveaxis(x, axis, 0), axes=(1, 0)), 0, axis)
    return out / n if inverse else out


def naive_dft3(x, inverse=False):
    for ax in (-3, -2, -1):
        x = naive_dft1(x, ax, inverse)
    return x


def integer_frequencies(n):
    """k in FFT order for an axis of n points."""
    k = np.arange(n)
    return np.where(k < (n + 1) // 2, k, k - n)


def frequencies(n, l):
    """xi vectors on the grid: array [3, n3, n2, n1] and the mask of zeroed modes."""
    n1, n2, n3 = n
    l1, l2, l3 = l
    k1, k2, k3 = integer_frequencies(n1), integer_frequencies(n2), integer_frequencies(n3)
    x1 = 2.0 * np.pi * k1 / l1
    x2 = 2.0 * np.pi * k2 / l2
    x3 = 2.0 * np.pi * k3 / l3
    xi = np.zeros((3, n3, n2, n1))
    xi[0] = x1[None, None, :]
    xi[1] = x2[None, :, None]
    xi[2] = x3[:, None, None]
    zero = (k3[:, None, None] == 0) & (k2[None, :, None] == 0) & (k1[None, None, :] == 0)
    nyq = np.zeros((n3, n2, n1), dtype=bool)
    if n1 % 2 == 0:
        nyq |= (k1 == -n1 // 2)[None, None, :]
    if n2 % 2 == 0:
        nyq |= (k2 == -n2 // 2)[None, :, None]
    if n3 % 2 == 0:
        nyq |= (k3 == -n3 // 2)[:, None, None]
    return xi, zero | nyq


def willot_frequencies(n, l):
    """Modified wave vectors of the rotated (HEX8R) scheme of Willot (2015), the
    discretization the paper's reference solutions use (Sec. 3, 6).

    The displacement lives at the voxel corners and the gradient at the voxel
    centre is the average of the four forward differences along each axis.  For a
    corner field u = exp(i theta . x / h) this gives, with theta_d = 2 pi k_d / n_d,
        grad_J u = k_J u,  k_J = (e^{i theta_J} - 1) / h_J  prod_{m != J} (1 + e^{i theta_m}) / 2,
    which is Willot's (i / 4h) tan(theta_J / 2) prod_m (1 + e^{i theta_m}) written
    without the tangent.  Returns complex k [3, n3, n2, n1] and the mask of modes
    with k = 0 (the mean, and modes on two or more Nyquist planes)."""
    n1, n2, n3 = n
    h = (l[0] / n1, l[1] / n2, l[2] / n3)
    th = [2.0 * np.pi * np.arange(m) / m for m in (n1, n2, n3)]
    shape = [(1, 1, n1), (1, n2, 1), (n3, 1, 1)]
    dif = [((np.exp(1j * t) - 1.0) / hh).reshape(sh) for t, hh, sh in zip(th, h, shape)]
    avg = [(0.5 * (1.0 + np.exp(1j * t))).reshape(sh) for t, sh in zip(th, shape)]
    k = np.zeros((3, n3, n2, n1), dtype=complex)
    k[0] = dif[0] * avg[1] * avg[2]
    k[1] = avg[0] * dif[1] * avg[2]
    k[2] = avg[0] * avg[1] * dif[2]
    nyq = [np.zeros(m, bool) if m % 2 else (np.arange(m) == m // 2) for m in (n1, n2, n3)]
    cnt = (nyq[0][None, None, :].astype(int) + nyq[1][None, :, None] + nyq[2][:, None, None])
    zero = np.zeros((n3, n2, n1), bool)
    zero[0, 0, 0] = True
    mask = zero | (cnt >= 2)
    k[:, mask] = 0.0
    return k, mask


def gamma0_hat_k(tau_hat, k, mask, mu0, kappa0):
    """Green operator for a complex gradient multiplier k (grad_J -> k_J):
    (Gamma^0_hat tau_hat)_iJ = k_J [K^{-1} (tau_hat conj(k))]_i with the acoustic
    tensor K_ik = C^0_iJkL conj(k_J) k_L = mu0 |k|^2 d_ik + kappa0 conj(k_i) k_k."""
    kc = np.conj(k)
    v = np.einsum("iJ...,J...->i...", tau_hat, kc)
    K = mu0 * np.einsum("...,ik->ik...", (kc * k).sum(axis=0).real, np.eye(3)) \
        + kappa0 * np.einsum("i...,k...->ik...", kc, k)
    K = np.where(mask[None, None], np.eye(3)[:, :, None, None, None], K)
    Km = np.moveaxis(K, (0, 1), (-2, -1))
    vm = np.moveaxis(v, 0, -1)[..., None]
    w = np.moveaxis(np.linalg.solve(Km, vm)[..., 0], -1, 0)
    out = np.einsum("i...,J...->iJ...", w, k)
    out[:, :, mask] = 0.0
    return out


def g_hat_k(tau_hat, k, mask):
    """(G_hat tau_hat)_iJ = k_J (tau_hat conj(k))_i / |k|^2."""
    v = np.einsum("iJ...,J...->i...", tau_hat, np.conj(k))
    k2 = (np.conj(k) * k).sum(axis=0).real
    k2 = np.where(mask, 1.0, k2)
    out = np.einsum("i...,J...->iJ...", v / k2, k)
    out[:, :, mask] = 0.0
    return out


def gamma0_hat(tau_hat, xi, mask, mu0, kappa0):
    """(Gamma^0_hat tau_hat)_iJ = xi_J [K^{-1} (tau_hat xi)]_i, zero on masked modes."""
    v = np.einsum("iJ...,J...->i...", tau_hat, xi)               # tau_hat xi
    K = mu0 * np.einsum("...,ik->ik...", (xi * xi).sum(axis=0), np.eye(3)) \
        + kappa0 * np.einsum("i...,k...->ik...", xi, xi)
    K = np.where(mask[None, None], np.eye(3)[:, :, None, None, None], K)   # placeholder where zeroed
    Km = np.moveaxis(K, (0, 1), (-2, -1))
    vm = np.moveaxis(v, 0, -1)[..., None]
    w = np.moveaxis(np.linalg.solve(Km, vm)[..., 0], -1, 0)
    out = np.einsum("i...,J...->iJ...", w, xi)
    out[:, :, mask] = 0.0
    return out


def g_hat(tau_hat, xi, mask):
    """(G_hat tau_hat)_iJ = xi_J (tau_hat xi)_i / |xi|^2, zero on masked modes."""
    v = np.einsum("iJ...,J...->i...", tau_hat, xi)
    x2 = (xi * xi).sum(axis=0)
    x2 = np.where(mask, 1.0, x2)
    out = np.einsum("i...,J...->iJ...", v / x2, xi)
    out[:, :, mask] = 0.0
    return out


def apply_gamma0(tau, n, l, mu0, kappa0, disc="ms"):
    """Gamma^0[tau] for a real field tau [3,3,n3,n2,n1]; disc "ms" (Fourier
    polynomials, Sec. 3) or "willot" (rotated scheme)."""
    if disc == "willot":
        k, mask = willot_frequencies(n, l)
        return ifftn(gamma0_hat_k(fftn(tau), k, mask, mu0, kappa0)).real
    xi, mask = frequencies(n, l)
    return ifftn(gamma0_hat(fftn(tau), xi, mask, mu0, kappa0)).real


def apply_g(tau, n, l, disc="ms"):
    """G[tau] for a real field tau [3,3,n3,n2,n1]."""
    if disc == "willot":
        k, mask = willot_frequencies(n, l)
        return ifftn(g_hat_k(fftn(tau), k, mask)).real
    xi, mask = frequencies(n, l)
    return ifftn(g_hat(fftn(tau), xi, mask)).real
