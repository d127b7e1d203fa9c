"""Spectral (Moulinec-Suquet) discretization of the Green operators (paper Sec. 3).

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


def apply_gamma0(tau, n, l, mu0, kappa0):
    """Gamma^0[tau] for a real field tau [3,3,n3,n2,n1]."""
    xi, mask = frequencies(n, l)
    return ifftn(gamma0_hat(fftn(tau), xi, mask, mu0, kappa0)).real


def apply_g(tau, n, l):
    """G[tau] for a real field tau [3,3,n3,n2,n1]."""
    xi, mask = frequencies(n, l)
    return ifftn(g_hat(fftn(tau), xi, mask)).real
