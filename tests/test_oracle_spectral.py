"""Pins of the oracle's spectral operators (paper Sec. 3): the library FFT against
a plain DFT, the frequency scaling and index order of the Green operators
against analytic gradients, and the projector identities."""
import numpy as np
import pytest

from oracle import spectral


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (5, 7, 3), (6, 9, 8), (16, 12, 9), (3, 1, 2)])
def test_fft_matches_naive_dft(shape):
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2,) + shape) + 1j * rng.normal(size=(2,) + shape)
    X = spectral.fftn(x)
    Xn = spectral.naive_dft3(x)
    assert np.abs(X - Xn).max() <= 1e-13 * np.abs(X).max()
    assert np.abs(spectral.ifftn(X) - spectral.naive_dft3(Xn, inverse=True)).max() <= 1e-13 * np.abs(x).max()


def _grid(n, l):
    n1, n2, n3 = n
    x1 = -l[0] / 2 + (np.arange(n1) + 0.5) * l[0] / n1
    x2 = -l[1] / 2 + (np.arange(n2) + 0.5) * l[1] / n2
    x3 = -l[2] / 2 + (np.arange(n3) + 0.5) * l[2] / n3
    return np.meshgrid(x3, x2, x1, indexing="ij")   # z, y, x


def _trig_displacement(n, l, rng):
    """A trigonometric periodic displacement u and its exact gradient F_iJ = du_i/dX_J."""
    Z, Y, X = _grid(n, l)
    coords = [X, Y, Z]
    u = np.zeros((3,) + X.shape)
    G = np.zeros((3, 3) + X.shape)
    for i in range(3):
        for _ in range(2):
            m = [int(rng.integers(0, (nd - 1) // 2 + 1)) for nd in n]   # below Nyquist
            if m == [0, 0, 0]:
                m[0] = min(1, (n[0] - 1) // 2)
            kvec = [2 * np.pi * m[d] / l[d] for d in range(3)]
            phi = rng.uniform(0, 2 * np.pi)
            amp = rng.normal()
            arg = kvec[0] * X + kvec[1] * Y + kvec[2] * Z + phi
            u[i] += amp * np.sin(arg)
            for J in range(3):
                G[i, J] += amp * kvec[J] * np.cos(arg)
    return u, G


@pytest.mark.parametrize("n,l", [((8, 6, 10), (1.0, 1.0, 1.0)), ((9, 7, 5), (2.0, 0.5, 1.3)),
                                 ((12, 12, 4), (1.0, 3.0, 0.25))])
def test_gamma0_inverts_reference_medium_on_gradients(n, l):
    """Gamma^0 C^0 is the identity on compatible zero-mean fields: checks 2 pi k / l
    and that the projection acts on the second (referential) index."""
    rng = np.random.default_rng(1)
    _, G = _trig_displacement(n, l, rng)
    mu0, kappa0 = 1.7, 5.3
    tr = G[0, 0] + G[1, 1] + G[2, 2]
    tau = mu0 * G + kappa0 * np.einsum("ij,...->ij...", np.eye(3), tr)
    out = spectral.apply_gamma0(tau, n, l, mu0, kappa0)
    assert np.abs(out - G).max() <= 1e-12 * np.abs(G).max()
    assert np.abs(spectral.apply_g(G, n, l) - G).max() <= 1e-12 * np.abs(G).max()


def test_g_annihilates_divergence_free_fields_and_not_their_transpose():
    n, l = (8, 8, 8), (1.0, 1.0, 1.0)
    Z, Y, X = _grid(n, l)
    g = np.cos(2 * np.pi * X)
    P = np.zeros((3, 3) + X.shape)
    P[0, 1] = g          # Div P = dP_iJ/dX_J = dP_01/dX_1 = 0
    assert np.abs(spectral.apply_g(P, n, l)).max() <= 1e-14
    Pt = np.zeros_like(P)
    Pt[1, 0] = g         # dP_10/dX_0 != 0
    assert np.abs(spectral.apply_g(Pt, n, l)).max() > 0.5


@pytest.mark.parametrize("n", [(6, 6, 6), (7, 5, 9), (8, 4, 6)])
def test_projector_identities_and_real_output(n):
    rng = np.random.default_rng(2)
    l = (1.0, 1.3, 0.7)
    tau = rng.normal(size=(3, 3) + (n[2], n[1], n[0]))
    xi, mask = spectral.frequencies(n, l)
    th = spectral.fftn(tau)
    G1 = spectral.g_hat(th, xi, mask)
    G2 = spectral.g_hat(G1, xi, mask)
    assert np.abs(G2 - G1).max() <= 1e-14 * np.abs(G1).max()          # G^2 = G
    # G real (Hermitian-preserving), symmetric in the L2 product
    g = spectral.ifftn(G1)
    assert np.abs(g.imag).max() <= 1e-14 * np.abs(g.real).max()
    sig = rng.normal(size=tau.shape)
    lhs = np.sum(spectral.apply_g(tau, n, l) * sig)
    rhs = np.sum(tau * spectral.apply_g(sig, n, l))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # Gamma^0 C^0 Gamma^0 = Gamma^0
    mu0, kappa0 = 0.8, 2.5
    g0 = spectral.apply_gamma0(tau, n, l, mu0, kappa0)
    trg = g0[0, 0] + g0[1, 1] + g0[2, 2]
    c0g0 = mu0 * g0 + kappa0 * np.einsum("ij,...->ij...", np.eye(3), trg)
    g0g0 = spectral.apply_gamma0(c0g0, n, l, mu0, kappa0)
    assert np.abs(g0g0 - g0).max() <= 1e-13 * np.abs(g0).max()
    # Gamma^0 output is compatible and zero-mean
    assert np.abs(g0.mean(axis=(2, 3, 4))).max() <= 1e-14
    assert np.abs(spectral.apply_g(g0, n, l) - g0).max() <= 1e-13 * np.abs(g0).max()


def test_frequencies_fft_order_and_nyquist_mask():
    xi, mask = spectral.frequencies((4, 3, 2), (2.0, 1.0, 1.0))
    # x axis: k = 0, 1, -2, -1 -> xi = 2 pi k / 2
    assert np.allclose(xi[0, 0, 0, :], np.pi * np.array([0, 1, -2, -1]))
    assert np.allclose(xi[1, 0, :, 0], 2 * np.pi * np.array([0, 1, -1]))
    assert mask[0, 0, 0] and mask[0, 0, 2] and mask[1, 0, 1]   # zero mode, x and z Nyquist
    assert not mask[0, 1, 1] and not mask[0, 2, 3]
