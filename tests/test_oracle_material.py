"""Pins of the oracle's Neo-Hookean law (paper Sec. 6.1) to the energy it is
derived from, to textbook linear elasticity and to frame invariance."""
import numpy as np
import pytest

from oracle import material

MATS = [(1.0, 2.0), (3.846153846153846, 5.769230769230769), (0.5, 0.0), (1.0, 1000.0)]


def rand_F(rng, m, amp=0.3):
    F = np.eye(3) + rng.uniform(-amp, amp, (m, 3, 3))
    F[np.linalg.det(F) < 0.2] = np.eye(3)
    return F


def rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


@pytest.mark.parametrize("mu,lam", MATS)
def test_stress_is_energy_gradient(mu, lam):
    rng = np.random.default_rng(1)
    F = rand_F(rng, 20)
    P = material.stress(F, mu, lam)
    h = 1e-6
    Pfd = np.zeros_like(P)
    for k in range(3):
        for L in range(3):
            E = np.zeros((3, 3))
            E[k, L] = h
            Pfd[:, k, L] = (material.energy(F + E, mu, lam) - material.energy(F - E, mu, lam)) / (2 * h)
    scale = np.abs(P).max() + mu + lam
    assert np.abs(P - Pfd).max() <= 1e-8 * scale


@pytest.mark.parametrize("mu,lam", MATS)
def test_tangent_is_stress_gradient(mu, lam):
    rng = np.random.default_rng(2)
    F = rand_F(rng, 20)
    A = material.tangent(F, mu, lam)
    h = 1e-6
    Afd = np.zeros_like(A)
    for kL in range(9):
        E = np.zeros((3, 3))
        E[kL // 3, kL % 3] = h
        dP = (material.stress(F + E, mu, lam) - material.stress(F - E, mu, lam)) / (2 * h)
        Afd[:, :, kL] = dP.reshape(-1, 9)
    scale = np.abs(A).max()
    assert np.abs(A - Afd).max() <= 1e-7 * scale


@pytest.mark.parametrize("mu,lam", MATS)
def test_tangent_at_identity_is_isotropic_stiffness(mu, lam):
    A = material.tangent(np.eye(3)[None], mu, lam)[0]
    # written out independently: C_iJkL = lam d_iJ d_kL + mu (d_ik d_JL + d_iL d_Jk)
    C = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for J in range(3):
            for k in range(3):
                for L in range(3):
                    C[i, J, k, L] = lam * (i == J) * (k == L) + mu * ((i == k) * (J == L) + (i == L) * (J == k))
    assert np.abs(A - C.reshape(9, 9)).max() <= 1e-14 * (mu + lam)
    assert np.abs(material.stress(np.eye(3)[None], mu, lam)).max() == 0.0


def test_tangent_major_symmetry():
    rng = np.random.default_rng(3)
    A = material.tangent(rand_F(rng, 50), 2.0, 7.0)
    assert np.abs(A - np.swapaxes(A, 1, 2)).max() <= 1e-13 * np.abs(A).max()


def test_objectivity():
    rng = np.random.default_rng(4)
    F = rand_F(rng, 30)
    for _ in range(3):
        Q = rotation(rng)
        P = material.stress(F, 1.3, 2.1)
        PQ = material.stress(np.einsum("ij,mjk->mik", Q, F), 1.3, 2.1)
        assert np.abs(PQ - np.einsum("ij,mjk->mik", Q, P)).max() <= 1e-14 * 10
        W = material.energy(F, 1.3, 2.1)
        WQ = material.energy(np.einsum("ij,mjk->mik", Q, F), 1.3, 2.1)
        assert np.abs(W - WQ).max() <= 1e-14 * 10


def test_uniaxial_closed_form():
    # F = diag(s, 1, 1): J = s, P11 = mu s + (lam ln s - mu)/s, P22 = P33 = lam ln s
    mu, lam, s = 1.7, 3.1, 1.23
    P = material.stress(np.diag([s, 1.0, 1.0])[None], mu, lam)[0]
    assert P[0, 0] == pytest.approx(mu * s + (lam * np.log(s) - mu) / s, rel=1e-14)
    assert P[1, 1] == pytest.approx(lam * np.log(s), rel=1e-14)
    assert P[2, 2] == pytest.approx(lam * np.log(s), rel=1e-14)
    assert abs(P[0, 1]) + abs(P[1, 2]) + abs(P[0, 2]) == 0.0
