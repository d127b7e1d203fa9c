"""Closed-form solutions used as pins by the oracle and GPU tests (no oracle code)."""
import numpy as np


def rotation_with_first_column(N):
    """Orthogonal Q (det +1) with Q e1 = N."""
    N = np.asarray(N, float) / np.linalg.norm(N)
    t = np.array([1.0, 0.0, 0.0]) if abs(N[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    b = t - (t @ N) * N
    b /= np.linalg.norm(b)
    return np.stack([N, b, np.cross(N, b)], axis=1)


def layered_stress(eps, f, mats):
    """Average stress of isotropic layers normal to e1 with inclusion fraction f
    under mean strain eps: in-plane strains and the traction sigma_1j are uniform,
    so sigma_11, sigma_12, sigma_13 follow from harmonic means of lambda + 2 mu
    and mu, and the in-plane stresses are volume averages."""
    fr = (1.0 - f, f)
    mu = (mats[0][0], mats[1][0])
    lam = (mats[0][1], mats[1][1])
    M = tuple(lam[p] + 2 * mu[p] for p in (0, 1))

    def avg(g):
        return sum(fr[p] * g(p) for p in (0, 1))

    e = eps[1, 1] + eps[2, 2]
    s = np.zeros((3, 3))
    s[0, 0] = (eps[0, 0] + e * avg(lambda p: lam[p] / M[p])) / avg(lambda p: 1.0 / M[p])
    s[0, 1] = s[1, 0] = 2.0 * eps[0, 1] / avg(lambda p: 1.0 / mu[p])
    s[0, 2] = s[2, 0] = 2.0 * eps[0, 2] / avg(lambda p: 1.0 / mu[p])
    e11 = [(s[0, 0] - lam[p] * e) / M[p] for p in (0, 1)]
    for k in (1, 2):
        s[k, k] = avg(lambda p: lam[p] * (e11[p] + e) + 2.0 * mu[p] * eps[k, k])
    s[1, 2] = s[2, 1] = 2.0 * avg(lambda p: mu[p]) * eps[1, 2]
    return s
