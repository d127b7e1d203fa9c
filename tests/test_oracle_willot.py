"""Pins of the oracle's rotated (Willot, HEX8R) discretization: the Fourier
multiplier against the corner-to-centre finite-difference stencil it stands for,
the Green operators as projections (real, idempotent, identity on compatible
fields, divergence preserving), exact layered RVEs on even grids (which the
Moulinec-Suquet reading cannot represent), and the whole solve against a direct
real-space assembly of reduced-integration hexahedra."""
import numpy as np
import pytest

from closed_forms import layered_stress, rotation_with_first_column
from oracle import laminate, material, solver, spectral
from paper_2204_13624_amd import synth

MATS = ((1.0, 2.0), (10.0, 20.0))


def stencil_grad(u, h):
    """Voxel-centre gradient of a corner field u [3, n3, n2, n1] (corner (k, j, i) is the
    lower corner of voxel (k, j, i)): the mean of the four edge differences per axis."""
    def sh(a, dz, dy, dx):
        return np.roll(a, (-dz, -dy, -dx), axis=(-3, -2, -1))

    H = np.zeros((3, 3) + u.shape[1:])
    for J, (dz, dy, dx) in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
        acc = 0.0
        others = [(a, b) for a in (0, 1) for b in (0, 1)]
        for a, b in others:
            if J == 0:
                o = (a, b, 0)
            elif J == 1:
                o = (a, 0, b)
            else:
                o = (0, a, b)
            acc = acc + sh(u, o[0] + dz, o[1] + dy, o[2] + dx) - sh(u, *o)
        H[:, J] = acc / (4.0 * h[J])
    return H


def stencil_div(tau, h):
    """Corner divergence: minus the adjoint of stencil_grad (per unit cell volume)."""
    def sh(a, dz, dy, dx):
        return np.roll(a, (dz, dy, dx), axis=(-3, -2, -1))

    d = np.zeros((3,) + tau.shape[2:])
    for J, (dz, dy, dx) in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
        for a in (0, 1):
            for b in (0, 1):
                o = (a, b, 0) if J == 0 else ((a, 0, b) if J == 1 else (0, a, b))
                d += (sh(tau[:, J], *o) - sh(tau[:, J], o[0] + dz, o[1] + dy, o[2] + dx)) / (4.0 * h[J])
    return -d


N_L = [((6, 5, 4), (1.0, 1.0, 1.0)), ((8, 6, 9), (0.8, 1.3, 0.7))]


@pytest.mark.parametrize("n,l", N_L)
def test_multiplier_is_the_corner_stencil(n, l):
    rng = np.random.default_rng(1)
    u = rng.normal(size=(3, n[2], n[1], n[0]))
    h = tuple(a / b for a, b in zip(l, n))
    k, mask = spectral.willot_frequencies(n, l)
    uh = spectral.fftn(u)
    Hf = spectral.ifftn(np.einsum("i...,J...->iJ...", uh, k))
    Hs = stencil_grad(u, h)
    assert np.abs(Hf.imag).max() <= 1e-12
    assert np.abs(Hf.real - Hs).max() <= 1e-12 * np.abs(Hs).max()
    # the masked modes are exactly those with a vanishing multiplier
    kk = np.abs(k).sum(axis=0)
    assert (kk[mask] == 0).all() and (kk[~mask] > 1e-12).all()


@pytest.mark.parametrize("n,l", N_L)
def test_green_operators_are_real_projections(n, l):
    rng = np.random.default_rng(2)
    mu0, kappa0 = 3.0, 7.0
    tau = rng.normal(size=(3, 3, n[2], n[1], n[0]))
    k, mask = spectral.willot_frequencies(n, l)
    raw = spectral.ifftn(spectral.gamma0_hat_k(spectral.fftn(tau), k, mask, mu0, kappa0))
    assert np.abs(raw.imag).max() <= 1e-12 * np.abs(raw.real).max()
    g = spectral.apply_gamma0(tau, n, l, mu0, kappa0, "willot")
    c0g = mu0 * g + kappa0 * np.einsum("ab,kk...->ab...", np.eye(3), g)
    gg = spectral.apply_gamma0(c0g, n, l, mu0, kappa0, "willot")
    assert np.abs(gg - g).max() <= 1e-12 * np.abs(g).max()
    G = spectral.apply_g(tau, n, l, "willot")
    assert np.abs(spectral.apply_g(G, n, l, "willot") - G).max() <= 1e-12 * np.abs(G).max()
    # G keeps the discrete divergence and maps stencil gradients to themselves
    h = tuple(a / b for a, b in zip(l, n))
    assert np.abs(stencil_div(G, h) - stencil_div(tau, h)).max() <= 1e-11 * np.abs(stencil_div(tau, h)).max()
    u = rng.normal(size=(3, n[2], n[1], n[0]))
    Hs = stencil_grad(u, h)
    assert np.abs(spectral.apply_g(Hs, n, l, "willot") - Hs).max() <= 1e-12 * np.abs(Hs).max()
    c0h = mu0 * Hs + kappa0 * np.einsum("ab,kk...->ab...", np.eye(3), Hs)
    assert np.abs(spectral.apply_gamma0(c0h, n, l, mu0, kappa0, "willot") - Hs).max() <= 1e-12 * np.abs(Hs).max()


H_BAR = np.array([[0.011, 0.004, -0.002], [0.001, -0.006, 0.003], [0.005, -0.001, 0.008]])
FBAR = np.array([[1.08, 0.12, -0.03], [0.05, 0.97, 0.04], [-0.02, 0.06, 1.02]])


@pytest.mark.parametrize("n,interfaces", [((8, 3, 2), (-0.5 + 3 / 8, -0.5 + 6 / 8)),        # odd width, even n
                                          ((10, 2, 4), (-0.5 + 2.3 / 10, -0.5 + 7.6 / 10))])  # composite columns
def test_layered_rve_is_exact_on_even_grids(n, interfaces):
    ms = synth.layered(n, (1.0, 1.0, 1.0), 0, interfaces)
    phi = float(ms.c.mean())
    tight = solver.Options(tol_newton=1e-12, tol_cg=1e-12)
    lin = solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS, law="linear", disc="willot")
    r = solver.solve(lin, np.eye(3) + H_BAR, tight)
    ref = layered_stress(0.5 * (H_BAR + H_BAR.T), phi, MATS)
    assert np.abs(r["Pbar"] - ref).max() <= 1e-12 * np.abs(ref).max()
    nh = solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS, disc="willot")
    r = solver.solve(nh, FBAR, tight)
    ref = laminate.solve(FBAR[None], np.array([phi]), np.array([[1.0, 0.0, 0.0]]), MATS[0], MATS[1])["P"][0]
    assert np.abs(r["Pbar"] - ref).max() <= 1e-12 * np.abs(ref).max()
    _ = rotation_with_first_column


def test_ms_reading_is_not_exact_on_the_same_even_grid():
    ms = synth.layered((8, 3, 2), (1.0, 1.0, 1.0), 0, (-0.5 + 3 / 8, -0.5 + 6 / 8))
    lin = solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS, law="linear")
    r = solver.solve(lin, np.eye(3) + H_BAR, solver.Options(tol_newton=1e-12, tol_cg=1e-12))
    ref = layered_stress(0.5 * (H_BAR + H_BAR.T), float(ms.c.mean()), MATS)
    assert np.abs(r["Pbar"] - ref).max() > 1e-6 * np.abs(ref).max()


def hex8r_solve(prob, Hbar):
    """Reduced-integration trilinear hexahedra on the periodic corner grid, assembled
    and solved directly (least squares: the hourglass modes are in the null space,
    the centre strains are unique).  Returns the centre gradient field [3, 3, ...]."""
    n1, n2, n3 = prob.n
    h = (prob.l[0] / n1, prob.l[1] / n2, prob.l[2] / n3)
    F0 = np.broadcast_to((np.eye(3) + Hbar)[:, :, None, None, None], (3, 3, n3, n2, n1))
    _, Av, ok, _, _ = solver.evaluate(np.ascontiguousarray(F0), prob)
    assert ok
    nn = n1 * n2 * n3
    K = np.zeros((3 * nn, 3 * nn))
    f = np.zeros(3 * nn)
    Bs = []
    vol = h[0] * h[1] * h[2]
    for k in range(n3):
        for j in range(n2):
            for i in range(n1):
                B = np.zeros((9, 3 * nn))
                for a in (0, 1):
                    for b in (0, 1):
                        for c in (0, 1):
                            node = (((k + c) % n3) * n2 + (j + b) % n2) * n1 + (i + a) % n1
                            g = ((2 * a - 1) / (4 * h[0]), (2 * b - 1) / (4 * h[1]), (2 * c - 1) / (4 * h[2]))
                            for comp in range(3):
                                for J in range(3):
                                    B[3 * comp + J, 3 * node + comp] += g[J]
                A = Av[(k * n2 + j) * n1 + i]
                K += vol * B.T @ A @ B
                f -= vol * B.T @ A @ Hbar.reshape(9)
                Bs.append(B)
    u = np.linalg.lstsq(K, f, rcond=1e-12)[0]
    H = np.stack([Hbar.reshape(9) + B @ u for B in Bs])            # [voxels, 9]
    return np.moveaxis(H, 0, -1).reshape(3, 3, n3, n2, n1)


def test_solve_equals_a_direct_hex8r_assembly():
    ms = synth.random_composite_field((4, 3, 5), 11, frac_composite=0.4)
    prob = solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, ((1.0, 2.0), (30.0, 60.0)), law="linear",
                          disc="willot")
    H = hex8r_solve(prob, H_BAR)
    r = solver.solve(prob, np.eye(3) + H_BAR, solver.Options(tol_newton=1e-13, tol_cg=1e-13))
    Hf = r["F"] - np.eye(3)[:, :, None, None, None]
    assert np.abs(Hf - H).max() <= 1e-10 * np.abs(H).max()
    sig = np.einsum("vab,vb->va", solver.evaluate(r["F"], prob)[1], solver.to_voxels(Hf).reshape(-1, 9))
    assert np.abs(sig.mean(axis=0).reshape(3, 3) - r["Pbar"]).max() <= 1e-12 * np.abs(r["Pbar"]).max()


def test_willot_and_ms_agree_on_smooth_fields():
    """A homogeneous RVE is exact under both; on a soft-contrast sphere the two
    discretizations differ only by the discretization error (a few percent here)."""
    ms = synth.homogeneous((6, 4, 5), phase_id=1)
    r = solver.solve(solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS, disc="willot"), FBAR)
    assert np.abs(r["Pbar"] - material.stress(FBAR[None], *MATS[1])[0]).max() <= 1e-14
    ms = synth.single_sphere((8, 8, 8), radius=0.3)
    o = solver.Options(tol_newton=1e-10, tol_cg=1e-12)
    a = solver.solve(solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS, disc="willot"), FBAR, o)["Pbar"]
    b = solver.solve(solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS), FBAR, o)["Pbar"]
    assert 0 < np.abs(a - b).max() <= 0.05 * np.abs(b).max()
