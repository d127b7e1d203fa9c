"""Pins of the small-strain ComBo path of the oracle (appendix cheat sheet,
infinitesimal strain column): the closed-form laminate against the small-load
limit of the finite-strain laminate, against the layered-medium formulas with
harmonic averages (written here from scalar equilibrium, not from tensors),
traction continuity and the Hadamard condition; the linear homogenization solve
against exact layered RVEs, the small-load limit of the Neo-Hooke solve and the
Voigt/Reuss bounds."""
import numpy as np
import pytest

from closed_forms import layered_stress, rotation_with_first_column
from oracle import laminate, material, solver
from paper_2204_13624_amd import synth

MATS = ((1.0, 2.0), (10.0, 20.0))
TIGHT = solver.Options(tol_newton=1e-12, tol_cg=1e-12)


def random_inputs(rng, m):
    H = rng.normal(scale=0.3, size=(m, 3, 3))
    c = rng.uniform(0.02, 0.98, size=m)
    N = rng.normal(size=(m, 3))
    N /= np.linalg.norm(N, axis=1)[:, None]
    return H, c, N


def sym(H):
    return 0.5 * (H + np.swapaxes(H, -1, -2))


def test_closed_form_is_the_layered_medium_in_the_frame_of_N():
    rng = np.random.default_rng(31)
    H, c, N = random_inputs(rng, 40)
    r = laminate.solve_small(H, c, N, MATS[0], MATS[1])
    for k in range(40):
        Q = rotation_with_first_column(N[k])
        ref = Q @ layered_stress(Q.T @ sym(H[k]) @ Q, c[k], MATS) @ Q.T
        assert np.abs(r["P"][k] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_traction_continuity_and_hadamard_jump():
    rng = np.random.default_rng(32)
    H, c, N = random_inputs(rng, 50)
    r = laminate.solve_small(H, c, N, MATS[0], MATS[1])
    tr = np.einsum("mij,mj->mi", r["Pp"] - r["Pm"], N)
    assert np.abs(tr).max() <= 1e-13 * np.abs(r["P"]).max()
    cp = c[:, None, None]
    assert np.abs(cp * r["eps_p"] + (1 - cp) * r["eps_m"] - sym(H)).max() <= 1e-14
    aN = np.einsum("mi,mj->mij", r["a"], N)
    jump = (1.0 / cp + 1.0 / (1 - cp)) * sym(aN)
    assert np.abs(r["eps_p"] - r["eps_m"] - jump).max() <= 1e-12 * np.abs(jump).max()
    # the phase stresses are the phase laws of the phase strains
    assert np.allclose(r["Pp"], material.linear_stress(np.eye(3) + r["eps_p"], *MATS[1]), rtol=0, atol=1e-13)


def test_tangent_reproduces_the_stress_and_has_both_symmetries():
    rng = np.random.default_rng(33)
    H, c, N = random_inputs(rng, 30)
    r = laminate.solve_small(H, c, N, MATS[0], MATS[1])
    sig = np.einsum("mab,mb->ma", r["A"], H.reshape(-1, 9)).reshape(-1, 3, 3)
    assert np.abs(sig - r["P"]).max() <= 1e-13 * np.abs(r["P"]).max()
    A = r["A"].reshape(-1, 3, 3, 3, 3)
    assert np.abs(A - A.transpose(0, 2, 1, 3, 4)).max() <= 1e-12 * np.abs(A).max()   # minor (left)
    assert np.abs(A - A.transpose(0, 3, 4, 1, 2)).max() <= 1e-12 * np.abs(A).max()   # major


def test_equal_phases_give_no_jump():
    rng = np.random.default_rng(34)
    H, c, N = random_inputs(rng, 10)
    r = laminate.solve_small(H, c, N, MATS[1], MATS[1])
    assert np.abs(r["a"]).max() <= 1e-15
    assert np.abs(r["A"] - material.isotropic_stiffness(*MATS[1])).max() <= 1e-13


def test_closed_form_is_the_small_load_limit_of_the_finite_strain_laminate():
    rng = np.random.default_rng(35)
    H, c, N = random_inputs(rng, 30)
    small = laminate.solve_small(H, c, N, MATS[0], MATS[1])
    t = 1e-6
    big = laminate.solve(np.eye(3) + t * H, c, N, MATS[0], MATS[1])
    assert (big["status"] == laminate.STATUS_OK).all()
    scale = np.abs(small["P"]).max()
    assert np.abs(big["P"] / t - small["P"]).max() <= 1e-4 * scale
    assert np.abs(big["a"] / t - small["a"]).max() <= 1e-4 * np.abs(small["a"]).max()
    at_identity = laminate.solve(np.repeat(np.eye(3)[None], 30, axis=0), c, N, MATS[0], MATS[1])
    assert np.abs(at_identity["A"] - small["A"]).max() <= 1e-12 * np.abs(small["A"]).max()


def linear_problem(ms, mats=MATS):
    return solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, mats, law="linear")


H_BAR = np.array([[0.011, 0.004, -0.002], [0.001, -0.006, 0.003], [0.005, -0.001, 0.008]])


@pytest.mark.parametrize("n,axis,interfaces", [
    ((9, 2, 3), 0, (-0.5 + 2.25 / 9, -0.5 + 6.5 / 9)),     # composite columns normal to e1
    ((3, 7, 2), 1, (-0.5 + 1.75 / 7, -0.5 + 4.75 / 7)),    # normal to e2
    ((9, 3, 4), 0, (-0.5 + 2 / 9, -0.5 + 6 / 9)),           # pure voxels only
])
def test_layered_rve_is_exact(n, axis, interfaces):
    ms = synth.layered(n, (1.0, 1.0, 1.0), axis, interfaces)
    phi = float(ms.c.mean())
    r = solver.solve(linear_problem(ms), np.eye(3) + H_BAR, TIGHT)
    Q = rotation_with_first_column(np.eye(3)[axis])
    ref = Q @ layered_stress(Q.T @ sym(H_BAR) @ Q, phi, MATS) @ Q.T
    assert np.abs(r["Pbar"] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert r["stats"]["newton_iters"] <= 2


def test_linear_solve_is_the_small_load_limit_of_the_neo_hooke_solve():
    ms = synth.single_sphere((8, 8, 8), radius=0.3, center=(0.05, -0.02, 0.03))
    lin = solver.solve(linear_problem(ms), np.eye(3) + H_BAR, TIGHT)
    t = 1e-4
    # the Newton test is relative to |Pbar| = O(t): round-off of P = O(eps mu) bounds it near 1e-11
    nh = solver.solve(solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS), np.eye(3) + t * H_BAR,
                      solver.Options(tol_newton=1e-9, tol_cg=1e-12))
    assert np.abs(nh["Pbar"] / t - lin["Pbar"]).max() <= 2e-3 * np.abs(lin["Pbar"]).max()
    assert lin["stats"]["newton_iters"] <= 2


def test_effective_stiffness_is_linear_and_within_voigt_reuss():
    ms = synth.single_sphere((8, 8, 8), radius=0.3, center=(0.05, -0.02, 0.03))
    prob = linear_problem(ms)
    r = solver.solve(prob, np.eye(3), solver.Options(tol_newton=1e-12, tol_cg=1e-13, want_tangent=True))
    C = r["Abar"]
    # the effective stiffness maps any mean strain to the solved mean stress
    s = solver.solve(prob, np.eye(3) + H_BAR, TIGHT)["Pbar"]
    assert np.abs(C @ H_BAR.reshape(9) - s.reshape(9)).max() <= 1e-9 * np.abs(s).max()
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    w = [1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)]

    def mandel(C9):
        C4 = C9.reshape(3, 3, 3, 3)
        return np.array([[w[a] * w[b] * C4[idx[a] + idx[b]] for b in range(6)] for a in range(6)])

    phi = float(ms.c.mean())
    Cm = mandel(material.isotropic_stiffness(*MATS[0]))
    Cp = mandel(material.isotropic_stiffness(*MATS[1]))
    CV = phi * Cp + (1 - phi) * Cm
    CR = np.linalg.inv(phi * np.linalg.inv(Cp) + (1 - phi) * np.linalg.inv(Cm))
    A6 = mandel(C)
    assert np.linalg.eigvalsh(CV - A6).min() > 0
    assert np.linalg.eigvalsh(A6 - CR).min() > 0
