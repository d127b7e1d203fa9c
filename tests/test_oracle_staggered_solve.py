"""Pins of the oracle's finite-strain solve on the staggered grid with the DFMG law
(paper App. A with the Newton-CG Lippmann-Schwinger solve of Sec. 3 and the
ComBo law of Sec. 4): the staggered Green operator's projection identities,
the DFMG tangent against finite differences of the DFMG stress (composite cells
included), the self-adjointness of the Newton operator, homogeneous RVEs,
grid-aligned laminates under loads normal to the layers (exact on this grid,
pure and composite cells), and the small-strain limit against the independent
linear staggered solve."""
import numpy as np
import pytest
from scipy import optimize

from oracle import material, solver, staggered as st
from paper_2204_13624_amd import synth

MATS = ((1.0, 2.0), (10.0, 20.0))
TIGHT = solver.Options(tol_newton=1e-12, tol_cg=1e-12)


def problem(ms, mats=MATS):
    return solver.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, mats, disc="staggered")


def rng_field(shape, seed, amp=1.0):
    return amp * np.random.default_rng(seed).normal(size=shape)


def compatible(n, l, seed, amp=0.05):
    """Grad U of a random periodic displacement on the staggered grid."""
    h = tuple(l[d] / n[d] for d in range(3))
    return st.grad(rng_field((3, n[2], n[1], n[0]), seed, amp), h)


N0, L0 = (6, 5, 4), (1.2, 0.9, 0.7)


def test_green_operator_projects_on_staggered_gradients():
    mu0, kappa0 = 3.0, 5.0
    C0 = st.c0_tensor(mu0, kappa0)
    E = compatible(N0, L0, 1)
    # Gamma0 [C0 : Grad U] = Grad U on the staggered grid
    tau = np.einsum("aAbB,bB...->aA...", C0, E)
    out = st.apply_gamma0(tau, N0, L0, mu0, kappa0)
    assert np.abs(out - E).max() <= 1e-12 * np.abs(E).max()
    # G is idempotent, Gamma0 lands on compatible fields, the mean is removed
    T = rng_field((3, 3, N0[2], N0[1], N0[0]), 2)
    g1 = st.apply_g(T, N0, L0)
    assert np.abs(st.apply_g(g1, N0, L0) - g1).max() <= 1e-12 * np.abs(g1).max()
    G0 = st.apply_gamma0(T, N0, L0, mu0, kappa0)
    assert np.abs(st.apply_g(G0, N0, L0) - G0).max() <= 1e-12 * np.abs(G0).max()
    assert np.abs(G0.mean(axis=(2, 3, 4))).max() <= 1e-14 * np.abs(G0).max()
    # G is the orthogonal projection on compatible fields: T - G T is orthogonal to Grad U
    assert abs(np.sum((T - g1) * E)) <= 1e-12 * np.abs(T).max() * np.abs(E).sum()


def composite_field(n, seed):
    ms = synth.random_composite_field(n, seed, frac_composite=0.5)
    return ms


def test_dfmg_tangent_matches_finite_differences():
    ms = composite_field((4, 3, 3), 5)
    assert ms.n_composite > 0 and (ms.phase == 0).any() and (ms.phase == 1).any()
    prob = problem(ms)
    F = np.eye(3)[:, :, None, None, None] + compatible(ms.n, ms.l, 6, 0.04) \
        + 0.03 * np.array([[0.5, 1.0, 0.2], [-0.3, 0.2, 0.4], [0.1, -0.6, -0.2]])[:, :, None, None, None]
    P, terms, ok, _, _ = st.evaluate(F, prob)
    assert ok
    dF = rng_field(F.shape, 7)
    h = 1e-6
    Pp = st.evaluate(F + h * dF, prob)[0]
    Pm = st.evaluate(F - h * dF, prob)[0]
    fd = (Pp - Pm) / (2 * h)
    an = st.tangent_action(terms, dF)
    assert np.abs(fd - an).max() <= 2e-7 * np.abs(an).max()


def test_newton_operator_is_self_adjoint_in_c0():
    ms = composite_field((4, 4, 3), 8)
    prob = problem(ms)
    mu0, kappa0 = solver.reference_medium(MATS)
    F = np.eye(3)[:, :, None, None, None] + compatible(ms.n, ms.l, 9, 0.03)
    _, terms, ok, _, _ = st.evaluate(F, prob)
    assert ok
    x = compatible(ms.n, ms.l, 10)
    y = compatible(ms.n, ms.l, 11)
    Ax = st.apply_gamma0(st.tangent_action(terms, x), ms.n, ms.l, mu0, kappa0)
    Ay = st.apply_gamma0(st.tangent_action(terms, y), ms.n, ms.l, mu0, kappa0)
    lhs = solver.inner_c0(y, Ax, mu0, kappa0)
    rhs = solver.inner_c0(Ay, x, mu0, kappa0)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    assert abs(lhs) > 0


FBAR = np.array([[1.08, 0.12, -0.03], [0.05, 0.97, 0.04], [-0.02, 0.06, 1.02]])


def test_homogeneous_rves_are_exact():
    for ph in (0, 1):
        ms = synth.homogeneous((4, 3, 5), phase_id=ph)
        r = solver.solve(problem(ms), FBAR, TIGHT)
        assert r["stats"]["newton_iters"] == 0
        assert np.abs(r["F"] - FBAR[:, :, None, None, None]).max() <= 1e-15
        assert np.abs(r["Pbar"] - material.stress(FBAR[None], *MATS[ph])[0]).max() <= 1e-14
    from oracle import laminate
    Nn = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    ms = synth.uniform_composite((3, 4, 2), 0.37, Nn)
    r = solver.solve(problem(ms), FBAR, TIGHT)
    ref = laminate.solve(FBAR[None], np.array([0.37]), Nn[None], MATS[0], MATS[1])["P"][0]
    assert np.abs(r["Pbar"] - ref).max() <= 1e-13


def exact_normal_laminate(Fdiag, phi, axis, mats):
    """Layers normal to e_axis under a diagonal mean deformation: the in-plane
    stretches are those of the mean, the normal stretches of the two layers differ
    and carry one normal stress (scipy root).  Returns the layer stresses (P+, P-)."""
    def parts(t):
        Fp = np.diag(Fdiag).astype(float).copy()
        Fm = Fp.copy()
        Fp[axis, axis] = Fdiag[axis] + (1 - phi) * t
        Fm[axis, axis] = Fdiag[axis] - phi * t
        return material.stress(Fp[None], *mats[1])[0], material.stress(Fm[None], *mats[0])[0]

    sol = optimize.brentq(lambda t: parts(t)[0][axis, axis] - parts(t)[1][axis, axis], -0.5, 0.5, xtol=1e-16,
                          rtol=1e-15)
    return parts(sol)


@pytest.mark.parametrize("n,l,axis,interfaces", [
    ((9, 2, 3), (1.0, 1.0, 1.0), 0, (-0.5 + 2 / 9, -0.5 + 6 / 9)),                  # pure cells
    ((9, 2, 3), (1.0, 1.0, 1.0), 0, (-0.5 + 2.25 / 9, -0.5 + 6.5 / 9)),             # composite columns
    ((3, 7, 2), (1.0, 1.4, 1.0), 1, (-0.7 + 1.4 * 1.75 / 7, -0.7 + 1.4 * 4.9 / 7)),  # normal e2, composites
    ((2, 3, 8), (1.0, 0.8, 2.0), 2, (-1.0 + 2 * 1.25 / 8, -1.0 + 2 * 5.5 / 8)),      # normal e3, composites
])
def test_laminate_under_normal_load_is_exact(n, l, axis, interfaces):
    """Under a diagonal load the shear components vanish in every cell and the DFMG
    terms reduce to the cell's own law: the layers' normal stretches solve the 1-D
    traction balance exactly, composite cells (normal e_axis) included."""
    ms = synth.layered(n, l, axis, interfaces)
    phi = float(ms.c.mean())
    Fd = np.array([1.06, 0.97, 1.02])
    r = solver.solve(problem(ms), np.diag(Fd), TIGHT)
    Pp, Pm = exact_normal_laminate(Fd, phi, axis, MATS)
    ref = phi * Pp + (1 - phi) * Pm
    assert np.abs(r["Pbar"] - ref).max() <= 1e-12 * np.abs(ref).max()
    scale = max(np.abs(Pp).max(), np.abs(Pm).max())
    assert np.abs(r["Pbar_phase"][0] - Pp).max() <= 1e-12 * scale
    assert np.abs(r["Pbar_phase"][1] - Pm).max() <= 1e-12 * scale
    assert np.abs(Pp - Pm).max() > 0.05 * scale


def test_small_load_limit_is_the_linear_staggered_solve():
    """Neo-Hooke linearises at F = I to the isotropic law with the same (mu, lambda):
    at a load of size t the finite-strain solve differs from the independent linear
    staggered solve (oracle.staggered.solve_linear) by O(t^2)."""
    ms = synth.single_sphere((6, 6, 6), radius=0.3)
    phase = np.where(ms.phase == 2, (ms.c > 0.5).astype(np.uint8), ms.phase).astype(np.uint8)
    pure = synth.Microstructure(n=ms.n, l=ms.l, phase=phase, c=phase.astype(float),
                                N=np.zeros_like(ms.N), info={})
    H0 = np.array([[0.5, 0.3, -0.1], [0.2, -0.4, 0.25], [-0.15, 0.1, 0.3]])
    errs, rels = [], []
    for t in (1e-3, 5e-4):
        lin = st.solve_linear(pure.phase, pure.l, MATS, t * H0)
        r = solver.solve(problem(pure), np.eye(3) + t * H0, TIGHT)
        d = np.abs(r["Pbar"] - lin["Pbar"]).max()
        errs.append(d)
        rels.append(d / np.abs(lin["Pbar"]).max())
    assert rels[0] < 2e-3                    # the two solves agree to first order
    assert 3.6 < errs[0] / errs[1] < 4.4     # and differ by a term quadratic in the load


def test_sphere_solve_equilibrium_and_mean():
    """A solve with composite cells: <F> = Fbar, Div P = 0 at the tolerance, and the
    phase averages recombine to Pbar."""
    ms = synth.single_sphere((6, 6, 6), radius=0.3)
    assert ms.n_composite > 0
    prob = problem(ms)
    r = solver.solve(prob, FBAR, TIGHT)
    assert np.abs(r["F"].mean(axis=(2, 3, 4)) - FBAR).max() <= 1e-14
    h = tuple(ms.l[d] / ms.n[d] for d in range(3))
    dv = st.div(r["P"], h)
    assert np.abs(dv).max() <= 1e-9 * np.abs(r["P"]).max() / min(h)
    vp = float((ms.phase == 1).sum() + ms.c[ms.phase == 2].sum())
    vm = float(ms.nvox) - vp
    rec = (vp * r["Pbar_phase"][0] + vm * r["Pbar_phase"][1]) / ms.nvox
    assert np.abs(rec - r["Pbar"]).max() <= 1e-13 * np.abs(r["Pbar"]).max()


def test_effective_tangent_matches_finite_differences_and_is_symmetric():
    """Abar of the staggered solve (nine CG solves with the DFMG tangent) against central
    differences of the solved Pbar, composite cells included; major symmetry holds
    because Abar is the second derivative of the averaged stored energy."""
    ms = synth.single_sphere((4, 4, 3), radius=0.3, center=(0.05, -0.03, 0.02))
    assert ms.n_composite > 0
    prob = problem(ms)
    r = solver.solve(prob, FBAR, solver.Options(tol_newton=1e-13, tol_cg=1e-13, want_tangent=True))
    A = r["Abar"]
    h = 1e-5
    Afd = np.zeros((9, 9))
    o = solver.Options(tol_newton=1e-13, tol_cg=1e-13)
    for kL in range(9):
        E = np.zeros((3, 3))
        E[kL // 3, kL % 3] = h
        Pp = solver.solve(prob, FBAR + E, o)["Pbar"]
        Pm = solver.solve(prob, FBAR - E, o)["Pbar"]
        Afd[:, kL] = ((Pp - Pm) / (2 * h)).reshape(9)
    assert np.abs(A - Afd).max() <= 1e-6 * np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-10 * np.abs(A).max()
