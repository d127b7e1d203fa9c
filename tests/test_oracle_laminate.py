"""Pins of the oracle's composite boxel law (paper Sec. 4) to what the paper and
the mathematics fix: volume preservation (matrix determinant lemma), traction
continuity, the energy the jump vector minimises (found here by an independent
root solve), the consistent tangent (finite differences), its symmetry, frame
invariance, the small-strain closed form of the appendix cheat sheet, and the
admissibility guarantee of the selective back-projection (Sec. 4.2, 6.4)."""
import numpy as np
import pytest
from scipy import optimize

from oracle import laminate, material

MINUS = (1.0, 2.0)
PLUS = (10.0, 20.0)


def rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def cases(seed, m, amp=0.2, crange=(0.05, 0.95)):
    rng = np.random.default_rng(seed)
    F = np.eye(3) + rng.uniform(-amp, amp, (m, 3, 3))
    F[np.linalg.det(F) < 0.3] = np.eye(3) * 1.05
    c = rng.uniform(*crange, m)
    N = rng.normal(size=(m, 3))
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    return F, c, N


def test_volume_average_and_determinant_lemma():
    rng = np.random.default_rng(0)
    F, c, N = cases(1, 40)
    a = rng.normal(scale=0.05, size=(40, 3))
    Fp, Fm = laminate.phase_deformations(F, a, c, N)
    # <F> over the voxel is F_box (Sec. 4.1)
    avg = c[:, None, None] * Fp + (1 - c)[:, None, None] * Fm
    assert np.abs(avg - F).max() <= 1e-15 * 10
    # c+ J+ + c- J- = J_box (lemma of Sec. 4.1), with J from plain determinants
    Jp, Jm, J = np.linalg.det(Fp), np.linalg.det(Fm), np.linalg.det(F)
    assert np.abs(c * Jp + (1 - c) * Jm - J).max() <= 1e-14
    # jump F+ - F- = (1/c+ + 1/c-) a (x) N (appendix cheat sheet)
    jump = Fp - Fm
    ref = ((1 / c + 1 / (1 - c))[:, None, None] * np.einsum("mi,mJ->miJ", a, N))
    assert np.abs(jump - ref).max() <= 1e-14


def test_jump_matrix_maps_a_to_a_outer_N():
    rng = np.random.default_rng(5)
    N = rng.normal(size=(7, 3))
    a = rng.normal(size=(7, 3))
    D = laminate.jump_matrix(N)
    lhs = np.einsum("mpk,mk->mp", D, a)
    assert np.abs(lhs - np.einsum("mi,mJ->miJ", a, N).reshape(7, 9)).max() == 0.0


def test_converged_traction_continuity_and_status():
    F, c, N = cases(2, 200)
    r = laminate.solve(F, c, N, MINUS, PLUS)
    assert np.all(r["status"] == laminate.STATUS_OK)
    f = np.einsum("miJ,mJ->mi", r["Pp"] - r["Pm"], N)
    tp = np.linalg.norm(np.einsum("miJ,mJ->mi", r["Pp"], N), axis=1)
    tm = np.linalg.norm(np.einsum("miJ,mJ->mi", r["Pm"], N), axis=1)
    scale = np.maximum(np.maximum(tp, tm), 1e-3 * 10)
    assert np.all(np.linalg.norm(f, axis=1) <= 1e-11 * scale)
    assert r["iters"].max() <= 12


def _independent_root(F, c, N, mats_minus, mats_plus):
    """Solve traction continuity by scipy's hybrid root finder, building F+-
    here from eq. Fpm without the oracle's helpers."""
    def res(a):
        Fp = F + np.outer(a, N) / c
        Fm = F - np.outer(a, N) / (1 - c)
        Pp = material.stress(Fp[None], *mats_plus)[0]
        Pm = material.stress(Fm[None], *mats_minus)[0]
        return (Pp - Pm) @ N
    sol = optimize.root(res, np.zeros(3), method="hybr", tol=1e-14)
    return sol.x


def test_jump_vector_is_independent_root_and_energy_minimiser():
    F, c, N = cases(3, 25)
    r = laminate.solve(F, c, N, MINUS, PLUS)
    for m in range(25):
        a_ref = _independent_root(F[m], c[m], N[m], MINUS, PLUS)
        assert np.abs(r["a"][m] - a_ref).max() <= 1e-9 * max(1.0, np.abs(a_ref).max())
        # Phi(a) = c+ W+ + c- W- has its minimum there: no coordinate step lowers it
        phi0 = laminate.potential(r["a"][m][None], F[m][None], c[m:m + 1], N[m][None], MINUS, PLUS)[0]
        for e in np.eye(3):
            for s in (1e-4, -1e-4):
                phi = laminate.potential((r["a"][m] + s * e)[None], F[m][None], c[m:m + 1], N[m][None],
                                         MINUS, PLUS)[0]
                assert phi >= phi0


def test_same_material_gives_zero_jump():
    F, c, N = cases(4, 30)
    r = laminate.solve(F, c, N, PLUS, PLUS)
    assert np.abs(r["a"]).max() == 0.0
    assert np.abs(r["P"] - material.stress(F, *PLUS)).max() <= 1e-14 * 100
    assert np.abs(r["A"] - material.tangent(F, *PLUS)).max() <= 1e-12 * 100


def test_consistent_tangent_matches_finite_differences():
    F, c, N = cases(6, 12)
    r = laminate.solve(F, c, N, MINUS, PLUS)
    h = 1e-6
    Afd = np.zeros((12, 9, 9))
    for kL in range(9):
        E = np.zeros((3, 3))
        E[kL // 3, kL % 3] = h
        Pp = laminate.solve(F + E, c, N, MINUS, PLUS)["P"]
        Pm = laminate.solve(F - E, c, N, MINUS, PLUS)["P"]
        Afd[:, :, kL] = ((Pp - Pm) / (2 * h)).reshape(12, 9)
    scale = np.abs(r["A"]).max()
    assert np.abs(r["A"] - Afd).max() <= 1e-7 * scale


def test_tangent_major_symmetry():
    F, c, N = cases(7, 100)
    A = laminate.solve(F, c, N, MINUS, PLUS)["A"]
    assert np.abs(A - np.swapaxes(A, 1, 2)).max() <= 1e-13 * np.abs(A).max()


def test_objectivity():
    rng = np.random.default_rng(8)
    F, c, N = cases(9, 40)
    r = laminate.solve(F, c, N, MINUS, PLUS)
    Q = rotation(rng)
    rq = laminate.solve(np.einsum("ij,mjk->mik", Q, F), c, N, MINUS, PLUS)
    assert np.abs(rq["P"] - np.einsum("ij,mjk->mik", Q, r["P"])).max() <= 1e-12
    assert np.abs(rq["a"] - np.einsum("ij,mj->mi", Q, r["a"])).max() <= 1e-12


def test_small_strain_limit_matches_cheat_sheet():
    """a(I + eps H)/eps -> Delta0^{-1} N.(C- - C+) sym(H) with Delta0 = N.(C+/c+ + C-/c-).N
    (appendix cheat sheet, infinitesimal column)."""
    rng = np.random.default_rng(10)
    Cm = material.isotropic_stiffness(*MINUS).reshape(3, 3, 3, 3)
    Cp = material.isotropic_stiffness(*PLUS).reshape(3, 3, 3, 3)
    for _ in range(10):
        H = rng.normal(size=(3, 3))
        c = rng.uniform(0.1, 0.9)
        N = rng.normal(size=3)
        N /= np.linalg.norm(N)
        eps = 1e-6
        r = laminate.solve((np.eye(3) + eps * H)[None], np.array([c]), N[None], MINUS, PLUS)
        e = 0.5 * (H + H.T)
        Delta0 = np.einsum("J,iJkL,L->ik", N, Cp / c + Cm / (1 - c), N)
        rhs = np.einsum("J,iJkL,kL->i", N, Cm - Cp, e)
        a_lin = np.linalg.solve(Delta0, rhs)
        assert np.abs(r["a"][0] / eps - a_lin).max() <= 1e-4 * np.abs(a_lin).max()


def _hard_cases():
    """High contrast, extreme fractions and compressive loads (Sec. 6.4 setting)."""
    rng = np.random.default_rng(11)
    m = 400
    F = np.eye(3) + rng.uniform(-0.45, 0.45, (m, 3, 3))
    F[:, 0, 0] -= 0.3
    keep = np.linalg.det(F) > 0.05
    F = F[keep]
    m = F.shape[0]
    c = np.where(rng.random(m) < 0.5, rng.uniform(0.97, 0.999, m), rng.uniform(0.001, 0.03, m))
    N = rng.normal(size=(m, 3))
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    return F, c, N


def test_backprojection_keeps_iterates_admissible_where_naive_newton_fails():
    F, c, N = _hard_cases()
    soft, stiff = (1.0, 2.0), (1000.0, 2000.0)
    naive = laminate.solve(F, c, N, soft, stiff, backprojection=False)
    failed = naive["status"] == laminate.STATUS_INADMISSIBLE
    assert failed.sum() >= 5          # the naive update does leave the admissible set
    r = laminate.solve(F, c, N, soft, stiff, trace=True)
    assert r["n_backproj"][failed].min() >= 1
    mb = r["m_beta"]
    bp, bm = r["beta_c"]
    for a in r["history"]:
        beta = np.einsum("mi,mi->m", a, mb)
        assert np.all((beta > bp) & (beta < bm))
        Fp, Fm = laminate.phase_deformations(F, a, c, N)
        assert np.all(np.linalg.det(Fp) > 0) and np.all(np.linalg.det(Fm) > 0)
    ok = r["status"] == laminate.STATUS_OK
    assert ok[failed].mean() >= 0.9
    # where both converge they agree
    both = ok & (naive["status"] == laminate.STATUS_OK)
    assert np.abs(r["P"][both] - naive["P"][both]).max() <= 1e-9 * np.abs(r["P"][both]).max()


def test_backprojection_step_matches_algorithm():
    # a0 admissible, a1 beyond beta_c^-: beta* is the midpoint of a0.m and beta_c^-,
    # and the component of a1 orthogonal to m is kept (eq. backproj:result).
    mb = np.array([[0.6, 0.8, 0.0]])
    a0 = np.array([[0.1, -0.2, 0.3]])
    a1 = np.array([[3.0, 4.0, -1.0]])
    bp, bm = np.array([-0.5]), np.array([0.7])
    a = laminate.backproject(a1, a0, mb, bp, bm)
    beta0 = (a0 * mb).sum()
    assert (a * mb).sum() == pytest.approx(0.5 * (beta0 + 0.7), abs=1e-15)
    perp = lambda v: v - (v * mb).sum() * mb
    assert np.abs(perp(a) - perp(a1)).max() <= 1e-15


def test_stop_bound_holds_between_two_stopping_solves():
    """The per-voxel bound the GPU back-projection parity test asserts holds between
    two oracle solves of the same hard cases (extreme fractions, contrast 1000,
    compression) that stop from different starts, and is tight (1e-12 of the
    stress scale) in the median voxel."""
    from laminate_bound import laminate_stop_bound
    rng = np.random.default_rng(7)
    nv = 512
    c = np.where(rng.random(nv) < 0.5, rng.uniform(0.97, 0.999, nv), rng.uniform(0.001, 0.03, nv))
    N = rng.normal(size=(3, nv))
    N /= np.linalg.norm(N, axis=0)
    mats = ((1.0, 2.0), (1000.0, 2000.0))
    F = np.eye(3)[:, :, None] + rng.uniform(-0.45, 0.45, (3, 3, nv))
    F[0, 0] -= 0.3
    bad = np.linalg.det(np.moveaxis(F, -1, 0)) < 0.05
    F[:, :, bad] = np.eye(3)[:, :, None]
    Fv = np.moveaxis(F, -1, 0)
    r = laminate.solve(Fv, c, N.T, mats[0], mats[1])
    ok = r["status"] == laminate.STATUS_OK
    assert ok.all()
    r2 = laminate.solve(Fv, c, N.T, mats[0], mats[1], a_init=r["a"] * (1.0 + 1e-9))
    bound = laminate_stop_bound(r, c, N.T, mats)
    scale = np.abs(r["P"]).max()
    diff = np.abs(r2["P"] - r["P"]).reshape(nv, 9).max(axis=1)
    assert np.all(diff <= bound + 1e-12 * scale)
    assert np.median(bound) <= 1e-12 * scale
    assert diff.max() > 1e-10 * scale    # the cases are hard: a flat 1e-10 bound would not hold
