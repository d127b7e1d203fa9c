"""The staggered grid with the doubly-fine material grid law (paper App. A) on the
GPU against the oracle (oracle/staggered.py through oracle.solver), through the
C-ABI: the staggered Green operators, the DFMG law (Neo-Hooke and laminate
cells), the CG operator with the DFMG tangent, and Newton-CG solves (FP64 and
mixed), plus the exact cases of the oracle's pins (homogeneous RVEs, laminates
under normal loads).

The GPU evaluates each doubly-fine cell once (eight per cell) and sums their
stresses; the oracle evaluates the 32 terms of the printed DFMG sum one by one.
Both are the same sum, so the laws agree to rounding: FP64 1e-12 (laminate cells
to their stopping tolerance), the CG operator 1e-11 (FP64) and 3e-6 (FP32), the
solves 1e-8 (FP64) and 1e-6 (mixed) relative to max |Pbar|."""
import numpy as np
import pytest

from oracle import solver as osol
from oracle import staggered as ost
from paper_2204_13624_amd import combo, synth

pytestmark = pytest.mark.gpu

MATS = ((1.0, 2.0), (10.0, 20.0))


@pytest.fixture
def ctx():
    c = combo.combo_create(0)
    yield c
    combo.combo_destroy(c)


def setup(ctx, ms, mats=MATS, **opt):
    combo.combo_set_grid(ctx, *ms.n, *ms.l)
    combo.combo_set_discretization(ctx, combo.COMBO_DISC_STAGGERED)
    combo.combo_set_materials(ctx, mats)
    combo.combo_set_microstructure(ctx, ms.phase, ms.c, ms.N)
    o = combo.combo_default_options()
    for k, v in opt.items():
        setattr(o, k, v)
    combo.combo_set_options(ctx, o)


def problem(ms, mats=MATS):
    return osol.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, mats, disc="staggered")


def rel(a, b):
    a, b = np.asarray(a, float).ravel(), np.asarray(b, float).ravel()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def compatible(n, l, seed, amp=0.05):
    """Grad U of a random displacement scaled so that the gradient entries are ~amp."""
    h = tuple(l[d] / n[d] for d in range(3))
    U = amp * min(h) * np.random.default_rng(seed).normal(size=(3, n[2], n[1], n[0]))
    return ost.grad(U, h)


@pytest.mark.parametrize("n,l", [((8, 6, 4), (1.0, 0.9, 0.7)), ((9, 8, 6), (1.2, 1.0, 0.8)),
                                 ((16, 12, 9), (1.0, 1.0, 1.0)), ((32, 8, 9), (2.0, 0.5, 0.6)),
                                 ((1, 4, 6), (0.3, 1.0, 1.0)), ((128, 6, 4), (1.0, 0.2, 0.1)),
                                 ((4, 128, 3), (0.2, 1.0, 0.3)), ((3, 4, 128), (0.2, 0.3, 1.0)),
                                 ((2, 96, 48), (0.1, 1.0, 0.5)), ((2, 64, 256), (0.1, 0.3, 1.0))])
@pytest.mark.parametrize("which", [combo.COMBO_GREEN_GAMMA0, combo.COMBO_GREEN_G])
def test_staggered_green_operators_match_oracle(ctx, n, l, which):
    rng = np.random.default_rng(3)
    combo.combo_set_grid(ctx, *n, *l)
    combo.combo_set_discretization(ctx, combo.COMBO_DISC_STAGGERED)
    combo.combo_set_materials(ctx, MATS)
    tau = rng.normal(size=(9, n[2], n[1], n[0]))
    t5 = tau.reshape(3, 3, n[2], n[1], n[0])
    mu0, kappa0 = osol.reference_medium(MATS)
    ref = (ost.apply_gamma0(t5, n, l, mu0, kappa0) if which == combo.COMBO_GREEN_GAMMA0
           else ost.apply_g(t5, n, l)).reshape(tau.shape)
    out = np.zeros_like(tau)
    combo.combo_apply_green(ctx, which, combo.COMBO_FP64, tau, out)
    assert rel(out, ref) <= 1e-12
    out32 = np.zeros_like(tau)
    combo.combo_apply_green(ctx, which, combo.COMBO_MIXED, tau, out32)
    assert rel(out32, ref) <= 2e-6


@pytest.mark.parametrize("n,seed,amp", [((6, 4, 4), 1, 0.05), ((9, 8, 6), 2, 0.08), ((16, 4, 3), 3, 0.06)])
def test_dfmg_law_matches_oracle(ctx, n, seed, amp):
    ms = synth.random_composite_field(n, seed, frac_composite=0.5)
    assert ms.n_composite > 0 and (ms.phase == 0).any() and (ms.phase == 1).any()
    setup(ctx, ms)
    l = ms.l
    F = np.eye(3)[:, :, None, None, None] + compatible(n, l, seed + 10, amp) \
        + amp * np.array([[0.3, 0.5, -0.1], [0.2, -0.4, 0.3], [-0.2, 0.1, 0.2]])[:, :, None, None, None]
    F9 = np.ascontiguousarray(F.reshape(9, n[2], n[1], n[0]))
    P = np.zeros_like(F9)
    st = combo.combo_eval_law(ctx, F9, P)
    assert st == combo.COMBO_OK, combo.combo_last_error(ctx)
    Po, _, ok, _, _ = ost.evaluate(F, problem(ms))
    assert ok
    assert rel(P, Po.reshape(P.shape)) <= 1e-11


# rows of 48, 96, 128 and 256 run the two-stage x passes on real fields (8x6, 8x12, 8x16, 16x16)
@pytest.mark.parametrize("n", [(8, 6, 4), (12, 9, 8), (32, 16, 8), (48, 6, 4), (96, 4, 3), (128, 4, 3), (256, 3, 2),
                               (4, 128, 3), (3, 4, 128), (2, 64, 48)])
@pytest.mark.parametrize("precision,tol", [(combo.COMBO_FP64, 1e-11), (combo.COMBO_MIXED, 3e-6)])
def test_staggered_cg_operator_matches_oracle(ctx, n, precision, tol):
    ms = synth.random_composite_field(n, 5, frac_composite=0.3)
    setup(ctx, ms, precision=precision)
    l = ms.l
    F = np.eye(3)[:, :, None, None, None] + compatible(n, l, 6, 0.05)
    F9 = np.ascontiguousarray(F.reshape(9, n[2], n[1], n[0]))
    assert combo.combo_eval_law(ctx, F9, None) == combo.COMBO_OK, combo.combo_last_error(ctx)
    _, terms, ok, _, _ = ost.evaluate(F, problem(ms))
    assert ok
    mu0, kappa0 = osol.reference_medium(MATS)
    p = compatible(n, l, 7, 1.0)
    ref = ost.apply_gamma0(ost.tangent_action(terms, p), n, l, mu0, kappa0)
    q = np.zeros((9, n[2], n[1], n[0]))
    combo.combo_apply_operator(ctx, precision, np.ascontiguousarray(p.reshape(q.shape)), q)
    assert rel(q, ref.reshape(q.shape)) <= tol


FBAR = np.array([[1.08, 0.12, -0.03], [0.05, 0.97, 0.04], [-0.02, 0.06, 1.02]])


def test_staggered_homogeneous_rves_are_exact(ctx):
    for ph in (0, 1):
        ms = synth.homogeneous((6, 4, 3), phase_id=ph)
        setup(ctx, ms, tol_newton=1e-12, tol_cg=1e-12)
        F = np.zeros((9, 3, 4, 6))
        r = combo.combo_solve(ctx, FBAR, F_out=F)
        assert r["stats"]["newton_iters"] == 0
        assert np.abs(F - FBAR.reshape(9, 1, 1, 1)).max() <= 1e-15
        ref = ost.evaluate(np.broadcast_to(FBAR[:, :, None, None, None], (3, 3, 3, 4, 6)).copy(),
                           problem(ms))[0].mean(axis=(2, 3, 4))
        assert rel(r["Pbar"], ref) <= 1e-14


@pytest.mark.parametrize("n,l,axis,interfaces", [
    ((9, 2, 3), (1.0, 1.0, 1.0), 0, (-0.5 + 2.25 / 9, -0.5 + 6.5 / 9)),
    ((3, 9, 2), (1.0, 1.4, 1.0), 1, (-0.7 + 1.4 * 2.25 / 9, -0.7 + 1.4 * 6.5 / 9)),
    ((2, 3, 8), (1.0, 0.8, 2.0), 2, (-1.0 + 2 * 1.25 / 8, -1.0 + 2 * 5.5 / 8)),
])
@pytest.mark.parametrize("precision,tol", [(combo.COMBO_FP64, 1e-11), (combo.COMBO_MIXED, 1e-6)])
def test_staggered_laminate_under_normal_load(ctx, n, l, axis, interfaces, precision, tol):
    """Layers through composite cells under a diagonal load: the staggered solve is the
    exact laminate (oracle pin), on the GPU as in the oracle."""
    ms = synth.layered(n, l, axis, interfaces)
    assert ms.n_composite > 0
    Fd = np.diag([1.06, 0.97, 1.02])
    setup(ctx, ms, precision=precision, tol_newton=1e-10 if precision == combo.COMBO_FP64 else 1e-8,
          tol_cg=1e-12 if precision == combo.COMBO_FP64 else 1e-5)
    r = combo.combo_solve(ctx, Fd)
    ref = osol.solve(problem(ms), Fd, osol.Options(tol_newton=1e-12, tol_cg=1e-12))
    assert rel(r["Pbar"], ref["Pbar"]) <= tol
    assert rel(r["Pbar_phase"], ref["Pbar_phase"]) <= tol


@pytest.mark.parametrize("n,K", [((8, 8, 8), 1), ((9, 8, 6), 2)])
@pytest.mark.parametrize("precision", [combo.COMBO_FP64, combo.COMBO_MIXED], ids=["fp64", "mixed"])
def test_staggered_sphere_solve_matches_oracle(ctx, n, K, precision):
    ms = synth.single_sphere(n, radius=0.3, center=(0.04, -0.02, 0.03))
    assert ms.n_composite > 0
    mats = synth.contrast_mats(20.0)
    fp64 = precision == combo.COMBO_FP64
    ref = osol.solve(problem(ms, mats), FBAR, osol.Options(tol_newton=1e-11, tol_cg=1e-12, n_increments=K))
    setup(ctx, ms, mats, precision=precision, n_increments=K, tol_newton=1e-10 if fp64 else 1e-8,
          tol_cg=1e-12 if fp64 else 1e-5)
    F = np.zeros((9, n[2], n[1], n[0]))
    P = np.zeros_like(F)
    r = combo.combo_solve(ctx, FBAR, F_out=F, P_out=P)
    bar = 1e-8 if fp64 else 1e-6
    assert rel(r["Pbar"], ref["Pbar"]) <= bar
    assert rel(r["Pbar_phase"], ref["Pbar_phase"]) <= bar
    assert rel(F, ref["F"].reshape(F.shape)) <= (1e-8 if fp64 else 1e-5)
    assert rel(P, ref["P"].reshape(P.shape)) <= (1e-8 if fp64 else 1e-5)
    assert np.abs(F.reshape(3, 3, -1).mean(axis=2) - FBAR).max() <= 1e-12


@pytest.mark.parametrize("precision,tol", [(combo.COMBO_FP64, 1e-9), (combo.COMBO_MIXED, 2e-5)],
                         ids=["fp64", "mixed"])
def test_staggered_effective_tangent_matches_oracle(ctx, precision, tol):
    ms = synth.single_sphere((8, 6, 6), radius=0.3, center=(0.04, -0.02, 0.03))
    assert ms.n_composite > 0
    mats = synth.contrast_mats(10.0)
    fp64 = precision == combo.COMBO_FP64
    ref = osol.solve(problem(ms, mats), FBAR, osol.Options(tol_newton=1e-11, tol_cg=1e-12, want_tangent=True))
    setup(ctx, ms, mats, precision=precision, tol_newton=1e-10 if fp64 else 1e-8, tol_cg=1e-12 if fp64 else 1e-6,
          want_tangent=1)
    r = combo.combo_solve(ctx, FBAR, want_tangent=True)
    assert r["stats"]["cg_iters_tangent"] > 0
    assert rel(r["Abar"], ref["Abar"]) <= tol, rel(r["Abar"], ref["Abar"])
    assert rel(r["Pbar"], ref["Pbar"]) <= (1e-8 if fp64 else 1e-6)


def test_staggered_refusals(ctx):
    ms = synth.single_sphere((6, 6, 6), radius=0.3)
    setup(ctx, ms)
    F = np.broadcast_to(np.eye(3).reshape(9, 1, 1, 1), (9, 6, 6, 6)).copy()
    A = np.zeros((81, 6, 6, 6))
    assert combo.combo_eval_law(ctx, F, None, A) == combo.COMBO_E_INVAL
    o = combo.combo_default_options()
    o.law = combo.COMBO_LAW_LINEAR
    combo.combo_set_options(ctx, o)
    with pytest.raises(combo.ComboError):
        combo.combo_solve(ctx, FBAR)
    b = combo.combo_batch_create(0)
    try:
        with pytest.raises(combo.ComboError):
            combo.combo_batch_set_discretization(b, combo.COMBO_DISC_STAGGERED)
    finally:
        combo.combo_batch_destroy(b)
