"""GPU (HIP, gfx950) against the FP64 CPU oracle, through the C-ABI.

Tolerances: the FP64 path computes the same quantities as the oracle with a
different operation order (FFT factorisation, laminate determinant by the
matrix-determinant lemma, blocked reductions), so pointwise results agree to
~1e2 ulp and solves to the Newton/CG tolerances.  The FP32 ("mixed") linear
solves carry float32 rounding (~6e-8 relative per operation, growing with
log n over the FFT passes).
"""
import numpy as np
import pytest

from oracle import laminate as olam
from oracle import material as omat
from oracle import solver as osol
from oracle import spectral as ospec
from paper_2204_13624_amd import combo, synth

from laminate_bound import laminate_stop_bound

pytestmark = pytest.mark.gpu

MATS = ((1.0, 2.0), (10.0, 20.0))


@pytest.fixture
def ctx():
    c = combo.combo_create(0)
    yield c
    combo.combo_destroy(c)


def setup(ctx, ms, mats=MATS, **opt):
    combo.combo_set_grid(ctx, *ms.n, *ms.l)
    combo.combo_set_materials(ctx, mats)
    combo.combo_set_microstructure(ctx, ms.phase, ms.c, ms.N)
    o = combo.combo_default_options()
    for k, v in opt.items():
        setattr(o, k, v)
    combo.combo_set_options(ctx, o)


def oracle_problem(ms, mats=MATS):
    return osol.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, mats)


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


# ---------------------------------------------------------------------------------
# pointwise law (pure Neo-Hooke + laminate) voxel by voxel
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed,amp", [((9, 6, 4), 1, 0.15), ((16, 12, 6), 2, 0.3), ((1, 1, 1), 3, 0.2)])
def test_law_matches_oracle_per_voxel(ctx, n, seed, amp):
    ms = synth.random_composite_field(n, seed, frac_composite=0.6)
    setup(ctx, ms)
    F = synth.random_F_field(n, seed + 100, amplitude=amp)
    nv = ms.nvox
    P = np.zeros_like(F)
    A = np.zeros((81,) + F.shape[1:])
    a = np.zeros((3,) + F.shape[1:])
    it = np.zeros(F.shape[1:], dtype=np.int32)
    st = combo.combo_eval_law(ctx, F, P, A, a, it)
    assert st == combo.COMBO_OK, combo.combo_last_error(ctx)
    prob = oracle_problem(ms)
    Fo = F.reshape(3, 3, *F.shape[1:])
    Po, Av, ok, _, lp = osol.evaluate(Fo, prob)
    assert ok
    assert rel(P.reshape(9, nv), Po.reshape(9, nv)) <= 1e-12
    Ag = np.moveaxis(A.reshape(81, nv), 0, 1)
    assert rel(Ag, Av.reshape(nv, 81)) <= 1e-10
    if lp:
        ag = a.reshape(3, nv)[:, lp["idx"]].T
        assert np.abs(ag - lp["a"]).max() <= 1e-11 * max(1.0, np.abs(lp["a"]).max())


def test_law_nearly_incompressible_matches_oracle(ctx):
    """lambda/mu = 1000 in both phases, fibre contrast 1000 (the fibre workload's materials): the FP64
    det F / ln J path and the laminate's round-off floor."""
    n = (16, 12, 6)
    mats = ((1.0, 1000.0), (1000.0, 1.0e6))
    ms = synth.random_composite_field(n, 4, frac_composite=0.6)
    setup(ctx, ms, mats)
    nv = ms.nvox
    for amp in (1e-4, 0.02):
        F = synth.random_F_field(n, 8, amplitude=amp)
        P = np.zeros_like(F)
        A = np.zeros((81,) + F.shape[1:])
        a = np.zeros((3,) + F.shape[1:])
        it = np.zeros(F.shape[1:], dtype=np.int32)
        assert combo.combo_eval_law(ctx, F, P, A, a, it) == combo.COMBO_OK, combo.combo_last_error(ctx)
        Po, Av, ok, st, lp = osol.evaluate(F.reshape(3, 3, *F.shape[1:]), oracle_problem(ms, mats))
        assert ok and st["lam_fail"] == 0
        assert rel(P.reshape(9, nv), Po.reshape(9, nv)) <= 1e-11, amp
        assert rel(np.moveaxis(A.reshape(81, nv), 0, 1), Av.reshape(nv, 81)) <= 1e-9, amp
        ag = a.reshape(3, nv)[:, lp["idx"]].T
        assert np.abs(ag - lp["a"]).max() <= 1e-9 * max(1e-3, np.abs(lp["a"]).max()), amp
        assert int(it.max()) < 50   # no laminate at the update cap


def test_law_backprojection_cases_match_oracle(ctx):
    """Extreme fractions, contrast 1000 and compression: the back-projection path."""
    n = (16, 8, 4)
    rng = np.random.default_rng(7)
    nv = n[0] * n[1] * n[2]
    phase = np.full((n[2], n[1], n[0]), 2, np.uint8)
    c = np.where(rng.random(nv) < 0.5, rng.uniform(0.97, 0.999, nv), rng.uniform(0.001, 0.03, nv))
    N = rng.normal(size=(3, nv))
    N /= np.linalg.norm(N, axis=0)
    ms = synth.Microstructure(n=n, l=(1.0, 1.0, 1.0), phase=phase, c=c.reshape(phase.shape),
                              N=N.reshape(3, *phase.shape), info={})
    mats = ((1.0, 2.0), (1000.0, 2000.0))
    setup(ctx, ms, mats)
    F = np.eye(3)[:, :, None] + rng.uniform(-0.45, 0.45, (3, 3, nv))
    F[0, 0] -= 0.3
    bad = np.linalg.det(np.moveaxis(F, -1, 0)) < 0.05
    F[:, :, bad] = np.eye(3)[:, :, None]
    F = F.reshape(9, *phase.shape)
    P = np.zeros_like(F)
    it = np.zeros(phase.shape, dtype=np.int32)
    st = combo.combo_eval_law(ctx, F, P, None, None, it)
    Fv = np.moveaxis(F.reshape(3, 3, nv), -1, 0)
    r = olam.solve(Fv, c, N.T, mats[0], mats[1])
    ok = r["status"] == olam.STATUS_OK
    assert st == combo.COMBO_OK or not ok.all()
    naive = olam.solve(Fv, c, N.T, mats[0], mats[1], backprojection=False)
    assert (naive["status"] == olam.STATUS_INADMISSIBLE).sum() >= 5
    Pg = np.moveaxis(P.reshape(3, 3, nv), -1, 0)
    bound = laminate_stop_bound(r, c, N.T, mats)
    scale = np.abs(r["P"][ok]).max()
    diff = np.abs(Pg - r["P"]).reshape(nv, 9).max(axis=1)
    assert np.all(diff[ok] <= bound[ok] + 1e-12 * scale), np.max(diff[ok] / (bound[ok] + 1e-12 * scale))
    # the bound is loose only where a soft phase is nearly collapsed
    assert np.median(bound[ok]) <= 1e-12 * scale



# ---------------------------------------------------------------------------------
# spectral operators
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("n,l", [((16, 16, 16), (1.0, 1.0, 1.0)), ((9, 6, 12), (2.0, 0.5, 1.3)),
                                 ((48, 18, 27), (1.0, 1.0, 2.0)), ((2, 1, 3), (1.0, 1.0, 1.0)),
                                 ((96, 8, 4), (1.0, 0.3, 0.3)), ((256, 6, 3), (2.0, 0.5, 0.25)),
                                 ((128, 32, 4), (1.0, 1.0, 1.0)), ((64, 64, 32), (1.0, 0.7, 1.0)),
                                 ((9, 256, 2), (1.0, 1.0, 1.0)), ((6, 4, 256), (0.5, 1.0, 3.0)),
                                 ((12, 128, 64), (1.0, 1.0, 1.0)), ((384, 2, 2), (1.0, 1.0, 1.0)),
                                 ((192, 3, 2), (1.0, 1.0, 1.0)), ((12, 48, 96), (1.0, 1.0, 1.0)),
                                 ((6, 96, 48), (1.0, 2.0, 1.0))])
@pytest.mark.parametrize("which", [combo.COMBO_GREEN_GAMMA0, combo.COMBO_GREEN_G])
def test_green_operators_match_oracle(ctx, n, l, which):
    rng = np.random.default_rng(11)
    combo.combo_set_grid(ctx, *n, *l)
    combo.combo_set_materials(ctx, MATS)
    tau = rng.normal(size=(9, n[2], n[1], n[0]))
    mu0, kappa0 = osol.reference_medium(MATS)
    t5 = tau.reshape(3, 3, n[2], n[1], n[0])
    ref = (ospec.apply_gamma0(t5, n, l, mu0, kappa0) if which == combo.COMBO_GREEN_GAMMA0
           else ospec.apply_g(t5, n, l)).reshape(9, n[2], n[1], n[0])
    out = np.zeros_like(tau)
    combo.combo_apply_green(ctx, which, combo.COMBO_FP64, tau, out)
    assert rel(out, ref) <= 1e-12
    out32 = np.zeros_like(tau)
    combo.combo_apply_green(ctx, which, combo.COMBO_MIXED, tau, out32)
    assert rel(out32, ref) <= 2e-6


@pytest.mark.parametrize("n", [(12, 9, 8), (64, 32, 16), (256, 4, 8), (48, 64, 32), (48, 48, 48), (12, 96, 96)])
@pytest.mark.parametrize("precision,tol", [(combo.COMBO_FP64, 1e-11), (combo.COMBO_MIXED, 3e-6)])
def test_cg_operator_matches_oracle(ctx, precision, tol, n):
    ms = synth.random_composite_field(n, 5, frac_composite=0.3)
    setup(ctx, ms, precision=precision)
    F = synth.random_F_field(n, 6, amplitude=0.15)
    assert combo.combo_eval_law(ctx, F, None, None, None, None) == combo.COMBO_OK
    prob = oracle_problem(ms)
    mu0, kappa0 = osol.reference_medium(MATS)
    _, Av, ok, _, _ = osol.evaluate(F.reshape(3, 3, *F.shape[1:]), prob)
    rng = np.random.default_rng(9)
    p = ospec.apply_g(rng.normal(size=(3, 3, n[2], n[1], n[0])), n, (1.0, 1.0, 1.0))   # compatible, zero mean
    ref = ospec.apply_gamma0(osol.apply_tangent(Av, p, prob.shape), n, (1.0, 1.0, 1.0), mu0, kappa0)
    q = np.zeros((9, n[2], n[1], n[0]))
    combo.combo_apply_operator(ctx, precision, np.ascontiguousarray(p.reshape(9, n[2], n[1], n[0])), q)
    assert rel(q, ref.reshape(q.shape)) <= tol


# ---------------------------------------------------------------------------------
# full solves
# ---------------------------------------------------------------------------------
FBAR = np.array([[1.08, 0.12, -0.03], [0.05, 0.97, 0.04], [-0.02, 0.06, 1.02]])


def test_single_sphere_16_fp64_and_mixed(ctx):
    ms, lc = synth.workload_single_sphere_16()
    ref = osol.solve(oracle_problem(ms, lc.mats), lc.Fbar, osol.Options(tol_newton=1e-10, tol_cg=1e-12))
    setup(ctx, ms, lc.mats, tol_newton=1e-10, tol_cg=1e-12)
    F = np.zeros((9, 16, 16, 16))
    P = np.zeros_like(F)
    r = combo.combo_solve(ctx, lc.Fbar, F_out=F, P_out=P)
    assert rel(r["Pbar"], ref["Pbar"]) <= 1e-8
    assert rel(F, ref["F"].reshape(9, 16, 16, 16)) <= 1e-8
    assert rel(P, ref["P"].reshape(9, 16, 16, 16)) <= 1e-7
    assert r["stats"]["eta_final"] <= 1e-10
    assert rel(r["Pbar_phase"], ref["Pbar_phase"]) <= 1e-8
    setup(ctx, ms, lc.mats, tol_newton=1e-9, tol_cg=1e-6, precision=combo.COMBO_MIXED)
    rm = combo.combo_solve(ctx, lc.Fbar)
    assert rel(rm["Pbar"], ref["Pbar"]) <= 1e-6


@pytest.mark.parametrize("n,l", [((24, 18, 12), (1.0, 1.0, 1.0)), ((9, 27, 6), (0.5, 1.5, 0.4))])
def test_ragged_grids_match_oracle(ctx, n, l):
    ms = synth.single_sphere(n, l=l, radius=0.3 * min(l), center=(0.02, -0.03, 0.01))
    ref = osol.solve(oracle_problem(ms), FBAR, osol.Options(tol_newton=1e-11, tol_cg=1e-12))
    setup(ctx, ms, tol_newton=1e-11, tol_cg=1e-12)
    r = combo.combo_solve(ctx, FBAR)
    assert rel(r["Pbar"], ref["Pbar"]) <= 1e-8


def test_homogeneous_and_laminate_pins_on_gpu(ctx):
    ms = synth.homogeneous((8, 6, 4), phase_id=1)
    setup(ctx, ms, tol_newton=1e-12, tol_cg=1e-12)
    F = np.zeros((9, 4, 6, 8))
    r = combo.combo_solve(ctx, FBAR, F_out=F)
    assert r["stats"]["newton_iters"] == 0
    assert np.abs(F - FBAR.reshape(9, 1, 1, 1)).max() <= 1e-15
    ms = synth.layered((9, 2, 3), (1.0, 1.0, 1.0), 0, (-0.5 + 2.25 / 9, -0.5 + 6.5 / 9))
    setup(ctx, ms, tol_newton=1e-12, tol_cg=1e-12)
    r = combo.combo_solve(ctx, FBAR)
    ref = osol.solve(oracle_problem(ms), FBAR, osol.Options(tol_newton=1e-12, tol_cg=1e-12))
    assert rel(r["Pbar"], ref["Pbar"]) <= 1e-11


def test_nearly_incompressible_solve_matches_oracle(ctx):
    """Stiff nearly incompressible sphere in a nearly incompressible matrix under shear."""
    ms = synth.single_sphere((12, 12, 12), radius=0.3, center=(0.03, -0.02, 0.01))
    mats = ((1.0, 1000.0), (30.0, 30000.0))
    Fb = synth.shear12(0.02)
    ref = osol.solve(oracle_problem(ms, mats), Fb, osol.Options(tol_newton=1e-10, tol_cg=1e-12, n_increments=2))
    setup(ctx, ms, mats, tol_newton=1e-10, tol_cg=1e-12, n_increments=2)
    r = combo.combo_solve(ctx, Fb)
    assert rel(r["Pbar"], ref["Pbar"]) <= 1e-8
    setup(ctx, ms, mats, tol_newton=1e-7, tol_cg=1e-5, n_increments=2, precision=combo.COMBO_MIXED)
    rm = combo.combo_solve(ctx, Fb)
    assert rel(rm["Pbar"], ref["Pbar"]) <= 1e-6


def test_effective_tangent_matches_oracle(ctx):
    ms = synth.single_sphere((8, 8, 8), radius=0.3)
    opts = osol.Options(tol_newton=1e-12, tol_cg=1e-12, want_tangent=True)
    ref = osol.solve(oracle_problem(ms), FBAR, opts)
    setup(ctx, ms, tol_newton=1e-12, tol_cg=1e-12, want_tangent=1)
    r = combo.combo_solve(ctx, FBAR, want_tangent=True)
    assert rel(r["Abar"], ref["Abar"]) <= 1e-9
    setup(ctx, ms, tol_newton=1e-11, tol_cg=1e-6, want_tangent=1, precision=combo.COMBO_MIXED)
    rm = combo.combo_solve(ctx, FBAR, want_tangent=True)
    assert rel(rm["Abar"], ref["Abar"]) <= 1e-5


def test_increments_match_oracle(ctx):
    ms = synth.single_sphere((12, 12, 12), radius=0.35)
    mats = ((1.0, 2.0), (100.0, 200.0))
    o = osol.Options(tol_newton=1e-10, tol_cg=1e-11, n_increments=4)
    ref = osol.solve(oracle_problem(ms, mats), synth.stretch(0.2), o)
    setup(ctx, ms, mats, tol_newton=1e-10, tol_cg=1e-11, n_increments=4)
    r = combo.combo_solve(ctx, synth.stretch(0.2))
    assert r["stats"]["increments_done"] == 4
    assert rel(r["Pbar"], ref["Pbar"]) <= 1e-8


NEGCURV_FBAR = np.eye(3) - 0.05 * np.array([[1.0, 0.3, 0.0], [0.2, -0.5, 0.0], [0.0, 0.0, 0.2]])


def test_negative_curvature_truncated_newton_matches_oracle(ctx):
    """Stiff sphere, 5 % compression in one increment: CG meets negative
    curvature at the predictor and the Newton step is truncated."""
    ms = synth.single_sphere((8, 8, 8), radius=0.3, center=(0.05, -0.02, 0.03))
    mats = synth.contrast_mats(100.0)
    ref = osol.solve(oracle_problem(ms, mats), NEGCURV_FBAR, osol.Options(tol_newton=1e-11, tol_cg=1e-12))
    assert ref["stats"]["cg_truncations"] >= 1
    setup(ctx, ms, mats, tol_newton=1e-11, tol_cg=1e-12)
    r = combo.combo_solve(ctx, NEGCURV_FBAR)
    assert r["stats"]["cg_truncations"] >= 1
    assert rel(r["Pbar"], ref["Pbar"]) <= 1e-8
    setup(ctx, ms, mats, tol_newton=1e-8, tol_cg=1e-6, precision=combo.COMBO_MIXED)
    rm = combo.combo_solve(ctx, NEGCURV_FBAR)
    assert rm["stats"]["cg_truncations"] >= 1
    assert rel(rm["Pbar"], ref["Pbar"]) <= 1e-6


def test_error_paths(ctx):
    ms = synth.single_sphere((8, 8, 8), radius=0.3)
    setup(ctx, ms)
    with pytest.raises(combo.ComboError) as e:
        combo.combo_solve(ctx, np.diag([1.0, 1.0, -1.0]))
    assert e.value.status == combo.COMBO_E_INADMISSIBLE
    with pytest.raises(combo.ComboError) as e:
        combo.combo_set_grid(ctx, 10, 8, 8)
    assert e.value.status == combo.COMBO_E_SIZE
    combo.combo_set_grid(ctx, 8, 8, 8)
    combo.combo_set_materials(ctx, MATS)
    combo.combo_set_microstructure(ctx, ms.phase, ms.c, ms.N)
    o = combo.combo_default_options()
    o.max_cg = 1
    combo.combo_set_options(ctx, o)
    with pytest.raises(combo.ComboError) as e:
        combo.combo_solve(ctx, FBAR)
    assert e.value.status == combo.COMBO_E_NOCONV


def test_profile_select_times_only_the_chosen_classes(ctx):
    ms = synth.single_sphere((16, 16, 16), radius=0.3)
    setup(ctx, ms, precision=combo.COMBO_MIXED, tol_newton=1e-8, tol_cg=1e-6)
    r0 = combo.combo_solve(ctx, FBAR)
    combo.combo_profile_select(ctx, [0])   # the x pass of the CG operator only
    combo.combo_profile_enable(ctx, True)
    r1 = combo.combo_solve(ctx, FBAR)
    prof = combo.combo_profile_all(ctx)
    combo.combo_profile_enable(ctx, False)
    assert prof["xpass_cg"][1] > 0 and prof["xpass_cg"][0] > 0
    assert all(v[1] == 0 for k, v in prof.items() if k != "xpass_cg")
    assert np.array_equal(r0["Pbar"], r1["Pbar"])
    combo.combo_profile_select(ctx, None)
    combo.combo_profile_enable(ctx, True)
    combo.combo_solve(ctx, FBAR)
    prof = combo.combo_profile_all(ctx)
    combo.combo_profile_enable(ctx, False)
    assert prof["ypass_fwd"][1] > 0 and prof["cg_update"][1] > 0 and prof["material"][1] > 0
