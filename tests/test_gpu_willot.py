"""Willot's rotated (HEX8R) discretization on the GPU (combo_set_discretization),
through the C-ABI, against the oracle: both Green operators and the CG operator
on even and odd grids (even n1 keeps its x-Nyquist plane), Newton-CG solves in
FP64 and mixed precision under both laws, the effective tangent, an exact layered
RVE on an even grid, and the 256^3 sphere workload.  Grids from about n1 = 100 on store
the half spectrum in rows padded to a multiple of 16 (zero modes): 128, 192 and 256 cover
that layout."""
import numpy as np
import pytest

from oracle import laminate as olam
from oracle import solver as osol
from oracle import spectral as ospec
from paper_2204_13624_amd import combo, synth

pytestmark = pytest.mark.gpu

MATS = ((1.0, 2.0), (10.0, 20.0))
FBAR = np.array([[1.08, 0.12, -0.03], [0.05, 0.97, 0.04], [-0.02, 0.06, 1.02]])


@pytest.fixture
def ctx():
    c = combo.combo_create(0)
    yield c
    combo.combo_destroy(c)


def setup(ctx, ms, mats=MATS, **opt):
    combo.combo_set_grid(ctx, *ms.n, *ms.l)
    combo.combo_set_discretization(ctx, combo.COMBO_DISC_WILLOT)
    combo.combo_set_materials(ctx, mats)
    combo.combo_set_microstructure(ctx, ms.phase, ms.c, ms.N)
    o = combo.combo_default_options()
    for k, v in opt.items():
        setattr(o, k, v)
    combo.combo_set_options(ctx, o)


def oracle_problem(ms, mats=MATS, law="neo_hooke"):
    return osol.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, mats, law=law, disc="willot")


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


SHAPES = [((8, 6, 4), (1.0, 1.0, 1.0)), ((9, 6, 4), (0.9, 1.2, 0.8)), ((12, 16, 9), (1.0, 1.3, 0.7)),
          ((2, 3, 8), (1.0, 1.0, 1.0)), ((1, 6, 4), (1.0, 1.0, 1.0)), ((16, 18, 12), (1.0, 1.0, 1.0))]


@pytest.mark.parametrize("n,l", SHAPES + [((128, 3, 4), (1.0, 0.7, 1.1))])
def test_green_operators_match_oracle(ctx, n, l):
    ms = synth.random_composite_field(n, 3, frac_composite=0.2, l=l)
    setup(ctx, ms)
    mu0, kappa0 = osol.reference_medium(MATS)
    rng = np.random.default_rng(sum(n))
    tau = rng.normal(size=(9, n[2], n[1], n[0]))
    t5 = tau.reshape(3, 3, n[2], n[1], n[0])
    refs = {combo.COMBO_GREEN_G: ospec.apply_g(t5, n, l, "willot").reshape(tau.shape),
            combo.COMBO_GREEN_GAMMA0: ospec.apply_gamma0(t5, n, l, mu0, kappa0, "willot").reshape(tau.shape)}
    for which, ref in refs.items():
        for prec, tol in ((combo.COMBO_FP64, 1e-12), (combo.COMBO_MIXED, 2e-6)):
            out = np.zeros_like(tau)
            combo.combo_apply_green(ctx, which, prec, tau, out)
            assert rel(out, ref) <= tol, (which, prec)


# x lengths 32, 48, 64 and 128 run the two-stage x pass (with the x-Nyquist bin); the others
# the LDS x pass; 128 and 192 pad the rows (65 -> 80 and 97 -> 112 values)
CG_SHAPES = SHAPES[:3] + [((32, 6, 4), (1.0, 1.0, 1.0)), ((64, 8, 6), (1.0, 0.5, 0.4)), ((48, 9, 4), (1.0, 1.0, 1.0)),
                          ((128, 4, 4), (1.0, 1.0, 1.0)), ((192, 3, 4), (1.2, 1.0, 0.9))]


@pytest.mark.parametrize("n,l", CG_SHAPES)
def test_cg_operator_matches_oracle(ctx, n, l):
    ms = synth.random_composite_field(n, 5, frac_composite=0.3, l=l)
    setup(ctx, ms)
    F = synth.random_F_field(n, 6, amplitude=0.15)
    prob = oracle_problem(ms)
    mu0, kappa0 = osol.reference_medium(MATS)
    _, Av, ok, _, _ = osol.evaluate(F.reshape(3, 3, *F.shape[1:]), prob)
    assert ok
    rng = np.random.default_rng(9)
    p = ospec.apply_g(rng.normal(size=(3, 3, n[2], n[1], n[0])), n, l, "willot")
    ref = ospec.apply_gamma0(osol.apply_tangent(Av, p, prob.shape), n, l, mu0, kappa0, "willot")
    pc = np.ascontiguousarray(p.reshape(9, n[2], n[1], n[0]))
    (_, _, _), (nxv, _, _) = combo.combo_get_schedule(ctx)
    for prec, tol in ((combo.COMBO_FP64, 1e-11), (combo.COMBO_MIXED, 3e-6)):
        o = combo.combo_default_options()
        o.precision = prec
        combo.combo_set_options(ctx, o)
        assert combo.combo_eval_law(ctx, F, None, None, None, None) == combo.COMBO_OK
        for xv in range(nxv):
            combo.combo_set_schedule(ctx, xv, 0, 0)
            q = np.zeros_like(pc)
            combo.combo_apply_operator(ctx, prec, pc, q)
            assert rel(q, ref.reshape(pc.shape)) <= tol, (prec, xv)


@pytest.mark.parametrize("n", [(16, 16, 16), (9, 12, 8), (128, 4, 4)])
def test_solves_match_oracle(ctx, n):
    ms = synth.single_sphere(n, radius=0.3, center=(0.02, -0.03, 0.01))
    ref = osol.solve(oracle_problem(ms), FBAR, osol.Options(tol_newton=1e-10, tol_cg=1e-12))
    setup(ctx, ms, tol_newton=1e-10, tol_cg=1e-12)
    F = np.zeros((9, n[2], n[1], n[0]))
    r = combo.combo_solve(ctx, FBAR, F_out=F)
    assert rel(r["Pbar"], ref["Pbar"]) <= 1e-8
    assert rel(F, ref["F"].reshape(F.shape)) <= 1e-8
    assert rel(r["Pbar_phase"], ref["Pbar_phase"]) <= 1e-8
    setup(ctx, ms, tol_newton=1e-9, tol_cg=1e-6, precision=combo.COMBO_MIXED)
    rm = combo.combo_solve(ctx, FBAR)
    assert rel(rm["Pbar"], ref["Pbar"]) <= 1e-6
    # small strain under the same discretization
    H = FBAR - np.eye(3)
    refl = osol.solve(oracle_problem(ms, law="linear"), np.eye(3) + 0.1 * H, osol.Options(tol_newton=1e-10, tol_cg=1e-12))
    setup(ctx, ms, tol_newton=1e-10, tol_cg=1e-12, law=combo.COMBO_LAW_LINEAR)
    rl = combo.combo_solve(ctx, np.eye(3) + 0.1 * H)
    assert rel(rl["Pbar"], refl["Pbar"]) <= 1e-8


def test_effective_tangent_matches_oracle(ctx):
    ms = synth.single_sphere((8, 8, 8), radius=0.3)
    ref = osol.solve(oracle_problem(ms), FBAR, osol.Options(tol_newton=1e-12, tol_cg=1e-12, want_tangent=True))
    setup(ctx, ms, tol_newton=1e-12, tol_cg=1e-12, want_tangent=1)
    r = combo.combo_solve(ctx, FBAR, want_tangent=True)
    assert rel(r["Abar"], ref["Abar"]) <= 1e-9


def test_layered_rve_is_exact_on_an_even_grid(ctx):
    """Odd layer widths on an even grid: exact under the rotated scheme."""
    ms = synth.layered((8, 2, 4), (1.0, 1.0, 1.0), 0, (-0.5 + 2.3 / 8, -0.5 + 5.6 / 8))
    phi = float(ms.c.mean())
    ref = olam.solve(FBAR[None], np.array([phi]), np.array([[1.0, 0.0, 0.0]]), MATS[0], MATS[1])["P"][0]
    setup(ctx, ms, tol_newton=1e-12, tol_cg=1e-12)
    r = combo.combo_solve(ctx, FBAR)
    assert rel(r["Pbar"], ref) <= 1e-11
    setup(ctx, ms, tol_newton=1e-9, tol_cg=1e-6, precision=combo.COMBO_MIXED)
    assert rel(combo.combo_solve(ctx, FBAR)["Pbar"], ref) <= 1e-7


def test_autotuned_schedule_matches_default(ctx):
    ms = synth.single_sphere((64, 48, 32), radius=0.25)
    setup(ctx, ms, precision=combo.COMBO_MIXED, tol_newton=1e-8, tol_cg=1e-6)
    r0 = combo.combo_solve(ctx, FBAR)
    (_, _, _), counts = combo.combo_get_schedule(ctx)
    sched = combo.combo_autotune(ctx, combo.COMBO_MIXED)
    assert all(0 <= v < c for v, c in zip(sched, counts))
    r1 = combo.combo_solve(ctx, FBAR)
    assert rel(r1["Pbar"], r0["Pbar"]) <= 1e-6
    for xv in range(counts[0]):
        for yv in range(counts[1]):
            combo.combo_set_schedule(ctx, xv, yv, counts[2] - 1)
            assert rel(combo.combo_solve(ctx, FBAR)["Pbar"], r0["Pbar"]) <= 1e-6, (xv, yv)


def test_discretization_switch_and_errors(ctx):
    ms = synth.single_sphere((8, 8, 8), radius=0.3)
    setup(ctx, ms, tol_newton=1e-10, tol_cg=1e-12)
    rw = combo.combo_solve(ctx, FBAR)
    # back to Moulinec-Suquet: the microstructure must be set again
    combo.combo_set_discretization(ctx, combo.COMBO_DISC_MS)
    with pytest.raises(combo.ComboError):
        combo.combo_solve(ctx, FBAR)
    combo.combo_set_materials(ctx, MATS)
    combo.combo_set_microstructure(ctx, ms.phase, ms.c, ms.N)
    rm = combo.combo_solve(ctx, FBAR)
    ref = osol.solve(osol.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS), FBAR,
                     osol.Options(tol_newton=1e-10, tol_cg=1e-12))
    assert rel(rm["Pbar"], ref["Pbar"]) <= 1e-8
    assert rel(rw["Pbar"], rm["Pbar"]) > 1e-6          # the two discretizations differ
    with pytest.raises(combo.ComboError):
        combo.combo_set_discretization(ctx, 7)


def test_full_size_sphere_workload(ctx):
    """The 256^3 sphere workload (first load increment) under the rotated scheme in
    mixed precision: converged, <F> = Fbar, and FP64 agreeing to 1e-6."""
    import torch
    ms, lc = synth.workload_spheres_256()
    dev = torch.device("cuda:0")
    combo.combo_set_grid(ctx, *ms.n, *ms.l)
    combo.combo_set_discretization(ctx, combo.COMBO_DISC_WILLOT)
    combo.combo_set_materials(ctx, lc.mats)
    combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(dev), torch.from_numpy(ms.c).to(dev),
                                   torch.from_numpy(np.ascontiguousarray(ms.N)).to(dev))
    Fb = np.eye(3) + (lc.Fbar - np.eye(3)) / lc.n_increments
    o = combo.combo_default_options()
    o.precision = combo.COMBO_MIXED
    o.tol_newton = 1e-6
    o.tol_cg = 1e-4
    o.max_cg = 20000
    combo.combo_set_options(ctx, o)
    F = torch.zeros((9,) + ms.phase.shape, dtype=torch.float64, device=dev)
    r = combo.combo_solve(ctx, Fb, F_out=F)
    assert r["stats"]["status"] == combo.COMBO_OK and r["stats"]["eta_final"] <= 1e-6
    assert np.abs(F.mean(dim=(1, 2, 3)).cpu().numpy() - Fb.reshape(9)).max() <= 1e-12
    o.precision = combo.COMBO_FP64
    o.tol_cg = 1e-6
    combo.combo_set_options(ctx, o)
    r64 = combo.combo_solve(ctx, Fb)
    assert rel(r["Pbar"], r64["Pbar"]) <= 1e-6


def test_batch_mixes_discretizations():
    """Three rotated-scheme members of different grids and one Moulinec-Suquet member in one
    batch: each equals its single solve and the oracle of its discretization."""
    cases = [(synth.single_sphere((16, 16, 16), radius=0.3), "willot"),
             (synth.random_spheres((24, 16, 12), 3, 0.2, seed=21), "willot"),
             (synth.single_sphere((16, 12, 8), radius=0.3), "ms"),
             (synth.random_spheres((128, 4, 6), 2, 0.2, seed=5), "willot")]   # padded rows
    o = combo.combo_default_options()
    o.tol_newton = 1e-10
    o.tol_cg = 1e-12
    b = combo.combo_batch_create(0)
    try:
        combo.combo_batch_set_options(b, o)
        for i, (ms, disc) in enumerate(cases):
            combo.combo_batch_set_discretization(b, combo.COMBO_DISC_WILLOT if disc == "willot" else combo.COMBO_DISC_MS)
            assert combo.combo_batch_add(b, ms.n, ms.l, MATS, ms.phase, ms.c, ms.N) == i
        with pytest.raises(combo.ComboError):
            combo.combo_batch_set_discretization(b, 5)
        res = combo.combo_batch_solve(b, np.stack([FBAR] * 4), n_increments=[1, 1, 1, 1])
    finally:
        combo.combo_batch_destroy(b)
    for i, (ms, disc) in enumerate(cases):
        assert res["stats"][i]["status"] == combo.COMBO_OK
        ref = osol.solve(osol.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS, disc=disc), FBAR,
                         osol.Options(tol_newton=1e-10, tol_cg=1e-12))
        assert rel(res["Pbar"][i], ref["Pbar"]) <= 1e-8, i
