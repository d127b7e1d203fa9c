"""Batched solves (many RVEs of uneven grids in shared launches) through the C-ABI.

A member solved in a batch runs the same kernel code on the same data, with
the same per-member reductions, as the member solved alone.  The batched
kernels are separately compiled instances of that code, and the compiler may
fuse multiply-adds differently in them, so FP64 results agree to rounding
rather than bit for bit: a stopping test (CG, laminate Newton) may move by an
iteration, so iteration totals agree within a small margin and the fields to
well below the solver tolerances; in mixed precision the effective stress is
compared at the mixed-mode accuracy.  Members are also checked against the FP64 oracle.
"""
import numpy as np
import pytest

from oracle import material as omat
from oracle import solver as osol
from paper_2204_13624_amd import combo, synth

pytestmark = pytest.mark.gpu

FBAR = np.array([[1.08, 0.12, -0.03], [0.05, 0.97, 0.04], [-0.02, 0.06, 1.02]])


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def members():
    """Uneven grids, two members per kernel shape in places, different loads and contrasts."""
    rng = np.random.Generator(np.random.PCG64(11))
    out = []
    out.append((synth.single_sphere((16, 16, 16), radius=0.3), ((1.0, 2.0), (10.0, 20.0)), FBAR, 1))
    out.append((synth.single_sphere((16, 16, 16), radius=0.22, center=(0.1, 0.0, -0.05)), synth.contrast_mats(100.0),
                synth.stretch(0.1), 2))
    out.append((synth.single_sphere((12, 9, 8), l=(1.0, 0.8, 0.6), radius=0.2), synth.contrast_mats(30.0),
                synth.shear12(0.08), 1))
    out.append((synth.single_sphere((6, 9, 8), l=(0.5, 0.8, 0.6), radius=0.15), synth.contrast_mats(5.0),
                synth.random_Fbar_ball(rng, 0.1), 1))
    out.append((synth.random_spheres((24, 24, 24), 3, 0.15, 5), synth.contrast_mats(300.0),
                synth.random_Fbar_ball(rng, 0.1), 3))
    out.append((synth.homogeneous((8, 6, 4), phase_id=1), ((1.0, 2.0), (10.0, 20.0)), FBAR, 1))
    # negative curvature at the predictor: a truncated Newton step
    out.append((synth.single_sphere((8, 8, 8), radius=0.3, center=(0.05, -0.02, 0.03)), synth.contrast_mats(100.0),
                np.eye(3) - 0.05 * np.array([[1.0, 0.3, 0.0], [0.2, -0.5, 0.0], [0.0, 0.0, 0.2]]), 1))
    out.append((synth.layered((9, 2, 3), (1.0, 1.0, 1.0), 0, (-0.5 + 2.25 / 9, -0.5 + 6.5 / 9)),
                ((1.0, 2.0), (10.0, 20.0)), FBAR, 2))
    return out


def options(**kw):
    o = combo.combo_default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def single_solve(ms, mats, Fbar, K, opts, want_tangent=False):
    ctx = combo.combo_create(0)
    try:
        combo.combo_set_grid(ctx, *ms.n, *ms.l)
        combo.combo_set_materials(ctx, mats)
        combo.combo_set_microstructure(ctx, ms.phase, ms.c, ms.N)
        o = options(**{k: getattr(opts, k) for k, _ in opts._fields_})
        o.n_increments = K
        combo.combo_set_options(ctx, o)
        n1, n2, n3 = ms.n
        F = np.zeros((9, n3, n2, n1))
        P = np.zeros_like(F)
        r = combo.combo_solve(ctx, Fbar, F_out=F, P_out=P, want_tangent=want_tangent)
        r["F"], r["P"] = F, P
        return r
    finally:
        combo.combo_destroy(ctx)


def make_batch(mem, opts):
    b = combo.combo_batch_create(0)
    combo.combo_batch_set_options(b, opts)
    for i, (ms, mats, _, _) in enumerate(mem):
        assert combo.combo_batch_add(b, ms.n, ms.l, mats, ms.phase, ms.c, ms.N) == i
    return b


COUNTERS = ("newton_iters", "increments_done", "step_halvings", "cutbacks", "cg_truncations")


def close_count(a, b, frac):
    return abs(a - b) <= max(2, frac * max(a, b))


@pytest.mark.parametrize("precision", [combo.COMBO_FP64, combo.COMBO_MIXED])
def test_batch_equals_single_solves(precision):
    mem = members()
    fp64 = precision == combo.COMBO_FP64
    if fp64:
        opts = options(precision=precision, tol_newton=1e-10, tol_cg=1e-11)
    else:
        opts = options(precision=precision, tol_newton=1e-7, tol_cg=1e-5)
    b = make_batch(mem, opts)
    try:
        Fb = np.stack([m[2] for m in mem])
        K = [m[3] for m in mem]
        rb = combo.combo_batch_solve(b, Fb, n_increments=K)
        for i, (ms, mats, Fbar, k) in enumerate(mem):
            print("member", i, ms.n, flush=True)
            rs = single_solve(ms, mats, Fbar, k, opts)
            sb, ss = rb["stats"][i], rs["stats"]
            assert sb["status"] == combo.COMBO_OK
            assert sb["increments_done"] == ss["increments_done"]
            n1, n2, n3 = ms.n
            F = np.zeros((9, n3, n2, n1))
            P = np.zeros_like(F)
            combo.combo_batch_fields(b, i, F, P)
            if fp64:
                for c in COUNTERS:
                    assert sb[c] == ss[c], (i, c)
                assert close_count(sb["cg_iters_total"], ss["cg_iters_total"], 0.01), i
                assert close_count(sb["laminate_iters_total"], ss["laminate_iters_total"], 0.005), i
                assert rel(rb["Pbar"][i], rs["Pbar"]) <= 1e-9, i
                assert rel(rb["Pbar_phase"][i], rs["Pbar_phase"]) <= 1e-9, i
                assert rel(F, rs["F"]) <= 1e-9, i
                assert rel(P, rs["P"]) <= 1e-8, i
            else:
                assert abs(sb["newton_iters"] - ss["newton_iters"]) <= 1, i
                assert rel(rb["Pbar"][i], rs["Pbar"]) <= 1e-6, i
                assert rel(F, rs["F"]) <= 1e-5, i
    finally:
        combo.combo_batch_destroy(b)


def test_batch_graph_chunks_equal_plain_launches():
    """Captured CG chunks (graph_chunk > 0) replay the same launches as plain ones."""
    mem = members()
    Fb = np.stack([m[2] for m in mem])
    K = [m[3] for m in mem]
    out = []
    for gc in (0, 8):
        opts = options(precision=combo.COMBO_FP64, tol_newton=1e-10, tol_cg=1e-11, graph_chunk=gc)
        b = make_batch(mem, opts)
        try:
            out.append(combo.combo_batch_solve(b, Fb, n_increments=K))
        finally:
            combo.combo_batch_destroy(b)
    for i in range(len(mem)):
        assert out[0]["stats"][i]["newton_iters"] == out[1]["stats"][i]["newton_iters"]
        assert out[0]["stats"][i]["cg_iters_total"] == out[1]["stats"][i]["cg_iters_total"]
        assert np.array_equal(out[0]["Pbar"][i], out[1]["Pbar"][i]), i


def test_batch_member_matches_oracle():
    mem = members()[:3]
    opts = options(tol_newton=1e-10, tol_cg=1e-12)
    b = make_batch(mem, opts)
    try:
        rb = combo.combo_batch_solve(b, np.stack([m[2] for m in mem]), n_increments=[m[3] for m in mem])
        for i in (0, 2):
            ms, mats, Fbar, K = mem[i]
            prob = osol.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, mats)
            ref = osol.solve(prob, Fbar, osol.Options(tol_newton=1e-10, tol_cg=1e-12, n_increments=K))
            assert rel(rb["Pbar"][i], ref["Pbar"]) <= 1e-8
            assert rel(rb["Pbar_phase"][i], ref["Pbar_phase"]) <= 1e-8
    finally:
        combo.combo_batch_destroy(b)


def test_batch_tangent_equals_single():
    mem = [(synth.single_sphere((8, 8, 8), radius=0.3), ((1.0, 2.0), (10.0, 20.0)), FBAR, 1),
           (synth.single_sphere((6, 9, 4), radius=0.2), synth.contrast_mats(50.0), synth.stretch(0.05), 1)]
    opts = options(tol_newton=1e-11, tol_cg=1e-12, want_tangent=1)
    b = make_batch(mem, opts)
    try:
        rb = combo.combo_batch_solve(b, np.stack([m[2] for m in mem]), want_tangent=True)
        for i, (ms, mats, Fbar, K) in enumerate(mem):
            rs = single_solve(ms, mats, Fbar, K, opts, want_tangent=True)
            assert rel(rb["Abar"][i], rs["Abar"]) <= 1e-9, i
            assert close_count(rb["stats"][i]["cg_iters_tangent"], rs["stats"]["cg_iters_tangent"], 0.01), i
    finally:
        combo.combo_batch_destroy(b)


def test_batch_failure_is_isolated():
    """A member that cannot converge fails alone; the others finish."""
    hom = synth.homogeneous((8, 6, 4), phase_id=0)
    hard = synth.single_sphere((8, 8, 8), radius=0.35)
    mats = ((1.0, 2.0), (10.0, 20.0))
    mem = [(hom, mats, FBAR, 1), (hard, synth.contrast_mats(1000.0), synth.stretch(0.3), 1), (hom, mats, FBAR, 1)]
    opts = options(tol_newton=1e-10, tol_cg=1e-11, max_newton=1, max_cutbacks=0)
    b = make_batch(mem, opts)
    try:
        with pytest.raises(combo.ComboError) as e:
            combo.combo_batch_solve(b, np.stack([m[2] for m in mem]))
        assert e.value.status == combo.COMBO_E_NOCONV
        assert "member 1" in str(e.value)
        r = e.value.result
        assert [s["status"] for s in r["stats"]] == [combo.COMBO_OK, combo.COMBO_E_NOCONV, combo.COMBO_OK]
        P_exact = omat.stress(FBAR, *mats[0])
        for i in (0, 2):
            assert rel(r["Pbar"][i], P_exact) <= 1e-14
            assert r["stats"][i]["newton_iters"] == 0
    finally:
        combo.combo_batch_destroy(b)


def test_batch_error_paths():
    b = combo.combo_batch_create(0)
    try:
        with pytest.raises(combo.ComboError) as e:
            combo.combo_batch_solve(b, np.zeros((0, 9)))
        assert e.value.status == combo.COMBO_E_STATE
        ms = synth.single_sphere((8, 8, 8), radius=0.3)
        with pytest.raises(combo.ComboError) as e:
            combo.combo_batch_add(b, (10, 8, 8), (1, 1, 1), ((1, 2), (10, 20)), ms.phase, ms.c, ms.N)
        assert e.value.status == combo.COMBO_E_SIZE
        assert combo.combo_batch_size(b) == 0
        combo.combo_batch_add(b, ms.n, ms.l, ((1, 2), (10, 20)), ms.phase, ms.c, ms.N)
        assert combo.combo_batch_size(b) == 1
        with pytest.raises(combo.ComboError) as e:
            combo.combo_batch_solve(b, np.diag([1.0, 1.0, -1.0]).reshape(1, 3, 3))
        assert e.value.status == combo.COMBO_E_INADMISSIBLE
        bad = combo.combo_default_options()
        bad.max_cg = 0
        with pytest.raises(combo.ComboError) as e:
            combo.combo_batch_set_options(b, bad)
        assert e.value.status == combo.COMBO_E_INVAL
    finally:
        combo.combo_batch_destroy(b)
