"""FFT schedule variants and the autotuner, through the C-ABI.

Every compiled variant of the x, y and z passes computes the same operator;
each is pinned against the FP64 oracle (CG operator and Green operators), the
autotuner must pick existing variants and reuse its cache, and a solve with
the tuned schedule must agree with the default one.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import solver as osol
from oracle import spectral as ospec
from paper_2204_13624_amd import combo, synth

pytestmark = pytest.mark.gpu

MATS = ((1.0, 2.0), (10.0, 20.0))
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def ctx():
    c = combo.combo_create(0)
    yield c
    combo.combo_destroy(c)


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def setup(ctx, ms, **opt):
    combo.combo_set_grid(ctx, *ms.n, *ms.l)
    combo.combo_set_materials(ctx, MATS)
    combo.combo_set_microstructure(ctx, ms.phase, ms.c, ms.N)
    o = combo.combo_default_options()
    for k, v in opt.items():
        setattr(o, k, v)
    combo.combo_set_options(ctx, o)


# every axis of these grids has two variants of its pass (x 256 and 64: rows per
# workgroup; the others: radix order or tile width)
GRIDS = [(64, 48, 32), (256, 32, 16), (32, 128, 96), (128, 96, 32), (32, 192, 48), (32, 48, 192)]


@pytest.mark.parametrize("n", GRIDS)
def test_every_schedule_variant_matches_oracle(ctx, n):
    ms = synth.random_composite_field(n, 5, frac_composite=0.1)
    setup(ctx, ms)
    (_, _, _), (nxv, nyv, nzv) = combo.combo_get_schedule(ctx)
    assert (nxv, nyv, nzv) == (2, 2 if n[1] != 16 else 1, 2 if n[2] != 16 else 1)
    F = synth.random_F_field(n, 6, amplitude=0.15)
    prob = osol.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS)
    mu0, kappa0 = osol.reference_medium(MATS)
    _, Av, ok, _, _ = osol.evaluate(F.reshape(3, 3, *F.shape[1:]), prob)
    assert ok
    rng = np.random.default_rng(9)
    p = ospec.apply_g(rng.normal(size=(3, 3, n[2], n[1], n[0])), n, (1.0, 1.0, 1.0))
    ref = ospec.apply_gamma0(osol.apply_tangent(Av, p, prob.shape), n, (1.0, 1.0, 1.0), mu0, kappa0)
    ref = ref.reshape(9, n[2], n[1], n[0])
    tau = rng.normal(size=(9, n[2], n[1], n[0]))
    gref = ospec.apply_gamma0(tau.reshape(3, 3, n[2], n[1], n[0]), n, (1.0, 1.0, 1.0), mu0, kappa0)
    gref = gref.reshape(tau.shape)
    pc = np.ascontiguousarray(p.reshape(9, n[2], n[1], n[0]))
    for prec, tol in ((combo.COMBO_MIXED, 3e-6), (combo.COMBO_FP64, 1e-11)):
        o = combo.combo_default_options()
        o.precision = prec
        combo.combo_set_options(ctx, o)
        assert combo.combo_eval_law(ctx, F, None, None, None, None) == combo.COMBO_OK
        for xv in range(nxv):
            for yv in range(nyv):
                for zv in range(nzv):
                    print("schedule", n, prec, xv, yv, zv, flush=True)
                    combo.combo_set_schedule(ctx, xv, yv, zv)
                    q = np.zeros_like(pc)
                    combo.combo_apply_operator(ctx, prec, pc, q)
                    assert rel(q, ref) <= tol, (prec, xv, yv, zv)
                    out = np.zeros_like(tau)
                    combo.combo_apply_green(ctx, combo.COMBO_GREEN_GAMMA0, prec, tau, out)
                    assert rel(out, gref) <= (2e-6 if prec == combo.COMBO_MIXED else 1e-12), (prec, xv, yv, zv)


def test_autotune_picks_existing_variants_and_caches(ctx, tmp_path):
    ms = synth.single_sphere((64, 48, 32), radius=0.25)
    setup(ctx, ms)
    (_, _, _), counts = combo.combo_get_schedule(ctx)
    sched = combo.combo_autotune(ctx, combo.COMBO_MIXED)
    assert all(0 <= v < c for v, c in zip(sched, counts))
    assert combo.combo_autotune(ctx, combo.COMBO_MIXED) == sched        # cached in the process
    assert combo.combo_get_schedule(ctx)[0] == sched
    assert combo.combo_autotune(ctx, combo.COMBO_FP64) == (0, 0, 0)     # FP64 passes: variant 0 only
    # the cache file: a fresh process tunes once and writes a line, the next reads it back
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, COMBO_TUNE_CACHE=str(cache))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2204_13624_amd import combo, synth\n"
            "ms = synth.single_sphere((96, 32, 48), radius=0.25)\n"
            "c = combo.combo_create(0)\n"
            "combo.combo_set_grid(c, *ms.n, *ms.l)\n"
            "combo.combo_set_materials(c, ((1.0, 2.0), (10.0, 20.0)))\n"
            "combo.combo_set_microstructure(c, ms.phase, ms.c, ms.N)\n"
            "print(*combo.combo_autotune(c, combo.COMBO_MIXED))\n") % ROOT
    r1 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r1.returncode == 0, r1.stderr
    lines = cache.read_text().split("\n")
    assert len([ln for ln in lines if ln.strip()]) == 1
    fields = lines[0].split()
    assert fields[1:5] == ["96", "32", "48", "mixed"]
    assert " ".join(fields[5:8]) == r1.stdout.strip()
    # a planted schedule in the file is what the next process uses, without tuning again
    cache.write_text(" ".join(fields[:5] + ["1", "1", "1"]) + "\n")
    r2 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r2.returncode == 0, r2.stderr
    assert r2.stdout.strip() == "1 1 1"
    assert len([ln for ln in cache.read_text().split("\n") if ln.strip()]) == 1


def test_solve_with_autotuned_schedule_matches_default(ctx):
    ms = synth.single_sphere((64, 48, 32), radius=0.25)
    setup(ctx, ms, precision=combo.COMBO_MIXED, tol_newton=1e-8, tol_cg=1e-6)
    r0 = combo.combo_solve(ctx, synth.stretch(0.05))
    setup(ctx, ms, precision=combo.COMBO_MIXED, tol_newton=1e-8, tol_cg=1e-6, autotune=1)
    r1 = combo.combo_solve(ctx, synth.stretch(0.05))
    assert rel(r1["Pbar"], r0["Pbar"]) <= 1e-6
    combo.combo_set_schedule(ctx, 1, 1, 1)
    setup_keep = combo.combo_default_options()
    setup_keep.precision = combo.COMBO_MIXED
    setup_keep.tol_newton = 1e-8
    setup_keep.tol_cg = 1e-6
    combo.combo_set_options(ctx, setup_keep)
    r2 = combo.combo_solve(ctx, synth.stretch(0.05))
    assert rel(r2["Pbar"], r0["Pbar"]) <= 1e-6
