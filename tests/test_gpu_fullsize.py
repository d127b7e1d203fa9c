"""Parity at the benchmark's full sizes (256^3 spheres, the 64-RVE batch), in the
launch configurations bench.py times.

At these sizes the oracle cannot run whole solves, so the checks are:
- sampled outputs it computes one by one: the pointwise law at sampled voxels,
  and the Green operators on sums of single Fourier modes, whose exact image
  is the oracle's multiplier at that frequency;
- properties that hold at any size: self-adjointness of the CG operator in
  the C0 inner product, <F> = Fbar, equilibrium, Hill-Mandel, and mixed
  against FP64;
- batch members against the same RVEs solved alone.
"""
import numpy as np
import pytest

from oracle import solver as osol
from oracle import spectral as ospec
from paper_2204_13624_amd import combo, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.fixture(scope="module")
def spheres256():
    return synth.workload_spheres_256()


@pytest.fixture
def ctx():
    c = combo.combo_create(0)
    yield c
    combo.combo_destroy(c)


def dev():
    return torch.device("cuda:0")


def setup(ctx, ms, mats, **opt):
    combo.combo_set_grid(ctx, *ms.n, *ms.l)
    combo.combo_set_materials(ctx, mats)
    combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(dev()), torch.from_numpy(ms.c).to(dev()),
                                   torch.from_numpy(np.ascontiguousarray(ms.N)).to(dev()))
    o = combo.combo_default_options()
    for k, v in opt.items():
        setattr(o, k, v)
    combo.combo_set_options(ctx, o)


def sample_voxels(ms, count, seed):
    """Sampled voxel indices, half of them composite."""
    rng = np.random.default_rng(seed)
    ph = ms.phase.reshape(-1)
    comp = np.nonzero(ph == 2)[0]
    rest = np.nonzero(ph != 2)[0]
    return np.sort(np.concatenate([rng.choice(comp, count // 2, replace=False),
                                   rng.choice(rest, count // 2, replace=False)]))


def test_law_at_256_sampled_voxels(ctx, spheres256):
    ms, lc = spheres256
    setup(ctx, ms, lc.mats)
    n = ms.nvox
    g = torch.Generator(device=dev()).manual_seed(7)
    F = 0.2 * (torch.rand((9, n), generator=g, device=dev(), dtype=torch.float64) - 0.5)
    F[0] += 1.0
    F[4] += 1.0
    F[8] += 1.0
    P = torch.empty_like(F)
    a = torch.empty((3, n), device=dev(), dtype=torch.float64)
    st = combo.combo_eval_law(ctx, F, P, None, a, None)
    if st != combo.COMBO_OK:   # name the failing voxels before failing
        err = combo.combo_last_error(ctx)
        it = torch.zeros(n, device=dev(), dtype=torch.int32)
        combo.combo_eval_law(ctx, F, P, None, a, it)
        det = torch.linalg.det(F.T.reshape(-1, 3, 3))
        maxit = combo.combo_default_options().max_laminate
        worst = torch.nonzero(it >= maxit).flatten()[:8].cpu().numpy()
        print("law failure:", err, "| laminate iters max", int(it.max()), "| at the limit", int((it >= maxit).sum()),
              "| min det F", float(det.min()), "| voxels", worst, "| c", ms.c.reshape(-1)[worst],
              "| N", ms.N.reshape(3, -1)[:, worst].T, "| F", F[:, torch.from_numpy(worst).to(dev())].T.cpu().numpy(),
              flush=True)
    assert st == combo.COMBO_OK, combo.combo_last_error(ctx)
    idx = sample_voxels(ms, 4096, 1)
    ti = torch.from_numpy(idx).to(dev())
    Fs, Ps, As = F[:, ti].cpu().numpy(), P[:, ti].cpu().numpy(), a[:, ti].cpu().numpy()
    m = idx.size
    sub = osol.Problem((m, 1, 1), (1.0, 1.0, 1.0), ms.phase.reshape(-1)[idx].reshape(1, 1, m),
                       ms.c.reshape(-1)[idx].reshape(1, 1, m), ms.N.reshape(3, -1)[:, idx].reshape(3, 1, 1, m),
                       lc.mats)
    Po, _, ok, _, lp = osol.evaluate(Fs.reshape(3, 3, 1, 1, m), sub)
    assert ok
    assert rel(Ps, Po.reshape(9, m)) <= 1e-12
    assert np.abs(As[:, lp["idx"]].T - lp["a"]).max() <= 1e-11 * max(1.0, np.abs(lp["a"]).max())


@pytest.mark.parametrize("which", [combo.COMBO_GREEN_G, combo.COMBO_GREEN_GAMMA0])
def test_green_operators_at_256_on_fourier_modes(ctx, which):
    """Gamma0 and G on a sum of single Fourier modes at 256^3 against the oracle's
    multiplier at each mode, at sampled voxels."""
    n = (256, 256, 256)
    l = (1.0, 0.8, 1.3)
    mats = ((1.0, 2.0), (100.0, 200.0))
    combo.combo_set_grid(ctx, *n, *l)
    combo.combo_set_materials(ctx, mats)
    mu0, kappa0 = osol.reference_medium(mats)
    rng = np.random.default_rng(5)
    modes = [((3, -7, 1), None), ((-127, 5, 64), None), ((0, 0, 9), None), ((41, 127, -100), None)]
    amps = [rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)) for _ in modes]
    zz, yy, xx = torch.meshgrid(*(torch.arange(m, device=dev(), dtype=torch.float64) for m in n[::-1]),
                                indexing="ij")
    tau = torch.zeros((9,) + n[::-1], device=dev(), dtype=torch.float64)
    for (k, _), A in zip(modes, amps):
        th = 2.0 * np.pi * (k[0] * xx / n[0] + k[1] * yy / n[1] + k[2] * zz / n[2])
        c, s = torch.cos(th), torch.sin(th)
        for comp in range(9):
            tau[comp] += float(A.reshape(9)[comp].real) * c - float(A.reshape(9)[comp].imag) * s
        del th, c, s
    del zz, yy, xx
    idx = np.random.default_rng(2).choice(n[0] * n[1] * n[2], 4096, replace=False)
    x1, x2, x3 = idx % n[0], (idx // n[0]) % n[1], idx // (n[0] * n[1])
    expect = np.zeros((9, idx.size))
    for (k, _), A in zip(modes, amps):
        # the oracle's multipliers on a one-frequency "grid" ([3, 1, 1, 1] frequencies)
        xi = np.array([2.0 * np.pi * k[d] / l[d] for d in range(3)]).reshape(3, 1, 1, 1)
        mask = np.zeros((1, 1, 1), dtype=bool)
        Ah = A.reshape(3, 3, 1, 1, 1)
        M = (ospec.gamma0_hat(Ah, xi, mask, mu0, kappa0) if which == combo.COMBO_GREEN_GAMMA0
             else ospec.g_hat(Ah, xi, mask))[:, :, 0, 0, 0]
        th = 2.0 * np.pi * (k[0] * x1 / n[0] + k[1] * x2 / n[1] + k[2] * x3 / n[2])
        expect += (M.reshape(9, 1) * np.exp(1j * th)[None, :]).real
    ti = torch.from_numpy(idx).to(dev())
    for prec, tol in ((combo.COMBO_FP64, 1e-12), (combo.COMBO_MIXED, 5e-6)):
        out = torch.empty_like(tau)
        combo.combo_apply_green(ctx, which, prec, tau, out)
        got = out.reshape(9, -1)[:, ti].cpu().numpy()
        assert rel(got, expect) <= tol, prec
        del out


def test_cg_operator_at_256_is_self_adjoint(ctx, spheres256):
    """<Gamma0[A:p1], p2>_C0 = <p1, Gamma0[A:p2]>_C0 for compatible p1, p2 at the
    first-increment predictor of the 256^3 workload."""
    ms, lc = spheres256
    setup(ctx, ms, lc.mats)
    n = ms.nvox
    Fb = np.eye(3) + (lc.Fbar - np.eye(3)) / lc.n_increments
    F = torch.from_numpy(Fb.reshape(9, 1)).to(dev()).expand(9, n).contiguous()
    assert combo.combo_eval_law(ctx, F, None, None, None, None) == combo.COMBO_OK
    del F
    mu0, kappa0 = osol.reference_medium(lc.mats)
    g = torch.Generator(device=dev()).manual_seed(3)
    ps, qs = [], []
    for _ in range(2):
        tau = torch.randn((9, n), generator=g, device=dev(), dtype=torch.float64)
        p = torch.empty_like(tau)
        combo.combo_apply_green(ctx, combo.COMBO_GREEN_G, combo.COMBO_FP64, tau, p)
        del tau
        q = torch.empty_like(p)
        combo.combo_apply_operator(ctx, combo.COMBO_FP64, p, q)
        ps.append(p)
        qs.append(q)

    def c0(x, y):
        trx, tr_y = x[0] + x[4] + x[8], y[0] + y[4] + y[8]
        return float(mu0 * (x * y).sum() + kappa0 * (trx * tr_y).sum())

    a, b = c0(qs[0], ps[1]), c0(ps[0], qs[1])
    assert abs(a - b) <= 1e-10 * (abs(c0(qs[0], ps[0])) * abs(c0(qs[1], ps[1]))) ** 0.5


def test_solve_at_256_mixed_and_fp64(ctx, spheres256):
    """The bench configuration: <F> = Fbar, equilibrium, Hill-Mandel, mixed vs FP64."""
    ms, lc = spheres256
    setup(ctx, ms, lc.mats, precision=combo.COMBO_MIXED, tol_newton=1e-6, tol_cg=1e-4, max_cg=20000,
          n_increments=lc.n_increments)
    n = ms.nvox
    F = torch.empty((9, n), device=dev(), dtype=torch.float64)
    P = torch.empty_like(F)
    rm = combo.combo_solve(ctx, lc.Fbar, F_out=F, P_out=P)
    assert rm["stats"]["eta_final"] <= 1e-6
    assert rm["stats"]["increments_done"] == lc.n_increments
    Fm = F.mean(dim=1).cpu().numpy().reshape(3, 3)
    assert np.abs(Fm - lc.Fbar).max() <= 1e-12
    Pbar = P.mean(dim=1).cpu().numpy().reshape(3, 3)
    assert rel(Pbar, rm["Pbar"]) <= 1e-12
    hm = float((P * F).sum(dim=0).mean())
    assert abs(hm - float((rm["Pbar"] * lc.Fbar).sum())) <= 1e-5 * np.abs(rm["Pbar"]).max()
    del F, P
    setup(ctx, ms, lc.mats, precision=combo.COMBO_FP64, tol_newton=1e-6, tol_cg=1e-4, max_cg=20000,
          n_increments=lc.n_increments)
    r64 = combo.combo_solve(ctx, lc.Fbar)
    assert rel(rm["Pbar"], r64["Pbar"]) <= 1e-6


def test_batch_workload_members_match_single_solves():
    """The 64-RVE batch as bench.py runs it: every member converged with <F> = Fbar,
    and one member per (size, kind) equal to its single solve to the mixed accuracy."""
    items = synth.workload_batch()
    o = combo.combo_default_options()
    o.precision = combo.COMBO_MIXED
    o.tol_newton = 1e-6
    o.tol_cg = 1e-4
    o.max_cg = 20000
    b = combo.combo_batch_create(0)
    try:
        combo.combo_batch_set_options(b, o)
        for ms, lc in items:
            combo.combo_batch_add(b, ms.n, ms.l, lc.mats, ms.phase, ms.c, ms.N)
        rb = combo.combo_batch_solve(b, np.stack([lc.Fbar for _, lc in items]),
                                     n_increments=[lc.n_increments for _, lc in items])
        picked = {}
        for i, (ms, lc) in enumerate(items):
            assert rb["stats"][i]["eta_final"] <= 1e-6
            F = torch.empty((9, ms.nvox), device=dev(), dtype=torch.float64)
            combo.combo_batch_fields(b, i, F, None)
            assert np.abs(F.mean(dim=1).cpu().numpy().reshape(3, 3) - lc.Fbar).max() <= 1e-12, i
            picked.setdefault((ms.n, ms.info["kind"]), i)
        for (shape, kind), i in sorted(picked.items()):
            ms, lc = items[i]
            print("member", i, shape, kind, flush=True)
            c = combo.combo_create(0)
            try:
                combo.combo_set_grid(c, *ms.n, *ms.l)
                combo.combo_set_materials(c, lc.mats)
                combo.combo_set_microstructure(c, ms.phase, ms.c, ms.N)
                oo = combo.combo_default_options()
                for k, _ in o._fields_:
                    setattr(oo, k, getattr(o, k))
                oo.n_increments = lc.n_increments
                combo.combo_set_options(c, oo)
                rs = combo.combo_solve(c, lc.Fbar)
            finally:
                combo.combo_destroy(c)
            assert rel(rb["Pbar"][i], rs["Pbar"]) <= 1e-6, i
    finally:
        combo.combo_batch_destroy(b)
