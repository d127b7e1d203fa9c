"""The fibre workload's load walk stops where its equilibrium branch loses stability.

The fibre workload (paper Sec. 6.5 stand-in: 60 random straight fibres, contrast
1000, near-incompressible matrix, simple shear) is walked on a 64^3 grid in FP64
with the adaptive rule of the benchmark (a converged step doubles the step, a failed
one halves it, the walk ends below 1/32 of an increment).  At the unloaded state and
at every converged load, Lanczos in the C0 inner product on the Newton operator
K = Gamma0[A : .] (combo_apply_operator) gives the lowest eigenvalue of K on
compatible zero-mean fields.  K is self-adjoint in that product on those fields, and
its eigenvalues are the values of p:A:p / p:C0:p there, so the sign of the lowest
one decides whether the equilibrium is stable.  Every Lanczos vector is projected
with G (combo_apply_green): rounding would otherwise leak components outside the
compatible fields, where K is not self-adjoint, and give spurious Ritz values.

- At F = I the lowest eigenvalue is mu_m / mu0.  Every phase is no softer than the
  matrix (a composite voxel holds a laminate of the two), and for gradient fields the
  sum of p:p^T equals that of tr(p)^2.  So the sum of p:C:p is at least
  mu_m |p|^2 + (lambda_m + mu_m) tr(p)^2, which is mu_m/mu0 times p:C0:p because the
  reference medium has kappa0 = mu0 (1 + lambda_m/mu_m) (both phases have
  lambda/mu = 1000).  Fields concentrated in the matrix reach the bound.
- Along the walk the lowest eigenvalue falls at every converged load, and at the last
  one it is below a tenth of the unloaded value: Newton starts to fail where the
  branch it follows is about to lose positive definiteness."""
import numpy as np
import pytest
import torch
from scipy.linalg import eigvalsh_tridiagonal

from paper_2204_13624_amd import combo, synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def lowest_eigenvalue(ctx, shape, mu0, kappa0, steps, seed=11):
    """Smallest Ritz value of K after `steps` Lanczos steps (and after 2/3 of them)."""
    def ip(x, y):
        return float(mu0 * torch.sum(x * y) + kappa0 * torch.sum((x[0] + x[4] + x[8]) * (y[0] + y[4] + y[8])))

    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    r = torch.randn(shape, dtype=torch.float64, device=DEV, generator=g)
    v = torch.empty_like(r)
    combo.combo_apply_green(ctx, combo.COMBO_GREEN_G, combo.COMBO_FP64, r, v)
    v /= np.sqrt(ip(v, v))
    v_old = torch.zeros_like(v)
    w = torch.empty_like(v)
    wp = torch.empty_like(v)
    alpha, beta = [], []
    b = 0.0
    ritz = []
    for j in range(steps):
        combo.combo_apply_operator(ctx, combo.COMBO_FP64, v, w)
        w -= b * v_old
        a = ip(w, v)
        w -= a * v
        combo.combo_apply_green(ctx, combo.COMBO_GREEN_G, combo.COMBO_FP64, w, wp)
        b = np.sqrt(ip(wp, wp))
        alpha.append(a)
        beta.append(b)
        v_old, v = v, wp / b
        if j + 1 in (2 * steps // 3, steps):
            ritz.append(float(eigvalsh_tridiagonal(np.array(alpha), np.array(beta[:-1]),
                                                   select="i", select_range=(0, 0))[0]))
    return ritz


def test_fibre_walk_stops_where_the_branch_loses_stability():
    n, steps = 64, 1500
    ms, lc = synth.workload_fibres_256(n)
    (mu_m, lam_m), (mu_p, lam_p) = lc.mats
    mu0 = float(np.sqrt(mu_m * mu_p))
    kappa0 = float(np.sqrt((lam_m + mu_m) * (lam_p + mu_p)))
    assert abs(kappa0 - mu0 * (1 + lam_m / mu_m)) <= 1e-9 * kappa0
    ctx = combo.combo_create(0)
    try:
        combo.combo_set_grid(ctx, *ms.n, *ms.l)
        combo.combo_set_materials(ctx, lc.mats)
        combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(DEV), torch.from_numpy(ms.c).to(DEV),
                                       torch.from_numpy(np.ascontiguousarray(ms.N)).to(DEV))
        o = combo.combo_default_options()
        o.precision = combo.COMBO_FP64
        o.tol_newton, o.tol_cg, o.max_newton, o.max_cg = 1e-8, 1e-10, 20, 20000
        o.n_increments, o.max_cutbacks = 1, 0
        combo.combo_set_options(ctx, o)
        shape = (9,) + ms.phase.shape

        def lowest(F, shear):
            combo.combo_eval_law(ctx, F)
            r = lowest_eigenvalue(ctx, shape, mu0, kappa0, steps)
            print("shear %.5f: lowest eigenvalue %.6f (%.6f after %d steps)" % (shear, r[1], r[0], 2 * steps // 3),
                  flush=True)
            assert abs(r[1] - r[0]) <= 0.02 * abs(r[1])        # converged
            return r[1]

        F = torch.zeros(shape, dtype=torch.float64, device=DEV)
        F[0] = F[4] = F[8] = 1.0
        Fn = torch.empty_like(F)
        lam = [lowest(F, 0.0)]
        assert abs(lam[0] - mu_m / mu0) <= 1e-4 * mu_m / mu0
        H = lc.Fbar - np.eye(3)
        K = lc.n_increments
        t, dt = 0.0, 1.0 / K
        while dt >= 1.0 / (32 * K):
            tn = t + dt
            try:
                combo.combo_solve(ctx, np.eye(3) + tn * H, F_init=F, F_out=Fn)
            except combo.ComboError:
                dt *= 0.5
                continue
            F, Fn = Fn, F
            t = tn
            dt = min(1.0 / K, 2 * dt)
            lam.append(lowest(F, 0.3 * t))
        print("walk stopped at shear %.5f" % (0.3 * t), flush=True)
        assert 0.0 < 0.3 * t < 0.02, t
        assert all(a > b for a, b in zip(lam, lam[1:])), lam
        assert 0.0 < lam[-1] < 0.1 * lam[0], lam
    finally:
        combo.combo_destroy(ctx)
