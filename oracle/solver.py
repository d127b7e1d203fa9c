"""Lippmann-Schwinger Newton-CG solve of the periodic homogenization problem
with composite boxels (paper Sec. 2, 3 and 4).

Problem (HOM, Sec. 2): given the macroscopic deformation gradient Fbar, find a
periodic fluctuation such that Div P = 0, with P = P(F) the pointwise material
law: compressible Neo-Hooke in pure voxels (Sec. 6.1), the ComBo laminate in
composite voxels (Sec. 4); or, with Problem.law = "linear", the infinitesimal
strain counterparts of the appendix cheat sheet (isotropic linear elasticity and
the closed-form laminate), where P is the stress of sym(F - I) and one Newton
step solves the problem up to the CG tolerance.  Outputs: Pbar = <P> (eq. Pbar), the phase averages
and the algorithmic effective tangent dPbar/dFbar (mentioned in Sec. 2).

Method (Sec. 3): Newton-Raphson on the Lippmann-Schwinger equation
F = Fbar - Gamma^0 (P - C^0:F) (eq. nonlinearLSE) with a conjugate gradient
linear solver.  Linearising at an F with F - Fbar compatible and zero-mean, and
using Gamma^0 C^0 = identity on such fields, each Newton step solves
    Gamma^0 [A : dF] = - Gamma^0 [P]
for a compatible zero-mean dF; Gamma^0 A is self-adjoint in the C^0 inner
product <x, y> = sum_voxels mu0 x:y + kappa0 tr(x) tr(y), so plain CG applies.

Readings where the paper is silent (the GPU solver uses the same ones):
  * reference medium C^0 = mu0 I + kappa0 I(x)I, default mu0 = sqrt(mu_min
    mu_max), kappa0 = sqrt((lambda+mu)_min (lambda+mu)_max); the result does
    not depend on it, only iteration counts do;
  * Newton test: eta = |G[P]|_2 / (sqrt(n) |Pbar|_F) <= tol_newton (root mean
    square equilibrium residual relative to the effective stress);
  * CG test: |r|_C0 / |b|_C0 <= tol_cg;
  * negative curvature: far from equilibrium (the homogeneous predictor puts
    stiff inclusions at the uniform-strain stress) the Neo-Hooke tangent can be
    indefinite on compatible fields, and CG meets <p, q> <= 0.  The Newton step
    then takes the CG iterate reached before that direction (truncated Newton);
    if that is the first CG iteration (no iterate yet), the Newton loop fails
    and the increment is halved.  A NaN <p, q> stays an error, and so does
    negative curvature in the effective-tangent solves;
  * load path Fbar_k = Fbar_0 + (k/K)(Fbar - Fbar_0), homogeneous predictor
    F += Fbar_k - Fbar_{k-1};
  * step control: F + s dF with s = 1, halved (at most 10 times) while any
    voxel has det F <= 0 or a laminate fails, or (line search, on by default)
    while the residual does not decrease, eta(s) > (1 - 1e-4 s) eta; if that,
    the predictor or the Newton loop fails, the increment is halved (at most
    5 times);
  * effective tangent: for each unit macro perturbation E = e_k (x) e_L solve
    Gamma^0 [A:dF] = -Gamma^0 [A:E] at the converged state and set
    Abar[:, 3k+L] = <A:(E + dF)>.
"""
import dataclasses

import numpy as np

from . import laminate, material, spectral, staggered

OK = 0
E_NOCONV = -5
E_INADMISSIBLE = -6
E_NUMERIC = -7
LS_ARMIJO = 1e-4   # sufficient decrease of the line search: eta(s) <= (1 - 1e-4 s) eta


@dataclasses.dataclass
class Options:
    tol_newton: float = 1e-8
    tol_cg: float = 1e-10
    max_newton: int = 30
    max_cg: int = 5000
    n_increments: int = 1
    mu0: float = 0.0          # <= 0: default rule
    kappa0: float = 0.0
    want_tangent: bool = False
    max_step_halvings: int = 10
    max_cutbacks: int = 5
    line_search: bool = True   # accept F + s dF only if the residual decreases (Armijo)


@dataclasses.dataclass
class Problem:
    n: tuple            # (n1, n2, n3)
    l: tuple            # (l1, l2, l3)
    phase: np.ndarray   # uint8 [n3, n2, n1]
    c: np.ndarray       # [n3, n2, n1]
    N: np.ndarray       # [3, n3, n2, n1]
    mats: tuple         # ((mu-, lam-), (mu+, lam+))
    law: str = "neo_hooke"   # or "linear": small strain, P = sigma(sym(F - I))
    disc: str = "ms"         # or "willot": rotated-scheme gradient (spectral.willot_frequencies);
                             # or "staggered": staggered grid with the DFMG law (App. A, oracle.staggered)

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def nvox(self):
        return self.n[0] * self.n[1] * self.n[2]


class NegativeCurvature(RuntimeError):
    """CG met a direction p with <p, Gamma^0[A:p]> <= 0; x is the iterate after `it` iterations."""

    def __init__(self, x, it, gam):
        super().__init__("CG negative curvature <p, q> = %r after %d iterations" % (gam, it))
        self.x = x
        self.it = it


class SolveError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


def reference_medium(mats, mu0=0.0, kappa0=0.0):
    (mu_m, lam_m), (mu_p, lam_p) = mats
    if mu0 <= 0.0:
        mu0 = float(np.sqrt(min(mu_m, mu_p) * max(mu_m, mu_p)))
    if kappa0 <= 0.0:
        k_m, k_p = lam_m + mu_m, lam_p + mu_p
        kappa0 = float(np.sqrt(min(k_m, k_p) * max(k_m, k_p)))
    return mu0, kappa0


def to_voxels(field):
    """[3,3,n3,n2,n1] -> [n,3,3] (voxels in z, y, x order)."""
    return np.moveaxis(field.reshape(3, 3, -1), -1, 0)


def to_field(vox, shape):
    return np.moveaxis(vox, 0, -1).reshape((3, 3) + tuple(shape))


def evaluate(F, prob):
    """Pointwise law on the whole field: P [3,3,...], A [n,9,9] and statistics
    (staggered grid: the DFMG law and its term tangents, oracle.staggered.evaluate)."""
    if prob.disc == "staggered":
        if prob.law != "neo_hooke":
            raise ValueError("the staggered-grid solve takes the finite-strain law")
        return staggered.evaluate(F, prob)
    Fv = to_voxels(F)
    n = Fv.shape[0]
    phase = prob.phase.reshape(-1)
    Pv = np.zeros((n, 3, 3))
    Av = np.zeros((n, 9, 9))
    ok = True
    stats = dict(lam_iters=0, lam_iters_max=0, lam_backproj=0, lam_fail=0)
    lam_parts = {}
    if prob.law == "linear":
        return _evaluate_linear(Fv, prob, phase, Pv, Av, stats)
    for ph in (0, 1):
        idx = np.nonzero(phase == ph)[0]
        if idx.size == 0:
            continue
        J = np.linalg.det(Fv[idx])
        if np.any(J <= 0):
            ok = False
            continue
        mu, lam = prob.mats[ph]
        Pv[idx] = material.stress(Fv[idx], mu, lam)
        Av[idx] = material.tangent(Fv[idx], mu, lam)
    idx = np.nonzero(phase == 2)[0]
    if idx.size:
        r = laminate.solve(Fv[idx], prob.c.reshape(-1)[idx], prob.N.reshape(3, -1)[:, idx].T,
                           prob.mats[0], prob.mats[1])
        bad = r["status"] != laminate.STATUS_OK
        stats["lam_iters"] = int(r["iters"].sum())
        stats["lam_iters_max"] = int(r["iters"].max())
        stats["lam_backproj"] = int(r["n_backproj"].sum())
        stats["lam_fail"] = int(bad.sum())
        if bad.any():
            ok = False
        Pv[idx] = r["P"]
        Av[idx] = r["A"]
        lam_parts = dict(idx=idx, Pp=r["Pp"], Pm=r["Pm"], a=r["a"])
    return to_field(Pv, prob.shape), Av, ok, stats, lam_parts


def _evaluate_linear(Fv, prob, phase, Pv, Av, stats):
    """Small-strain law: isotropic linear elasticity in pure voxels, the closed-form
    laminate of the appendix cheat sheet in composite voxels (no admissibility)."""
    for ph in (0, 1):
        idx = np.nonzero(phase == ph)[0]
        mu, lam = prob.mats[ph]
        Pv[idx] = material.linear_stress(Fv[idx], mu, lam)
        Av[idx] = material.isotropic_stiffness(mu, lam)
    lam_parts = {}
    idx = np.nonzero(phase == 2)[0]
    if idx.size:
        r = laminate.solve_small(Fv[idx] - np.eye(3), prob.c.reshape(-1)[idx],
                                 prob.N.reshape(3, -1)[:, idx].T, prob.mats[0], prob.mats[1])
        Pv[idx] = r["P"]
        Av[idx] = r["A"]
        lam_parts = dict(idx=idx, Pp=r["Pp"], Pm=r["Pm"], a=r["a"])
    return to_field(Pv, prob.shape), Av, True, stats, lam_parts


def apply_tangent(Av, p, shape):
    """(A : p) as a field, A [n,9,9] per voxel (a dict of DFMG term tangents on the
    staggered grid)."""
    if isinstance(Av, dict):
        return staggered.tangent_action(Av, p)
    pv = to_voxels(p).reshape(-1, 9)
    return to_field(np.einsum("nab,nb->na", Av, pv).reshape(-1, 3, 3), shape)


def inner_c0(x, y, mu0, kappa0):
    """<x, y>_C0 = sum over voxels of mu0 x:y + kappa0 tr(x) tr(y)."""
    trx = x[0, 0] + x[1, 1] + x[2, 2]
    tr_y = y[0, 0] + y[1, 1] + y[2, 2]
    return float(mu0 * np.sum(x * y) + kappa0 * np.sum(trx * tr_y))


def gamma0(tau, prob, mu0, kappa0):
    """Gamma^0[tau] of the problem's discretization."""
    if prob.disc == "staggered":
        return staggered.apply_gamma0(tau, prob.n, prob.l, mu0, kappa0)
    return spectral.apply_gamma0(tau, prob.n, prob.l, mu0, kappa0, prob.disc)


def residual(P, prob):
    """eta = |G[P]|_2 / (sqrt(n) |Pbar|_F)."""
    if prob.disc == "staggered":
        R = staggered.apply_g(P, prob.n, prob.l)
    else:
        R = spectral.apply_g(P, prob.n, prob.l, prob.disc)
    Pbar = P.mean(axis=(2, 3, 4))
    den = np.sqrt(prob.nvox) * max(np.linalg.norm(Pbar), 1e-300)
    return float(np.linalg.norm(R) / den)


def cg(Av, b, prob, mu0, kappa0, tol, maxit):
    """CG in the C^0 inner product on Gamma^0 [A : x] = b (b compatible, zero mean)."""
    shape = prob.shape
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = inner_c0(r, r, mu0, kappa0)
    rho0 = rho
    if rho0 == 0.0:
        return x, 0
    it = 0
    while True:
        if it >= maxit:
            raise SolveError(E_NOCONV, "CG did not converge in %d iterations" % maxit)
        q = gamma0(apply_tangent(Av, p, shape), prob, mu0, kappa0)
        gam = inner_c0(p, q, mu0, kappa0)
        if gam != gam:
            raise SolveError(E_NUMERIC, "CG breakdown: <p, q> = %r" % gam)
        if not (gam > 0.0):
            raise NegativeCurvature(x, it, gam)
        alpha = rho / gam
        x += alpha * p
        r -= alpha * q
        rho_n = inner_c0(r, r, mu0, kappa0)
        it += 1
        if np.sqrt(rho_n / rho0) <= tol:
            return x, it
        p = r + (rho_n / rho) * p
        rho = rho_n


def effective_tangent(F, prob, opts, mu0, kappa0):
    P, Av, ok, _, _ = evaluate(F, prob)
    shape = prob.shape
    Abar = np.zeros((9, 9))
    cg_total = 0
    for kL in range(9):
        E = np.zeros((3, 3) + tuple(shape))
        E[kL // 3, kL % 3] = 1.0
        tau = apply_tangent(Av, E, shape)
        b = -gamma0(tau, prob, mu0, kappa0)
        try:
            dF, it = cg(Av, b, prob, mu0, kappa0, opts.tol_cg, opts.max_cg)
        except NegativeCurvature as e:
            raise SolveError(E_NUMERIC, "effective tangent: %s" % e)
        cg_total += it
        Abar[:, kL] = apply_tangent(Av, E + dF, shape).mean(axis=(2, 3, 4)).reshape(9)
    return Abar, cg_total


def phase_averages(P, prob, lam_parts):
    """Volume-weighted averages of P over the inclusion (+) and matrix (-) phases,
    counting c+ P+ and c- P- inside composite voxels (staggered grid: computed by
    the DFMG law over its doubly-fine cells)."""
    if "Pphase" in lam_parts:
        return lam_parts["Pphase"]
    Pv = to_voxels(P)
    phase = prob.phase.reshape(-1)
    sp = Pv[phase == 1].sum(axis=0)
    sm = Pv[phase == 0].sum(axis=0)
    vp = float(np.count_nonzero(phase == 1))
    vm = float(np.count_nonzero(phase == 0))
    if lam_parts:
        c = prob.c.reshape(-1)[lam_parts["idx"]]
        sp = sp + np.einsum("m,mij->ij", c, lam_parts["Pp"])
        sm = sm + np.einsum("m,mij->ij", 1.0 - c, lam_parts["Pm"])
        vp += float(c.sum())
        vm += float((1.0 - c).sum())
    Pp = sp / vp if vp > 0 else np.zeros((3, 3))
    Pm = sm / vm if vm > 0 else np.zeros((3, 3))
    return Pp, Pm


def solve(prob, Fbar, opts=None, F_init=None):
    """Full solve along the load path.  Returns a dict with F, P, Pbar, Pbar_phase,
    Abar (if requested) and statistics; raises SolveError on failure."""
    opts = opts or Options()
    shape = prob.shape
    Fbar = np.asarray(Fbar, float).reshape(3, 3)
    if prob.law != "linear" and np.linalg.det(Fbar) <= 0:
        raise SolveError(E_INADMISSIBLE, "det Fbar <= 0")
    mu0, kappa0 = reference_medium(prob.mats, opts.mu0, opts.kappa0)
    if F_init is None:
        F = np.broadcast_to(np.eye(3)[:, :, None, None, None], (3, 3) + tuple(shape)).copy()
    else:
        F = np.array(F_init, float).reshape((3, 3) + tuple(shape))
    Fbar0 = F.mean(axis=(2, 3, 4))
    stats = dict(newton_iters=0, cg_iters=0, increments=0, step_halvings=0, cutbacks=0, cg_truncations=0,
                 lam_iters=0, lam_iters_max=0, lam_backproj=0, lam_fail=0, eta=[])

    def load(t):
        return Fbar0 + t * (Fbar - Fbar0)

    K = max(1, int(opts.n_increments))
    P = None
    lam_parts = {}
    for k in range(1, K + 1):
        t_start, t_end = (k - 1) / K, k / K
        depth = 0
        t = t_start
        dt = t_end - t_start
        while t < t_end - 1e-15:
            t_next = min(t_end, t + dt)
            F_save = F.copy()
            F = F + (load(t_next) - load(t))[:, :, None, None, None]
            converged = False
            P, Av, ok, lst, lam_parts = evaluate(F, prob)
            if ok:
                for _ in range(opts.max_newton + 1):
                    eta = residual(P, prob)
                    stats["eta"].append(eta)
                    if eta <= opts.tol_newton:
                        converged = True
                        break
                    if _ == opts.max_newton:
                        break
                    b = -gamma0(P, prob, mu0, kappa0)
                    try:
                        dF, it = cg(Av, b, prob, mu0, kappa0, opts.tol_cg, opts.max_cg)
                    except NegativeCurvature as e:
                        dF, it = e.x, e.it
                        stats["cg_truncations"] += 1
                        if it == 0:
                            stats["cg_iters"] += it
                            break
                    stats["cg_iters"] += it
                    stats["newton_iters"] += 1
                    s = 1.0
                    accepted = False
                    for h in range(opts.max_step_halvings + 1):
                        Ft = F + s * dF
                        P_t, Av_t, ok_t, lst, lp_t = evaluate(Ft, prob)
                        if ok_t and (not opts.line_search or
                                     residual(P_t, prob) <= (1.0 - LS_ARMIJO * s) * eta):
                            accepted = True
                            break
                        s *= 0.5
                        stats["step_halvings"] += 1
                    if not accepted:
                        break
                    F, P, Av, lam_parts = Ft, P_t, Av_t, lp_t
            if converged:
                for key in ("lam_iters", "lam_backproj", "lam_fail"):
                    stats[key] += lst[key]
                stats["lam_iters_max"] = max(stats["lam_iters_max"], lst["lam_iters_max"])
                t = t_next
                stats["increments"] += 1
            else:
                F = F_save
                depth += 1
                stats["cutbacks"] += 1
                if depth > opts.max_cutbacks:
                    raise SolveError(E_NOCONV, "increment %d failed after %d cutbacks" % (k, opts.max_cutbacks))
                dt *= 0.5
    Pbar = P.mean(axis=(2, 3, 4))
    Pp, Pm = phase_averages(P, prob, lam_parts)
    out = dict(F=F, P=P, Pbar=Pbar, Pbar_phase=np.stack([Pp, Pm]), stats=stats, mu0=mu0, kappa0=kappa0,
               a=lam_parts.get("a"))
    if opts.want_tangent:
        Abar, it = effective_tangent(F, prob, opts, mu0, kappa0)
        out["Abar"] = Abar
        stats["cg_iters_tangent"] = it
    return out
