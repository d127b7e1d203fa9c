"""Composite boxel (ComBo) rank-one laminate law at finite strain (paper Sec. 4),
and its infinitesimal-strain closed form (appendix cheat sheet, solve_small).

A composite voxel with inclusion fraction c+ = c, matrix fraction c- = 1 - c and
interface normal N (out of the inclusion) receives the voxel deformation F_box.
The phases deform as (eq. Fpm, Sec. 4.1)
    F+- = F_box +- (a (x) N) / c+-
so that <F> = F_box, and the jump vector a solves traction continuity
(eqs. hadamard:T, tractionbalance)
    f(a) = (P+ - P-) N = 0
under the admissibility constraint J+ > 0, J- > 0 (eq. Jpm:volumeConstraint).

Newton-Raphson (Alg. 1) uses the Hessian of eq. Hessian:F,
    Delta = D^T (A+/c+ + A-/c-) D,
with D the 9x3 matrix that maps a to the row-major vector of a (x) N, i.e.
D[3i+J, k] = delta_ik N_J.  (The matrix printed in Sec. 4.1.1 lists its rows in
an order that contradicts the row-major vector of Sec. 1.5; the definition
"D a = vec(a (x) N)" that the paper states above it is what is used.)

Admissibility (Sec. 4.2, eq. matrixlemma): with v = F_box^{-T} N,
m = v/|v|, beta_c^+ = -c+/|v|, beta_c^- = +c-/|v|, an iterate is admissible iff
beta_c^+ < a.m < beta_c^-.  An inadmissible naive update a1 from the admissible
previous iterate a0 is replaced by the selective back-projection of Alg. 2:
beta* = (a0.m + beta_c)/2 with beta_c the bound that a1.m crossed, and
a* = (I - m (x) m) a1 + beta* m.

At convergence (Sec. 4.1.1, eq. Peff:Seff and the tangent that follows it)
    P_box = c+ P+ + c- P-
    A_box = c+ A+ + c- A- - dA D Delta^{-1} D^T dA,   dA = A+ - A-.
(The paper prints "c+ A+ + c- A+" in the first term; the cheat sheet of the
appendix writes the volume average of the two tangents, which is what is used.)

Readings where the paper is silent:
  * the stopping tolerance eps is not given: |f| <= 1e-12 max(|P+ N|, |P- N|,
    1e-3 max(mu+, mu-), 1e-2 max(lambda+, lambda-)) -- the last term keeps the
    test above the round-off of lambda ln J (about eps lambda) in nearly
    incompressible phases -- or, where round-off in f stalls above that, as for
    a nearly collapsed soft phase -- a Newton correction |Delta^{-1} f| <=
    1e-13 max(|a|, 1e-3) (the current iterate is kept); at most 50 updates;
  * the oracle always starts from a = 0 (the paper's stated initialisation);
  * admissibility is strict, as in eq. matrixlemma; J_box > 0 is required first.
"""
import numpy as np

from . import material

STATUS_OK = 0
STATUS_MAXIT = 1
STATUS_BAD_FBOX = 2
STATUS_INADMISSIBLE = 3

MAX_ITERS = 50
REL_TOL = 1e-12
STEP_TOL = 1e-13


def jump_matrix(N):
    """D with D a = vec(a (x) N): D[3i+J, k] = delta_ik N_J.  N [m,3] -> D [m,9,3]."""
    m = N.shape[0]
    D = np.zeros((m, 3, 3, 3))
    for i in range(3):
        D[:, i, :, i] = N          # D[i, J, k=i] = N_J
    return D.reshape(m, 9, 3)


def phase_deformations(Fbox, a, c, N):
    """F+ and F- of eq. Fpm."""
    aN = np.einsum("mi,mJ->miJ", a, N)
    Fp = Fbox + aN / c[:, None, None]
    Fm = Fbox - aN / (1.0 - c)[:, None, None]
    return Fp, Fm


def admissibility_data(Fbox, c, N):
    """m_beta and the two critical values beta_c^+ < 0 < beta_c^- (Sec. 4.2)."""
    FinvT = np.swapaxes(np.linalg.inv(Fbox), -1, -2)
    v = np.einsum("mij,mj->mi", FinvT, N)
    nv = np.linalg.norm(v, axis=1)
    mb = v / nv[:, None]
    return mb, -c / nv, (1.0 - c) / nv


def backproject(a1, a0, mb, beta_p, beta_m):
    """Alg. 2: move only the m_beta component of an inadmissible a1."""
    beta1 = np.einsum("mi,mi->m", a1, mb)
    beta0 = np.einsum("mi,mi->m", a0, mb)
    beta_c = np.where(beta1 <= beta_p, beta_p, beta_m)
    beta_s = 0.5 * (beta0 + beta_c)
    return a1 - beta1[:, None] * mb + beta_s[:, None] * mb


def solve(Fbox, c, N, mat_minus, mat_plus, backprojection=True, maxit=MAX_ITERS, a_init=None,
          trace=False):
    """Evaluate the laminate law for m composite voxels.

    Fbox [m,3,3], c [m] (= c+), N [m,3] unit normals, materials (mu, lambda).
    Returns dict with P [m,3,3], A [m,9,9], a [m,3], iters [m], n_backproj [m],
    status [m] and, with trace=True, the list of iterates.
    """
    Fbox = np.asarray(Fbox, float)
    c = np.asarray(c, float)
    N = np.asarray(N, float)
    m = Fbox.shape[0]
    (mu_m, lam_m), (mu_p, lam_p) = mat_minus, mat_plus
    cp, cm = c, 1.0 - c
    Jbox = np.linalg.det(Fbox)
    status = np.full(m, STATUS_MAXIT, dtype=int)
    good = Jbox > 0
    status[~good] = STATUS_BAD_FBOX
    Fsafe = np.where(good[:, None, None], Fbox, np.eye(3))
    mb, beta_p, beta_m = admissibility_data(Fsafe, c, N)
    D = jump_matrix(N)
    DT = np.swapaxes(D, 1, 2)
    a = np.zeros((m, 3)) if a_init is None else np.array(a_init, float)
    iters = np.zeros(m, dtype=int)
    nbp = np.zeros(m, dtype=int)
    active = good.copy()
    history = [a.copy()] if trace else None
    # scale floor of the traction test: 1e-3 max mu for small loads, and 1e-2 max lambda
    # so that the tolerance (1e-14 lambda ~ 45 eps lambda) stays above the round-off of
    # lambda ln J in nearly incompressible phases, where |f| cannot get below ~eps lambda
    floor = max(1e-3 * max(mu_m, mu_p), 1e-2 * max(lam_m, lam_p))
    while True:
        Fp, Fm = phase_deformations(Fsafe, a, c, N)
        with np.errstate(invalid="ignore", divide="ignore"):
            Pp = material.stress(Fp, mu_p, lam_p)
            Pm = material.stress(Fm, mu_m, lam_m)
            Ap = material.tangent(Fp, mu_p, lam_p)
            Am = material.tangent(Fm, mu_m, lam_m)
        tp = np.einsum("miJ,mJ->mi", Pp, N)
        tm = np.einsum("miJ,mJ->mi", Pm, N)
        f = tp - tm
        err = np.linalg.norm(f, axis=1)
        tol = REL_TOL * np.maximum(np.maximum(np.linalg.norm(tp, axis=1), np.linalg.norm(tm, axis=1)), floor)
        bad = active & ~np.isfinite(err)
        status[bad] = STATUS_INADMISSIBLE
        active &= ~bad
        done = active & (err <= tol)
        status[done] = STATUS_OK
        active &= ~done
        if not active.any():
            break
        Delta = DT @ (Ap / cp[:, None, None] + Am / cm[:, None, None]) @ D
        da = np.zeros_like(a)
        da[active] = np.linalg.solve(Delta[active], f[active][..., None])[..., 0]
        # stagnation at round-off: the Newton correction is negligible against a
        small = active & (np.linalg.norm(da, axis=1) <= STEP_TOL * np.maximum(np.linalg.norm(a, axis=1), 1e-3))
        status[small] = STATUS_OK
        active &= ~small
        upd = active & (iters < maxit)
        if not upd.any():
            break
        a1 = a - da
        if backprojection:
            beta1 = np.einsum("mi,mi->m", a1, mb)
            inadm = upd & ~((beta_p < beta1) & (beta1 < beta_m))
            if inadm.any():
                a1[inadm] = backproject(a1[inadm], a[inadm], mb[inadm], beta_p[inadm], beta_m[inadm])
                nbp[inadm] += 1
        a = np.where(upd[:, None], a1, a)
        iters[upd] += 1
        if trace:
            history.append(a.copy())
    Pbox = cp[:, None, None] * Pp + cm[:, None, None] * Pm
    Delta = DT @ (Ap / cp[:, None, None] + Am / cm[:, None, None]) @ D
    dA = Ap - Am
    with np.errstate(invalid="ignore"):
        Dinv = np.linalg.inv(np.where(np.isfinite(Delta), Delta, np.eye(3)))
    corr = dA @ D @ Dinv @ DT @ dA
    Abox = cp[:, None, None] * Ap + cm[:, None, None] * Am - corr
    out = dict(P=Pbox, A=Abox, a=a, iters=iters, n_backproj=nbp, status=status,
               Pp=Pp, Pm=Pm, Fp=Fp, Fm=Fm)
    if trace:
        out["history"] = history
        out["m_beta"] = mb
        out["beta_c"] = (beta_p, beta_m)
    return out


def solve_small(Hbox, c, N, mat_minus, mat_plus):
    """Small-strain ComBo laminate in closed form (appendix cheat sheet, right column).

    Hbox [m,3,3] displacement gradient of the voxel (eps_box = sym(Hbox)),
    c [m] = c+, N [m,3], materials (mu, lambda) of isotropic phases.  With
    C+- the stiffnesses (isotropic_stiffness) and dC = C+ - C-:
        Delta_ik = N_j (C+/c+ + C-/c-)_ijkl N_l              (Hessian row)
        a = Delta^{-1} [(C- - C+) : eps_box] N               (update of a)
        eps+- = eps_box +- sym(a (x) N) / c+-                (deformation row)
        sigma_box = c+ C+ : eps+ + c- C- : eps-              (stress row)
        C_box = c+ C+ + c- C- - dC D Delta^{-1} D^T dC       (tangent row)
    with D the 9x3 map a -> vec(a (x) N) of the finite-strain law.  The law is
    linear, so no iteration is needed and C_box : eps_box = sigma_box.
    Returns P (= sigma_box) [m,3,3], A (= C_box) [m,9,9], a [m,3] and the
    phase strains and stresses (Pp, Pm are sigma+-)."""
    H = np.asarray(Hbox, float)
    c = np.asarray(c, float)
    N = np.asarray(N, float)
    (mu_m, lam_m), (mu_p, lam_p) = mat_minus, mat_plus
    cp, cm = c, 1.0 - c
    Cp = material.isotropic_stiffness(mu_p, lam_p).reshape(3, 3, 3, 3)
    Cm = material.isotropic_stiffness(mu_m, lam_m).reshape(3, 3, 3, 3)
    eps = 0.5 * (H + np.swapaxes(H, -1, -2))
    Delta = (np.einsum("mj,ijkl,ml->mik", N, Cp, N) / cp[:, None, None]
             + np.einsum("mj,ijkl,ml->mik", N, Cm, N) / cm[:, None, None])
    rhs = np.einsum("ijkl,mkl,mj->mi", Cm - Cp, eps, N)
    a = np.linalg.solve(Delta, rhs[..., None])[..., 0]
    aN = np.einsum("mi,mj->mij", a, N)
    saN = 0.5 * (aN + np.swapaxes(aN, 1, 2))
    eps_p = eps + saN / cp[:, None, None]
    eps_m = eps - saN / cm[:, None, None]
    sig_p = np.einsum("ijkl,mkl->mij", Cp, eps_p)
    sig_m = np.einsum("ijkl,mkl->mij", Cm, eps_m)
    P = cp[:, None, None] * sig_p + cm[:, None, None] * sig_m
    D = jump_matrix(N)
    dC = (Cp - Cm).reshape(9, 9)
    Cbar = (cp[:, None, None] * Cp.reshape(1, 9, 9) + cm[:, None, None] * Cm.reshape(1, 9, 9))
    A = Cbar - dC @ D @ np.linalg.inv(Delta) @ np.swapaxes(D, 1, 2) @ dC
    m = H.shape[0]
    return dict(P=P, A=A, a=a, iters=np.zeros(m, dtype=int), n_backproj=np.zeros(m, dtype=int),
                status=np.full(m, STATUS_OK, dtype=int), Pp=sig_p, Pm=sig_m, eps_p=eps_p, eps_m=eps_m)


def potential(a, Fbox, c, N, mat_minus, mat_plus):
    """Phi(a) = c+ W+(F+) + c- W-(F-); f = dPhi/da (used only by the tests)."""
    Fp, Fm = phase_deformations(Fbox, a, c, N)
    return (c * material.energy(Fp, *mat_plus) + (1.0 - c) * material.energy(Fm, *mat_minus))
