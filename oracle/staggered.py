"""Staggered-grid finite differences and the doubly-fine material grid (DFMG) law
(paper App. A).  Test infrastructure: only tests/ use it.  It holds the
operators, the DFMG law, the staggered-grid Green operators, the DFMG law of the
finite-strain ComBo problem (Neo-Hooke cells and laminate cells) with its
tangent action for the Newton-CG solve of oracle.solver (Problem.disc =
"staggered"), and a small-strain CG solve on the same operators.

Fields are arrays [3, n3, n2, n1] (vectors) and [3, 3, n3, n2, n1] (tensors), x
the last array axis, cell xi = (i, j, k) at array index [k, j, i].

Placement (App. A): U_a sits on the face of cell xi normal to e_a; the diagonal
F_aa (and P_aa) at the cell centre; F_ab = F_ba (a != b) on the edge of cell xi
parallel to the third axis at the lower corner in a and b, e.g. F_12 at
(i h1, j h2, (k + 1/2) h3).

Forward and backward differences (eq. forward_backward_difference):
    D_j^+ phi[I] = (phi[I + e_j] - phi[I]) / h_j,   D_j^- phi[I] = (phi[I] - phi[I - e_j]) / h_j.
Gradient (eq. gradient_operator): F_aA = D_A^+ U_a on the diagonal, D_A^- U_a off it.

Readings (the printed formulas are not all consistent with that placement):
  * Div: the printed matrix pairs D_B with P_Ba (derivative on the first index),
    the gradient D_A with F_aA (derivative on the second).  Taken here as the
    negative adjoint of Grad, (Div P)_a = sum_A D_A^{-s} P_aA with s the sign
    Grad uses for (a, A); for a symmetric P the two agree.
  * DFMG material offsets: P^{ab}_l[xi] for a < b is printed as the law of cell
    xi + l^{+a,+b}, while the same formula takes the diagonal entries of
    F^{ab}_l from cells xi + l^{-a,-b}.  The edge of F_ab borders the cells
    xi - l^{a,b} (l_a, l_b in {0, 1}), so the law of cell xi + l^{-a,-b} is used.
  * Finite strain (the appendix states the small-strain placement and the DFMG
    formula; the finite-strain problem is read from Sec. 2-4 on this grid): the
    Lippmann-Schwinger Newton-CG solve of Sec. 3 with the staggered gradient's
    Fourier symbols g[a, A] in the Green operator,
    Gamma0_hat = g (g^H C0 g)^{-1} g^H (only the mean mode projected out), and
    the DFMG stress as the material law; the law of a cell is Neo-Hooke (Sec. 6.1)
    in pure cells and the rank-one laminate (Sec. 4, Alg. 1 and 2) in composite
    cells, evaluated at the deformation F^{ab}_l of every term of the DFMG sum.
  * Phase averages under the DFMG: each (cell, l) term of the "aa" sum is one
    doubly-fine cell of that cell's material; P+ and P- average the stress of the
    doubly-fine cells of each phase (c+ P+ and c- P- inside composite cells).
"""
import numpy as np

from . import laminate, material

AXIS = {0: -1, 1: -2, 2: -3}     # direction (x, y, z) -> array axis


def shift(phi, d, s):
    """phi[I + s e_d] for a periodic field (d = 0, 1, 2 for x, y, z)."""
    return np.roll(phi, -s, axis=AXIS[d])


def d_fwd(phi, d, h):
    return (shift(phi, d, 1) - phi) / h[d]


def d_bwd(phi, d, h):
    return (phi - shift(phi, d, -1)) / h[d]


def grad(U, h):
    """Staggered gradient [3, 3, ...] of U [3, ...] (eq. gradient_operator)."""
    F = np.empty((3, 3) + U.shape[1:])
    for a in range(3):
        for A in range(3):
            F[a, A] = d_fwd(U[a], A, h) if a == A else d_bwd(U[a], A, h)
    return F


def div(P, h):
    """Staggered divergence [3, ...] of P [3, 3, ...]: the negative adjoint of grad."""
    out = np.zeros((3,) + P.shape[2:])
    for a in range(3):
        for A in range(3):
            out[a] += d_bwd(P[a, A], A, h) if a == A else d_fwd(P[a, A], A, h)
    return out


def grad_symbols(n, l):
    """Fourier multipliers g[a, A] (shape [3, 3, n3, n2, n1], complex) of grad for
    numpy's fftn convention: fftn(grad(U))[a, A] = g[a, A] * fftn(U[a]).
    Forward difference: (e^{i theta} - 1) / h, backward: (1 - e^{-i theta}) / h,
    theta_d = 2 pi k_d / n_d."""
    h = [l[d] / n[d] for d in range(3)]
    th = []
    for d in range(3):
        t = 2.0 * np.pi * np.arange(n[d]) / n[d]
        shape = [1, 1, 1]
        shape[2 - d] = n[d]
        th.append(t.reshape(shape))
    g = np.empty((3, 3, n[2], n[1], n[0]), complex)
    for a in range(3):
        for A in range(3):
            if a == A:
                sym = (np.exp(1j * th[A]) - 1.0) / h[A]
            else:
                sym = (1.0 - np.exp(-1j * th[A])) / h[A]
            g[a, A] = np.broadcast_to(sym, (n[2], n[1], n[0]))
    return g


def _offset(l, a, b, sa, sb):
    """The cell offset l^{sa a, sb b}: l_a sa on axis a, l_b sb on axis b, 0 elsewhere."""
    o = [0, 0, 0]
    o[a] = sa * l[a]
    o[b] = sb * l[b]
    return o


def _at(field, o):
    """field[xi + o] for an offset o = (ox, oy, oz)."""
    out = field
    for d in range(3):
        if o[d]:
            out = shift(out, d, o[d])
    return out


# Sign pattern of App. A: in the matrix F^{ab}_l (a < b, or "aa" for the one of the
# diagonal stresses), entry (c, d) -> (p, q, sp, sq) is F_cd at xi + l^{sp p, sq q};
# entries not listed are F_cd[xi].
def _pattern(pair):
    if pair == "aa":
        return {(0, 1): (0, 1, +1, +1), (0, 2): (0, 2, +1, +1), (1, 2): (1, 2, +1, +1),
                (1, 0): (1, 0, +1, +1), (2, 0): (2, 0, +1, +1), (2, 1): (2, 1, +1, +1)}
    if pair == (0, 1):
        return {(0, 0): (0, 1, -1, -1), (1, 1): (0, 1, -1, -1), (2, 2): (0, 1, -1, -1),
                (0, 2): (1, 2, -1, +1), (2, 0): (1, 2, -1, +1),
                (1, 2): (0, 2, -1, +1), (2, 1): (0, 2, -1, +1)}
    if pair == (0, 2):
        return {(0, 0): (0, 2, -1, -1), (1, 1): (0, 2, -1, -1), (2, 2): (0, 2, -1, -1),
                (0, 1): (1, 2, +1, -1), (1, 0): (1, 2, +1, -1),
                (1, 2): (0, 1, -1, +1), (2, 1): (0, 1, -1, +1)}
    if pair == (1, 2):
        return {(0, 0): (1, 2, -1, -1), (1, 1): (1, 2, -1, -1), (2, 2): (1, 2, -1, -1),
                (0, 1): (0, 2, +1, -1), (1, 0): (0, 2, +1, -1),
                (0, 2): (0, 1, +1, -1), (2, 0): (0, 1, +1, -1)}
    raise ValueError(pair)


LSET = [(l1, l2, l3) for l3 in (0, 1) for l2 in (0, 1) for l1 in (0, 1)]


def dfmg_F(F, pair, l):
    """The deformation F^{pair}_l[xi] [3, 3, ...] of App. A for pair = "aa" or (a, b), a < b."""
    out = np.array(F, copy=True)
    for (c, d), (p, q, sp, sq) in _pattern(pair).items():
        out[c, d] = _at(F[c, d], _offset(l, p, q, sp, sq))
    return out


def dfmg_stress(F, law):
    """DFMG stress (eq. constitutive_law): P_ab[xi] = 1/8 sum_l (P^{ab}_l(F^{ab}_l[xi]))_ab.
    law(Fm, cell_offset) returns the stress [3, 3, ...] of the laws of cells
    xi + cell_offset evaluated at the field Fm."""
    P = np.zeros_like(F)
    for l in LSET:
        Pd = law(dfmg_F(F, "aa", l), (0, 0, 0))
        for a in range(3):
            P[a, a] += Pd[a, a] / 8.0
        for a, b in ((0, 1), (0, 2), (1, 2)):
            Po = law(dfmg_F(F, (a, b), l), _offset(l, a, b, -1, -1))
            P[a, b] += Po[a, b] / 8.0
            P[b, a] += Po[b, a] / 8.0
    return P


def linear_cells(phase, mats):
    """Law callback for dfmg_stress: the small-strain isotropic law
    sigma = lambda tr(eps) I + 2 mu eps, eps = sym(F - I), of cell xi + offset.
    Pure cells only (phase 0 or 1): composite cells have no law here."""
    bad = (phase != 0) & (phase != 1)
    if np.any(bad):
        raise ValueError("linear_cells: phase ids other than 0 and 1 (%d cells)" % int(np.count_nonzero(bad)))
    mu = np.where(phase == 1, mats[1][0], mats[0][0])
    lam = np.where(phase == 1, mats[1][1], mats[0][1])

    def law(Fm, off):
        m, la = _at(mu, off), _at(lam, off)
        Hm = Fm - np.eye(3)[:, :, None, None, None]
        eps = 0.5 * (Hm + np.swapaxes(Hm, 0, 1))
        tr = eps[0, 0] + eps[1, 1] + eps[2, 2]
        return la * tr * np.eye(3)[:, :, None, None, None] + 2.0 * m * eps
    return law


def solve_linear(phase, l, mats, Hbar, tol=1e-12, maxit=20000):
    """Small-strain equilibrium on the staggered grid with the DFMG law: find the
    periodic displacement U (zero mean) with Div P(I + Hbar + Grad U) = 0, by plain
    CG on the symmetric positive semi-definite operator U -> -Div(P(I + Grad U) - P(I)).
    Returns U, F = I + Hbar + Grad U, P and the mean stress per component."""
    n = (phase.shape[2], phase.shape[1], phase.shape[0])
    h = tuple(l[d] / n[d] for d in range(3))
    law = linear_cells(phase, mats)
    I = np.broadcast_to(np.eye(3)[:, :, None, None, None], (3, 3) + phase.shape)
    P0 = dfmg_stress(np.array(I), law)

    def A(U):
        return -div(dfmg_stress(I + grad(U, h), law) - P0, h)

    Fbar = I + np.asarray(Hbar)[:, :, None, None, None]
    b = div(dfmg_stress(Fbar, law), h)
    U = np.zeros((3,) + phase.shape)
    r = b.copy()
    p = r.copy()
    rr = np.sum(r * r)
    r0 = np.sqrt(rr)
    it = 0
    while r0 > 0 and np.sqrt(rr) > tol * r0 and it < maxit:
        Ap = A(p)
        alpha = rr / np.sum(p * Ap)
        U += alpha * p
        r -= alpha * Ap
        rr_new = np.sum(r * r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    if r0 > 0 and np.sqrt(rr) > tol * r0:
        raise RuntimeError("solve_linear: CG did not reach %g in %d iterations (%g)" % (tol, maxit, np.sqrt(rr) / r0))
    F = Fbar + grad(U, h)
    P = dfmg_stress(F, law)
    return {"U": U, "F": F, "P": P, "Pbar": P.mean(axis=(2, 3, 4)), "iters": it}


# ---- Green operators of the staggered grid -----------------------------------

def c0_tensor(mu0, kappa0):
    """C0_aAbB = mu0 d_ab d_AB + kappa0 d_aA d_bB (the reference medium of the solver)."""
    I = np.eye(3)
    return mu0 * np.einsum("ab,AB->aAbB", I, I) + kappa0 * np.einsum("aA,bB->aAbB", I, I)


def green_hat(tau_hat, g, mu0, kappa0):
    """Gamma0_hat tau_hat = g w with w = (g^H C0 g)^{-1} (g^H tau_hat), i.e.
    w_a solves sum_b K_ab w_b = sum_A conj(g_aA) tau_hat_aA with
    K_ab = sum_AB conj(g_aA) C0_aAbB g_bB; the output is F_aA = g_aA w_a.  Modes
    where every symbol vanishes (the mean) are set to zero."""
    gc = np.conj(g)
    v = np.einsum("aA...,aA...->a...", gc, tau_hat)
    K = np.einsum("aA...,aAbB,bB...->ab...", gc, c0_tensor(mu0, kappa0), g)
    mask = np.abs(g).reshape(9, -1).max(axis=0).reshape(g.shape[2:]) == 0.0
    K = np.where(mask[None, None], np.eye(3)[:, :, None, None, None], K)
    w = np.moveaxis(np.linalg.solve(np.moveaxis(K, (0, 1), (-2, -1)), np.moveaxis(v, 0, -1)[..., None])[..., 0],
                    -1, 0)
    out = g * w[:, None]
    out[:, :, mask] = 0.0
    return out


def apply_gamma0(tau, n, l, mu0, kappa0):
    """Gamma0[tau] of the staggered grid for a real field tau [3,3,n3,n2,n1]."""
    g = grad_symbols(n, l)
    th = np.fft.fftn(tau, axes=(-3, -2, -1))
    return np.fft.ifftn(green_hat(th, g, mu0, kappa0), axes=(-3, -2, -1)).real


def apply_g(tau, n, l):
    """G[tau]: Gamma0 of the reference medium mu0 = 1, kappa0 = 0."""
    return apply_gamma0(tau, n, l, 1.0, 0.0)


# ---- the finite-strain DFMG law -------------------------------------------------

def _pairs():
    """The terms of the DFMG sum: ("aa", offset rule) and the three off-diagonal pairs."""
    return ["aa", (0, 1), (0, 2), (1, 2)]


def _law_offset(pair, l):
    """Offset of the cell whose law enters term (pair, l): the cell itself for the
    diagonal stresses, xi + l^{-a,-b} for the pair (a, b) (reading above)."""
    if pair == "aa":
        return (0, 0, 0)
    a, b = pair
    return tuple(_offset(l, a, b, -1, -1))


def _comps(pair):
    if pair == "aa":
        return [(0, 0), (1, 1), (2, 2)]
    a, b = pair
    return [(a, b), (b, a)]


def cell_law(Fm, off, prob):
    """Law of the cells xi + off evaluated at Fm [3,3,n3,n2,n1]: Neo-Hooke in pure
    cells (Sec. 6.1), the laminate of Sec. 4 (Alg. 1 and 2, from a = 0) in composite
    cells.  Returns P [3,3,...], A [n,9,9], ok, laminate statistics and, for the
    composite cells, their indices with c+, P+ and P-."""
    shape = Fm.shape[2:]
    Fv = np.moveaxis(Fm.reshape(3, 3, -1), -1, 0)
    n = Fv.shape[0]
    ph = _at(prob.phase, off).reshape(-1)
    Pv = np.zeros((n, 3, 3))
    Av = np.zeros((n, 9, 9))
    ok = True
    st = dict(lam_iters=0, lam_iters_max=0, lam_backproj=0, lam_fail=0)
    for p in (0, 1):
        idx = np.nonzero(ph == p)[0]
        if idx.size == 0:
            continue
        if np.any(np.linalg.det(Fv[idx]) <= 0):
            ok = False
            continue
        Pv[idx] = material.stress(Fv[idx], *prob.mats[p])
        Av[idx] = material.tangent(Fv[idx], *prob.mats[p])
    idx = np.nonzero(ph == 2)[0]
    parts = None
    if idx.size:
        c = _at(prob.c, off).reshape(-1)[idx]
        N = np.stack([_at(prob.N[d], off).reshape(-1)[idx] for d in range(3)], axis=1)
        r = laminate.solve(Fv[idx], c, N, prob.mats[0], prob.mats[1])
        bad = r["status"] != laminate.STATUS_OK
        st.update(lam_iters=int(r["iters"].sum()), lam_iters_max=int(r["iters"].max()),
                  lam_backproj=int(r["n_backproj"].sum()), lam_fail=int(bad.sum()))
        if bad.any():
            ok = False
        Pv[idx] = r["P"]
        Av[idx] = r["A"]
        parts = dict(idx=idx, c=c, Pp=r["Pp"], Pm=r["Pm"])
    return np.moveaxis(Pv, 0, -1).reshape((3, 3) + shape), Av, ok, st, parts


def evaluate(F, prob):
    """DFMG stress (eq. constitutive_law) of the finite-strain ComBo law at the
    staggered field F, term by term as printed: for every l in L and every pair
    ("aa", (0,1), (0,2), (1,2)) the law of the cell given by _law_offset at
    F^{pair}_l[xi], of which the pair's components enter with weight 1/8.
    Returns P, the tangents of all 32 terms (the tangent object of
    tangent_action), ok, laminate statistics and the phase averages."""
    P = np.zeros_like(F)
    terms = {}
    ok = True
    st = dict(lam_iters=0, lam_iters_max=0, lam_backproj=0, lam_fail=0)
    phase = prob.phase.reshape(-1)
    sp, sm = np.zeros((3, 3)), np.zeros((3, 3))
    for l in LSET:
        for pair in _pairs():
            Pm, Am, okm, s, parts = cell_law(dfmg_F(F, pair, l), _law_offset(pair, l), prob)
            ok = ok and okm
            for k in ("lam_iters", "lam_backproj", "lam_fail"):
                st[k] += s[k]
            st["lam_iters_max"] = max(st["lam_iters_max"], s["lam_iters_max"])
            for (c, d) in _comps(pair):
                P[c, d] += Pm[c, d] / 8.0
            terms[(pair, l)] = Am
            if pair == "aa":
                # doubly-fine cells (xi, l) of the cell xi's material
                Pv = np.moveaxis(Pm.reshape(3, 3, -1), -1, 0)
                sp += Pv[phase == 1].sum(axis=0) / 8.0
                sm += Pv[phase == 0].sum(axis=0) / 8.0
                if parts is not None:
                    sp += np.einsum("m,mij->ij", parts["c"], parts["Pp"]) / 8.0
                    sm += np.einsum("m,mij->ij", 1.0 - parts["c"], parts["Pm"]) / 8.0
    vp = float(np.count_nonzero(phase == 1)) + float(prob.c.reshape(-1)[phase == 2].sum())
    vm = float(np.count_nonzero(phase == 0)) + float((1.0 - prob.c.reshape(-1)[phase == 2]).sum())
    phase_avg = (sp / vp if vp > 0 else np.zeros((3, 3)), sm / vm if vm > 0 else np.zeros((3, 3)))
    return P, terms, ok, st, dict(Pphase=phase_avg)


def tangent_action(terms, dF):
    """Linearised DFMG stress: sum over the terms of (A_term : dF^{pair}_l)_pair / 8."""
    out = np.zeros_like(dF)
    shape = dF.shape[2:]
    for (pair, l), A in terms.items():
        dFm = dfmg_F(dF, pair, l)
        v = np.moveaxis(dFm.reshape(9, -1), -1, 0)
        t = np.moveaxis(np.einsum("nab,nb->na", A, v), -1, 0).reshape((3, 3) + shape)
        for (c, d) in _comps(pair):
            out[c, d] += t[c, d] / 8.0
    return out
