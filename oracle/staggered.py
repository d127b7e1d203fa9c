"""Staggered-grid finite differences and the doubly-fine material grid (DFMG) law
(paper App. A).  Test infrastructure: only tests/ use it.  It holds the
operators, the DFMG law and a small-strain CG solve on them; the finite-strain
Newton solve and a GPU path of this discretization do not exist yet.

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
"""
import numpy as np

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
