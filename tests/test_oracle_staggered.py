"""Pins of the oracle's staggered-grid operators and DFMG law (paper App. A):
summation by parts between Grad and Div (which also shows why the printed
divergence is read as the adjoint form), the real-space stencils against their
Fourier symbols derived separately, the DFMG law equal to the pointwise law for a
homogeneous material (uniform F: any law; any F: a linear law), and, for two
phases under the small-strain law, the shear stress on an edge equal to the mean
shear modulus of the four cells around that edge (which fixes the reading of the
material offsets), and the whole DFMG law under Neo-Hooke against a construction
of the doubly-fine grid from the variables' coordinates."""
import numpy as np
import pytest

from oracle import material, staggered as st

N = (6, 5, 4)
L = (1.2, 0.9, 0.7)
H = tuple(a / b for a, b in zip(L, N))
MATS = ((1.0, 2.0), (30.0, 45.0))


def rand_field(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def test_div_is_negative_adjoint_of_grad():
    U = rand_field((3, N[2], N[1], N[0]), 1)
    P = rand_field((3, 3, N[2], N[1], N[0]), 2)            # not symmetric
    lhs = np.sum(st.grad(U, H) * P)
    rhs = -np.sum(U * st.div(P, H))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the printed divergence (derivative on the first index of P) is not the adjoint
    # for a non-symmetric P; it is for a symmetric one
    Pt = np.swapaxes(P, 0, 1)
    assert abs(np.sum(U * st.div(Pt, H)) + lhs) > 1e-3 * abs(lhs)
    S = P + Pt
    assert abs(np.sum(st.grad(U, H) * S) + np.sum(U * st.div(np.swapaxes(S, 0, 1), H))) <= 1e-12 * abs(lhs)


def test_stencils_match_fourier_symbols():
    U = rand_field((3, N[2], N[1], N[0]), 3)
    g = st.grad_symbols(N, L)
    Fh = np.fft.fftn(st.grad(U, H), axes=(-3, -2, -1))
    Uh = np.fft.fftn(U, axes=(-3, -2, -1))
    ref = g * Uh[:, None]
    assert np.abs(Fh - ref).max() <= 1e-12 * np.abs(ref).max()
    # Div has the symbol -conj(g) (its negative adjoint)
    P = rand_field((3, 3, N[2], N[1], N[0]), 4)
    Dh = np.fft.fftn(st.div(P, H), axes=(-3, -2, -1))
    refd = np.einsum("aA...,aA...->a...", -np.conj(g), np.fft.fftn(P, axes=(-3, -2, -1)))
    assert np.abs(Dh - refd).max() <= 1e-12 * np.abs(refd).max()
    # symbols of the mean mode vanish; the gradient of a constant field is zero
    assert np.abs(g[..., 0, 0, 0]).max() == 0.0
    assert np.abs(st.grad(np.ones_like(U), H)).max() <= 1e-15


def law_cells(phase, law):
    """A law callback for dfmg_stress: the law of cell xi + offset at each xi."""
    def f(Fm, off):
        ph = st._at(phase, off)
        m = Fm.reshape(3, 3, -1).transpose(2, 0, 1)
        out = np.empty_like(m)
        for p in (0, 1):
            sel = ph.reshape(-1) == p
            if sel.any():
                out[sel] = law(m[sel], *MATS[p])
        return out.transpose(1, 2, 0).reshape(Fm.shape)
    return f


def pointwise(F, law, mu, lam):
    m = F.reshape(3, 3, -1).transpose(2, 0, 1)
    return law(m, mu, lam).transpose(1, 2, 0).reshape(F.shape)


def test_dfmg_is_the_law_for_uniform_F_in_one_material():
    Fbar = np.array([[1.08, 0.12, -0.03], [0.05, 0.97, 0.04], [-0.02, 0.06, 1.02]])
    F = np.broadcast_to(Fbar[:, :, None, None, None], (3, 3, N[2], N[1], N[0])).copy()
    phase = np.ones((N[2], N[1], N[0]), int)
    P = st.dfmg_stress(F, law_cells(phase, material.stress))
    ref = material.stress(Fbar[None], *MATS[1])[0]
    assert np.abs(P - ref[:, :, None, None, None]).max() <= 1e-14 * np.abs(ref).max()


def test_dfmg_of_a_homogeneous_linear_law_is_pointwise():
    """The linear law reads only the colocated entries of F^{ab}_l: the diagonal of
    F^{aa}_l (all unshifted) for P_aa and F_ab, F_ba (unshifted in F^{ab}_l) for P_ab."""
    F = np.eye(3)[:, :, None, None, None] + 0.1 * rand_field((3, 3, N[2], N[1], N[0]), 5)
    phase = np.zeros((N[2], N[1], N[0]), int)
    P = st.dfmg_stress(F, law_cells(phase, material.linear_stress))
    ref = pointwise(F, material.linear_stress, *MATS[0])
    assert np.abs(P - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("seed", [6, 7])
def test_dfmg_shear_on_an_edge_uses_the_four_cells_around_it(seed):
    """Two phases, small strain: P_aa[xi] is the law of cell xi; P_ab[xi] (a < b) is
    mu_edge (F_ab + F_ba)[xi] with mu_edge the mean shear modulus of the cells
    xi - (l_a e_a + l_b e_b), l in {0, 1}^2, which border the edge of F_ab."""
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, 2, size=(N[2], N[1], N[0]))
    F = np.eye(3)[:, :, None, None, None] + 0.1 * rng.normal(size=(3, 3, N[2], N[1], N[0]))
    P = st.dfmg_stress(F, law_cells(phase, material.linear_stress))
    mu = np.where(phase == 1, MATS[1][0], MATS[0][0])
    lam = np.where(phase == 1, MATS[1][1], MATS[0][1])
    tr = F[0, 0] + F[1, 1] + F[2, 2] - 3.0
    for a in range(3):
        ref = lam * tr + 2.0 * mu * (F[a, a] - 1.0)
        assert np.abs(P[a, a] - ref).max() <= 1e-13 * np.abs(ref).max()
    for a, b in ((0, 1), (0, 2), (1, 2)):
        mu_e = np.zeros_like(mu)
        for la in (0, 1):
            for lb in (0, 1):
                o = [0, 0, 0]
                o[a] = -la
                o[b] = -lb
                mu_e += st._at(mu, o) / 4.0
        ref = mu_e * (F[a, b] + F[b, a])
        assert np.abs(P[a, b] - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(P[b, a] - ref).max() <= 1e-13 * np.abs(ref).max()
        # the offsets as printed (cells xi + l^{+a,+b}) give another average
        mu_p = np.zeros_like(mu)
        for la in (0, 1):
            for lb in (0, 1):
                o = [0, 0, 0]
                o[a] = la
                o[b] = lb
                mu_p += st._at(mu, o) / 4.0
        assert np.abs(mu_p - mu_e).max() > 1.0


def dfmg_by_geometry(F, phase, law):
    """The DFMG law built from the placement alone: each of the 8 n doubly-fine cells
    S = (X, Y, Z) takes every F_cd from the variable on its boundary (diagonal: its
    cell's centre; F_ab = F_ba: the edge of the a-b plane through the nearest grid
    lines in a and b), is evaluated with its cell's law, and each P_ab is the mean
    over the 8 doubly-fine cells that share its variable."""
    n3, n2, n1 = phase.shape
    Xs, Ys, Zs = np.meshgrid(np.arange(2 * n1), np.arange(2 * n2), np.arange(2 * n3), indexing="ij")
    Xs, Ys, Zs = Xs.ravel(), Ys.ravel(), Zs.ravel()
    cell = (Xs // 2, Ys // 2, Zs // 2)
    edge = ((Xs + 1) // 2 % n1, (Ys + 1) // 2 % n2, (Zs + 1) // 2 % n3)   # nearest grid line per axis
    def idx(d, on_line):
        return edge[d] if on_line else cell[d]
    Fs = np.empty((Xs.size, 3, 3))
    for c in range(3):
        for d in range(3):
            lines = {c, d} if c != d else set()
            i, j, k = (idx(0, 0 in lines), idx(1, 1 in lines), idx(2, 2 in lines))
            Fs[:, c, d] = F[c, d][k, j, i]
    ph = phase[cell[2], cell[1], cell[0]]
    Ps = np.empty_like(Fs)
    for p in (0, 1):
        sel = ph == p
        Ps[sel] = law(Fs[sel], *MATS[p])
    P = np.zeros_like(F)
    cnt = np.zeros((3, 3) + phase.shape)
    for c in range(3):
        for d in range(3):
            lines = {c, d} if c != d else set()
            i, j, k = (idx(0, 0 in lines), idx(1, 1 in lines), idx(2, 2 in lines))
            np.add.at(P[c, d], (k, j, i), Ps[:, c, d])
            np.add.at(cnt[c, d], (k, j, i), 1.0)
    assert (cnt == 8).all()
    return P / 8.0


@pytest.mark.parametrize("n,seed", [((4, 3, 3), 8), ((3, 4, 5), 9)])
def test_dfmg_equals_the_doubly_fine_grid_construction(n, seed):
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, 2, size=(n[2], n[1], n[0]))
    F = np.eye(3)[:, :, None, None, None] + 0.15 * rng.normal(size=(3, 3, n[2], n[1], n[0]))
    P = st.dfmg_stress(F, law_cells(phase, material.stress))
    ref = dfmg_by_geometry(F, phase, material.stress)
    assert np.abs(P - ref).max() <= 1e-13 * np.abs(ref).max()


def test_linear_operator_is_symmetric():
    rng = np.random.default_rng(10)
    n = (5, 4, 3)
    phase = rng.integers(0, 2, size=(n[2], n[1], n[0]))
    h = tuple(a / b for a, b in zip(L, n))
    law = st.linear_cells(phase, MATS)
    I = np.broadcast_to(np.eye(3)[:, :, None, None, None], (3, 3) + phase.shape)
    P0 = st.dfmg_stress(np.array(I), law)
    A = lambda U: -st.div(st.dfmg_stress(I + st.grad(U, h), law) - P0, h)
    u, v = rng.normal(size=(2, 3) + phase.shape)
    assert abs(np.sum(A(u) * v) - np.sum(u * A(v))) <= 1e-12 * abs(np.sum(A(u) * v))
    assert np.sum(A(u) * u) > 0


def test_linear_solve_homogeneous_is_uniform():
    phase = np.zeros((3, 4, 5), int)
    Hb = np.array([[0.01, 0.004, -0.002], [0.001, -0.006, 0.003], [0.005, -0.001, 0.008]])
    r = st.solve_linear(phase, L, MATS, Hb)
    mu, lam = MATS[0]
    eps = 0.5 * (Hb + Hb.T)
    ref = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
    assert np.abs(r["U"]).max() <= 1e-14
    assert np.abs(r["Pbar"] - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("seed", [11, 12])
def test_linear_solve_of_a_shear_laminate_has_the_closed_form(seed):
    """Layers normal to x (phase depends on i only) under H = gamma e2 (x) e1: only U_2(i)
    moves; P_21 = mu_e F_21 on the edges x = i h1 with mu_e = (mu[i-1] + mu[i]) / 2 (DFMG
    edge modulus); Div P = 0 makes P_21 uniform, and sum_i (F_21 - gamma) = 0 gives
    P_21 = P_12 = gamma / mean_i(1 / mu_e), every other stress 0."""
    rng = np.random.default_rng(seed)
    n = (8, 3, 2)
    layers = rng.integers(0, 2, size=n[0])
    layers[:2] = (0, 1)
    phase = np.broadcast_to(layers[None, None, :], (n[2], n[1], n[0])).copy()
    gamma = 0.02
    Hb = np.zeros((3, 3))
    Hb[1, 0] = gamma
    r = st.solve_linear(phase, L, MATS, Hb)
    mu = np.where(layers == 1, MATS[1][0], MATS[0][0])
    mu_e = 0.5 * (np.roll(mu, 1) + mu)
    tau = gamma / np.mean(1.0 / mu_e)
    assert abs(r["Pbar"][1, 0] - tau) <= 1e-10 * tau
    assert abs(r["Pbar"][0, 1] - tau) <= 1e-10 * tau
    assert np.abs(r["P"][1, 0] - tau).max() <= 1e-10 * tau
    others = [(a, b) for a in range(3) for b in range(3) if (a, b) not in ((1, 0), (0, 1))]
    assert max(np.abs(r["P"][a, b]).max() for a, b in others) <= 1e-10 * tau


def test_linear_cells_and_solve_refuse_what_they_cannot_do():
    """Composite cells (phase 2) have no law in the small-strain DFMG callback, and
    a CG that stops at its iteration cap is an error, not a result."""
    phase = np.zeros((3, 4, 5), np.uint8)
    phase[1, 2, 3] = 2
    with pytest.raises(ValueError):
        st.linear_cells(phase, ((1.0, 2.0), (10.0, 20.0)))
    phase[1, 2, 3] = 1
    with pytest.raises(RuntimeError):
        st.solve_linear(phase, (1.0, 1.0, 1.0), ((1.0, 2.0), (10.0, 20.0)),
                               np.array([[0.0, 0.01, 0], [0.01, 0, 0], [0, 0, 0.0]]), maxit=2)
