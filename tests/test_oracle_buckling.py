"""Loss of stability of a straight stiff inclusion in compression, on the oracle.

The fibre workload (paper Sec. 6.5 stand-in) pairs a near-incompressible matrix
(mu = 1, lambda = 1000) with stiff fibres (contrast 1000), and its load walk stops
where Newton steps meet negative curvature and the line search cannot lower the
residual.  This test shows the mechanism on a problem small enough for dense linear
algebra: a stiff layer two voxels thick in that matrix (a 16 x 8 x 1 grid, the
layer normal along y, the cell twice as long along x as along y), compressed along
the layer by Fbar = diag(1 - eps, 1, 1).

- The solve from F = I follows the straight branch: by symmetry F stays uniform along x.
- The second variation of the energy on compatible fields (paper Sec. 3: the
  tangent A of the law, restricted to the range of the compatibility projector
  G) is positive definite at 0.4 % compression and indefinite at 1 %, with
  lambda_min falling monotonically in between.
- The unstable mode is a degenerate pair made only of the longest wave the cell
  admits along the layer (kx = +-1): the layer bends and the matrix follows.
- Past that load, a solve started a little off the straight branch fails (Newton
  cannot find an equilibrium nearby).  Below it, the same start returns to the
  straight solution.

The critical compression found here belongs to a layer only two voxels thick: with
strains sampled at voxel centres such a layer is far softer in bending than a
continuum plate, and the same layer resolved by four or eight voxels is still stable
at 3 % compression.  The test shows the mechanism, not a critical load.

The oracle alone is used; the inputs come from the seeded generators."""
import numpy as np
import pytest

from oracle import solver as osol
from oracle import spectral as ospec
from paper_2204_13624_amd import synth

MATS = ((1.0, 1000.0), (1000.0, 1.0e6))     # matrix, stiff phase (mu, lambda)
N = (16, 8, 1)
L = (2.0, 1.0, 0.125)
OPTS = dict(tol_newton=1e-9, tol_cg=1e-12)


@pytest.fixture(scope="module")
def setup():
    h2 = L[1] / N[1]
    ms = synth.layered(N, L, 1, (-0.5 + 3 * h2, -0.5 + 5 * h2))
    assert ms.n_composite == 0 and int((ms.phase == 1).sum()) == 2 * N[0]
    prob = osol.Problem(ms.n, ms.l, ms.phase, ms.c, ms.N, MATS)
    nv = int(np.prod(N))
    G = np.empty((9 * nv, 9 * nv))
    e = np.zeros(9 * nv)
    for k in range(9 * nv):
        e[k] = 1.0
        G[:, k] = ospec.apply_g(e.reshape((3, 3) + tuple(prob.shape)), N, L).reshape(-1)
        e[k] = 0.0
    w, V = np.linalg.eigh(0.5 * (G + G.T))
    Q = V[:, w > 0.5]                       # orthonormal basis of the compatible fields
    return ms, prob, Q


def spectrum(F, prob, Q):
    """Eigenvalues and eigenvectors of Q^T A Q, A the pointwise tangent at F."""
    _, Av, ok, _, _ = osol.evaluate(F, prob)
    assert ok
    nv = prob.nvox
    A = np.zeros((9 * nv, 9 * nv))
    for v in range(nv):                     # field layout [3,3,n3,n2,n1]: entry c*nv + v
        idx = np.arange(9) * nv + v
        A[np.ix_(idx, idx)] = Av[v]
    M = Q.T @ A @ Q
    lam, U = np.linalg.eigh(0.5 * (M + M.T))
    return lam, Q @ U


def straight_solution(prob, eps):
    r = osol.solve(prob, np.diag([1.0 - eps, 1.0, 1.0]), osol.Options(**OPTS))
    return r["F"]


def test_compatible_space_is_the_gradient_space(setup):
    """The range of G holds three displacement components per frequency with a
    non-zero, non-Nyquist wave vector (the Nyquist planes carry no gradient)."""
    _, prob, Q = setup
    n1, n2, n3 = N
    freqs = n1 * n2 * n3 - 1 - (n2 * n3 + n1 * n3 - n3)     # drop zero and the kx, ky Nyquist planes
    assert Q.shape[1] == 3 * freqs
    # At F = I the tangent is the small-strain stiffness C.  Every phase is no softer
    # than the matrix, and for gradient fields the sum of p:p^T equals that of
    # tr(p)^2, so the sum of p:C:p is at least mu_m |p|^2 + (lambda_m + mu_m) tr(p)^2:
    # lambda_min >= mu_m.  The bound is reached by antiplane fields u3(y) whose
    # gradient vanishes at the layer's voxel centres (the quadratic form only sees
    # voxel values).
    lam, _ = spectrum(np.broadcast_to(np.eye(3)[:, :, None, None, None], (3, 3) + tuple(prob.shape)).copy(),
                      prob, Q)
    assert abs(lam[0] - MATS[0][0]) <= 1e-8


def test_straight_branch_loses_stability(setup):
    ms, prob, Q = setup
    lam_min = []
    for eps in (0.004, 0.007, 0.01):
        F = straight_solution(prob, eps)
        assert np.abs(F - F.mean(axis=-1, keepdims=True)).max() <= 1e-12     # uniform along the layer
        lam, H = spectrum(F, prob, Q)
        lam_min.append(lam[0])
        # the two lowest modes: a degenerate pair (sine and cosine of one wave)
        assert abs(lam[0] - lam[1]) <= 1e-8 * max(1.0, abs(lam[0])) and lam[2] - lam[1] > 0.1
        for j in (0, 1):
            h = H[:, j].reshape((3, 3) + tuple(prob.shape))
            px = (np.abs(np.fft.fft(h, axis=-1)) ** 2).sum(axis=(0, 1, 2, 3))
            assert (px[1] + px[-1]) / px.sum() > 1 - 1e-10                    # kx = +-1 only
            assert (h[..., ms.phase == 1] ** 2).sum() < 0.2                   # mostly in the matrix
        if eps == 0.004:
            assert lam[0] > 0.3
        if eps == 0.01:
            assert lam[0] < -0.3 and lam[2] > 0                               # exactly the pair is unstable
    assert lam_min[0] > lam_min[1] > lam_min[2]


@pytest.mark.parametrize("eps,stable", [(0.004, True), (0.01, False)])
def test_perturbed_start(setup, eps, stable):
    _, prob, _ = setup
    F = straight_solution(prob, eps)
    p = ospec.apply_g(np.random.default_rng(3).normal(size=(3, 3) + tuple(prob.shape)), N, L)
    F0 = F + 1e-3 * p / np.abs(p).max()    # compatible, zero mean: the same Fbar
    if stable:
        r = osol.solve(prob, np.diag([1.0 - eps, 1.0, 1.0]), osol.Options(**OPTS), F_init=F0)
        assert np.abs(r["F"] - F).max() <= 1e-9
    else:
        with pytest.raises(osol.SolveError):
            osol.solve(prob, np.diag([1.0 - eps, 1.0, 1.0]), osol.Options(**OPTS), F_init=F0)
