"""Pins of the oracle's normal detection from fine images (paper Sec. 5): the
Laplacian weights against the Fourier-domain convolution and against their
support, exact normals of axis-aligned and symmetric planes, recovery of random
planes in equiaxed and non-equiaxed boxels (better than the barycentre normal of
eq. normal:kabel), the sign rule, equivariance under axis permutations and
reflections, the paper's composite-voxel count of the coarsened sphere, and the
rejected boxel-centre reading."""
import numpy as np
import pytest

from oracle import normals
from paper_2204_13624_amd import synth


def unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def centre_boxel(s, h, N0, off, method=normals.METHOD_LAPLACE):
    """The middle boxel of a 3 x 3 x 3-boxel image of the half space x.N0 < off (x from
    the image centre = that boxel's centre).  The image is periodic, but its outer
    faces are more than one fine voxel away from the middle boxel."""
    N = tuple(3 * x for x in s)
    l = tuple(3 * x * hh for x, hh in zip(s, h))
    img = synth.plane_image(N, l, N0, off)
    p, c, n = normals.detect_at(img, s, l, [(1, 1, 1)], method)
    return int(p[0]), float(c[0]), n[0], img, l


def test_fourier_and_direct_weights_agree():
    rng = np.random.default_rng(1)
    chi = (rng.random((8, 10, 12)) < 0.4).astype(np.uint8)
    h = (0.3, 0.5, 0.7)
    w1 = normals.laplace_weights(chi, h)
    w2 = normals.laplace_weights_fft(chi, h)
    assert np.abs(w1 - w2).max() <= 1e-12 * w1.max()


def test_anisotropic_weights_of_one_inclusion_voxel():
    """Fine voxel 1 x 2 x 4: r = (h2 h3 / h1, h1 h3 / h2, h1 h2 / h3) = (8, 2, 1/2), so the
    lone inclusion voxel weighs 2 (8 + 2 + 1/2) = 21 and its x, y, z neighbours 8, 2, 1/2;
    the same as the fine voxel volume times the plain second differences (1/h^2)."""
    chi = np.zeros((5, 5, 5), np.uint8)
    chi[2, 2, 2] = 1
    w = normals.laplace_weights(chi, (1.0, 2.0, 4.0))
    assert w[2, 2, 2] == 21.0
    assert w[2, 2, 1] == w[2, 2, 3] == 8.0
    assert w[2, 1, 2] == w[2, 3, 2] == 2.0
    assert w[1, 2, 2] == w[3, 2, 2] == 0.5
    assert w.sum() == 21.0 + 2 * (8.0 + 2.0 + 0.5)
    rng = np.random.default_rng(4)
    chi = (rng.random((6, 7, 8)) < 0.5).astype(np.uint8)
    h = (0.3, 0.5, 0.7)
    f = chi.astype(float)
    lap = sum((np.roll(f, 1, a) - 2 * f + np.roll(f, -1, a)) / hh ** 2 for a, hh in ((2, h[0]), (1, h[1]), (0, h[2])))
    assert np.abs(normals.laplace_weights(chi, h) - np.prod(h) * np.abs(lap)).max() <= 1e-14


def test_weights_vanish_exactly_away_from_the_interface():
    rng = np.random.default_rng(2)
    chi = (rng.random((9, 7, 11)) < 0.5).astype(np.uint8)
    w = normals.laplace_weights(chi, (1.0, 2.0, 0.5))
    differs = np.zeros(chi.shape, bool)
    for ax in range(3):
        for sh in (1, -1):
            differs |= np.roll(chi, sh, axis=ax) != chi
    assert np.array_equal(w > 0, differs)


@pytest.mark.parametrize("axis,side", [(0, 1), (0, -1), (1, 1), (2, -1)])
@pytest.mark.parametrize("cut", [1, 3, 5])
def test_axis_aligned_plane_gives_the_axis(axis, side, cut):
    s = (8, 6, 7)
    N0 = side * np.eye(3)[axis]
    off = (cut - 0.5 * s[axis]) * 0.1 * side
    phase, c, N, _, _ = centre_boxel(s, (0.1, 0.1, 0.1), N0, off)
    assert phase == 2
    assert np.abs(N - N0).max() <= 1e-13


def test_diagonal_plane_by_symmetry():
    s = (8, 8, 6)
    for off in (-0.31, -0.05, 0.0, 0.2):
        N0 = unit([1.0, 1.0, 0.0])
        _, _, N, _, _ = centre_boxel(s, (0.125, 0.125, 0.125), N0, off)
        assert np.abs(N - N0).max() <= 1e-12


def _angle_errors(s, h, rng, count, method):
    errs = []
    while len(errs) < count:
        N0 = unit(rng.normal(size=3))
        off = rng.uniform(-0.4, 0.4) * min(x * hh for x, hh in zip(s, h))
        phase, c, N, _, _ = centre_boxel(s, h, N0, off, method)
        if phase != 2 or not (0.05 < c < 0.95):
            continue
        errs.append(float(N @ N0))
    return np.array(errs)


@pytest.mark.parametrize("s", [(16, 16, 16), (16, 6, 8), (4, 12, 20)])
def test_random_planes_are_recovered_better_than_by_barycentres(s):
    h = (0.05, 0.05, 0.05)                  # equiaxed fine voxels, non-equiaxed boxels
    new = _angle_errors(s, h, np.random.default_rng(3), 40, normals.METHOD_LAPLACE)
    old = _angle_errors(s, h, np.random.default_rng(3), 40, normals.METHOD_BARYCENTRE)
    assert new.min() > 0.99                 # every normal within ~8 degrees, out of the inclusion
    assert np.median(new) > 0.999
    assert np.mean(np.arccos(np.minimum(new, 1))) < np.mean(np.arccos(np.minimum(old, 1)))


def test_boxel_centre_reading_fails_at_low_volume_fraction():
    """A corner cut (c ~ 3 %): moments about the boxel centre give an in-plane vector."""
    s = (16, 16, 16)
    h = (1 / 16, 1 / 16, 1 / 16)
    N0 = unit([1.0, 0.8, 0.6])
    img = synth.plane_image((48, 48, 48), (3.0, 3.0, 3.0), N0, -0.3 * np.sqrt(3) * (N0 @ unit([1, 1, 1])))
    w = normals.laplace_weights(img, h)[16:32, 16:32, 16:32]
    cb = img[16:32, 16:32, 16:32].astype(np.float64)
    x = normals._local_coords(s, h)
    assert 0.01 < cb.mean() < 0.06
    good = normals.boxel_normal(cb, w, x, about="interface")
    bad = normals.boxel_normal(cb, w, x, about="centre")
    assert good @ N0 > 0.99
    assert bad @ N0 < 0.9


def test_sphere_normals_point_out_of_the_inclusion_and_radially():
    n, S = (8, 8, 8), 12
    img = synth.sphere_image(tuple(x * S for x in n), 0.33, center=(0.02, -0.01, 0.03))
    phase, c, N = normals.detect(img, (S, S, S), (1.0, 1.0, 1.0))
    _, _, Nt = normals.detect(img, (S, S, S), (1.0, 1.0, 1.0), normals.METHOD_BARYCENTRE)
    comp = np.argwhere(phase == 2)
    assert len(comp) > 100
    cos_new, cos_old = [], []
    for k, j, i in comp:
        centre = (np.array([i, j, k]) + 0.5) / 8 - 0.5
        r = unit(centre - np.array([0.02, -0.01, 0.03]))
        cos_new.append(N[:, k, j, i] @ r)
        cos_old.append(Nt[:, k, j, i] @ r)
        assert N[:, k, j, i] @ Nt[:, k, j, i] > 0
    cos_new = np.array(cos_new)
    assert np.median(cos_new) > 0.99 and cos_new.min() > 0.8
    assert np.median(cos_new) > np.median(cos_old)


def test_paper_composite_count_of_the_coarsened_sphere():
    """Sphere R = 0.4 L on a 256^3 image coarsened to 32^3: 2624 composite voxels."""
    img = synth.sphere_image((256, 256, 256), 0.4)
    phase, c, N = normals.detect(img, (8, 8, 8), (1.0, 1.0, 1.0))
    assert int((phase == 2).sum()) == 2624
    comp = phase == 2
    assert np.abs(np.linalg.norm(N[:, comp], axis=0) - 1).max() <= 1e-13
    assert abs(c.mean() - img.mean()) <= 1e-15


def test_permutation_and_reflection_equivariance():
    s = (6, 6, 6)
    img = synth.sphere_image((24, 24, 24), 0.31, center=(0.03, 0.05, -0.02))
    img = img | synth.sphere_image((24, 24, 24), 0.12, center=(-0.4, 0.37, 0.41))
    ref = normals.detect(img, s, (1.0, 1.0, 1.0))
    # permuted array axes: new array axis a is old array axis perm[a]
    perm = (2, 0, 1)
    img_p = np.transpose(img, perm)
    out = normals.detect(img_p, s, (1.0, 1.0, 1.0))
    assert np.array_equal(out[0], np.transpose(ref[0], perm))
    # array axis a of the new image is array axis perm[a] of the old one; physical axis d = 2 - a
    phys = [2 - perm[2 - d] for d in range(3)]
    Np = np.transpose(ref[2], (0,) + tuple(p + 1 for p in perm))[phys]
    comp = out[0] == 2
    assert np.abs(out[2][:, comp] - Np[:, comp]).max() <= 1e-12
    # reflection x -> -x (array axis 2 reversed): N_x flips, the boxel order reverses
    img_r = img[:, :, ::-1]
    out = normals.detect(img_r, s, (1.0, 1.0, 1.0))
    Nr = ref[2][:, :, :, ::-1].copy()
    Nr[0] *= -1
    comp = out[0] == 2
    assert np.abs(out[2][:, comp] - Nr[:, comp]).max() <= 1e-12


def test_detect_at_matches_whole_image():
    img = synth.sphere_image((30, 24, 18), 0.3, center=(0.4, -0.45, 0.1))   # crosses the periodic faces
    s, l = (5, 4, 3), (1.0, 0.8, 0.6)
    phase, c, N = normals.detect(img, s, l)
    boxels = [tuple(b) for b in np.argwhere(np.ones_like(phase, bool))]
    p2, c2, N2 = normals.detect_at(img, s, l, boxels)
    assert np.array_equal(p2, phase.reshape(-1))
    assert np.array_equal(c2, c.reshape(-1))
    assert np.abs(N2 - N.reshape(3, -1).T).max() <= 1e-13
