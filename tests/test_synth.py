"""Pins of the input generator: the composite-voxel count the paper reports for
its sphere example (Sec. 6.2), unit outward normals, and determinism."""
import numpy as np

from paper_2204_13624_amd import synth


def test_sphere_composite_count_matches_paper():
    # Sphere R = 0.4 L on a 256^3 image coarsened to 32^3: the paper reports
    # 2624 composite voxels (Sec. 6.2).  With 8^3 subsamples per voxel:
    ms = synth.single_sphere((32, 32, 32), radius=0.4, S=8)
    assert ms.n_composite == 2624


def test_normals_point_out_of_the_inclusion():
    ms = synth.single_sphere((16, 16, 16), radius=0.3, S=4)
    comp = ms.phase == synth.PHASE_COMPOSITE
    n1 = ms.n[0]
    x = -0.5 + (np.arange(n1) + 0.5) / n1
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    radial = np.stack([X, Y, Z])
    radial /= np.linalg.norm(radial, axis=0, keepdims=True)
    dots = (ms.N * radial).sum(axis=0)[comp]
    assert np.allclose(np.linalg.norm(ms.N[:, comp], axis=0), 1.0)
    assert dots.min() > 0.8
    assert 0.0 < ms.c[comp].min() and ms.c[comp].max() < 1.0


def test_sphere_fraction_and_determinism():
    a, _ = synth.workload_spheres_64()
    b, _ = synth.workload_spheres_64()
    assert np.array_equal(a.phase, b.phase) and np.array_equal(a.N, b.N)
    assert abs(a.c.mean() - 0.25) < 2e-3


def test_layered_normals_and_fractions():
    ms = synth.layered((9, 2, 3), (1.0, 1.0, 1.0), 0, (-0.5 + 2.25 / 9, -0.5 + 6.5 / 9))
    comp = np.nonzero(ms.phase[0, 0] == 2)[0]
    assert list(comp) == [2, 6]
    assert np.allclose(ms.N[:, 0, 0, 2], [-1, 0, 0]) and np.allclose(ms.N[:, 0, 0, 6], [1, 0, 0])
    assert np.isclose(ms.c[0, 0, 2], 0.75) and np.isclose(ms.c[0, 0, 6], 0.5)


def test_batch_workload_shapes():
    rves = synth.workload_batch(n_rve=3, sizes=(32,))
    for ms, lc in rves:
        assert ms.n[0] == 32
        assert 1 <= lc.n_increments <= 5
        assert np.linalg.norm(lc.Fbar - np.eye(3)) <= 0.1 + 1e-12
