"""combo_image_to_boxels_static (no allocation, static device scratch) against
combo_image_to_boxels on the same context and inputs, through the C-ABI.

Both run the same boxel kernels (paper Sec. 5: volume fractions, phases and the
Laplacian or barycentre normals) on the same data, so their outputs must agree
bit for bit.  Two calls in a row, the second on a smaller grid, check that the
scratch left behind by one call does not leak into the next; the size limits
are refused on the host."""
import ctypes

import numpy as np
import pytest

from paper_2204_13624_amd import combo, synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _outputs(n, dev):
    torch = _torch()
    n1, n2, n3 = n
    return (torch.full((n3, n2, n1), 7, dtype=torch.uint8, device=dev),
            torch.full((n3, n2, n1), -1.0, dtype=torch.float64, device=dev),
            torch.full((3, n3, n2, n1), -1.0, dtype=torch.float64, device=dev))


def _compare(ctx, img, s, method):
    torch = _torch()
    dev = torch.device("cuda:0")
    (n1, n2, n3), _ = combo.combo_get_grid(ctx)
    dimg = torch.from_numpy(img).to(dev)
    got = combo.combo_image_to_boxels_static(ctx, dimg, s, _outputs((n1, n2, n3), dev), method=method)
    ref = combo.combo_image_to_boxels(ctx, dimg, s, method=method, out=_outputs((n1, n2, n3), dev))
    torch.cuda.synchronize()
    for g, r in zip(got, ref):
        assert torch.equal(g, r)
    ph = got[0].cpu().numpy()
    assert (ph == 2).sum() > 0 and (ph == 0).sum() > 0
    return int((ph == 2).sum())


@pytest.mark.parametrize("method", [combo.COMBO_NORMALS_LAPLACE, combo.COMBO_NORMALS_BARYCENTRE])
def test_static_scratch_matches_allocating_path_two_calls(method):
    ctx = combo.combo_create(0)
    try:
        # call 1: 32^3 boxels of 4^3 fine voxels (four-boxel pass with packed words)
        combo.combo_set_grid(ctx, 32, 32, 32, 1.0, 1.0, 1.0)
        img = synth.sphere_image((128, 128, 128), 0.31, center=(0.05, -0.02, 0.01))
        n1c = _compare(ctx, img, (4, 4, 4), method)
        # call 2, smaller: 12 x 16 x 8 boxels of 3 x 2 x 2 fine voxels (one boxel per thread)
        combo.combo_set_grid(ctx, 12, 16, 8, 1.0, 1.2, 0.7)
        img2 = synth.sphere_image((36, 32, 16), 0.25, center=(0.1, 0.0, 0.0), l=(1.0, 1.2, 0.7))
        n2c = _compare(ctx, img2, (3, 2, 2), method)
        assert n2c < n1c
    finally:
        combo.combo_destroy(ctx)


def test_static_scratch_size_limits():
    torch = _torch()
    dev = torch.device("cuda:0")
    lib = combo.load_library()
    ctx = combo.combo_create(0)
    try:
        # 384^3 boxels: the composite list alone (4 B per boxel) exceeds 64 MiB -> refused before GPU work
        combo.combo_set_grid(ctx, 384, 384, 384, 1.0, 1.0, 1.0)
        chi = torch.zeros((384, 384, 384), dtype=torch.uint8, device=dev)
        out = _outputs((384, 384, 384), dev)
        st = lib.combo_image_to_boxels_static(ctx, ctypes.c_void_p(chi.data_ptr()), 1, 1, 1, 0,
                                              ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()),
                                              ctypes.c_void_p(out[2].data_ptr()))
        assert st == combo.COMBO_E_SIZE
        assert "static scratch" in combo.combo_last_error(ctx)
        del chi, out
        # 192^3 boxels of 2^3 fine voxels of a random image: almost every boxel is a composite and
        # their moments (104 B each) do not fit -> refused after pass 1, phase and c written
        combo.combo_set_grid(ctx, 192, 192, 192, 1.0, 1.0, 1.0)
        rng = np.random.Generator(np.random.PCG64(11))
        chi = torch.from_numpy(rng.integers(0, 2, size=(384, 384, 384), dtype=np.uint8)).to(dev)
        out = _outputs((192, 192, 192), dev)
        torch.cuda.synchronize()
        st = lib.combo_image_to_boxels_static(ctx, ctypes.c_void_p(chi.data_ptr()), 2, 2, 2, 0,
                                              ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()),
                                              ctypes.c_void_p(out[2].data_ptr()))
        assert st == combo.COMBO_E_SIZE
        assert "composite" in combo.combo_last_error(ctx)
        ph = out[0].cpu().numpy()
        ref_c = chi.view(192, 2, 192, 2, 192, 2).to(torch.float64).mean(dim=(1, 3, 5)).cpu().numpy()
        assert np.array_equal(out[1].cpu().numpy(), ref_c)
        assert set(np.unique(ph)) <= {0, 1, 2}
        # the context still works with the static path on a grid that fits
        combo.combo_set_grid(ctx, 16, 16, 16, 1.0, 1.0, 1.0)
        _compare(ctx, synth.sphere_image((64, 64, 64), 0.3), (4, 4, 4), combo.COMBO_NORMALS_LAPLACE)
    finally:
        combo.combo_destroy(ctx)
