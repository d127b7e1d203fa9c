"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/*.h, and its host-only functions behave."""
import glob
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2204_13624_amd import combo, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(combo_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    lib = os.path.join(ROOT, "paper_2204_13624_amd", "libcombo.so")
    assert os.path.exists(lib), "build libcombo.so first"
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    names = declared_functions()
    assert len(names) >= 15
    missing = sorted(n for n in names if n not in exported)
    assert not missing, missing
    combo.load_library()


def test_host_only_calls():
    assert combo.combo_abi_version() == 7
    assert combo.combo_strerror(combo.COMBO_E_SIZE) == "unsupported grid size"
    o = combo.combo_default_options()
    assert o.tol_newton == 1e-8 and o.max_laminate == 50 and o.warm_start_laminate == 1
    assert o.law == combo.COMBO_LAW_NEO_HOOKE and o.line_search == 1
    for n in (1, 2, 3, 6, 9, 16, 48, 96, 256, 384, 432, 486, 512):
        assert combo.combo_check_size(n) == combo.COMBO_OK
    for n in (0, 5, 7, 10, 11, 576, 648, 768, 1024):
        assert combo.combo_check_size(n) == combo.COMBO_E_SIZE


def test_microstructure_validation():
    ms = synth.single_sphere((8, 8, 8), radius=0.3)
    assert combo.combo_validate_microstructure(ms.phase, ms.c, ms.N)[0] == combo.COMBO_OK
    bad = ms.phase.copy()
    bad[0, 0, 0] = 3
    st, msg = combo.combo_validate_microstructure(bad, ms.c, ms.N)
    assert st == combo.COMBO_E_INVAL and "phase id" in msg
    c = ms.c.copy()
    comp = np.argwhere(ms.phase == 2)[0]
    c[tuple(comp)] = 1.0
    st, msg = combo.combo_validate_microstructure(ms.phase, c, ms.N)
    assert st == combo.COMBO_E_INVAL and "(0, 1)" in msg
    N = ms.N.copy()
    N[:, comp[0], comp[1], comp[2]] *= 2.0
    st, msg = combo.combo_validate_microstructure(ms.phase, ms.c, N)
    assert st == combo.COMBO_E_INVAL and "unit" in msg


def test_create_without_gpu_fails_cleanly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(combo.ComboError) as e:
        combo.combo_create(0)
    assert e.value.status in (combo.COMBO_E_HIP, combo.COMBO_E_INVAL)
