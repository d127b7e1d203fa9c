"""Per-voxel bound on the difference of two laminate solves that each stop by the
rule of Alg. 1 as read here (test helper; uses the oracle's tangent)."""
import numpy as np

from oracle import laminate as olam
from oracle import material as omat


def laminate_stop_bound(r, c, N, mats):
    """Per-voxel bound on |P_box| differences between two laminate solves that each
    stopped by the rule of Alg. 1 as read here: |f| <= tol_f, or a Newton correction
    |Delta^-1 f| <= 1e-13 max(|a|, 1e-3).  Each side's jump vector is then within
    da = |Delta^-1| (tol_f + 64 eps (|P+| + |P-|)) + 1e-13 max(|a|, 1e-3) of the root
    (the eps term is the round-off of f itself, which is what triggers the second
    stop), and dP_box/da = (A+ - A-) D, so |dP_box| <= 2 |(A+ - A-) D| da."""
    D = olam.jump_matrix(N)
    Ap = omat.tangent(r["Fp"], *mats[1])
    Am = omat.tangent(r["Fm"], *mats[0])
    Delta = np.swapaxes(D, 1, 2) @ (Ap / c[:, None, None] + Am / (1.0 - c)[:, None, None]) @ D
    dinv = np.linalg.norm(np.linalg.inv(Delta), 2, axis=(1, 2))
    dad = np.linalg.norm((Ap - Am) @ D, 2, axis=(1, 2))
    tp = np.linalg.norm(np.einsum("miJ,mJ->mi", r["Pp"], N), axis=1)
    tm = np.linalg.norm(np.einsum("miJ,mJ->mi", r["Pm"], N), axis=1)
    floor = max(1e-3 * max(mats[0][0], mats[1][0]), 1e-2 * max(mats[0][1], mats[1][1]))
    tol_f = olam.REL_TOL * np.maximum(np.maximum(tp, tm), floor)
    pn = np.linalg.norm(r["Pp"].reshape(-1, 9), axis=1) + np.linalg.norm(r["Pm"].reshape(-1, 9), axis=1)
    da = dinv * (tol_f + 64 * np.finfo(float).eps * pn) + olam.STEP_TOL * np.maximum(np.linalg.norm(r["a"], axis=1), 1e-3)
    return 2.0 * dad * da
