"""Composite boxels from a fine binary image (paper Sec. 5).  Test infrastructure:
only tests/, the package's smoke check and the bench's CPU baseline use it.

A fine periodic image chi (1 = inclusion, 0 = matrix) of N_m = n_m s_m voxels
per axis, each fine voxel of size h_m = l_m / N_m, is cut into n1 x n2 x n3
boxels of s1 x s2 x s3 fine voxels.  Per boxel:
  * c+ = mean of chi; phase 1 if c+ = 1, 0 if c+ = 0, 2 (composite) otherwise;
  * the barycentre normal (eq. normal:kabel)
        N~ = (c- - c+) / |c- - c+|,
    c+- the barycentres of the fine voxels of each phase in the boxel;
  * the interface weights [N.1]: w = |S * chi| with the periodic stencil
        (S * chi)_p = sum_m r_m (chi_{p - e_m} - 2 chi_p + chi_{p + e_m}),
        r_m = h_i h_j / h_m  ({i, j, m} = {1, 2, 3}),
    i.e. the 3-point second differences of each axis (Sec. 5.2) weighted by the
    fine voxel's face area over its edge length;
  * [N.2]: M = sum_p w_p x_p (x) x_p over the fine voxels of the boxel, N = the
    eigenvector of the smallest eigenvalue of M, and N <- -N unless N~ . N > 0
    (eq. normal:flip), so that N points out of the inclusion.

Reading: x_p is taken relative to the weighted barycentre of the interface,
c_S = sum w x / sum w (the barycentre of the interface drawn with the method's
figure).  The footnote on M speaks of the barycentre of the boxel; measured from
the boxel centre, M of an interface patch far from the centre is dominated by the
offset, its smallest eigenvector turns in-plane, and low volume fractions (the
case the method is meant to fix) get wrong normals (tests/test_oracle_normals.py
shows it).  For pure boxels N = 0.  Where the two phase barycentres coincide,
N~ is taken as 0 (so eq. normal:flip returns -N) and the barycentre method
returns e1.
"""
import numpy as np

METHOD_LAPLACE = 0      # Sec. 5.2 ([N.1] + [N.2] + eq. normal:flip)
METHOD_BARYCENTRE = 1   # eq. normal:kabel


def stencil_ratios(h):
    """r_m = h_i h_j / h_m for the fine voxel size h = (h1, h2, h3)."""
    h1, h2, h3 = h
    return np.array([h2 * h3 / h1, h1 * h3 / h2, h1 * h2 / h3])


def laplace_weights(chi, h):
    """w = |S * chi| on the whole periodic fine image chi [N3, N2, N1] (direct stencil)."""
    f = chi.astype(np.float64)
    r = stencil_ratios(h)
    lap = np.zeros_like(f)
    for m, axis in ((0, 2), (1, 1), (2, 0)):      # x is the last array axis
        lap += r[m] * (np.roll(f, 1, axis=axis) - 2.0 * f + np.roll(f, -1, axis=axis))
    return np.abs(lap)


def laplace_weights_fft(chi, h):
    """The same convolution carried out in the Fourier domain, as the paper does."""
    f = chi.astype(np.float64)
    r = stencil_ratios(h)
    N3, N2, N1 = f.shape
    sym = np.zeros(f.shape)
    for m, (axis, n) in enumerate(((2, N1), (1, N2), (0, N3))):
        k = np.arange(n)
        s = 2.0 * np.cos(2.0 * np.pi * k / n) - 2.0
        shape = [1, 1, 1]
        shape[axis] = n
        sym = sym + r[m] * s.reshape(shape)
    return np.abs(np.fft.ifftn(np.fft.fftn(f) * sym).real)


def _boxel_blocks(a, s):
    """[N3, N2, N1] -> [n3, n2, n1, s3, s2, s1]."""
    N3, N2, N1 = a.shape
    s1, s2, s3 = s
    return a.reshape(N3 // s3, s3, N2 // s2, s2, N1 // s1, s1).transpose(0, 2, 4, 1, 3, 5)


def _local_coords(s, h):
    """Fine voxel centres relative to the boxel centre, [s3, s2, s1, 3] (x, y, z)."""
    s1, s2, s3 = s
    x = (np.arange(s1) + 0.5 - 0.5 * s1) * h[0]
    y = (np.arange(s2) + 0.5 - 0.5 * s2) * h[1]
    z = (np.arange(s3) + 0.5 - 0.5 * s3) * h[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def boxel_normal(chi_b, w_b, x, method=METHOD_LAPLACE, about="interface"):
    """Normal of one composite boxel from its fine values chi_b, weights w_b [s3, s2, s1]
    and local coordinates x [s3, s2, s1, 3].  about = "interface" (the reading used)
    or "centre" (the footnote's wording, kept for the test that rejects it)."""
    chi_b = chi_b.astype(np.float64)
    cp = (chi_b[..., None] * x).sum(axis=(0, 1, 2)) / chi_b.sum()
    cm = ((1.0 - chi_b)[..., None] * x).sum(axis=(0, 1, 2)) / (1.0 - chi_b).sum()
    d = cm - cp
    nd = np.linalg.norm(d)
    Nt = d / nd if nd > 0 else np.zeros(3)      # coinciding barycentres: no orientation
    if method == METHOD_BARYCENTRE:
        return Nt if nd > 0 else np.array([1.0, 0.0, 0.0])
    wsum = w_b.sum()
    xs = x
    if about == "interface":
        xs = x - (w_b[..., None] * x).sum(axis=(0, 1, 2)) / wsum
    M = np.einsum("abc,abci,abcj->ij", w_b, xs, xs)
    _, vec = np.linalg.eigh(M)
    N = vec[:, 0]
    return N if Nt @ N > 0 else -N


def detect(chi, s, l, method=METHOD_LAPLACE, about="interface"):
    """Phase [n3, n2, n1] uint8, c [n3, n2, n1] and N [3, n3, n2, n1] of the boxels of chi."""
    chi = np.asarray(chi, dtype=np.uint8)
    N3, N2, N1 = chi.shape
    s1, s2, s3 = s
    assert N1 % s1 == 0 and N2 % s2 == 0 and N3 % s3 == 0
    h = (l[0] / N1, l[1] / N2, l[2] / N3)
    w = laplace_weights(chi, h)
    cb = _boxel_blocks(chi, s)
    wb = _boxel_blocks(w, s)
    n3, n2, n1 = cb.shape[:3]
    cnt = cb.reshape(n3, n2, n1, -1).sum(axis=-1, dtype=np.int64)
    vol = s1 * s2 * s3
    c = cnt / float(vol)
    phase = np.where(cnt == 0, 0, np.where(cnt == vol, 1, 2)).astype(np.uint8)
    Nf = np.zeros((3, n3, n2, n1))
    x = _local_coords(s, h)
    for k, j, i in np.argwhere(phase == 2):
        Nf[:, k, j, i] = boxel_normal(cb[k, j, i], wb[k, j, i], x, method, about)
    return phase, c, Nf


def detect_at(chi, s, l, boxels, method=METHOD_LAPLACE):
    """Like detect, for a list of boxels (k, j, i) only: each boxel's weights come from
    its block with a one-voxel periodic halo, so large images need not be filtered
    whole.  Returns phase [m], c [m], N [m, 3]."""
    N3, N2, N1 = chi.shape
    s1, s2, s3 = s
    h = (l[0] / N1, l[1] / N2, l[2] / N3)
    x = _local_coords(s, h)
    out_p, out_c, out_n = [], [], []
    for k, j, i in boxels:
        zi = np.arange(k * s3 - 1, k * s3 + s3 + 1) % N3
        yi = np.arange(j * s2 - 1, j * s2 + s2 + 1) % N2
        xi = np.arange(i * s1 - 1, i * s1 + s1 + 1) % N1
        blk = chi[np.ix_(zi, yi, xi)]
        w = laplace_weights_block(blk, h)
        cb = blk[1:-1, 1:-1, 1:-1]
        cnt = int(cb.sum(dtype=np.int64))
        vol = s1 * s2 * s3
        out_c.append(cnt / float(vol))
        if cnt == 0 or cnt == vol:
            out_p.append(0 if cnt == 0 else 1)
            out_n.append(np.zeros(3))
            continue
        out_p.append(2)
        out_n.append(boxel_normal(cb, w, x, method))
    return np.array(out_p, dtype=np.uint8), np.array(out_c), np.array(out_n)


def laplace_weights_block(blk, h):
    """w on the interior of a block that carries a one-voxel halo."""
    f = blk.astype(np.float64)
    r = stencil_ratios(h)
    c = f[1:-1, 1:-1, 1:-1]
    lap = (r[0] * (f[1:-1, 1:-1, :-2] - 2.0 * c + f[1:-1, 1:-1, 2:])
           + r[1] * (f[1:-1, :-2, 1:-1] - 2.0 * c + f[1:-1, 2:, 1:-1])
           + r[2] * (f[:-2, 1:-1, 1:-1] - 2.0 * c + f[2:, 1:-1, 1:-1]))
    return np.abs(lap)
