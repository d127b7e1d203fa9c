"""Seeded synthetic microstructures and load cases for the ComBo solver.

This module is the only code shared between the GPU path's callers and the CPU
oracle's callers.  It holds geometry sampling only (no constitutive law, no
laminate, no spectral operator): it turns analytic inclusions into the per-voxel
ComBo inputs (phase id, inclusion volume fraction c, unit normal N).

Conventions (paper Sec. 2 and Sec. 4):
  * the RVE is [-l1/2, l1/2] x [-l2/2, l2/2] x [-l3/2, l3/2];
  * voxel (i, j, k) has its centre at -l/2 + (i + 1/2) h along each axis;
  * arrays are indexed [z][y][x] (x fastest), vectors/tensors lead: N is [3][n3][n2][n1];
  * phase 0 = matrix ("-"), 1 = inclusion ("+"), 2 = composite boxel;
  * c = c_plus, the inclusion fraction of the boxel;
  * N points out of the inclusion into the matrix (paper Sec. 2, Sec. 5.1).

Composite data come from S^3 subsamples per voxel (S = 4 by default): c is the
fraction of subsample centres strictly inside an inclusion, and N = -g/|g| where
g is the sum over the boxel's subsamples of the periodic central-difference
gradient of the indicator on the subsample grid (physical units, so boxels are
handled).  If g vanishes, the barycentre rule of paper Sec. 5.1 (matrix minus
inclusion barycentre) is used; if that vanishes too, e1.  This is a stand-in
for the image-based normal detection of paper Sec. 5, not that method.

Every generator uses numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PHASE_MATRIX = 0
PHASE_INCLUSION = 1
PHASE_COMPOSITE = 2


@dataclasses.dataclass
class Microstructure:
    n: tuple          # (n1, n2, n3)
    l: tuple          # (l1, l2, l3)
    phase: np.ndarray  # uint8 [n3, n2, n1]
    c: np.ndarray      # float64 [n3, n2, n1]
    N: np.ndarray      # float64 [3, n3, n2, n1]
    info: dict

    @property
    def nvox(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_composite(self) -> int:
        return int(np.count_nonzero(self.phase == PHASE_COMPOSITE))


@dataclasses.dataclass
class LoadCase:
    """Materials (mu, lambda) per phase and the macroscopic load path."""
    mats: tuple        # ((mu_minus, lam_minus), (mu_plus, lam_plus))
    Fbar: np.ndarray   # final macroscopic deformation gradient (3x3)
    n_increments: int


# ----------------------------------------------------------------------------
# fine indicator grids
# ----------------------------------------------------------------------------

def _fine_coords(n: int, l: float, S: int) -> np.ndarray:
    """Subsample centres along one axis: -l/2 + (s + 1/2) h/S."""
    h = l / n
    return -0.5 * l + (np.arange(n * S) + 0.5) * (h / S)


def _wrap(d: np.ndarray, l: float) -> np.ndarray:
    """Minimum-image displacement in a periodic box of length l."""
    return d - l * np.round(d / l)


def _axis_window(center: float, radius: float, n: int, l: float, S: int):
    """Fine indices (wrapped) whose centres may lie within radius of center."""
    hf = l / (n * S)
    nf = n * S
    lo = math.floor((center - radius + 0.5 * l) / hf - 0.5) - 1
    hi = math.ceil((center + radius + 0.5 * l) / hf - 0.5) + 1
    if hi - lo + 1 >= nf:
        idx = np.arange(nf)
    else:
        idx = np.arange(lo, hi + 1) % nf
    x = -0.5 * l + (idx + 0.5) * hf
    return idx, _wrap(x - center, l)


def paint_spheres(chi: np.ndarray, n, l, S, centers, radii) -> None:
    """Set chi = 1 at subsample centres strictly inside any sphere (periodic)."""
    for cen, r in zip(centers, radii):
        ix, dx = _axis_window(cen[0], r, n[0], l[0], S)
        iy, dy = _axis_window(cen[1], r, n[1], l[1], S)
        iz, dz = _axis_window(cen[2], r, n[2], l[2], S)
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        inside = d2 < r * r
        sub = chi[np.ix_(iz, iy, ix)]
        chi[np.ix_(iz, iy, ix)] = sub | inside


def paint_aligned_cylinders(chi: np.ndarray, n, l, S, axis, centers2d, radii) -> None:
    """Infinite cylinders along coordinate axis `axis` (0=x, 1=y, 2=z), periodic."""
    a, b = [d for d in range(3) if d != axis]          # physical axes, a < b
    xa = _fine_coords(n[a], l[a], S)
    xb = _fine_coords(n[b], l[b], S)
    m2 = np.zeros((len(xa), len(xb)), dtype=bool)
    for cen, r in zip(centers2d, radii):
        da = _wrap(xa - cen[0], l[a])
        db = _wrap(xb - cen[1], l[b])
        m2 |= (da[:, None] ** 2 + db[None, :] ** 2) < r * r
    # chi is indexed [z, y, x]: physical axis d is array axis 2 - d, so the
    # cross-section appears in array order (b, a).
    shape = list(chi.shape)
    shape[2 - axis] = 1
    chi |= m2.T.reshape(shape)


def paint_fibres(chi: np.ndarray, n, l, S, starts, dirs, length, radius) -> None:
    """Straight flat-ended fibres (periodically wrapped), swept in short pieces."""
    piece = 2.0 * radius
    for p0, d in zip(starts, dirs):
        d = np.asarray(d, float) / np.linalg.norm(d)
        npieces = int(math.ceil(length / piece))
        for q in range(npieces):
            t0 = q * piece
            t1 = min(length, t0 + piece)
            mid = np.asarray(p0) + 0.5 * (t0 + t1) * d
            half = 0.5 * (t1 - t0)
            ext = half * np.abs(d) + radius
            ix, dx = _axis_window(mid[0], ext[0], n[0], l[0], S)
            iy, dy = _axis_window(mid[1], ext[1], n[1], l[1], S)
            iz, dz = _axis_window(mid[2], ext[2], n[2], l[2], S)
            # coordinates relative to the piece midpoint
            t = (dz[:, None, None] * d[2] + dy[None, :, None] * d[1] + dx[None, None, :] * d[0])
            r2 = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2) - t * t
            inside = (r2 < radius * radius) & (t >= -half) & (t < half)
            blk = np.ix_(iz, iy, ix)
            chi[blk] = chi[blk] | inside


# ----------------------------------------------------------------------------
# coarsening: fine indicator -> (phase, c, N)
# ----------------------------------------------------------------------------

def coarsen(chi: np.ndarray, n, l, S: int, info=None) -> Microstructure:
    n1, n2, n3 = n
    l1, l2, l3 = l
    assert chi.shape == (n3 * S, n2 * S, n1 * S)
    cnt = chi.reshape(n3, S, n2, S, n1, S).sum(axis=(1, 3, 5), dtype=np.int64)
    c = cnt.astype(np.float64) / float(S ** 3)
    phase = np.where(cnt == 0, PHASE_MATRIX,
                     np.where(cnt == S ** 3, PHASE_INCLUSION, PHASE_COMPOSITE)).astype(np.uint8)

    # Block sums of the periodic central difference (chi[s+1] - chi[s-1]) / (2 hf)
    # telescope to the two first and two last subsample planes of each block.
    def grad_sum(axis_arr: int, hf: float) -> np.ndarray:
        first = np.take(chi, np.arange(0, chi.shape[axis_arr], S), axis=axis_arr).astype(np.int16)
        last = np.take(chi, np.arange(S - 1, chi.shape[axis_arr], S), axis=axis_arr).astype(np.int16)
        nxt = np.roll(first, -1, axis=axis_arr)   # plane S*(i+1)
        prv = np.roll(last, 1, axis=axis_arr)     # plane S*i - 1
        tel = nxt + last - first - prv            # one plane per block along axis
        shp = [n3, S, n2, S, n1, S]
        shp[2 * axis_arr + 1] = 1
        return tel.reshape(shp).sum(axis=(1, 3, 5), dtype=np.int64) / (2.0 * hf)

    gx = grad_sum(2, l1 / (n1 * S))
    gy = grad_sum(1, l2 / (n2 * S))
    gz = grad_sum(0, l3 / (n3 * S))
    g = np.stack([gx, gy, gz])
    gn = np.sqrt((g * g).sum(axis=0))
    N = np.zeros((3, n3, n2, n1))
    comp = phase == PHASE_COMPOSITE
    ok = comp & (gn >= 1e-12)
    N[:, ok] = -g[:, ok] / gn[ok]
    bad = np.argwhere(comp & (gn < 1e-12))
    n_fallback = 0
    for (k, j, i) in bad:
        n_fallback += 1
        blk = chi[k * S:(k + 1) * S, j * S:(j + 1) * S, i * S:(i + 1) * S].astype(bool)
        zz, yy, xx = np.meshgrid(np.arange(S), np.arange(S), np.arange(S), indexing="ij")
        pos = np.stack([(xx + 0.5) * l1 / (n1 * S), (yy + 0.5) * l2 / (n2 * S), (zz + 0.5) * l3 / (n3 * S)])
        cp = pos[:, blk].mean(axis=1)
        cm = pos[:, ~blk].mean(axis=1)
        d = cm - cp
        nd = np.linalg.norm(d)
        N[:, k, j, i] = d / nd if nd > 1e-14 else np.array([1.0, 0.0, 0.0])
    c = np.where(phase == PHASE_COMPOSITE, c, np.where(phase == PHASE_INCLUSION, 1.0, 0.0))
    inf = dict(info or {})
    inf.update(S=S, c_total=float(c.mean()), n_composite=int(comp.sum()), n_normal_fallback=n_fallback)
    return Microstructure(n=tuple(n), l=tuple(l), phase=phase, c=c, N=N, info=inf)


# ----------------------------------------------------------------------------
# inclusion placement
# ----------------------------------------------------------------------------

def _min_image_dist(a: np.ndarray, b: np.ndarray, l) -> np.ndarray:
    d = a[None, :] - b
    for ax in range(len(l)):
        d[:, ax] = _wrap(d[:, ax], l[ax])
    return np.sqrt((d * d).sum(axis=1))


def rsa_spheres(rng, radii, l, gap, max_tries=200000):
    """Random sequential addition, largest first, periodic minimum-image gap."""
    order = np.argsort(-np.asarray(radii), kind="stable")
    radii = np.asarray(radii, float)[order]
    centers = np.zeros((0, 3))
    rs = np.zeros(0)
    for r in radii:
        for _ in range(max_tries):
            p = (rng.random(3) - 0.5) * np.asarray(l, float)
            if len(rs) == 0 or np.all(_min_image_dist(p, centers, l) >= rs + r + gap):
                centers = np.vstack([centers, p])
                rs = np.append(rs, r)
                break
        else:
            raise RuntimeError("RSA failed to place a sphere")
    return centers, rs


def rsa_disks(rng, radii, l2d, gap, max_tries=200000):
    radii = np.sort(np.asarray(radii, float))[::-1]
    centers = np.zeros((0, 2))
    rs = np.zeros(0)
    for r in radii:
        for _ in range(max_tries):
            p = (rng.random(2) - 0.5) * np.asarray(l2d, float)
            if len(rs) == 0 or np.all(_min_image_dist(p, centers, l2d) >= rs + r + gap):
                centers = np.vstack([centers, p])
                rs = np.append(rs, r)
                break
        else:
            raise RuntimeError("RSA failed to place a disk")
    return centers, rs


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def single_sphere(n=(16, 16, 16), l=(1.0, 1.0, 1.0), radius=0.3, center=(0.0, 0.0, 0.0), S=4):
    """One sphere (default: centred, r = 0.3 L) -- the 16^3 single-inclusion case."""
    chi = np.zeros((n[2] * S, n[1] * S, n[0] * S), dtype=bool)
    paint_spheres(chi, n, l, S, [np.asarray(center, float)], [radius])
    return coarsen(chi, n, l, S, info=dict(kind="sphere", radius=radius))


def random_spheres(n, n_spheres, c_target, seed, l=(1.0, 1.0, 1.0), radius_range=None, S=4, return_image=False):
    """Non-overlapping random spheres (RSA with a gap of one voxel).

    Equal radii when radius_range is None, else radii ~ U[radius_range]*L rescaled
    by one common factor so that the analytic sphere volume fraction is c_target.
    With return_image, the fine indicator image [n3 S, n2 S, n1 S] (bool) is
    returned instead of the coarsened microstructure.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    L = float(min(l))
    vol = float(np.prod(l))
    if radius_range is None:
        r = (c_target * vol * 3.0 / (4.0 * math.pi * n_spheres)) ** (1.0 / 3.0)
        radii = np.full(n_spheres, r)
        scale = 1.0
    else:
        radii = rng.uniform(radius_range[0], radius_range[1], n_spheres) * L
        v = (4.0 / 3.0) * math.pi * np.sum(radii ** 3)
        scale = (c_target * vol / v) ** (1.0 / 3.0)
        radii = radii * scale
    gap = max(li / ni for li, ni in zip(l, n))
    centers, rs = rsa_spheres(rng, radii, l, gap)
    chi = np.zeros((n[2] * S, n[1] * S, n[0] * S), dtype=bool)
    paint_spheres(chi, n, l, S, centers, rs)
    if return_image:
        return chi
    return coarsen(chi, n, l, S, info=dict(kind="spheres", n_spheres=n_spheres, radius_scale=scale,
                                           c_analytic=float((4.0 / 3.0) * math.pi * np.sum(rs ** 3) / vol),
                                           seed=seed))


def random_fibres(n, n_fibres, radius, c_target, seed, l=(1.0, 1.0, 1.0), S=4):
    """Straight fibres of one radius, isotropic directions, periodic wrap, overlaps allowed.

    The common length is chosen so that the analytic (overlap-free) volume
    fraction equals c_target; the achieved fraction is reported in info.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    vol = float(np.prod(l))
    length = c_target * vol / (n_fibres * math.pi * radius ** 2)
    starts = (rng.random((n_fibres, 3)) - 0.5) * np.asarray(l, float)
    dirs = rng.normal(size=(n_fibres, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    chi = np.zeros((n[2] * S, n[1] * S, n[0] * S), dtype=bool)
    paint_fibres(chi, n, l, S, starts, dirs, length, radius)
    return coarsen(chi, n, l, S, info=dict(kind="fibres", n_fibres=n_fibres, radius=radius,
                                           length=length, seed=seed))


def layered(n, l, normal_axis, interfaces, S=4):
    """Planar layers orthogonal to a coordinate axis; interfaces = sorted positions
    (in [-l/2, l/2)) alternating matrix -> inclusion -> matrix ... along the axis."""
    chi = np.zeros((n[2] * S, n[1] * S, n[0] * S), dtype=bool)
    x = _fine_coords(n[normal_axis], l[normal_axis], S)
    inside = np.zeros_like(x, dtype=bool)
    iv = list(interfaces)
    for a, b in zip(iv[0::2], iv[1::2]):
        inside |= (x > a) & (x < b)
    arr_axis = {0: 2, 1: 1, 2: 0}[normal_axis]
    shape = [1, 1, 1]
    shape[arr_axis] = len(x)
    chi |= np.broadcast_to(inside.reshape(shape), chi.shape)
    return coarsen(chi, n, l, S, info=dict(kind="layers", axis=normal_axis, interfaces=list(interfaces)))


def uniform_composite(n, c, N, l=(1.0, 1.0, 1.0)):
    """Every voxel the same composite boxel (c, N)."""
    n1, n2, n3 = n
    N = np.asarray(N, float)
    N = N / np.linalg.norm(N)
    phase = np.full((n3, n2, n1), PHASE_COMPOSITE, np.uint8)
    cc = np.full((n3, n2, n1), float(c))
    NN = np.broadcast_to(N.reshape(3, 1, 1, 1), (3, n3, n2, n1)).copy()
    return Microstructure(n=tuple(n), l=tuple(l), phase=phase, c=cc, N=NN, info=dict(kind="uniform_composite"))


def homogeneous(n, phase_id=0, l=(1.0, 1.0, 1.0)):
    n1, n2, n3 = n
    phase = np.full((n3, n2, n1), phase_id, np.uint8)
    c = np.full((n3, n2, n1), 1.0 if phase_id == 1 else 0.0)
    return Microstructure(n=tuple(n), l=tuple(l), phase=phase, c=c, N=np.zeros((3, n3, n2, n1)),
                          info=dict(kind="homogeneous"))


def random_composite_field(n, seed, frac_composite=0.5, c_range=(0.02, 0.98), l=(1.0, 1.0, 1.0)):
    """Unstructured random phases, fractions and normals (for per-voxel law tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n1, n2, n3 = n
    u = rng.random((n3, n2, n1))
    phase = np.where(u < frac_composite, PHASE_COMPOSITE,
                     np.where(u < frac_composite + 0.5 * (1 - frac_composite), PHASE_MATRIX, PHASE_INCLUSION)
                     ).astype(np.uint8)
    c = rng.uniform(c_range[0], c_range[1], (n3, n2, n1))
    c = np.where(phase == PHASE_COMPOSITE, c, np.where(phase == PHASE_INCLUSION, 1.0, 0.0))
    N = rng.normal(size=(3, n3, n2, n1))
    N /= np.linalg.norm(N, axis=0, keepdims=True)
    N = np.where(phase[None] == PHASE_COMPOSITE, N, 0.0)
    return Microstructure(n=tuple(n), l=tuple(l), phase=phase, c=c, N=N, info=dict(kind="random", seed=seed))


def random_F_field(n, seed, amplitude=0.1):
    """Random deformation gradients I + H with |H_ij| <= amplitude, [9][n3][n2][n1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n1, n2, n3 = n
    H = rng.uniform(-amplitude, amplitude, (3, 3, n3, n2, n1))
    F = H + np.eye(3).reshape(3, 3, 1, 1, 1)
    return F.reshape(9, n3, n2, n1)


def random_Fbar_ball(rng, radius=0.1):
    """F = I + H with H uniform in the Frobenius ball of the given radius."""
    g = rng.normal(size=9)
    g /= np.linalg.norm(g)
    r = radius * rng.random() ** (1.0 / 9.0)
    return np.eye(3) + (r * g).reshape(3, 3)


def stretch(e: float) -> np.ndarray:
    F = np.eye(3)
    F[0, 0] += e
    return F


def shear12(g: float) -> np.ndarray:
    F = np.eye(3)
    F[0, 1] += g
    return F


# Materials as (mu, lambda): index 0 = matrix ("-"), 1 = inclusion ("+").
def contrast_mats(contrast: float, base=(1.0, 2.0)):
    mu, lam = base
    return ((mu, lam), (contrast * mu, contrast * lam))


def paper_mats():
    """E+ = 10, nu+ = 0.3 and E- = 1, nu- = 0 (paper Sec. 6.1) as (mu, lambda)."""
    def lame(E, nu):
        return (E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)))
    return (lame(1.0, 0.0), lame(10.0, 0.3))


# ---- the five workloads ------------------------------------------------------

def workload_single_sphere_16():
    """16^3, centred sphere r = 0.3 L, inclusion 10x stiffer, F = I + 0.05 e1(x)e1, one step."""
    ms = single_sphere((16, 16, 16), radius=0.3)
    return ms, LoadCase(mats=contrast_mats(10.0), Fbar=stretch(0.05), n_increments=1)


def workload_spheres_64():
    """64^3, 20 equal spheres (c = 0.25), contrast 100, 20 % stretch in 10 increments."""
    ms = random_spheres((64, 64, 64), 20, 0.25, seed=2)
    return ms, LoadCase(mats=contrast_mats(100.0), Fbar=stretch(0.2), n_increments=10)


def workload_spheres_256(n=256):
    """256^3, 200 spheres r ~ U[0.03, 0.06] L rescaled to c = 0.30, contrast 100, 20 % stretch / 10 incr."""
    ms = random_spheres((n, n, n), 200, 0.30, seed=3, radius_range=(0.03, 0.06))
    return ms, LoadCase(mats=contrast_mats(100.0), Fbar=stretch(0.2), n_increments=10)


def workload_spheres_256_image(n=256, S=4):
    """The fine (S n)^3 indicator image the 256^3 sphere workload is coarsened from."""
    return random_spheres((n, n, n), 200, 0.30, seed=3, radius_range=(0.03, 0.06), S=S, return_image=True)


def sphere_image(N, radius, center=(0.0, 0.0, 0.0), l=(1.0, 1.0, 1.0)):
    """Fine image [N3, N2, N1] (uint8) of one periodic sphere, voxel centres strictly inside."""
    chi = np.zeros((N[2], N[1], N[0]), dtype=bool)
    paint_spheres(chi, N, l, 1, [np.asarray(center, float)], [radius])
    return chi.astype(np.uint8)


def plane_image(N, l, normal, offset, point=(0.0, 0.0, 0.0)):
    """Fine image [N3, N2, N1] (uint8): 1 where (x - point).normal < offset, x the voxel
    centres of the box [-l/2, l/2)^3 (not periodic: a half space cut to the box)."""
    xs = [(np.arange(N[d]) + 0.5) * l[d] / N[d] - 0.5 * l[d] - point[d] for d in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return ((X * normal[0] + Y * normal[1] + Z * normal[2]) < offset).astype(np.uint8)


def workload_fibres_256(n=256, S=4):
    """256^3, 60 fibres r = 0.025 L, c = 0.35, near-incompressible matrix, shear 0.3 in 30 incr."""
    ms = random_fibres((n, n, n), 60, 0.025, 0.35, seed=5, S=S)
    return ms, LoadCase(mats=((1.0, 1000.0), (1000.0, 1.0e6)), Fbar=shear12(0.3), n_increments=30)


def workload_batch(n_rve=64, seed=4, sizes=(32, 48, 64, 96), S=4):
    """Batch of RVEs with uneven grids, spheres or aligned cylinders, log-uniform contrast."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n_rve):
        n = int(sizes[rng.integers(len(sizes))])
        kind = "spheres" if rng.random() < 0.5 else "cylinders"
        count = int(rng.integers(5, 31))
        c_target = float(rng.uniform(0.1, 0.3))
        contrast = float(10.0 ** rng.uniform(1.0, 3.0))
        Fbar = random_Fbar_ball(rng, 0.1)
        K = int(rng.integers(1, 6))
        sub_seed = int(rng.integers(0, 2 ** 31 - 1))
        sub = np.random.Generator(np.random.PCG64(sub_seed))
        l = (1.0, 1.0, 1.0)
        gap = 1.0 / n
        chi = np.zeros((n * S, n * S, n * S), dtype=bool)
        # keep random sequential addition well below jamming: the spheres (disks)
        # grown by half the gap may cover at most 30 % (40 %) of the box
        if kind == "spheres":
            r_cap = (0.30 * 3.0 / (4.0 * math.pi * count)) ** (1.0 / 3.0) - 0.5 * gap
            c_target = min(c_target, count * (4.0 / 3.0) * math.pi * r_cap ** 3)
            r = (c_target * 3.0 / (4.0 * math.pi * count)) ** (1.0 / 3.0)
            centers, rs = rsa_spheres(sub, np.full(count, r), l, gap)
            paint_spheres(chi, (n, n, n), l, S, centers, rs)
            extra = dict(radius=r)
        else:
            axis = int(sub.integers(3))
            r_cap = math.sqrt(0.40 / (math.pi * count)) - 0.5 * gap
            c_target = min(c_target, count * math.pi * r_cap ** 2)
            r = math.sqrt(c_target / (math.pi * count))
            centers, rs = rsa_disks(sub, np.full(count, r), (1.0, 1.0), gap)
            paint_aligned_cylinders(chi, (n, n, n), l, S, axis, centers, rs)
            extra = dict(radius=r, axis=axis)
        ms = coarsen(chi, (n, n, n), l, S, info=dict(kind=kind, count=count, c_target=c_target, **extra))
        out.append((ms, LoadCase(mats=contrast_mats(contrast), Fbar=Fbar, n_increments=K)))
    return out
