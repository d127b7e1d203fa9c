"""Benchmark: ComBo Lippmann-Schwinger Newton-CG solve on one MI355X.

Workload (default): 256^3 RVE, 200 random spheres (radii U[0.03, 0.06] L
rescaled to c = 0.30), composite boxels from 4^3 subsamples, Neo-Hooke matrix
(mu, lambda) = (1, 2) and inclusions 100x stiffer, uniaxial stretch to 20 % in
10 increments, Newton tolerance eta <= 1e-6.  One step = one full solve.

value = voxel-CG-iterations per second of the mixed-precision solve (FP32
linear solves, FP64 law and residual) over the K timed solves (default 3, after
one warm-up); time-to-solution is their median, and the FP64 solve's is reported
beside it.  Per-kernel durations come from HIP event pairs the library records
on its stream: around the x pass (the roofline kernel) in the timed solves, and
around every kernel class in the last warm-up solve.

Further sections of the same JSON line (each can be switched off): the same RVE
twice in one batch (the batched form against the single mixed and FP64 solves), the
rotated scheme and the staggered grid on the same RVE, the small-strain law, composite
boxels from the 1024^3 image, the 64-RVE batch, the fibre workload's load walk
with its effective tangent and stability, and the CPU oracle's CG throughput.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64] [--no-willot]
       [--no-staggered] [--no-small-strain] [--no-image] [--no-batch] [--no-batched-256] [--no-fibres]
"""
import argparse
import json
import os
import platform
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(name, n, nspec, nc, s):
    """Algorithmic HBM bytes of one launch of a CG kernel class (s = bytes per real)."""
    c2 = 2 * s * nspec            # one complex component of the half spectrum / one CG vector component
    table = {
        "xpass_cg": 18 * c2 + 4 * n + 10 * s * (n - nc) + 45 * s * nc,
        "ypass_inv": 15 * c2,
        "ypass_fwd": 15 * c2,
        "zpass_inv": 15 * c2,
        "zpass_fwd": 12 * c2,
        "cg_update": 18 * c2,
    }
    return table.get(name)


def measured_traffic(kernel):
    """HBM bytes per launch of a CG kernel class from the committed PMC record
    (FETCH_SIZE / WRITE_SIZE scaled by a plain-copy calibration), or None if the
    record is missing or the kernel sources changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_spheres_256_mixed.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return rec["kernels"][kernel]["traffic_bytes"]
    except (OSError, ValueError, KeyError, AttributeError):
        return None


def tts(times, key):
    """Time-to-solution over the timed runs: the median, with the minimum, maximum and count."""
    ts = sorted(times)
    return {key: float(np.median(ts)), key + "_min": ts[0], key + "_max": ts[-1], key + "_runs": len(ts)}


def cpu_cores_used(cpu_s, wall_s):
    return max(1, int(round(cpu_s / max(wall_s, 1e-9))))


def host_cpu():
    """CPU model (from /proc/cpuinfo) and the number of cores this process may use."""
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return model, nproc


def cpu_baseline(ms, lc, sub=128, iters=8):
    """Time the FP64 oracle's CG iterations on a sub-block of the same workload."""
    from oracle import solver as osol
    from oracle import spectral as ospec
    from paper_2204_13624_amd import synth
    crop = synth.Microstructure(n=(sub, sub, sub), l=(sub / ms.n[0],) * 3,
                                phase=np.ascontiguousarray(ms.phase[:sub, :sub, :sub]),
                                c=np.ascontiguousarray(ms.c[:sub, :sub, :sub]),
                                N=np.ascontiguousarray(ms.N[:, :sub, :sub, :sub]), info={})
    prob = osol.Problem(crop.n, crop.l, crop.phase, crop.c, crop.N, lc.mats)
    mu0, kappa0 = osol.reference_medium(lc.mats)
    Fb1 = np.eye(3) + (lc.Fbar - np.eye(3)) / lc.n_increments
    F = np.broadcast_to(Fb1[:, :, None, None, None], (3, 3, sub, sub, sub)).copy()
    P, Av, ok, _, _ = osol.evaluate(F, prob)
    b = -ospec.apply_gamma0(P, prob.n, prob.l, mu0, kappa0)
    t0, c0 = time.perf_counter(), time.process_time()
    try:
        osol.cg(Av, b, prob, mu0, kappa0, 1e-30, iters)
    except (osol.SolveError, osol.NegativeCurvature):
        pass
    wall, cpu = time.perf_counter() - t0, time.process_time() - c0
    nv = sub ** 3
    model, nproc = host_cpu()
    cores = cpu_cores_used(cpu, wall)
    return {"value": nv * iters / wall, "unit": "voxel-CG-iters/s", "cores": cores,
            "kind": "oracle", "host_cpu": model, "host_nproc": nproc,
            "sample": "%d CG iterations of the FP64 numpy oracle (numpy FFT and einsum: one thread; %d core(s) "
                      "busy on average) on a %d^3 block of the same microstructure, a cropped (not periodic) "
                      "RVE, at the first load increment; %.1f s wall on %s, %d cores available"
                      % (iters, cores, sub, wall, model, nproc)}


def image_bench(combo, synth, ms, steps):
    """Composite boxels of the 256^3 workload from its 1024^3 fine image (s = 4, paper
    Sec. 5 normals), image resident in HBM; per-kernel times from HIP events."""
    import torch
    t = time.time()
    img = synth.workload_spheres_256_image()
    log("image generated in %.1f s" % (time.time() - t))
    dimg = torch.from_numpy(img.view(np.uint8)).to("cuda:0")
    del img
    n = ms.n
    ctx = combo.combo_create(0)
    combo.combo_set_grid(ctx, *n, *ms.l)
    out = combo.combo_image_to_boxels(ctx, dimg, (4, 4, 4))          # warm-up
    combo.combo_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(3, steps)
    for _ in range(reps):
        combo.combo_image_to_boxels(ctx, dimg, (4, 4, 4), out=out)
    el = (time.perf_counter() - t0) / reps
    prof = combo.combo_profile_all(ctx)
    combo.combo_destroy(ctx)
    phase = out[0].cpu().numpy()
    nb = phase.size
    ncomp = int((phase == 2).sum())
    exact = bool(np.array_equal(phase, ms.phase) and np.array_equal(out[1].cpu().numpy(), ms.c))
    img_bytes = int(dimg.numel())
    del dimg
    ms1, n1 = prof["boxel_count"]
    ms2, n2 = prof["boxel_normals"]
    avg1, avg2 = ms1 / n1, ms2 / n2
    # pass 1: the image once; phase (1 B), c (8 B) and the packed fine values (one 8-B word) of every boxel
    b1 = img_bytes + nb * (9 + 8)
    # pass 2: phase (1 B) in and N (24 B) out for every boxel; per composite the seven packed words of
    # its boxel and the six face neighbours (56 B) and the list entry (written and read once)
    b2 = nb * 25 + ncomp * (56 + 8)
    res = {"workload": "1024^3 image of spheres_256 -> 256^3 boxels (4^3 fine voxels each), Laplacian normals",
           "composites": ncomp, "phase_and_c_equal_generator": exact,
           "ms_per_call": el * 1e3,
           "kernels": {"boxel_count": {"avg_us": round(avg1 * 1e3, 2), "bytes_per_launch": b1,
                                       "GBps": round(b1 / (avg1 * 1e-3) / 1e9, 1)},
                       "boxel_normals": {"avg_us": round(avg2 * 1e3, 2), "bytes_per_launch": b2,
                                         "GBps": round(b2 / (avg2 * 1e-3) / 1e9, 1)}},
           "image_GB_per_s": round(img_bytes / el / 1e9, 1)}
    dom = max(("boxel_count", "boxel_normals"), key=lambda k: res["kernels"][k]["avg_us"])
    res["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": res["kernels"][dom]["GBps"],
                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(res["kernels"][dom]["GBps"] / HBM_PEAK_GBS, 4)}
    log("image -> boxels: %.3f ms per call (count %.1f us, normals %.1f us), composites %d, exact %s"
        % (el * 1e3, avg1 * 1e3, avg2 * 1e3, ncomp, exact))
    return res


def batch_bench(combo, synth, steps):
    """The many-RVE workload: 64 RVEs of 32^3..96^3 in one batch, against the same
    RVEs solved one after another on one context each (setup excluded)."""
    import torch
    t = time.time()
    items = synth.workload_batch()
    log("batch workload generated in %.1f s: %d RVEs, %d voxels" % (time.time() - t, len(items),
                                                                    sum(ms.nvox for ms, _ in items)))
    o = combo.combo_default_options()
    o.precision = combo.COMBO_MIXED
    o.tol_newton = 1e-6
    o.tol_cg = 1e-4
    o.max_cg = 20000
    o.autotune = 1
    o.graph_chunk = 0   # plain launches: captured chunks measured no faster (GPU-bound)
    b = combo.combo_batch_create(0)
    combo.combo_batch_set_options(b, o)
    for ms, lc in items:
        combo.combo_batch_add(b, ms.n, ms.l, lc.mats, ms.phase, ms.c, ms.N)
    Fb = np.stack([lc.Fbar for _, lc in items])
    K = [lc.n_increments for _, lc in items]
    nv = [ms.nvox for ms, _ in items]
    combo.combo_batch_solve(b, Fb, n_increments=K)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = combo.combo_batch_solve(b, Fb, n_increments=K)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    cg = [s["cg_iters_total"] for s in r["stats"]]
    vox_it = sum(n * c for n, c in zip(nv, cg))
    combo.combo_batch_destroy(b)
    # the same members one at a time
    ctxs = []
    for ms, lc in items:
        c = combo.combo_create(0)
        combo.combo_set_grid(c, *ms.n, *ms.l)
        combo.combo_set_materials(c, lc.mats)
        combo.combo_set_microstructure(c, ms.phase, ms.c, ms.N)
        oo = combo.combo_default_options()
        for k, _ in o._fields_:
            setattr(oo, k, getattr(o, k))
        oo.n_increments = lc.n_increments
        oo.graph_chunk = 0
        combo.combo_set_options(c, oo)
        combo.combo_autotune(c, combo.COMBO_MIXED)   # cached: same schedules as the batch
        ctxs.append(c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_it = 0
    for c, (ms, lc) in zip(ctxs, items):
        rr = combo.combo_solve(c, lc.Fbar)
        seq_it += ms.nvox * rr["stats"]["cg_iters_total"]
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    for c in ctxs:
        combo.combo_destroy(c)
    log("batch: %.3f s (%.3e voxel-CG-iters/s), one by one: %.3f s" % (wall, vox_it / wall, seq))
    return {"workload": "64 RVEs, grids from {32,48,64,96}^3, 5-30 spheres or aligned cylinders each, contrast "
                        "10^U[1,3], |Fbar-I|<=0.1, 1-5 increments, mixed precision, eta<=1e-6, tol_cg 1e-4",
            "n_rve": len(items), "voxels": int(sum(nv)), "value": vox_it / wall, "unit": "voxel-CG-iters/s",
            "time_s": wall, "cg_iters": int(sum(cg)), "newton_iters": int(sum(s["newton_iters"] for s in r["stats"])),
            "cg_truncations": int(sum(s["cg_truncations"] for s in r["stats"])),
            "one_by_one_time_s": seq, "one_by_one_value": seq_it / seq, "speedup_vs_one_by_one": seq / wall}


def batched_256(combo, ms, lc, o, out, members=2):
    """The 256^3 workload in the batched form: `members` copies of the RVE under the
    same load in one batch (mixed precision, the main solve's options), one warm-up and
    one timed batch solve.  The per-RVE time is compared with the single mixed and the
    FP64 solves of the same workload; Pbar of every member against the FP64 solve."""
    import torch
    b = combo.combo_batch_create(0)
    try:
        combo.combo_batch_set_options(b, o)
        for _ in range(members):
            combo.combo_batch_add(b, ms.n, ms.l, lc.mats, ms.phase, ms.c, ms.N)
        Fb = np.stack([lc.Fbar] * members)
        K = [lc.n_increments] * members
        combo.combo_batch_solve(b, Fb, n_increments=K)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = combo.combo_batch_solve(b, Fb, n_increments=K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        combo.combo_batch_destroy(b)
    cg = [st["cg_iters_total"] for st in r["stats"]]
    per = wall / members
    res = {"members": members, "wall_s": wall, "per_rve_s": per, "cg_iters": cg,
           "value": ms.nvox * sum(cg) / wall, "unit": "voxel-CG-iters/s"}
    tts_ = out.get("time_to_solution_s", {})
    if "mixed" in tts_:
        res["single_mixed_over_per_rve"] = tts_["mixed"] / per
    if "fp64" in tts_:
        res["fp64_over_per_rve"] = tts_["fp64"] / per
    if out.get("_Pbar_fp64") is not None:
        P64 = out["_Pbar_fp64"]
        res["pbar_rel_diff_vs_fp64"] = float(max(np.abs(np.asarray(r["Pbar"][i]) - P64).max()
                                                 for i in range(members)) / np.abs(P64).max())
    log("batched 256^3: %d members %.2f s (%.2f s per RVE)" % (members, wall, per))
    return res


def lowest_eigenvalue(combo, ctx, shape, mu0, kappa0, steps, seed=11):
    """Smallest Ritz value of K = Gamma0[A:.] (the tangent state of the last
    combo_eval_law) on compatible zero-mean fields, in the C0 inner product
    mu0 x:y + kappa0 tr x tr y, after 2/3 of `steps` and after `steps` Lanczos steps.
    K is self-adjoint in that product on those fields; each vector is projected with
    G so that rounding does not leak it outside them."""
    import torch
    from scipy.linalg import eigvalsh_tridiagonal
    dev = torch.device("cuda:0")

    def ip(x, y):
        return float(mu0 * torch.sum(x * y) + kappa0 * torch.sum((x[0] + x[4] + x[8]) * (y[0] + y[4] + y[8])))

    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    r = torch.randn(shape, dtype=torch.float64, device=dev, generator=g)
    v = torch.empty_like(r)
    combo.combo_apply_green(ctx, combo.COMBO_GREEN_G, combo.COMBO_FP64, r, v)
    del r
    v /= np.sqrt(ip(v, v))
    v_old = torch.zeros_like(v)
    w = torch.empty_like(v)
    wp = torch.empty_like(v)
    alpha, beta, ritz = [], [], []
    b = 0.0
    for j in range(steps):
        combo.combo_apply_operator(ctx, combo.COMBO_FP64, v, w)
        w -= b * v_old
        a = ip(w, v)
        w -= a * v
        combo.combo_apply_green(ctx, combo.COMBO_GREEN_G, combo.COMBO_FP64, w, wp)
        b = np.sqrt(ip(wp, wp))
        alpha.append(a)
        beta.append(b)
        v_old, v = v, wp / b
        if j + 1 in (2 * steps // 3, steps):
            ritz.append(float(eigvalsh_tridiagonal(np.array(alpha), np.array(beta[:-1]),
                                                   select="i", select_range=(0, 0))[0]))
    return ritz


def fibres_bench(combo, synth, seconds):
    """The fibre workload (256^3, 60 random straight fibres, near-incompressible matrix,
    fibre contrast 1000, simple shear 0.3 e1 (x) e2 in 30 increments), mixed precision
    (FP64 det F, ln J, laminates, residual).  The load path is walked with an adaptive
    step: from the converged state at fraction t one solve to t + dt (one increment, no
    internal cutbacks); a converged step doubles dt up to 1/30, a failed one halves it.
    The walk ends when dt drops below 1/(32 x 30) (the solver's own cutback limit), at
    the end of the path, or after `seconds`.  The effective tangent Abar is computed at
    the last converged load, and so is the lowest eigenvalue of the Newton operator
    there (how close the branch is to losing stability)."""
    import torch
    t = time.time()
    ms, lc = synth.workload_fibres_256()
    gen_s = time.time() - t
    dev = torch.device("cuda:0")
    ctx = combo.combo_create(0)
    combo.combo_set_grid(ctx, *ms.n, *ms.l)
    combo.combo_set_materials(ctx, lc.mats)
    combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(dev), torch.from_numpy(ms.c).to(dev),
                                   torch.from_numpy(np.ascontiguousarray(ms.N)).to(dev))
    o = combo.combo_default_options()
    o.precision = combo.COMBO_MIXED
    o.tol_newton = 1e-6
    o.tol_cg = 1e-4
    o.max_cg = 4000
    o.max_newton = 15
    o.n_increments = 1
    o.max_cutbacks = 0
    combo.combo_set_options(ctx, o)
    H = lc.Fbar - np.eye(3)
    K = lc.n_increments
    F = torch.zeros((9,) + ms.phase.shape, dtype=torch.float64, device=dev)
    F[0] = F[4] = F[8] = 1.0
    Fn = torch.empty_like(F)
    tt, dt = 0.0, 1.0 / K
    tot = dict(newton=0, cg=0, trunc=0, attempts=0, converged=0)
    walk = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stop = "end of load path"
    while tt < 1.0 - 1e-12:
        if dt < 1.0 / (32 * K):
            stop = "step below 1/32 of an increment"
            break
        if time.perf_counter() - t0 > seconds:
            stop = "time cap"
            break
        tn = min(1.0, tt + dt)
        try:
            r = combo.combo_solve(ctx, np.eye(3) + tn * H, F_init=F, F_out=Fn)
            ok = True
        except combo.ComboError as e:
            r, ok = e.result, False
        s = r["stats"]
        tot["newton"] += s["newton_iters"]
        tot["cg"] += s["cg_iters_total"]
        tot["trunc"] += s["cg_truncations"]
        tot["attempts"] += 1
        walk.append([round(0.3 * tn, 6), int(ok)])
        if ok:
            F, Fn = Fn, F
            tt = tn
            tot["converged"] += 1
            Pbar_last = r["Pbar"]
            dt = min(1.0 / K, 2 * dt)
        else:
            dt *= 0.5
    torch.cuda.synchronize()
    walk_s = time.perf_counter() - t0
    res = {"workload": "fibres_256: 256^3, 60 fibres r=0.025 L (c=%.3f after overlaps), %d composites, "
                       "matrix (mu, lambda) = (1, 1000), fibres (1000, 1e6), simple shear 0.3 e1 (x) e2 in 30 "
                       "increments" % (ms.info.get("c_total", float(ms.c.mean())), ms.n_composite),
           "precision": "mixed (FP64 det F, ln J, laminates, residual), eta<=1e-6, tol_cg 1e-4",
           "generation_s": round(gen_s, 1), "walk_s": walk_s, "stop": stop,
           "last_converged_shear": 0.3 * tt, "attempts": tot["attempts"], "converged_steps": tot["converged"],
           "newton_iters": tot["newton"], "cg_iters": tot["cg"], "cg_truncations": tot["trunc"],
           "voxel_cg_iters_per_s": ms.nvox * tot["cg"] / walk_s, "walk": walk}
    if tt > 0:
        o.want_tangent = 1
        combo.combo_set_options(ctx, o)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = combo.combo_solve(ctx, np.eye(3) + tt * H, F_init=F, F_out=Fn, want_tangent=True)
        torch.cuda.synchronize()
        res["tangent_s"] = time.perf_counter() - t1
        res["tangent_cg_iters"] = r["stats"]["cg_iters_tangent"]
        res["Pbar_last"] = [[float("%.6g" % v) for v in row] for row in Pbar_last]
        res["Abar_last"] = [[float("%.6g" % v) for v in row] for row in r["Abar"]]
        (mu_m, lam_m), (mu_p, lam_p) = lc.mats
        mu0 = float(np.sqrt(mu_m * mu_p))
        kappa0 = float(np.sqrt((lam_m + mu_m) * (lam_p + mu_p)))
        o.precision = combo.COMBO_FP64
        combo.combo_set_options(ctx, o)
        t1 = time.perf_counter()
        combo.combo_eval_law(ctx, F)
        ritz = lowest_eigenvalue(combo, ctx, tuple(F.shape), mu0, kappa0, 1000)
        res["stability"] = {
            "what": "lowest eigenvalue of the Newton operator Gamma0[A:.] on compatible fields (C0 product, "
                    "FP64, Lanczos with G re-projection) at the last converged load; unloaded it is mu_m/mu0",
            "unloaded": mu_m / mu0, "last_converged": ritz[1], "after_2_3_of_steps": ritz[0],
            "ratio": ritz[1] / (mu_m / mu0), "lanczos_steps": 1000, "seconds": time.perf_counter() - t1}
    combo.combo_destroy(ctx)
    log("fibres: %s at shear %.5f after %d attempts, %.1f s" % (stop, 0.3 * tt, tot["attempts"], walk_s))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--tol-cg", type=float, default=1e-4)
    ap.add_argument("--graph-chunk", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-batched-256", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-small-strain", action="store_true")
    ap.add_argument("--no-image", action="store_true")
    ap.add_argument("--no-willot", action="store_true")
    ap.add_argument("--no-staggered", action="store_true")
    ap.add_argument("--no-fibres", action="store_true")
    ap.add_argument("--fibre-seconds", type=float, default=120.0,
                    help="time cap of the fibre workload's load walk")
    ap.add_argument("--increments", type=int, default=0,
                    help="override the workload's load increments (shorter runs for counter collection)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_13624_amd import combo, synth

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t = time.time()
    ms, lc = synth.workload_spheres_256(args.n)
    if args.increments > 0:
        lc.n_increments = args.increments
    log("workload generated in %.1f s: n=%d, composites=%d, c=%.4f" % (time.time() - t, ms.nvox, ms.n_composite,
                                                                       ms.info["c_total"]))
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    ctx = combo.combo_create(0)
    combo.combo_set_grid(ctx, *ms.n, *ms.l)
    combo.combo_set_materials(ctx, lc.mats)
    combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(dev), torch.from_numpy(ms.c).to(dev),
                                   torch.from_numpy(np.ascontiguousarray(ms.N)).to(dev))

    def options(precision):
        o = combo.combo_default_options()
        o.precision = precision
        o.tol_newton = 1e-6
        o.tol_cg = args.tol_cg
        o.n_increments = lc.n_increments
        o.max_cg = 20000
        o.graph_chunk = args.graph_chunk
        o.autotune = 1 if precision == combo.COMBO_MIXED and not args.no_autotune else 0
        return o

    combo.combo_set_options(ctx, options(combo.COMBO_MIXED))

    def profiled_solve():
        """One untimed solve with every kernel class timed: the per-kernel table."""
        combo.combo_profile_select(ctx, None)
        combo.combo_profile_enable(ctx, True)
        combo.combo_solve(ctx, lc.Fbar)
        out = combo.combo_profile_all(ctx), combo.combo_profile_all_idle(ctx)
        combo.combo_profile_enable(ctx, False)
        return out

    prof_all = idle_all = None
    for w in range(args.warmup):
        if w == args.warmup - 1 and not args.no_profile:
            prof_all, idle_all = profiled_solve()
            r = None
        else:
            r = combo.combo_solve(ctx, lc.Fbar)
        if r is not None:
            log("warmup %d: %.2f s, newton %d, cg %d" % (w, r["stats"]["time_ms_total"] / 1e3,
                                                       r["stats"]["newton_iters"], r["stats"]["cg_iters_total"]))
    if not args.no_profile:
        # the timed solves time the dominant kernel only (one event pair per launch)
        combo.combo_profile_select(ctx, [combo.KERNEL_NAMES.index("xpass_cg")])
        combo.combo_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cg_total = 0
    results = []
    for k in range(args.steps):
        r = combo.combo_solve(ctx, lc.Fbar)
        cg_total += r["stats"]["cg_iters_total"]
        results.append(r)
        log("step %d: %.2f s, newton %d, cg %d, eta %.2e" % (k, r["stats"]["time_ms_total"] / 1e3,
                                                            r["stats"]["newton_iters"], r["stats"]["cg_iters_total"],
                                                            r["stats"]["eta_final"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof_timed = combo.combo_profile_all(ctx) if not args.no_profile else {}
    idle_timed = combo.combo_profile_all_idle(ctx) if not args.no_profile else {}
    schedule = combo.combo_get_schedule(ctx)[0]
    combo.combo_profile_enable(ctx, False)
    if not args.no_profile and prof_all is None:
        prof_all, idle_all = profiled_solve()
    # per-kernel table from the fully profiled (untimed) solve; the dominant kernel from the timed solves
    prof = dict(prof_all or {})
    idle = dict(idle_all or {})
    if prof_timed.get("xpass_cg", (0, 0))[1]:
        prof["xpass_cg"] = prof_timed["xpass_cg"]
        idle["xpass_cg"] = idle_timed["xpass_cg"]
    n = ms.nvox
    nh = ms.n[0] // 2 if ms.n[0] % 2 == 0 else (ms.n[0] + 1) // 2
    nspec = nh * ms.n[1] * ms.n[2]
    nc = ms.n_composite
    value = n * cg_total / elapsed
    Pbar_mixed = results[-1]["Pbar"]

    # roofline of the dominant CG kernel
    roof = None
    kernels = {}
    for name, (msec, cnt) in prof.items():
        if cnt == 0:
            continue
        avg = msec / cnt
        b = kernel_bytes(name, n, nspec, nc, 4)
        # launches that did work; the launches of chunk iterations after the CG had
        # finished return at once and are listed apart
        kernels[name] = {"ms_total": round(msec, 3), "launches": cnt, "avg_us": round(avg * 1e3, 2)}
        if idle.get(name, (0, 0))[1]:
            kernels[name]["idle_launches"] = idle[name][1]
            kernels[name]["idle_ms_total"] = round(idle[name][0], 3)
        if b is not None:
            kernels[name]["GBps"] = round(b / (avg * 1e-3) / 1e9, 1)
            kernels[name]["bytes_per_launch"] = b
            kernels[name]["frac"] = round(b / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    cg_kernels = {k: v for k, v in kernels.items() if "GBps" in v}
    if cg_kernels:
        dom = max(cg_kernels, key=lambda k: cg_kernels[k]["ms_total"])
        ach = cg_kernels[dom]["GBps"]
        traffic = measured_traffic(dom) if args.n == 256 else None
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": cg_kernels[dom]["bytes_per_launch"], "avg_us": cg_kernels[dom]["avg_us"]}
    b_cg = sum(kernel_bytes(k, n, nspec, nc, 4) for k in
               ("xpass_cg", "ypass_inv", "ypass_fwd", "zpass_inv", "zpass_fwd", "cg_update")) / n

    out = {
        "metric": "voxel-CG-iters/s at 256³ + time-to-solution (rel. residual 1e-6), mixed vs FP64",
        "value": value,
        "unit": "voxel-CG-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 linear solves (FFT, Green operator, tangent action, CG) + f64 law, laminate, residual",
        "data": "synthetic",
        "config": {"workload": "spheres_256: %d^3 RVE, 200 spheres c=0.30 (RSA, radii U[0.03,0.06]L rescaled), "
                               "4^3-subsample composite boxels, Neo-Hooke (1,2) / contrast 100, uniaxial stretch "
                               "to 20%% in 10 increments, eta<=1e-6, tol_cg %.0e" % (args.n, args.tol_cg),
                   "n_vox": n, "n_composite": nc, "precision": "mixed", "parallelism": "1 GPU"},
        "fft_schedule_xyz": list(schedule),
        "cg_iters_per_step": cg_total / args.steps,
        "newton_iters_per_step": results[-1]["stats"]["newton_iters"],
        "bytes_per_voxel_cg_iter": round(b_cg, 1),
        "hbm_frac_whole_cg": round(value * b_cg / (HBM_PEAK_GBS * 1e9), 4),
        "kernels": kernels,
        "kernels_timing": "HIP event pairs on the library's stream: xpass_cg in the timed solves (the only class "
                          "timed there); the other classes in one untimed solve of the same workload with every "
                          "class timed",
        "roofline": roof,
        "time_to_solution_s": tts([r["stats"]["time_ms_total"] / 1e3 for r in results], "mixed"),
    }
    if not args.no_fp64:
        combo.combo_set_options(ctx, options(combo.COMBO_FP64))
        runs64 = [combo.combo_solve(ctx, lc.Fbar) for _ in range(args.steps)]
        r64 = runs64[-1]
        out["time_to_solution_s"].update(tts([r["stats"]["time_ms_total"] / 1e3 for r in runs64], "fp64"))
        out["fp64_cg_iters"] = r64["stats"]["cg_iters_total"]
        out["fp64_voxel_cg_iters_per_s"] = n * r64["stats"]["cg_iters_total"] / out["time_to_solution_s"]["fp64"]
        out["pbar_rel_diff_mixed_vs_fp64"] = float(np.abs(Pbar_mixed - r64["Pbar"]).max() /
                                                   np.abs(r64["Pbar"]).max())
        out["_Pbar_fp64"] = r64["Pbar"]
        log("fp64: %.2f s, cg %d" % (out["time_to_solution_s"]["fp64"], r64["stats"]["cg_iters_total"]))
    if not args.no_batched_256:
        out["batched_256"] = batched_256(combo, ms, lc, options(combo.COMBO_MIXED), out)
    if not args.no_willot:
        # the same workload under Willot's rotated scheme
        combo.combo_set_discretization(ctx, combo.COMBO_DISC_WILLOT)
        combo.combo_set_materials(ctx, lc.mats)
        combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(dev), torch.from_numpy(ms.c).to(dev),
                                       torch.from_numpy(np.ascontiguousarray(ms.N)).to(dev))
        combo.combo_set_options(ctx, options(combo.COMBO_MIXED))
        combo.combo_profile_enable(ctx, True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rw = combo.combo_solve(ctx, lc.Fbar)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        pw = combo.combo_profile_all(ctx)
        combo.combo_profile_enable(ctx, False)
        out["willot"] = {"discretization": "rotated (HEX8R) scheme, two-stage FFT passes, mixed",
                         "time_to_solution_s": el, "newton_iters": rw["stats"]["newton_iters"],
                         "cg_iters": rw["stats"]["cg_iters_total"],
                         "voxel_cg_iters_per_s": n * rw["stats"]["cg_iters_total"] / el,
                         "pbar_rel_diff_vs_ms": float(np.abs(rw["Pbar"] - Pbar_mixed).max() /
                                                      np.abs(Pbar_mixed).max()),
                         "kernels_avg_us": {k: round(v[0] / v[1] * 1e3, 1) for k, v in pw.items() if v[1]}}
        log("willot: %.2f s, newton %d, cg %d" % (el, rw["stats"]["newton_iters"], rw["stats"]["cg_iters_total"]))
        combo.combo_set_discretization(ctx, combo.COMBO_DISC_MS)
        combo.combo_set_materials(ctx, lc.mats)
        combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(dev), torch.from_numpy(ms.c).to(dev),
                                       torch.from_numpy(np.ascontiguousarray(ms.N)).to(dev))
    if not args.no_staggered:
        # the same workload on the staggered grid with the DFMG law (App. A), mixed: the
        # first five increments of the load path (10 % stretch, same increment size)
        combo.combo_set_discretization(ctx, combo.COMBO_DISC_STAGGERED)
        combo.combo_set_materials(ctx, lc.mats)
        combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(dev), torch.from_numpy(ms.c).to(dev),
                                       torch.from_numpy(np.ascontiguousarray(ms.N)).to(dev))
        o = options(combo.COMBO_MIXED)
        o.autotune = 0
        K_st = max(1, lc.n_increments // 2)
        o.n_increments = K_st
        combo.combo_set_options(ctx, o)
        Fb_st = np.eye(3) + (lc.Fbar - np.eye(3)) * K_st / lc.n_increments
        combo.combo_profile_enable(ctx, True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rs = combo.combo_solve(ctx, Fb_st)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        ps = combo.combo_profile_all(ctx)
        combo.combo_profile_enable(ctx, False)
        cg_st = rs["stats"]["cg_iters_total"]
        # algorithmic bytes of one CG iteration's tangent part, FP32 fields: x inverse (9 complex
        # half spectra in, dH 36 B/voxel out), DFMG action (dH 36 B, F in FP64 72 B, slot 4 B in;
        # own + parts 108 B out; 8 packed 45-entry tangents, 1440 B, per composite), DFMG sum
        # (108 B in, dQ 36 B out), x forward (dQ 36 B in, 9 complex half spectra out)
        nspec_st = (ms.n[0] // 2 + 1) * ms.n[1] * ms.n[2]
        xb = 2 * 9 * 8 * nspec_st + n * (36 + 36 + 72 + 4 + 108 + 108 + 36 + 36) + 1440 * ms.n_composite
        xms, xcnt = ps.get("xpass_cg", (0.0, 0))
        out["staggered"] = {"discretization": "staggered grid, DFMG law (8 doubly-fine cells per cell), mixed",
                            "load": "first %d of %d increments (%.0f %% stretch)" % (
                                K_st, lc.n_increments, 100 * (Fb_st[0, 0] - 1.0)),
                            "time_to_solution_s": el, "newton_iters": rs["stats"]["newton_iters"],
                            "cg_iters": cg_st, "voxel_cg_iters_per_s": n * cg_st / el,
                            "laminate_solves_per_composite_per_eval": 8,
                            "kernels_avg_us": {k: round(v[0] / v[1] * 1e3, 1) for k, v in ps.items() if v[1]},
                            "tangent_part_GBps": round(xb / (xms / xcnt * 1e-3) / 1e9, 1) if xcnt else None}
        log("staggered: %.2f s, newton %d, cg %d" % (el, rs["stats"]["newton_iters"], cg_st))
        combo.combo_set_discretization(ctx, combo.COMBO_DISC_MS)
        combo.combo_set_materials(ctx, lc.mats)
        combo.combo_set_microstructure(ctx, torch.from_numpy(ms.phase).to(dev), torch.from_numpy(ms.c).to(dev),
                                       torch.from_numpy(np.ascontiguousarray(ms.N)).to(dev))
    if not args.no_small_strain:
        # the same RVE under the small-strain law (closed-form laminate): one linear solve
        o = options(combo.COMBO_MIXED)
        o.law = combo.COMBO_LAW_LINEAR
        o.n_increments = 1
        combo.combo_set_options(ctx, o)
        combo.combo_solve(ctx, lc.Fbar)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cg_lin = 0
        for k in range(args.steps):
            rl = combo.combo_solve(ctx, lc.Fbar)
            cg_lin += rl["stats"]["cg_iters_total"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        out["small_strain"] = {"law": "linear (closed-form laminate)", "precision": "mixed",
                               "load": "H = 0.2 e1 (x) e1, eta<=1e-6, tol_cg %.0e" % args.tol_cg,
                               "time_to_solution_s": el / args.steps, "newton_iters": rl["stats"]["newton_iters"],
                               "cg_iters": cg_lin / args.steps, "voxel_cg_iters_per_s": n * cg_lin / el,
                               "laminate_ms": rl["stats"]["time_ms_material"]}
        log("small strain: %.3f s, newton %d, cg %d" % (el / args.steps, rl["stats"]["newton_iters"],
                                                         rl["stats"]["cg_iters_total"]))
    combo.combo_destroy(ctx)
    out["image_to_boxels"] = None if args.no_image else image_bench(combo, synth, ms, args.steps)
    out["batch"] = None if args.no_batch else batch_bench(combo, synth, args.steps)
    out["fibres"] = None if args.no_fibres else fibres_bench(combo, synth, args.fibre_seconds)
    if not args.no_cpu:
        t = time.time()
        out["cpu_baseline"] = cpu_baseline(ms, lc)
        log("cpu baseline in %.1f s" % (time.time() - t))
    else:
        out["cpu_baseline"] = None
    out.pop("_Pbar_fp64", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
