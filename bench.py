"""Benchmark: the null-space-free eigensolver's hot path on one MI355X.

A step is one invert-Lanczos eigensolve of the HHPD pencil (Thm 4.2) for the
10 smallest positive eigenvalues at 128^3 (every row of the hot path: basis
tables, basis synthesis, twisted FFTs, constitutive step, projection, CG,
Lanczos).  The reported value is the whole-job SVD-FFT matvec throughput: the
algorithmic bytes of every A_r apply the steps performed (336 n B each) over
the wall time of the timed steps.  The isolated A_r apply, its per-kernel
times (HIP events on the plan's stream) and the CPU oracle timed on the host
are reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere128|rods128|sphere64]

After the timed steps the default run adds, outside the timed region: the other
configurations (128^3 rods apply, 64^3 and 16^3 eigensolves), the batched-vs-plain
legs (the 40-point Gamma-X-M-Gamma-R path of the 128^3 rods, the 32-instance uneven
batch), the gradient with central differences at 50 voxels (64^3), the paper's
band-structure path G-X-M-R-G at 128^3 for both of its media, the chirality
sweep (64^3), the NFSEP path (64^3) and the CPU oracle.

Every plan (and batch) first autotunes its pass tiling, outside the timed
regions, with the results cached for the run by grid shape, medium kind and
vacuum share (NSF_TUNE_CACHE); --no-autotune, or an explicit --mid-cols /
--yz-cols / --x-rows, keeps the given tiling.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SVD-FFT matvec GB/s at 128^3; eigenpairs/s batched vs plain at res≤1e-8"
HBM_PEAK_GBPS = 8000.0
MAX_RESTARTS = 100  # per eigensolve in the secondary legs (a converging 128^3 solve needs about 10)
BYTES_PER_APPLY_PER_N = 336  # y in (64n) + 6 fields out (96n) + in (96n) + medium (16n) + out (64n)
NFSEP_FIELD_BYTES_PER_N = 320  # the same field traffic; the NFSEP medium adds 576 B (per voxel) or 2 B (palette)

WORKLOADS = {
    "sphere128": dict(grid=(128, 128, 128), k=(0.1, 0.2, 0.3), kind="chiral",
                      desc="chiral sphere r=0.3 eps 13 gamma 0.5, background eps 1, 128^3, k=(0.1,0.2,0.3)"),
    "rods128": dict(grid=(128, 128, 128), k=(0.1, 0.2, 0.3), kind="pseudo",
                    desc="pseudochiral x-y rods r=0.2 eps 13 gamma 0.4, 128^3, k=(0.1,0.2,0.3)"),
    "sphere64": dict(grid=(64, 64, 64), k=(0.25, 0.0, 0.0), kind="chiral",
                     desc="chiral sphere r=0.3 eps 13 gamma 0.5, 64^3, k=(0.25,0,0)"),
    "scsc128": dict(grid=(128, 128, 128), k=(0.1, 0.2, 0.3), kind="scsc",
                    desc="simple cubic spheres r=0.345 joined by cylinders s=0.11, (eps_i, eps_o, gamma) = "
                         "(13, 1, 0.5), 128^3, k=(0.1,0.2,0.3)"),
}


def make_medium(w):
    from paper_1402_6297_amd import media

    n1 = w["grid"][0]
    if w["kind"] == "chiral":
        return media.sphere_chiral(n1)
    if w["kind"] == "scsc":
        return media.spheres_cylinders_chiral(n1)
    return media.rods_pseudochiral(n1)


AUTOTUNE = True  # every leg tunes its plans' pass tiling first (outside the timed regions)


def tune(obj):
    """Autotune a plan or batch (per grid shape; NSF_TUNE_CACHE makes repeats free)."""
    if AUTOTUNE:
        obj.autotune(reps=5)


def batch_instances(name):
    """(grids, ks, media, nev) of the batched workloads."""
    from paper_1402_6297_amd import media

    if name == "kpath128":  # Gamma-X-M-Gamma-R, 10 per segment, x-y rods at 128^3
        ks = media.kpath_gxmgr(10)
        eps, gam = media.rods_pseudochiral(128)
        return [(128, 128, 128)] * len(ks), ks, [("pseudo", eps, gam)] * len(ks), 10
    if name.startswith("uneven"):  # mixed 48..128^3 chiral spheres
        count = int(name[len("uneven"):] or 32)
        out = media.uneven_batch(count=count, seed=0)
        grids = [o["grid"] for o in out]
        ks = [o["k"] for o in out]
        med = [("chiral",) + media.sphere_chiral(o["grid"][0], radius=o["radius"], eps_in=o["eps_in"],
                                                gamma_in=o["gamma_in"]) for o in out]
        return grids, ks, med, 8
    raise ValueError(name)


def batch_leg(name, log=sys.stderr):
    """Eigenpairs/s of one batched schedule against the plain per-instance loop."""
    import torch

    from paper_1402_6297_amd import nsf

    grids, ks, med, nev = batch_instances(name)
    kw = dict(res_tol=1e-8, cg_rtol=1e-10, seed=0, max_restarts=MAX_RESTARTS)
    # plain: one plan at a time; plan set-up (tables, medium upload) is outside
    # the timed region in both schedules, only the eigensolves are timed
    t_plain = 0.0
    plain_pairs, plain_mv = 0, 0
    for i, (g, k, m) in enumerate(zip(grids, ks, med)):
        with nsf.Plan(g, k) as P:
            if m[0] == "chiral":
                P.set_chiral(m[1], m[2])
            else:
                P.set_pseudochiral(0, 1, m[1], m[2])
            tune(P)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, om, res, stats = P.eigs(nev, seed=kw["seed"] + 1000003 * i, res_tol=kw["res_tol"],
                                        cg_rtol=kw["cg_rtol"], max_restarts=kw["max_restarts"])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            t_plain += dt
            plain_pairs += stats["converged"]
            plain_mv += stats["matvecs"]
        print(f"[bench] {name} plain {i}: {g[0]}^3 k={np.round(k, 4).tolist()} status {st}, "
              f"{stats['lanczos_steps']} steps, {dt:.2f} s", file=log, flush=True)
    print(f"[bench] {name} plain: {len(grids)} instances, {t_plain:.1f} s", file=log, flush=True)
    with nsf.Batch(grids, ks) as B:
        for i, m in enumerate(med):
            if m[0] == "chiral":
                B.set_chiral(i, m[1], m[2])
            else:
                B.set_pseudochiral(i, 0, 1, m[1], m[2])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        shapes = B.autotune(reps=5) if AUTOTUNE else 0  # tiling per grid shape (set-up, reported apart)
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
        t0 = time.perf_counter()
        st, om, res, stats, wave = B.eigs(nev, **kw)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
    pairs = sum(s["converged"] for s in stats)
    print(f"[bench] {name} batched: {t_batch:.1f} s, wave {wave}, {shapes} shapes autotuned", file=log, flush=True)
    return {"workload": name, "instances": len(grids), "nev": nev, "wave": wave,
            "eigenpairs_per_s_batched": round(pairs / t_batch, 4),
            "eigenpairs_per_s_plain": round(plain_pairs / t_plain, 4),
            "s_batched": round(t_batch, 3), "s_plain": round(t_plain, 3), "s_autotune": round(t_tune, 3),
            "max_residual": float(res.max()), "status": st,
            "grids": sorted(set(f"{g[0]}^3" for g in grids))}


def kpath_warm_leg(log=sys.stderr, nev=10):
    """The 40-point k-path of the 128^3 rods with warm starts: the plain loop starts
    each k-point from the previous one's Ritz vectors (nsf_eigs_set_start); the
    batched schedule is one nsf_batch_eigs call over the path with
    NSF_OPT_WARM_CHAIN on k-points 1..39, which chains the same starts inside the
    batch (each 128^3 instance runs in a wave of its own)."""
    import torch

    from paper_1402_6297_amd import media, nsf

    ks = media.kpath_gxmgr(10)
    eps, gam = media.rods_pseudochiral(128)
    g = (128, 128, 128)
    n = 128 ** 3
    kw = dict(res_tol=1e-8, cg_rtol=1e-10, seed=0)
    t_plain, pairs_plain, steps_plain, prev = 0.0, 0, 0, None
    for i, k in enumerate(ks):
        with nsf.Plan(g, k) as P:
            P.set_pseudochiral(0, 1, eps, gam)
            tune(P)
            Y = torch.empty((nev, 4 * n), dtype=torch.complex128, device="cuda")
            if prev is not None:
                P.set_start(prev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, om, res, stats = P.eigs(nev, Y=Y, **kw)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t0
            pairs_plain += stats["converged"]
            steps_plain += stats["lanczos_steps"]
            prev = Y
        print(f"[bench] kpath128 warm plain {i}: {stats['lanczos_steps']} steps", file=log, flush=True)
    del prev, Y
    print(f"[bench] kpath128 warm plain: {t_plain:.1f} s", file=log, flush=True)
    with nsf.Batch([g] * len(ks), ks) as B:
        for i in range(len(ks)):
            B.set_pseudochiral(i, 0, 1, eps, gam)
            nsf.nsf_plan_set_option(B.plan(i), nsf.NSF_OPT_WARM_CHAIN, int(i > 0))
        tune(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, om, res, stats, wave = B.eigs(nev, **kw)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
    pairs_batch = sum(s["converged"] for s in stats)
    steps_batch = sum(s["lanczos_steps"] for s in stats)
    print(f"[bench] kpath128 warm batched: {t_batch:.1f} s, status {st}", file=log, flush=True)
    return {"workload": "kpath128 with warm starts", "instances": len(ks), "nev": nev,
            "schedule": "batched: one call, starts chained inside the batch; plain: chained nsf_eigs calls",
            "eigenpairs_per_s_batched": round(pairs_batch / t_batch, 4),
            "eigenpairs_per_s_plain": round(pairs_plain / t_plain, 4),
            "s_batched": round(t_batch, 3), "s_plain": round(t_plain, 3),
            "lanczos_steps_plain": steps_plain, "lanczos_steps_batched": steps_batch,
            "max_residual": float(res.max()), "status": st}


def gamma_sweep_leg(n1=64, log=sys.stderr, nev=10):
    """CG conditioning against the chirality (the paper's second test set): the
    spheres-and-cylinders structure at k = (1/2, 0, 0), eps_i = 13 with gamma from
    0.25 to 3 and eps_i = 1 with gamma from 0.05 to 0.9 (Phi -> 0 as gamma ->
    sqrt(eps_i)).  Reports CG iterations per solve and the eigenvalues."""
    import torch

    from paper_1402_6297_amd import media, nsf

    out = []
    for eps_i, gammas in ((13.0, (0.25, 1.0, 2.0, 3.0)), (1.0, (0.05, 0.3, 0.6, 0.9))):
        for gmm in gammas:
            eps, gam = media.spheres_cylinders_chiral(n1, eps_in=eps_i, eps_out=1.0, gamma=gmm)
            with nsf.Plan((n1, n1, n1), (0.5, 0.0, 0.0)) as P:
                P.set_chiral(eps, gam)
                tune(P)
                P.set_option(nsf.NSF_OPT_VERIFY, 16)  # k on a lattice axis of a cubic structure
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, om, res, stats = P.eigs(nev, res_tol=1e-8, cg_rtol=1e-10, max_restarts=MAX_RESTARTS)
                torch.cuda.synchronize()
                out.append({"eps_i": eps_i, "gamma": gmm, "status": st, "s": round(time.perf_counter() - t0, 3),
                            "cg_iters_avg": round(stats["cg_iters_avg"], 2), "lanczos_steps": stats["lanczos_steps"],
                            "omega": [round(x, 8) for x in om.tolist()], "max_residual": float(res.max())})
            print(f"[bench] gamma sweep eps_i {eps_i} gamma {gmm}: cg avg {out[-1]['cg_iters_avg']}",
                  file=log, flush=True)
    return {"workload": f"spheres+cylinders {n1}^3, k=(0.5,0,0), nev={nev}, multiplicity check on",
            "paper_pcg_iters_avg_128": {"eps_i=13, gamma 0.25->3": "39->90", "eps_i=1, gamma 0.05->0.9": "9->59",
                                        "note": "MATLAB pcg to 1e-14 at 128^3 (context)"},
            "points": out}


# The paper's band-structure runs (Sec. 5, first test set): 128^3, spheres joined
# by cylinders, G-X-M-R-G with ten wave vectors per segment, 10 smallest positive
# omega; Lanczos iterations and CPU hours per k-point as printed there (MATLAB
# eigs + pcg on 2x Intel Xeon X5687, 8 cores, 3.6 GHz).  Context, not targets.
PAPER_BAND = (
    ((13.0, 1.0, 0.5), {"lanczos_iters": "120-190", "lanczos_iters_avg": 143, "hours_per_k": "2.75-4",
                        "hours_per_k_avg": 3.2}),
    ((1.0, 1.0, 0.8), {"lanczos_iters": "100-200", "lanczos_iters_avg": 136, "hours_per_k": "2.1-4.1",
                       "hours_per_k_avg": 2.8}),
)


def band_leg(per_seg, n1=128, log=sys.stderr, nev=10):
    """The paper's band-structure workload on the GPU: both media along G-X-M-R-G
    (per_seg wave vectors per segment, segment midpoints), each k-point one plain
    eigensolve with the multiplicity check on (the path's symmetric k-points can
    carry multiple eigenvalues).  Per-k Lanczos steps, CG iterations and seconds,
    beside the paper's ranges."""
    import torch

    from paper_1402_6297_amd import media, nsf

    ks = media.kpath_gxmrg(per_seg)
    grid = (n1, n1, n1)
    out = []
    for (ei, eo, g), paper in PAPER_BAND:
        eps, gam = media.spheres_cylinders_chiral(n1, eps_in=ei, eps_out=eo, gamma=g)
        eps_d, gam_d = torch.from_numpy(eps).to("cuda"), torch.from_numpy(gam).to("cuda")
        pts = []
        for k in ks:
            with nsf.Plan(grid, tuple(k)) as P:
                P.set_chiral(eps_d, gam_d)
                tune(P)
                P.set_option(nsf.NSF_OPT_VERIFY, 16)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, om, res, stats = P.eigs(nev, res_tol=1e-8, cg_rtol=1e-10, max_restarts=MAX_RESTARTS)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            print(f"[bench] band ({ei:g},{eo:g},{g:g}) k={np.round(k, 4).tolist()}: status {st}, "
                  f"{stats['lanczos_steps']} steps, {dt:.2f} s", file=log, flush=True)
            pts.append({"k": [round(x, 6) for x in k.tolist()], "status": st, "s": round(dt, 3),
                        "lanczos_steps": stats["lanczos_steps"], "cg_iters_avg": round(stats["cg_iters_avg"], 2),
                        "applies": stats["matvecs"], "max_residual": float(res.max()),
                        "omega_over_2pi": [round(x / (2 * np.pi), 8) for x in om.tolist()]})
        steps = np.array([p["lanczos_steps"] for p in pts])
        secs = np.array([p["s"] for p in pts])
        summ = {"medium": f"(eps_i, eps_o, gamma) = ({ei:g}, {eo:g}, {g:g})", "k_points": len(pts),
                "status_all_ok": all(p["status"] == 0 for p in pts),
                "lanczos_steps_min_max_avg": [int(steps.min()), int(steps.max()), round(float(steps.mean()), 1)],
                "cg_iters_avg": round(float(np.mean([p["cg_iters_avg"] for p in pts])), 2),
                "s_per_k_min_max_avg": [round(float(secs.min()), 3), round(float(secs.max()), 3),
                                        round(float(secs.mean()), 3)],
                "max_residual": max(p["max_residual"] for p in pts),
                "paper_matlab_2x_xeon_x5687": paper, "points": pts}
        out.append(summ)
        print(f"[bench] band {summ['medium']}: {len(pts)} k, Lanczos steps {summ['lanczos_steps_min_max_avg']}, "
              f"{summ['s_per_k_min_max_avg'][2]} s per k", file=log, flush=True)
        del eps_d, gam_d
    return {"workload": f"spheres r=0.345 joined by cylinders s=0.11 (simple cubic), {n1}^3, G-X-M-R-G with "
                        f"{per_seg} k per segment, nev={nev}, residual <= 1e-8, multiplicity check on",
            "media": out}


def nfsep_leg(n1=64, log=sys.stderr, nev=10):
    """The NFSEP path (Thm 3.2; Algorithm 1, else-branch) on a lossy chiral sphere
    (eps_in = 13 + 0.5i, gamma 0.5, r = 0.3) at n1^3, k = (0.1, 0.2, 0.3), a medium
    outside the HHPD assumption: median K apply and median Kern apply (the A_r
    pipeline with the full 6x6 factor, 896 n B algorithmic), and one zero-shift
    shift-invert Arnoldi eigensolve (nev, residual <= 1e-8, GMRES rtol 1e-10)."""
    import torch

    from paper_1402_6297_amd import media, nsf

    grid, k = (n1, n1, n1), (0.1, 0.2, 0.3)
    n = n1 ** 3
    tens = media.lossy_sphere_tensors(n1)
    u = torch.from_numpy(media.random_vector(4 * n, 0)).to("cuda")
    o = torch.empty_like(u)
    with nsf.Plan(grid, k) as P:  # factors stored per voxel, for comparison
        P.set_option(nsf.NSF_OPT_MEDIUM_PALETTE, 0)
        P.set_nfsep(*tens)
        kern_full_us = median_apply_us(P, u, o)
    with nsf.Plan(grid, k) as P:
        P.set_nfsep(*tens)
        info = P.medium_info()
        kern_us = median_apply_us(P, u, o)
        for _ in range(5):
            P.K(u, o)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
        for a, b in ev:
            a.record()
            P.K(u, o)
            b.record()
        torch.cuda.synchronize()
        k_us = float(np.median([a.elapsed_time(b) * 1e3 for a, b in ev]))
        del u, o
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, om, res, stats = P.eigs_nfsep(nev, res_tol=1e-8, inner_rtol=1e-10)
        dt = time.perf_counter() - t0
    b = (NFSEP_FIELD_BYTES_PER_N + info["voxel_bytes"]) * n
    b_full = (NFSEP_FIELD_BYTES_PER_N + 576) * n
    out = {"workload": f"lossy chiral sphere {n1}^3 (eps 13+0.5i, gamma 0.5), k=(0.1,0.2,0.3), nev={nev}",
           "palette": info["palette"], "bytes_alg_per_apply": b,
           "kern_apply_us": round(kern_us, 2), "kern_GBps_alg": round(b / (kern_us * 1e-6) / 1e9, 2),
           "kern_frac": round(b / (kern_us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4),
           "kern_per_voxel_factors_us": round(kern_full_us, 2),
           "kern_per_voxel_factors_GBps_alg": round(b_full / (kern_full_us * 1e-6) / 1e9, 2),
           "K_apply_us": round(k_us, 2),
           "eigs_status": st, "s_per_solve": round(dt, 3),
           "omega": [[round(w.real, 10), round(w.imag, 10)] for w in om],
           "max_residual": float(res.max()), "applies": stats["matvecs"],
           "gmres_iters_avg": round(stats["cg_iters_avg"], 2), "arnoldi_steps": stats["lanczos_steps"],
           "restarts": stats["restarts"], "value_GBps": round(b * stats["matvecs"] / dt / 1e9, 2),
           "ms_phases": {"gmres": round(stats["ms_cg"], 1), "gram_schmidt": round(stats["ms_orth"], 1),
                         "restart_refine": round(stats["ms_restart"], 1)}}
    print(f"[bench] nfsep {n1}^3: {out['s_per_solve']} s, {out['applies']} applies, "
          f"kern apply {out['kern_apply_us']} us", file=log, flush=True)
    return out


def median_apply_us(P, u, out, reps=100, warm=10):
    """Median of `reps` individually timed A_r applies (HIP events on the plan's
    stream, which is torch's current stream), after `warm` untimed ones."""
    import torch

    for _ in range(warm):
        P.Ar(u, out)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        P.Ar(u, out)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) * 1e3 for a, b in ev]))


def extra_workloads(log=sys.stderr):
    """The other configurations, one small measurement each: the 128^3 rods apply
    (second headline medium), the 64^3 sphere eigensolve and the 16^3 one."""
    import torch

    from paper_1402_6297_amd import media, nsf

    out = {}
    n = 128 ** 3
    with nsf.Plan((128, 128, 128), (0.1, 0.2, 0.3)) as P:
        P.set_pseudochiral(0, 1, *media.rods_pseudochiral(128))
        tune(P)
        u = torch.from_numpy(media.random_vector(4 * n, 0)).to("cuda")
        o = torch.empty_like(u)
        us = median_apply_us(P, u, o)
        out["rods128_apply"] = {"us_median": round(us, 2),
                                "GBps_alg": round(BYTES_PER_APPLY_PER_N * n / (us * 1e-6) / 1e9, 2),
                                "frac": round(BYTES_PER_APPLY_PER_N * n / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)}
        del u, o
    for name, grid, k in (("sphere64_eigs", (64, 64, 64), (0.25, 0.0, 0.0)),
                          ("sphere16_eigs", (16, 16, 16), (0.1, 0.2, 0.3))):
        with nsf.Plan(grid, k) as P:
            P.set_chiral(*media.sphere_chiral(grid[0]))
            tune(P)
            P.eigs(10, res_tol=1e-8, cg_rtol=1e-10)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, om, res, stats = P.eigs(10, res_tol=1e-8, cg_rtol=1e-10)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            nn = grid[0] * grid[1] * grid[2]
            nn_apply = None
            if grid[0] >= 64:
                u = torch.from_numpy(media.random_vector(4 * nn, 0)).to("cuda")
                nn_apply = median_apply_us(P, u, torch.empty_like(u))
            out[name] = {"status": st, "s_per_solve": round(dt, 4), "omega": [round(x, 10) for x in om.tolist()],
                         "max_residual": float(res.max()), "matvecs": stats["matvecs"],
                         "cg_iters_avg": round(stats["cg_iters_avg"], 2), "lanczos_steps": stats["lanczos_steps"],
                         "restarts": stats["restarts"],
                         "value_GBps": round(BYTES_PER_APPLY_PER_N * nn * stats["matvecs"] / dt / 1e9, 2)}
            if nn_apply:
                out[name]["apply_us_median"] = round(nn_apply, 2)
        print(f"[bench] {name}: {out[name]['s_per_solve']} s", file=log, flush=True)
    return out


def grad_leg(nvox, log=sys.stderr, h=1e-6, nev=4):
    """Gradient of S = sum of the 4 smallest omega on the 64^3 noise medium
    (Gaussian-filtered eps in [1, 13], gamma = 0.3 (eps - 1) / 12, k = (0.1, 0.1, 0.1)):
    cost of the gradient kernel against the eigensolve, and central differences
    (step h, every perturbed solve in one batch) at nvox seeded voxels."""
    import torch

    from paper_1402_6297_amd import media, nsf

    grid, k = (64, 64, 64), (0.1, 0.1, 0.1)
    eps, gam = media.noise_chiral(64, sigma_vox=2.0, seed=0)
    n = eps.size
    kw = dict(res_tol=1e-11, cg_rtol=1e-12, max_restarts=MAX_RESTARTS)
    vox = np.random.default_rng(1).choice(n, size=nvox, replace=False)
    with nsf.Plan(grid, k) as P:
        P.set_chiral(eps, gam)
        tune(P)
        Y = torch.empty(nev * 4 * n, dtype=torch.complex128, device="cuda")
        P.eigs(nev, Y=Y, **kw)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, om, res, stats = P.eigs(nev, Y=Y, **kw)
        torch.cuda.synchronize()
        t_eigs = time.perf_counter() - t0
        de = torch.empty(n, dtype=torch.float64, device="cuda")
        dg = torch.empty_like(de)
        P.eig_grad(om, Y, np.ones(nev), de, dg)
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.eig_grad(om, Y, np.ones(nev), de, dg)
        e1.record()
        torch.cuda.synchronize()
        t_grad = e0.elapsed_time(e1) / reps * 1e-3
        an = np.stack([de.cpu().numpy()[vox], dg.cpu().numpy()[vox]])
    print(f"[bench] grad64: eigensolve {t_eigs:.3f} s, gradient {t_grad * 1e6:.0f} us", file=log, flush=True)
    fields = []
    for which in range(2):
        for v in vox:
            for s in (+1, -1):
                e, g = eps.copy().ravel(), gam.copy().ravel()
                (e if which == 0 else g)[v] += s * h
                fields.append((e.reshape(eps.shape), g.reshape(eps.shape)))
    t0 = time.perf_counter()
    with nsf.Batch([grid] * len(fields), [k] * len(fields)) as B:
        for i, (e, g) in enumerate(fields):
            B.set_chiral(i, e, g)
        tune(B)
        stb, omb, resb, _, wave = B.eigs(nev, **kw)
    t_fd = time.perf_counter() - t0
    S = omb.sum(axis=1).reshape(2, nvox, 2)
    fd = (S[:, :, 0] - S[:, :, 1]) / (2 * h)
    err = np.abs(an - fd)
    relerr = err / np.abs(an)
    scale = np.abs(an).max(axis=1, keepdims=True)
    ok = (err <= 5e-3 * np.abs(an)) | (err <= 1e-3 * scale)
    print(f"[bench] grad64: {2 * nvox} FD pairs in {t_fd:.1f} s (wave {wave}), pass {int(ok.sum())}/{ok.size}",
          file=log, flush=True)
    return {"workload": "grad64: 64^3 Gaussian-filtered noise eps in [1,13], gamma=0.3(eps-1)/12, "
                        "k=(0.1,0.1,0.1), S = sum of 4 smallest omega",
            "omega": [round(x, 12) for x in om.tolist()], "eigs_status": st,
            "s_eigensolve": round(t_eigs, 4), "s_gradient": round(t_grad, 6),
            "gradient_over_eigensolve": round(t_grad / t_eigs, 6),
            "fd_voxels": int(nvox), "fd_h": h, "fd_status": stb, "fd_pass": int(ok.sum()), "fd_total": int(ok.size),
            "fd_max_rel_err_eps": float(relerr[0].max()), "fd_max_rel_err_gamma": float(relerr[1].max()),
            "fd_median_rel_err": float(np.median(relerr)), "max_abs_grad_eps": float(scale[0, 0]),
            "max_abs_grad_gamma": float(scale[1, 0]), "s_fd_batch": round(t_fd, 2)}


def _oracle_apply_worker(job):
    """One host process of the CPU baseline: build the oracle's medium tensors for
    the workload, then time `reps` matrix-free A_r applies (numpy, one thread)."""
    if job is None:
        return None  # pool warm-up: the workers start before the GPU is touched
    grid, k, kind, reps = job
    from oracle import medium, nfgep
    from paper_1402_6297_amd import media

    eps, gam = media.sphere_chiral(grid[0]) if kind == "chiral" else media.rods_pseudochiral(grid[0])
    tens = (medium.tensors_chiral(eps, gam) if kind in ("chiral", "scsc")
            else medium.tensors_pseudochiral(eps, gam, (0, 1)))
    u = media.random_vector(4 * grid[0] * grid[1] * grid[2], 0)
    t0 = time.perf_counter()
    for _ in range(reps):
        nfgep.apply_Ar(u, grid, k, tens)
    return reps, time.perf_counter() - t0


def host_workers():
    """Host processes for the all-cores baseline: the CPUs this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, eps, gam, pool=None, nproc=1, budget_s=12.0):
    """The oracle's matrix-free A_r apply on the host, as it stands: one process
    (bounded to ~budget_s), then one process per host core running the same
    applies at once (whole-host throughput), plus the oracle eigensolve times
    stored with the golden files (measured on the build host)."""
    from oracle import medium, nfgep
    from paper_1402_6297_amd import media

    grid, k = w["grid"], w["k"]
    n = grid[0] * grid[1] * grid[2]
    tens = (medium.tensors_chiral(eps, gam) if w["kind"] in ("chiral", "scsc")
            else medium.tensors_pseudochiral(eps, gam, (0, 1)))
    u = media.random_vector(4 * n, 0)
    reps, t0 = 0, time.perf_counter()
    while True:
        nfgep.apply_Ar(u, grid, k, tens)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 10:
            break
    del tens, u
    one = BYTES_PER_APPLY_PER_N * n * reps / el / 1e9
    out = dict(value=one, unit="GB/s", cores=1, kind="oracle",
               sample=f"{reps} oracle A_r applies (numpy FFT, one thread) on the same {grid[0]}^3 "
                      f"workload, {el:.1f} s; {el / reps * 1e3:.0f} ms per apply",
               host_cpu=host_cpu_model())
    if pool is not None and nproc > 1:
        jobs = [(tuple(grid), tuple(k), w["kind"], 2)] * nproc
        t0 = time.perf_counter()
        res = list(pool.map(_oracle_apply_worker, jobs))
        wall = time.perf_counter() - t0
        span = max(r[1] for r in res)
        allv = BYTES_PER_APPLY_PER_N * n * sum(r[0] for r in res) / span / 1e9
        out.update(value=allv, cores=nproc,
                   sample=f"{nproc} host processes at once, each running 2 oracle A_r applies (numpy FFT, "
                          f"one thread) on the same {grid[0]}^3 workload: {span:.1f} s for the slowest "
                          f"({wall:.1f} s with medium set-up); one process alone: {el / reps * 1e3:.0f} ms "
                          f"per apply",
                   value_one_core=one)
    gold = {}
    for name, f in (("eigensolve_16", "config1_16.json"), ("eigensolve_64", "config2_64.json")):
        try:
            g = json.load(open(os.path.join(ROOT, "tests", "golden", f)))
        except OSError:
            continue
        secs = g["seconds"]
        if isinstance(secs, list):  # [sparse shift-invert on the 6n GEP, ARPACK + CG (1e-13) on the pencil]
            e = {"s_shift_invert_6n_gep": round(secs[0], 1), "s_arpack_cg_pencil": round(secs[1], 1)}
        else:
            e = {"s_arpack_cg_pencil": round(secs, 1), "route": g["route"]}
        e.update(grid=g["grid"], k=g["k"], nev=10, timed="stored with the golden file, not in this run",
                 host="8-core Intel Xeon @ 2.7 GHz (build host), one process")
        gold[name] = e
    out["oracle_eigensolve"] = gold
    return out


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


# Sources the A_r apply kernels are compiled from (the passes and their shared
# device code); stored traffic figures apply only while these are unchanged.
APPLY_SOURCES = ("fft_fast.hip", "fft_passes.hip", "fft_wave.hip", "fft_common.h", "nsf_internal.h")


def kernel_source_hash():
    """Hash of the A_r apply kernel sources."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_1402_6297_amd", "csrc")
    h = hashlib.sha256()
    for f in APPLY_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def _kernel_key(name):
    import re

    m = re.search(r"::(k_\w+(<[^>]*>)?)", name)
    return m.group(1) if m else name.split("(")[0][:60]


def summarize_trace(d):
    """Markdown table of a rocprofv3 --kernel-trace --stats CSV directory."""
    import csv
    import glob

    path = glob.glob(os.path.join(d, "*kernel_stats.csv"))[0]
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{_kernel_key(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def summarize_pmc(fetch_dir, write_dir, applies, workload, tiling):
    """Per-kernel HBM bytes from FETCH_SIZE / WRITE_SIZE runs, calibrated on the
    1 GiB device copy of the same run (known: 1 GiB read, 1 GiB written)."""
    import collections
    import csv
    import glob

    def load(d, ctr):
        rows = list(csv.DictReader(open(glob.glob(os.path.join(d, "*counter_collection.csv"))[0])))
        acc = collections.defaultdict(list)
        for r in rows:
            if r["Counter_Name"] == ctr:
                acc[_kernel_key(r["Kernel_Name"])].append(float(r["Counter_Value"]) * 1024.0)
        return acc

    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy = "__amd_rocclr_copyBuffer"
    f_scale = (1 << 30) / (sum(fe[copy]) / len(fe[copy]))
    w_scale = (1 << 30) / (sum(wr[copy]) / len(wr[copy]))
    kernels = {}
    for k in fe:
        if not k.startswith("k_"):
            continue
        fb = sum(fe[k]) / len(fe[k]) * f_scale
        wb = sum(wr.get(k, [0.0])) / max(len(wr.get(k, [1])), 1) * w_scale
        kernels[k] = {"fetch_bytes": fb, "write_bytes": wb, "launches": len(fe[k])}
    per_apply = sum((v["fetch_bytes"] + v["write_bytes"]) * v["launches"] for v in kernels.values()) / applies
    return {"workload": workload, "source_hash": kernel_source_hash(), "tiling": tiling, "fetch_scale": f_scale,
            "write_scale": w_scale, "kernels": kernels, "bytes_per_apply": per_apply}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere128", choices=sorted(WORKLOADS))
    ap.add_argument("--nev", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the rods / 64^3 / 16^3 measurements")
    ap.add_argument("--matvec-reps", type=int, default=50)
    ap.add_argument("--fft-path", type=int, default=0, help="nsf_plan_set_option(NSF_OPT_FFT_PATH)")
    ap.add_argument("--mid-cols", type=int, default=0, help="nsf_plan_set_option(NSF_OPT_MID_COLS)")
    ap.add_argument("--mid-pairs", type=int, default=-1, help="nsf_plan_set_option(NSF_OPT_MID_PAIRS)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default pass tiling (every leg autotunes its plans otherwise)")
    ap.add_argument("--yz-cols", type=int, default=0, help="nsf_plan_set_option(NSF_OPT_YZ_COLS)")
    ap.add_argument("--x-rows", type=int, default=0, help="nsf_plan_set_option(NSF_OPT_X_ROWS)")
    ap.add_argument("--profile-applies", type=int, default=0,
                    help="only run this many A_r applies plus a 1 GiB device copy (for rocprofv3)")
    ap.add_argument("--summarize-trace", metavar="DIR", help="print a rocprofv3 kernel-stats table and exit")
    ap.add_argument("--batch", default="kpath128,uneven32",
                    help="comma-separated batched-vs-plain legs after the steps: kpath128, kpath128warm, "
                         "uneven32, unevenN; or none")
    ap.add_argument("--gamma-sweep", type=int, default=64, metavar="N",
                    help="CG iterations against chirality at N^3 (0 skips it)")
    ap.add_argument("--band", type=int, default=3, metavar="PER_SEG",
                    help="the paper's 128^3 band-structure leg, PER_SEG k-points per segment of G-X-M-R-G "
                         "(the paper uses 10; 0 skips it)")
    ap.add_argument("--nfsep", type=int, default=64, metavar="N",
                    help="NFSEP leg (lossy sphere, shift-invert Arnoldi) at N^3; 0 skips it")
    ap.add_argument("--nfsep-only", action="store_true",
                    help="run only the NFSEP leg (at --nfsep N) and print its JSON")
    ap.add_argument("--grad", type=int, default=50, metavar="NVOX",
                    help="gradient leg at 64^3: kernel cost and central differences at NVOX voxels")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/ar_apply_traffic_<workload>.json from two --pmc runs and exit")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_pmc:
        tiling = {"mid_cols": args.mid_cols or 16, "yz_cols": args.yz_cols or 16, "x_rows": args.x_rows or 4}
        res = summarize_pmc(*args.summarize_pmc, applies=args.profile_applies or 3, workload=args.workload,
                            tiling=tiling)
        path = os.path.join(ROOT, "profiles", f"ar_apply_traffic_{args.workload}.json")
        with open(path, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent k-points and instances shard across GPUs without communication; one grid "
              "split in z-slabs would need an all-to-all before and after the fused z pass",
              file=sys.stderr)
        sys.exit(2)
    global AUTOTUNE
    AUTOTUNE = not args.no_autotune and not args.mid_cols and not args.yz_cols and not args.x_rows
    if AUTOTUNE and not os.environ.get("NSF_TUNE_CACHE"):
        # one tuning per grid shape, medium kind and vacuum share for this run
        fd, cache = tempfile.mkstemp(prefix="nsf_tune_", suffix=".txt")
        os.close(fd)
        os.environ["NSF_TUNE_CACHE"] = cache

    pool, nproc = None, 1
    if not args.no_cpu and not args.nfsep_only and not args.profile_applies:
        # host processes for the all-cores CPU baseline, started (and idle) before
        # anything touches the GPU
        import concurrent.futures
        import multiprocessing

        nproc = host_workers()
        if nproc > 1:
            pool = concurrent.futures.ProcessPoolExecutor(nproc, mp_context=multiprocessing.get_context("spawn"))
            list(pool.map(_oracle_apply_worker, [None] * nproc))

    import torch

    from paper_1402_6297_amd import media, nsf

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.nfsep_only:
        print(json.dumps(nfsep_leg(args.nfsep or 128)), flush=True)
        return
    w = WORKLOADS[args.workload]
    grid, k = w["grid"], w["k"]
    n = grid[0] * grid[1] * grid[2]
    eps, gam = make_medium(w)
    print(f"[bench] workload {args.workload}: {w['desc']}", file=sys.stderr, flush=True)
    P = nsf.Plan(grid, k)
    P.set_option(nsf.NSF_OPT_FFT_PATH, args.fft_path)
    if args.mid_cols:
        P.set_option(nsf.NSF_OPT_MID_COLS, args.mid_cols)
    if args.mid_pairs >= 0:
        P.set_option(nsf.NSF_OPT_MID_PAIRS, args.mid_pairs)
    dev_info = nsf.nsf_device_info(0)
    print(f"[bench] device {dev_info}", file=sys.stderr, flush=True)
    if w["kind"] in ("chiral", "scsc"):
        P.set_chiral(eps, gam)
    else:
        P.set_pseudochiral(0, 1, eps, gam)

    if args.yz_cols:
        P.set_option(nsf.NSF_OPT_YZ_COLS, args.yz_cols)
    if args.x_rows:
        P.set_option(nsf.NSF_OPT_X_ROWS, args.x_rows)
    tuned = None
    if AUTOTUNE:
        tuned = P.autotune(reps=5)
        print(f"[bench] autotune: {tuned}", file=sys.stderr, flush=True)
    # ---- isolated A_r apply: per-kernel HIP-event times and the whole apply
    u = torch.from_numpy(media.random_vector(4 * n, 0)).to("cuda")
    out = torch.empty_like(u)
    if args.profile_applies:
        # short run for hardware counters: the applies, then a plain copy of
        # known size whose FETCH_SIZE / WRITE_SIZE calibrate the counters
        for _ in range(args.profile_applies):
            P.Ar(u, out)
        src = torch.empty(1 << 26, dtype=torch.complex128, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_applies": args.profile_applies, "copy_bytes": 2 * src.numel() * 16}))
        return
    for _ in range(10):
        P.Ar(u, out)
    torch.cuda.synchronize()
    pass_ms, apply_ms = P.profile_Ar(u, out, reps=args.matvec_reps)
    b_alg = BYTES_PER_APPLY_PER_N * n
    apply_ms = median_apply_us(P, u, out) * 1e-3  # headline: median of 100 timed applies
    apply_gbps = b_alg / (apply_ms * 1e-3) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", f"ar_apply_traffic_{args.workload}.json")
    if os.path.exists(tpath):
        t = json.load(open(tpath))
        used = {"mid_cols": tuned["mid_cols"], "yz_cols": tuned["yz_cols"], "x_rows": tuned["x_rows"]} if tuned else \
            {"mid_cols": args.mid_cols or 16, "yz_cols": args.yz_cols or 16, "x_rows": args.x_rows or 4}
        # the counters hold for these kernels at this tiling only
        if t.get("source_hash") == kernel_source_hash() and args.fft_path == 0 and t.get("tiling") == used:
            traffic = round(t["bytes_per_apply"])
    print(f"[bench] A_r apply {apply_ms * 1e3:.1f} us, {apply_gbps:.0f} GB/s algorithmic; "
          f"kernels (us): {[round(x * 1e3, 1) for x in pass_ms]}", file=sys.stderr, flush=True)

    # ---- steps: full eigensolves
    nev = args.nev
    kw = dict(res_tol=1e-8, cg_rtol=1e-10, seed=0)
    for i in range(args.warmup):
        st, om, res, stats = P.eigs(nev, **kw)
        print(f"[bench] warmup {i}: status {st}, {stats['matvecs']} applies, {stats['ms_total']:.0f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tot_mv, tot_pairs, results = 0, 0, []
    t0 = time.perf_counter()
    for i in range(args.steps):
        st, om, res, stats = P.eigs(nev, **kw)
        tot_mv += stats["matvecs"]
        tot_pairs += stats["converged"]
        results.append((st, om, res, stats))
        print(f"[bench] step {i}: status {st}, {stats['matvecs']} applies, "
              f"cg avg {stats['cg_iters_avg']:.1f}, {stats['ms_total']:.0f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = b_alg * tot_mv / elapsed / 1e9
    st, om, res, stats = results[-1]

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['desc']}; invert Lanczos nev={nev}, "
                               f"CG rtol 1e-10, residual <= 1e-8, complex128",
                   "grid": list(grid), "k": list(k), "nev": nev, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": round(apply_gbps, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(apply_gbps / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "A_r apply (all five kernels of one apply, 336 n B algorithmic; median of 100 applies timed with HIP events)",
                     "traffic_note": "bytes per apply between the L2 caches and the memory fabric (HBM plus the "
                                     "Infinity Cache), rocprofv3 FETCH_SIZE + WRITE_SIZE calibrated on a 1 GiB copy",
                     "kernel_us": [round(x * 1e3, 2) for x in pass_ms]},
        "device": dev_info,
        "autotune": tuned,
        "matvec": {"us_per_apply_median": round(apply_ms * 1e3, 2), "GBps_alg": round(apply_gbps, 2),
                   "bytes_alg": b_alg, "traffic_bytes": traffic,
                   "traffic_GBps": round(traffic / (apply_ms * 1e-3) / 1e9, 2) if traffic else None},
        "eigs": {"status": st, "omega": [round(x, 12) for x in om.tolist()],
                 "max_residual": float(res.max()), "eigenpairs_per_s": round(tot_pairs / elapsed, 4),
                 "matvecs_per_solve": stats["matvecs"], "cg_iters_avg": round(stats["cg_iters_avg"], 2),
                 "lanczos_steps": stats["lanczos_steps"], "restarts": stats["restarts"],
                 "s_per_solve": round(elapsed / args.steps, 3),
                 "ms_phases": {"cg": round(stats["ms_cg"], 1), "gram_schmidt": round(stats["ms_orth"], 1),
                               "restart_refine": round(stats["ms_restart"], 1)}},
    }
    if not args.no_extra:
        line["other_configs"] = extra_workloads()
    batches = []
    for name in [b for b in args.batch.split(",") if b and b != "none"]:
        batches.append(kpath_warm_leg() if name == "kpath128warm" else batch_leg(name))
    if batches:
        line["batch"] = batches[0] if len(batches) == 1 else batches
    if args.grad:
        line["grad"] = grad_leg(args.grad)
    if args.band:
        line["band"] = band_leg(args.band)
    if args.gamma_sweep:
        line["gamma_sweep"] = gamma_sweep_leg(args.gamma_sweep)
    if args.nfsep:
        line["nfsep"] = nfsep_leg(args.nfsep)
    P.close()
    if not args.no_cpu:
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, eps, gam, pool, nproc)
    if pool is not None:
        pool.shutdown()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
