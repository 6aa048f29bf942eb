"""Benchmark: the exact block-Toeplitz PMCHW product (fast-solver appendix),
mixed-precision batched solves and the adjoint sigma gradient on one GPU.

Workload: two parallel 0.4 x 0.2 dielectric channels (eps 12.25 in air, gap
0.3), 30 long, quartic surface-conductivity absorbers of length 4 at both
ends, mesh edge 0.072 (N = 102,852 unknowns; 417 periodic rings of 108 RWG
edges, circulant length 864); lengths in wavelengths inside the guide.
Synthetic, seeded inputs (synth package).

One step = one pass of the whole hot path: a batched mixed-precision solve of
B = 8 seeded dipoles in channel 0 to relative residual 1e-6 (FP32 block-
Toeplitz products inside GMRES, FP64 orthogonalisation and FP64 refinement
residual, right Schwarz preconditioner), then, for dipole 0, the reflected
amplitude at 16 monitor points on the channel axis, its adjoint (transposed)
mixed solve with the exact transposed block-Toeplitz product and the sigma
gradient from the Galerkin matrix's own point fields.  value = operator
products per second over the timed steps (forward and transposed, FP32 and
FP64, all right-hand sides).

Also reported: single-dipole mixed and FP64 solve times (the mixed/FP64
comparison), standalone product rates (1 and 8 vectors), per-stage averages
from HIP events (one extra untimed step with every stage recorded), the
rooflines of the FP32 per-frequency block products (forward and transposed)
and the FP32 Schwarz apply; "roofline" is the one
with the largest total, measured with HIP events on the library stream over
the timed steps, during which only its stage records events; the oracle
timed on the host; and the solution error against the dense Galerkin LU on a
one-wavelength section of the same geometry (oracle leg).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BATCH = 8


def kernel_src_sha(name: str) -> str:
    p = os.path.join(ROOT, "paper_1004_5076_amd", "csrc", name)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


# kernels whose roofline is reported: stage record, kernel name, source file
ROOFLINE_KERNELS = {
    "toeapply32": ("toe_apply_mfma_kernel", "kernels_toeplitz.hip"),
    "precond": ("precond_apply32_mfma_kernel", "kernels_precond.hip"),
    "toeapplyt32": ("toe_t_apply_kernel<float, 1>", "kernels_toeplitz_t.hip"),
}


def measured_ratio(stage: str):
    """HBM bytes over algorithmic bytes of a kernel from committed rocprofv3
    counter runs (FETCH_SIZE and WRITE_SIZE, calibrated on a device copy),
    only if they were taken on the current source of the kernel."""
    p = os.path.join(ROOT, "profiles", "traffic_%s_two_channel.json" % stage)
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_src_sha") != kernel_src_sha(ROOFLINE_KERNELS[stage][1]):
        return None
    return d.get("ratio")


def roofline(prof: dict, stage: str) -> dict:
    """Roofline of one kernel from the stage records of the timed region:
    algorithmic bytes per launch (summed by the library per record) over the
    average launch time from HIP events on the library stream."""
    rec = prof[stage]
    n = max(rec["count"], 1)
    avg_s = rec["ms"] / n * 1e-3
    bytes_launch = rec["bytes"] / n
    achieved = bytes_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    ratio = measured_ratio(stage)
    return {"kernel": ROOFLINE_KERNELS[stage][0], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": ratio * bytes_launch if ratio is not None else None,
            "bytes_per_launch": bytes_launch, "avg_launch_us": avg_s * 1e6, "launches": rec["count"],
            "total_ms": rec["ms"]}


def product_roofline(prof: dict, stage: str = "toeproduct32") -> dict:
    """Roofline of the whole FP32 block-Toeplitz product (every kernel of it,
    transforms, block products and sparse rows), from its stage records:
    tables, stored sparse entries, vectors and ring-axis spectra once each,
    over the average product time."""
    rec = prof[stage]
    n = max(rec["count"], 1)
    avg_s = rec["ms"] / n * 1e-3
    bytes_prod = rec["bytes"] / n
    achieved = bytes_prod / avg_s / 1e9 if avg_s > 0 else 0.0
    return {"kernel": "block-Toeplitz product, all kernels", "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "bytes_per_product": bytes_prod, "avg_product_us": avg_s * 1e6, "products": rec["count"]}


def _host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(w_full_N: int, budget_s: float = 12.0, gpu_check=None) -> dict:
    """The oracle on the host cores, unscaled, on two bounded cases: the
    4-long single guide (configuration 0, N = 2135) and a one-wavelength
    section of the benchmark geometry (two channels, quartic absorber on
    x in [0.5, 1], N = 4338).  Timed: dense Galerkin assembly (OpenMP C),
    LU factorisation (zgetrf) and solve (zgetrs), the dense product (zgemv),
    and the oracle's precorrected-FFT product (numpy FFT + C loops), on all
    host cores and (configuration 0 only, plus the section's product) on one
    core.  value: the dense product rate on all cores extrapolated O(N^2) to
    the benchmark's N (labelled as an extrapolation; the dense matrix would
    need 170 GB there)."""
    import numpy as np
    import scipy.linalg as sla
    from threadpoolctl import threadpool_limits
    import oracle
    import synth
    cores = _host_cores()
    L = oracle.lib()

    def section():
        w = synth.workload_two_channel(length=1.0, absorber=0.5, edge=0.072)
        w.sigma = [synth.SigmaEnd(axis=0, x0=0.5, length=0.5, direction=+1, degree=4, sigma0=1.0)]
        w.dipoles = [synth.seeded_dipole(2000, base=(0.25, -0.35, 0.0), jitter=(0.05, 0.02, 0.02), body=0)]
        w.h, w.r_near = 30.0 / 508, 3.61 * 30.0 / 508
        return w

    def timed(fn, min_s=0.3):
        n, t0 = 0, time.perf_counter()
        while True:
            fn()
            n += 1
            dt = time.perf_counter() - t0
            if dt >= min_s or n >= 50:
                return dt / n

    cases = {}
    for name, wf, one_core in (("config0_guide4", synth.workload_small, True), ("section_1lambda", section, False)):
        w = wf()
        o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
        o.set_sigma(w.sigma)
        rec = {"N": o.N}
        for nthreads in ([cores, 1] if one_core else [cores]):
            L.or_set_threads(nthreads)
            with threadpool_limits(nthreads):
                t0 = time.perf_counter()
                A = o.dense()
                ta = time.perf_counter() - t0
                t0 = time.perf_counter()
                lu = sla.lu_factor(A)
                tf = time.perf_counter() - t0
                b = o.rhs_dipole(w.dipoles[0])
                ts = timed(lambda: sla.lu_solve(lu, b), 0.1)
                x = synth.random_complex(77, o.N)
                tm = timed(lambda: A @ x)
                if gpu_check is not None and nthreads == cores:
                    rec["gpu_solution_error_vs_dense_lu"] = gpu_check(w, sla.lu_solve(lu, b), b)
            rec[f"threads{nthreads}"] = {"assembly_s": ta, "zgetrf_s": tf, "zgetrs_s": ts, "zgemv_s": tm,
                                         "dense_matvecs_per_s": 1.0 / tm}
            del A, lu
        # the oracle's precorrected product (one thread: numpy FFT, C loops)
        L.or_set_threads(1)
        with threadpool_limits(1):
            P = o.pfft(w.h, w.r_near)
            x = synth.random_complex(78, o.N)
            tp = timed(lambda: P.matvec(x), 1.0)
        rec["pfft_product_s_1thread"] = tp
        cases[name] = rec
    L.or_set_threads(cores)
    ref = cases["section_1lambda"]
    rate_ext = ref[f"threads{cores}"]["dense_matvecs_per_s"] * (ref["N"] / w_full_N) ** 2
    pfft_ext = 1.0 / ref["pfft_product_s_1thread"] * (ref["N"] / w_full_N)
    return {"value": rate_ext, "unit": "matvecs/s", "cores": cores, "kind": "oracle",
            "extrapolated": True,
            "sample": (f"dense Galerkin oracle (zgemv) on a one-wavelength two-channel section, N={ref['N']}, "
                       f"{cores} threads; value extrapolated O(N^2) to N={w_full_N}"),
            "cases": cases,
            "pfft_oracle_matvecs_per_s_1thread_extrapolated_linear": pfft_ext,
            "lu_extrapolated_s": ref[f"threads{cores}"]["zgetrf_s"] * (w_full_N / ref["N"]) ** 3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--edge", type=float, default=0.072)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--restart", type=int, default=400)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the untimed single-solve and product-rate runs")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the untimed step with every stage recorded (the roofline kernel is then the "
                         "largest of the roofline kernels over the timed steps)")
    ap.add_argument("--products-only", type=int, default=0,
                    help="run this many FP32 products and preconditioner applies, then a device copy of known "
                         "size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; runs on several GPUs are not supported", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1004_5076_amd as pk
    import synth

    dev = torch.device("cuda", 0)
    w = synth.workload_two_channel(edge=args.edge)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ctx = pk.context_for(w, device=0, product=pk.SCABS_PRODUCT_TOEPLITZ)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = ctx.info()
    log("setup", f"{setup_s:.2f}s", info)
    # the library's autotuner picks the product's launch choices on this
    # context (part of the setup, outside the timed region)
    t1 = time.perf_counter()
    tune = ctx.autotune(reps=3)
    tune_s = time.perf_counter() - t1
    tune_chosen = {str(r["nrhs"]): {k: r[k] for k in ("apply_form", "groups", "lines", "overlap", "us")}
                   for r in tune if r["chosen"]}
    log("autotune", f"{tune_s:.2f}s", tune_chosen)
    N = ctx.N
    d0 = w.dipoles[0]

    if args.products_only:
        # the roofline kernels alone, for counter runs: batched FP32 products,
        # single-vector transposed FP32 products and one GMRES step of the
        # batch (one FP32 Schwarz apply to 8 vectors)
        X = torch.from_numpy(np.stack([synth.random_complex(3 + k, N) for k in range(BATCH)])).to(dev)
        b = ctx.rhs_dipole(d0.pos, d0.moment, d0.body)
        bb = torch.stack([b] * BATCH).contiguous()
        ctx.matvec(X, prec=pk.SCABS_FP32)
        torch.cuda.synchronize()
        ctx.profile_begin()
        for _ in range(args.products_only):
            ctx.matvec(X, prec=pk.SCABS_FP32)
        for _ in range(args.products_only):
            ctx.matvec(X[0], prec=pk.SCABS_FP32, transpose=True)
        for _ in range(args.products_only):
            ctx.solve(bb, tol=0.5, max_iter=1, restart=1, mode=pk.SCABS_MIXED)
        prof = ctx.profile_end()
        a = torch.ones(1 << 26, dtype=torch.float32, device=dev)   # 2^28 bytes read, 2^28 written
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"products": args.products_only, "N": N, "copy_bytes": 1 << 28, "info": info,
                          "stages": {k: prof[k] for k in ROOFLINE_KERNELS},
                          "kernels": {k: v[0] for k, v in ROOFLINE_KERNELS.items()},
                          "kernel_src_sha": {k: kernel_src_sha(v[1]) for k, v in ROOFLINE_KERNELS.items()}}))
        ctx.close()
        return

    # seeded dipoles in channel 0 within its first wavelength; monitor points on its axis
    dips = [d0] + [synth.seeded_dipole(600 + k, base=(0.5, float(d0.pos[1]), 0.0), body=d0.body)
                   for k in range(BATCH - 1)]
    B = torch.stack([ctx.rhs_dipole(d.pos, d.moment, d.body) for d in dips]).contiguous()
    xs_m = np.linspace(6.0, 24.0, 16)
    pts = np.stack([xs_m, np.full_like(xs_m, float(d0.pos[1])), np.zeros_like(xs_m)], 1)
    beta = 0.9 * w.omega * math.sqrt(w.eps_in)
    fit = np.stack([np.exp(-1j * beta * xs_m), np.exp(1j * beta * xs_m)], axis=1)
    wE = np.zeros((len(xs_m), 3), complex)
    wE[:, 1] = np.linalg.pinv(fit)[1]
    wE_t = torch.from_numpy(wE).to(dev)
    Einc_y = ctx.dipole_field(d0.pos, d0.moment, d0.body, pts, int(d0.body))[0][:, 1].contiguous()
    einc = ctx.incident_dipole_points(d0.pos, d0.moment, d0.body)
    region = int(d0.body)

    def step():
        X, infos = ctx.solve(B, tol=args.tol, restart=args.restart, mode=pk.SCABS_MIXED, max_iter=6000)
        x0 = X[0].contiguous()
        E, _ = ctx.eval_field(x0, pts, region)
        bh = (wE_t[:, 1] * (Einc_y + E[:, 1])).sum()
        q = ctx.eval_field_transpose(pts, region, wE_t)
        g = (torch.conj(bh) * q).contiguous()
        lam, ia = ctx.solve(g, tol=args.tol, restart=args.restart, mode=pk.SCABS_MIXED, max_iter=6000,
                            transpose=True)
        _, dpar = ctx.sigma_gradient(x0, lam, einc)
        return infos, ia, dpar

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    full = None
    if not args.no_breakdown:
        # one untimed step with every stage recorded: the per-stage breakdown
        # and the choice of the roofline kernel (largest total among
        # ROOFLINE_KERNELS)
        ctx.profile_mask(None)
        ctx.profile_begin()
        step()
        full = ctx.profile_end()
        log("stages avg us (profiled step)",
            {k: (v["ms"] / v["count"] * 1e3 if v["count"] else 0.0) for k, v in full.items()})
        top = max(ROOFLINE_KERNELS, key=lambda k: full[k]["ms"])
        timed_stages = [top, "toeproduct32"]
    else:
        timed_stages = list(ROOFLINE_KERNELS) + ["toeproduct32"]
    # timed steps: only the roofline kernel's stage and the whole FP32
    # product record events (two per launch; events around every stage would
    # add ~75 ms per step)
    ctx.profile_mask(timed_stages)
    torch.cuda.synchronize()
    ctx.profile_begin()
    all_infos, adj_infos = [], []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        infos, ia, dpar = step()
        all_infos += infos
        adj_infos.append(ia)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    prof = ctx.profile_end()
    ctx.profile_mask(None)
    if full is None:
        top = max(ROOFLINE_KERNELS, key=lambda k: prof[k]["ms"])
        full = prof
    stage_avg_us = {k: (v["ms"] / v["count"] * 1e3 if v["count"] else 0.0) for k, v in full.items()}
    stage_total_ms = {k: v["ms"] for k, v in full.items()}
    nprod = sum(i["matvecs32"] + i["matvecs64"] for i in all_infos + adj_infos)
    ok = all(i["status"] == 0 for i in all_infos + adj_infos)
    log("batched solves", all_infos[:BATCH], "adjoint", adj_infos[0], "gradient", list(dpar),
        f"{dt / args.steps:.3f}s per step")

    extras = {}
    if not args.no_extras:
        b0 = B[0].clone()
        xsol = {}
        for mode, name in ((pk.SCABS_MIXED, "mixed"), (pk.SCABS_FP64, "fp64")):
            ctx.solve(b0, tol=args.tol, restart=args.restart, mode=mode, max_iter=6000)   # warm
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            x1, si = ctx.solve(b0, tol=args.tol, restart=args.restart, mode=mode, max_iter=6000)
            torch.cuda.synchronize()
            extras[f"solve_single_{name}"] = {"seconds": time.perf_counter() - t2, **si}
            xsol[name] = x1
        extras["mixed_vs_fp64_rel_diff"] = (torch.linalg.norm(xsol["mixed"] - xsol["fp64"]) /
                                            torch.linalg.norm(xsol["fp64"])).item()
        x8 = torch.from_numpy(np.stack([synth.random_complex(3 + k, N) for k in range(BATCH)])).to(dev)
        rates = {}
        for prec, name in ((pk.SCABS_FP32, "fp32"), (pk.SCABS_FP64, "fp64")):
            for nb in (1, BATCH):
                xb = x8[:nb].contiguous()
                for _ in range(2):
                    ctx.matvec(xb, prec=prec)
                torch.cuda.synchronize()
                n = 10
                t3 = time.perf_counter()
                for _ in range(n):
                    ctx.matvec(xb, prec=prec)
                torch.cuda.synchronize()
                rates[f"{name}_x{nb}"] = n * nb / (time.perf_counter() - t3)
        extras["product_rates_per_s"] = rates
        log("extras", extras)

    # rooflines of the kernels with the largest shares of the step (the FP32
    # per-frequency block products, forward and transposed, the FP32 Schwarz
    # apply): "roofline" is the one with the
    # largest total, measured over the timed steps; "rooflines" all of them
    # from the profiled step
    roofs = {k: roofline(full, k) for k in ROOFLINE_KERNELS}
    single_m = extras.get("solve_single_mixed", {}).get("seconds")
    single_d = extras.get("solve_single_fp64", {}).get("seconds")
    out = {
        "metric": "PMCHW matvecs/s + solve time @1e-6 resid, N~100k: mixed/batched vs FP64, 1 GPU",
        "value": nprod / dt,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 products and inner Krylov basis / f64 sums, rotations, refinement",
        "data": "synthetic",
        "config": {"workload": "two_channel_30x0.4x0.2_quartic_absorbers_edge%.3g" % args.edge, "N": N,
                   "product": "block_toeplitz", "rings": info["rings"], "circulant_length": info["circulant_length"],
                   "ring_edges": info["ring_edges"], "nnz_nonperiodic": info["nnz_nonperiodic"],
                   "grid_phys": info["grid_phys"], "grid_fft": info["grid_fft"], "h": w.h, "r_near": w.r_near,
                   "tol": args.tol, "restart": args.restart, "batch_rhs": BATCH,
                   "step": "batched mixed solve of 8 dipoles + adjoint solve + sigma gradient"},
        "solve_converged": ok,
        "step_s_per_rhs": dt / args.steps / BATCH,
        "solve_single_mixed_s": single_m,
        "solve_single_fp64_s": single_d,
        "mixed_speedup_vs_fp64": (single_d / single_m) if single_m and single_d else None,
        "iters_mixed": all_infos[0]["inner_iters"],
        "adjoint_iters": adj_infos[0]["inner_iters"],
        "extras": extras,
        "setup_s": setup_s,
        "stage_avg_us": stage_avg_us,
        "stage_total_ms": stage_total_ms,
        "roofline": roofline(prof, top),
        "autotune": {"seconds": tune_s, "chosen": tune_chosen, "candidates": len(tune)},
        "rooflines": roofs,
        "product_roofline": product_roofline(prof),
        "rooflines_source": ("the timed steps (roofline kernels only)" if args.no_breakdown
                             else "one untimed step with every stage recorded"),
        "product_roofline_source": "the timed steps",
    }
    def gpu_check(ws, x_lu, b):
        """solution of the same system on the GPU (mixed, to 1e-10), exact
        block-Toeplitz product and lattice product, against the dense LU"""
        res = {}
        for name, prod in (("toeplitz", pk.SCABS_PRODUCT_TOEPLITZ), ("lattice", pk.SCABS_PRODUCT_PFFT)):
            cs = pk.context_for(ws, device=0, product=prod)
            xg, si = cs.solve(torch.from_numpy(b).to(dev), tol=1e-10, restart=200, max_iter=4000,
                              mode=pk.SCABS_MIXED)
            res[name] = float(np.linalg.norm(xg.cpu().numpy() - x_lu) / np.linalg.norm(x_lu))
            cs.close()
        return res

    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(N, gpu_check=gpu_check)
        except Exception as e:  # the baseline is informative only
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
