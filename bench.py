"""Benchmark: precorrected-FFT PMCHW products and mixed-precision solves.

Workload: two parallel 0.4 x 0.2 dielectric channels (eps 12.25 in air),
30 long, quartic surface-conductivity absorbers of length 4 at both ends,
mesh edge 0.072 (N ~ 1e5 unknowns), one seeded dipole in channel 0; lengths in
wavelengths inside the guide.  Synthetic, seeded inputs (synth.py).

One step = one mixed-precision solve of A x = b to relative residual 1e-6
(FP32 products inside GMRES, FP64 orthogonalisation and refinement residual,
right preconditioner), i.e. one pass of every stage of the hot path.
value = operator products per second over the timed steps (the solve's
products, FP32 and FP64).  Also reported: standalone FP32/FP64 product rates,
the FP64-only solve time, the roofline of the dominant kernel measured with
HIP events over the timed region, and the oracle timed on the host.

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


def near_rows_bytes(info: dict, real_bytes: int) -> float:
    """Algorithmic bytes of one near-correction-row launch (the dominant
    kernel): CSR row pointers and columns, four complex exact-minus-grid values
    per entry (eight on absorber rows), per-edge currents and triangle partial
    rows read once, edge records, and the FP64 output rows written."""
    cplx = 2 * real_bytes
    ne, nt, N = info["n_edges"], info["n_tris"], info["N"]
    nnz, nnzr = info["nnz_near"], info["nnz_near_r"]
    return ((ne + 1) * 8 + nnz * 4 + nnz * 4 * cplx + nnzr * 4 * cplx + ne * 3 * cplx + ne * 56
            + nt * 9 * cplx + N * 16)


def kernel_src_sha() -> str:
    p = os.path.join(ROOT, "paper_1004_5076_amd", "csrc", "kernels_matvec.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def measured_traffic(bytes_alg: float):
    """HBM bytes per launch from committed rocprofv3 counter runs, only if they
    were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "near_rows_two_channel_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_src_sha") != kernel_src_sha():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(w_full_N: int, budget_s: float = 20.0) -> dict:
    """The oracle's precorrected-FFT product (numpy FFT + plain C loops) on a
    1-long two-channel section of the same geometry, mesh and grid; scaled
    linearly in N to the benchmark size (the product's cost is ~linear)."""
    import numpy as np
    import oracle
    import synth
    w = synth.workload_two_channel(length=0.6, absorber=0.3, edge=0.072)
    wf = synth.workload_two_channel(edge=0.072)
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    P = o.pfft(wf.h, wf.r_near)
    x = synth.random_complex(77, o.N)
    P.matvec(x)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s or n < 2:
        P.matvec(x)
        n += 1
    dt = (time.perf_counter() - t0) / n
    rate = 1.0 / dt * (o.N / w_full_N)
    return {"value": rate, "unit": "matvecs/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle pFFT product, two-channel 0.6-long section N={o.N}, {n} products "
                      f"({dt * 1e3:.1f} ms each), rate scaled by N_sample/N={o.N}/{w_full_N}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--edge", type=float, default=0.072)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--restart", type=int, default=240)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-solve", action="store_true")
    ap.add_argument("--products-only", type=int, default=0,
                    help="run this many FP32 products, then a device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1004_5076_amd as pk
    import synth

    dev = torch.device("cuda", 0)
    w = synth.workload_two_channel(edge=args.edge)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ctx = pk.context_for(w, device=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = ctx.info()
    log("setup", f"{setup_s:.2f}s", info)
    N = ctx.N
    d = w.dipoles[0]
    b = ctx.rhs_dipole(d.pos, d.moment, d.body)

    if args.products_only:
        x = torch.from_numpy(synth.random_complex(3, N)).to(dev)
        for _ in range(args.products_only):
            ctx.matvec(x, prec=pk.SCABS_FP32)
        torch.cuda.synchronize()
        # calibration copy: 2^28 bytes read and 2^28 bytes written
        a = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"products": args.products_only, "N": N, "copy_bytes": 1 << 28, "info": info,
                          "near_rows_alg_bytes": near_rows_bytes(info, 4), "kernel_src_sha": kernel_src_sha()}))
        ctx.close()
        return

    # standalone product rates
    x = torch.from_numpy(synth.random_complex(3, N)).to(dev)
    rates = {}
    for prec, name in ((pk.SCABS_FP32, "fp32"), (pk.SCABS_FP64, "fp64")):
        for _ in range(3):
            ctx.matvec(x, prec=prec)
        torch.cuda.synchronize()
        n = 30
        t1 = time.perf_counter()
        for _ in range(n):
            ctx.matvec(x, prec=prec)
        torch.cuda.synchronize()
        rates[name] = n / (time.perf_counter() - t1)
    log("product rates /s", rates)

    # warmup solves
    for _ in range(args.warmup):
        ctx.solve(b, tol=args.tol, restart=args.restart, mode=pk.SCABS_MIXED)
    torch.cuda.synchronize()
    # timed steps, stage events recorded on the library stream
    ctx.profile_begin()
    infos = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        xs, si = ctx.solve(b, tol=args.tol, restart=args.restart, mode=pk.SCABS_MIXED)
        infos.append(si)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    prof = ctx.profile_end()
    nprod = sum(i["matvecs32"] + i["matvecs64"] for i in infos)
    ok = all(i["status"] == 0 for i in infos)
    log("mixed solves", infos, f"{dt / args.steps:.4f}s per solve")
    log("stages", prof)

    fp64_solve = None
    if not args.no_fp64_solve:
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x64, si64 = ctx.solve(b, tol=args.tol, restart=args.restart, mode=pk.SCABS_FP64)
        torch.cuda.synchronize()
        fp64_solve = {"seconds": time.perf_counter() - t2, **si64}
        rel = (torch.linalg.norm(xs - x64) / torch.linalg.norm(x64)).item()
        fp64_solve["mixed_vs_fp64_rel_diff"] = rel
        log("fp64 solve", fp64_solve)

    # dominant kernel: near-correction rows of the FP32 product
    near = prof["near32"]
    avg_s = near["ms"] / max(near["count"], 1) * 1e-3
    bytes_alg = near_rows_bytes(info, 4)
    achieved = bytes_alg / avg_s / 1e9 if avg_s > 0 else 0.0
    tr = measured_traffic(bytes_alg)
    stage_avg_us = {k: (v["ms"] / v["count"] * 1e3 if v["count"] else 0.0) for k, v in prof.items()}

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
        "dtype": "c64 products / f64 Krylov",
        "data": "synthetic",
        "config": {"workload": "two_channel_30x0.4x0.2_quartic_absorbers_edge%.3g" % args.edge, "N": N,
                   "grid_phys": info["grid_phys"], "grid_fft": info["grid_fft"], "h": w.h, "r_near": w.r_near,
                   "tol": args.tol, "restart": args.restart},
        "solve_mixed_s": dt / args.steps,
        "solve_mixed_iters": infos[0]["inner_iters"],
        "solve_converged": ok,
        "solve_fp64": fp64_solve,
        "matvec_fp32_per_s": rates["fp32"],
        "matvec_fp64_per_s": rates["fp64"],
        "setup_s": setup_s,
        "stage_avg_us": stage_avg_us,
        "roofline": {"kernel": "near_rows_kernel<float>", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": tr, "bytes_per_launch": bytes_alg, "avg_launch_us": avg_s * 1e6},
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(N)
        except Exception as e:  # the baseline is informative only
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
