#!/usr/bin/env python3
"""Throughput benchmark of the batched semilinear lens solve on one MI355X.

Workload (one "step"): the c3 population -- 256 SIE + external-shear lens
parameter sets drawn from the prior box, per-member source grids of 32..96
nodes per side, scored against the 128x128 c2 mock image with a 15x15 PSF,
curvature regularisation and a 16-lambda L-curve (1e-4..1e2), FP32 bulk
arithmetic with FP64 inner products, chi^2 and L-curve, CG to 1e-7.  One
step is the whole hot path: trace + compaction + right-hand sides, 4096 CG
solves, chi^2/||Hs||^2 and the L-curve corner of every member.

Prints one JSON line (rank 0, N = 1).  value = lens-model evaluations per
second over the timed steps.  Also reported: the unbatched ("plain") rate of
the same library called one member at a time, the persistent kernel's
roofline position measured with HIP events, and the FP64 C oracle timed on
the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lens-model evals/s (128² image, 16-λ L-curve) vs plain; χ² rel err vs FP64"
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
SOLVE_SRC = os.path.join(ROOT, "paper_1101_5803_amd", "csrc", "solve.hip")
LARGE_SRC = os.path.join(ROOT, "paper_1101_5803_amd", "csrc", "large.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_solve_c3_hbm_traffic.txt")
LARGE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "large_shape_hbm_traffic.txt")


def source_hash(text: str | None = None, path: str = SOLVE_SRC) -> str:
    """Hash of the kernel source with // comments and whitespace removed."""
    if text is None:
        with open(path) as f:
            text = f.read()
    code = re.sub(r"//[^\n]*", "", text)
    code = re.sub(r"\s+", "", code)
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE, src=SOLVE_SRC, hash_key="solve_hip_sha256_16",
                     value_key="hbm_bytes_per_launch"):
    """HBM bytes from a committed counter summary (per k_solve launch by default), or None.

    The summary records the hash of the kernel source it was measured on; a
    different source (the kernel changed since) gives None.
    """
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get(hash_key) != source_hash(path=src):
        return None
    try:
        return float(kv[value_key])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c3", "c4"],
                    help="c3 (default, the headline): 256 members on the 128x128 image; c4: 1024 members on the "
                         "200x200 image")
    ap.add_argument("--members", type=int, default=0, help="members (default: 256 for c3, 1024 for c4)")
    ap.add_argument("--plain-members", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-member-per-call comparison")
    ap.add_argument("--cpu-members", type=int, default=0, help="oracle sample size (default: one per host core, "
                                                                "at most 16)")
    ap.add_argument("--no-autotune", action="store_true", help="default kernel variant instead of the autotuned one")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"],
                    help="bulk arithmetic of the timed solve (f32: FP32 with FP64 reductions)")
    ap.add_argument("--psf", default="gauss", choices=["gauss", "sinc-moffat"],
                    help="gauss: the workload's Gaussian PSF (separable: banded blur); sinc-moffat: a non-separable "
                         "PSF of the same size (direct K x K blur)")
    ap.add_argument("--search", action="store_true",
                    help="instead of the throughput line: plain vs surrogate-screened GA on the c5 settings")
    ap.add_argument("--search-seeds", type=int, default=3)
    ap.add_argument("--large", action="store_true",
                    help="instead of the throughput line: the large-scale shape (640x640 image, 512x512 source, "
                         "65x65 PSF, 40 CGLS iterations, blur in Fourier space)")
    ap.add_argument("--ga-loop", action="store_true",
                    help="c4's GA generation loop: population 1024, 50 generations, every offspring fully solved")
    ap.add_argument("--gens", type=int, default=30)
    ap.add_argument("--pop", type=int, default=819)
    ap.add_argument("--fanout", type=int, default=10)
    ap.add_argument("--pretrain", type=int, default=100000, help="surrogate pre-training solves (the c5 training set)")
    ap.add_argument("--select", default="per_parent", choices=["per_parent", "global"])
    ap.add_argument("--clip-quantile", type=float, default=0.1, help="surrogate targets clipped at this quantile")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (a known-size kernel that scales "
                         "hardware byte counters)")
    return ap.parse_args()


def algorithmic_work(info, iters, nsub, ck, elem=4, direct=False):
    """Bytes and flops of the CG phase (the persistent kernels) for one step.

    The unit of work is one member's CG iteration.  Its algorithmic bytes are
    the per-iteration traffic of the matrix-free CG of Sec. 2.2 with the image
    restricted to the M pixels that map onto the source grid (the only pixels
    that enter L, Sec. 2.2), for a member of I nodes and n x n subpixels:
        bytes_it = 16 M n^2      the (u, v) positions of the M n^2 subpixels, FP32, read by L and by L^T
                 + 8 M           one image-space vector written by B and read by B^T
                 + 56 I          CG vectors (s, r, p, q and the H^T H and update passes), FP32
    Also returned: the bytes of this implementation's own table encoding
    (cell index and two FP32 fractions per subpixel plus the packed pixel
    index, read once by L and once by L^T: 2 M (4 + 12 n^2)), and the flops
        flops_it = 2 passes * (4ck+1) FMAs * h*w * 2      (B^T B, banded, in LDS)
                 + 2 * 12 * M n^2                          (L and L^T bilinear)
                 + 23 * I                                  (H^T H stencil and CG updates)
    for a mapped bounding box of h x w pixels.  Preconditioned iterations read
    the same tables and count the same; the sine transforms of their
    preconditioner run in LDS on MFMA and their 8 n^3 flops are not counted.
    With the direct blur (a non-separable PSF) the blur term is
    2 K^2 ((h + 2ck)(w + 2ck) + h w) instead.  elem = 8 (FP64 bulk) doubles
    every FP32 vector and table term.
    """
    n2 = nsub * nsub
    flops = 0.0
    nbytes = 0.0
    tbytes = 0.0
    for m in range(info.shape[0]):
        ns, I, M, r0, r1, c0, c1, st = info[m][:8]
        if st != 0:
            continue
        h, w = r1 - r0 + 1, c1 - c0 + 1
        it = float(iters[m].sum())
        K = 2 * ck + 1
        blur = (2 * K * K * ((h + 2 * ck) * (w + 2 * ck) + h * w)) if direct else (2 * (4 * ck + 1) * h * w * 2)
        flops += it * (blur + 2 * 12 * M * n2 + 23 * I)
        nbytes += it * (16.0 * M * n2 + 8.0 * M + 56.0 * I) * (elem / 4.0)
        tbytes += it * (2 * M * (4 + 12 * n2)) * (elem / 4.0)
    return nbytes, tbytes, flops


def host_cores():
    """Cores this process may use (its affinity set, capped at the box's 16-core share) and lscpu's count."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    lscpu = None
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            if line.startswith("CPU(s):"):
                lscpu = int(line.split(":")[1])
    except Exception:   # lscpu missing: report the affinity count only
        pass
    return min(avail, 16), lscpu


def cpu_baseline(w, z, pop, grids, n_members, gpu):
    """The plain-C FP64 oracle on the host cores, on a bounded sample of the c3 step.

    All cores: the first n_members members (one per OpenMP thread), full
    16-lambda sweep each, CG to 1e-10 (the oracle's own tolerance).  Single
    core: member 0 at CG tol 1e-6 (about the work of the FP32 GPU path).  The
    all-core results also serve as a parity check of the timed GPU run on the
    same members: chi^2 at every lambda, ||H s||^2 from two indices below the
    corner, and the corner solution.
    """
    from oracle import coracle, lcurve
    cores, lscpu = host_cores()
    n = min(n_members, cores) if n_members else cores
    t0 = time.perf_counter()
    ref = coracle.evaluate(pop[:n], grids[:n], w.half_width, w.nx, w.ny, w.pix, w.nsub_model, z["d"],
                           float(z["sigma"]), z["psf"], w.reg, w.lambdas, tol=1e-10, want_s=True, threads=n)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    coracle.evaluate(pop[:1], grids[:1], w.half_width, w.nx, w.ny, w.pix, w.nsub_model, z["d"], float(z["sigma"]),
                     z["psf"], w.reg, w.lambdas, tol=1e-6, threads=1)
    dt1 = time.perf_counter() - t1
    chi2, reg, ks, s, off = gpu
    rel = np.abs(chi2[:n] - ref["chi2"]) / ref["chi2"]
    reg_err, s_err, agree = 0.0, 0.0, 0
    for m in range(n):
        k = int(ks[m])
        agree += int(k == lcurve.corner(ref["reg"][m], ref["chi2"][m])[0])
        lo = max(0, k - 2)
        reg_err = max(reg_err, float(np.max(np.abs(reg[m, lo:] - ref["reg"][m, lo:]) / ref["reg"][m, lo:])))
        sr = ref["s"][m, k, :grids[m] ** 2]
        s_err = max(s_err, float(np.linalg.norm(s[off[m]:off[m + 1]] - sr) / np.linalg.norm(sr)))
    return {"value": n / dt, "unit": "evals/s", "cores": n, "kind": "oracle",
            "sample": f"first {n} of the 256 c3 members, full 16-lambda sweep each, plain-C FP64 matrix-free CG to "
                      f"1e-10, one member per OpenMP thread ({dt:.1f} s wall)",
            "host_cpus_lscpu": lscpu, "host_cpus_available": cores,
            "single_core_tol1e-6": {"value": 1.0 / dt1, "unit": "evals/s", "cores": 1,
                                    "sample": f"member 0, full 16-lambda sweep, CG to 1e-6 ({dt1:.1f} s)"},
            "gpu_fp32_vs_oracle_on_sample": {"members": n, "chi2_rel_max": float(rel.max()),
                                             "reg_rel_max_from_kstar_minus_2": reg_err,
                                             "s_corner_rel_l2_max": s_err, "corner_index_agree": agree}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the batched solve shards "
              "members across GPUs by design but runs on one GPU here)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1101_5803_amd as sl
    import synthgen

    if args.search:
        return search_main(args, torch, sl, synthgen)
    if args.ga_loop:
        return ga_loop_main(args, torch, sl, synthgen)
    if args.large:
        return large_main(args, torch, sl, synthgen)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "c3":
        w = synthgen.C3
        z = np.load(os.path.join(ROOT, "tests", "data", "c2.npz"))
        M = args.members or 256
        pop = synthgen.population(w.seed, 256)[:M]
        grids = synthgen.member_grids(w.seed, 256)[:M]
        max_ns = 96
        desc = ("c3: 256 SIE+shear lens sets, 128x128 image at 0.05\", 2x2 subpixels, source grids 32..96 nodes per "
                "side over +-1\", 15x15 Gaussian PSF (FWHM 3 px), curvature H, 16 lambdas 1e-4..1e2, CG tol 1e-7")
    else:
        w = synthgen.C4
        z = np.load(os.path.join(ROOT, "tests", "data", "c4.npz"))
        M = args.members or 1024
        pop = synthgen.population(w.seed, M)
        grids = np.full(M, w.ns, dtype=np.int32)
        max_ns = w.ns
        desc = ("c4: 1024 SIE+shear lens sets, 200x200 image at 0.05\", 2x2 subpixels, 100x100 source nodes over "
                "+-1\", 21x21 Gaussian PSF (FWHM 4 px), curvature H, 24 lambdas 1e-4..1e2, CG tol 1e-7")
    f64 = args.dtype == "f64"
    psf = z["psf"]
    if args.psf == "sinc-moffat":
        psf = synthgen.sinc_moffat_psf(w.k_psf)
        desc = desc.replace("Gaussian PSF", "non-separable sinc x elliptical-Moffat PSF (direct blur)")
        desc = desc.replace(" (FWHM 3 px)", "").replace(" (FWHM 4 px)", "")
    if f64:
        desc = desc.replace("CG tol 1e-7", "CG tol 1e-7, FP64 throughout")
    grid = sl.Grid(w.nx, w.ny, w.pix, w.nsub_model)
    solver = sl.Solver(torch.tensor(z["d"], device=dev), float(z["sigma"]), torch.tensor(psf, device=dev),
                       grid, w.half_width, reg=w.reg, dtype=torch.float64 if f64 else torch.float32)
    lens_d = torch.tensor(pop, device=dev)
    ns_d = torch.tensor(grids, device=dev)
    out = solver.alloc_result(M * max_ns * max_ns, M, len(w.lambdas))

    chi2_h = torch.empty((M, len(w.lambdas)), dtype=torch.float64, pin_memory=True)
    k_h = torch.empty(M, dtype=torch.int32, pin_memory=True)

    def step():
        # one evaluation of every member: the solve, and its fitness (chi^2, k*) back on the host
        solver.solve_semilinear(lens_d, ns_d, w.lambdas, tol=w.tol, maxit=4000, max_ns=max_ns, out=out, tuning={})
        chi2_h.copy_(out["chi2"], non_blocking=True)
        k_h.copy_(out["k_star"], non_blocking=True)

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] warmup {args.warmup} step(s) of {M} members", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sl.profile_enable(True)
    print(f"[bench] timing {args.steps} step(s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = sl.profile_solve_ms()
    sl.profile_enable(False)
    value = M * args.steps / dt
    ms_per_step = 1e3 * dt / args.steps
    iters = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    info = solver.member_info(max_ns, M, len(w.lambdas))
    abytes, tbytes, flops = algorithmic_work(info, iters, w.nsub_model, (w.k_psf - 1) // 2, 8 if f64 else 4,
                                             args.psf != "gauss")
    kern_s = kern_ms / max(launches, 1) / 1e3
    tflops = flops / kern_s / 1e12
    gbs = abytes / kern_s / 1e9
    traffic = measured_traffic() if args.workload == "c3" and not f64 and args.psf == "gauss" else None
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": "CG phase: k_split, then the plain and the preconditioned persistent k_solve side by side",
            "kernel_ms": round(kern_s * 1e3, 3), "launches_timed": launches,
            "algorithmic_bytes": abytes,
            "byte_model": "per member CG iteration 16 M n^2 + 8 M + 56 I (M mapped pixels, n^2 subpixels, I nodes)"
                          + (", doubled for FP64" if f64 else ""),
            "table_encoding_bytes": tbytes, "table_encoding_GBps": round(tbytes / kern_s / 1e9, 1),
            "measured_hbm_GBps": round(traffic / kern_s / 1e9, 1) if traffic else None,
            "measured_hbm_frac": round(traffic / kern_s / 1e9 / PEAK_HBM_GBS, 4) if traffic else None,
            "fp32_TFLOPs": round(tflops, 3), "fp32_frac": round(tflops / PEAK_FP32_TFLOPS, 4)}
    if f64:
        roof["fp64_TFLOPs"] = roof.pop("fp32_TFLOPs")
        roof["fp64_frac"] = round(tflops / PEAK_FP64_TFLOPS, 4)
        roof.pop("fp32_frac")
    # the autotuner's table on the same problem, after the timed region (the timed steps run the default
    # variant, the one the committed counter profiles describe)
    tune = None
    if not args.no_autotune:
        os.environ.setdefault("SL_AUTOTUNE_VERBOSE", "1")
        print("[bench] autotune", file=sys.stderr, flush=True)
        tout = solver.alloc_result(M * max_ns * max_ns, M, len(w.lambdas))
        tuned, tms, _ = solver.autotune(lens_d, ns_d, w.lambdas, tol=w.tol, maxit=4000, max_ns=max_ns, out=tout)
        tune = {"best": tuned, "ms_per_variant": [round(t, 2) for t in tms],
                "best_vs_default": round(min(t for t in tms if t > 0) / tms[0], 4) if tms[0] > 0 else None}
        del tout
    # the same step replayed from a captured HIP graph
    plan = solver.plan(lens_d, ns_d, w.lambdas, tol=w.tol, maxit=4000, max_ns=max_ns, out=out, tuning={})
    plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    plan.close()
    prec = None if f64 or args.psf != "gauss" else precision_vs_f64(sl, torch, z, grid, w, dev, pop, grids, out,
                                                                     max_ns)
    mc = mc_dof_step(sl, torch, solver, lens_d, ns_d, w, max_ns, M, args.steps)
    imp = implicit_step(torch, solver, lens_d, ns_d, max_ns, M, args.steps)
    ref = refine_step(torch, solver, z, w, args.steps)
    big = large_step(torch, sl, synthgen, dev, args.steps)
    # plain: the same library, one member per call
    plain_value = None
    kpo = None
    if not args.no_plain:
        plain_value = run_plain(args, sl, torch, z, grid, w, dev, lens_d, ns_d, max_ns)
        if args.workload == "c3" and not f64:
            kv, kfit = run_plain_kpo(sl, torch, z, grid, w, dev, lens_d, ns_d)
            kc = out["chi2"].cpu().numpy()
            ks = out["k_star"].cpu().numpy()
            kref = np.array([kc[m, ks[m]] for m in range(len(kfit))])
            kpo = {"value": round(kv, 3), "unit": "evals/s", "members": len(kfit),
                   "vs_batched": round(value / kv, 1),
                   "corner_chi2_rel_diff_max": float(np.max(np.abs(np.array(kfit) - kref) / kref))}
    rec = {
        "metric": METRIC, "value": round(value, 2), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": desc,
                   "members": M, "n_lambda": len(w.lambdas), "reductions": "f64", "kernel_variant": "default",
                   "cg_iterations": int(iters.sum()),
                   "status_counts": {int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))}},
        "plain_value": round(plain_value, 3) if plain_value else None,
        "vs_plain": round(value / plain_value, 2) if plain_value else None,
        "plain_kernel_per_operator": kpo,
        "graph_ms_per_step": round(graph_ms, 3),
        "chi2_rel_err_vs_f64": prec,
        "autotune": tune,
        "mc_dof": mc,
        "implicit": imp,
        "refine": ref,
        "large_scale": big,
        "roofline": roof,
    }
    if not args.no_cpu_baseline and args.workload == "c3" and not f64 and args.psf == "gauss":
        print(f"[bench] cpu baseline: oracle on the host cores", file=sys.stderr, flush=True)
        gpu = (out["chi2"].cpu().numpy(), out["reg"].cpu().numpy(), out["k_star"].cpu().numpy(),
               out["s_corner"].cpu().numpy(), out["s_off"].cpu().numpy())
        rec["cpu_baseline"] = cpu_baseline(w, z, pop, grids, args.cpu_members, gpu)
    print(json.dumps(rec), flush=True)


def large_bytes_per_iteration(w, entries, elem=4, tiled=True):
    """Algorithmic HBM bytes of one CGLS iteration of the large solve (sl_solve_large):
    every array read or written once by each kernel that touches it.

    Common to both blur forms: the subpixel table read by the gather L p (cell
    int32 and two fractions per subpixel: (4 + 2 elem) J n^2) with one read of
    p (elem I); L^T over the node-major table (entries x (4 + elem)), its row
    starts (4 I), one read of w (elem J) and g written (elem I); the update
    reading s, p, g and writing s, p and the kept iterate (6 elem I).

    tiled (FP32 with a PSF of at most 65 x 65, overlap-save tiles): y = L p
    written and read, q written, the residual and q read and the new residual
    and w written by the B^T tiles (7 elem J), plus the tile's PSF spectrum
    (65 x 96 complex) read by both blur launches.

    frame (the 1024 x 1024 frame FFT): the half spectra of the ny image rows
    (ny Nh complex values each) written by the row FFT of L p, read and
    written by its column pass, read by the inverse rows that write q's
    spectra, then the residual's spectra and q's read and the residual's and
    the column output written by the B^T column pass, which the last inverse
    rows read: ten such arrays, plus the PSF spectrum (Nh Ny) read twice, and
    w written (elem J).
    """
    J, I, n2 = w.nx * w.ny, w.ns * w.ns, w.nsub_model ** 2
    common = (4 + 2 * elem) * J * n2 + elem * I + entries * (4 + elem) + 4 * I + elem * J + elem * I + 6 * elem * I
    if tiled:
        return common + 7 * elem * J + 2 * 65 * 96 * 2 * elem
    ck = (w.k_psf - 1) // 2
    Nx = 4
    while Nx < w.nx + ck:
        Nx *= 2
    Ny = 4
    while Ny < w.ny + ck:
        Ny *= 2
    Nh = Nx // 2 + 1
    spectra = 10 * w.ny * Nh * 2 * elem + 2 * Nh * Ny * 2 * elem
    return common - elem * I + spectra + J * elem


def _large_setup(torch, sl, synthgen, dev):
    w = synthgen.LARGE
    z = np.load(os.path.join(ROOT, "tests", "data", "large.npz"))
    solver = sl.Solver(torch.tensor(z["d"].astype(np.float64), device=dev), float(z["sigma"]),
                       torch.tensor(z["psf"], device=dev), sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width,
                       reg=w.reg, dtype=torch.float32)
    lens = torch.tensor(z["lens"], device=dev)
    return w, z, solver, lens


def _time_large(torch, solver, lens, ns, n_iter, reps):
    """ms per call of sl_solve_large, HIP events on the stream it runs on (torch's current stream)."""
    out = solver.solve_large(lens, ns, n_iter)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        solver.solve_large(lens, ns, n_iter, out=out)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps, out


def large_step(torch, sl, synthgen, dev, steps):
    """GPU-only summary of the large-scale shape for the throughput line: ms per solve (trace, table, 40 CGLS
    iterations, corner) and per CGLS iteration (the 40-iteration call minus the 1-iteration call, over 39)."""
    print("[bench] large-scale shape (640^2 image, 512^2 source, 65^2 PSF)", file=sys.stderr, flush=True)
    w, z, solver, lens = _large_setup(torch, sl, synthgen, dev)
    reps = max(3, steps)
    ms40, out = _time_large(torch, solver, lens, w.ns, synthgen.LARGE_ITERS, reps)
    ms1, _ = _time_large(torch, solver, lens, w.ns, 1, reps)
    it_ms = (ms40 - ms1) / (synthgen.LARGE_ITERS - 1)
    k = int(out["k_star"].cpu().numpy()[0])
    chi2 = out["chi2"].cpu().numpy()[0]
    return {"ms_per_solve": round(ms40, 3), "ms_per_cgls_iteration": round(it_ms, 4),
            "setup_ms": round(ms1 - it_ms, 3), "corner_iterate": k + 1, "chi2_corner": float(chi2[k]),
            "chi2_r_corner": float(chi2[k] / (w.nx * w.ny))}


def large_main(args, torch, sl, synthgen):
    """The large-scale shape as its own JSON line: solves per second, the roofline of one CGLS iteration, and
    the oracle (FP64, blur in Fourier space) timed on the host for the same solve."""
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w, z, solver, lens = _large_setup(torch, sl, synthgen, dev)
    n_iter = synthgen.LARGE_ITERS
    if args.copy_calibration:   # a device copy of known size, for the counter calibration of a profiled run
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] large: warmup {args.warmup}, timing {args.steps} solve(s)", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        solver.solve_large(lens, w.ns, n_iter)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = solver.solve_large(lens, w.ns, n_iter)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms40, out = _time_large(torch, solver, lens, w.ns, n_iter, max(3, args.steps))
    ms1, _ = _time_large(torch, solver, lens, w.ns, 1, max(3, args.steps))
    it_ms = (ms40 - ms1) / (n_iter - 1)
    # the same solve replayed from a captured HIP graph (launch overheads out of the loop)
    gout = solver.alloc_result(w.ns * w.ns, 1, n_iter)
    solver.solve_large(lens, w.ns, n_iter, out=gout)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        solver.solve_large(lens, w.ns, n_iter, out=gout)
    graph.replay()
    torch.cuda.synchronize()
    ga, gb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ga.record()
    for _ in range(max(3, args.steps)):
        graph.replay()
    gb.record()
    torch.cuda.synchronize()
    graph_ms = ga.elapsed_time(gb) / max(3, args.steps)
    graph_same = bool(torch.equal(gout["chi2"], out["chi2"]) and torch.equal(gout["s_corner"], out["s_corner"]))
    del graph
    # the same solve in FP64 throughout: its time, and how far the FP32 corner chi^2 lies from it
    s64 = sl.Solver(torch.tensor(z["d"].astype(np.float64), device=dev), float(z["sigma"]),
                    torch.tensor(z["psf"], device=dev), sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width,
                    reg=w.reg, dtype=torch.float64)
    ms64, out64 = _time_large(torch, s64, lens, w.ns, n_iter, max(3, args.steps))
    c32, c64 = out["chi2"].cpu().numpy()[0], out64["chi2"].cpu().numpy()[0]
    k32, k64 = int(out["k_star"].cpu().numpy()[0]), int(out64["k_star"].cpu().numpy()[0])
    fp64 = {"ms_per_solve": round(ms64, 3), "corner_iterate": k64 + 1,
            "chi2_rel_diff_fp32_vs_fp64_per_iterate_max": float(np.max(np.abs(c32 - c64) / c64)),
            "chi2_rel_diff_first_10_iterates_max": float(np.max(np.abs(c32[:10] - c64[:10]) / c64[:10]))}
    del s64, out64
    # L^T table entries: the distinct nodes among the four bilinear taps of a pixel's subpixels, per pixel
    # (the library merges a pixel's terms for one node), from the library's own trace
    uv = sl.lens_trace(lens.reshape(1, 7), sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), [w.ns], w.half_width)
    uv = uv.reshape(w.nx * w.ny, w.nsub_model ** 2, 2)
    ok = torch.isfinite(uv[..., 0])
    c0 = torch.clamp(torch.nan_to_num(uv[..., 0]).floor().long(), max=w.ns - 2)
    r0 = torch.clamp(torch.nan_to_num(uv[..., 1]).floor().long(), max=w.ns - 2)
    nodes = torch.stack([(r0 + dr) * w.ns + c0 + dc for dr in (0, 1) for dc in (0, 1)], dim=-1)
    nodes = torch.where(ok[..., None], nodes, torch.full_like(nodes, -1)).reshape(w.nx * w.ny, -1)
    nodes, _ = torch.sort(nodes, dim=1)
    first = torch.ones_like(nodes, dtype=torch.bool)
    first[:, 1:] = nodes[:, 1:] != nodes[:, :-1]
    entries = int((first & (nodes >= 0)).sum().item())
    del uv, nodes, first
    res = {k: v.cpu().numpy() for k, v in out.items()}
    rec_cpu = None
    if not args.no_cpu_baseline:
        print("[bench] large: oracle on the host", file=sys.stderr, flush=True)
        from oracle import implicit, solve
        c0 = time.perf_counter()
        pb = solve.Problem(z["lens"], z["d"].astype(np.float64), float(z["sigma"]), z["psf"], w.nx, w.ny, w.pix,
                           w.nsub_model, w.ns, w.half_width, w.reg, blur="fft")
        ref = implicit.cgls_iterates(pb, n_iter)
        cpu_s = time.perf_counter() - c0
        k = int(res["k_star"][0])
        rec_cpu = {"value": round(1.0 / cpu_s, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
                   "sample": f"one full solve ({n_iter} CGLS iterations, FP64, numpy FFT blur) on one host core",
                   "chi2_rel_diff_at_gpu_corner": float(abs(res["chi2"][0][k] - ref["chi2"][k]) / ref["chi2"][k])}
    abytes = large_bytes_per_iteration(w, entries)
    gbs = abytes / (it_ms * 1e-3) / 1e9
    traffic = measured_traffic(LARGE_TRAFFIC_FILE, LARGE_SRC, "large_hip_sha256_16", "hbm_bytes_per_iteration")
    rec = {"metric": "large-scale CGLS solves/s (640² image, 512² source, 65² PSF, 40 iterations)",
           "value": round(args.steps / dt, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "large-scale shape of Sec. 4: 640x640 image at 0.008\", 2x2 subpixels, "
                                  "512x512 nodes over +-1.6\", 65x65 sinc-Moffat PSF, identity H, 40 CGLS "
                                  "iterations, blur in Fourier space (overlap-save 96x128 tiles)"},
           "ms_per_solve_events": round(ms40, 3), "ms_per_cgls_iteration": round(it_ms, 4),
           "graph_ms_per_solve": round(graph_ms, 3), "graph_matches_eager": graph_same,
           "setup_ms": round(ms1 - it_ms, 3),
           "corner_iterate": int(res["k_star"][0]) + 1,
           "fp64": fp64,
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
                        "measured_hbm_GBps": round(traffic / (it_ms * 1e-3) / 1e9, 1) if traffic else None,
                        "kernel": "one CGLS iteration: 5 kernels (L p; tile blur q = B y with |q|^2; tile blur "
                                  "with the residual update, |e|^2 and w = B^T e; L^T; update)",
                        "algorithmic_bytes": abytes, "table_entries": entries},
           "cpu_baseline": rec_cpu}
    print(json.dumps(rec), flush=True)


def refine_step(torch, solver, z, w, steps, P=1024):
    """The source-refinement fitness (Sec. 3.2): image chi^2 of P candidate sources for the true lens on a
    64 x 64 grid (c2's), one sl_chi2_sources call per generation; candidates per second."""
    print("[bench] source-refinement chi^2", file=sys.stderr, flush=True)
    ns = 64
    rng = np.random.default_rng(12)
    S = torch.tensor(rng.uniform(0.0, 1.0, (P, ns * ns)), device=solver.device)
    out = torch.empty(P, dtype=torch.float64, device=solver.device)
    solver.chi2_sources(z["lens"], ns, S, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.chi2_sources(z["lens"], ns, S, out=out)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    return {"candidates": P, "ns": ns, "ms_per_generation": round(ms, 3), "candidates_per_s": round(P / ms * 1e3, 1)}


def implicit_step(torch, solver, lens_d, ns_d, max_ns, M, steps, n_iter=40):
    """The paper's own fitness (Sec. 2.4, 2.6): 40 unregularised CG iterations per member and the L-curve over
    the iterates, on the same members; time per step and the corner iterates."""
    print("[bench] implicit regularisation (40 iterations)", file=sys.stderr, flush=True)
    out = solver.alloc_result(M * max_ns * max_ns, M, n_iter)
    solver.solve_implicit(lens_d, ns_d, n_iter, max_ns=max_ns, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.solve_implicit(lens_d, ns_d, n_iter, max_ns=max_ns, out=out)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    k = out["k_star"].cpu().numpy()
    return {"n_iter": n_iter, "ms_per_step": round(ms, 3), "evals_per_s": round(M / ms * 1e3, 2),
            "corner_iterate_median": float(np.median(k + 1))}


def mc_dof_step(sl, torch, solver, lens_d, ns_d, w, max_ns, M, steps):
    """The same step with the Monte Carlo degrees of freedom at every corner (Sec. 2.5).

    Returns its time per step and the reduced chi^2 = chi^2(k*) / dof over the
    members (one seeded Gaussian draw bhat for the whole batch).
    """
    import synthgen
    print("[bench] Monte Carlo degrees of freedom", file=sys.stderr, flush=True)
    noise = torch.tensor(synthgen.mc_draws(w.seed, w.ny, w.nx).reshape(-1), device=lens_d.device)
    out = solver.alloc_result(M * max_ns * max_ns, M, len(w.lambdas))
    solver.solve_semilinear(lens_d, ns_d, w.lambdas, tol=w.tol, maxit=4000, max_ns=max_ns, out=out, mc_noise=noise,
                            tuning={})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.solve_semilinear(lens_d, ns_d, w.lambdas, tol=w.tol, maxit=4000, max_ns=max_ns, out=out,
                                mc_noise=noise, tuning={})
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    dof = out["dof"].cpu().numpy()
    k = out["k_star"].cpu().numpy()
    chi2 = out["chi2"].cpu().numpy()[np.arange(M), k]
    ok = np.isfinite(dof) & (dof > 0)
    chi2r = chi2[ok] / dof[ok]
    return {"ms_per_step": round(ms, 3), "evals_per_s": round(M / ms * 1e3, 2), "members": int(ok.sum()),
            "dof_median": float(np.median(dof[ok])), "chi2_r_min": float(chi2r.min()),
            "chi2_r_median": float(np.median(chi2r))}


def precision_vs_f64(sl, torch, z, grid, w, dev, pop, grids, out, max_ns, n=16):
    """chi^2 of the FP32 path (the timed run's results) against the FP64 path at tol 1e-10.

    Members 0, M/n, 2M/n, ... of the batch are re-solved in FP64.
    """
    M = pop.shape[0]
    idx = np.arange(0, M, max(1, M // n))[:n]
    print(f"[bench] precision: {len(idx)} members in FP64", file=sys.stderr, flush=True)
    s64 = sl.Solver(torch.tensor(z["d"], device=dev), float(z["sigma"]), torch.tensor(z["psf"], device=dev), grid,
                    w.half_width, reg=w.reg, dtype=torch.float64)
    o64 = s64.solve_semilinear(torch.tensor(pop[idx], device=dev), torch.tensor(grids[idx], device=dev), w.lambdas,
                               tol=1e-10, maxit=20000, max_ns=max_ns)
    c64 = o64["chi2"].cpu().numpy()
    k64 = o64["k_star"].cpu().numpy()
    c32 = out["chi2"].cpu().numpy()[idx]
    k32 = out["k_star"].cpu().numpy()[idx]
    ok = (o64["status"].cpu().numpy() == 0) & (out["status"].cpu().numpy()[idx] == 0)
    rel = np.abs(c32 - c64) / c64
    rows = np.arange(len(idx))
    corner = np.abs(c32[rows, k32] - c64[rows, k32]) / c64[rows, k32]
    return {"members": int(len(idx)), "per_lambda_max": float(rel[ok].max()),
            "per_lambda_median": float(np.median(rel[ok])), "at_corner_max": float(corner.max()),
            "corner_index_agree": int((k32 == k64).sum())}


def ga_loop_main(args, torch, sl, synthgen, pop=1024, gens=50):
    """c4 at scale: the GA generation loop (Sec. 3.1.1) with population 1024 for 50 generations on the c4 image
    (200^2, 100^2 nodes, 21^2 PSF, 24 lambdas), every offspring scored by the batched solve (corner chi^2).
    Prints one JSON line: wall time, fitness evaluations per second over the whole loop, best chi^2 by generation."""
    from paper_1101_5803_amd import search
    w = synthgen.C4
    z = np.load(os.path.join(ROOT, "tests", "data", "c4.npz"))
    dev = torch.device("cuda:0")
    solver = sl.Solver(torch.tensor(z["d"], device=dev), float(z["sigma"]), torch.tensor(z["psf"], device=dev),
                       sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width, reg=w.reg, dtype=torch.float32)
    box = search.Box(synthgen.PRIOR_LO, synthgen.PRIOR_HI)
    fit = search.SolverFitness(solver, box, w.ns, w.lambdas, tol=w.tol)
    X0 = box.to_unit(synthgen.population(w.seed, pop))
    draws = synthgen.ga_draws(w.seed, pop, gens)
    t0 = time.perf_counter()
    ga = search.GeneticSearch(fit, X0, log=lambda r: print(f"[ga] generation {r['generation']}: best {r['best']:.1f}",
                                                           file=sys.stderr, flush=True))
    for g in range(gens):
        ga.step({k: v[g] for k, v in draws.items()})
    dt = time.perf_counter() - t0
    truth_f = float(fit(box.to_unit(np.atleast_2d(z["lens"])))[0])
    best_u = ga.X[int(np.argmin(ga.fX))]
    # reduced chi^2 at the corner (Sec. 2.5): chi^2 / dof with the Monte Carlo degrees of freedom, which is how
    # the paper compares solutions at the end of a run
    pair = torch.tensor(np.vstack([box.to_phys(best_u[None])[0], z["lens"]]), device=dev)
    noise = torch.tensor(synthgen.mc_draws(w.seed, w.ny, w.nx).reshape(-1), device=dev)
    o = solver.solve_semilinear(pair, torch.full((2,), w.ns, dtype=torch.int32, device=dev), w.lambdas, tol=w.tol,
                                max_ns=w.ns, mc_noise=noise)
    k = o["k_star"].cpu().numpy()
    c2 = o["chi2"].cpu().numpy()[np.arange(2), k]
    dof = o["dof"].cpu().numpy()
    rec = {"experiment": "c4 GA generation loop", "pop": pop, "generations": gens, "full_solves": ga.full_solves,
           "wall_s": round(dt, 2), "evals_per_s": round(ga.full_solves / dt, 1),
           "best_chi2": float(ga.history[-1]), "true_lens_chi2": truth_f,
           "best_lens": box.to_phys(best_u[None])[0].round(4).tolist(), "true_lens": np.asarray(z["lens"]).tolist(),
           "best_dof": float(dof[0]), "true_dof": float(dof[1]), "best_chi2_r": float(c2[0] / dof[0]),
           "true_chi2_r": float(c2[1] / dof[1]),
           "history": [round(h, 1) for h in ga.history]}
    print(json.dumps(rec), flush=True)


def search_main(args, torch, sl, synthgen):
    """c5: plain GA vs surrogate-screened GA, same seeds; counts full solves to reach the plain search's best."""
    from paper_1101_5803_amd import search
    w = synthgen.C5
    z = np.load(os.path.join(ROOT, "tests", "data", "c2.npz"))
    dev = torch.device("cuda:0")
    solver = sl.Solver(torch.tensor(z["d"], device=dev), float(z["sigma"]), torch.tensor(z["psf"], device=dev),
                       sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width, reg=w.reg, dtype=torch.float32)
    box = search.Box(synthgen.PRIOR_LO, synthgen.PRIOR_HI)
    fit = search.SolverFitness(solver, box, w.ns, w.lambdas, tol=w.tol)
    P, G, F = args.pop, args.gens, args.fanout
    # surrogate training set: solves of genomes drawn uniformly in the prior box
    t0 = time.perf_counter()
    U0 = box.to_unit(synthgen.population(w.seed, args.pretrain))
    f0 = np.concatenate([fit(U0[i:i + 4096]) for i in range(0, len(U0), 4096)])
    ok = np.isfinite(f0)
    sur0 = search.Surrogate(dev, seed=w.seed, clip_quantile=args.clip_quantile)
    sur0.train(U0[ok], np.log(f0[ok]), steps=2000, seed=0)
    pre_s = time.perf_counter() - t0
    print(f"[search] pre-training: {args.pretrain} solves + 2000 Adam steps in {pre_s:.1f} s", file=sys.stderr,
          flush=True)
    runs = []
    for seed in range(100, 100 + args.search_seeds):
        X0 = box.to_unit(synthgen.population(seed, P))
        dp = synthgen.ga_draws(seed, P, G)
        ds = synthgen.ga_draws(seed, P * F, G)
        t1 = time.perf_counter()
        plain = search.GeneticSearch(fit, X0)
        for g in range(G):
            plain.step({k: v[g] for k, v in dp.items()})
        t_plain = time.perf_counter() - t1
        sur = search.Surrogate(dev, seed=w.seed, clip_quantile=args.clip_quantile)
        sur.load_state(sur0.state())
        t1 = time.perf_counter()
        scr = search.ScreenedSearch(fit, X0, sur, fanout=F, train_steps=50, pretrain_steps=0, select=args.select)
        for g in range(G):
            scr.step({k: v[g] for k, v in ds.items()})
        t_scr = time.perf_counter() - t1
        target = plain.history[-1] * 1.01
        hit = [i for i, h in enumerate(scr.history) if h <= target]
        solves_to_target = (hit[0] + 1) * P if hit else None
        runs.append({"seed": seed, "plain_best": plain.history[-1], "screened_best": scr.history[-1],
                     "plain_solves": plain.full_solves, "screened_solves_to_plain_best_1pct": solves_to_target,
                     "plain_s": round(t_plain, 2), "screened_s": round(t_scr, 2),
                     "plain_history": [round(h, 2) for h in plain.history],
                     "screened_history": [round(h, 2) for h in scr.history]})
        print(f"[search] seed {seed}: plain {plain.history[-1]:.1f} screened {scr.history[-1]:.1f} "
              f"solves-to-target {solves_to_target}", file=sys.stderr, flush=True)
    print(json.dumps({"experiment": "c5 screened vs plain GA", "pop": P, "gens": G, "fanout": F,
                      "select": args.select, "clip_quantile": args.clip_quantile,
                      "pretrain_solves": args.pretrain, "pretrain_s": round(pre_s, 1), "runs": runs}), flush=True)


def run_plain(args, sl, torch, z, grid, w, dev, lens_d, ns_d, max_ns):
    """Evals/s of the same library called with one member per call."""
    print(f"[bench] plain: {args.plain_members} members one at a time", file=sys.stderr, flush=True)
    if args.plain_members <= 0:
        args.plain_members = 1
    plain = sl.Solver(torch.tensor(z["d"], device=dev), float(z["sigma"]), torch.tensor(z["psf"], device=dev),
                      grid, w.half_width, reg=w.reg, dtype=torch.float32)
    pout = plain.alloc_result(max_ns * max_ns, 1, len(w.lambdas))
    plain.solve_semilinear(lens_d[:1], ns_d[:1], w.lambdas, tol=w.tol, maxit=4000, max_ns=max_ns, out=pout)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m in range(args.plain_members):
        plain.solve_semilinear(lens_d[m:m + 1], ns_d[m:m + 1], w.lambdas, tol=w.tol, maxit=4000, max_ns=max_ns,
                               out=pout)
    torch.cuda.synchronize()
    return args.plain_members / (time.perf_counter() - t0)


def run_plain_kpo(sl, torch, z, grid, w, dev, lens_d, ns_d, n=3):
    """Evals/s of the plain GPU solve: one member at a time, one kernel per operator (the stand-alone
    sl_lens_trace, sl_apply_L / B / B^T / L^T (scatter) / H^T H launches), CG driven from the host with FP32
    vectors, FP64 inner products and a host-side stop test every iteration, the L-curve corner on the host.
    Returns (evals/s, largest relative chi^2 difference at the corner against the batched solve)."""
    print(f"[bench] plain kernel-per-operator: {n} members", file=sys.stderr, flush=True)
    psf = torch.tensor(z["psf"], device=dev)
    d = torch.tensor(z["d"], device=dev, dtype=torch.float32).reshape(1, -1)
    sigma = float(z["sigma"])

    def normal(uv, ns, p, lam):
        y = sl.apply_L(uv, grid, [ns], p.reshape(1, -1)).reshape(1, grid.ny, grid.nx)
        y = sl.apply_BT(psf, sl.apply_B(psf, y))
        q = sl.apply_LT(uv, grid, [ns], y.reshape(1, -1)).reshape(-1)
        return q + lam * sl.apply_HtH(w.reg, [ns], p.reshape(1, -1)).reshape(-1)

    def one(m):
        ns = int(ns_d[m].item())
        uv = sl.lens_trace(lens_d[m:m + 1], grid, [ns], w.half_width)
        b = sl.apply_LT(uv, grid, [ns], sl.apply_BT(psf, d.reshape(1, grid.ny, grid.nx)).reshape(1, -1)).reshape(-1)
        bb = float(torch.dot(b.double(), b.double()))
        chi2, reg = [], []
        for lam in w.lambdas:
            s = torch.zeros_like(b)
            r = b.clone()
            p = r.clone()
            rr = bb
            for _ in range(4000):
                if rr <= w.tol * w.tol * bb:
                    break
                q = normal(uv, ns, p, lam)
                alpha = rr / float(torch.dot(p.double(), q.double()))
                s += alpha * p
                r -= alpha * q
                rn = float(torch.dot(r.double(), r.double()))
                p = r + (rn / rr) * p
                rr = rn
            res = sl.apply_B(psf, sl.apply_L(uv, grid, [ns], s.reshape(1, -1)).reshape(1, grid.ny, grid.nx))
            res = res.reshape(-1).double() - d.reshape(-1).double()
            chi2.append(float(torch.dot(res, res)) / sigma ** 2)
            reg.append(float(torch.dot(s.double(), sl.apply_HtH(w.reg, [ns], s.reshape(1, -1)).reshape(-1).double())))
        k = sl.lcurve_corner(np.array(reg), np.array(chi2))[0]
        return chi2[k] if k >= 0 else float("nan")

    one(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fits = [one(m) for m in range(n)]
    torch.cuda.synchronize()
    return n / (time.perf_counter() - t0), fits


if __name__ == "__main__":
    main()
