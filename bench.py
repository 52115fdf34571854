#!/usr/bin/env python3
"""Benchmark: filtered subspace iteration on one MI355X.

One step = one iteration of the solver on the 3D Laplacian + potential workload
(n = 100^3, p = 256, Jackson degree 120): the Clenshaw filter (120 fused sparse x
block products), CholQR2 orthonormalisation, Rayleigh-Ritz, residual norms and
the locking test.  Inputs are resident on the GPU before timing starts.

value = algorithmic filter bytes moved per step / wall time per step (GB/s),
i.e. the filter's throughput with the rest of the iteration counted as overhead.
The roofline object reports the steady-state Clenshaw kernel alone, timed with
HIP events on the stream it runs on.  cpu_baseline times the oracle's filter on
a bounded sample of the same workload on the host cores.

Usage: python bench.py [--steps K] [--warmup W] [--form fp64|mixed] [--gpus 1]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# pencil side of the grid ordering (afsi_grid_order): 25 x 25 tiles put the +-x neighbours
# 625 rows away, so the products run each XCD on rows 76 apart (the matrix's median row
# reach / 8) and reuse those rows from its L2; 20-50 measured within 2% of each other
PENCIL = 25
# pencil side for the 96-column slices of the serving path (768-byte rows): 50 x 50 tiles
# (2500 rows apart; runs of 304 rows, a whole number of the grouped kernel's 16-row
# workgroups) gave the grouped step 10.33 ms against 11.03 ms with 25 x 25 and 10.63 ms
# in the natural order
SLICE_PENCIL = 50


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha1():
    """Hash of the Clenshaw kernel sources (ties stored counter data to the kernel it measured)."""
    import hashlib

    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2604_00914_amd", "csrc")
    for f in ("vec_types.h", "clenshaw_kernels.h", "clenshaw_dispatch.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def filter_bytes(nnz, n, p, sx, sval, coeffs, degree):
    """Algorithmic (compulsory) bytes of one filter application and of one steady launch.

    Per product: the CSR matrix once (values, int32 columns, int32 row pointers) plus
    one pass over each dense block it touches: the gathered source once, the block
    b_{j+2} read in place, X when its coefficient is nonzero, and the output write.
    """
    a_bytes = nnz * (sval + 4) + 4 * (n + 1)
    pb = n * p * sx
    total = 0
    for s in range(degree):
        j = degree - 1 - s
        if s == 0:
            passes = 2                                   # read X, write b_{k-1}
        elif s == 1:
            passes = 2 + (1 if coeffs[j] - coeffs[degree] != 0 else 0)
        else:
            passes = 3 + (1 if coeffs[j] != 0 else 0)    # src, V in place, write (+ X)
        total += a_bytes + passes * pb
    steady = a_bytes + 4 * pb
    return total, steady


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--workload", default="lap3d_pot_100")
    ap.add_argument("--size", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--order", choices=["pencil", "natural"], default="pencil",
                    help="row order of a grid workload: the 25 x 25 pencil ordering of afsi_grid_order "
                         "(default) or the natural one")
    ap.add_argument("--no-natural", action="store_true",
                    help="skip the natural-order comparison steps (profiling runs)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run three plain device copies of one block (counter calibration)")
    ap.add_argument("--cpu-baseline-sweep", default=None, metavar="OUT",
                    help="only time the oracle (host cores, all threads and one) on every "
                         "workload plus full converging solves; one JSON line per case into OUT")
    ap.add_argument("--sweep", default=None, metavar="OUT",
                    help="only measure the filter alone on every workload and precision; "
                         "one JSON line per case into OUT")
    ap.add_argument("--slices", default=None, metavar="OUT",
                    help="only measure the slice steps (16 slices x 96 columns of the 100^3 matrix: "
                         "side by side in one block, and each in its own block); one JSON line into OUT")
    ap.add_argument("--sensitivity", default=None, metavar="OUT",
                    help="only run the parameter-sensitivity solves (damping exponent m, "
                         "tau_a, C_r adaptive vs fixed); one JSON line per solve into OUT")
    ap.add_argument("--bandwidth", default=None, metavar="OUT",
                    help="only measure a device copy and a 3-read/1-write pass against the "
                         "working-set size (memory-side cache vs HBM); one JSON line per size")
    ap.add_argument("--irregular", default=None, metavar="OUT",
                    help="only measure the steady product of the irregular n = 2e6 matrix at "
                         "p = 640 FP32; one JSON line into OUT")
    ap.add_argument("--gather-cost", default=None, metavar="OUT",
                    help="only measure the steady product on the 100^3 matrix restricted to "
                         "its diagonal, +-1, +-N and all neighbours; one JSON line per case into OUT")
    args = ap.parse_args()
    if args.cpu_baseline_sweep:
        cpu_sweep(args.cpu_baseline_sweep)   # host only: the oracle on every workload
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_00914_amd import afsi
    from paper_2604_00914_amd import build as hipbuild
    from workloads import build_config, start_block

    if not os.path.exists(afsi.LIB_PATH):
        hipbuild.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.sweep:
        filter_sweep(afsi, torch, dev, args.sweep)
        return
    if args.gather_cost:
        gather_cost(afsi, torch, dev, args.gather_cost)
        return
    if args.sensitivity:
        sensitivity(afsi, torch, dev, args.sensitivity)
        return
    if args.bandwidth:
        bandwidth_sweep(torch, dev, args.bandwidth)
        return
    if args.irregular:
        rec = irregular_record(afsi, torch, dev)
        with open(args.irregular, "w") as fh:
            fh.write(json.dumps(rec) + "\n")
        return
    if args.slices:
        rec = batched_record(afsi, torch, dev)
        log(f"slices: {rec}")
        with open(args.slices, "w") as fh:
            fh.write(json.dumps(rec) + "\n")
        return

    t0 = time.time()
    A, (lmin, lmax), (a, b), cfg = build_config(args.workload, size=args.size, seed=0)
    n, p, k = A.n, cfg.p, cfg.degree
    cplx = A.is_complex
    log(f"workload {cfg.name}: n={n} nnz={A.nnz} p={p} k={k} bounds=({lmin:.4g},{lmax:.4g}) "
        f"interval=({a:.6g},{b:.6g}) gen {time.time() - t0:.1f}s")
    # grid workloads run in the pencil ordering (P A P^T; afsi_grid_order, afsi_csr_permute):
    # same spectrum, start block moved to the same order
    gsize = args.size or cfg.size
    order = args.order if cfg.extra.get("grid") == 3 else "natural"
    perm = None
    A_run = A
    if order == "pencil":
        perm = afsi.afsi_grid_order(gsize, gsize, gsize, PENCIL, PENCIL)
        A_run = afsi.afsi_csr_permute(A, perm)
        log(f"pencil ordering {PENCIL} x {PENCIL}: median row reach {PENCIL * PENCIL}")
    M = afsi.Matrix(A_run, device=0, bounds=(lmin, lmax))
    mh = [M.handle]   # the matrix the timed steps use
    coeffs = afsi.afsi_filter_coefficients(lmin, lmax, a, b, k, cfg.damping)
    X0 = start_block(n, p, seed=0, complex_=cplx)
    f64 = torch.complex128 if cplx else torch.float64
    f32 = torch.complex64 if cplx else torch.float32
    fdt = f64 if args.form == "fp64" else f32
    B0 = torch.from_numpy(X0).to(dev)
    del X0
    B1, B2 = torch.empty_like(B0), torch.empty_like(B0)
    if perm is not None:
        afsi.afsi_permute_rows(B0, perm, B1)
        B0.copy_(B1)
    F0 = torch.empty((n, p), dtype=f32, device=dev)    # filter blocks of the mixed form
    F1, F2 = torch.empty_like(F0), torch.empty_like(F0)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        # a plain device copy of one n x p block: reference for the HBM byte counters
        for _ in range(3):
            B1.copy_(B0)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": B0.numel() * B0.element_size()}), flush=True)
        return
    afsi.afsi_orthonormalize(None, B0, B1)
    torch.cuda.synchronize()

    sx = {torch.float64: 8, torch.float32: 4, torch.complex128: 16, torch.complex64: 8}[fdt]
    sval = sx  # the matrix values are read in the filter's precision
    fbytes, steady_bytes = filter_bytes(A.nnz, n, p, sx, sval, coeffs, k)

    # every product of the filter is bracketed by HIP events on this stream
    steady_ms = []   # products that gather src, read V in place and read X (the dominant kernel)

    cur_form = [args.form]

    def run_filter(deg):
        if cur_form[0] == "fp64":
            ms, kind = afsi.afsi_filter_block_profiled(mh[0], coeffs, deg, B0, B1, B2)
        else:
            afsi.afsi_convert_block(B0, F0)
            ms, kind = afsi.afsi_filter_block_profiled(mh[0], coeffs, deg, F0, F1, F2)
            afsi.afsi_convert_block(F1, B1)
        steady_ms.extend(ms[2:][kind[2:] == 3].tolist())

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    filt_ms = []
    phase_ms = []    # (Cholesky QR fused with Rayleigh-Ritz, residuals) per step
    n_check = [0]

    def step():
        ev[0].record(stream)
        run_filter(k)
        ev[1].record(stream)
        # CholQR2 of the filtered block and Rayleigh-Ritz on its (implicit) basis, as
        # afsi_solve's iteration runs them: V -> B0, AV -> B2
        ritz = afsi.afsi_orthonormalize_rayleigh_ritz(mh[0], B1, B2, B0, B2)
        ev[2].record(stream)
        res = afsi.afsi_residual_norms(B0, B2, ritz)
        ev[3].record(stream)
        inside = (ritz >= a) & (ritz <= b)
        if inside.any():
            normA = max(abs(lmin), abs(lmax))
            _, _, _, n_check[0] = afsi.afsi_lock_select(ritz, res, inside, a, b, 1e-10 * normA, 0, n_check[0])
        filt_ms.append(ev[0].elapsed_time(ev[1]))
        phase_ms.append([ev[i].elapsed_time(ev[i + 1]) for i in (1, 2)])

    for w in range(max(args.warmup, 1)):
        step()
    filt_ms.clear()
    phase_ms.clear()
    steady_ms.clear()
    torch.cuda.synchronize()
    log(f"warmup done; timing {args.steps} steps")
    tstart = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - tstart
    ms_per_step = 1e3 * elapsed / args.steps
    value = fbytes * args.steps / elapsed / 1e9
    filt_med = float(np.median(filt_ms))
    steady_launch_ms = float(np.mean(steady_ms))
    steady_launches = len(steady_ms)
    achieved = steady_bytes / (steady_launch_ms * 1e-3) / 1e9
    filter_gbs = fbytes / (filt_med * 1e-3) / 1e9
    log(f"step {ms_per_step:.2f} ms, filter {filt_med:.2f} ms ({filter_gbs:.0f} GB/s), "
        f"dominant kernel {steady_launch_ms * 1e3:.1f} us avg over {steady_launches} launches ({achieved:.0f} GB/s)")
    orth_rr_ms, res_ms = (float(v) for v in np.median(np.array(phase_ms), axis=0))

    # the same iteration in the other form (FP64 filter vs FP32 / complex-FP32 filter;
    # everything else FP64), same number of steps
    other = "mixed" if args.form == "fp64" else "fp64"
    cur_form[0] = other
    step()
    torch.cuda.synchronize()
    filt_ms.clear()
    phase_ms.clear()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    other_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    osx = {("fp64", False): 8, ("fp64", True): 16, ("mixed", False): 4, ("mixed", True): 8}[(other, cplx)]
    other_fbytes, _ = filter_bytes(A.nnz, n, p, osx, osx, coeffs, k)
    other_rec = {"form": other, "ms_per_step": round(other_ms, 3),
                 "filter_ms": round(float(np.median(filt_ms)), 3),
                 "value": round(other_fbytes / (other_ms * 1e-3) / 1e9, 2),
                 "step_speedup_vs_" + args.form: round(ms_per_step / other_ms, 3)}
    log(f"{other} form: {other_rec}")
    cur_form[0] = args.form
    del F0, F1, F2

    # the same iteration on the matrix in its natural order (the ordering's effect)
    natural_rec = None
    if perm is not None and not args.no_natural:
        Mn = afsi.Matrix(A, device=0, bounds=(lmin, lmax))
        mh[0] = Mn.handle
        step()
        torch.cuda.synchronize()
        steady_ms.clear()
        filt_ms.clear()
        phase_ms.clear()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        nat_step = 1e3 * (time.perf_counter() - t2) / args.steps
        nat_k1 = float(np.mean(steady_ms))
        natural_rec = {"ms_per_step": round(nat_step, 3), "value": round(fbytes / (nat_step * 1e-3) / 1e9, 2),
                       "filter_ms": round(float(np.median(filt_ms)), 3),
                       "dominant_launch_us": round(nat_k1 * 1e3, 2),
                       "dominant_frac": round(steady_bytes / (nat_k1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "pencil_speedup_step": round(nat_step / ms_per_step, 3),
                       "pencil_speedup_dominant": round(nat_k1 / steady_launch_ms, 3)}
        log(f"natural order: {natural_rec}")
        mh[0] = M.handle
        Mn.close()

    # measured copy bandwidth: a plain device copy of one block, same stream, HIP events
    for _ in range(2):
        B2.copy_(B1)
    ev[0].record(stream)
    for _ in range(10):
        B2.copy_(B1)
    ev[1].record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * B1.numel() * B1.element_size() * 10 / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9
    # K1's dense access mix without the gather: read three blocks, write one in place
    # (torch's elementwise addcmul_: B2 <- B2 + B0 * B1)
    for _ in range(2):
        B2.addcmul_(B0, B1)
    ev[0].record(stream)
    for _ in range(10):
        B2.addcmul_(B0, B1)
    ev[1].record(stream)
    torch.cuda.synchronize()
    stream3_gbs = 4 * B1.numel() * B1.element_size() * 10 / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9
    log(f"phases: Cholesky QR + Rayleigh-Ritz {orth_rr_ms:.2f} ms, residuals {res_ms:.2f} ms; "
        f"device copy {copy_gbs:.0f} GB/s; 3-read/1-write pass {stream3_gbs:.0f} GB/s")

    traffic = None
    tpath = os.path.join(ROOT, "profiles", f"traffic_{cfg.name}_{order}_{args.form}.json")
    if os.path.exists(tpath):
        rec = json.load(open(tpath))
        if rec.get("kernel_source_sha1") == kernel_source_sha1():
            traffic = rec.get("hbm_bytes_per_launch")
        else:
            log("stored HBM traffic was taken for other kernel sources: reporting traffic = null")

    out = {
        "metric": "SpMM-filter GB/s (% HBM peak); eigenpairs/s mixed vs FP64; p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "c128" if cplx else "f64", "mixed": "c64" if cplx else "f32"}[args.form],
        "data": "synthetic",
        "config": {
            "workload": cfg.name,
            "description": cfg.description,
            "n": n, "nnz": A.nnz, "p": p, "degree": k, "damping": cfg.damping, "form": args.form,
            "ordering": (f"pencil {PENCIL}x{PENCIL} (afsi_grid_order: P A P^T, same spectrum)"
                         if perm is not None else "natural"),
            "step": f"one solver iteration: filter ({k} products) + CholQR2 fused with Rayleigh-Ritz + residuals",
        },
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "filter_only_gbs": round(filter_gbs, 1),
        "filter_ms": round(filt_med, 3),
        "other_form": other_rec,
        "natural_order": natural_rec,
        "phase_ms": {"filter": round(filt_med, 3), "cholqr_rayleigh_ritz": round(orth_rr_ms, 3),
                     "residuals": round(res_ms, 3)},
        "measured_copy_gbs": round(copy_gbs, 1),
        "measured_3r1w_gbs": round(stream3_gbs, 1),
        "dominant_frac_of_copy": round(achieved / copy_gbs, 4),
        "dominant_frac_of_3r1w": round(achieved / stream3_gbs, 4),
        "roofline": {
            "kernel": "clenshaw_step_staged_kernel<HAS_V=1,HAS_X=1> (gather src, read V in place, read X, write V)",
            "launches": steady_launches,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": steady_bytes,
            "launch_us": round(steady_launch_ms * 1e3, 2),
        },
    }

    if not args.no_solve:
        out["solve"] = solve_rates(afsi, torch, dev)
        out["lanczos"] = lanczos_rates(afsi, torch, dev)
        out["eigencount"] = eigencount_rates(afsi, torch, dev)
        out["irregular"] = irregular_record(afsi, torch, dev)
        out["complex"] = complex_record(afsi, torch, dev)
    if not args.no_serve:
        # the slices of the serving stream run on the matrix in the pencil ordering for
        # 96-column rows (SLICE_PENCIL), as in the slice-step record
        Ms = M
        if perm is not None:
            Ms = afsi.Matrix(afsi.afsi_csr_permute(A, afsi.afsi_grid_order(gsize, gsize, gsize, SLICE_PENCIL,
                                                                           SLICE_PENCIL)),
                             device=0, bounds=(lmin, lmax))
        out["serve"] = serve_rates(afsi, Ms, args.serve_requests)
        out["serve"]["slice_ordering"] = f"pencil {SLICE_PENCIL}x{SLICE_PENCIL}" if perm is not None else "natural"
        if Ms is not M:
            Ms.close()

    out["paper_context"] = paper_context()
    # the same rate for this GPU's steady product (nonzeros x block columns per second)
    out["paper_context"]["this_gpu_steady_product_nnz_per_s"] = float(
        f"{A.nnz * p / (steady_launch_ms * 1e-3):.3g}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, p, k, lmin, lmax, a, b, cfg, sx, args.cpu_sample_steps)
    M.close()
    print(json.dumps(out), flush=True)


SWEEP = [("lap2d_64", "fp64"), ("lap3d_pot_100", "fp64"), ("lap3d_pot_100", "fp32"),
         ("tb3d_64", "fp64"), ("tb3d_64", "fp32"), ("rand_2m", "fp32"), ("rand_2m", "fp64")]


def filter_sweep(afsi, torch, dev, path, reps=3):
    """Filter-only throughput of every workload in both precisions (inputs resident).

    Per case: one warm-up filter, then `reps` filters, each product bracketed by HIP
    events; reports the median filter time, its algorithmic GB/s and the steady
    kernel's average launch time and GB/s.
    """
    from workloads import build_config, start_block

    with open(path, "w") as fh:
        for name, prec in SWEEP:
            t0 = time.time()
            A, (lmin, lmax), (a, b), cfg = build_config(name, seed=0)
            n, p, k = A.n, cfg.p, cfg.degree
            cplx = A.is_complex
            M = afsi.Matrix(A, device=0, bounds=(lmin, lmax))
            coeffs = afsi.afsi_filter_coefficients(lmin, lmax, a, b, k, cfg.damping)
            dt = {("fp64", False): torch.float64, ("fp32", False): torch.float32,
                  ("fp64", True): torch.complex128, ("fp32", True): torch.complex64}[(prec, cplx)]
            X = torch.from_numpy(start_block(n, p, seed=0, complex_=cplx)).to(dev).to(dt)
            Y, W = torch.empty_like(X), torch.empty_like(X)
            sx = X.element_size()
            fbytes, steady_bytes = filter_bytes(A.nnz, n, p, sx, sx, coeffs, k)
            tot, steady = [], []
            for r in range(reps + 1):
                ms, kind = afsi.afsi_filter_block_profiled(M.handle, coeffs, k, X, Y, W)
                if r:
                    tot.append(float(np.sum(ms)))
                    steady.extend(ms[2:][kind[2:] == 3].tolist())
            fmed = float(np.median(tot))
            sms = float(np.mean(steady))
            rec = {"workload": name, "precision": prec, "dtype": str(dt).replace("torch.", ""),
                   "n": n, "nnz": A.nnz, "p": p, "degree": k,
                   "filter_ms": round(fmed, 3), "filter_gbs": round(fbytes / (fmed * 1e-3) / 1e9, 1),
                   "steady_launch_us": round(sms * 1e3, 2),
                   "steady_gbs": round(steady_bytes / (sms * 1e-3) / 1e9, 1),
                   "steady_frac_hbm_peak": round(steady_bytes / (sms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "bytes_per_filter": fbytes, "bytes_per_steady_launch": steady_bytes}
            log(f"sweep {name} {prec}: {rec} (setup {time.time() - t0:.1f}s)")
            fh.write(json.dumps(rec) + "\n")
            fh.flush()
            del X, Y, W
            M.close()
            torch.cuda.empty_cache()
        rec = batched_record(afsi, torch, dev)
        log(f"sweep batched slices: {rec}")
        fh.write(json.dumps(rec) + "\n")


def sensitivity(afsi, torch, dev, path, max_iter=400):
    """Parameter sensitivity of the adaptive solver (the experiments of Section 4.2, on
    synthetic matrices): the damping exponent m in [0, 3] step 0.1 and tau_a in
    [1e-4, 0.5] with k^(1) from eq. (compute_k_1) (C = 1.4) and k = ceil(2.5 k^(1));
    then C_r = C / (alpha - beta) over 13 values in [10, 120], k^(1) = ceil(C_r) - 1,
    for the adaptive filter (k = ceil(2.5 k^(1))) and for the fixed degree k^(1).
    Workloads: lap3d_pot_27 (196 eigenvalues) and lap2d_64 (40), FP64, tau_c = 1e-10.
    Per solve: wall time, iterations, average degree, products with A, the filter's and
    the other phases' time, and whether the count and every eigenvalue are right."""
    from workloads import build_config, start_block

    with open(path, "w") as fh:
        for name in ("lap3d_pot_27", "lap2d_64"):
            A, (lmin, lmax), (a, b), cfg = build_config(name)
            exact = _window_fixture(name)
            normA = max(abs(lmin), abs(lmax))
            M = afsi.Matrix(A, device=0, bounds=(lmin, lmax))
            X0 = start_block(A.n, cfg.p, seed=0)
            k1_paper = paper_initial_degree(lmin, lmax, a, b)

            def run(study, value, k1, kmax, adaptive, m_exp=0.5, tau_a=1e-3):
                o = afsi.afsi_options_default(kmax)
                o.k_init = k1
                o.adaptive = adaptive
                o.damping = afsi.DAMP_LANCZOS
                o.m_exp = m_exp
                o.tau_a = tau_a
                o.max_iter = max_iter
                X = torch.from_numpy(X0).to(dev)
                E = torch.zeros((A.n, cfg.p), dtype=torch.float64, device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, lam, res, r = afsi.afsi_solve(M.handle, a, b, o, X, E, cfg.p)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                ok = bool(st == 0 and lam.size == exact.size and np.max(np.abs(lam - exact)) <= 1e-10 * normA)
                other = r.time_orth_ms + r.time_rr_ms + r.time_resid_ms + r.time_host_ms
                rec = {"workload": name, "study": study, "value": value, "adaptive": adaptive,
                       "k1": k1, "kmax": kmax, "m_exp": m_exp, "tau_a": tau_a, "status": st,
                       "correct": ok, "seconds": round(dt, 4), "iterations": r.iterations,
                       "avg_degree": round(r.avg_degree, 2), "spmv": r.spmv,
                       "filter_ms": round(r.time_filter_ms, 2), "other_ms": round(other, 2)}
                log(f"sensitivity {name} {study}={value} adaptive={adaptive}: {rec}")
                fh.write(json.dumps(rec) + "\n")
                fh.flush()

            kmax_paper = math.ceil(2.5 * k1_paper)
            for i in range(31):
                run("m", round(0.1 * i, 1), k1_paper, kmax_paper, 1, m_exp=0.1 * i)
            for ta in (1e-4, 3e-4, 1e-3, 3e-3, 1e-2, 3e-2, 1e-1, 5e-1):
                run("tau_a", ta, k1_paper, kmax_paper, 1, tau_a=ta)
            for cr in np.linspace(10.0, 120.0, 13):
                k1 = max(1, math.ceil(cr) - 1)
                run("C_r", round(float(cr), 2), k1, math.ceil(2.5 * k1), 1)
                run("C_r", round(float(cr), 2), k1, k1, 0)
            M.close()


def gather_cost(afsi, torch, dev, path, degree=24, reps=3):
    """What the gathers cost the steady product: the FP64 lap3d_pot_100 matrix (p = 256)
    restricted to the entries at column offsets {0}, {0, +-1}, {0, +-1, +-N} and all
    seven, each filtered with the same schedule.  With the diagonal alone the product
    is a pure 3-read/1-write stream in the kernel's own access pattern; the rate lost
    with each pair of neighbours is what gathering those rows costs.  Bytes are the
    compulsory model of each restricted matrix."""
    from workloads import CSR, build_config, start_block

    A, (lmin, lmax), (a, b), cfg = build_config("lap3d_pot_100", seed=0)
    n, p = A.n, cfg.p
    N = round(n ** (1.0 / 3.0))
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))
    off = A.col.astype(np.int64) - rows
    coeffs = afsi.afsi_filter_coefficients(lmin, lmax, a, b, degree, cfg.damping)
    X = torch.from_numpy(start_block(n, p, seed=0)).to(dev)
    Y, W = torch.empty_like(X), torch.empty_like(X)
    cases = [("diagonal", {0}), ("+-1", {0, 1, -1}), ("+-1,+-N", {0, 1, -1, N, -N}),
             ("+-1,+-N,+-N^2", {0, 1, -1, N, -N, N * N, -N * N})]
    with open(path, "w") as fh:
        for name, offs in cases:
            keep = np.isin(off, list(offs))
            counts = np.bincount(rows[keep], minlength=n)
            rp = np.zeros(n + 1, dtype=np.int64)
            np.cumsum(counts, out=rp[1:])
            sub = CSR(n, rp, A.col[keep].copy(), A.val[keep].copy())
            M = afsi.Matrix(sub, device=0, bounds=(lmin, lmax))
            _, steady_bytes = filter_bytes(sub.nnz, n, p, 8, 8, coeffs, degree)
            steady = []
            for r in range(reps + 1):
                ms, kind = afsi.afsi_filter_block_profiled(M.handle, coeffs, degree, X, Y, W)
                if r:
                    steady.extend(ms[2:][kind[2:] == 3].tolist())
            sms = float(np.mean(steady))
            rec = {"workload": "lap3d_pot_100 restricted", "offsets": name, "nnz": sub.nnz, "p": p,
                   "steady_launch_us": round(sms * 1e3, 2), "bytes_per_steady_launch": steady_bytes,
                   "steady_gbs": round(steady_bytes / (sms * 1e-3) / 1e9, 1),
                   "steady_frac_hbm_peak": round(steady_bytes / (sms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            log(f"gather cost {name}: {rec}")
            fh.write(json.dumps(rec) + "\n")
            fh.flush()
            M.close()
    del X, Y, W
    torch.cuda.empty_cache()


def batched_record(afsi, torch, dev, groups=16, cols=96, launches=30):
    """Batched slice filter: 16 spectrum slices x 96 columns of the 100^3 matrix advanced
    by one launch per step (A read once), against the same groups as 16 launches.
    `batched`: every group at the same step, so all read one source block;
    `batched_mixed_sources`: odd groups one step ahead, so the launch mixes two sources;
    `grouped*`: the same slices each in its own contiguous n x 96 blocks, advanced by one
    grouped launch per step (or one launch per slice).

    Every group is in the steady part of its own filter (steps 2..), with its own
    slice coefficients; bytes per launch = A once + per group one pass over each block
    it touches (gathered source, V in place, X when alpha != 0, write)."""
    from workloads import build_config, start_block
    from workloads.stream import slice_intervals

    A, (lo, hi), _, cfg = build_config("lap3d_pot_100", seed=0)
    # in the pencil ordering for 96-column rows (random blocks need no reordering)
    A = afsi.afsi_csr_permute(A, afsi.afsi_grid_order(cfg.size, cfg.size, cfg.size, SLICE_PENCIL,
                                                      SLICE_PENCIL))
    M = afsi.Matrix(A, device=0, bounds=(lo, hi))
    k = cfg.degree
    l1, l2 = 2.0 / (hi - lo), -(hi + lo) / (hi - lo)
    ivs = slice_intervals(A.n, 0.5 * (lo + hi), groups, 50)
    coeffs = [afsi.afsi_filter_coefficients(lo, hi, a, b, k, "jackson") for a, b in ivs]
    ptot = groups * cols
    X = torch.from_numpy(start_block(A.n, ptot, seed=0)).to(dev)
    P0, P1 = torch.zeros_like(X), torch.zeros_like(X)
    a_bytes = A.nnz * 12 + 4 * (A.n + 1)
    col_pass = A.n * cols * 8

    def step_groups(s, stagger=0):
        # stagger = 1: odd groups one step ahead, so neighbouring groups read different
        # source blocks in the same launch
        gs = [afsi.afsi_clenshaw_step_params(coeffs[g], k, s + stagger * (g % 2), l1, l2, g * cols, cols)
              for g in range(groups)]
        for g in gs:
            g.active = 1
        return gs

    def bytes_of(gs, with_a):
        tot = a_bytes if with_a else 0
        for g in gs:
            tot += (2 + int(g.has_v) + int(g.alpha != 0.0)) * col_pass
        return tot

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {"workload": "lap3d_pot_100 slices", "ordering": f"pencil {SLICE_PENCIL}x{SLICE_PENCIL}", "kernel": "clenshaw_batched_kernel", "groups": groups,
           "cols_per_group": cols, "n": A.n, "degree": k, "launches": launches}
    for mode in ("batched", "batched_mixed_sources", "one_launch_per_group"):
        steps = list(range(2, 2 + launches))
        total = 0
        for warm in (True, False):
            ev[0].record()
            for s in steps:
                gs = step_groups(s, 1 if mode == "batched_mixed_sources" else 0)
                if mode != "one_launch_per_group":
                    afsi.afsi_clenshaw_step_batched(M.handle, gs, X, P0, P1)
                    total += bytes_of(gs, True)
                else:
                    for g in gs:
                        afsi.afsi_clenshaw_step_batched(M.handle, [g], X, P0, P1)
                    total += sum(bytes_of([g], True) for g in gs)
            ev[1].record()
            torch.cuda.synchronize()
            if warm:
                total = 0
        ms = ev[0].elapsed_time(ev[1])
        out[mode] = {"ms_per_step": round(ms / launches, 3),
                     "gbs": round(total / (ms * 1e-3) / 1e9, 1)}
    out["batched_speedup"] = round(out["one_launch_per_group"]["ms_per_step"] / out["batched"]["ms_per_step"], 3)
    X0 = X.cpu()
    del X, P0, P1
    torch.cuda.empty_cache()
    # the same slices, each in its own contiguous n x 96 blocks (the serving pool's layout):
    # one grouped launch per step, and one launch per slice
    own = []
    for g in range(groups):
        Xg = X0[:, g * cols:(g + 1) * cols].contiguous().to(dev)
        own.append((Xg, torch.zeros_like(Xg), torch.zeros_like(Xg)))
    del X0
    for mode in ("grouped", "grouped_mixed_sources", "grouped_one_launch_per_slice"):
        steps = list(range(2, 2 + launches))
        total = 0
        for warm in (True, False):
            ev[0].record()
            for s in steps:
                gs = step_groups(s, 1 if mode == "grouped_mixed_sources" else 0)
                sl = [(gs[g], *own[g]) for g in range(groups)]
                if mode != "grouped_one_launch_per_slice":
                    afsi.afsi_clenshaw_step_grouped(M.handle, sl)
                    total += bytes_of(gs, True)
                else:
                    for g in range(groups):
                        afsi.afsi_clenshaw_step_grouped(M.handle, [sl[g]])
                    total += sum(bytes_of([x], True) for x in gs)
            ev[1].record()
            torch.cuda.synchronize()
            if warm:
                total = 0
        ms = ev[0].elapsed_time(ev[1])
        out[mode] = {"ms_per_step": round(ms / launches, 3),
                     "gbs": round(total / (ms * 1e-3) / 1e9, 1)}
    del own
    M.close()
    torch.cuda.empty_cache()
    return out


def _window_fixture(name):
    """Expected eigenvalues of a workload's window from its stored fixture."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_window.txt")
    vals = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        vals.append(float(line.split()[-1]))
    return np.array(vals)


# (label, filter form, tau_c, adaptive paper mode)
SOLVE_MODES = [
    ("fp64", "fp64", 1e-10, False),
    ("fp64_tau1e-6", "fp64", 1e-6, False),
    ("mixed", "mixed", 1e-6, False),
    ("fp64_adaptive", "fp64", 1e-10, True),
    ("fp64_adaptive_tau1e-6", "fp64", 1e-6, True),
    ("mixed_adaptive", "mixed", 1e-6, True),
]


def paper_initial_degree(lmin, lmax, a, b, C=1.4):
    """k^(1) = ceil(C / (alpha - beta)) - 1 of eq. (compute_k_1), alpha = arccos l(a),
    beta = arccos l(b) with l(.) clipped into [-1, 1] (the experiment's parameter, as the
    solver computes it when it is not given)."""
    t = lambda x: min(1.0, max(-1.0, (2 * x - lmax - lmin) / (lmax - lmin)))
    return max(1, math.ceil(C / (math.acos(t(a)) - math.acos(t(b)))) - 1)


def solve_rates(afsi, torch, dev, seeds=(0, 1, 2, 3, 4)):
    """Eigenpairs/s of the full solver on the converging workloads, FP64 vs mixed.

    lap2d_64 (40 eigenvalues, closed form) and lap3d_pot_27 (196 eigenvalues from the
    banded eigensolver), each from its stored fixture.  Modes: fixed Jackson degree (the
    workload's) and the paper's adaptive mode (Section 4: Lanczos damping m = 0.5,
    tau_a = 1e-3, k^(1) from eq. (compute_k_1) with C = 1.4, maximum degree
    k = ceil(2.5 k^(1)), Algorithm 3 after every iteration); FP64 at
    tau_c = 1e-10 (full accuracy) and at tau_c = 1e-6 (the mixed form's accuracy, for an
    equal-accuracy comparison).  A run counts its eigenpairs only if the count is exact
    and every eigenvalue is within 1e-10 ||A|| (tau_c 1e-10) or 1e-5 ||A|| (tau_c 1e-6).
    Wall time runs from the resident start block to results on the host.  As in the
    paper's experiments (Section 4), every mode runs once per start-block seed 0..4 and
    the averages are reported (after one untimed solve per workload).
    """
    from workloads import build_config, start_block

    out = {}
    for name in ("lap2d_64", "lap3d_pot_27"):
        A, (lmin, lmax), (a, b), cfg = build_config(name)
        exact = _window_fixture(name)
        normA = max(abs(lmin), abs(lmax))
        M = afsi.Matrix(A, device=0, bounds=(lmin, lmax))
        X0s = {sd: start_block(A.n, cfg.p, seed=sd) for sd in seeds}
        rec_w = {"n": A.n, "p": cfg.p, "degree": cfg.degree, "eigenvalues": int(exact.size),
                 "seeds": list(seeds)}
        k1 = paper_initial_degree(lmin, lmax, a, b)
        rec_w["adaptive_k1_kmax"] = [k1, math.ceil(2.5 * k1)]

        def solve(o, X0):
            X = torch.from_numpy(X0).to(dev)
            E = torch.zeros((A.n, cfg.p), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, lam, res, r = afsi.afsi_solve(M.handle, a, b, o, X, E, cfg.p)
            torch.cuda.synchronize()
            return st, lam, res, r, time.perf_counter() - t0

        for label, form, tau_c, adaptive in SOLVE_MODES:
            o = afsi.afsi_options_default(math.ceil(2.5 * k1) if adaptive else cfg.degree)
            o.max_iter = 1500
            o.tau_c = tau_c
            if form == "mixed":
                o.filter_dtype = afsi.R32
            if adaptive:
                o.adaptive = 1
                o.damping = afsi.DAMP_LANCZOS
            if label == SOLVE_MODES[0][0]:
                solve(o, X0s[seeds[0]])  # untimed: first-use allocations
            tol = (1e-10 if tau_c <= 1e-10 else 1e-5) * normA
            runs = []
            for sd in seeds:
                st, lam, res, r, dt = solve(o, X0s[sd])
                err = float(np.max(np.abs(lam - exact))) if lam.size == exact.size else None
                good = int(lam.size) if (st == 0 and err is not None and err <= tol) else 0
                runs.append({"seed": sd, "seconds": round(dt, 4), "eigenpairs": good,
                             "iterations": r.iterations, "eigenpairs_per_s": round(good / dt, 2),
                             "max_abs_eig_err": err,
                             "max_residual": float(np.max(res)) if res.size else None})
            rate = [x["eigenpairs_per_s"] for x in runs]
            rec = {"eigenpairs_per_s": round(float(np.mean(rate)), 2),
                   "eigenpairs_per_s_min_max": [min(rate), max(rate)],
                   "seconds": round(float(np.mean([x["seconds"] for x in runs])), 4),
                   "iterations": round(float(np.mean([x["iterations"] for x in runs])), 1),
                   "all_correct": all(x["eigenpairs"] == exact.size for x in runs), "tau_c": tau_c,
                   "max_abs_eig_err": max((x["max_abs_eig_err"] or 0.0) for x in runs),
                   "max_residual": max((x["max_residual"] or 0.0) for x in runs)}
            rec_w[label] = rec
            log(f"solve {name} {label}: {rec}")
        for fast, slow in (("mixed", "fp64_tau1e-6"), ("mixed_adaptive", "fp64_adaptive_tau1e-6")):
            if rec_w[slow]["eigenpairs_per_s"] > 0:
                rec_w[f"{fast}_vs_fp64_equal_accuracy"] = round(
                    rec_w[fast]["eigenpairs_per_s"] / rec_w[slow]["eigenpairs_per_s"], 3)
        M.close()
        out[name] = rec_w
    return out


def eigencount_rates(afsi, torch, dev, probes=64):
    """Setup step of Section 3.4: the eigenvalue count in [a, b] by trace estimation of
    the filter (Lanczos damping m = 0.5 at the workload's degree) over `probes` +-1
    probe vectors, and the block size p = ceil(1.8 * estimate) it implies.  Reports the
    estimate, its standard error, the exact count where a fixture holds it, and the
    wall time of the call (inputs resident)."""
    from workloads import build_config, probe_block

    out = {}
    for name in ("lap2d_64", "lap3d_pot_27", "lap3d_pot_100"):
        A, (lmin, lmax), (a, b), cfg = build_config(name)
        M = afsi.Matrix(A, device=0, bounds=(lmin, lmax))
        Z = torch.from_numpy(probe_block(A.n, probes, seed=1)).to(dev)
        Y, W = torch.empty_like(Z), torch.empty_like(Z)
        afsi.afsi_estimate_eigencount(M.handle, a, b, cfg.degree, Z, Y, W, "lanczos", 0.5)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        est, per = afsi.afsi_estimate_eigencount(M.handle, a, b, cfg.degree, Z, Y, W, "lanczos", 0.5)
        dt = time.perf_counter() - t0
        rec = {"n": A.n, "degree": cfg.degree, "probes": probes, "estimate": round(est, 2),
               "std_error": round(float(np.std(per, ddof=1) / np.sqrt(per.size)), 2),
               "block_size": afsi.afsi_block_size(est, 1.8, A.n), "configured_p": cfg.p,
               "ms": round(dt * 1e3, 2)}
        if name != "lap3d_pot_100":
            rec["exact_count"] = int(_window_fixture(name).size)
        else:
            # the other setup step: Lanczos bounds (40 steps, one vector) against Gershgorin
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lo, hi = afsi.afsi_estimate_spectral_bounds(M.handle, 40, 7)
            rec["bounds_estimate"] = {"steps": 40, "lmin": round(lo, 6), "lmax": round(hi, 6),
                                      "gershgorin": [round(lmin, 6), round(lmax, 6)],
                                      "ms": round((time.perf_counter() - t0) * 1e3, 2)}
        log(f"eigencount {name}: {rec}")
        out[name] = rec
        del Z, Y, W
        M.close()
        torch.cuda.empty_cache()
    return out


# (workload, block s, basis m, degree, form, tau_c): filtered thick-restart block Lanczos
# (the mixed form only where the filter separates the window's eigenvalues: on the 27^3
# window the degree-200 filter is flat to ~1e-7 over its interior, below what an FP32
# operator resolves, and the mixed Lanczos does not lock those pairs)
LANCZOS_RUNS = [("lap2d_64", 8, 128, 60, "fp64", 1e-10), ("lap2d_64", 8, 128, 60, "fp64", 1e-6),
                ("lap2d_64", 8, 128, 60, "mixed", 1e-6), ("lap3d_pot_27", 32, 512, 120, "fp64", 1e-10),
                ("lap3d_pot_27", 32, 512, 200, "fp64", 1e-10), ("lap3d_pot_27", 32, 512, 300, "fp64", 1e-10),
                ("lap3d_pot_27", 32, 512, 200, "fp64", 1e-6)]


def lanczos_rates(afsi, torch, dev, seeds=(0, 1, 2, 3, 4)):
    """Eigenpairs/s of the filtered thick-restart block Lanczos (Jackson filter of a fixed
    degree) on the converging workloads, from resident start blocks, mean over start-block
    seeds 0-4: FP64 at tau_c = 1e-10, and FP64 against the mixed form (FP32 filter) at
    tau_c = 1e-6; a run counts its pairs only with the fixture's exact count and every
    eigenvalue within 1e-10 ||A|| (1e-5 ||A|| at tau_c = 1e-6).  The subspace-iteration
    figures of the same workloads are in the solve record."""
    from workloads import build_config, start_block

    out = {}
    for name, s_blk, m, deg, form, tau_c in LANCZOS_RUNS:
        A, (lmin, lmax), (a, b), cfg = build_config(name)
        exact = _window_fixture(name)
        normA = max(abs(lmin), abs(lmax))
        tol = 1e-10 if tau_c <= 1e-10 else 1e-5
        M = afsi.Matrix(A, device=0, bounds=(lmin, lmax))
        E = torch.zeros((A.n, 2 * exact.size + m), dtype=torch.float64, device=dev)
        o = afsi.afsi_lanczos_options_default(deg)
        o.block, o.basis, o.max_cycles, o.tau_c = s_blk, m, 300, tau_c
        o.mixed = int(form == "mixed")
        runs = []
        for i, sd in enumerate((seeds[0],) + tuple(seeds)):
            X0 = torch.from_numpy(start_block(A.n, s_blk, seed=sd)).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, lam, res, r = afsi.afsi_filtered_lanczos(M.handle, a, b, o, X0, E)
            dt = time.perf_counter() - t0
            if i == 0:
                continue  # untimed: first-use allocations
            ok = st == 0 and lam.size == exact.size and np.max(np.abs(lam - exact)) <= tol * normA
            runs.append({"seed": sd, "seconds": round(dt, 4), "eigenpairs": int(lam.size) if ok else 0,
                         "cycles": r.cycles, "filter_columns": r.filter_columns})
        rate = [x["eigenpairs"] / x["seconds"] for x in runs]
        rec = {"n": A.n, "block": s_blk, "basis": m, "degree": deg, "form": form, "tau_c": tau_c,
               "eigenvalues": int(exact.size),
               "eigenpairs_per_s": round(float(np.mean(rate)), 2),
               "seconds": round(float(np.mean([x["seconds"] for x in runs])), 4),
               "cycles": round(float(np.mean([x["cycles"] for x in runs])), 1),
               "filter_products_x_columns": int(np.mean([x["filter_columns"] for x in runs])) * deg,
               "all_correct": all(x["eigenpairs"] == exact.size for x in runs)}
        log(f"lanczos {name} s={s_blk} m={m} k={deg} {form} tau {tau_c}: {rec}")
        out[f"{name}_s{s_blk}_m{m}_k{deg}_{form}_tau{tau_c:g}"] = rec
        M.close()
        del E
        torch.cuda.empty_cache()
    f, m_ = out.get("lap2d_64_s8_m128_k60_fp64_tau1e-06"), out.get("lap2d_64_s8_m128_k60_mixed_tau1e-06")
    if f and m_ and f["eigenpairs_per_s"] > 0:
        out["mixed_vs_fp64_equal_accuracy"] = round(m_["eigenpairs_per_s"] / f["eigenpairs_per_s"], 3)
    return out


def bandwidth_sweep(torch, dev, path):
    """Plain streaming references against working-set size: torch's device copy (read one
    FP64 buffer, write one) and addcmul_ (read three, write one in place), repeated back
    to back and timed with HIP events; sets up to ~256 MB stay in the memory-side cache."""
    with open(path, "w") as fh:
        for mb in (16, 32, 64, 96, 128, 256, 512, 2048, 4096):
            n = mb * (1 << 20) // 8
            a = torch.randn(n, dtype=torch.float64, device=dev)
            b, c, d = torch.empty_like(a), torch.randn_like(a), torch.randn_like(a)
            reps = max(5, 20000 // mb)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            rec = {"MB_per_buffer": mb, "copy_ws_MB": 2 * mb, "3r1w_ws_MB": 3 * mb}
            for name, fn, passes in (("copy_GBs", lambda: b.copy_(a), 2),
                                     ("3r1w_GBs", lambda: b.addcmul_(c, d), 4)):
                for _ in range(3):
                    fn()
                e0.record()
                for _ in range(reps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                rec[name] = round(passes * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9)
            log(f"bandwidth: {rec}")
            fh.write(json.dumps(rec) + "\n")
            del a, b, c, d
            torch.cuda.empty_cache()


def irregular_record(afsi, torch, dev, products=8):
    """The irregular matrix (n = 2e6, ~24 nnz/row, half of each row's columns uniform at
    random) at its full block width p = 640 in FP32: steady Clenshaw products (HIP events),
    against the compulsory bytes and the gather-inclusive model (every off-band entry
    gathers its source row from HBM).  The block is N(0,1) drawn on the device."""
    from workloads import build_config

    A, (lmin, lmax), (a, b), cfg = build_config("rand_2m")
    M = afsi.Matrix(A, device=0, bounds=(lmin, lmax))
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    X = torch.randn((A.n, cfg.p), dtype=torch.float32, device=dev, generator=gen)
    Y, W = torch.empty_like(X), torch.empty_like(X)
    coeffs = afsi.afsi_filter_coefficients(lmin, lmax, a, b, products, cfg.damping)
    afsi.afsi_filter_block_profiled(M.handle, coeffs, products, X, Y, W)  # warm-up
    ms, kind = afsi.afsi_filter_block_profiled(M.handle, coeffs, products, X, Y, W)
    steady = float(np.mean(ms[2:][kind[2:] == 3]))
    pb = A.n * cfg.p * 4
    a_bytes = A.nnz * 8 + 4 * (A.n + 1)
    compulsory = a_bytes + 4 * pb
    # off-band entries (|col - row| > 64) gather a whole row from HBM each
    rp, ci = A.row_ptr, A.col
    rows = np.repeat(np.arange(A.n), np.diff(rp))
    far = int(np.count_nonzero(np.abs(ci.astype(np.int64) - rows) > 64))
    gathered = compulsory + far * cfg.p * 4
    rec = {"n": A.n, "nnz": A.nnz, "p": cfg.p, "dtype": "f32", "steady_product_us": round(steady * 1e3, 1),
           "compulsory_bytes": compulsory, "compulsory_gbs": round(compulsory / (steady * 1e-3) / 1e9, 1),
           "far_entries": far, "gather_inclusive_bytes": gathered,
           "gather_inclusive_gbs": round(gathered / (steady * 1e-3) / 1e9, 1)}
    rec["compulsory_frac"] = round(rec["compulsory_gbs"] / HBM_PEAK_GBS, 4)
    # the same products in 256-byte column blocks of the dense operand (MaSpMM's loop over
    # column blocks, afsi_matrix_set_column_block): A is read once per block, each block's
    # gathered rows are reused from the memory-side cache while every row of A passes
    afsi.afsi_matrix_set_column_block(M.handle, 256)
    afsi.afsi_filter_block_profiled(M.handle, coeffs, products, X, Y, W)  # warm-up
    ms, kind = afsi.afsi_filter_block_profiled(M.handle, coeffs, products, X, Y, W)
    afsi.afsi_matrix_set_column_block(M.handle, 0)
    blk = float(np.mean(ms[2:][kind[2:] == 3]))
    blocks = -(-cfg.p * 4 // 256)
    comp_blk = compulsory + (blocks - 1) * a_bytes
    rec["column_blocks_256B"] = {"steady_product_us": round(blk * 1e3, 1),
                                 "compulsory_bytes": comp_blk,
                                 "compulsory_gbs": round(comp_blk / (blk * 1e-3) / 1e9, 1),
                                 "speedup_vs_whole_rows": round(steady / blk, 3)}
    log(f"irregular rand_2m fp32: {rec}")
    M.close()
    del X, Y, W
    torch.cuda.empty_cache()
    return rec


def complex_record(afsi, torch, dev, products=8):
    """The complex lattice (64^3 periodic tight binding, n = 262144, 7 complex entries per
    row) at its block width p = 192: steady Clenshaw products in complex FP64 (C128) and
    complex FP32 (C64), HIP events, against the compulsory bytes (A once + four passes of
    the block); in folded 16 x 16 pencils (afsi_grid_order with fold_x: the periodic x
    neighbours at most two cross-sections apart) and, for comparison, the natural order.
    The block is N(0,1) + i N(0,1) drawn on the device."""
    from workloads import build_config

    A, (lmin, lmax), (a, b), cfg = build_config("tb3d_64")
    L = cfg.size
    orders = {"folded_pencil_16x16": afsi.afsi_csr_permute(A, afsi.afsi_grid_order(L, L, L, 16, 16, fold_x=True)),
              "natural": A}
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    coeffs = afsi.afsi_filter_coefficients(lmin, lmax, a, b, products, cfg.damping)
    rec = {"n": A.n, "nnz": A.nnz, "p": cfg.p}
    for name, dt, sx in (("c128", torch.complex128, 16), ("c64", torch.complex64, 8)):
        X = torch.randn((A.n, cfg.p), dtype=dt, device=dev, generator=gen)
        Y, W = torch.empty_like(X), torch.empty_like(X)
        comp = A.nnz * (sx + 4) + 4 * (A.n + 1) + 4 * A.n * cfg.p * sx
        rec[name] = {"compulsory_bytes": comp}
        for oname, B in orders.items():
            M = afsi.Matrix(B, device=0, bounds=(lmin, lmax))
            afsi.afsi_filter_block_profiled(M.handle, coeffs, products, X, Y, W)  # warm-up
            ms, kind = afsi.afsi_filter_block_profiled(M.handle, coeffs, products, X, Y, W)
            M.close()
            steady = float(np.mean(ms[2:][kind[2:] == 3]))
            gbs = comp / (steady * 1e-3) / 1e9
            r = {"steady_product_us": round(steady * 1e3, 1), "gbs": round(gbs, 1),
                 "frac": round(gbs / HBM_PEAK_GBS, 4)}
            if oname == "natural":
                rec[name]["natural"] = r
            else:
                rec[name].update(r)
                rec[name]["ordering"] = oname
        del X, Y, W
        torch.cuda.empty_cache()
    log(f"complex tb3d_64: {rec}")
    return rec


def serve_rates(afsi, M_slices, num, loads=(0.5, 0.8, 0.95)):
    """p50/p99 latency and throughput of the continuous-batching server.

    (a) the serving mix (the literal stream): half spectrum slices of the 100^3 matrix
        (16 slices, p = 96, degree 120, slices of one matrix share grouped launches),
        half independent 3D Laplacian + potential matrices (n log-uniform in [1e4, 1e6],
        p in {32..256}, degree in [40, 200]); a fixed budget of 2 iterations per
        request.  The capacity is measured first (all `num` requests submitted at once,
        requests finished per second); then `num` Poisson arrivals at each offered load
        (a fraction of that capacity) give the latency percentiles.  FP64 and mixed.
    (b) a converging stream at equal accuracy (tau_c = 1e-6 in both forms, plus FP64 at
        1e-10): 2D Laplacian window requests (40 eigenpairs, fixed Jackson degree 60)
        and 27^3 Laplacian + potential requests (196 eigenpairs, the paper's adaptive
        mode); eigenpairs/s counts a request's pairs only when its count equals the
        fixture's and every eigenvalue is within 1e-5 ||A|| (1e-10 ||A|| at tau_c 1e-10).
    """
    from paper_2604_00914_amd import serve
    from tests.golden_util import lap2d_window, lap3d27_window
    from workloads import build_config, laplacian_3d_dirichlet
    from workloads.stream import serving_stream

    reqs = serving_stream(num, rate_hz=1.0, seed=0)   # arrivals rescaled per load below
    base = np.array([r.arrival for r in reqs])
    mats = {}
    for r in reqs:
        if r.kind == "matrix" and r.grid not in mats:
            mats[r.grid] = afsi.Matrix(laplacian_3d_dirichlet(r.grid, 2.0, seed=r.seed), bounds=(0.0, 14.0))
    out = {"mix": {"requests": num, "max_iter": 2, "slices": sum(r.kind == "slice" for r in reqs),
                   "loads": list(loads)}}

    def jobs_for(form, arrivals):
        jobs = []
        for r, t in zip(reqs, arrivals):
            o = afsi.afsi_options_default(r.degree)
            o.max_iter = 2
            if form == "mixed":
                o.filter_dtype, o.tau_c = afsi.R32, 1e-6
            M = M_slices if r.kind == "slice" else mats[r.grid]
            jobs.append((float(t), M, r.a, r.b, r.p, o, r.seed, r.kind))
        return jobs

    def run(jobs):
        with serve.Server(hbm_budget_bytes=200 << 30) as S:
            S.set_pool_columns(M_slices, 16 * 96)
            return serve.run_stream(S, jobs).summary()

    for form in ("fp64", "mixed"):
        burst = run(jobs_for(form, np.zeros(num)))
        cap = burst["throughput_req_per_s"]
        rec = {"capacity_req_per_s": cap, "burst": burst}
        for load in loads:
            s = run(jobs_for(form, base / (load * cap)))
            s["offered_req_per_s"] = round(load * cap, 3)
            rec[f"load_{load}"] = s
            log(f"serve mix {form} load {load}: {s}")
        out["mix"][form] = rec

    # (b) converging stream
    specs = []
    A1, (lo1, hi1), (a1, b1), cfg1 = build_config("lap2d_64")
    A2, (lo2, hi2), (a2, b2), cfg2 = build_config("lap3d_pot_27")
    M1, M2 = afsi.Matrix(A1, bounds=(lo1, hi1)), afsi.Matrix(A2, bounds=(lo2, hi2))
    ref = {"lap2d_64": lap2d_window(), "lap3d_pot_27": lap3d27_window()}
    norm = {"lap2d_64": max(abs(lo1), abs(hi1)), "lap3d_pot_27": max(abs(lo2), abs(hi2))}
    k1 = paper_initial_degree(lo2, hi2, a2, b2)
    rng = np.random.default_rng(1)
    arrivals = np.cumsum(rng.exponential(1.0 / 40.0, size=24))
    for i, t in enumerate(arrivals):
        if i % 3 == 2:
            specs.append((float(t), "lap3d_pot_27", M2, a2, b2, cfg2.p, math.ceil(2.5 * k1), True))
        else:
            specs.append((float(t), "lap2d_64", M1, a1, b1, cfg1.p, cfg1.degree, False))
    out["converging"] = {"requests": len(specs), "rate_hz": 40.0,
                         "workloads": {"lap2d_64": "fixed Jackson degree 60, p = 64",
                                       "lap3d_pot_27": f"adaptive (Lanczos m = 0.5, k1 = {k1}, "
                                                       f"kmax = {math.ceil(2.5 * k1)}), p = {cfg2.p}"}}
    for form, tau_c in (("fp64", 1e-10), ("fp64", 1e-6), ("mixed", 1e-6)):
        jobs = []
        for i, (t, name, M, a, b, p, kmax, adaptive) in enumerate(specs):
            o = afsi.afsi_options_default(kmax)
            o.tau_c, o.max_iter = tau_c, 1500
            if adaptive:
                o.adaptive, o.damping = 1, afsi.DAMP_LANCZOS
            if form == "mixed":
                o.filter_dtype = afsi.R32
            jobs.append((t, M, a, b, p, o, 500 + i, name))
        with serve.Server(hbm_budget_bytes=64 << 30) as S:
            S.set_pool_columns(M1, 8 * cfg1.p)
            S.set_pool_columns(M2, 4 * cfg2.p)
            rep = serve.run_stream(S, jobs)
        s = rep.summary()
        tol = 1e-10 if tau_c <= 1e-10 else 1e-5
        good = 0
        wrong = 0
        for c in rep.completed:
            r = ref[c.tag]
            ok = c.eigenvalues.size == r.size and np.max(np.abs(c.eigenvalues - r)) <= tol * norm[c.tag]
            good += r.size if ok else 0
            wrong += 0 if ok else 1
        s["correct_eigenpairs_per_s"] = round(good / max(rep.wall_s, 1e-9), 2)
        s["requests_not_exact"] = wrong
        s["tau_c"] = tau_c
        key = form if tau_c > 1e-10 else "fp64_tau1e-10"
        out["converging"][key] = s
        log(f"serve converging {key}: {s}")
    c = out["converging"]
    if c["fp64"]["correct_eigenpairs_per_s"] > 0:
        c["mixed_vs_fp64_equal_tau"] = round(c["mixed"]["correct_eigenpairs_per_s"] /
                                             c["fp64"]["correct_eigenpairs_per_s"], 3)
    for M in mats.values():
        M.close()
    M1.close()
    M2.close()
    return out


# Table 1 of the paper (Section 4.1): rows, nonzeros and eigenvalue count of each test matrix
PAPER_TABLE1 = {"Ge87H76": (112985, 7892195, 212), "Ge99H100": (112985, 8451395, 250),
                "Si41Ge41H72": (185639, 15011265, 218), "Si87H76": (240369, 10661631, 213),
                "Ga41As41H72": (268096, 18488476, 201)}


def paper_context():
    """The paper's own AdaPolySI figures as context (Tables 1 and 2, Section 4.1: one CPU
    socket, 28 OpenMP threads, FP64, SuiteSparse DFT Hamiltonians of 1.1e5-2.7e5 rows,
    residual 1e-10 ||A||): eigenpairs/s (#evals / runtime) and the rate of sparse
    matrix-vector products (SpMVs x nnz / runtime, nonzeros x vectors per second, a
    lower bound on its SpMM rate since the whole solve is timed).  Different hardware
    and matrices: not a target."""
    rows = [l.strip().split(",") for l in open(os.path.join(ROOT, "tests", "golden", "paper_table2.csv"))
            if l.strip() and not l.startswith("#") and not l.startswith("matrix")]
    out = {"hardware": "one CPU socket, 28 OpenMP threads, FP64 (Section 4)", "per_matrix": {}}
    for m, method, avgdeg, it, spmvs, rt, res in rows:
        if method != "AdaPolySI":
            continue
        n, nnz, ev = PAPER_TABLE1[m]
        out["per_matrix"][m] = {"n": n, "eigenpairs": ev, "runtime_s": float(rt),
                                "eigenpairs_per_s": round(ev / float(rt), 2),
                                "spmv_nnz_per_s": float(f"{int(spmvs) * nnz / float(rt):.3g}")}
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sweep(path, budget_s=10.0):
    """The oracle on the host cores: per workload a bounded sample of FP64 Clenshaw
    products with all threads and with one thread (one-thread samples on a column
    subset for the wide workloads, scaled to full width), extrapolated to one full
    filter; plus full oracle solves of the converging lap2d_64 workload."""
    from oracle import coefficients as co
    from oracle import native
    from oracle import solver as osolver
    from oracle.filter import clenshaw_steps
    from workloads import build_config, start_block

    native.build(force=False)
    all_threads = native.num_threads()
    out = open(path, "w")

    def sample(A, X0, c, l1, l2, k, secs):
        gen = clenshaw_steps(A, X0, c, l1, l2)
        t0 = time.perf_counter()
        next(gen)
        one = time.perf_counter() - t0
        steps = max(1, min(k - 1, int(secs / max(one, 1e-4))))
        t0 = time.perf_counter()
        for _ in range(steps):
            next(gen)
        return steps, (time.perf_counter() - t0) / steps

    for name in ("lap2d_64", "lap3d_pot_100", "tb3d_64", "rand_2m"):
        A, (lmin, lmax), (a, b), cfg = build_config(name, seed=0)
        n, p, k = A.n, cfg.p, cfg.degree
        cplx = A.is_complex
        s = 16 if cplx else 8
        c = co.filter_coefficients(lmin, lmax, a, b, k, cfg.damping)
        l1, l2 = co.affine_map(lmin, lmax)
        rec = {"workload": name, "n": n, "nnz": A.nnz, "p": p, "degree": k, "dtype": "c128" if cplx else "f64",
               "cpu": cpu_model(), "threads": all_threads}
        step_bytes = A.nnz * (s + 4) + 4 * (n + 1) + 4 * n * p * s
        for label, threads, cols in (("all_threads", all_threads, p), ("one_thread", 1, min(p, 64 if n > 1e5 else p))):
            native.set_num_threads(threads)
            X0 = start_block(n, cols, seed=1, complex_=cplx)
            steps, per = sample(A, X0, c, l1, l2, k, budget_s)
            del X0
            scale = p / cols
            per_full = per * scale
            rec[label] = {"threads": threads, "sample_products": steps, "sample_cols": cols,
                          "s_per_product": round(per_full, 4), "filter_s_extrapolated": round(per_full * k, 2),
                          "gbs": round(step_bytes / per_full / 1e9, 3)}
            log(f"cpu oracle {name} {label}: {rec[label]}")
        native.set_num_threads(all_threads)
        out.write(json.dumps(rec) + "\n")
        out.flush()
    # full oracle solves where they converge
    A, (lmin, lmax), (a, b), cfg = build_config("lap2d_64")
    for threads in (all_threads, 1):
        native.set_num_threads(threads)
        X0 = start_block(A.n, cfg.p, seed=0)
        o = osolver.Options(kmax=cfg.degree)
        t0 = time.perf_counter()
        res = osolver.solve(A, a, b, lmin, lmax, X0, o)
        dt = time.perf_counter() - t0
        rec = {"workload": "lap2d_64 solve", "threads": threads, "seconds": round(dt, 3),
               "eigenpairs": int(len(res.eigenvalues)), "iterations": int(res.iterations),
               "eigenpairs_per_s": round(len(res.eigenvalues) / dt, 2), "cpu": cpu_model()}
        log(f"cpu oracle solve: {rec}")
        out.write(json.dumps(rec) + "\n")
    native.set_num_threads(all_threads)
    out.close()


def cpu_baseline(A, p, k, lmin, lmax, a, b, cfg, sx, sample_steps):
    """The oracle's Clenshaw filter on the same matrix, a few products, on the host cores."""
    from oracle import coefficients as co
    from oracle import native
    from oracle.filter import clenshaw_steps
    from workloads import start_block

    native.build(force=False)
    threads = native.num_threads()
    X0 = start_block(A.n, p, seed=1)
    c = co.filter_coefficients(lmin, lmax, a, b, k, cfg.damping)
    l1, l2 = co.affine_map(lmin, lmax)
    # size the sample to roughly 10-30 s of work: time one product first
    gen = clenshaw_steps(A, X0, c, l1, l2)
    t0 = time.perf_counter()
    next(gen)
    one = time.perf_counter() - t0
    steps = sample_steps or max(2, min(k - 1, int(15.0 / max(one, 1e-3))))
    t0 = time.perf_counter()
    for _ in range(steps):
        next(gen)
    dt = time.perf_counter() - t0
    del gen, X0
    step_bytes = A.nnz * (8 + 4) + 4 * (A.n + 1) + 4 * A.n * p * 8
    # one thread, on a 64-column sample of the block (bytes scaled to the full width)
    cols = min(p, 64)
    native.set_num_threads(1)
    try:
        X1 = start_block(A.n, cols, seed=1)
        gen = clenshaw_steps(A, X1, c, l1, l2)
        next(gen)
        t1 = time.perf_counter()
        n1 = 2
        for _ in range(n1):
            next(gen)
        per1 = (time.perf_counter() - t1) / n1 * (p / cols)
    finally:
        native.set_num_threads(threads)
    return {
        "value": round(steps * step_bytes / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{steps} Clenshaw products (of {k}) of the FP64 oracle on the full "
                  f"{cfg.name} matrix, n={A.n}, p={p}; {dt:.1f} s",
        "seconds_per_product": round(dt / steps, 4),
        "cpu": cpu_model(),
        "one_thread": {"value": round(step_bytes / per1 / 1e9, 3), "unit": "GB/s",
                       "seconds_per_product": round(per1, 3),
                       "sample": f"{n1} products on a {cols}-column block, scaled to p={p}"},
    }


if __name__ == "__main__":
    main()
