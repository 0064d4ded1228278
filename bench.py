"""Benchmark of the Chebyshev-filter hot path on one MI355X.

One step = one pass of the hot path over the resident synthetic block: the
degree-m Chebyshev filter (m fused BSR-SpMM + recurrence launches) followed,
when available, by the FP64 Rayleigh-Ritz step (Cholesky-QR twice, X^T H X,
dense eigensolve, rotation).  Prints ONE JSON line.  Beside the timed steps it
reports the occupancies and density on the step's Ritz pairs, the filter's
adjoint on the adjoint workload, the reduced-precision filters against FP64 and
the CPU oracle's rate.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision f64|f32|bf16|bf16x3] [--no-cpu-baseline] [--no-rr]
                    [--no-mixed] [--no-adjoint] [--solve] [--calib-copy]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Chebyshev-filter GFLOP/s + HBM GB/s (% roofline); mixed vs FP64 at ≤1e-6 Ha"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}   # dense MFMA peaks, MI355X
PEAK_HBM_GBS = 8000.0

# HBM-side bytes per launch of the dominant kernel from the two rocprofv3 counter
# passes (FETCH_SIZE, WRITE_SIZE), calibrated against a plain copy of known size;
# see profiles/cheb_step_<precision>_lattice60_h4_n2048_m20_bytes.md.  Valid only while
# the kernel source is the one that was profiled.
COUNTED_TRAFFIC = {
    ("f64", "lattice60_h4_n2048_m20"): {"read_bytes": 89.384e9, "write_bytes": 3.539e9,
                                        "kernel_sha256_16": "59b3b427be3be9de"},
    ("bf16", "lattice60_h4_n2048_m20"): {"read_bytes": 16.201e9, "write_bytes": 1.774e9,
                                        "kernel_sha256_16": "59b3b427be3be9de"},
    ("bf16x3", "lattice60_h4_n2048_m20"): {"read_bytes": 16.922e9, "write_bytes": 1.771e9,
                                        "kernel_sha256_16": "59b3b427be3be9de"},
}


def kernel_source_sha16():
    import hashlib
    path = os.path.join(ROOT, "paper_2110_15853_amd", "csrc", "cheb_step.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(Hc, X, cfg, n_cols, threads=None):
    """The FP64 oracle (SciPy CSR) on a column sample of the same workload, as
    it stands: first on one core (n_cols columns), then on all host cores with
    one thread per n_cols-column slice (the filter is column-independent, so
    the slices are independent oracle runs; SciPy's sparse product and NumPy's
    array arithmetic release the GIL).  Reported as algorithmic GFLOP/s."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    threads = threads or min(16, os.cpu_count() or 1)

    def run(j):
        Xs = np.ascontiguousarray(X[:, j * n_cols:(j + 1) * n_cols])
        oracle.cheb_filter(Hc, Xs, cfg.m, cfg.a, cfg.b, cfg.a0)

    t0 = time.perf_counter()
    run(0)
    dt1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(threads)))
    dtn = time.perf_counter() - t0
    flops1 = 2.0 * Hc.nnz * n_cols * cfg.m
    # the same definition in plain C with OpenMP, threads x n_cols-column blocks
    Xc = np.ascontiguousarray(X[:, :threads * n_cols])
    t0 = time.perf_counter()
    oracle.cheb_filter_c(Hc, Xc, cfg.m, cfg.a, cfg.b, cfg.a0, threads=threads, blk=n_cols)
    dtc = time.perf_counter() - t0
    return {"value": flops1 * threads / dtn / 1e9, "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{threads * n_cols} of {cfg.n} columns as {threads} threads x {n_cols} columns, "
                      f"full m={cfg.m} filter, SciPy CSR FP64 ({dtn:.1f} s); algorithmic flops "
                      f"2*nnz*cols*m",
            "one_core": {"value": flops1 / dt1 / 1e9, "sample": f"{n_cols} columns ({dt1:.1f} s)"},
            "c_openmp": {"value": flops1 * threads / dtc / 1e9, "cores": threads,
                         "sample": f"the same {threads * n_cols} columns by the C/OpenMP oracle "
                                   f"(CSR FP64, {n_cols}-column blocks, {dtc:.1f} s)"},
            "host_cpus": os.cpu_count(), "host": platform.processor() or platform.machine()}


STEP_KERNEL = {"f64": "cheb_step_mfma<double>", "f32": "cheb_step_mfma<float>",
               "bf16": "cheb_step_bf16_patch<float, false>", "bf16x3": "cheb_step_bf16_patch<float, true>"}


def step_roofline(prec, alg_flops, alg_bytes, launch_s, traffic=None):
    """Roofline entry of one step-kernel launch.  FP64 and FP32 tiles are bound
    by the matrix cores (arithmetic intensity 43.6 flop/B against ridges of 9.8
    and 19.7); BF16 tiles with FP32 iterates are bound by HBM (ridge about 315
    flop/B), so they are reported as algorithmic bytes per launch time."""
    if prec in ("f64", "f32"):
        ach = alg_flops / launch_s / 1e12
        return {"bound": "mfma", "kernel": STEP_KERNEL[prec], "achieved": round(ach, 3),
                "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s", "frac": round(ach / PEAK_TFLOPS[prec], 4),
                "traffic": traffic}
    ach = alg_bytes / launch_s / 1e9
    return {"bound": "hbm", "kernel": STEP_KERNEL[prec], "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic}


def issued_flops(H, prec):
    """Matrix-core flop issued per vector by one step launch: FP64/FP32 tiles
    issue the 16x4 fragments whose mask bit is set (2*64 flop each per vector);
    BF16 tiles issue the 16x32 fragments holding any set 16x4 sub-block (2*512
    flop each), three times for the bf16x3 split products."""
    fm = H.frag_mask.cpu().numpy().view(np.uint64)
    if prec in ("f64", "f32"):
        return 2.0 * 64 * int(np.unpackbits(fm.view(np.uint8)).sum())
    bits = np.unpackbits(fm.view(np.uint8), bitorder="little").reshape(-1, 64)   # bit 4*kk4 + mb
    frag = bits.reshape(-1, 2, 8, 4).any(axis=2)                                   # [tile, kk, mb]
    return 2.0 * 512 * int(frag.sum()) * (3 if prec == "bf16x3" else 1)


def mixed_precision_report(P, torch, ip, ix, d, cfg, H64, Xb64, keep_frac=1800 / 2048, reps=3,
                           m_late=(4, 18)):
    """Low-precision filters followed by the FP64 Rayleigh-Ritz with FP64 H,
    against the FP64 pipeline from the same start block (the FP64 pipeline is
    itself checked against the oracle at this size by the tests): FP32 tiles;
    BF16 tiles; bf16x3 split products; and the precision schedules BF16 tiles
    for the first m - m_late steps then FP32 or bf16x3 tiles for the last
    m_late, for each m_late given (FP32 iterates throughout).  For each: the filter time, its
    roofline entry, and the error of the lowest Ritz values and the largest
    principal angle between the Ritz subspaces, from a random start (cold) and
    from the FP64 Ritz vectors of one previous pass (warm)."""
    keep = int(round(keep_frac * cfg.n))
    out = {"keep": keep, "m_late": list(m_late), "reference": "GPU FP64 pipeline (filter + Rayleigh-Ritz)"}

    def time_filter(fn, X):
        Y = fn(X)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            fn(X)
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps, Y

    def angle(U, V):
        S = torch.linalg.svdvals((U.T @ V).cpu())
        return float(torch.arccos(torch.clamp(S.min(), -1.0, 1.0)))

    f64 = lambda X: P.cheb_filter(H64, X, cfg.m, cfg.a, cfg.b, cfg.a0)
    t64, _ = time_filter(f64, Xb64)
    out["f64_filter_ms"] = round(t64, 3)
    lam_c, psi_c = P.rayleigh_ritz(H64, f64(Xb64))
    Xw = psi_c.clone()
    lam_w, psi_w = P.rayleigh_ritz(H64, f64(Xw))
    tiles = {"f32": P.bsr_astype(H64, torch.float32), "bf16": P.bsr_astype(H64, torch.bfloat16),
             "bf16x3": P.bsr_astype(H64, "bf16x3")}
    elt = 4
    x_bytes = 3.0 * H64.rows * cfg.n * elt
    nnz = len(d)
    runs = [("f32", "f32", 0), ("bf16", "bf16", 0), ("bf16x3", "bf16x3", 0)]
    for ml in m_late:
        runs += [(f"bf16x{cfg.m - ml}+f32x{ml}", "f32", ml), (f"bf16x{cfg.m - ml}+bf16x3x{ml}", "bf16x3", ml)]
    for name, late, ml in runs:
        early = name.split("x")[0] if "+" in name else name
        He, Hl = tiles[early], tiles[late]
        fn = lambda X, He=He, Hl=Hl, ml=ml: P.cheb_filter_schedule(He, Hl, ml, X, cfg.m, cfg.a, cfg.b, cfg.a0)
        Xl = P.cast(Xb64, torch.float32)
        tl, _ = time_filter(fn, Xl)
        steps = [(early, cfg.m - ml), (late, ml)] if ml else [(early, cfg.m)]
        rec = {"filter_ms": round(tl, 3), "steps": {k: v for k, v in steps if v},
               "speedup_vs_f64_filter": round(t64 / tl, 3),
               "alg_gflops": round(2.0 * nnz * cfg.n * cfg.m / (tl / 1e3) / 1e9, 1)}
        if ml == 0:
            hb = tiles[early].vals.numel() * tiles[early].vals.element_size()
            counted = COUNTED_TRAFFIC.get((early, cfg.name))
            traffic = (counted["read_bytes"] + counted["write_bytes"]
                       if counted and counted["kernel_sha256_16"] == kernel_source_sha16() else None)
            rec["roofline"] = step_roofline(early, 2.0 * nnz * cfg.n, hb + x_bytes, tl / 1e3 / cfg.m, traffic)
            rec["roofline"]["alg_bytes_per_launch"] = hb + x_bytes
        for regime, X0, lam_ref, psi_ref in (("cold", Xl, lam_c, psi_c),
                                             ("warm", P.cast(Xw, torch.float32), lam_w, psi_w)):
            lam, psi = P.rayleigh_ritz(H64, fn(X0))
            err = float((lam[:keep] - lam_ref[:keep]).abs().max())
            rec[regime] = {"max_ritz_err_Ha": err, "max_angle_rad": angle(psi_ref[:, :keep], psi[:, :keep]),
                           "meets_1e-6_Ha": err <= 1e-6}
        out[name] = rec
        torch.cuda.empty_cache()
        log(f"mixed {name}: {rec}")
    del tiles
    torch.cuda.empty_cache()
    return out


def symmetric_formed_tiles(rowptr, tcol):
    """Tiles a symmetric sampled product forms (P = P^T: each mirror pair once):
    (B, B') with B' >= B, and those with B' < B whose mirror (B', B) is not stored."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    nbr = len(rowptr) - 1
    brow = np.repeat(np.arange(nbr, dtype=np.int64), np.diff(rowptr))
    bcol = np.asarray(tcol, dtype=np.int64)
    mirrored = np.isin(bcol * nbr + brow, brow * nbr + bcol)
    return (bcol >= brow) | ~mirrored


def density_report(P, torch, H, lam, psi, cfg):
    """Occupancies at the paper's smearing temperature (500 K) for N_e = 1.5 n
    electrons, the density matrix on the pattern of H and the site density,
    each timed with HIP events; tr(P H) is checked against 2 sum f lambda."""
    ne = 1.5 * cfg.n
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    times = {"fermi_ms": [], "density_matrix_ms": [], "electron_density_ms": []}
    for _ in range(3):
        ev[0].record()
        f, mu = P.fermi_level(lam, ne, P.KT_500K_HARTREE)
        ev[1].record()
        Pv = P.density_matrix(H, psi, f)
        ev[2].record()
        rho = P.electron_density(psi, f)
        ev[3].record()
        torch.cuda.synchronize()
        for k, (i, j) in zip(times, [(0, 1), (1, 2), (2, 3)]):
            times[k].append(ev[i].elapsed_time(ev[j]))
    tr = float((Pv * H.vals).sum())
    want = 2.0 * float((f * lam).sum())
    # the sampled product issues 2 * 256 * n flop per 16 x 16 block that holds a
    # pattern entry (the other blocks are skipped), over the tiles it forms
    m = H.mask.view(H.n_tiles, 4, 16).cpu().numpy().view(np.uint64)
    formed = symmetric_formed_tiles(H.tile_rowptr.cpu().numpy(), H.tile_col.cpu().numpy())
    rows_or = np.bitwise_or.reduce(m[formed], axis=2)               # [formed tile, row block]
    live = sum(int(np.count_nonzero((rows_or >> np.uint64(16 * jb)) & np.uint64(0xFFFF)))
               for jb in range(4))
    dm_s = float(np.median(times["density_matrix_ms"])) / 1e3
    return {"n_electrons": ne, "kT_hartree": P.KT_500K_HARTREE, "mu": mu,
            **{k: round(float(np.median(v)), 3) for k, v in times.items()},
            "density_matrix_issued_tflops": round(2.0 * 256 * cfg.n * live / dm_s / 1e12, 2),
            "density_matrix_live_blocks": live, "density_matrix_blocks": 16 * int(formed.sum()),
            "sum_rho": float(rho.sum()), "trace_PH": tr, "two_sum_f_lambda": want}


def adjoint_report(P, torch, workload, dtypes=("f64", "f32")):
    """The filter's adjoint on the adjoint workload (r = 40, h = 3, 512 vectors,
    m = 16, loss sum(w * Y) with w ~ N(0,1)): the forward filter and the backward
    with every iterate stored and with a checkpoint every 4 steps, FP64 and FP32,
    each timed with HIP events (median of 3).  Algorithmic work of the backward:
    m reverse products and m products sampled on the pattern, 4 m nnz n flop."""
    cfg = workload.CONFIGS["lattice40_h3_n512_m16"]
    ip, ix, d, N = workload.lattice_hamiltonian(cfg.r, cfg.h, cfg.seed)
    nnz = int(len(ix))
    X = torch.from_numpy(workload.gaussian_block(N, cfg.n, cfg.seed)).cuda()
    W = torch.from_numpy(workload.gaussian_block(N, cfg.n, cfg.seed, stream="W")).cuda()
    H64 = P.bsr_build(ip, ix, d, cfg.r, dtype=torch.float64, device="cuda")
    out = {"workload": cfg.name, "N": N, "n_vec": cfg.n, "m": cfg.m, "nnz": nnz}
    for name in dtypes:
        dt = {"f64": torch.float64, "f32": torch.float32}[name]
        H = H64 if dt == torch.float64 else P.bsr_astype(H64, dt)
        Xb, Wb = P.to_blocked(X.to(dt), H), P.to_blocked(W.to(dt), H)
        runs = {
            "forward_ms": lambda: P.cheb_filter(H, Xb, cfg.m, cfg.a, cfg.b, cfg.a0),
            "backward_store_all_ms": lambda: P.cheb_filter_backward(H, Xb, Wb, cfg.m, cfg.a, cfg.b,
                                                                    cfg.a0, ckpt_every=0),
            "backward_ckpt4_ms": lambda: P.cheb_filter_backward(H, Xb, Wb, cfg.m, cfg.a, cfg.b,
                                                                cfg.a0, ckpt_every=4),
        }
        r = {}
        for key, f in runs.items():
            f()
            torch.cuda.synchronize()
            ms = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                f()
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            r[key] = round(float(np.median(ms)), 3)
        r["forward_alg_tflops"] = round(2.0 * cfg.m * nnz * cfg.n / r["forward_ms"] / 1e9, 2)
        r["backward_alg_tflops"] = round(4.0 * cfg.m * nnz * cfg.n / r["backward_store_all_ms"] / 1e9, 2)
        out[name] = r
        del H, Xb, Wb
        torch.cuda.empty_cache()
    return out


def run_large(args, P, torch, workload):
    """Large workload: ChFSI passes with a reduced-precision filter and FP64
    Rayleigh-Ritz; every pass starts from the previous pass's Ritz vectors with
    bounds updated from its Ritz values (a0 = lowest, a = highest)."""
    cfg = workload.CONFIGS[args.workload]
    prec = args.precision if args.precision != "f64" else "f32"
    fdt = {"f32": torch.float32, "bf16": torch.bfloat16}[prec]
    t0 = time.perf_counter()
    ip, ix, d, N = workload.lattice_hamiltonian(cfg.r, cfg.h, cfg.seed)
    H64 = P.bsr_build(ip, ix, d, cfg.r, dtype=torch.float64, device="cuda")
    Hf = P.bsr_astype(H64, fdt)
    X = workload.gaussian_block(N, cfg.n, cfg.seed, dtype=np.float32)
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), H64)
    del X
    rr_work = torch.empty(P.rayleigh_ritz_workspace(H64, cfg.n, torch.float32), dtype=torch.uint8,
                          device="cuda")
    torch.cuda.synchronize()
    log(f"large inputs resident ({time.perf_counter() - t0:.1f} s), "
        f"{torch.cuda.memory_allocated() / 1e9:.1f} GB allocated")
    a, b, a0 = cfg.a, cfg.b, cfg.a0
    recs = []
    for it in range(args.warmup + args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ev[0].record()
        Y = P.cheb_filter(Hf, Xb, cfg.m, a, b, a0)
        ev[1].record()
        del Xb
        lam, Psi = P.rayleigh_ritz(H64, Y, work=rr_work)
        ev[2].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        del Y
        rec = {"pass": it + 1, "a0": a0, "a": a, "filter_ms": ev[0].elapsed_time(ev[1]),
               "rr_ms": ev[1].elapsed_time(ev[2]), "wall_ms": wall * 1e3,
               "lowest_ritz": float(lam[0]), "highest_ritz": float(lam[-1])}
        log(f"large pass {it + 1}: {rec}")
        if it >= args.warmup:
            recs.append(rec)
        a0, a = P.updated_bounds(lam, b)
        Xb = P.cast(Psi, torch.float32)
        del Psi
        torch.cuda.empty_cache()
    filt_s = float(np.mean([r["filter_ms"] for r in recs])) / 1e3
    alg = 2.0 * len(d) * cfg.n * cfg.m
    value = alg / filt_s / 1e9
    launch_s = filt_s / cfg.m
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(float(np.mean([r["wall_ms"] for r in recs])), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{prec} filter, f64 Rayleigh-Ritz", "data": "synthetic",
        "config": {"workload": cfg.name, "N": N, "rows_blocked": H64.rows, "n_vec": cfg.n,
                   "m": cfg.m, "h": cfg.h, "nnz": len(d), "tiles": H64.n_tiles,
                   "step": "one ChFSI pass: filter + FP64 Rayleigh-Ritz, bounds from the previous pass"},
        "passes": recs,
        "roofline": {"bound": "mfma", "kernel": STEP_KERNEL[prec], "achieved": round(2.0 * len(d) * cfg.n / launch_s / 1e12, 3),
                     "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                     "frac": round(2.0 * len(d) * cfg.n / launch_s / 1e12 / PEAK_TFLOPS[prec], 4),
                     "traffic": None},
    }
    print(json.dumps(out), flush=True)


def run_solve(args, P, torch, workload):
    """Algorithm 1 repeated to convergence on the workload: a random start, first
    bounds from Lanczos, then passes from the previous Ritz vectors until the
    Ritz residual norms of the lowest 80% of the block are at most --tol."""
    cfg = workload.CONFIGS[args.workload]
    prec = args.precision if args.precision != "bf16" else "f32"
    tol = args.tol if args.tol else (1e-8 if prec == "f64" else 1e-5)
    t0 = time.perf_counter()
    ip, ix, d, N = workload.lattice_hamiltonian(cfg.r, cfg.h, cfg.seed)
    H64 = P.bsr_build(ip, ix, d, cfg.r, dtype=torch.float64, device="cuda")
    Hf = H64 if prec == "f64" else P.bsr_astype(H64, torch.float32)
    X = workload.gaussian_block(N, cfg.n, cfg.seed, dtype=np.float64 if prec == "f64" else np.float32)
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), H64)
    del X
    torch.cuda.synchronize()
    log(f"solve inputs resident ({time.perf_counter() - t0:.1f} s)")
    n_conv = int(0.8 * cfg.n)
    t1 = time.perf_counter()
    lam, Psi, res, hist = P.chfsi_solve(Hf, H64, Xb, cfg.m, tol, n_conv=n_conv, max_iter=args.max_passes,
                                        lanczos_k=40)
    torch.cuda.synchronize()
    total = time.perf_counter() - t1
    done = [h for h in hist if not h.get("rank_deficient")]
    for h in hist:
        if h.get("rank_deficient"):
            log(f"solve pass {h['pass']}: m={h['m']} filtered block rank-deficient, degree halved")
            continue
        log(f"solve pass {h['pass']}: m={h['m']} max residual {h['max_residual']:.3e} "
            f"filter {h['filter_ms']:.1f} ms, Rayleigh-Ritz {h['rr_ms']:.1f} ms, residuals {h['residual_ms']:.1f} ms")
    flops = sum(2.0 * len(d) * cfg.n * h["m"] for h in done)
    filt_s = sum(h["filter_ms"] for h in done) / 1e3
    launch_s = filt_s / sum(h["m"] for h in done)
    hist = done
    value = flops / filt_s / 1e9
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": len(hist), "warmup": 0, "ms_per_step": round(total / len(hist) * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{prec} filter, f64 Rayleigh-Ritz", "data": "synthetic",
        "config": {"workload": cfg.name, "N": N, "rows_blocked": H64.rows, "n_vec": cfg.n,
                   "m": cfg.m, "h": cfg.h, "nnz": len(d),
                   "step": "one ChFSI pass: filter + FP64 Rayleigh-Ritz + Ritz residuals"},
        "solve": {"converged": hist[-1]["max_residual"] <= tol, "passes": len(hist), "tol": tol,
                  "n_conv": n_conv, "max_residual": hist[-1]["max_residual"], "total_s": round(total, 3),
                  "lowest_ritz": float(lam[0]), "history": hist},
        "roofline": {"bound": "mfma", "kernel": f"cheb_step_mfma<{'double' if prec == 'f64' else 'float'}>",
                     "achieved": round(2.0 * len(d) * cfg.n / launch_s / 1e12, 3),
                     "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                     "frac": round(2.0 * len(d) * cfg.n / launch_s / 1e12 / PEAK_TFLOPS[prec], 4),
                     "traffic": None},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lattice60_h4_n2048_m20")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "bf16", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=8)
    ap.add_argument("--no-rr", action="store_true", help="time the filter alone")
    ap.add_argument("--solve", action="store_true",
                    help="run the subspace iteration to convergence instead of timing steps")
    ap.add_argument("--tol", type=float, default=0.0, help="residual tolerance of --solve")
    ap.add_argument("--max-passes", type=int, default=40)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the reduced-precision filters and their Ritz-value errors")
    ap.add_argument("--m-late", default="4,18",
                    help="comma-separated counts of late FP32 / bf16x3 steps of the precision schedules")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint report (forward and backward on the adjoint workload)")
    ap.add_argument("--adjoint-only", default="",
                    help="run only the adjoint report for these iterate types (e.g. f64 or "
                         "f64,f32) and print it as one JSON line")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain device copy of the X block (known bytes) before the timed "
                         "steps, to scale hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the build has no multi-GPU path "
              "(the filter shards by columns with no communication).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2110_15853_amd as P
    import workload

    cfg = workload.CONFIGS[args.workload]
    if args.adjoint_only:
        if args.calib_copy:                 # known bytes for scaling byte counters
            a = torch.ones(64000 * 512, dtype=torch.float64, device="cuda")
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            log(f"calibration copy: {a.numel() * 8} bytes read and written")
            del a, b
        print(json.dumps({"adjoint": adjoint_report(P, torch, workload,
                                                    tuple(args.adjoint_only.split(",")))}))
        return
    log(f"workload {cfg}")
    if args.solve:
        run_solve(args, P, torch, workload)
        return
    if cfg.name == "lattice90_h3_n8000_m24":
        run_large(args, P, torch, workload)
        return
    t0 = time.perf_counter()
    ip, ix, d, N = workload.lattice_hamiltonian(cfg.r, cfg.h, cfg.seed)
    log(f"H generated: N={N} nnz={len(d)} ({time.perf_counter() - t0:.1f} s)")
    hdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
           "bf16x3": "bf16x3"}[args.precision]
    xdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32,
           "bf16x3": torch.float32}[args.precision]
    H = P.bsr_build(ip, ix, d, cfg.r, dtype=hdt, device="cuda")
    log(f"BSR built: {H.n_block_rows} block rows, {H.n_tiles} tiles")
    X = workload.gaussian_block(N, cfg.n, cfg.seed)
    log("X generated")
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), H)
    if xdt != torch.float64:
        Xb = P.cast(Xb, xdt)
    Y = torch.empty_like(Xb)
    work = torch.empty(Xb.numel() * Xb.element_size(), dtype=torch.uint8, device="cuda")
    do_rr = not args.no_rr
    if do_rr:
        H64 = H if args.precision == "f64" else P.bsr_build(ip, ix, d, cfg.r, dtype=torch.float64,
                                                             device="cuda")
        rr_work = torch.empty(P.rayleigh_ritz_workspace(H64, cfg.n, Xb.dtype), dtype=torch.uint8,
                              device="cuda")
    torch.cuda.synchronize()
    log("inputs resident on the GPU")
    rr_out = {}

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        P.cheb_filter(H, Xb, cfg.m, cfg.a, cfg.b, cfg.a0, out=Y, work=work)
        if ev is not None:
            ev[1].record()
        if do_rr:
            rr_out["lam"], rr_out["psi"] = P.rayleigh_ritz(H64, Y, work=rr_work)
            if ev is not None:
                ev[2].record()

    if args.calib_copy:
        calib = torch.empty_like(Xb)
        calib.copy_(Xb)
        torch.cuda.synchronize()
        log(f"calibration copy: {Xb.numel() * Xb.element_size()} bytes read and written")
        del calib

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup}")

    events = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    filt_ms = [ev[0].elapsed_time(ev[1]) for ev in events]
    rr_ms = [ev[1].elapsed_time(ev[2]) for ev in events] if do_rr else []
    log(f"timed {args.steps} steps: wall {wall:.3f} s, filter ms {['%.1f' % v for v in filt_ms]}, "
        f"Rayleigh-Ritz ms {['%.1f' % v for v in rr_ms]}")

    nnz = len(d)
    n = cfg.n
    alg_flops_launch = 2.0 * nnz * n                      # one H*Y_k product
    issued_flops_launch = issued_flops(H, args.precision) * n
    elt = Xb.element_size()
    h_bytes = H.vals.numel() * H.vals.element_size() + 4 * (H.n_tiles + H.n_block_rows + 1)
    alg_bytes_launch = h_bytes + 3.0 * H.rows * n * elt    # read Y_k, Y_{k-1}, write Y_{k+1}
    filt_s = float(np.mean(filt_ms)) / 1e3
    launch_s = filt_s / cfg.m
    value = alg_flops_launch * cfg.m / filt_s / 1e9
    counted = COUNTED_TRAFFIC.get((args.precision, cfg.name))
    traffic = None
    if counted and counted["kernel_sha256_16"] == kernel_source_sha16():
        traffic = counted["read_bytes"] + counted["write_bytes"]
    roofline = step_roofline(args.precision, alg_flops_launch, alg_bytes_launch, launch_s, traffic)
    peak = PEAK_TFLOPS["bf16" if args.precision == "bf16x3" else args.precision]
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16xf32", "bf16x3": "bf16x3xf32"}.get(args.precision, args.precision),
        "data": "synthetic",
        "config": {"workload": cfg.name, "N": N, "rows_blocked": H.rows, "n_vec": n, "m": cfg.m,
                   "h": cfg.h, "nnz": nnz, "tiles": H.n_tiles, "fill": nnz / (H.n_tiles * 4096),
                   "a": cfg.a, "b": cfg.b, "a0": cfg.a0,
                   "step": "chebyshev filter + FP64 Rayleigh-Ritz" if do_rr else "chebyshev filter"},
        "filter_ms": round(filt_s * 1e3, 3),
        "rayleigh_ritz_ms": round(float(np.mean(rr_ms)), 3) if do_rr else None,
        "hbm_gbs_algorithmic": round(alg_bytes_launch / launch_s / 1e9, 1),
        "issued_tflops": round(issued_flops_launch / launch_s / 1e12, 2),
        "issued_frac": round(issued_flops_launch / launch_s / 1e12 / peak, 4),
        "roofline": {**roofline,
                     "per_launch": {"alg_flops": alg_flops_launch, "alg_bytes": alg_bytes_launch,
                                    "issued_flops": issued_flops_launch,
                                    "avg_launch_ms": round(launch_s * 1e3, 4),
                                    "traffic_unit": "bytes (L2-miss reads + writes, counter-calibrated)"}},
    }
    if do_rr and args.precision == "f64":
        out["density"] = density_report(P, torch, H, rr_out["lam"], rr_out["psi"], cfg)
        log(f"density: {out['density']}")
    if not args.no_adjoint and args.precision == "f64" and do_rr:
        out["adjoint"] = adjoint_report(P, torch, workload)
        log(f"adjoint: {out['adjoint']}")
    if not args.no_mixed and args.precision == "f64" and do_rr:
        del rr_work, work
        rr_out.clear()
        torch.cuda.empty_cache()
        out["mixed_vs_f64"] = mixed_precision_report(
            P, torch, ip, ix, d, cfg, H, Xb, m_late=tuple(int(v) for v in args.m_late.split(",") if v))
    if not args.no_cpu_baseline:
        import oracle
        log("CPU baseline (oracle) ...")
        Hc = oracle.csr_from_arrays(ip, ix, d, N)
        out["cpu_baseline"] = cpu_baseline(Hc, X, cfg, args.cpu_cols)
        log("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
