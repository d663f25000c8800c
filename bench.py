#!/usr/bin/env python3
"""Throughput of the selected Green's-function solve on one MI355X.

One step = one qtx_rgf_solve call over the realistic workload: a synthetic
device with n_b = 32 diagonal blocks of size b = 416 (complex128, S = I,
random Hermitian H, eta = 1e-3, contact broadening gamma = 0.5) at all 256
energies of linspace(-2, 2, 256) -- forward and backward passes for G^R and
G^< with every block inversion, inputs resident in HBM.  The metric is energy
points per second.  Precision schemes: fp64 (reference) and the mixed schemes
of the complex block products; `value` is the fastest scheme whose per-block
error against the FP64 oracle on sampled energies is <= 1e-6 and whose error
against FP64 solves of all energies (every output block type, T_L, j_L; the
FP64 solves run again in chunks after the timed region) is <= 1e-6 as well (the
FP64 path always qualifies; it is itself checked against the oracle on the
sample), and every scheme's rate and error is reported beside it.  If no scheme
qualifies, the line carries "meets_tolerance": false.

Also reported:
  roofline     the dominant kernel (the b x b x b complex block products),
               algorithmic flops per launch / average launch duration, both from
               HIP events recorded by the library on the launch stream
  cpu_baseline the FP64 oracle (numpy/LAPACK) on the host cores, on a bounded
               sample of the same workload's energies, in energy points per second
  p50/p99_latency_ms  per-solve latency of the K back-to-back timed solves (HIP
               events on the solve's stream); request latency under load is the
               serve workload's, one-energy latency the latency workload's

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precs fp64,...]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RGF energy points/sec: mixed-prec vs FP64 at rel err ≤1e-6; p50/p99 latency"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "int8": 5000.0}   # dense TFLOP/s (TOP/s), MI355X
TOL_MIXED = 1e-6
# rocprofv3 --pmc summaries of each scheme's product kernel on the realistic workload,
# with the kernel source they were taken on
PMC = {"fp64": ("zgemm_f64_product_realistic_pmc.md", "zgemm_mfma.hip"),
       "int8": ("zgemm_o2_product_realistic_pmc.md", "zgemm_ozaki2.hip")}


def parse_scheme(spec):
    """"fp64", "bf16:5", "int8:11", or "<retarded>/<lesser>", e.g. "int8:10/int8:11"."""
    parts = spec.split("/")

    def one(p):
        name, _, ns = p.partition(":")
        return name, int(ns or 0)
    r = one(parts[0])
    kw = dict(prec=r[0], n_slices=r[1])
    if len(parts) > 1:
        lsr = one(parts[1])
        kw.update(prec_lesser=lsr[0], n_slices_lesser=lsr[1])
    return kw


def autotune(ctx, skw, shapes):
    """Autotuner pass (outside any timed region): for each scheme of `skw` (retarded
    and lesser chain) and each (b, batch) in `shapes`, time the product kernel's tile
    variants (INT8: 14 tile shapes; FP64, FP32, split: 32 x 32 or 64 x 64 tiles) and
    keep the fastest in the context."""
    out = {}
    chains = [(skw["prec"], skw.get("n_slices", 0))]
    if skw.get("prec_lesser"):
        chains.append((skw["prec_lesser"], skw.get("n_slices_lesser", 0)))
    for prec, ns in sorted(set(chains)):
        for b, batch in shapes:
            v, ms = ctx.tune(b, prec, ns, batch=batch)
            out["%s:%d b=%d batch=%d" % (prec, ns, b, batch)] = {"variant": v, "ms_per_product": [round(t, 4) for t in ms]}
            log("bench: autotune %s:%d b=%d batch=%d -> variant %d (%s ms)" % (prec, ns, b, batch, v,
                                                                                 " ".join("%.3f" % t for t in ms)))
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(src):
    with open(os.path.join(ROOT, "paper_2606_25595_amd", "csrc", src), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_from_profile(scheme, variant=None):
    """HBM bytes per product-kernel launch from the committed rocprofv3 --pmc
    summary, if it was taken for this scheme and tile variant on the current kernel
    source (else None)."""
    prec = parse_scheme(scheme)["prec"]
    if prec not in PMC:
        return None
    fname, src = PMC[prec]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash(src) or kv.get("scheme") != scheme:
        return None
    try:
        if variant is not None and "hbm_bytes_per_launch_variant_%d" % variant in kv:
            return float(kv["hbm_bytes_per_launch_variant_%d" % variant])
        if "tile_variant" in kv and variant is not None and int(kv["tile_variant"]) != variant:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_one_energy(args):
    """Process-pool worker of the CPU baseline: the FP64 oracle on one energy of a named
    workload with one BLAS thread; returns (start, end) wall-clock times of the oracle
    call (the problem is built before the clock starts)."""
    name, e, eta = args
    from threadpoolctl import threadpool_limits
    import oracle
    from paper_2606_25595_amd import inputs
    p = inputs.config_problem(name, energy_index=[e], eta=eta)
    with threadpool_limits(1):
        t0 = time.time()
        oracle.rgf_selected(p)
        t1 = time.time()
    return t0, t1


def host_cores():
    """CPU cores this process may use (its affinity mask), at most 16 (one GPU's share
    of the host's cores on an eight-GPU node)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_pool_rate(name, energies, eta, workers):
    """Energy points/s of the oracle run as a process pool over the energies, one BLAS
    thread per process (wall time from the first oracle start to the last end)."""
    import multiprocessing as mp
    ctxp = mp.get_context("spawn")
    with ctxp.Pool(workers) as pool:
        spans = pool.map(_oracle_one_energy, [(name, e, eta) for e in energies], chunksize=1)
    wall = max(t1 for _, t1 in spans) - min(t0 for t0, _ in spans)
    return len(energies) / wall, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precs", default="fp64,fp32,bf16:5,int8:11,int8:10/int8:11,int8:10/int8:10",
                    help="comma list of schemes: fp64 | fp32 | bf16:NS | fp16:NS | int8:P (P moduli) | "
                         "<retarded>/<lesser>")
    ap.add_argument("--cpu-energies", type=int, default=16, help="energies in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-full-check", action="store_true",
                    help="skip the all-energy error check of the mixed schemes (then none qualifies)")
    ap.add_argument("--workload", default="realistic",
                    choices=["realistic", "hard", "kappa", "w", "fpx", "batch", "serve", "latency", "tiny", "memory",
                             "longchain", "products"],
                    help="realistic (default, the headline line) | hard (the realistic shapes at eta = 1e-6, "
                         "condition numbers up to ~5e6) | kappa (error against the exact condition number, "
                         "n_b=8, b=128, eta 1e-3..1e-6) | w (screened Coulomb system: assembly + solve, n_b=16, "
                         "b=256, 128 energies) | fpx (FPX storage codec GB/s on G^R blocks) | batch (512 uneven "
                         "problems, one graph launch) | "
                         "serve (Poisson arrivals, continuous batching, p50/p99) | latency (few energies) | "
                         "tiny (n_b=8, b=16, 32 energies; both CPU oracles) | memory (energies resident per GPU "
                         "under dense / diagonal Sigma and complex128 / FPX32 outputs) | longchain (latency of "
                         "few energies on a long device: one chain, split, P-way partitions) | products (INT8 "
                         "product kernel per tile variant, operands per entry or shared by the whole batch)")
    ap.add_argument("--workspace-gb", type=float, default=0.0,
                    help="realistic/hard: library workspace cap in GiB (0 = a quarter of free HBM)")
    ap.add_argument("--split", action="store_true",
                    help="realistic/hard/serve: two half-chains per energy (QTX_SPLIT_CHAIN)")
    ap.add_argument("--eta", type=float, default=None, help="realistic/hard: broadening (default 1e-3 / 1e-6)")
    ap.add_argument("--latency-ne", default="1,2,4,8,16,32", help="latency workload: energy counts")
    ap.add_argument("--latency-precs", default="fp64,int8:10/int8:10", help="latency workload: schemes")
    ap.add_argument("--latency-split", default="0,1", help="latency workload: 0 = one chain, 1 = split")
    ap.add_argument("--problems", type=int, default=512, help="batch workload: number of problems")
    ap.add_argument("--rate", type=float, default=200.0, help="serve workload: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serve workload: arrival window (s)")
    ap.add_argument("--time-limit", type=float, default=150.0, help="serve workload: wall-clock cap (s)")
    ap.add_argument("--serve-slots", type=int, default=3, help="serve workload: launches in flight (library contexts)")
    ap.add_argument("--serve-chunk", type=int, default=16, help="serve workload: energies per chunk")
    ap.add_argument("--serve-policy", default="fifo", choices=["fifo", "sjf"],
                    help="serve workload: admission order (arrival order, or least work first with aging)")
    ap.add_argument("--serve-compact", type=int, default=0,
                    help="serve workload: X in 16..56 stores the self-energies as b-vectors and the off-diagonal "
                         "outputs as FPX X-bit bytes (0: dense complex128)")
    ap.add_argument("--prec", default="fp64", help="batch workload scheme (fp64 | int8:11 | int8:10/int8:11 | ...)")
    ap.add_argument("--int8-variant", type=int, default=-1,
                    help="realistic workload: force this INT8 product tile variant after the tuner ran (-1: the "
                         "tuner's choice; counter runs use it, since a profiler's serialisation perturbs the "
                         "tuner's timings)")
    ap.add_argument("--mem-prec", default="int8:10/int8:10", help="memory workload scheme")
    ap.add_argument("--long-nb", type=int, default=128, help="longchain workload: blocks of the device")
    ap.add_argument("--long-ne", default="1,4", help="longchain workload: energy counts")
    ap.add_argument("--long-modes", default="chain,split,p2,p4,p8,p16",
                    help="longchain workload: chain | split | pP (P-way partitions)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: energies shard across GPUs with no exchange inside a solve, "
              "so the per-GPU rate is the single-GPU figure; multi-GPU runs are not supported.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2606_25595_amd import inputs, qtx

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "kappa":
        return bench_kappa(args)
    if args.workload == "w":
        return bench_w(args)
    if args.workload == "fpx":
        return bench_fpx(args)
    if args.workload == "latency":
        return bench_latency(args)
    if args.workload == "tiny":
        return bench_tiny(args)
    if args.workload == "memory":
        return bench_memory(args)
    if args.workload == "longchain":
        return bench_longchain(args)
    if args.workload == "products":
        return bench_products(args)

    cfg = inputs.CONFIGS["realistic"]
    n_b, b, n_e = cfg["n_b"], cfg["b"], cfg["n_e"]
    eta = args.eta if args.eta is not None else (1e-6 if args.workload == "hard" else 1e-3)
    sample = list(range(0, n_e, max(1, n_e // args.cpu_energies)))[: args.cpu_energies]
    pool = None
    if not args.no_cpu:
        # the oracle as a process pool (one BLAS thread per process), started before this
        # process touches the GPU
        workers = host_cores()
        log("bench: oracle process pool, %d workers, %d energies" % (workers, len(sample)))
        rate, wall = oracle_pool_rate("realistic", sample, eta, workers)
        pool = {"value": rate, "cores": workers, "wall_s": wall}
    gamma, mu_L, kT = 0.5, 0.1, 0.025
    grid = np.linspace(-2.0, 2.0, n_e)
    log("bench: building realistic workload n_b=%d b=%d n_e=%d eta=%g on the device" % (n_b, b, n_e, eta))
    d = inputs.device_random_problem(n_b, b, grid, seed=0, eta=eta)
    kw = dict(dtype=torch.complex128, device="cuda")
    dp = qtx.DeviceProblem(energies=d["energies"], H_d=d["H_d"], H_u=d["H_u"], H_l=d["H_l"], SR_d=d["SR_d"],
                           SL_d=d["SL_d"], GR_d=torch.empty((n_e, n_b, b, b), **kw),
                           GR_u=torch.empty((n_e, n_b - 1, b, b), **kw), GR_l=torch.empty((n_e, n_b - 1, b, b), **kw),
                           GL_d=torch.empty((n_e, n_b, b, b), **kw), GL_u=torch.empty((n_e, n_b - 1, b, b), **kw),
                           status=torch.full((n_e,), -1, dtype=torch.int32, device="cuda"), split=args.split)
    ctx = qtx.Context(0, workspace_bytes=int(args.workspace_gb * (1 << 30)))
    gamma_L = 2.0 * gamma * np.eye(b, dtype=np.complex128)
    f_L = inputs.fermi(grid, mu_L, kT)
    kappa = None

    # ---- CPU oracle on the sample (also the parity reference for the sampled outputs)
    ref = None
    cpu = None
    if not args.no_cpu:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            threads = max([t.get("num_threads", 1) for t in threadpool_info() if t.get("user_api") == "blas"] or [1])
        except Exception:
            threads = os.cpu_count() or 1
        p_s = inputs.config_problem("realistic", energy_index=sample, eta=eta)
        log("bench: oracle on %d sampled energies (%d BLAS threads)" % (len(sample), threads))
        t0 = time.perf_counter()
        ref = oracle.rgf_selected(p_s)
        t_cpu = time.perf_counter() - t0
        ref["T_L"] = oracle.transmission_left(ref["GR_d"][:, 0], p_s.gamma_L)
        ref["j_L"] = oracle.contact_current_left(ref["GR_d"][:, 0], ref["GL_d"][:, 0], p_s.gamma_L, p_s.f_L)
        kappa = kappa_bounds(p_s, ref, eta) if args.workload == "hard" else None
        seq = {"value": len(sample) / t_cpu, "cores": int(threads), "wall_s": t_cpu}
        best = "pool" if pool and pool["value"] > seq["value"] else "threads"
        top = pool if best == "pool" else seq
        cpu = {"value": top["value"], "unit": "energy points/s", "cores": int(top["cores"]), "kind": "oracle",
               "sample": "%d of the 256 energies (every %dth) of the realistic workload, block recurrences in "
                         "numpy/LAPACK FP64; faster of: one energy at a time on %d BLAS threads (%.1f s), a pool of "
                         "%d processes with one BLAS thread each (%s)"
                         % (len(sample), n_e // len(sample), seq["cores"], seq["wall_s"],
                            pool["cores"] if pool else 0, ("%.1f s" % pool["wall_s"]) if pool else "not run"),
               "mode": best, "modes": {"threads": seq, "pool": pool},
               "host_cpus": os.cpu_count(), "host_cpus_usable": host_cores()}

    results = {}
    tuned = {}
    KEYS = ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")
    chunk_e = 32

    def full_errors():
        """Error of the current outputs over ALL energies against FP64 solves of the same
        energies, run again here in chunks of 32 energies (every output block type:
        max relative Frobenius error per (energy, block); T_L and j_L relative to their
        largest magnitude over all energies).  Outside the timed region."""
        worst = {k: 0.0 for k in KEYS}
        dT = dj = mT = mj = 0.0
        sub = None
        for e0 in range(0, n_e, chunk_e):
            e1 = min(n_e, e0 + chunk_e)
            c = e1 - e0
            if sub is None or sub.n_e != c:
                sub = qtx.DeviceProblem(
                    energies=grid[e0:e1], H_d=dp.H_d, H_u=dp.H_u, H_l=dp.H_l, SR_d=dp.SR_d[e0:e1],
                    SL_d=dp.SL_d[e0:e1], GR_d=torch.empty((c, n_b, b, b), **kw),
                    GR_u=torch.empty((c, n_b - 1, b, b), **kw), GR_l=torch.empty((c, n_b - 1, b, b), **kw),
                    GL_d=torch.empty((c, n_b, b, b), **kw), GL_u=torch.empty((c, n_b - 1, b, b), **kw),
                    status=torch.full((c,), -1, dtype=torch.int32, device="cuda"))
            sub.energies = grid[e0:e1]
            sub.SR_d, sub.SL_d = dp.SR_d[e0:e1], dp.SL_d[e0:e1]
            ctx.solve(sub, prec="fp64")
            for key in KEYS:
                X, R = getattr(dp, key)[e0:e1], getattr(sub, key)
                d = (X - R).abs().pow(2).sum((-1, -2)).sqrt()
                nr = R.abs().pow(2).sum((-1, -2)).sqrt()
                worst[key] = max(worst[key], float((d / nr.clamp_min(1e-300)).max().item()))
            Tr, jr = ctx.observables(sub, gamma_L, f_L[e0:e1])
            Tg, jg = ctx.observables_blocks(dp.GR_d[e0:e1], dp.GL_d[e0:e1], gamma_L, f_L[e0:e1])
            dT = max(dT, float((Tg - Tr).abs().max().item()))
            dj = max(dj, float((jg - jr).abs().max().item()))
            mT = max(mT, float(Tr.abs().max().item()))
            mj = max(mj, float(jr.abs().max().item()))
        worst["T_L"] = dT / max(mT, 1e-300)
        worst["j_L"] = dj / max(mj, 1e-300)
        return worst
    for prec in args.precs.split(","):
        skw = parse_scheme(prec)
        tuned.update(autotune(ctx, skw, [(b, n_e)]))
        if args.int8_variant >= 0:
            ctx.set_int8_tile_variant(args.int8_variant)
            log("bench: INT8 tile variant forced to %d" % args.int8_variant)
        log("bench: %s warmup x%d" % (prec, args.warmup))
        for _ in range(args.warmup):
            ctx.solve(dp, **skw)
        torch.cuda.synchronize()
        ctx.profile(True)
        for fam in (qtx.QTX_KERNEL_GEMM, qtx.QTX_KERNEL_INV, qtx.QTX_KERNEL_CONVERT):
            ctx.profile_read(fam)
        log("bench: %s timed x%d" % (prec, args.steps))
        # one event after each solve on the solve's stream: per-solve latency of back-to-back
        # solves (recording events does not synchronise the host)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record()
        for k in range(args.steps):
            ctx.solve(dp, **skw)
            evs[k + 1].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.profile(False)
        lat_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
        g_ms, g_n, g_fl = ctx.profile_read(qtx.QTX_KERNEL_GEMM)
        i_ms, i_n, i_fl = ctx.profile_read(qtx.QTX_KERNEL_INV)
        c_ms, c_n, c_by = ctx.profile_read(qtx.QTX_KERNEL_CONVERT)
        ms_step = (t1 - t0) * 1e3 / args.steps
        st = dp.status.cpu().numpy()
        errs = None
        if ref is not None:
            import oracle
            errs = {}
            for key in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u"):
                got = getattr(dp, key)[sample].cpu().numpy()
                errs[key] = float(oracle.rel_fro_err(got, ref[key]).max())
            # observables from the library's own kernel on the GPU outputs; error relative
            # to the largest magnitude over the sample
            T, j = ctx.observables(dp, gamma_L, f_L)
            for key, got in (("T_L", T), ("j_L", j)):
                g = got.cpu().numpy()[sample]
                errs[key] = float(np.abs(g - ref[key]).max() / max(np.abs(ref[key]).max(), 1e-300))
        errs_full = None
        if prec != "fp64" and not args.no_full_check:
            log("bench: %s all-energy check against chunked FP64 solves" % prec)
            errs_full = full_errors()
        results[prec] = dict(ms_per_step=ms_step, value=n_e / (ms_step / 1e3), status_ok=bool(np.all(st == 0)),
                             gemm=(g_ms, g_n, g_fl), inv=(i_ms, i_n, i_fl), conv=(c_ms, c_n, c_by), errs=errs,
                             errs_full=errs_full,
                             latency_ms={"p50": float(np.percentile(lat_ms, 50)),
                                         "p99": float(np.percentile(lat_ms, 99)), "solves": len(lat_ms)})
        log("bench: %s %.1f ms/step, %.1f energies/s, product kernel avg %.3f ms x%d, conversion %.1f ms/step, "
            "inv avg %.3f ms x%d, err %s, all-energy err vs fp64 %s" % (
                prec, ms_step, n_e / (ms_step / 1e3), g_ms / max(g_n, 1), g_n, c_ms / args.steps,
                i_ms / max(i_n, 1), i_n, errs, errs_full))

    # headline: fastest scheme meeting the error bar (FP64 always qualifies)
    def qualifies(p):
        r = results[p]
        if not r["status_ok"]:
            return False
        if p == "fp64":
            return True
        if r["errs"] is None or max(r["errs"].values()) > TOL_MIXED:
            return False
        # every output block type and the observables over all energies, too
        return r["errs_full"] is not None and max(r["errs_full"].values()) <= TOL_MIXED
    # without the oracle (--no-cpu) or the all-energy check no mixed scheme qualifies:
    # the line then reports the fastest scheme that ran, flagged meets_tolerance = false
    qual = [p for p in results if qualifies(p)]
    cands = qual or [p for p in results if results[p]["status_ok"]] or list(results)
    best = max(cands, key=lambda p: results[p]["value"])
    r = results[best]
    g_ms, g_n, g_fl = r["gemm"]
    achieved = (g_fl / max(g_n, 1)) / (g_ms / max(g_n, 1) / 1e3) / 1e12 if g_n else None
    peak = PEAK[parse_scheme(best)["prec"]]
    bsk = parse_scheme(best)
    if bsk["prec"] == "int8" and args.int8_variant >= 0:
        variant = args.int8_variant
    else:
        variant = tuned.get("%s:%d b=%d batch=%d" % (bsk["prec"], bsk.get("n_slices", 0), b, n_e), {}).get("variant")
    traffic = traffic_from_profile(best, variant)
    kernel_name = {"fp64": "zgemm_mfma_kernel (v_mfma_f64_16x16x4)", "fp32": "zgemm_mfma_kernel (v_mfma_f32)",
                   "bf16": "zgemm_split_kernel (v_mfma_f32_16x16x32_bf16)",
                   "fp16": "zgemm_split_kernel (v_mfma_f32_16x16x32_f16)",
                   "int8": "zgemm_o2_kernel (v_mfma_i32_32x32x32_i8)"}[parse_scheme(best)["prec"]]
    gemm_fp64eq = (136 * (n_b - 1) + 16) * b ** 3 * n_e   # FP64-equivalent product flops per step
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "energy points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "f64+" + best.replace(":", "x"),
        "data": "synthetic",
        "config": {"workload": "%sselected RGF solve: n_b=32 blocks, b=416, N_E=256 energies in [-2,2], "
                               "complex128, S=I, random Hermitian H (seed 0), eta=%g, gamma=0.5"
                               % ("realistic " if args.workload == "realistic" else "hard (ill-conditioned) ", eta),
                   "precision": best, "energies_per_step": n_e, "split_chain": bool(args.split),
                   "workspace_gb": args.workspace_gb or None},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": (achieved / peak) if achieved else None, "traffic": traffic,
                     "kernel": "%s: matrix-core kernel of the complex b x b x b block products (%s scheme); "
                               "operations counted in its own arithmetic" % (kernel_name, best),
                     "flops_per_launch": g_fl / max(g_n, 1), "avg_launch_ms": g_ms / max(g_n, 1),
                     "launches": g_n},
        "cpu_baseline": cpu,
        "meets_tolerance": best in qual,
        "p50_latency_ms": r["latency_ms"]["p50"], "p99_latency_ms": r["latency_ms"]["p99"],
        "latency": "one solve of all energies of the step, back to back (HIP events on the solve's stream)",
        "schemes": {p: {"energies_per_s": v["value"], "ms_per_step": v["ms_per_step"], "max_rel_err": v["errs"],
                        "max_rel_err_all_energies_vs_fp64": v["errs_full"],
                        "status_ok": v["status_ok"], "solve_latency_ms": v["latency_ms"],
                        "products_tflops_fp64eq": gemm_fp64eq * args.steps / ((v["gemm"][0] + v["conv"][0]) / 1e3)
                        / 1e12 if v["gemm"][1] else None,
                        "product_kernel_ms_per_step": v["gemm"][0] / args.steps,
                        "product_kernel_rate_own_arith": (v["gemm"][2] / (v["gemm"][0] / 1e3) / 1e12)
                        if v["gemm"][1] else None,
                        "conversion_ms_per_step": v["conv"][0] / args.steps,
                        "conversion_GBps": (v["conv"][2] / (v["conv"][0] / 1e3) / 1e9) if v["conv"][1] else None,
                        "inversion_ms_per_step": v["inv"][0] / args.steps}
                    for p, v in results.items()},
        "fp64_energies_per_s": results["fp64"]["value"] if "fp64" in results else None,
        "autotune": tuned,
        "algorithmic_tflops_fp64eq": (144 * (n_b - 1) + 24) * b ** 3 * n_e / (r["ms_per_step"] / 1e3) / 1e12,
    }
    if kappa is not None:
        line["kappa_sampled"] = kappa
    print(json.dumps(line), flush=True)
    ctx.close()


def _spec_norm(mv, rmv, n, iters=40, seed=0):
    """Largest singular value of the operator x -> mv(x) by power iteration on
    rmv(mv(.)) (a lower bound that converges from below)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x /= np.linalg.norm(x)
    s = 0.0
    for _ in range(iters):
        y = rmv(mv(x))
        s = np.sqrt(np.linalg.norm(y))
        x = y / np.linalg.norm(y)
    return float(s)


def kappa_bounds(p, ref, eta):
    """Bounds on the 2-norm condition number of M(E) = E - H - Sigma^R at the
    sampled energies: sigma_min(M) >= eta (the anti-Hermitian part of M is at
    least eta), so kappa <= ||M|| / eta; and ||M^-1|| >= max_i ||G^R_ii||, so
    kappa >= ||M|| max_i ||G^R_ii||.  Norms by power iteration."""
    import numpy as np
    n_b, b = p.n_b, p.b
    lo, hi = [], []
    for k in range(p.n_e):
        E = p.energies[k]
        D = [E * np.eye(b) - p.H_d[i] - p.SR_d[k, i] for i in range(n_b)]
        U = [-p.H_u[i] for i in range(n_b - 1)]
        L = [-p.H_l[i] for i in range(n_b - 1)]

        def mv(x, D=D, U=U, L=L, adj=False):
            X = x.reshape(n_b, b)
            Y = np.empty_like(X)
            for i in range(n_b):
                y = (D[i].conj().T if adj else D[i]) @ X[i]
                if i + 1 < n_b:
                    y = y + ((L[i].conj().T if adj else U[i]) @ X[i + 1])
                if i > 0:
                    y = y + ((U[i - 1].conj().T if adj else L[i - 1]) @ X[i - 1])
                Y[i] = y
            return Y.reshape(-1)
        nM = _spec_norm(mv, lambda x: mv(x, adj=True), n_b * b)
        g = max(_spec_norm(lambda x, G=G: G @ x, lambda x, G=G: G.conj().T @ x, b, iters=30)
                for G in ref["GR_d"][k])
        lo.append(nM * g)
        hi.append(nM / eta)
    return {"lower_max": max(lo), "lower_min": min(lo), "upper": max(hi),
            "note": "kappa_2(M) per sampled energy lies in [||M|| max_i ||G^R_ii||, ||M||/eta]"}


def bench_kappa(args):
    """Error of each scheme against the exact 2-norm condition number of M(E)
    (singular values of the dense matrix), as the paper relates emulation error to
    conditioning.  The synthetic device with n_b = 8, b = 128 (N = 1024) is closed
    (no contact broadening, gamma = 0), so that sigma_min(M) is set by eta alone at
    an eigenvalue of H: 4 energies are eigenvalues of H (kappa ~ ||M|| / eta) and 4
    lie on the grid linspace(-1.9, 1.9, 4), for eta = 1e-2 ... 1e-7.  Reference: the
    FP64 oracle's block recurrences."""
    import numpy as np
    import torch
    import oracle
    from paper_2606_25595_amd import inputs, qtx
    n_b, b = 8, 128
    H_d, H_u, H_l = inputs.random_hamiltonian(n_b, b, 0)
    Hd = np.zeros((n_b * b, n_b * b), complex)
    for i in range(n_b):
        Hd[i * b:(i + 1) * b, i * b:(i + 1) * b] = H_d[i]
        if i + 1 < n_b:
            Hd[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = H_u[i]
            Hd[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = H_l[i]
    lam = np.linalg.eigvalsh(Hd)
    on = np.array([lam[np.argmin(np.abs(lam - x))] for x in np.linspace(-1.5, 1.5, 4)])
    grid = np.concatenate([on, np.linspace(-1.9, 1.9, 4)])
    n_e = grid.size
    precs = args.precs.split(",")
    ctx = qtx.Context(0)
    rows = []
    for eta in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
        p = inputs.random_bt_problem(n_b, b, grid, seed=0, eta=eta, gamma=0.0)
        ref = oracle.rgf_selected(p)
        kap = np.array([(lambda s: s[0] / s[-1])(np.linalg.svd(oracle.assemble_dense(p, e)[0], compute_uv=False))
                        for e in range(n_e)])
        kap_s = np.array([max(np.linalg.cond(S) for S in oracle.schur_complements(p, e)) for e in range(n_e)])
        dp = qtx.to_device(p)
        for prec in precs:
            ctx.solve(dp, **parse_scheme(prec))
            torch.cuda.synchronize()
            out = dp.outputs()
            for e in range(n_e):
                err = {k: float(oracle.rel_fro_err(out[k][e], ref[k][e]).max())
                       for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")}
                rows.append({"eta": eta, "E": float(grid[e]), "on_eigenvalue": bool(e < 4), "kappa": float(kap[e]),
                             "kappa_schur": float(kap_s[e]), "scheme": prec, "err": err})
        log("bench kappa: eta=%g kappa(M) %.2e .. %.2e, max_i kappa(S_i) %.2e .. %.2e" % (
            eta, kap.min(), kap.max(), kap_s.min(), kap_s.max()))
    ctx.close()
    # error envelope per scheme and decade of kappa(M), then of max_i kappa(S_i)
    def envelope(kkey):
        table = {}
        for r in rows:
            dec = int(np.floor(np.log10(r[kkey])))
            key = "%s|1e%d" % (r["scheme"], dec)
            t = table.setdefault(key, {"scheme": r["scheme"], "decade": "1e%d" % dec, "n": 0,
                                       "max_err_GR": 0.0, "max_err_GL": 0.0})
            t["n"] += 1
            t["max_err_GR"] = max(t["max_err_GR"], r["err"]["GR_d"], r["err"]["GR_u"], r["err"]["GR_l"])
            t["max_err_GL"] = max(t["max_err_GL"], r["err"]["GL_d"], r["err"]["GL_u"])
        env = sorted(table.values(), key=lambda t: (t["scheme"], float(t["decade"])))
        for t in env:
            log("bench kappa: %-18s %s~%-5s (%2d points): G^R %.2e  G^< %.2e" % (
                t["scheme"], kkey, t["decade"], t["n"], t["max_err_GR"], t["max_err_GL"]))
        return env
    env = envelope("kappa")
    env_s = envelope("kappa_schur")
    line = {"metric": "max relative error per block type against the exact condition number of M(E)",
            "unit": "relative Frobenius error", "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "kappa: closed device n_b=8, b=128, 4 energies on eigenvalues of H + 4 on "
                                   "linspace(-1.9,1.9,4), eta in {1e-2..1e-7}, gamma=0, seed 0"},
            "envelope_kappa_M": env, "envelope_kappa_schur": env_s, "points": rows}
    print(json.dumps(line), flush=True)


def bench_w(args):
    """Screened Coulomb (W) system, the W row of Table I: per step, qtx_w_assemble
    (BT blocks of V P^R and V P^< V^H) and qtx_rgf_solve of the assembled system, for
    n_b = 16 blocks of b = 256 at 128 energies in [-2, 2].  V, P0 and K come from
    inputs.w_base_matrices (seed 0); the per-energy P^R = a(E) P0 - i g(E) K and
    P^< = -f (P^R - P^A) are built on the device.  Errors on 4 sampled energies
    against the FP64 oracle (dense assembly, block recurrences) on the same inputs."""
    import numpy as np
    import torch
    import oracle
    from paper_2606_25595_amd import inputs, qtx
    n_b, b, n_e = 16, 256, 128
    E = np.linspace(-2.0, 2.0, n_e)
    V_d, V_u, (P0_d, P0_u, P0_l), (K_d, K_u) = inputs.w_base_matrices(n_b, b, 0)
    a, g, f = inputs.w_scalars(E)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    A = dev(a).view(-1, 1, 1, 1)
    G = dev(g.astype(np.complex128)).view(-1, 1, 1, 1)
    F = dev(f.astype(np.complex128)).view(-1, 1, 1, 1)
    K_l = np.conj(np.transpose(K_u, (0, 2, 1)))
    PR = [A * dev(P)[None] - 1j * G * dev(Kx)[None] for P, Kx in ((P0_d, K_d), (P0_u, K_u), (P0_l, K_l))]
    Hh = lambda X: X.conj().transpose(-1, -2)
    PL_d = -F * (PR[0] - Hh(PR[0]))
    PL_u = -F * (PR[1] - Hh(PR[2]))
    dw = qtx.DeviceW(n_e=n_e, V_d=dev(V_d), V_u=dev(V_u), PR_d=PR[0].contiguous(), PR_u=PR[1].contiguous(),
                     PR_l=PR[2].contiguous(), PL_d=PL_d.contiguous(), PL_u=PL_u.contiguous())
    torch.cuda.synchronize()
    sample = [0, 43, 85, 127]
    log("bench w: oracle on %d sampled energies" % len(sample))
    host = lambda t: t[sample].cpu().numpy()
    w_s = inputs.WProblem(energies=E[sample], V_d=V_d, V_u=V_u, PR_d=host(dw.PR_d), PR_u=host(dw.PR_u),
                          PR_l=host(dw.PR_l), PL_d=host(dw.PL_d), PL_u=host(dw.PL_u),
                          PL_l=-np.conj(np.swapaxes(host(dw.PL_u), -1, -2)))
    t0 = time.perf_counter()
    ref = oracle.w_selected(w_s, "rgf")
    t_cpu = time.perf_counter() - t0
    ctx = qtx.Context(0)
    results = {}
    for spec in args.precs.split(","):
        asm_prec, _, solve_spec = spec.partition("+")      # "<assembly scheme>+<solve scheme>"
        akw = parse_scheme(asm_prec)
        skw = parse_scheme(solve_spec or asm_prec)
        autotune(ctx, skw, [(b, n_e)])
        autotune(ctx, akw, [(b, n_e)])

        def step():
            asm = ctx.w_assemble(dw, prec=akw["prec"], n_slices=akw.get("n_slices", 0))
            dp = ctx.w_problem(dw, asm)
            ctx.solve(dp, **skw)
            return dp
        for _ in range(args.warmup):
            dp = step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dp = step()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        out = {k: getattr(dp, k)[sample].cpu().numpy() for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")}
        errs = {k: float(oracle.rel_fro_err(out[k], ref[k]).max()) for k in out}
        results[spec] = {"energies_per_s": n_e / t, "ms_per_step": t * 1e3, "max_rel_err": errs,
                         "status_ok": bool((dp.status == 0).all().item())}
        log("bench w: %s %.1f ms/step, %.1f energies/s, err %s" % (spec, t * 1e3, n_e / t, errs))
        del dp
    ctx.close()
    ok = [k for k, v in results.items() if v["status_ok"] and max(v["max_rel_err"].values()) <= TOL_MIXED]
    best = max(ok or list(results), key=lambda k: results[k]["energies_per_s"])
    line = {"metric": "W-system energy points/sec (assembly + selected solve) at rel err <= 1e-6",
            "value": results[best]["energies_per_s"], "unit": "energy points/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": results[best]["ms_per_step"], "higher_is_better": True,
            "dtype": "f64" if best == "fp64" else "f64+" + best, "data": "synthetic",
            "config": {"workload": "w: screened Coulomb system, n_b=16, b=256, 128 energies in [-2,2], seed 0",
                       "precision": best},
            "schemes": results,
            "cpu_baseline": {"value": len(sample) / t_cpu, "unit": "energy points/s", "kind": "oracle",
                             "sample": "%d energies, dense assembly + block recurrences, %.1f s" % (len(sample), t_cpu)}}
    print(json.dumps(line), flush=True)


def bench_fpx(args):
    """FPX storage codec (Section V-A): encode and decode of the diagonal G^R blocks
    of 64 energies of the realistic workload's shape (64 x 32 x 416 x 416 complex128,
    5.67 GB, values of a synthetic spread over the FP32 range), for every X.  HBM
    roofline: algorithmic bytes = 8 read + X/8 written per value (encode), the
    reverse for decode; each launch timed by HIP events on its stream.  The oracle
    checks a sample bitwise."""
    import numpy as np
    import torch
    import oracle
    from paper_2606_25595_amd import qtx
    n_vals = 64 * 32 * 416 * 416 * 2
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x = torch.randn(n_vals, dtype=torch.float64, device="cuda", generator=g)
    x.mul_(torch.pow(10.0, torch.randint(-30, 30, (n_vals,), device="cuda", generator=g).double()))
    ctx = qtx.Context(0)
    rows = {}
    y = torch.empty_like(x)
    for bits in (16, 24, 32, 40, 48, 56):
        enc = torch.empty(n_vals * bits // 8, dtype=torch.uint8, device="cuda")
        ctx.fpx_encode(x, bits, out=enc)
        ctx.fpx_decode(enc, bits, n_vals, out=y)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        te = td = 0.0
        for _ in range(args.steps):
            ev[0].record()
            ctx.fpx_encode(x, bits, out=enc)
            ev[1].record()
            ctx.fpx_decode(enc, bits, n_vals, out=y)
            ev[2].record()
            torch.cuda.synchronize()
            te += ev[0].elapsed_time(ev[1]) / args.steps
            td += ev[1].elapsed_time(ev[2]) / args.steps
        nbytes = n_vals * (8 + bits // 8)
        ok_e = np.array_equal(enc[: 8 * 4096 * bits // 8].cpu().numpy(),
                              oracle.fpx_encode(x[: 8 * 4096].cpu().numpy(), bits))
        rows[bits] = {"encode_ms": te, "decode_ms": td, "encode_GBps": nbytes / te / 1e6,
                      "decode_GBps": nbytes / td / 1e6, "sample_bitwise_ok": bool(ok_e),
                      "max_rel_roundtrip": float(((y - x).abs() / x.abs()).max().item())}
        log("bench fpx: X=%d encode %.3f ms (%.0f GB/s), decode %.3f ms (%.0f GB/s), sample ok %s, "
            "max rel round trip %.2e" % (bits, te, rows[bits]["encode_GBps"], td, rows[bits]["decode_GBps"], ok_e,
                                         rows[bits]["max_rel_roundtrip"]))
        del enc
    ctx.close()
    best = max(rows, key=lambda k: rows[k]["encode_GBps"])
    line = {"metric": "FPX codec HBM throughput (encode + decode of complex128 blocks)", "unit": "GB/s",
            "value": min(min(r["encode_GBps"], r["decode_GBps"]) for r in rows.values()), "n_gpus": 1,
            "higher_is_better": True, "data": "synthetic",
            "config": {"workload": "fpx: 64 x 32 blocks of 416 x 416 complex128 (5.67 GB of FP64)"},
            "roofline": {"bound": "hbm", "peak": 8000.0, "unit": "GB/s",
                         "achieved": rows[best]["encode_GBps"], "frac": rows[best]["encode_GBps"] / 8000.0,
                         "kernel": "fpx_encode_kernel<%d>" % best},
            "formats": rows}
    print(json.dumps(line), flush=True)


def bench_memory(args):
    """Energies a GPU keeps resident under each HBM storage form of the realistic device
    (n_b = 32, b = 416, eta = 1e-3, the grid linspace(-2, 2, n_e)), the memory lever of
    Section V-A (Table IV):
      dense_sigma_c128   Sigma^R_ii, Sigma^<_ii as b x b blocks, every output complex128;
      diag_sigma_c128    the diagonal self-energy blocks as b-vectors (QTX_SIGMA_DIAG);
      diag_sigma_fpx32   and the off-diagonal outputs G^R_{i,i+1}, G^R_{i+1,i}, G^<_{i,i+1}
                         as FPX32 (out_bits = 32; the diagonal outputs carry recurrence
                         state and stay complex128).
    With the library workspace fixed (--workspace-gb, default 24 GiB, reserved first), each
    form gets the largest energy count whose inputs and outputs fit the free HBM (less
    2 GiB); that many energies are then allocated, built on the device and solved (one
    warm-up solve, one timed), which shows that they fit.  The FPX error: the decoded
    off-diagonal blocks of 32 energies against the complex128 outputs of the same scheme,
    for X = 32, 40, 48, next to the scheme's own error against FP64 solves."""
    import numpy as np
    import torch
    from paper_2606_25595_amd import inputs, qtx
    cfg = inputs.CONFIGS["realistic"]
    n_b, b = cfg["n_b"], cfg["b"]
    skw = parse_scheme(args.mem_prec)
    ws = int((args.workspace_gb or 24.0) * (1 << 30))
    ctx = qtx.Context(0, workspace_bytes=ws)
    ctx.reserve_workspace(ws)
    tuned = autotune(ctx, skw, [(b, 256)])
    blk = b * b * 16
    forms = {"dense_sigma_c128": dict(sigma_diag=False, out_bits=64),
             "diag_sigma_c128": dict(sigma_diag=True, out_bits=64),
             "diag_sigma_fpx32": dict(sigma_diag=True, out_bits=32)}

    def per_energy(f):
        s_in = 2 * n_b * (b * 16 if f["sigma_diag"] else blk)
        off = 3 * (n_b - 1) * (blk if f["out_bits"] == 64 else b * b * f["out_bits"] // 4)
        return s_in + 2 * n_b * blk + off + 4

    H_d, H_u, H_l = (torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in inputs.random_hamiltonian(n_b, b, 0))

    def build(n_e, f, grid=None):
        grid = np.linspace(-2.0, 2.0, n_e) if grid is None else grid
        sr, sl = inputs.random_bt_scalars(n_b, grid, eta=1e-3)
        if f["sigma_diag"]:
            def vec(x):
                return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")[:, :, None].expand(n_e, n_b, b).contiguous()
            SR, SL = vec(sr), vec(sl)
        else:
            SR, SL = inputs.diag_blocks_device(sr, b), inputs.diag_blocks_device(sl, b)
        kw = dict(dtype=torch.complex128, device="cuda")

        def offd():
            if f["out_bits"] == 64:
                return torch.empty((n_e, n_b - 1, b, b), **kw)
            return torch.empty((n_e, n_b - 1, b * b * f["out_bits"] // 4), dtype=torch.uint8, device="cuda")
        return qtx.DeviceProblem(energies=grid, H_d=H_d, H_u=H_u, H_l=H_l, SR_d=SR, SL_d=SL,
                                 GR_d=torch.empty((n_e, n_b, b, b), **kw), GR_u=offd(), GR_l=offd(),
                                 GL_d=torch.empty((n_e, n_b, b, b), **kw), GL_u=offd(),
                                 status=torch.full((n_e,), -1, dtype=torch.int32, device="cuda"),
                                 sigma_diag=f["sigma_diag"], out_bits=f["out_bits"])

    rows = {}
    for name, f in forms.items():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free, total = torch.cuda.mem_get_info()
        n_e = int((free - (2 << 30)) // per_energy(f))
        log("bench memory: %s: %.1f MB per energy, %.1f GiB free -> %d energies"
            % (name, per_energy(f) / 1e6, free / 2 ** 30, n_e))
        dp = build(n_e, f)
        ctx.solve(dp, **skw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.solve(dp, **skw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = bool((dp.status == 0).all().item())
        rows[name] = {"bytes_per_energy": per_energy(f), "energies_resident": n_e, "solve_s": dt,
                      "energies_per_s": n_e / dt, "status_ok": ok, "hbm_free_gib": free / 2 ** 30}
        log("bench memory: %s: %d energies solved in %.2f s (%.1f energies/s), status ok %s"
            % (name, n_e, dt, n_e / dt, ok))
        del dp
    # FPX error on 32 energies: decoded blocks against the complex128 outputs of the same
    # scheme, and that scheme against FP64
    grid = np.linspace(-2.0, 2.0, 256)[::8]
    ref64 = build(32, forms["diag_sigma_c128"], grid)
    ctx.solve(ref64, prec="fp64")
    mixed = build(32, forms["diag_sigma_c128"], grid)
    ctx.solve(mixed, **skw)

    def rel(X, R):
        d = (X - R).abs().pow(2).sum((-1, -2)).sqrt()
        return float((d / R.abs().pow(2).sum((-1, -2)).sqrt().clamp_min(1e-300)).max().item())
    err = {"scheme_vs_fp64": {k: rel(getattr(mixed, k), getattr(ref64, k)) for k in ("GR_u", "GR_l", "GL_u")}}
    for bits in (32, 40, 48):
        fx = build(32, dict(sigma_diag=True, out_bits=bits), grid)
        ctx.solve(fx, **skw)
        e_fmt, e_tot = {}, {}
        for k in ("GR_u", "GR_l", "GL_u"):
            raw = getattr(fx, k)
            dec = ctx.fpx_decode(raw.reshape(-1), bits, raw.numel() * 8 // bits)
            dec = torch.view_as_complex(dec.view(-1, 2)).view(32, n_b - 1, b, b)
            e_fmt[k] = rel(dec, getattr(mixed, k))
            e_tot[k] = rel(dec, getattr(ref64, k))
        err["fpx%d" % bits] = {"decoded_vs_scheme_c128": e_fmt, "decoded_vs_fp64": e_tot}
        log("bench memory: FPX%d decoded vs %s complex128 %s, vs fp64 %s" % (bits, args.mem_prec, e_fmt, e_tot))
        del fx
    ctx.close()
    base = rows["dense_sigma_c128"]["energies_resident"]
    best = rows["diag_sigma_fpx32"]
    line = {"metric": "energies resident per GPU (inputs + selected outputs in HBM), realistic device",
            "value": best["energies_resident"], "unit": "energies", "n_gpus": 1, "higher_is_better": True,
            "data": "synthetic", "dtype": "f64+" + args.mem_prec.replace(":", "x"),
            "config": {"workload": "memory: realistic device n_b=32, b=416, eta=1e-3, library workspace %.0f GiB"
                                   % (ws / 2 ** 30), "precision": args.mem_prec},
            "gain_vs_dense_c128": best["energies_resident"] / base,
            "forms": rows, "fpx_error": err, "autotune": tuned}
    print(json.dumps(line), flush=True)


def bench_latency(args):
    """Latency of solves with few energies on the realistic device (n_b = 32,
    b = 416, eta = 1e-3, seed 0): one chain per energy against the two-sided split
    (QTX_SPLIT_CHAIN), FP64 and INT8 10/10, n_e in {1, 2, 4, 8, 16, 32} energies
    spread over [-2, 2], eager and hipGraph replay.  Each configuration: 2 warmup
    solves, then `reps` solves timed one by one (host clock, synchronised);
    p50 and max.  The split and unsplit outputs are compared (max relative
    Frobenius difference over the diagonal blocks of G^R and G^<)."""
    import numpy as np
    import torch
    from paper_2606_25595_amd import inputs, qtx
    n_b, b = 32, 416
    grid = np.linspace(-2.0, 2.0, 256)
    ctx = qtx.Context(0)
    stream = torch.cuda.Stream()
    rows = []
    precs = args.latency_precs.split(",")
    kw = dict(dtype=torch.complex128, device="cuda")
    for n_e in [int(x) for x in args.latency_ne.split(",")]:
        E = grid[np.linspace(0, 255, n_e + 2).astype(int)[1:-1]]
        d = inputs.device_random_problem(n_b, b, E, seed=0, eta=1e-3)
        outs = {}
        for split in [bool(int(x)) for x in args.latency_split.split(",")]:
            dp = qtx.DeviceProblem(energies=d["energies"], H_d=d["H_d"], H_u=d["H_u"], H_l=d["H_l"],
                                   SR_d=d["SR_d"], SL_d=d["SL_d"], GR_d=torch.empty((n_e, n_b, b, b), **kw),
                                   GR_u=torch.empty((n_e, n_b - 1, b, b), **kw),
                                   GR_l=torch.empty((n_e, n_b - 1, b, b), **kw),
                                   GL_d=torch.empty((n_e, n_b, b, b), **kw),
                                   GL_u=torch.empty((n_e, n_b - 1, b, b), **kw),
                                   status=torch.full((n_e,), -1, dtype=torch.int32, device="cuda"), split=split)
            for prec in precs:
                skw = parse_scheme(prec)
                for graph in (False, True):
                    if graph and n_e > 8:
                        continue
                    ctx.set_graph(graph)
                    reps = 12 if n_e <= 4 else 6
                    ts = []
                    with torch.cuda.stream(stream):
                        for k in range(2 + reps):
                            torch.cuda.synchronize()
                            t0 = time.perf_counter()
                            ctx.solve(dp, stream=stream, **skw)
                            stream.synchronize()
                            if k >= 2:
                                ts.append(time.perf_counter() - t0)
                    ctx.set_graph(False)
                    ts = np.array(ts) * 1e3
                    ok = bool((dp.status == 0).all().item())
                    row = {"n_e": n_e, "split": split, "prec": prec, "graph": graph, "p50_ms": float(np.median(ts)),
                           "max_ms": float(ts.max()), "energies_per_s": n_e / float(np.median(ts)) * 1e3,
                           "status_ok": ok}
                    if not graph:
                        outs[(split, prec)] = (dp.GR_d.clone(), dp.GL_d.clone())
                    rows.append(row)
                    log("bench latency: n_e=%d %s %s %s p50 %.1f ms max %.1f ms (%.1f energies/s)%s"
                        % (n_e, "split" if split else "chain", prec, "graph" if graph else "eager",
                           row["p50_ms"], row["max_ms"], row["energies_per_s"], "" if ok else " STATUS FAIL"))
            del dp
        for prec in precs:
            if (False, prec) not in outs or (True, prec) not in outs:
                continue
            a, s_ = outs[(False, prec)], outs[(True, prec)]
            diff = 0.0
            for x, y in zip(a, s_):
                dn = (x - y).abs().pow(2).sum((-1, -2)).sqrt()
                nr = x.abs().pow(2).sum((-1, -2)).sqrt().clamp_min(1e-300)
                diff = max(diff, float((dn / nr).max().item()))
            for r in rows:
                if r["n_e"] == n_e and r["prec"] == prec:
                    r["split_vs_chain_max_rel"] = diff
            log("bench latency: n_e=%d %s split vs chain max rel diff %.2e" % (n_e, prec, diff))
        del d, outs
        torch.cuda.empty_cache()
    ctx.close()
    best = {}
    for r in rows:
        key = (r["n_e"], r["split"], r["prec"])
        if key not in best or r["p50_ms"] < best[key]["p50_ms"]:
            best[key] = r
    n0 = min(r["n_e"] for r in rows)
    head = best.get((n0, True, precs[0])) or best.get((n0, False, precs[0]))
    line = {"metric": "selected-solve latency (p50) at %d energies, %s" % (n0, precs[0]), "value": head["p50_ms"],
            "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "latency: realistic device n_b=32, b=416, eta=1e-3, %s energies"
                                   % args.latency_ne, "split_chain": head["split"]},
            "speedup_split": {"%d:%s" % (n, pr): best[(n, False, pr)]["p50_ms"] / best[(n, True, pr)]["p50_ms"]
                              for (n, sp, pr) in best if sp and (n, False, pr) in best},
            "rows": rows}
    print(json.dumps(line), flush=True)


def bench_longchain(args):
    """Latency of solves with few energies on a long device (random BT device of
    --long-nb blocks, b = 416, eta = 1e-3, seed 0, energies spread over [-2, 2]): one
    chain per energy, the two-sided split (QTX_SPLIT_CHAIN), and P-way partitions;
    FP64 and INT8 10/10; each configuration captured once into a hipGraph and replayed
    (2 warm-up, then `reps` timed one by one, host clock, synchronised): p50 and max.
    Each mode's outputs against the one-chain solve of the same scheme: max relative
    Frobenius difference per block of G^R_ii, and per block of G^<_ii over the energy's
    largest G^<_ii block."""
    import numpy as np
    import torch
    from paper_2606_25595_amd import inputs, qtx
    n_b, b = args.long_nb, 416
    grid = np.linspace(-2.0, 2.0, 256)
    ctx = qtx.Context(0)
    stream = torch.cuda.Stream()
    modes = args.long_modes.split(",")
    precs = args.latency_precs.split(",")
    kw = dict(dtype=torch.complex128, device="cuda")
    rows = []
    for n_e in [int(x) for x in args.long_ne.split(",")]:
        E = grid[np.linspace(0, 255, n_e + 2).astype(int)[1:-1]]
        d = inputs.device_random_problem(n_b, b, E, seed=0, eta=1e-3)
        dp = qtx.DeviceProblem(energies=d["energies"], H_d=d["H_d"], H_u=d["H_u"], H_l=d["H_l"],
                               SR_d=d["SR_d"], SL_d=d["SL_d"], GR_d=torch.empty((n_e, n_b, b, b), **kw),
                               GR_u=torch.empty((n_e, n_b - 1, b, b), **kw),
                               GR_l=torch.empty((n_e, n_b - 1, b, b), **kw),
                               GL_d=torch.empty((n_e, n_b, b, b), **kw),
                               GL_u=torch.empty((n_e, n_b - 1, b, b), **kw),
                               status=torch.full((n_e,), -1, dtype=torch.int32, device="cuda"))
        for prec in precs:
            skw = parse_scheme(prec)
            ref = None
            for mode in modes:
                dp.split = mode == "split"
                dp.partitions = int(mode[1:]) if mode.startswith("p") else 0
                ctx.set_graph(True)
                reps = 8
                ts = []
                with torch.cuda.stream(stream):
                    for k in range(2 + reps):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        ctx.solve(dp, stream=stream, **skw)
                        stream.synchronize()
                        if k >= 2:
                            ts.append(time.perf_counter() - t0)
                ctx.set_graph(False)
                ts = np.array(ts) * 1e3
                ok = bool((dp.status == 0).all().item())
                row = {"n_e": n_e, "mode": mode, "prec": prec, "p50_ms": float(np.median(ts)),
                       "max_ms": float(ts.max()), "status_ok": ok}
                if ref is None:
                    ref = (dp.GR_d.clone(), dp.GL_d.clone())
                else:
                    dn = (dp.GR_d - ref[0]).abs().pow(2).sum((-1, -2)).sqrt()
                    nr = ref[0].abs().pow(2).sum((-1, -2)).sqrt().clamp_min(1e-300)
                    row["GR_d_vs_chain"] = float((dn / nr).max().item())
                    dn = (dp.GL_d - ref[1]).abs().pow(2).sum((-1, -2)).sqrt()
                    nr = ref[1].abs().pow(2).sum((-1, -2)).sqrt().amax(dim=1, keepdim=True).clamp_min(1e-300)
                    row["GL_d_vs_chain"] = float((dn / nr).max().item())
                rows.append(row)
                log("bench longchain: n_b=%d n_e=%d %s %s p50 %.1f ms max %.1f ms%s%s"
                    % (n_b, n_e, prec, mode, row["p50_ms"], row["max_ms"],
                       (" vs chain G^R %.1e G^< %.1e" % (row["GR_d_vs_chain"], row["GL_d_vs_chain"]))
                       if "GR_d_vs_chain" in row else "", "" if ok else " STATUS FAIL"))
        del d, dp, ref
        torch.cuda.empty_cache()
    ctx.close()
    n0 = min(r["n_e"] for r in rows)
    chain = {(r["n_e"], r["prec"]): r["p50_ms"] for r in rows if r["mode"] == "chain"}
    best = min((r for r in rows if r["n_e"] == n0 and r["prec"] == precs[0]), key=lambda r: r["p50_ms"])
    line = {"metric": "selected-solve latency (p50) at %d energies on a %d-block device, %s" % (n0, n_b, precs[0]),
            "value": best["p50_ms"], "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "longchain: random BT device n_b=%d, b=416, eta=1e-3, %s energies"
                                   % (n_b, args.long_ne), "mode": best["mode"]},
            "speedup_vs_chain": {"%d:%s:%s" % (r["n_e"], r["prec"], r["mode"]): chain[(r["n_e"], r["prec"])] / r["p50_ms"]
                                 for r in rows if (r["n_e"], r["prec"]) in chain},
            "rows": rows}
    print(json.dumps(line), flush=True)


def bench_products(args):
    """The INT8 product kernel alone (416^3 complex products over 256 entries, 10 moduli,
    the library's per-launch HIP-event timer): every tile variant with operands per entry
    and with the left, the right or both operands shared by the whole batch (batch
    stride 0: every tile then reads the same residues, which stay in L2).  The shared
    cases separate the cost of L2 misses from the rest of the strip pipeline."""
    import torch
    from paper_2606_25595_amd import qtx
    b, batch, p = 416, 256, 10
    ctx = qtx.Context(0)
    g = torch.Generator(device="cuda").manual_seed(0)
    A = torch.randn(batch, b, b, dtype=torch.complex128, device="cuda", generator=g)
    B = torch.randn(batch, b, b, dtype=torch.complex128, device="cuda", generator=g)
    A1, B1 = A[:1].clone(), B[:1].clone()
    C = torch.empty_like(A)
    rows = []
    for v in range(64):
        try:
            ctx.set_int8_tile_variant(v)
        except qtx.QtxError:
            break                      # past the last variant
        for name, a, bb in (("per_entry", A, B), ("shared_A", A1, B), ("shared_B", A, B1), ("shared_AB", A1, B1)):
            ctx.zgemm(a, bb, C, prec="int8", n_slices=p)
            torch.cuda.synchronize()
            ctx.profile(True)
            ctx.profile_read(qtx.QTX_KERNEL_GEMM)
            for _ in range(max(3, args.steps)):
                ctx.zgemm(a, bb, C, prec="int8", n_slices=p)
            torch.cuda.synchronize()
            ctx.profile(False)
            ms, n, ops = ctx.profile_read(qtx.QTX_KERNEL_GEMM)
            rows.append({"variant": v, "operands": name, "ms": ms / n, "tops": ops / n / (ms / n * 1e-3) / 1e12})
            log("bench products: variant %2d %-9s %.4f ms (%.0f TOP/s)" % (v, name, ms / n, rows[-1]["tops"]))
    ctx.set_int8_tile_variant(-1)
    ctx.close()
    best = min((r for r in rows if r["operands"] == "per_entry"), key=lambda r: r["ms"])
    line = {"metric": "INT8 product kernel, 416^3 x 256 complex, 10 moduli", "value": best["ms"], "unit": "ms",
            "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "int8x10",
            "config": {"workload": "products: 256 products of 416^3, operands per entry or shared"},
            "best_variant": best["variant"], "rows": rows}
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """Batching workload: independent problems with b in {128, 256, 384, 512} and
    n_b in {16, 24, 32}, one energy each (E uniform in [-2, 2]), random devices
    generated on the GPU from per-problem seeds, all solved by one qtx_rgf_solve
    captured into a hipGraph and replayed."""
    import numpy as np
    import torch
    import oracle
    from paper_2606_25595_amd import inputs, qtx
    from paper_2606_25595_amd.serve import GpuExecutor, Request
    rng = np.random.default_rng(0)
    n = args.problems
    spec = [(int(rng.choice([128, 256, 384, 512])), int(rng.choice([16, 24, 32])), float(rng.uniform(-2, 2)))
            for _ in range(n)]
    need = sum((8 * nb - 5) * b * b * 16 for b, nb, _ in spec)
    log("bench batch: %d problems, %.1f GB of inputs and outputs" % (n, need / 1e9))
    ex = GpuExecutor(n_slots=1)              # only its device generator is used here
    kw = dict(dtype=torch.complex128, device="cuda")
    dps, reqs = [], []
    for q, (b, nb, E) in enumerate(spec):
        r = Request(rid=q, b=b, n_b=nb, n_e=1, seed=5000 + q)
        ex.start_request(r)
        H_d, H_u, H_l = ex.H.pop(q)
        sr, sl = inputs.random_bt_scalars(nb, [E])
        dps.append(qtx.DeviceProblem(
            energies=np.array([E]), H_d=H_d, H_u=H_u, H_l=H_l, SR_d=inputs.diag_blocks_device(sr, b),
            SL_d=inputs.diag_blocks_device(sl, b), GR_d=torch.empty((1, nb, b, b), **kw),
            GR_u=torch.empty((1, nb - 1, b, b), **kw), GR_l=torch.empty((1, nb - 1, b, b), **kw),
            GL_d=torch.empty((1, nb, b, b), **kw), GL_u=torch.empty((1, nb - 1, b, b), **kw),
            status=torch.full((1,), -1, dtype=torch.int32, device="cuda")))
    ex.close()
    torch.cuda.synchronize()
    skw = parse_scheme(args.prec)
    ctx = qtx.Context(0)
    counts = {}
    for b, _, _ in spec:
        counts[b] = counts.get(b, 0) + 1
    tuned = autotune(ctx, skw, sorted(counts.items()))
    ctx.set_graph(True)
    stream = torch.cuda.Stream()
    flops = sum((144 * (nb - 1) + 24) * b ** 3 for b, nb, _ in spec)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        ctx.solve(dps, stream=stream, **skw)     # capture + first run
        stream.synchronize()
        t_first = time.perf_counter() - t0
        for _ in range(args.warmup):
            ctx.solve(dps, stream=stream, **skw)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.solve(dps, stream=stream, **skw)
        stream.synchronize()
        t = (time.perf_counter() - t0) / args.steps
    ok = all(int(dp.status.item()) == 0 for dp in dps)
    sample = list(range(0, n, max(1, n // 16)))[:16]
    errs = {k: 0.0 for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")}
    for q in sample:
        dp = dps[q]
        b, nb, E = spec[q]
        sr, sl = inputs.random_bt_scalars(nb, [E])
        p = inputs.BTProblem(energies=np.array([E]), H_d=dp.H_d.cpu().numpy(), H_u=dp.H_u.cpu().numpy(),
                             H_l=dp.H_l.cpu().numpy(), SR_d=inputs._diag_blocks(sr, b), SL_d=inputs._diag_blocks(sl, b))
        ref = oracle.rgf_selected(p)
        out = dp.outputs()
        for k in errs:
            errs[k] = max(errs[k], float(oracle.rel_fro_err(out[k], ref[k]).max()))
    line = {"metric": "batched RGF energy points/sec (uneven problems, one hipGraph launch)",
            "value": n / t, "unit": "energy points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": t * 1e3, "higher_is_better": True, "dtype": "f64" if args.prec == "fp64" else "f64+" + args.prec,
            "data": "synthetic",
            "config": {"workload": "batch: %d problems, b in {128,256,384,512}, n_b in {16,24,32}, 1 energy each" % n,
                       "precision": args.prec},
            "fp64eq_tflops": flops / t / 1e12, "first_call_ms": t_first * 1e3, "status_ok": ok,
            "graph_captures": ctx.stat(qtx.QTX_STAT_GRAPH_CAPTURES),
            "graph_launches": ctx.stat(qtx.QTX_STAT_GRAPH_LAUNCHES),
            "sampled_max_rel_err": errs, "sampled_problems": len(sample), "autotune": tuned}
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_tiny(args):
    """The tiny workload (n_b = 8, b = 16, all 32 energies of [-2, 2]): GPU solve latency
    of all 32 energies (eager and replayed as a hipGraph; the launch-bound case), the
    error of every output block against the dense FP64 oracle, and both CPU oracles
    (dense inverse and block recurrences) timed on all 32 energies."""
    import numpy as np
    import torch
    import oracle
    from paper_2606_25595_amd import inputs, qtx
    p = inputs.config_problem("tiny")
    t0 = time.perf_counter()
    dense = oracle.dense_selected(p)
    t_dense = time.perf_counter() - t0
    t0 = time.perf_counter()
    rgf = oracle.rgf_selected(p)
    t_rgf = time.perf_counter() - t0
    ctx = qtx.Context(0)
    dp = qtx.to_device(p)
    stream = torch.cuda.Stream()
    res = {}
    for graph in (False, True):
        ctx.set_graph(graph)
        with torch.cuda.stream(stream):
            for _ in range(max(1, args.warmup)):
                ctx.solve(dp, stream=stream)
            stream.synchronize()
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
            evs[0].record(stream)
            for k in range(args.steps):
                ctx.solve(dp, stream=stream)
                evs[k + 1].record(stream)
            stream.synchronize()
        lat = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
        res["graph" if graph else "eager"] = {"p50_ms": float(np.percentile(lat, 50)),
                                              "p99_ms": float(np.percentile(lat, 99)),
                                              "energies_per_s": p.n_e / (float(np.median(lat)) / 1e3)}
    ctx.set_graph(False)
    out = dp.outputs()
    errs = {k: float(oracle.rel_fro_err(out[k], dense[k]).max()) for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")}
    errs_rgf = {k: float(oracle.rel_fro_err(rgf[k], dense[k]).max()) for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")}
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info() if t.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    best = res["graph"] if res["graph"]["p50_ms"] < res["eager"]["p50_ms"] else res["eager"]
    line = {"metric": "RGF energy points/sec, tiny workload (launch-bound)", "value": best["energies_per_s"],
            "unit": "energy points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": best["p50_ms"], "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "tiny: n_b=8 blocks, b=16, N_E=32 energies in [-2,2], complex128, S=I, seed 0"},
            "gpu": res, "max_rel_err_vs_dense_oracle": errs, "status_ok": bool(np.all(out["status"] == 0)),
            "cpu_oracles": {"dense_s": t_dense, "rgf_s": t_rgf, "dense_energies_per_s": p.n_e / t_dense,
                            "rgf_energies_per_s": p.n_e / t_rgf, "blas_threads": int(threads),
                            "rgf_vs_dense_max_rel_err": errs_rgf,
                            "note": "all 32 energies, one at a time, numpy/LAPACK FP64"},
            "flops_per_energy": (144 * (p.n_b - 1) + 24) * p.b ** 3}
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_serve(args):
    """Serving workload: Poisson arrivals (b in 128..512 step 32, n_b in 8..48,
    N_E in 16..128, FP64 or mixed with probability 1/2, seed 1000 + id), continuous
    batching by HBM footprint, p50/p99 latency of completed requests."""
    import torch
    from paper_2606_25595_amd.serve import PRECISIONS, GpuExecutor, Server, request_stream
    free, total = torch.cuda.mem_get_info()
    budget = int(free * 0.55)
    reqs = request_stream(rate=args.rate, duration=args.duration, seed=0)
    log("bench serve: %d requests over %.1f s at %.1f/s, budget %.1f GB" % (len(reqs), args.duration, args.rate,
                                                                           budget / 1e9))
    compact = dict(sigma_diag=True, out_bits=args.serve_compact) if args.serve_compact else {}
    ex = GpuExecutor(n_slots=args.serve_slots, workspace_per_slot=int(free * 0.24 / args.serve_slots), split=args.split,
                     **compact)
    n_done = [0]

    def done(r):
        n_done[0] += 1
        if n_done[0] % 20 == 0:
            log("bench serve: %d requests completed (latest: id %d, %d energies, %.2f s)"
                % (n_done[0], r.rid, r.n_e, r.latency))

    srv = Server(ex, hbm_budget=budget, chunk_energies=args.serve_chunk, max_pending=512, on_done=done,
                 policy=args.serve_policy)
    rep = srv.run(reqs, time_limit=args.time_limit)
    ex.close()
    line = {"metric": "served RGF energy points/sec with p50/p99 request latency",
            "value": rep["energy_points_per_s"], "unit": "energy points/s", "n_gpus": 1,
            "higher_is_better": True, "data": "synthetic",
            "dtype": " / ".join("f64" if x["prec"] == "fp64" else
                                "f64+%s:%d/%s:%d" % (x["prec"], x.get("n_slices", 0), x.get("prec_lesser", x["prec"]),
                                                     x.get("n_slices_lesser", x.get("n_slices", 0)))
                                for x in PRECISIONS.values()),
            "config": {"workload": "serve: Poisson %.1f/s for %.1f s, b 128..512, n_b 8..48, N_E 16..128"
                                   % (args.rate, args.duration), "split_chain": bool(args.split),
                       "compact_out_bits": int(args.serve_compact) or None, "slots": args.serve_slots,
                       "policy": args.serve_policy,
                       "chunk_energies": args.serve_chunk},
            "p50_latency_s": rep["p50_latency_s"], "p99_latency_s": rep["p99_latency_s"], "report": rep}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
