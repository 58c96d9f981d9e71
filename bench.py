"""Throughput of the per-sample PEPS evaluation (psi, dpsi, E_loc) on one MI355X.

One step = one pepsgo_evaluate over the whole batch of the 10x10 D=6 Dc=12
workload (16384 configurations from 1024 W^2 Metropolis chains of 16
nearest-neighbour-exchange steps, random N(0,1)/sqrt(D) tensors, J1 = 1,
J2 = 0.5; psi, every Delta_ij and E_loc), inputs resident in HBM before timing
starts.  Default precision: float32 two-row strips on the matrix cores with
float64 truncation, sandwiches, log-scales and float64 re-evaluation of any
strip that fails its accuracy check.  A short serving leg (Poisson arrivals
through the library's request loop) adds p50/p99 latency, and the float64
CPU reference is timed on a bounded sample.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def progress(msg: str) -> None:
    """A progress line on stderr (the result is the one JSON line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


METRIC = "samples/s (ψ+∂ψ+E_loc) at 10x10 D=6 Dc=12; serving p50/p99 latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name: str, Dc: int, J2: float, seconds: float = 20.0):
    """The oracle, untuned, on the host cores over a bounded sample of the workload,
    and on one core (one worker process with one BLAS thread)."""
    import multiprocessing as mp

    from paper_1611_09467_amd import workloads as wl

    cores = min(16, os.cpu_count() or 1)
    T, S = wl.workload_inputs(name)
    # per-sample cost of the oracle: calibrate on one sample, then size the sample
    t0 = time.perf_counter()
    _oracle_one((T, S[0], Dc, J2))
    per = time.perf_counter() - t0
    n = int(max(cores, min(len(S), round(seconds / max(per, 1e-3)))))
    idx = [int(k) for k in (len(S) * (i + 0.5) / n for i in range(n))]
    ctxm = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctxm.Pool(cores, initializer=_one_thread) as pool:
        pool.map(_oracle_one, [(T, S[k], Dc, J2) for k in idx], chunksize=1)
    wall = time.perf_counter() - t0
    n1 = 4
    with ctxm.Pool(1, initializer=_one_thread) as pool:
        pool.map(_oracle_one, [(T, S[idx[0]], Dc, J2)])  # imports and warm-up
        t0 = time.perf_counter()
        pool.map(_oracle_one, [(T, S[k], Dc, J2) for k in idx[1:n1 + 1]], chunksize=n1)
        wall1 = time.perf_counter() - t0
    return {"value": n / wall, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "single_core_value": n1 / wall1,
            "sample": f"{n} samples spread over the {len(S)}-sample batch (psi, Delta, E_loc; "
                      f"float64 numpy/LAPACK, one process per core, one BLAS thread each); "
                      f"single core: {n1} of them in one process"}


SERVE_L = (6, 8, 10, 12, 16)
SERVE_D = (4, 6, 8, 10)


def serving_leg(ctx, seconds: float, load: float, seed: int = 7, max_D: int = 10,
                precision: str = "fp64"):
    """Poisson arrivals of evaluation requests through the library's request loop.

    The mix: L uniform in SERVE_L, D uniform in SERVE_D (up to max_D), Dc = 2D,
    L x L lattices, batch ~ Geometric(1/256), uniform S^z = 0 configurations
    seeded by the request id, J1 = 1, J2 = 0.5, psi + Delta + E_loc (strips in
    ``precision``; everything else float64).
    Tensors are N(0,1)/sqrt(D), one resident PEPS per (L, D) class.  Capacity
    is measured first (each class alone at batch 256), and arrivals are offered
    at `load` times it for `seconds`.  Latency = completion observed by the
    server's thread minus submission.
    """
    import numpy as np
    import torch

    from paper_1611_09467_amd import binding as bd
    from paper_1611_09467_amd import workloads as wl

    classes = [(L, D) for L in SERVE_L for D in SERVE_D if D <= max_D]
    peps = {}
    for k, (L, D) in enumerate(classes):
        peps[(L, D)] = bd.Peps(ctx, L, L, D, wl.pack_peps(wl.make_peps(L, L, D, seed=100 + k)))
    # capacity: per-sample device time of each class alone at the mean batch
    per_sample = {}
    prec = bd.PRECISIONS[precision]
    for (L, D), P in peps.items():
        S = torch.from_numpy(wl.random_sz0_configs(L, L, 256, 5)).cuda()
        P.evaluate(S[:8], 2 * D, 1.0, 0.5, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.evaluate(S, 2 * D, 1.0, 0.5, precision=prec)
        torch.cuda.synchronize()
        per_sample[(L, D)] = (time.perf_counter() - t0) / 256
        P._ws = None
        progress(f"serving: capacity of {L}x{L} D={D}: {1e3 * per_sample[(L, D)]:.3f} ms/sample")
    progress(f"serving: capacity of {len(per_sample)} classes measured")
    mean_req = 256 * float(np.mean(list(per_sample.values())))
    rate = load / mean_req  # requests per second
    rng = np.random.Generator(np.random.PCG64(seed))
    srv = bd.Server(ctx, pool_bytes=64 << 30, streams=8, max_chunk=512, min_chunk=32)
    n_req = max(8, int(rate * seconds))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    picks = rng.integers(0, len(classes), size=n_req)
    batches = rng.geometric(1.0 / 256, size=n_req)
    inputs = []
    for q in range(n_req):
        L, D = classes[picks[q]]
        S = wl.random_sz0_configs(L, L, int(batches[q]), 10_000 + q)
        inputs.append(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    lat, done_cls, samples = {}, {}, 0
    ids = {}
    t_start = time.perf_counter()
    t_note = t_start
    q = 0
    while len(lat) < n_req:
        if time.perf_counter() - t_note > 20.0:
            t_note = time.perf_counter()
            progress(f"serving: {len(lat)} of {n_req} requests done, {q} submitted")
        now = time.perf_counter() - t_start
        while q < n_req and arrivals[q] <= now:
            L, D = classes[picks[q]]
            ids[srv.submit(peps[(L, D)], inputs[q], 2 * D, 1.0, 0.5, precision=prec)] = q
            q += 1
        wait = (arrivals[q] - (time.perf_counter() - t_start)) if q < n_req else 0.05
        for d, _ in srv.poll(timeout_s=max(0.0, min(wait, 0.05))):
            r = ids.pop(d.id)
            lat[r] = (d.t_done_ns - d.t_submit_ns) / 1e6
            done_cls[r] = classes[picks[r]]
            samples += d.batch
            if len(lat) % 100 == 0:
                progress(f"serving: {len(lat)} of {n_req} requests done")
    wall = time.perf_counter() - t_start
    stats = srv.stats()
    srv.close()
    for P in peps.values():
        P.free()
    v = np.array([lat[r] for r in range(n_req)])
    per_class = {}
    for (L, D) in classes:
        sel = [lat[r] for r in range(n_req) if done_cls[r] == (L, D)]
        if sel:
            per_class[f"{L}x{L}_D{D}_Dc{2 * D}"] = {"n": len(sel), "p50_ms": float(np.percentile(sel, 50)),
                                                    "p99_ms": float(np.percentile(sel, 99))}
    return {"requests": n_req, "offered_load": load, "arrival_rate_per_s": rate,
            "precision": precision, "server_stats": stats,
            "p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)),
            "samples_per_s": samples / wall, "wall_s": wall,
            "capacity_ms_per_sample": {f"{L}x{L}_D{D}": 1e3 * t for (L, D), t in per_sample.items()},
            "per_class": per_class,
            "mix": "L in {6,8,10,12,16} x D in {4,6,8,10} (<= max_D), Dc = 2D, batch ~ Geometric(1/256), "
                   f"Poisson arrivals, strips in {precision}, psi + Delta + E_loc"}


TRACE_NAMES = {"zip": "pg::k_zip<", "sandwich": "pg::k_sandwich<", "strip": "pg::k_strip<"}


def optimiser_leg(P, cfg, out, Dc: int, J2: float, prec: int, eval_ms: float) -> dict:
    """Device times of the kernels around the evaluation on the same batch: the
    Eq. (3) accumulation and Eq. (6) update, one Metropolis step (an evaluation
    plus the accept/move kernel), one sweep, one simple-update step of the same
    lattice, and the correlations on the bulk window (the transverse part on the
    first 1024 samples)."""
    import numpy as np
    import torch
    dev = cfg.device
    B = cfg.shape[0]

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r = fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b), r

    saved = P.read()
    P.go_accumulate(cfg, out)  # warm-up
    acc_ms, sums = timed(lambda: P.go_accumulate(cfg, out))
    p = torch.rand(P.nparams, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(1))
    upd_ms, _ = timed(lambda: P.go_update(sums, 0.001, p))
    P.update(saved)
    bonds = torch.from_numpy(np.random.default_rng(3).integers(
        0, P.N * (P.M - 1) + (P.N - 1) * P.M, B).astype(np.int32)).to(dev)
    u = torch.rand(B, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(2))
    chain = cfg.clone()
    met_ms, _ = timed(lambda: P.metropolis_step(chain, bonds, u, Dc, 1.0, J2, precision=prec,
                                                want_grad=True))
    # one sweep over every bond of every chain (environments reused)
    us = torch.rand((B, P.nbonds), dtype=torch.float64, device=dev,
                    generator=torch.Generator(dev).manual_seed(4))
    chain2 = cfg.clone()
    sweep_ms, (sacc, _) = timed(lambda: P.metropolis_sweep(chain2, us, Dc))
    sweep_acc = float(sacc.double().mean().item())
    gam, lam = P.su_start()
    P.su_evolve(gam, lam, 1.0, 0.01, 1)  # warm-up
    su_ms, _ = timed(lambda: P.su_evolve(gam, lam, 1.0, 0.01, 1))
    P.update(saved)
    import math
    from paper_1611_09467_amd import binding as bd
    win = (1, 1, P.N - 2, P.M - 2)
    bd.sz_correlations(cfg, P.N, P.M, win, out["flags"])  # warm-up
    corr_ms, counts = timed(lambda: bd.sz_correlations(cfg, P.N, P.M, win, out["flags"]))
    sf_ms, m2 = timed(lambda: bd.structure_factor(counts, math.pi, math.pi))
    # transverse part of <S_p . S_q> over the same bulk window, on a share of the batch
    nt = min(B, 1024)
    sub = cfg[:nt].contiguous()
    P.transverse(sub[:8], win, Dc)  # warm-up
    tr_ms, (trans, tflags, _) = timed(lambda: P.transverse(sub, win, Dc))
    counts_t = bd.sz_correlations(sub, P.N, P.M, win, tflags)
    ms2 = bd.spin_structure_factor(counts_t, trans, math.pi, math.pi)
    torch.cuda.synchronize()
    grad_bytes = B * P.grad_elems * 8
    return {"batch": B,
            "evaluate_ms": eval_ms,
            "metropolis_step_ms": met_ms,
            "metropolis_sweep_ms": sweep_ms,
            "sweep_proposals_per_s": B * P.nbonds / (sweep_ms / 1e3),
            "sweep_accepted_fraction": sweep_acc,
            "go_accumulate_ms": acc_ms,
            "go_accumulate_GBps": grad_bytes / (acc_ms / 1e3) / 1e9,
            "go_update_ms": upd_ms,
            "su_step_ms": su_ms,
            "sz_counts_ms": corr_ms,
            "structure_factor_ms": sf_ms,
            "staggered_zz_structure_factor": float(m2.item()),
            "transverse_samples": nt,
            "transverse_window_sites": win[2] * win[3],
            "transverse_ms": tr_ms,
            "transverse_samples_per_s": nt / (tr_ms / 1e3),
            "transverse_pair_ratios_per_s": nt * (win[2] * win[3]) ** 2 / 4 / (tr_ms / 1e3),
            "staggered_structure_factor_ms2": float(ms2.item())}


def measured_traffic(workload: str, precision: str, cls: str):
    """HBM bytes per launch of a kernel class from the committed counter summary.

    None when no summary exists for this workload and precision, or when the
    kernel sources changed since the counters were taken.
    """
    import glob
    import hashlib
    f = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{precision}.json")
    if not os.path.exists(f):
        return None
    data = json.load(open(f))
    h = hashlib.sha256()
    for src in sorted(glob.glob(os.path.join(ROOT, "paper_1611_09467_amd", "csrc", "*"))):
        h.update(open(src, "rb").read())
    if h.hexdigest() != data.get("source_sha256"):
        return None
    tot = 0.0
    for name, v in data["bytes_per_launch"].items():
        if TRACE_NAMES[cls] in name:
            tot += v["fetch"] + v["write"]
    return tot or None


def timed_passes(P, cfg, Dc, J2, prec, passes=2, tune=False):
    """samples/s of whole evaluations of cfg (one warm-up, then `passes` timed)."""
    import torch
    if tune:
        P.autotune(cfg[: min(cfg.shape[0], 2048)], Dc, 1.0, J2, precision=prec)
    out = P.evaluate(cfg, Dc, 1.0, J2, precision=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(passes):
        out = P.evaluate(cfg, Dc, 1.0, J2, precision=prec, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / passes
    flags = out["flags"].cpu().numpy()
    return {"samples_per_s": cfg.shape[0] / dt, "ms_per_pass": dt * 1e3, "batch": int(cfg.shape[0]),
            "refined_in_fp64": int(((flags & 8) != 0).sum())}


PUBLISHED_PEAKS_TFLOPS = {"fp64_vector_fma": 78.6, "fp64_mfma_16x16x4": 78.6,
                          "fp32_mfma_16x16x4": 157.3, "bf16_mfma_16x16x16": 2500.0}
STRIP_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x6": 2500.0, "bf16": 2500.0}


def measured_peaks() -> dict:
    """On-device throughput of the units the roofline divides by: the library's probe
    kernels (independent FMA / MFMA chains, 2048 workgroups of 256 threads) and a plain
    4 GiB device copy, each timed with HIP events over three launches after a warm-up."""
    import torch
    from paper_1611_09467_amd import binding as bd
    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream(dev)
    blocks = 2048
    sink = torch.zeros(blocks, dtype=torch.float64, device=dev)
    iters = {"fp64_vector_fma": 100000, "fp64_mfma_16x16x4": 5000, "fp32_mfma_16x16x4": 10000,
             "bf16_mfma_16x16x16": 10000}
    out = {}
    for name, kind in bd.PROBES.items():
        bd.pepsgo_peak_probe(kind, blocks, 100, sink.data_ptr(), s.cuda_stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        flops = sum(bd.pepsgo_peak_probe(kind, blocks, iters[name], sink.data_ptr(), s.cuda_stream)
                    for _ in range(3))
        b.record(s)
        torch.cuda.synchronize()
        tf = flops / (a.elapsed_time(b) / 1e3) / 1e12
        out[name] = {"measured_tflops": tf, "published_tflops": PUBLISHED_PEAKS_TFLOPS[name],
                     "fraction_of_published": tf / PUBLISHED_PEAKS_TFLOPS[name]}
    src = torch.ones(1 << 30, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(3):
        dst.copy_(src)
    b.record(s)
    torch.cuda.synchronize()
    gbps = 3 * 2 * src.numel() * 4 / (a.elapsed_time(b) / 1e3) / 1e9
    out["hbm_copy"] = {"measured_GBps": gbps, "published_GBps": 8000.0,
                       "fraction_of_published": gbps / 8000.0}
    del src, dst
    torch.cuda.empty_cache()
    return out


def reduced_passes(P, cfg, Dc, J2, prec, passes=2):
    """samples/s of whole evaluations in the REDUCED gradient mode (the Eq. (3) sums
    formed inside the call, no per-sample Delta written), beside the per-sample mode."""
    import torch
    sums = P.new_sums()
    out = P.evaluate(cfg, Dc, 1.0, J2, precision=prec, sums=sums)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(passes):
        out = P.evaluate(cfg, Dc, 1.0, J2, precision=prec, sums=sums, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / passes
    return {"samples_per_s": cfg.shape[0] / dt, "ms_per_pass": dt * 1e3, "batch": int(cfg.shape[0]),
            "per_sample_delta_bytes_not_written": int(cfg.shape[0]) * P.grad_elems * 8}


def other_workloads(ctx) -> dict:
    """The other lattices of the benchmark set, timed the same way (autotuned):
    8x8 D=4 Dc=8 on its 4096 chain samples (float64 and float32 strips), and
    16x16 D=8 Dc=16 on 512 of its 8192 chain samples (the per-sample cost
    depends only on the shape; float64, float32 and split-bfloat16 strips,
    default tuning)."""
    import numpy as np
    import torch

    from paper_1611_09467_amd import binding as bd
    from paper_1611_09467_amd import workloads as wl
    res = {}
    for name, count, precs, tune in (("8x8_D4_Dc8", None, ("fp64", "fp32"), True),
                                     ("16x16_D8_Dc16", 512, ("fp64", "fp32", "bf16x6"), False)):
        w = wl.WORKLOADS[name]
        T, S = wl.workload_inputs(name)
        if count:
            S = S[:: len(S) // count][:count]
        P = bd.Peps(ctx, w["N"], w["M"], w["D"], wl.pack_peps(T))
        cfg = torch.from_numpy(np.ascontiguousarray(S)).cuda()
        res[name] = {}
        for p in precs:
            res[name][p] = timed_passes(P, cfg, w["Dc"], w["J2"], bd.PRECISIONS[p], tune=tune,
                                        passes=2 if tune else 1)
            progress(f"{name} {p}: {res[name][p]['samples_per_s']:.1f} samples/s")
        P.free()
        torch.cuda.empty_cache()
    return res


def _one_thread():
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass


def _oracle_one(args):
    from oracle import peps as op
    T, s, Dc, J2 = args
    return op.evaluate(T, s, Dc, 1.0, J2)["logabs"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="10x10_D6_Dc12")
    ap.add_argument("--batch", type=int, default=0, help="0: the workload's full batch")
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16x6", "bf16"],
                    help="strip contractions: float64, float32, split-bfloat16 or bfloat16 "
                         "matrix-core products (truncation and logs are float64 in all)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the LDS-budget autotuner (default budgets)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-optimiser", action="store_true",
                    help="skip timing the sampler / gradient-step / simple-update kernels")
    ap.add_argument("--serve-seconds", type=float, default=15.0,
                    help="seconds of Poisson arrivals through the request loop (0: no serving leg)")
    ap.add_argument("--serve-load", type=float, default=0.75)
    ap.add_argument("--serve-max-d", type=int, default=6,
                    help="largest D of the serving mix (the full mix goes to 10)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other precision modes and the other lattices")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving leg (with --serve-loads), e.g. for the full mix")
    ap.add_argument("--serve-precisions", default="fp64",
                    help="--serve-only: comma-separated strip precisions to serve in")
    ap.add_argument("--serve-loads", default="",
                    help="comma-separated offered loads for a serving sweep (default: --serve-load)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="run one plain device copy of this many bytes before timing "
                         "(a calibration dispatch for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1 (samples are "
                                   "independent: the batch shards by sample, each GPU holding a "
                                   "replica of the tensors)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1611_09467_amd import binding as bd
    from paper_1611_09467_amd import workloads as wl
    from paper_1611_09467_amd.workmodel import evaluation_flops

    if args.serve_only:
        ctx = bd.Context(0)
        loads = [float(x) for x in args.serve_loads.split(",")] if args.serve_loads else [args.serve_load]
        for pn in args.serve_precisions.split(","):
            for ld in loads:
                r = serving_leg(ctx, args.serve_seconds, ld, max_D=args.serve_max_d, precision=pn)
                print(json.dumps({"serving": r}), flush=True)
        return

    w = wl.WORKLOADS[args.workload]
    N, M, D, Dc, J2 = w["N"], w["M"], w["D"], w["Dc"], w["J2"]
    T, S = wl.workload_inputs(args.workload, count=args.batch or None)
    B = S.shape[0]
    ctx = bd.Context(0)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(T))
    dev = torch.device("cuda:0")
    cfg = torch.from_numpy(np.ascontiguousarray(S)).to(dev)
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prec = bd.PRECISIONS[args.precision]
    prm = bd.make_params(Dc, 1.0, J2, precision=prec)
    tuning = None
    if not args.no_tune:
        # the tuner times each candidate on a slice of the same batch (untimed here)
        tuning = P.autotune(cfg[: min(B, 2048)], Dc, 1.0, J2, precision=prec)
        progress(f"tuned: {tuning}")
    ws = torch.empty(P.workspace_bytes(prm, B), dtype=torch.uint8, device=dev)
    out = None
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        out = P.evaluate(cfg, Dc, 1.0, J2, precision=prec, workspace=ws, out=out)
    torch.cuda.synchronize()
    progress(f"{args.warmup} warm-up steps done; timing {args.steps} steps")
    bd.pepsgo_profile(ctx.handle, 1)
    bd.pepsgo_profile(ctx.handle, -1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = P.evaluate(cfg, Dc, 1.0, J2, precision=prec, workspace=ws, out=out,
                         stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress(f"timed steps done: {(t1 - t0) * 1e3 / args.steps:.1f} ms per step")
    bd.pepsgo_profile(ctx.handle, 0)
    kern = {}
    for k, name in enumerate(bd.KERNEL_CLASSES):
        ms, n = bd.pepsgo_profile_read(ctx.handle, k)
        kern[name] = {"total_ms": ms, "launches": n, "avg_ms": ms / n if n else 0.0}
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = B / (ms_step / 1e3)

    flops = evaluation_flops(N, M, D, Dc, S, J2=J2)
    per_class = {
        "zip": flops["zip"] + flops["zip_truncation"] + flops["zip_lq"],
        "sandwich": flops["sandwich"],
        "strip": flops["strip"],
    }
    dom = max(per_class, key=lambda k: kern[k]["total_ms"])
    launches_per_step = kern[dom]["launches"] / args.steps
    per_launch = per_class[dom] / launches_per_step
    achieved = per_launch / (kern[dom]["avg_ms"] / 1e3) / 1e12
    flags = out["flags"].cpu().numpy()
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64+f32", "bf16x6": "f64+bf16x6",
                  "bf16": "f64+bf16"}[args.precision],
        "data": "synthetic (seeded random tensors and exchange-chain configurations)",
        "config": {"workload": f"{N}x{M} OBC D={D} Dc={Dc}, {B} samples, J1=1 J2={J2}, "
                               f"psi + per-sample Delta + E_loc",
                   "batch": B},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(args.workload, args.precision, dom),
                     "flops_per_launch": per_launch,
                     "avg_launch_ms": kern[dom]["avg_ms"]},
        "kernels": kern,
        "tuning": tuning,
        "flops_per_sample": {k: v / B for k, v in flops.items()},
        "flagged": {"zero_psi": int(((flags & 1) != 0).sum()),
                    "nonfinite": int(((flags & 2) != 0).sum()),
                    "near_tie": int(((flags & 4) != 0).sum()),
                    "refined_in_fp64": int(((flags & 8) != 0).sum())},
    }
    # every kernel class against its own unit, and the path as a whole
    cls_peak = {"zip": FP64_VECTOR_PEAK_TFLOPS, "sandwich": FP64_VECTOR_PEAK_TFLOPS,
                "strip": STRIP_PEAK_TFLOPS[args.precision]}
    util = {}
    t_roof = 0.0
    for cls, peak in cls_peak.items():
        tf = per_class[cls] / (kern[cls]["total_ms"] / args.steps / 1e3) / 1e12
        util[cls] = {"achieved_tflops": tf, "peak_tflops": peak, "frac": tf / peak}
        t_roof += per_class[cls] / (peak * 1e12)
    rec["class_utilisation"] = util
    rec["path_fraction"] = {"roofline_ms_per_step": t_roof * 1e3, "measured_ms_per_step": ms_step,
                            "fraction": t_roof * 1e3 / ms_step}
    rec["reduced_gradient_mode"] = reduced_passes(P, cfg, Dc, J2, prec)
    progress(f"REDUCED mode: {rec['reduced_gradient_mode']['samples_per_s']:.1f} samples/s")
    # the same evaluation captured once as a HIP graph and replayed
    g = P.capture(cfg, Dc, 1.0, J2, precision=prec, workspace=P._ws, out=out)
    g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        g.launch()
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / 2
    g.free()
    rec["graph_replay"] = {"ms_per_step": gms, "samples_per_s": B / (gms / 1e3)}
    progress(f"graph replay: {gms:.1f} ms per step")
    rec["measured_peaks"] = measured_peaks()
    progress("peak probes done")
    if not args.no_optimiser:
        rec["optimiser"] = optimiser_leg(P, cfg, out, Dc, J2, prec, ms_step)
        progress("optimiser leg done")
    if not args.no_extra:
        # the same batch with the other strip precisions (default tuning of each), and
        # the other lattices of the benchmark set
        ws = out = None
        torch.cuda.empty_cache()
        rec["precision_modes"] = {args.precision: {"samples_per_s": value, "ms_per_pass": ms_step}}
        for pn in ("fp64", "fp32", "bf16x6"):
            if pn != args.precision:
                rec["precision_modes"][pn] = timed_passes(P, cfg, Dc, J2, bd.PRECISIONS[pn])
                progress(f"{pn}: {rec['precision_modes'][pn]['samples_per_s']:.1f} samples/s")
        rec["other_workloads"] = other_workloads(ctx)
    if args.serve_seconds > 0:
        ws = out = None
        P.free()
        torch.cuda.empty_cache()
        rec["serving"] = serving_leg(ctx, args.serve_seconds, args.serve_load,
                                     max_D=args.serve_max_d)
        progress("serving leg done")
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(args.workload, Dc, J2)
        progress("cpu baseline done")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
