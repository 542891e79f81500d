"""Benchmark of the LSMS tau00 hot path on one MI355X.

One step = the whole path over one batch: LIZ extraction for every
(site, energy) instance, KKR matrix assembly and FP64 LU/Schur elimination
with tau00, for the 8192 instances of the fcc NiAu 50/50 workload with a
135-atom LIZ (N = 2160, lmax = 3, 256 sites x 32 contour energies).  Inputs
are synthetic and resident on the GPU before the timed region.

Prints one JSON line: metric, value (solves/s), timing, the roofline of the
dominant kernel (HIP-event timing, measured HBM traffic when the kernel
sources match the profiled ones), the other forms timed on the same
instances, and the CPU oracle baseline.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

# HBM bytes per instance moved by the fused kernel (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, each scaled by the counts of a plain copy of known size), valid
# only for the kernel code whose hash is given; null otherwise.
TRAFFIC_PER_INSTANCE = {("fp64", "08af91cf900550a5"): 2.031e9, ("fp32ir", "08af91cf900550a5"): 1.290e9}
KERNEL_SOURCES = ("kkr_device.h", "lu_device.h", "lu_fp64.hip", "lsms_common.h")


def kernel_source_hash(csrc: str = "") -> str:
    """Hash of the fused kernel's sources (in `csrc`, default the package's)
    with comments and white space removed, so that an edit of comments alone
    keeps the measured figures."""
    import hashlib
    import re

    csrc = csrc or os.path.join(ROOT, "paper_2308_16317_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(re.sub(r"\s+", "", src).encode())
    return h.hexdigest()[:16]

METRIC = "τ00 solves/s at N=2160, 1e-10 rel: mixed/batched vs plain FP64; TFLOP/s vs peak"

# The paper's own GPU-over-CPU speedups, for context only: ratios of the
# whole-program MuST wall-clock times (I/O excluded) in its table of
# performance results (Sec. 4.2), complex FP64 throughout, against its
# 32-core EPYC 7742 reference (28 cores for the five-element alloy).  The
# paper gives no per-inverse time, so none of these is comparable with the
# solves/s measured here.
PAPER_SPEEDUPS = [
    {"workload": "NiAu 30/70 non-spin-canted, lmax=4, KKR rank 6225", "gpu": "2x A100-40G, 16 MPI ranks",
     "cpu": "32 EPYC 7742 cores", "seconds": [1014, 2489], "speedup": 2.45},
    {"workload": "NiAu 30/70 non-spin-canted, lmax=4, KKR rank 6225", "gpu": "8x V100-16G, 32 MPI ranks",
     "cpu": "32 EPYC 7742 cores", "seconds": [593, 2489], "speedup": 4.20},
    {"workload": "NiAu 30/70 spin-canted, lmax=4, KKR rank 12450", "gpu": "8x A100-80G, 32 MPI ranks",
     "cpu": "32 EPYC 7742 cores", "seconds": [1821, 19002], "speedup": 10.4},
    {"workload": "NiAu 30/70 spin-canted, lmax=4, KKR rank 12450", "gpu": "8x V100-32G, 16 MPI ranks",
     "cpu": "32 EPYC 7742 cores", "seconds": [3375, 19002], "speedup": 5.63},
    {"workload": "CoCrFeMnNi spin-canted, lmax=4, KKR rank 6750", "gpu": "2x A100-40G, 16 MPI ranks",
     "cpu": "28 EPYC 7742 cores", "seconds": [1401, 4647], "speedup": 3.32},
]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, n_threads: int):
    """The oracle on a bounded sample of the same workload: one instance per
    thread (OpenMP over instances), at both contour ends and mid-contour."""
    import inputs
    import oracle

    n = max(1, n_threads)
    idx = np.linspace(0, w.n_inst - 1, n).astype(int)
    ws = inputs.subset(w, idx)
    liz_off, pos, spec = oracle.liz_batch(ws)
    oracle.set_threads(n_threads)
    t0 = time.perf_counter()
    tau, info = oracle.tau00_batch(ws.lmax, liz_off, pos, spec, ws.energies, ws.e_idx, ws.delta, refine=2)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "solves/s", "cores": n_threads, "kind": "oracle",
            "sample": f"{n} instances of the same workload (N=2160), one per OpenMP thread, "
                      f"{dt:.1f} s wall"}


def rel_f_rows(a, b):
    import torch

    return (torch.linalg.vector_norm(a - b, dim=1) / torch.linalg.vector_norm(b, dim=1)).max().item()


def time_forms(args, P, h, w, liz, energy, e_idx, delta, max_liz, tau64, fp64_rate):
    """The precision and learned forms on the same instances (one warm-up and
    one timed pass each, persistent launch), with their speedup over the FP64
    path and the largest per-instance deviation of their tau00 from it."""
    import torch

    import inputs
    from paper_2308_16317_amd import learned

    prob = P.Problem(w.lmax, liz["liz_off"], liz["pos"], liz["species"], energy, e_idx, delta, max_liz=max_liz)
    res = {"fp64": {"solves_per_s": fp64_rate, "reference": "the FP64 path of this run"}}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    try:
        opts = P.Opts(P.PREC_FP32_IR, args.nb, 0, P.PERSISTENT, 0, 0, args.tol)
        work = torch.empty(P.workspace_size(h, prob, 0, opts), dtype=torch.uint8, device="cuda")
        t32 = torch.empty_like(tau64)
        i32 = torch.empty(w.n_inst, dtype=torch.int32, device="cuda")
        _, dt = timed(lambda: P.tau00_solve(h, prob, work, opts, tau=t32, info=i32))
        del work
        fb = int((i32 == P.INFO_FP64_FALLBACK).sum().item())
        res["fp32ir"] = {"solves_per_s": w.n_inst / dt, "speedup_vs_fp64": w.n_inst / dt / fp64_rate,
                         "max_rel_F_vs_fp64": rel_f_rows(t32, tau64), "fp64_fallbacks": fb,
                         "errors": int((i32 != 0).sum().item()) - fb,
                         "peak_tflops": FP32_PEAK_TFLOPS}
        log(f"[bench] fp32ir: {res['fp32ir']}")
    except Exception as e:  # reported, not fatal: the FP64 line stands on its own
        res["fp32ir"] = {"error": repr(e)}
    if args.forms == "all":
        try:
            t0 = time.perf_counter()
            net, losses = learned.train_on(h, inputs.config2(seed=1), inputs.A_LAT, inputs.mlp_init(seed=0),
                                           steps=3000)
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
            restart = 8
            work = torch.empty(P.gmres_workspace_size(h, prob, restart), dtype=torch.uint8, device="cuda")
            tl = torch.empty(w.n_inst * 256, dtype=torch.complex128, device="cuda")
            il = torch.empty(w.n_inst, dtype=torch.int32, device="cuda")
            sl = torch.empty(w.n_inst, dtype=torch.int32, device="cuda")

            def run():
                feat = P.mlp_features(h, prob, inputs.A_LAT)
                seed = net.seeds(feat)
                return P.tau00_gmres(h, prob, work, seed=seed, restart=restart, max_cycles=20, tol=1e-12, tau=tl,
                                     info=il, steps=sl)

            _, dt = timed(run)
            fb = int((il == P.INFO_LU_FALLBACK).sum().item())
            res["learned"] = {"solves_per_s": w.n_inst / dt, "speedup_vs_fp64": w.n_inst / dt / fp64_rate,
                              "max_rel_F_vs_fp64": rel_f_rows(tl.view(-1, 256), tau64), "lu_fallbacks": fb,
                              "errors": int((il != 0).sum().item()) - fb,
                              "mean_gmres_block_steps": float(sl.double().mean().item()),
                              "train_loss_first_last": [losses[0], float(np.mean(losses[-50:]))],
                              "train_seconds": t_train, "restart": restart}
            log(f"[bench] learned: {res['learned']}")
        except Exception as e:
            res["learned"] = {"error": repr(e)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["chunked", "persistent", "graph"], default="persistent",
                    help="chunked: build_kkr + tau00_batched per pass; persistent: tau00_solve with one "
                         "fused persistent kernel; graph: the same, replayed from a captured hipGraph")
    ap.add_argument("--precision", choices=["fp64", "fp32ir"], default="fp64",
                    help="fp64: complex FP64 elimination; fp32ir: complex FP32 factorisation and solves with "
                         "FP64 iterative refinement (persistent and graph modes)")
    ap.add_argument("--tol", type=float, default=0.0, help="refinement tolerance of fp32ir (0 = library default)")
    ap.add_argument("--chunk", type=int, default=1024, help="instances per build/LU launch (chunked)")
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--n-inst", type=int, default=0, help="limit the batch (0 = all 8192)")
    ap.add_argument("--workload", choices=["benchmark", "ragged", "lmax4"], default="benchmark",
                    help="benchmark: 8192 instances at N = 2160 (the metric's workload); ragged: 1024 instances of "
                         "the vacancy/noise supercell with cutoffs 1.7a-2.1a (N = 1200-2400); lmax4: the benchmark "
                         "systems at lmax = 4 (N = 3375)")
    ap.add_argument("--forms", choices=["none", "fp32ir", "all"], default="all",
                    help="also time the other forms on the same instances (persistent launch) and report them "
                         "with their speedup over the FP64 path and their deviation from it")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run three plain device copies of MIB MiB (the reference kernel whose "
                         "FETCH_SIZE / WRITE_SIZE counters scale the HBM-traffic measurement) and exit")
    args = ap.parse_args()
    if args.copy_calib:
        import torch

        a = torch.ones((args.copy_calib << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calib} MiB three times")
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.precision == "fp32ir" and args.mode == "chunked":
        print(json.dumps({"error": "--precision fp32ir runs through tau00_solve: use --mode persistent or graph"}))
        sys.exit(2)

    import torch

    import inputs
    import paper_2308_16317_amd as P

    w = {"benchmark": inputs.config2, "ragged": inputs.config4, "lmax4": inputs.config3}[args.workload]()
    if args.n_inst:
        w = inputs.subset(w, np.arange(args.n_inst))
    log(f"[bench] workload {w.name}: {w.n_inst} instances")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    h = P.Handle()
    # inputs resident on the device
    atom_pos = torch.as_tensor(w.atom_pos, device=dev)
    atom_spec = torch.as_tensor(w.atom_species, device=dev)
    centre = torch.as_tensor(w.centre, device=dev)
    rc = torch.as_tensor(w.rc, device=dev)
    energy = torch.as_tensor(w.energies, device=dev)
    e_idx = torch.as_tensor(w.e_idx, device=dev)
    delta = torch.as_tensor(w.delta, device=dev)
    max_liz = 160  # bound on the 135-atom LIZ of this workload (checked every step)
    kk = w.kk
    tau = torch.empty((w.n_inst, kk * kk), dtype=torch.complex128, device=dev)
    info = torch.empty(w.n_inst, dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream(device=dev) if args.mode == "graph" else torch.cuda.current_stream()
    events = []  # (start, end, instances, N per instance) around each launch of the dominant kernel
    if args.mode == "chunked":
        chunk = min(args.chunk, w.n_inst)
        nslot = kk * max_liz
        M = torch.empty(chunk * nslot * nslot, dtype=torch.complex128, device=dev)
        opts = P.Opts(0, args.nb, 0, 0)
        kernel = "lu_schur_fp64_kernel"
    else:
        chunk = w.n_inst
        flags = P.PERSISTENT | (P.GRAPH if args.mode == "graph" else 0)
        if args.precision == "fp32ir":
            opts = P.Opts(P.PREC_FP32_IR, args.nb, 0, flags, 0, 0, args.tol)
            kernel = "tau00_mixed_persistent_kernel (LIZ-to-tau00: build + FP32 LU + FP64 refinement)"
        else:
            opts = P.Opts(P.PREC_FP64, args.nb, 0, flags)
            kernel = "tau00_persistent_kernel (LIZ-to-tau00: build + elimination)"
        work = None

    liz_buf = None

    def step(record: bool):
        nonlocal work, liz_buf
        liz = P.build_liz(h, atom_pos, atom_spec, w.box, centre, rc, max_liz, out=liz_buf)
        liz_buf = liz
        N = kk * (liz["liz_off"][1:] - liz["liz_off"][:-1])
        for i0 in range(0, w.n_inst, chunk):
            n = min(chunk, w.n_inst - i0)
            sl = slice(i0, i0 + n)
            # instance i of the pass owns LIZ rows liz_off[i0+i] .. liz_off[i0+i+1]-1
            prob = P.Problem(w.lmax, liz["liz_off"][i0:i0 + n + 1], liz["pos"], liz["species"], energy,
                             e_idx[sl], delta, max_liz=max_liz)
            if args.mode == "chunked":
                Nc = N[sl]
                m_off = torch.cumsum(Nc * Nc, 0) - Nc * Nc
                P.build_kkr(h, prob, M, m_off)
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            if args.mode == "chunked":
                P.tau00_batched(h, prob, M, m_off, opts, tau=tau[sl], info=info[sl])
            else:
                if work is None:
                    work = torch.empty(P.workspace_size(h, prob, 0, opts), dtype=torch.uint8, device=dev)
                P.tau00_solve(h, prob, work, opts, tau=tau[sl], info=info[sl])
            if record:
                e1.record(stream)
                events.append((e0, e1, n, N[sl]))
        return liz

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            liz = step(True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    sizes = (liz["liz_n"]).cpu().numpy()
    if sizes.max() > max_liz:
        raise RuntimeError("LIZ larger than the bench's max_liz")
    fallback = int((info == P.INFO_FP64_FALLBACK).sum().item()) if args.precision == "fp32ir" else 0
    bad = int((info != 0).sum().item()) - fallback
    if bad:
        raise RuntimeError(f"{bad} instances reported an error in info")
    n_inst = w.n_inst
    Ns = kk * sizes.astype(np.float64)
    flops_step = float(np.sum(8.0 / 3.0 * Ns ** 3))
    ms = 1e3 * dt / args.steps
    lu_ms = [e0.elapsed_time(e1) for (e0, e1, _, _) in events]
    lu_flops = [float(np.sum(8.0 / 3.0 * (Nc.double().cpu().numpy()) ** 3)) for (_, _, _, Nc) in events]
    ach = float(np.sum(lu_flops) / (np.sum(lu_ms) * 1e-3) / 1e12)
    peak = FP32_PEAK_TFLOPS if args.precision == "fp32ir" else FP64_PEAK_TFLOPS
    per_inst = TRAFFIC_PER_INSTANCE.get((args.precision, kernel_source_hash()))
    # measured on the N = 2160 benchmark instances only
    traffic = None if (per_inst is None or args.mode == "chunked" or args.workload != "benchmark") else per_inst * chunk
    form = ("complex FP32 LU + FP64 iterative refinement to 1e-12 (FP64 fallback per instance)"
            if args.precision == "fp32ir" else "complex FP64 LU/Schur")
    out = {
        "metric": METRIC,
        "value": n_inst * args.steps / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32ir" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"{w.name}: fcc NiAu 50/50, 256 sites x 32 energies = {n_inst} instances, "
                                f"135-atom LIZ, N={int(Ns.max())}, lmax={w.lmax}, {form}")
                   if args.workload != "ragged" else
                               (f"{w.name}: 10x10x10 fcc NiAu supercell, 3% vacancies, 0.02a noise, {n_inst} "
                                f"(site, E) instances, cutoff 1.7a-2.1a, N={int(Ns.min())}-{int(Ns.max())}, "
                                f"lmax=3, {form}"),
                   "n_inst": n_inst, "N": int(Ns.max()), "lmax": w.lmax, "mode": args.mode,
                   "precision": args.precision, "instances_per_launch": chunk,
                   "fp64_fallbacks": fallback},
        "tflops": flops_step / (ms * 1e-3) / 1e12,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": traffic,
                     "kernel": kernel, "ms_per_launch": float(np.mean(lu_ms)),
                     "instances_per_launch": chunk},
    }
    if args.forms != "none" and args.precision == "fp64" and args.mode != "chunked":
        out["forms"] = time_forms(args, P, h, w, liz, energy, e_idx, delta, max_liz, tau, n_inst * args.steps / dt)
    if not args.no_cpu:
        nthr = args.cpu_threads or min(16, os.cpu_count() or 1)
        log(f"[bench] cpu baseline: oracle on {nthr} threads")
        out["cpu_baseline"] = cpu_baseline(w, nthr)
    out["paper_speedups"] = PAPER_SPEEDUPS
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
