"""Benchmark of the LSMS tau00 hot path on one MI355X.

One step = the whole path over one batch: LIZ extraction for every
(site, energy) instance, KKR matrix assembly and FP64 LU/Schur elimination
with tau00, for the 8192 instances of the fcc NiAu 50/50 workload with a
135-atom LIZ (N = 2160, lmax = 3, 256 sites x 32 contour energies).  Inputs
are synthetic and resident on the GPU before the timed region.

Prints one JSON line: metric, value (solves/s), timing, the roofline of the
dominant kernel (HIP-event timing, measured HBM traffic when the kernel
sources match the profiled ones), the other forms timed on the same
instances, the block row with ln det M, the phases of the path (build,
elimination, fused, fused plus the copy of tau00 to the host), the CPU
baselines (the oracle and LAPACK) and the check of the GPU's tau00 against
the oracle.
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
TRAFFIC_PER_INSTANCE = {("fp64", "90c86cd25f803934"): 2.0338e+09, ("fp32ir", "90c86cd25f803934"): 1.1884e+09}
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


def host_cores() -> int:
    """Cores the CPU legs use: the cores this process may run on, at most 16
    (the CPU share of one GPU on the benchmark hosts, whatever the machine's
    total core count)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_sample_indices(w, n_sites: int = 2):
    """The oracle sample: every contour energy of the first Ni and the first
    Au centre of the workload (2 sites x 32 energies = 64 instances of the
    benchmark workload)."""
    sites = []
    for sp in (0, 1):
        cand = [c for c in np.unique(w.centre) if w.atom_species[c] == sp]
        if cand:
            sites.append(int(cand[0]))
    idx = [i for i in range(w.n_inst) if int(w.centre[i]) in sites[:n_sites]]
    return np.asarray(idx, dtype=int)


def cpu_baseline(w, n_threads: int, idx):
    """The oracle on a bounded sample of the same workload (the instances
    `idx`), OpenMP over instances, in batches of one instance per thread;
    returns the baseline record and the oracle's tau00 of the sample."""
    import inputs
    import oracle

    ws = inputs.subset(w, idx)
    liz_off, pos, spec = oracle.liz_batch(ws)
    oracle.set_threads(n_threads)
    taus, infos, rates = [], [], []
    t_all = time.perf_counter()
    for b0 in range(0, len(idx), n_threads):
        sl = slice(b0, min(len(idx), b0 + n_threads))
        wb = inputs.subset(ws, np.arange(sl.start, sl.stop))
        lo, po, sp = oracle.liz_batch(wb)
        t0 = time.perf_counter()
        tau, info = oracle.tau00_batch(wb.lmax, lo, po, sp, wb.energies, wb.e_idx, wb.delta, refine=2)
        rates.append((sl.stop - sl.start) / (time.perf_counter() - t0))
        taus.append(tau)
        infos.append(info)
    dt = time.perf_counter() - t_all
    rec = {"value": float(np.median(rates)), "unit": "solves/s", "cores": n_threads, "kind": "oracle",
           "sample": f"{len(idx)} instances of the same workload (every contour energy of two sites, N="
                     f"{w.kk * int(np.diff(liz_off).max())}), in {len(rates)} batches of one instance per "
                     f"OpenMP thread; value = median batch rate, {dt:.1f} s wall",
           "batch_rates": [float(r) for r in rates]}
    return rec, np.concatenate(taus), np.concatenate(infos)


def cpu_lapack(w, n_threads: int, idx, n_mats: int = 8):
    """Second CPU number: LAPACK zgetrf + zgetrs with kk right-hand sides (the
    first block column of M^-1) on matrices built by the oracle, BLAS threads
    over the same cores; the analog of the paper's AOCL CPU path."""
    import numpy
    import scipy
    from scipy.linalg import lapack
    from threadpoolctl import threadpool_limits

    import inputs
    import oracle

    ws = inputs.subset(w, idx[np.linspace(0, len(idx) - 1, n_mats).astype(int)])
    liz_off, pos, spec = oracle.liz_batch(ws)
    C, _ = oracle.gaunt(ws.lmax)
    kk = ws.kk
    dts = []
    with threadpool_limits(limits=n_threads):
        for i in range(ws.n_inst):
            a, b = liz_off[i], liz_off[i + 1]
            e = int(ws.e_idx[i])
            M, _ = oracle.build_m(ws.lmax, pos[a:b], spec[a:b], ws.energies[e], ws.delta[:, e, :], C)
            B = np.zeros((M.shape[0], kk), np.complex128, order="F")
            B[:kk, :kk] = np.eye(kk)
            t0 = time.perf_counter()
            lu, piv, inf = lapack.zgetrf(M, overwrite_a=True)
            x, inf2 = lapack.zgetrs(lu, piv, B, overwrite_b=True)
            dts.append(time.perf_counter() - t0)
    cfg = scipy.show_config(mode="dicts")["Build Dependencies"]["lapack"]
    return {"value": float(1.0 / np.median(dts)), "unit": "solves/s", "cores": n_threads, "kind": "lapack",
            "routine": "zgetrf + zgetrs, 16 right-hand sides" if kk == 16 else f"zgetrf + zgetrs, {kk} rhs",
            "lapack": f"{cfg.get('name')} {cfg.get('version')}", "numpy": numpy.__version__,
            "sample": f"{ws.n_inst} matrices of the same workload, one at a time with BLAS threads over the "
                      f"cores; value = 1 / median time per matrix (factor + solve, build excluded)"}


def oracle_check(w, idx, ref, rinfo, tau, info, precision, outputs):
    """Compares the timed run's tau00 (and each other form's) on the oracle's
    sample: per-instance rel_F and the elementwise error of [M^-1]_00 =
    tau00 diag(t_0)^-1 relative to its largest entry; the bar is 1e-12 for
    the FP64 path and 1e-10 for the other forms."""
    import oracle

    kk = w.kk
    lv = np.floor(np.sqrt(np.arange(kk)) + 1e-9).astype(int)
    t0 = np.stack([oracle.tmat(w.lmax, w.energies[w.e_idx[i]], w.delta[w.atom_species[w.centre[i]], w.e_idx[i]])[lv]
                   for i in idx])
    res = {"instances": int(len(idx)), "oracle_info_nonzero": int(np.count_nonzero(rinfo)), "pass": True}
    runs = {"timed_" + precision: (tau, 1e-12 if precision == "fp64" else 1e-10)}
    for k, v in outputs.items():
        runs[k] = (v, 1e-10)
    for name, (t, bar) in runs.items():
        got = t.view(-1, kk * kk)[torch_index(idx, t)].cpu().numpy().reshape(-1, kk, kk).transpose(0, 2, 1)
        rf = np.linalg.norm((got - ref).reshape(len(idx), -1), axis=1) / np.linalg.norm(ref.reshape(len(idx), -1),
                                                                                          axis=1)
        xe = np.array([np.abs(got[q] / t0[q][None, :] - ref[q] / t0[q][None, :]).max() /
                       np.abs(ref[q] / t0[q][None, :]).max() for q in range(len(idx))])
        ok = bool(rf.max() <= bar and xe.max() <= bar)
        res[name] = {"max_rel_F_vs_oracle": float(rf.max()), "max_M_inv_00_err_vs_oracle": float(xe.max()),
                     "bar": bar, "pass": ok}
        res["pass"] = res["pass"] and ok
    return res


def torch_index(idx, t):
    import torch

    return torch.as_tensor(np.asarray(idx), device=t.device)


def rel_f_rows(a, b):
    import torch

    return (torch.linalg.vector_norm(a - b, dim=1) / torch.linalg.vector_norm(b, dim=1)).max().item()


def time_forms(args, P, h, w, liz, energy, e_idx, delta, max_liz, tau64, fp64_rate, outputs):
    """The precision and learned forms on the same instances (one warm-up and
    one timed pass each, persistent launch), with their speedup over the FP64
    path and the largest per-instance deviation of their tau00 from it; each
    form's tau00 goes to outputs[form] (device)."""
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
        outputs["fp32ir"] = t32
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
            # routing calibrated on the training alloy: 8 sites x 32 energies
            pt = P.problem_for_workload(h, inputs.subset(inputs.config2(seed=1), np.arange(256)))
            cal = learned.calibrate_routing(h, pt, net.seeds(P.mlp_features(h, pt, inputs.A_LAT)), None, None,
                                            w.energies.shape[0], restart)
            del pt
            route = torch.as_tensor(cal["route_by_energy"]).to("cuda")[e_idx.long()].contiguous()
            work = torch.empty(P.gmres_workspace_size(h, prob, restart), dtype=torch.uint8, device="cuda")
            tl = torch.empty(w.n_inst * 256, dtype=torch.complex128, device="cuda")
            il = torch.empty(w.n_inst, dtype=torch.int32, device="cuda")
            sl = torch.empty(w.n_inst, dtype=torch.int32, device="cuda")
            centre = torch.as_tensor(w.centre, device="cuda")
            n_atoms = w.atom_pos.shape[0]

            def run():
                # every site of the benchmark alloy is a centre at every energy, so the
                # batch's own seeds hold the preconditioner block of every LIZ site
                lz = P.build_liz(h, torch.as_tensor(w.atom_pos, device="cuda"),
                                 torch.as_tensor(w.atom_species, device="cuda"), w.box, centre,
                                 torch.as_tensor(w.rc, device="cuda"), max_liz, with_atoms=True)
                prow = P.site_blocks(h, prob, lz["atom"][:int(prob.liz_off[-1].item())], centre, n_atoms)
                feat = P.mlp_features(h, prob, inputs.A_LAT)
                seed = net.seeds(feat)
                return P.tau00_gmres(h, prob, work, seed=seed, restart=restart, max_cycles=cal["max_cycles"],
                                     tol=1e-12, tau=tl, info=il, steps=sl, precond=seed, precond_row=prow,
                                     route=route)

            _, dt = timed(run)
            routed = int(((il & P.INFO_ROUTED) != 0).sum().item())
            fb = int(((il & P.INFO_LU_FALLBACK) != 0).sum().item())
            ran = (il & P.INFO_ROUTED) == 0
            res["learned"] = {"solves_per_s": w.n_inst / dt, "speedup_vs_fp64": w.n_inst / dt / fp64_rate,
                              "max_rel_F_vs_fp64": rel_f_rows(tl.view(-1, 256), tau64), "routed_to_lu": routed,
                              "lu_fallbacks": fb,
                              "errors": int(((il & ~(P.INFO_ROUTED | P.INFO_LU_FALLBACK)) != 0).sum().item()),
                              "mean_gmres_block_steps_unrouted": float(sl[ran].double().mean().item())
                              if bool(ran.any()) else 0.0,
                              "routing": {"t_block_step_ms": 1e3 * cal["t_step_s"], "t_direct_ms": 1e3 * cal["t_lu_s"],
                                          "max_cycles": cal["max_cycles"],
                                          "gmres_energies": [int(e) for e in np.flatnonzero(cal["route_by_energy"] == 0)],
                                          "calibration_mean_steps_by_energy":
                                              [round(float(x), 1) for x in cal["mean_steps_by_energy"]]},
                              "preconditioner": "block-diagonal, the network's [M^-1]_00 at each LIZ site",
                              "train_loss_first_last": [losses[0], float(np.mean(losses[-50:]))],
                              "train_seconds": t_train, "restart": restart}
            outputs["learned"] = tl.view(-1, 256)
            log(f"[bench] learned: {res['learned']}")
        except Exception as e:
            res["learned"] = {"error": repr(e)}
    return res


def time_row(args, P, h, w, liz, energy, e_idx, delta, max_liz, n: int = 256):
    """The block row of tau with ln det M (tau_row_batched) against tau00
    alone (tau00_batched) on the first n instances of the workload, both on
    M built by build_kkr (one pass each, HIP events around the elimination
    launches; M rebuilt before each).  With the CPU legs, the block rows and
    ln det M of instances 0 and 31 (both contour ends of the first site) are
    compared with the oracle."""
    import torch

    import inputs
    import oracle

    dev = torch.device("cuda:0")
    prob = P.Problem(w.lmax, liz["liz_off"][:n + 1], liz["pos"], liz["species"], energy, e_idx[:n], delta,
                     max_liz=max_liz)
    N = w.kk * (liz["liz_off"][1:n + 1] - liz["liz_off"][:n])
    m_off = torch.cumsum(N * N, 0) - N * N
    M = torch.empty(int((N * N).sum().item()), dtype=torch.complex128, device=dev)
    xg = torch.empty(n * P.BATCHED_WORK_PER_INST, dtype=torch.uint8, device=dev)
    rw = torch.empty(P.row_workspace_size(h, prob), dtype=torch.uint8, device=dev)
    opts = P.Opts(0, args.nb, 0, 0)

    def timed(fn):
        P.build_kkr(h, prob, M, m_off)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1) * 1e-3

    timed(lambda: P.tau00_batched(h, prob, M, m_off, opts, work=xg))
    _, t_tau = timed(lambda: P.tau00_batched(h, prob, M, m_off, opts, work=xg))
    (rows, roff, ld, tau, info), t_row = timed(lambda: P.tau_row_batched(h, prob, M, m_off, opts, work=rw))
    res = {"instances": n, "N": int(N.max().item()), "row_and_logdet_solves_per_s": n / t_row,
           "tau00_batched_solves_per_s": n / t_tau, "time_ratio_row_over_tau00": t_row / t_tau,
           "errors": int((info != 0).sum().item()),
           "kernels": "tau_row_fp64_kernel vs lu_schur_fp64_kernel, one launch each"}
    if not args.no_cpu:
        pick = [0, 31]
        wp = inputs.subset(w, pick)
        oracle.set_threads(2)
        ref_rows, rinfo = oracle.tau_row_workload(wp)
        ref_ld, linfo = oracle.logdet_workload(wp)
        kk = w.kk
        r = rows.cpu().numpy()
        ro = roff.cpu().numpy()
        Nn = N.cpu().numpy()
        rf = [float(np.linalg.norm(r[ro[i]:ro[i] + kk * Nn[i]].reshape(Nn[i], kk).T - ref_rows[q]) /
                    np.linalg.norm(ref_rows[q])) for q, i in enumerate(pick)]
        ldg = ld.cpu().numpy()[pick]
        dld = np.abs(ldg.real - ref_ld.real).max(), np.abs(np.angle(np.exp(1j * (ldg.imag - ref_ld.imag)))).max()
        res["oracle_check"] = {"instances": pick, "max_row_rel_F": max(rf), "max_logdet_abs_err": float(max(dld)),
                               "bars": [1e-12, 1e-10],
                               "pass": bool(max(rf) <= 1e-12 and max(dld) <= 1e-10 and np.all(rinfo == 0))}
    del M, xg, rw
    return res


def time_phases(args, P, h, w, liz, energy, e_idx, delta, max_liz, n: int = 256):
    """The phases of the path on the first n instances (one per compute unit),
    each one pass after a warm-up, HIP events on the current stream: the
    build of M alone (build_kkr into a caller buffer), the elimination alone
    (tau00_batched on that M), the fused path that the benchmark times
    (tau00_solve, persistent: build and elimination in one kernel, M in a
    workspace slot), and the fused path plus the copy of tau00 to host
    memory (end to end, wall clock)."""
    import torch

    dev = torch.device("cuda:0")
    prob = P.Problem(w.lmax, liz["liz_off"][:n + 1], liz["pos"], liz["species"], energy, e_idx[:n], delta,
                     max_liz=max_liz)
    N = w.kk * (liz["liz_off"][1:n + 1] - liz["liz_off"][:n])
    m_off = torch.cumsum(N * N, 0) - N * N
    M = torch.empty(int((N * N).sum().item()), dtype=torch.complex128, device=dev)
    xg = torch.empty(n * P.BATCHED_WORK_PER_INST, dtype=torch.uint8, device=dev)
    opts = P.Opts(0, args.nb, 0, 0)
    fopts = P.Opts(P.PREC_FP64, args.nb, 0, P.PERSISTENT)
    work = torch.empty(P.workspace_size(h, prob, 0, fopts), dtype=torch.uint8, device=dev)
    tau = torch.empty((n, w.kk * w.kk), dtype=torch.complex128, device=dev)
    info = torch.empty(n, dtype=torch.int32, device=dev)
    host = torch.empty((n, w.kk * w.kk), dtype=torch.complex128, pin_memory=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    t_build = timed(lambda: P.build_kkr(h, prob, M, m_off))
    t_factor = timed(lambda: (P.build_kkr(h, prob, M, m_off),
                              P.tau00_batched(h, prob, M, m_off, opts, tau=tau, info=info, work=xg))) - t_build
    t_fused = timed(lambda: P.tau00_solve(h, prob, work, fopts, tau=tau, info=info))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.tau00_solve(h, prob, work, fopts, tau=tau, info=info)
    host.copy_(tau, non_blocking=True)
    torch.cuda.synchronize()
    t_e2e = (time.perf_counter() - t0) * 1e3
    res = {"instances": n, "N": int(N.max().item()),
           "build_ms": t_build, "factor_ms": t_factor, "fused_ms": t_fused,
           "fused_plus_tau00_d2h_ms": t_e2e, "tau00_bytes": int(tau.numel() * 16),
           "build_share_of_separate": t_build / (t_build + t_factor),
           "errors": int((info != 0).sum().item()),
           "kernels": "build_kkr_kernel; lu_schur_fp64_kernel; tau00_persistent_kernel (build + elimination)"}
    del M, xg, work
    return res


def bench_large(args, canted: bool = False):
    """One matrix across the whole GPU (tau00_large) at the paper's
    non-canted NiAu rank N = 6225 (lmax = 4, 249-atom LIZ), or with `canted`
    at its spin-canted NiAu rank 12450 (canted moments, spin-split wells):
    the instances are solved one after another (build, then tau00_large),
    HIP events around each tau00_large; the golden oracle instances are
    checked."""
    import torch

    import inputs
    import paper_2308_16317_amd as P

    w_all = inputs.config_large_canted() if canted else inputs.config_large()
    gname = "large_canted_tau00.npz" if canted else "large_tau00.npz"
    g = np.load(os.path.join(ROOT, "tests", "golden", gname), allow_pickle=False)
    idx = list(g["idx"]) + list(range(1, 1 + max(0, (args.n_inst or (4 if canted else 6)) - 2)))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    h = P.Handle()
    probs = [P.problem_for_workload(h, inputs.subset(w_all, [i])) for i in idx]
    N = probs[0].kc * probs[0].max_liz
    M = torch.empty(N * N, dtype=torch.complex128, device=dev)
    m_off = torch.zeros(1, dtype=torch.int64, device=dev)
    build = P.build_kkr_spin if canted else P.build_kkr
    work = None
    ms, taus = [], []
    for it in range(args.warmup + args.steps):
        for q, prob in enumerate(probs):
            build(h, prob, M, m_off)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            tau, info = P.tau00_large(h, prob, M, work=work)
            e1.record()
            torch.cuda.synchronize()
            if int(info.item()) != 0:
                raise RuntimeError(f"tau00_large info {int(info.item())}")
            if it >= args.warmup:
                ms.append(e0.elapsed_time(e1))
                if it == args.warmup and q < 2:
                    taus.append(tau.cpu().numpy()[0])
    flops = 8.0 / 3.0 * float(N) ** 3
    med = float(np.median(ms))
    rf = [float(np.linalg.norm(t - r) / np.linalg.norm(r)) for t, r in zip(taus, g["tau"])]
    kind = ("spin-canted (cone 60 deg, spin-split wells), rank 2 kk 249" if canted else "non-canted")
    out = {"metric": f"single-instance {'spin-canted ' if canted else ''}τ00 solves/s at N={N} (whole GPU)",
           "value": 1e3 / med,
           "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": med,
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{w_all.name}: one (site, E) instance at a time, 6x6x6 fcc NiAu 50/50, 249-atom "
                                  f"LIZ, {kind}, N={N}, lmax=4, complex FP64 LU/Schur over all compute units",
                      "instances": len(idx), "N": N},
           "roofline": {"bound": "mfma", "achieved": flops / (med * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": flops / (med * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "traffic": None, "kernel": "tau00_large (panel, U12 and MFMA update kernels, look-ahead)",
                        "ms_per_launch": med, "ms_min": float(np.min(ms))},
           "oracle_check": {"instances": [int(i) for i in g["idx"]], "max_rel_F_vs_oracle": max(rf), "bar": 1e-12,
                            "pass": bool(max(rf) <= 1e-12), "source": f"tests/golden/{gname} (oracle)"}}
    print(json.dumps(out), flush=True)
    if not out["oracle_check"]["pass"]:
        sys.exit(1)


def bench_canted(args, lmax: int):
    """The spin-canted path (tau00_spin_solve, persistent fused kernel, FP64)
    on the spin-canted recipe: the 135-atom-LIZ systems with canted moments,
    rank 2 kk 135 (4320 at lmax = 3, 6750 at lmax = 4).  The timed batch is
    the first n instances (every energy of the first n / 32 sites); the
    instances of tests/golden/canted_tau00.npz are solved by the same call
    and compared with those oracle values."""
    import torch

    import inputs
    import paper_2308_16317_amd as P

    w_all = inputs.config_canted(lmax=lmax)
    n = args.n_inst or (1024 if lmax == 3 else 256)
    w = inputs.subset(w_all, np.arange(n))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    h = P.Handle()
    prob = P.problem_for_workload(h, w)
    kc = prob.kc
    opts = P.Opts(0, args.nb, 0, P.PERSISTENT)
    work = torch.empty(P.spin_workspace_size(h, prob, 0, opts), dtype=torch.uint8, device=dev)
    tau = torch.empty(n * kc * kc, dtype=torch.complex128, device=dev)
    info = torch.empty(n, dtype=torch.int32, device=dev)
    log(f"[bench] canted lmax={lmax}: {n} instances, rank {kc * prob.max_liz}, workspace {work.numel() / 2**30:.1f} GiB")
    ev = []
    for it in range(args.warmup + args.steps):
        if it == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        P.tau00_spin_solve(h, prob, work, opts, tau=tau, info=info)
        e1.record()
        if it >= args.warmup:
            ev.append((e0, e1))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if int((info != 0).sum().item()):
        raise RuntimeError(f"canted: info values {torch.unique(info).tolist()}")
    Ns = kc * np.diff(prob.liz_off.cpu().numpy()).astype(np.float64)
    flops = float(np.sum(8.0 / 3.0 * Ns ** 3))
    ms = [a.elapsed_time(b) for a, b in ev]
    ach = flops / (np.mean(ms) * 1e-3) / 1e12
    del work
    # oracle values of the golden instances, solved by the same entry point
    check = {"pass": None}
    gpath = os.path.join(ROOT, "tests", "golden", "canted_tau00.npz")
    if os.path.exists(gpath):
        g = np.load(gpath, allow_pickle=False)
        gi, gref = g[f"idx_l{lmax}"], g[f"tau_l{lmax}"]
        wg = inputs.subset(w_all, gi)
        pg = P.problem_for_workload(h, wg)
        wk = torch.empty(P.spin_workspace_size(h, pg, 0, opts), dtype=torch.uint8, device=dev)
        tg, ig = P.tau00_spin_solve(h, pg, wk, opts)
        torch.cuda.synchronize()
        tg = tg.cpu().numpy()
        rf = np.linalg.norm((tg - gref).reshape(len(gi), -1), axis=1) / np.linalg.norm(gref.reshape(len(gi), -1),
                                                                                          axis=1)
        check = {"instances": [int(x) for x in gi], "max_rel_F_vs_oracle": float(rf.max()), "bar": 1e-12,
                 "pass": bool(rf.max() <= 1e-12 and np.all(ig.cpu().numpy() == 0)),
                 "source": "tests/golden/canted_tau00.npz (oracle)"}
    out = {
        "metric": f"spin-canted τ00 solves/s at rank {int(Ns.max())}",
        "value": n * args.steps / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w_all.name}: fcc NiAu 50/50 with canted moments (cone 60 deg), spin-split "
                               f"square wells, first {n} (site, E) instances, 135-atom LIZ, rank "
                               f"{int(Ns.max())}, lmax={lmax}, complex FP64 LU/Schur",
                   "n_inst": n, "N": int(Ns.max()), "lmax": lmax, "mode": "persistent", "precision": "fp64"},
        "tflops": flops * args.steps / dt / 1e12,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / FP64_PEAK_TFLOPS, "traffic": None,
                     "traffic_source": "no counters taken on this workload",
                     "kernel": "tau00_persistent_kernel (spin-canted build + elimination)",
                     "ms_per_launch": float(np.mean(ms)), "instances_per_launch": n},
        "oracle_check": check,
    }
    print(json.dumps(out), flush=True)
    if check["pass"] is False:
        log("[bench] canted tau00 outside the tolerance against the oracle")
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
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
    ap.add_argument("--workload", choices=["benchmark", "ragged", "lmax4", "canted", "canted4", "large", "large_canted"],
                    default="benchmark",
                    help="benchmark: 8192 instances at N = 2160 (the metric's workload); ragged: 1024 instances of "
                         "the vacancy/noise supercell with cutoffs 1.7a-2.1a (N = 1200-2400); lmax4: the benchmark "
                         "systems at lmax = 4 (N = 3375); canted / canted4: the spin-canted path at rank 4320 / "
                         "6750 (first 1024 / 256 instances unless --n-inst); large: one N = 6225 matrix at a "
                         "time across the whole GPU (tau00_large); large_canted: the same at the spin-canted "
                         "rank 12450")
    ap.add_argument("--forms", choices=["none", "fp32ir", "all"], default="all",
                    help="also time the other forms on the same instances (persistent launch) and report them "
                         "with their speedup over the FP64 path and their deviation from it")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU legs (oracle baseline, LAPACK number) and the oracle check of tau00")
    ap.add_argument("--cpu-threads", type=int, default=0, help="threads of the CPU legs (0 = host_cores())")
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="oracle sample: at most this many instances (every contour energy of two sites)")
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

    if args.workload in ("large", "large_canted"):
        bench_large(args, canted=args.workload == "large_canted")
        return
    if args.workload in ("canted", "canted4"):
        bench_canted(args, 3 if args.workload == "canted" else 4)
        return

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
        raise RuntimeError(f"{bad} instances reported an error in info (values {torch.unique(info).tolist()})")
    n_inst = w.n_inst
    Ns = kk * sizes.astype(np.float64)
    flops_step = float(np.sum(8.0 / 3.0 * Ns ** 3))
    ms = 1e3 * dt / args.steps
    lu_ms = [e0.elapsed_time(e1) for (e0, e1, _, _) in events]
    lu_flops = [float(np.sum(8.0 / 3.0 * (Nc.double().cpu().numpy()) ** 3)) for (_, _, _, Nc) in events]
    ach = float(np.sum(lu_flops) / (np.sum(lu_ms) * 1e-3) / 1e12)
    peak = FP32_PEAK_TFLOPS if args.precision == "fp32ir" else FP64_PEAK_TFLOPS
    src_hash = kernel_source_hash()
    per_inst = TRAFFIC_PER_INSTANCE.get((args.precision, src_hash))
    # measured on the N = 2160 benchmark instances only
    traffic = None if (per_inst is None or args.mode == "chunked" or args.workload != "benchmark") else per_inst * chunk
    # bound: algorithmic intensity (8/3 N^3 flops over the 32 N^2 bytes of
    # reading and writing M once) against the ridge peak / 8 TB/s
    intensity = float(np.sum(8.0 / 3.0 * Ns ** 3) / np.sum(32.0 * Ns ** 2))
    bound = "mfma" if intensity > peak / 8.0 else "hbm"
    form = ("complex FP32 LU + FP64 iterative refinement to 1e-12 (FP64 fallback per instance)"
            if args.precision == "fp32ir" else "complex FP64 LU/Schur")
    lu_s = np.asarray(lu_ms) * 1e-3
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
        "solves_per_s_median_launch": float(np.median([e[2] / t for e, t in zip(events, lu_s)])),
        "roofline": {"bound": bound, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": traffic,
                     "traffic_source": (f"rocprofv3 FETCH_SIZE/WRITE_SIZE per instance, calibrated on a copy "
                                        f"kernel, profiles/{'tau00_mixed_persistent' if args.precision == 'fp32ir' else 'tau00_persistent_fp64'}"
                                        f"_n2160_hbm_traffic.md, kernel source hash {src_hash}")
                                       if traffic is not None else
                                       f"no counters for kernel source hash {src_hash} on this workload",
                     "algorithmic_intensity_flop_per_byte": intensity,
                     "kernel": kernel, "ms_per_launch": float(np.mean(lu_ms)),
                     "ms_per_launch_median": float(np.median(lu_ms)),
                     "instances_per_launch": chunk},
    }
    outputs = {}
    if args.forms != "none" and args.precision == "fp64" and args.mode != "chunked":
        out["forms"] = time_forms(args, P, h, w, liz, energy, e_idx, delta, max_liz, tau, n_inst * args.steps / dt,
                                  outputs)
    if args.forms == "all" and args.workload == "benchmark":
        try:
            out["block_row_logdet"] = time_row(args, P, h, w, liz, energy, e_idx, delta, max_liz)
            log(f"[bench] block row: {out['block_row_logdet']}")
        except Exception as e:  # reported, not fatal
            out["block_row_logdet"] = {"error": repr(e)}
    if args.forms == "all" and args.workload == "benchmark" and args.mode != "chunked":
        try:
            out["phases"] = time_phases(args, P, h, w, liz, energy, e_idx, delta, max_liz)
            log(f"[bench] phases: {out['phases']}")
        except Exception as e:  # reported, not fatal
            out["phases"] = {"error": repr(e)}
    if not args.no_cpu:
        nthr = args.cpu_threads or host_cores()
        idx = cpu_sample_indices(w)[:args.cpu_sample]
        log(f"[bench] cpu baseline: oracle on {nthr} threads, {len(idx)} instances")
        out["cpu_baseline"], ref, rinfo = cpu_baseline(w, nthr, idx)
        log(f"[bench] cpu baseline: {out['cpu_baseline']}")
        out["oracle_check"] = oracle_check(w, idx, ref, rinfo, tau, info, args.precision, outputs)
        log(f"[bench] oracle check: {out['oracle_check']}")
        try:
            out["cpu_lapack"] = cpu_lapack(w, nthr, idx)
            log(f"[bench] cpu lapack: {out['cpu_lapack']}")
        except Exception as e:  # reported, not fatal
            out["cpu_lapack"] = {"error": repr(e)}
    out["paper_speedups"] = PAPER_SPEEDUPS
    print(json.dumps(out), flush=True)
    if "oracle_check" in out and not out["oracle_check"]["pass"]:
        log("[bench] tau00 outside the tolerance against the oracle")
        sys.exit(1)


if __name__ == "__main__":
    main()
