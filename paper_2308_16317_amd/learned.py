"""Learned form: a small network that maps an instance's local environment
and energy to an approximation of tau00 and of [M^{-1}]_{00}; the latter
seeds the block-GMRES solve (`tau00_gmres`), whose fallback is the direct
FP64 path.

Training data are tau00 values the solver itself produced (`tau00_solve`);
training runs on the GPU through the library's own kernels (forward,
backward, MSE, AdamW).  The same network's outputs at every LIZ site's own
environment give a block-diagonal preconditioner, and a routing table,
calibrated on the training alloy, sends the energies where GMRES would cost
more than the direct elimination straight to it.  This module only sequences
the library's calls.
"""

from __future__ import annotations

import numpy as np
import torch

from . import lsms


class SeedNet:
    """The network's parameters (FP32 master, bf16 copy), its AdamW state and
    the target normalisation."""

    def __init__(self, h: lsms.Handle, init_params):
        self.h = h
        p = torch.as_tensor(np.asarray(init_params, dtype=np.float32)).to("cuda")
        if p.numel() != lsms.MLP_PARAMS:
            raise ValueError(f"expected {lsms.MLP_PARAMS} parameters, got {p.numel()}")
        self.params = p.contiguous()
        self.w_bf16 = torch.empty(lsms.MLP_PARAMS, dtype=torch.int16, device="cuda")
        lsms.mlp_cast(h, self.params, self.w_bf16)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.scale = None
        self.shift = None

    def set_normalisation(self, targets_raw: torch.Tensor):
        self.scale, self.shift = lsms.mlp_norm_stats(self.h, targets_raw)

    def forward(self, feat: torch.Tensor):
        return lsms.mlp_forward(self.h, self.params, self.w_bf16, feat)

    def train(self, feat: torch.Tensor, target: torch.Tensor, steps: int, batch: int = 512, lr: float = 2e-3,
              wd: float = 0.0, seed: int = 0, lr_final: float | None = None):
        """AdamW on the MSE between the network's outputs and the normalised
        targets; minibatches drawn from a seeded permutation.  Returns the
        per-step losses (host floats)."""
        n = feat.shape[0]
        batch = min(batch, n)
        g = torch.Generator(device="cpu").manual_seed(seed)
        act = torch.empty((batch, lsms.MLP_ACT), dtype=torch.float32, device="cuda")
        out = torch.empty((batch, 1024), dtype=torch.float32, device="cuda")
        dout = torch.empty((batch, 1024), dtype=torch.float32, device="cuda")
        grad = torch.empty(lsms.MLP_PARAMS, dtype=torch.float32, device="cuda")
        work = torch.empty((batch, 1280), dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        losses = []
        perm = torch.randperm(n, generator=g)
        pos = 0
        for it in range(steps):
            if pos + batch > n:
                perm = torch.randperm(n, generator=g)
                pos = 0
            idx = perm[pos:pos + batch].to("cuda")
            pos += batch
            fb = feat.index_select(0, idx).contiguous()
            tb = target.index_select(0, idx).contiguous()
            lsms.mlp_forward(self.h, self.params, self.w_bf16, fb, act=act, out=out)
            lsms.mlp_mse(self.h, out, tb, dout=dout, loss=loss)
            lsms.mlp_backward(self.h, self.w_bf16, fb, act, dout, grad=grad, work=work)
            self.step += 1
            rate = lr if lr_final is None else lr * (lr_final / lr) ** (it / max(1, steps - 1))
            lsms.mlp_adamw(self.h, self.params, self.w_bf16, self.m, self.v, grad, rate, self.step, wd=wd)
            losses.append(loss.clone())
        return [float(x.item()) for x in losses]

    def seeds(self, feat: torch.Tensor) -> torch.Tensor:
        """Approximations of [M^{-1}]_{00} ([n, 256] complex128) for tau00_gmres."""
        out, _ = self.forward(feat)
        return lsms.mlp_seed(self.h, out, self.scale, self.shift)


def solve_direct(h: lsms.Handle, prob: lsms.Problem) -> torch.Tensor:
    """tau00 of every instance by the FP64 path (persistent launch), as the
    [n, 256] complex128 column-major buffer the library writes."""
    opts = lsms.Opts(lsms.PREC_FP64, 0, 0, lsms.PERSISTENT)
    work = torch.empty(lsms.workspace_size(h, prob, 0, opts), dtype=torch.uint8, device="cuda")
    tau, info = lsms.tau00_solve(h, prob, work, opts)
    del work
    if int((info != 0).sum().item()):
        raise RuntimeError("the direct solver reported errors on the training set")
    return tau.transpose(1, 2).contiguous().reshape(-1, 256)


def train_on(h: lsms.Handle, w, a_lat: float, init_params, steps: int, batch: int = 512, lr: float = 2e-3,
             lr_final: float | None = 2e-4, max_liz: int = 1024):
    """Generate the training set of workload `w` with the direct solver,
    normalise it, and train a fresh network on it.  Returns (net, losses)."""
    prob = lsms.problem_for_workload(h, w, max_liz)
    tau = solve_direct(h, prob)
    feat = lsms.mlp_features(h, prob, a_lat)
    net = SeedNet(h, init_params)
    net.set_normalisation(lsms.mlp_targets(h, prob, tau))
    target = lsms.mlp_targets(h, prob, tau, net.scale, net.shift)
    losses = net.train(feat, target, steps, batch=batch, lr=lr, lr_final=lr_final)
    return net, losses


def preconditioner(h: lsms.Handle, prob: lsms.Problem, liz_atom: torch.Tensor, centre, n_atoms: int,
                   seeds: torch.Tensor):
    """Block-diagonal preconditioner of tau00_gmres_pc from the network's
    seeds of the batch itself: the block of a LIZ site is the seed of the
    instance centred on that site's atom at the same energy (identity where
    the batch has no such instance).  Returns (precond, precond_row)."""
    return seeds, lsms.site_blocks(h, prob, liz_atom, centre, n_atoms)


def _timed(fn):
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    r = fn()
    e1.record()
    torch.cuda.synchronize()
    return r, e0.elapsed_time(e1) * 1e-3


def calibrate_routing(h: lsms.Handle, prob: lsms.Problem, seeds, precond, precond_row, n_energy: int,
                      restart: int = 8, tol: float = 1e-12):
    """Routing table and step cap from a calibration batch (training alloy,
    at most one instance per compute unit so that one launch is one wave):
    the time of one block step t and of the direct elimination T follow from
    two GMRES launches that never converge (tol 1e-300) with 1 and 3 restart
    cycles (time = steps t + T); then GMRES with the seeds and the
    preconditioner gives each instance's steps and convergence.  An energy is
    routed to the direct path when the mean GMRES cost of its instances
    (steps t, plus T for those that did not converge within the cap of
    ceil(T / t) steps) is not below T.  Returns a dict with the table
    (int8 per energy index), the cycle cap, t, T and the per-energy means."""
    n = prob.n_inst
    work = torch.empty(lsms.gmres_workspace_size(h, prob, restart), dtype=torch.uint8, device="cuda")
    _, t1 = _timed(lambda: lsms.tau00_gmres(h, prob, work, seed=seeds, restart=restart, max_cycles=1, tol=1e-300))
    _, t3 = _timed(lambda: lsms.tau00_gmres(h, prob, work, seed=seeds, restart=restart, max_cycles=3, tol=1e-300))
    t_step = max((t3 - t1) / (2 * restart), 1e-9)
    t_lu = max(t1 - restart * t_step, t_step)
    cap_cycles = max(1, int(np.ceil(t_lu / t_step / restart)))
    _, info, steps = lsms.tau00_gmres(h, prob, work, seed=seeds, restart=restart, max_cycles=cap_cycles, tol=tol,
                                      precond=precond, precond_row=precond_row)
    torch.cuda.synchronize()
    steps = steps.cpu().numpy().astype(np.float64)
    fell = (info.cpu().numpy() & lsms.INFO_LU_FALLBACK) != 0
    e_idx = prob.e_idx.cpu().numpy()
    route = np.ones(n_energy, np.int8)
    mean_steps = np.full(n_energy, np.nan)
    frac_conv = np.full(n_energy, np.nan)
    for e in range(n_energy):
        sel = e_idx == e
        if not np.any(sel):
            continue
        cost = np.mean(steps[sel] * t_step + fell[sel] * t_lu)
        mean_steps[e] = float(np.mean(steps[sel]))
        frac_conv[e] = float(1.0 - np.mean(fell[sel]))
        route[e] = 0 if cost < t_lu else 1
    del work
    return {"route_by_energy": route, "max_cycles": cap_cycles, "t_step_s": t_step, "t_lu_s": t_lu,
            "mean_steps_by_energy": mean_steps, "converged_by_energy": frac_conv, "instances": n}
