"""GPU checks of the learned form through the C ABI: features, network
forward/backward, loss and AdamW against the CPU reference (oracle/mlp.py);
block GMRES against the oracle's tau00; and what the trained network gains
over GMRES without it.

Bars: features bit-exact; network outputs and gradients within relative
Frobenius 1e-4 of the FP64 reference with the same bf16 rounding points (FP32
accumulation of up to 256 bf16 products per output, plus rare one-ulp bf16
flips of an activation computed in FP32 rather than FP64); GMRES tau00
within 1e-10 of the oracle (the bar of the reduced forms), FP64-fallback
instances within 1e-12.
"""

import numpy as np
import pytest

import inputs
import oracle
from oracle import mlp as omlp
from parity import rel_f, t0_of, x_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def P():
    _torch()
    import paper_2308_16317_amd as P

    return P


@pytest.fixture(scope="module")
def h(P):
    return P.Handle()


def _err(tau, ref, w):
    """Per instance: the larger of rel_F and the elementwise [M^-1]_00 error."""
    return np.maximum(rel_f(tau, ref), x_err(tau, ref, t0_of(w)))


def _net(P, h, theta):
    torch = _torch()
    params = torch.as_tensor(theta.astype(np.float32)).cuda()
    wb = torch.empty(P.MLP_PARAMS, dtype=torch.int16, device="cuda")
    P.mlp_cast(h, params, wb)
    return params, wb


def test_features_bit_exact(P, h):
    for w in (inputs.subset(inputs.config2(), [0, 1, 2, 100, 8191]), inputs.subset(inputs.config4(), np.arange(0, 1024, 97))):
        prob = P.problem_for_workload(h, w)
        feat = P.mlp_features(h, prob, inputs.A_LAT).cpu().numpy()
        liz_off, pos, spec = oracle.liz_batch(w)
        ref = omlp.features(liz_off, pos, spec, w.energies, w.e_idx, inputs.A_LAT).astype(np.float32)
        assert np.array_equal(feat, ref), np.abs(feat - ref).max()


def test_forward_backward_match_reference(P, h):
    torch = _torch()
    theta = inputs.mlp_init(seed=5)
    rng = np.random.default_rng(2)
    n = 37  # ragged against the 64-row tiles
    X = rng.standard_normal((n, 18)).astype(np.float32)
    params, wb = _net(P, h, theta)
    feat = torch.as_tensor(X).cuda()
    out, act = P.mlp_forward(h, params, wb, feat)
    ref, cache = omlp.forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float64), round_bf16=True)
    err = np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref)
    print("forward rel_F", err)
    assert err <= 1e-4
    dY = rng.standard_normal((n, 1024)).astype(np.float32)
    grad = P.mlp_backward(h, wb, feat, act, torch.as_tensor(dY).cuda()).cpu().numpy()
    gref = omlp.backward(theta.astype(np.float32).astype(np.float64), cache, dY.astype(np.float64))
    off = 0
    for i, o in zip(omlp.LAYERS[:-1], omlp.LAYERS[1:]):
        for seg in (slice(off, off + o * i), slice(off + o * i, off + o * i + o)):
            e = np.linalg.norm(grad[seg] - gref[seg]) / np.linalg.norm(gref[seg])
            print("grad layer", i, o, e)
            assert e <= 1e-4
        off += o * i + o


def test_mse_and_adamw_match_reference(P, h):
    torch = _torch()
    rng = np.random.default_rng(4)
    out = rng.standard_normal((5, 1024)).astype(np.float32)
    tgt = rng.standard_normal((5, 1024)).astype(np.float32)
    dout, loss = P.mlp_mse(h, torch.as_tensor(out).cuda(), torch.as_tensor(tgt).cuda())
    d = out.astype(np.float64) - tgt
    assert abs(loss.item() - np.mean(d * d)) <= 1e-5 * np.mean(d * d)
    assert np.allclose(dout.cpu().numpy(), 2 * d / d.size, rtol=1e-5, atol=1e-12)
    theta = inputs.mlp_init(seed=9)
    params, wb = _net(P, h, theta)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    tref = theta.astype(np.float32).astype(np.float64)
    mref = np.zeros_like(tref)
    vref = np.zeros_like(tref)
    for step in (1, 2, 3):
        g = rng.standard_normal(P.MLP_PARAMS).astype(np.float32)
        P.mlp_adamw(h, params, wb, m, v, torch.as_tensor(g).cuda(), 1e-3, step, wd=1e-2)
        tref, mref, vref = omlp.adamw(tref, mref, vref, g.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, 1e-2, step)
    assert np.max(np.abs(params.cpu().numpy() - tref)) <= 1e-6
    # the bf16 copy is the rounded master copy
    wb_f = (wb.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(wb_f.astype(np.float64), omlp.bf16(params.cpu().numpy()))


def _gmres(P, h, w, seed=None, restart=8, max_cycles=20, tol=1e-12):
    torch = _torch()
    prob = P.problem_for_workload(h, w)
    work = torch.empty(P.gmres_workspace_size(h, prob, restart), dtype=torch.uint8, device="cuda")
    print(f"gmres: n_inst={prob.n_inst} max_liz={prob.max_liz} restart={restart} seed={seed is not None}",
          flush=True)
    tau, info, steps = P.tau00_gmres(h, prob, work, seed=seed, restart=restart, max_cycles=max_cycles, tol=tol)
    torch.cuda.synchronize()
    return tau.cpu().numpy(), info.cpu().numpy(), steps.cpu().numpy()


def test_gmres_matches_oracle_tiny(P, h):
    w = inputs.config1()
    ref, _ = oracle.tau00_workload(w)
    tau, info, steps = _gmres(P, h, w)
    assert np.all((info == 0) | (info == P.INFO_LU_FALLBACK)), np.unique(info)
    err = _err(tau, ref, w)
    print("tiny gmres: fallbacks", int((info != 0).sum()), "steps", steps.min(), np.median(steps), steps.max(),
          "max rel_F", err.max())
    assert err[info == 0].max(initial=0.0) <= 1e-10
    assert err[info != 0].max(initial=0.0) <= 1e-12
    assert (info == 0).mean() >= 0.5


def test_gmres_small_restart_and_fallback(P, h):
    # restart 2 with 1 cycle cannot converge: every instance takes the FP64 path
    w = inputs.subset(inputs.config1(), np.arange(0, 128, 13))
    ref, _ = oracle.tau00_workload(w)
    tau, info, steps = _gmres(P, h, w, restart=2, max_cycles=1, tol=1e-14)
    assert np.all(info == P.INFO_LU_FALLBACK)
    assert np.all(steps == 2)
    assert _err(tau, ref, w).max() <= 1e-12


def test_gmres_full_size_sample(P, h):
    w = inputs.subset(inputs.config2(), [0, 16, 31, 77 * 32 + 1, 200 * 32 + 30])
    ref, _ = oracle.tau00_workload(w)
    tau, info, steps = _gmres(P, h, w)
    err = _err(tau, ref, w)
    print("N=2160 gmres: info", info, "steps", steps, "rel_F", err)
    assert np.all((info == 0) | (info == P.INFO_LU_FALLBACK))
    assert err[info == 0].max(initial=0.0) <= 1e-10
    assert err[info != 0].max(initial=0.0) <= 1e-12


def _all_centre_batch(w, energies):
    """Every atom of the supercell as a centre at each of `energies`: the
    batch holds a block for every LIZ site of every instance."""
    import dataclasses

    n_at = w.atom_pos.shape[0]
    centre = np.repeat(np.arange(n_at), len(energies)).astype(np.int32)
    e_idx = np.tile(np.asarray(energies), n_at).astype(np.int32)
    return dataclasses.replace(w, centre=centre, rc=np.full(centre.size, float(w.rc[0])), e_idx=e_idx)


def test_gmres_preconditioner_and_routing(P, h):
    # blocks from the direct solution of the batch itself ([M^-1]_00 of the
    # instance centred on each site): GMRES with them converges to the oracle
    # (on these 13-site LIZs the centred block is a poor stand-in for an edge
    # site's own diagonal block, and the steps are printed, not compared);
    # routed instances take the FP64 path
    torch = _torch()
    from paper_2308_16317_amd import learned

    w = _all_centre_batch(inputs.config1(), [0, 5, 10, 15])  # 32 atoms x 4 energies
    ref, rinfo = oracle.tau00_workload(w)
    prob = P.problem_for_workload(h, w)
    tau_d = learned.solve_direct(h, prob).cpu().numpy().reshape(-1, 16, 16).transpose(0, 2, 1)
    lv = np.floor(np.sqrt(np.arange(16)) + 1e-9).astype(int)
    t0 = np.stack([oracle.tmat(3, w.energies[w.e_idx[i]], w.delta[w.atom_species[w.centre[i]], w.e_idx[i]])[lv]
                   for i in range(w.n_inst)])
    D = tau_d / t0[:, None, :]  # [M^-1]_00, natural indexing
    blocks = torch.as_tensor(np.ascontiguousarray(D.transpose(0, 2, 1)).reshape(-1)).to("cuda")
    liz = P.build_liz(h, w.atom_pos, w.atom_species, w.box, w.centre, w.rc, 1024, with_atoms=True)
    rows = int(prob.liz_off[-1].item())
    prow = P.site_blocks(h, prob, liz["atom"][:rows], w.centre, w.atom_pos.shape[0])
    assert int((prow < 0).sum().item()) == 0
    work = torch.empty(P.gmres_workspace_size(h, prob, 8), dtype=torch.uint8, device="cuda")
    out = {}
    for name, kw in (("none", {}), ("blocks", dict(precond=blocks, precond_row=prow))):
        tau, info, steps = P.tau00_gmres(h, prob, work, restart=8, max_cycles=20, tol=1e-12, **kw)
        torch.cuda.synchronize()
        tau, info, steps = tau.cpu().numpy(), info.cpu().numpy(), steps.cpu().numpy()
        err = _err(tau, ref, w)
        print(f"preconditioner {name}: mean steps {steps.mean():.2f}, converged {(info == 0).mean():.2f}, "
              f"max rel_F {err.max():.2e}")
        assert np.all((info == 0) | (info == P.INFO_LU_FALLBACK))
        assert err[info == 0].max(initial=0.0) <= 1e-10 and err[info != 0].max(initial=0.0) <= 1e-12
        out[name] = steps
    # routing: every other instance straight to the FP64 path
    route = torch.as_tensor((np.arange(w.n_inst) % 2).astype(np.int8)).to("cuda")
    tau, info, steps = P.tau00_gmres(h, prob, work, restart=8, max_cycles=20, tol=1e-12, route=route)
    torch.cuda.synchronize()
    tau, info, steps = tau.cpu().numpy(), info.cpu().numpy(), steps.cpu().numpy()
    r = np.arange(w.n_inst) % 2 == 1
    assert np.all(info[r] == P.INFO_ROUTED) and np.all(steps[r] == 0)
    assert np.all(info[~r] != P.INFO_ROUTED)
    err = _err(tau, ref, w)
    assert err[r].max() <= 1e-12 and err[~r][info[~r] == 0].max(initial=0.0) <= 1e-10


def test_trained_seed_reduces_gmres_steps(P, h):
    """Train the network on tau00 the direct solver produced for a different
    random alloy (seed 1), then solve the evaluation alloy (seed 0, every site
    at five energies across the contour, so that every LIZ site has its own
    block) by GMRES: no seed, the untrained network (its output is the
    training-set mean after the normalisation), the trained network, each
    with and without the block-diagonal preconditioner built from the same
    network's outputs.  The direct FP64 path is the reference."""
    torch = _torch()
    from paper_2308_16317_amd import learned

    net, losses = learned.train_on(h, inputs.config2(seed=1), inputs.A_LAT, inputs.mlp_init(seed=0), steps=3000)
    print("training loss: first", losses[0], "last 50 mean", np.mean(losses[-50:]))
    assert np.mean(losses[-50:]) < 0.6 * losses[0]
    w = _all_centre_batch(inputs.config2(seed=0), [4, 8, 12, 16, 20])
    prob = P.problem_for_workload(h, w)
    ref = learned.solve_direct(h, prob).cpu().numpy().reshape(-1, 16, 16).transpose(0, 2, 1)
    feat = P.mlp_features(h, prob, inputs.A_LAT)
    net0 = learned.SeedNet(h, inputs.mlp_init(seed=0))
    net0.scale, net0.shift = net.scale, net.shift
    sd = {"trained": net.seeds(feat), "mean": net0.seeds(feat)}
    liz = P.build_liz(h, w.atom_pos, w.atom_species, w.box, w.centre, w.rc, 1024, with_atoms=True)
    prow = P.site_blocks(h, prob, liz["atom"][:int(prob.liz_off[-1].item())], w.centre, w.atom_pos.shape[0])
    work = torch.empty(P.gmres_workspace_size(h, prob, 8), dtype=torch.uint8, device="cuda")
    variants = {"none": {}, "mean": dict(seed=sd["mean"]), "trained": dict(seed=sd["trained"]),
                "mean+pc": dict(seed=sd["mean"], precond=sd["mean"], precond_row=prow),
                "trained+pc": dict(seed=sd["trained"], precond=sd["trained"], precond_row=prow)}
    res = {}
    for k, kw in variants.items():
        tau, info, steps = P.tau00_gmres(h, prob, work, restart=8, max_cycles=20, tol=1e-12, **kw)
        torch.cuda.synchronize()
        tau, info, steps = tau.cpu().numpy(), info.cpu().numpy(), steps.cpu().numpy()
        err = _err(tau, ref, w)
        res[k] = (steps, info)
        print(f"{k}: mean steps {steps.mean():.2f}, fallbacks {int((info != 0).sum())}, max rel_F {err.max():.2e}")
        assert np.all((info == 0) | (info == P.INFO_LU_FALLBACK))
        assert err[info == 0].max(initial=0.0) <= 1e-10
    conv = np.logical_and.reduce([v[1] == 0 for v in res.values()])
    means = {k: float(v[0][conv].mean()) for k, v in res.items()}
    print("jointly converged", int(conv.sum()), "mean steps:", means)
    assert conv.sum() >= 0.5 * w.n_inst
    # what the network gains: its seed and its per-site preconditioner cut
    # the block steps below the unseeded, unpreconditioned solve, and the
    # trained network's per-site blocks beat the untrained network's (the
    # training-set mean) by at least one block step on average (measured:
    # 38.8 against 42.3)
    assert means["trained"] < means["none"]
    assert means["trained+pc"] < means["trained"]
    assert means["trained+pc"] <= means["mean+pc"] - 1.0


@pytest.mark.xfail(strict=False, reason="negative result: as a seed alone the trained network is no better than "
                                        "the training-set mean (31.4 against 31.2 block steps measured); its gain "
                                        "shows through the preconditioner (test above)")
def test_training_beats_mean_seed(P, h):
    """Training against the untrained network (the training-set mean), seed
    only: the trained seed would save at least one block step on average."""
    torch = _torch()
    from paper_2308_16317_amd import learned

    net, _ = learned.train_on(h, inputs.config2(seed=1), inputs.A_LAT, inputs.mlp_init(seed=0), steps=3000)
    w = _all_centre_batch(inputs.config2(seed=0), [8, 16])
    prob = P.problem_for_workload(h, w)
    feat = P.mlp_features(h, prob, inputs.A_LAT)
    net0 = learned.SeedNet(h, inputs.mlp_init(seed=0))
    net0.scale, net0.shift = net.scale, net.shift
    work = torch.empty(P.gmres_workspace_size(h, prob, 8), dtype=torch.uint8, device="cuda")
    st = {}
    for k, n_ in (("trained", net), ("mean", net0)):
        _, info, steps = P.tau00_gmres(h, prob, work, seed=n_.seeds(feat), restart=8, max_cycles=20, tol=1e-12)
        torch.cuda.synchronize()
        st[k] = steps.cpu().numpy().astype(float)
    print("mean block steps: trained", st["trained"].mean(), "mean seed", st["mean"].mean())
    assert st["trained"].mean() <= st["mean"].mean() - 1.0
