"""GPU parity of tau00_large: one instance's elimination spread over the whole
GPU (panel kernel, strip U12 kernel, row-block MFMA update, one panel of
look-ahead on a second stream), against the CPU oracle.

Bar: tau00 rel_F <= 1e-12 and the scale-free [M^{-1}]_00 elementwise within
1e-12 of its largest entry (the plain FP64 bar).  The paper's non-canted NiAu
rank N = 6225 (lmax = 4, 249-atom LIZ) is checked against
tests/golden/large_tau00.npz, written by make_large_golden.py beside it with
the oracle alone; the spin-canted ranks 4320 and 6750 against
canted_tau00.npz, and
the paper's spin-canted NiAu rank 12450 (2 kk 249, lmax = 4) against
large_canted_tau00.npz (same script, argument `canted`).
"""

import dataclasses
import os

import numpy as np
import pytest

import inputs
import oracle
from parity import check_tau, oracle_cached

pytestmark = pytest.mark.gpu

TOL = 1e-12
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _large(P, h, w, i, nb=0):
    """tau00_large of instance i of workload w (its own single-instance problem)."""
    torch = _torch()
    wi = inputs.subset(w, [i])
    prob = P.problem_for_workload(h, wi)
    N = prob.kc * prob.max_liz
    M = torch.zeros(N * N, dtype=torch.complex128, device="cuda")
    moff = torch.zeros(1, dtype=torch.int64, device="cuda")
    binfo = (P.build_kkr_spin if prob.spin is not None else P.build_kkr)(h, prob, M, moff)
    tau, info = P.tau00_large(h, prob, M, P.Opts(0, nb, 0, 0))
    torch.cuda.synchronize()
    assert int(binfo.cpu().numpy()[0]) == 0
    return tau.cpu().numpy()[0], int(info.cpu().numpy()[0]), N


def _run(P, h, w, idx):
    out, Ns = [], []
    for i in idx:
        t, inf, N = _large(P, h, w, i)
        assert inf == 0, (i, inf)
        out.append(t)
        Ns.append(N)
    print(f"tau00_large on N = {sorted(set(Ns))}", flush=True)
    return np.stack(out)


def test_large_config1_against_oracle_and_batched(P, h):
    # N = 208 (Nd = 192: three full panels)
    torch = _torch()
    w = inputs.config1()
    ref, _ = oracle_cached("cfg1", w)
    idx = [0, 15, 37, 64, 127]
    got = _run(P, h, w, idx)
    check_tau(got, ref[idx], inputs.subset(w, idx), TOL, "tau00_large config1")
    # the batched path with 64-column panels (same pivot rule, its own panel
    # arithmetic)
    ws = inputs.subset(w, idx)
    prob = P.problem_for_workload(h, ws)
    N = prob.kk * np.diff(prob.liz_off.cpu().numpy())
    m_off = torch.as_tensor(np.concatenate([[0], np.cumsum(N * N)[:-1]]).astype(np.int64), device="cuda")
    M = torch.zeros(int((N * N).sum()), dtype=torch.complex128, device="cuda")
    P.build_kkr(h, prob, M, m_off)
    tb, ib = P.tau00_batched(h, prob, M, m_off, P.Opts(0, 64, 0, 0))
    torch.cuda.synchronize()
    tb = tb.cpu().numpy()
    d = np.abs(got - tb).max() / np.abs(tb).max()
    print(f"tau00_large vs tau00_batched (64-wide panels): max rel diff {d:.2e}")
    assert d <= 1e-12


@pytest.mark.parametrize("lmax", [0, 1, 2, 4])
def test_large_other_lmax(P, h, lmax):
    # N = 13 (one 12-column panel: the narrow-panel update), 52, 117, 325
    w = inputs.config1().with_lmax(lmax)
    idx = [3, 50, 126]
    ref, rinfo = oracle.tau00_workload(inputs.subset(w, idx))
    got = _run(P, h, w, idx)
    check_tau(got, ref, inputs.subset(w, idx), TOL, f"tau00_large lmax={lmax}")


def test_large_ragged_and_full_size(P, h):
    # a ragged-workload instance (N 1184..2400) and the benchmark's N = 2160
    # at the left contour end
    w4 = inputs.config4(n_inst=1024)
    i4 = [0, 511]
    ref4, _ = oracle.tau00_workload(inputs.subset(w4, i4))
    check_tau(_run(P, h, w4, i4), ref4, inputs.subset(w4, i4), TOL, "tau00_large ragged")
    w2 = inputs.config2()
    ref2, _ = oracle.tau00_workload(inputs.subset(w2, [0]))
    check_tau(_run(P, h, w2, [0]), ref2, inputs.subset(w2, [0]), TOL, "tau00_large N=2160")


def test_large_n6225(P, h):
    # the paper's non-canted NiAu rank: lmax = 4 over a 249-atom LIZ
    path = os.path.join(GOLD, "large_tau00.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/large_tau00.npz not written")
    g = np.load(path, allow_pickle=False)
    w = inputs.config_large()
    got = _run(P, h, w, list(g["idx"]))
    check_tau(got, g["tau"], inputs.subset(w, g["idx"]), TOL, "tau00_large N=6225")


def test_large_spin(P, h):
    # spin-canted: a tiny instance against the oracle, rank 4320 against the
    # golden oracle values
    w1 = inputs.config1()
    up, dn = inputs.spin_phase_shift_tables(w1.energies, 3)
    wc = dataclasses.replace(w1, delta=up, delta_dn=dn, atom_moment=inputs.canted_moments(32, 0))
    idx = [5, 77]
    ref, _ = oracle.tau00_spin_workload(inputs.subset(wc, idx))
    got = _run(P, h, wc, idx)
    d = np.linalg.norm((got - ref).reshape(2, -1), axis=1) / np.linalg.norm(ref.reshape(2, -1), axis=1)
    print(f"tau00_large canted tiny: rel_F max {d.max():.2e}")
    assert d.max() <= TOL
    path = os.path.join(GOLD, "canted_tau00.npz")
    if os.path.exists(path):
        g = np.load(path, allow_pickle=False)
        w = inputs.config_canted(lmax=3)
        i0 = int(g["idx_l3"][0])
        got = _run(P, h, w, [i0])
        ref = g["tau_l3"][:1]
        d = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"tau00_large canted rank 4320: rel_F {d:.2e}")
        assert d <= TOL
        # rank 6750 (lmax = 4: a 50 x 50 central block), both contour ends
        w4 = inputs.config_canted(lmax=4)
        i4 = [int(i) for i in g["idx_l4"]]
        got = _run(P, h, w4, i4)
        ref = g["tau_l4"]
        d = np.linalg.norm((got - ref).reshape(len(i4), -1), axis=1) / np.linalg.norm(ref.reshape(len(i4), -1), axis=1)
        print(f"tau00_large canted rank 6750: rel_F max {d.max():.2e}")
        assert d.max() <= TOL


def test_large_spin_n12450(P, h):
    # the paper's spin-canted NiAu rank: 2 kk 249 = 12450 (98 panel
    # workgroups in the first panels, 195 panels)
    path = os.path.join(GOLD, "large_canted_tau00.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/large_canted_tau00.npz not written")
    g = np.load(path, allow_pickle=False)
    w = inputs.config_large_canted()
    got = _run(P, h, w, list(g["idx"]))
    ref = g["tau"]
    d = np.linalg.norm((got - ref).reshape(len(ref), -1), axis=1) / np.linalg.norm(ref.reshape(len(ref), -1), axis=1)
    print(f"tau00_large canted rank 12450: rel_F {d.max():.2e}")
    assert d.max() <= TOL


def test_large_errors(P, h):
    torch = _torch()
    w = inputs.subset(inputs.config1(), [0, 1])
    prob = P.problem_for_workload(h, w)
    M = torch.zeros(208 * 208, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError):  # two instances
        P.tau00_large(h, prob, M)
    w1 = inputs.subset(inputs.config1(), [0])
    p1 = P.problem_for_workload(h, w1)
    with pytest.raises(RuntimeError):  # panel width other than 64
        P.tau00_large(h, p1, M, P.Opts(0, 32, 0, 0))
    # rank limit: 16384 rows (max_liz 656 at lmax = 4 is 16400)
    w4 = inputs.subset(inputs.config1().with_lmax(4), [0])
    p4 = P.problem_for_workload(h, w4)
    big = P.Problem(4, p4.liz_off, p4.pos, p4.species, w4.energies, w4.e_idx, w4.delta, max_liz=656)
    with pytest.raises(RuntimeError):
        P.tau00_large(h, big, M)
    # a LIZ smaller than max_liz: info -3, tau00 NaN
    p2 = P.Problem(3, p1.liz_off, p1.pos, p1.species, w1.energies, w1.e_idx, w1.delta, max_liz=14)
    M2 = torch.zeros((16 * 14) ** 2, dtype=torch.complex128, device="cuda")
    tau, info = P.tau00_large(h, p2, M2)
    torch.cuda.synchronize()
    assert int(info.cpu().numpy()[0]) == -3 and np.all(np.isnan(tau.cpu().numpy()))
    # an exactly zero pivot (M = I with one zero row of M) at steps 1, 70, 193
    for step in (1, 70, 193):
        N, Nd, kk = 208, 192, 16
        v = step - 1
        phys = v + kk if v < Nd else v - Nd
        Mz = np.eye(N, dtype=np.complex128)
        Mz[phys, :] = 0.0
        Md = torch.as_tensor(Mz.ravel(order="F")).to("cuda")
        tau, info = P.tau00_large(h, p1, Md)
        torch.cuda.synchronize()
        assert int(info.cpu().numpy()[0]) == step, (step, int(info.cpu().numpy()[0]))
        assert np.all(np.isnan(tau.cpu().numpy()))


def test_large_spin_limit_gives_up(P, h):
    # a barrier wait allowed a single poll gives up (the first workgroup to
    # arrive never finds the others there): every kernel still ends, the
    # instance reports info -4 with tau00 NaN; with the default limit the next
    # call on the same handle and workspace is exact again
    torch = _torch()
    w = inputs.subset(inputs.config2(), [0])
    prob = P.problem_for_workload(h, w)
    N = prob.kk * prob.max_liz
    M = torch.zeros(N * N, dtype=torch.complex128, device="cuda")
    moff = torch.zeros(1, dtype=torch.int64, device="cuda")
    P.build_kkr(h, prob, M, moff)
    P.large_set_spin_limit(h, 1)
    try:
        tau, info = P.tau00_large(h, prob, M)
        torch.cuda.synchronize()
        print("spin limit 1: info", int(info.cpu().numpy()[0]), flush=True)
        assert int(info.cpu().numpy()[0]) == -4
        assert np.all(np.isnan(tau.cpu().numpy()))
    finally:
        P.large_set_spin_limit(h, 0)
    P.build_kkr(h, prob, M, moff)
    tau, info = P.tau00_large(h, prob, M)
    torch.cuda.synchronize()
    assert int(info.cpu().numpy()[0]) == 0
    ref, _ = oracle.tau00_workload(w)
    check_tau(tau.cpu().numpy(), ref, w, TOL, "tau00_large after a give-up")
