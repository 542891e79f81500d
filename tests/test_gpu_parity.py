"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Bars: bit-exact for the LIZ (indices, order, relative vectors); M elementwise
within 1e-13 of max|M|; tau00 within rel_F = ||tau - tau_ref||_F / ||tau_ref||_F
<= 1e-12 per instance (the plain FP64 target).  The oracle's tau00 is refined
with 80-bit residuals, so its own error is far below that bar.
"""

import os

import numpy as np
import pytest

import inputs
import oracle
from parity import check_tau, config2_two_sites, config4_sample, oracle_cached, rel_f

pytestmark = pytest.mark.gpu

TOL_TAU = 1e-12
TOL_M = 1e-13


def _bits(x):
    # the raw 64-bit words of a complex array (any strides)
    return np.ascontiguousarray(x).view(np.uint64)


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


def _oracle_tau(w):
    return oracle.tau00_workload(w)


_CACHE = {}


def oracle_tau_cached(key, w):
    if key not in _CACHE:
        _CACHE[key] = _oracle_tau(w)
    return _CACHE[key]


def _solve(P, h, w, nb=0, chunk=0, work_gb=None):
    torch = _torch()
    prob = P.problem_for_workload(h, w)
    opts = P.Opts(0, nb, chunk, 0)
    one = P.workspace_size(h, prob, 1, opts)
    n_slots = prob.n_inst if chunk == 0 else min(chunk, prob.n_inst)
    if work_gb is not None:
        n_slots = max(1, min(prob.n_inst, int(work_gb * 2 ** 30 // one)))
    work = torch.empty(one * max(1, n_slots), dtype=torch.uint8, device="cuda")
    tau, info = P.tau00_solve(h, prob, work, opts)
    torch.cuda.synchronize()
    return tau.cpu().numpy(), info.cpu().numpy()


# ---------------------------------------------------------------- a1 LIZ
@pytest.mark.parametrize("which", ["config1", "config4"])
def test_liz_bit_exact(P, h, which):
    w = inputs.config1() if which == "config1" else inputs.config4(n_inst=96)
    liz = P.build_liz(h, w.atom_pos, w.atom_species, w.box, w.centre, w.rc, 256, with_atoms=True)
    off = liz["liz_off"].cpu().numpy()
    n = liz["liz_n"].cpu().numpy()
    pos = liz["pos"].cpu().numpy()
    atom = liz["atom"].cpu().numpy()
    spec = liz["species"].cpu().numpy()
    for i, (c, rc) in enumerate(zip(w.centre, w.rc)):
        rel, idx = oracle.liz(w.atom_pos, w.box, int(c), float(rc))
        assert n[i] == rel.shape[0]
        a, b = off[i], off[i + 1]
        assert b - a == rel.shape[0]
        np.testing.assert_array_equal(atom[a:b], idx)
        np.testing.assert_array_equal(pos[a:b], rel)
        np.testing.assert_array_equal(spec[a:b], w.atom_species[idx])


# ---------------------------------------------------------- a2 + a3 build
@pytest.mark.parametrize("lmax", [0, 1, 3, 4])
def test_build_kkr_matches_oracle(P, h, lmax):
    torch = _torch()
    w = inputs.config1()
    if lmax != 3:
        w = w.with_lmax(lmax)
    w = inputs.subset(w, np.arange(0, 128, 9))
    prob = P.problem_for_workload(h, w)
    liz_off = prob.liz_off.cpu().numpy()
    N = prob.kk * np.diff(liz_off)
    m_off = np.concatenate([[0], np.cumsum(N * N)[:-1]]).astype(np.int64)
    M = torch.zeros(int((N * N).sum()), dtype=torch.complex128, device="cuda")
    info = P.build_kkr(h, prob, M, torch.as_tensor(m_off, device="cuda"))
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    Mh = M.cpu().numpy()
    pos = prob.pos.cpu().numpy()
    spec = prob.species.cpu().numpy()
    C, _ = oracle.gaunt(lmax)
    for i in range(prob.n_inst):
        a, b = liz_off[i], liz_off[i + 1]
        e = w.e_idx[i]
        ref, st = oracle.build_m(lmax, pos[a:b], spec[a:b], w.energies[e], w.delta[:, e, :], C)
        got = Mh[m_off[i]:m_off[i] + N[i] * N[i]].reshape(N[i], N[i]).T  # column-major
        assert st == 0
        assert np.abs(got - ref).max() <= TOL_M * np.abs(ref).max()


# ---------------------------------------------------------- a4 + a5 tau00
def test_tau00_batched_config1_all(P, h):
    torch = _torch()
    w = inputs.config1()
    ref, rinfo = oracle_tau_cached("cfg1", w)
    assert np.all(rinfo == 0)
    prob = P.problem_for_workload(h, w)
    N = prob.kk * np.diff(prob.liz_off.cpu().numpy())
    m_off = np.concatenate([[0], np.cumsum(N * N)[:-1]]).astype(np.int64)
    M = torch.zeros(int((N * N).sum()), dtype=torch.complex128, device="cuda")
    moff = torch.as_tensor(m_off, device="cuda")
    info_b = P.build_kkr(h, prob, M, moff)
    tau, info = P.tau00_batched(h, prob, M, moff)
    torch.cuda.synchronize()
    assert np.all(info_b.cpu().numpy() == 0) and np.all(info.cpu().numpy() == 0)
    check_tau(tau.cpu().numpy(), ref, w, TOL_TAU, "config1 batched")


@pytest.mark.parametrize("nb,chunk", [(0, 0), (16, 7), (32, 50), (48, 1), (96, 5), (128, 0)])
def test_tau00_solve_config1_nb_chunk(P, h, nb, chunk):
    w = inputs.config1()
    ref, _ = oracle_tau_cached("cfg1", w)
    tau, info = _solve(P, h, w, nb=nb, chunk=chunk)
    assert np.all(info == 0)
    check_tau(tau, ref, w, TOL_TAU, f"config1 nb={nb} chunk={chunk}")


@pytest.mark.parametrize("lmax", [0, 1, 2, 4])
def test_tau00_other_lmax(P, h, lmax):
    # N = 13, 52, 117, 325: ragged tails smaller than one 16-row tile, and kk = 25
    w = inputs.subset(inputs.config1().with_lmax(lmax), np.arange(0, 128, 5))
    ref, rinfo = _oracle_tau(w)
    tau, info = _solve(P, h, w)
    assert np.all(info == 0) and np.all(rinfo == 0)
    check_tau(tau, ref, w, TOL_TAU, f"lmax={lmax}")


def test_tau00_ragged_config4(P, h):
    # 32 instances of the ragged workload spread over the batch, N 1184..2400
    w = config4_sample(32)
    ref, rinfo = oracle_cached("cfg4-32", w)
    tau, info = _solve(P, h, w)
    assert np.all(info == 0) and np.all(rinfo == 0)
    check_tau(tau, ref, w, TOL_TAU, "config4 32-instance sample")


def test_tau00_config2_full_size_sample(P, h):
    # the benchmarked workload (N = 2160): all 32 energies of two sites,
    # through tau00_solve with the default panel width and with 128
    w = config2_two_sites()
    ref, rinfo = oracle_cached("cfg2-2sites", w)
    for nb in (0, 128):
        tau, info = _solve(P, h, w, nb=nb)
        assert np.all(info == 0) and np.all(rinfo == 0)
        rf, xe = check_tau(tau, ref, w, TOL_TAU, f"config2 two sites nb={nb}")
        e = w.energies[w.e_idx]
        for k in np.argsort(-xe)[:4]:
            print(f"  worst: E={e[k]:.4f} rel_F {rf[k]:.2e} [M^-1]00 {xe[k]:.2e}")
    # tau00 is complex symmetric
    sym = np.abs(tau - tau.transpose(0, 2, 1)).max(axis=(1, 2)) / np.abs(tau).max(axis=(1, 2))
    assert sym.max() <= TOL_TAU


def _pivot_sensitive_matrix(rng, N, kk, eps=1e-8):
    """M whose elimination (Sec. 3.2: partial pivoting, the central block
    last) has a known and unambiguous pivot sequence.  In elimination order
    (non-central rows and columns first, the central block last) the matrix
    read as A = M^T is P L U: P a random permutation inside each of the two
    row groups, L unit lower triangular with |L_ij| ~ eps, U upper triangular
    and well conditioned.  Partial pivoting recovers P; any other pivot gives
    multipliers of order 1/eps and errors far above the FP64 bar."""
    Nd = N - kk
    cn = lambda *s: (rng.standard_normal(s) + 1j * rng.standard_normal(s)) / np.sqrt(2)
    L = np.eye(N, dtype=np.complex128) + np.tril(eps * cn(N, N), -1)
    U = np.triu(0.3 / np.sqrt(N) * cn(N, N), 1)
    U += np.diag((1.0 + 0.5 * rng.random(N)) * np.exp(2j * np.pi * rng.random(N)))
    perm = np.concatenate([rng.permutation(Nd), Nd + rng.permutation(kk)])
    A = (L @ U)[np.argsort(perm)]  # row perm[i] of A is row i of L U
    ph = np.where(np.arange(N) < Nd, np.arange(N) + kk, np.arange(N) - Nd)  # elimination -> storage index
    M = np.empty((N, N), np.complex128)
    M[np.ix_(ph, ph)] = A.T
    return M


@pytest.mark.parametrize("which", ["config1", "config2"])
def test_pivot_choice_caller_matrix(P, h, which):
    # the largest candidate sits at random rows, so every lane, wave and
    # reduction stage of the pivot search is the winner somewhere
    torch = _torch()
    w = inputs.config1() if which == "config1" else inputs.config2()
    w = inputs.subset(w, [0, 37])
    prob = P.problem_for_workload(h, w)
    kk = prob.kk
    liz_off = prob.liz_off.cpu().numpy()
    N = kk * np.diff(liz_off)
    rng = np.random.default_rng(2024)
    mats = [_pivot_sensitive_matrix(rng, int(n), kk) for n in N]
    m_off = np.concatenate([[0], np.cumsum(N * N)[:-1]]).astype(np.int64)
    M = torch.as_tensor(np.concatenate([m.ravel(order="F") for m in mats])).to("cuda")
    tau, info = P.tau00_batched(h, prob, M, torch.as_tensor(m_off, device="cuda"))
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    liz_off_o, pos, spec = oracle.liz_batch(w)
    l_of = np.floor(np.sqrt(np.arange(kk))).astype(int)
    ref = []
    for i, m in enumerate(mats):
        E = w.energies[w.e_idx[i]]
        t = oracle.tmat(w.lmax, E, w.delta[spec[liz_off_o[i]], w.e_idx[i]])[l_of]
        X = np.linalg.solve(m, np.eye(m.shape[0], kk))  # first block column of M^-1
        ref.append(X[:kk] * t[None, :])
    check_tau(tau.cpu().numpy(), np.stack(ref), w, TOL_TAU, f"{which} pivot-sensitive")


# --------------------------------------------------------- edge cases
def test_one_atom_and_zero_t(P, h):
    torch = _torch()
    w = inputs.config1()
    e = np.array([0, 5, 15], np.int32)
    prob = P.Problem(3, [0, 1, 2, 3], np.zeros((3, 3)), [0, 1, 0], w.energies, e, w.delta)
    work = torch.empty(P.workspace_size(h, prob, 3), dtype=torch.uint8, device="cuda")
    tau, info = P.tau00_solve(h, prob, work)
    torch.cuda.synchronize()
    tau = tau.cpu().numpy()
    lv = np.array([int(np.floor(np.sqrt(L) + 1e-9)) for L in range(16)])
    for q, s in enumerate([0, 1, 0]):
        t = oracle.tmat(3, w.energies[e[q]], w.delta[s, e[q]])
        np.testing.assert_allclose(tau[q], np.diag(t[lv]), rtol=0, atol=1e-15 * np.abs(t).max())
    assert np.all(info.cpu().numpy() == 0)
    # t = 0 everywhere: tau00 = 0
    w0 = inputs.subset(inputs.config1(), [0, 1])
    w0.delta = np.zeros_like(w0.delta)
    tau0, info0 = _solve(P, h, w0)
    assert np.all(info0 == 0) and np.all(tau0 == 0)


def test_dimer_closed_form(P, h):
    torch = _torch()
    E = 0.25 + 0.1j
    delta = np.array([[[0.3 + 0.02j]], [[-0.7 + 0.05j]]])
    R = np.array([[0, 0, 0], [2.0, -3.0, 1.5]])
    prob = P.Problem(0, [0, 2], R, [0, 1], [E], [0], delta)
    work = torch.empty(P.workspace_size(h, prob, 1), dtype=torch.uint8, device="cuda")
    tau, info = P.tau00_solve(h, prob, work)
    torch.cuda.synchronize()
    tA = oracle.tmat(0, E, delta[0, 0])[0]
    tB = oracle.tmat(0, E, delta[1, 0])[0]
    r = np.linalg.norm(R[1])
    g = -np.exp(1j * np.sqrt(E) * r) / r
    ref = tA / (1 - tA * tB * g * g)
    assert info.cpu().numpy()[0] == 0
    assert abs(tau.cpu().numpy()[0, 0, 0] - ref) <= 1e-14 * abs(ref)


def test_error_codes(P, h):
    torch = _torch()
    w = inputs.subset(inputs.config1(), [0, 1, 2])
    prob = P.problem_for_workload(h, w)
    # coincident sites in instance 1, NaN phase shift for instance 2's energy
    pos = prob.pos.clone()
    off = prob.liz_off.cpu().numpy()
    pos[off[1] + 4] = pos[off[1] + 3]
    delta = torch.as_tensor(w.delta.copy())
    delta[1, w.e_idx[2], 2] = float("nan")
    bad = P.Problem(3, prob.liz_off, pos, prob.species, w.energies, w.e_idx, delta, max_liz=prob.max_liz)
    work = torch.empty(P.workspace_size(h, bad, 3), dtype=torch.uint8, device="cuda")
    tau, info = P.tau00_solve(h, bad, work)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    tau = tau.cpu().numpy()
    assert info[0] == 0 and info[1] == -2 and info[2] == -1
    assert np.all(np.isnan(tau[1]))
    # empty batch is a no-op; an undersized workspace is rejected
    empty = P.Problem(3, [0], np.zeros((0, 3)), np.zeros(0), w.energies, np.zeros(0), w.delta, max_liz=13)
    t0, i0 = P.tau00_solve(h, empty, work)
    assert t0.shape[0] == 0
    with pytest.raises(RuntimeError):
        P.tau00_solve(h, prob, work[:16])


@pytest.mark.parametrize("step", [1, 256, 257, 300, 512, 2144, 2145, 2160])
def test_zero_pivot_info_beyond_flag_bits(P, h, step):
    # M = I with one row of zeros: reading M as A = M^T, the column of A at
    # internal index step - 1 is zero, so elimination step `step` meets an
    # exactly zero pivot (steps 1..2144 are non-central columns of a
    # 135-site LIZ, 2145..2160 the central block).  info must report the
    # step itself, never a value that reads as a fallback flag.
    torch = _torch()
    w = inputs.subset(inputs.config2(), [3])
    prob = P.problem_for_workload(h, w)
    kk = prob.kk
    N = kk * 135
    Nd = N - kk
    v = step - 1
    phys = v + kk if v < Nd else v - Nd
    M = np.eye(N, dtype=np.complex128)
    M[phys, :] = 0.0
    Md = torch.as_tensor(M.ravel(order="F")).to("cuda")
    tau, info = P.tau00_batched(h, prob, Md, torch.zeros(1, dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    got = int(info.cpu().numpy()[0])
    print("zero pivot at step", step, "info", got)
    assert got == step
    assert got & ~P.INFO_PIVOT_MASK == 0
    assert np.all(np.isnan(tau.cpu().numpy()))


def test_deterministic(P, h):
    w = inputs.subset(inputs.config1(), np.arange(0, 128, 3))
    t1, _ = _solve(P, h, w)
    t2, _ = _solve(P, h, w, chunk=5)
    assert np.array_equal(np.ascontiguousarray(t1).view(np.uint64), np.ascontiguousarray(t2).view(np.uint64))


# ------------------------------------------- persistent ragged batch (a7)
def _solve_flags(P, h, w, flags, nb=0, stream=None):
    torch = _torch()
    prob = P.problem_for_workload(h, w)
    opts = P.Opts(0, nb, 0, flags)
    work = torch.empty(P.workspace_size(h, prob, prob.n_inst, opts), dtype=torch.uint8, device="cuda")
    tau, info = P.tau00_solve(h, prob, work, opts)
    torch.cuda.synchronize()
    return tau.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("which", ["config1", "config1-lmax4", "config4"])
def test_persistent_matches_oracle(P, h, which):
    if which == "config1":
        w = inputs.config1()
        ref, rinfo = oracle_tau_cached("cfg1", w)
    elif which == "config1-lmax4":
        w = inputs.subset(inputs.config1().with_lmax(4), np.arange(0, 128, 7))
        ref, rinfo = _oracle_tau(w)
    else:
        w = inputs.subset(inputs.config4(n_inst=1024), [5, 6, 7, 8, 700])
        ref, rinfo = _oracle_tau(w)
    for nb in (0, 128):
        tau, info = _solve_flags(P, h, w, P.PERSISTENT, nb=nb)
        assert np.all(info == 0) and np.all(rinfo == 0)
        check_tau(tau, ref, w, TOL_TAU, f"persistent {which} nb={nb}")


def test_persistent_error_codes(P, h):
    # An instance that fails its build takes the kernel's error path and the
    # workgroup goes on to the next instance (regression: that path once left
    # all but one thread re-reading a stale work counter).
    torch = _torch()
    w = inputs.subset(inputs.config1(), [0, 1, 2])
    prob = P.problem_for_workload(h, w)
    pos = prob.pos.clone()
    off = prob.liz_off.cpu().numpy()
    pos[off[1] + 4] = pos[off[1] + 3]
    bad = P.Problem(3, prob.liz_off, pos, prob.species, w.energies, w.e_idx, w.delta, max_liz=prob.max_liz)
    opts = P.Opts(0, 0, 0, P.PERSISTENT)
    work = torch.empty(P.workspace_size(h, bad, 0, opts), dtype=torch.uint8, device="cuda")
    tau, info = P.tau00_solve(h, bad, work, opts)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert info[0] == 0 and info[1] == -2 and info[2] == 0
    assert np.all(np.isnan(tau.cpu().numpy()[1]))


def test_graph_replay(P, h):
    # captured once, replayed with eager work and an input change between
    # replays; every replay is checked against the oracle
    torch = _torch()
    w = inputs.subset(inputs.config1(), np.arange(0, 128, 4))
    ref, _ = _oracle_tau(w)
    w2 = inputs.subset(inputs.config1(), np.arange(0, 128, 4))
    w2.e_idx = (w2.e_idx + 5) % 16
    ref2, _ = _oracle_tau(w2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        prob = P.problem_for_workload(h, w)
        opts = P.Opts(0, 0, 0, P.PERSISTENT | P.GRAPH)
        work = torch.empty(P.workspace_size(h, prob, 0, opts), dtype=torch.uint8, device="cuda")
        tau = torch.empty(prob.n_inst * 256, dtype=torch.complex128, device="cuda")
        info = torch.empty(prob.n_inst, dtype=torch.int32, device="cuda")
        for rep in range(4):
            if rep == 2:
                prob.e_idx.copy_(torch.as_tensor(w2.e_idx, device="cuda"))
            tau.fill_(0)
            t, i = P.tau00_solve(h, prob, work, opts, tau=tau, info=info)
            s.synchronize()
            junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
            s.synchronize()
            assert np.all(i.cpu().numpy() == 0)
            check_tau(t.cpu().numpy(), ref if rep < 2 else ref2, w if rep < 2 else w2, TOL_TAU, f"replay {rep}")
        del junk


def test_autotune(P, h, tmp_path):
    torch = _torch()
    w = inputs.subset(inputs.config1(), np.arange(0, 128, 2))
    ref, _ = _oracle_tau(w)
    prob = P.problem_for_workload(h, w)
    n = prob.kk * prob.max_liz
    before32 = P.get_tuned_nb(h, n, P.PREC_FP32_IR)
    opts = P.Opts(0, 0, 0, P.PERSISTENT)
    work = torch.empty(P.workspace_size(h, prob, 0, opts), dtype=torch.uint8, device="cuda")
    best, ms = P.autotune(h, prob, work, opts)
    assert best in (32, 64, 96, 128) and all(v > 0 for v in ms.values())
    # keyed by (size bucket, precision): the FP64 tuning leaves the precision form's entry alone
    assert P.get_tuned_nb(h, n, P.PREC_FP64) == best
    assert P.get_tuned_nb(h, n, P.PREC_FP32_IR) == before32
    tau, info = P.tau00_solve(h, prob, work, opts)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    check_tau(tau.cpu().numpy(), ref, w, TOL_TAU, "after autotune")
    # the tuning cache survives a save / load into another handle
    P.set_tuned_nb(h, 2160, 96, P.PREC_FP32_IR)
    path = str(tmp_path / "tune.json")
    P.autotune_save(h, path)
    import json

    entries = json.load(open(path))
    assert {"n_max": 2176, "precision": 1, "nb": 96} in entries
    h2 = P.Handle()
    assert P.autotune_load(h2, path) == len(entries)
    assert P.get_tuned_nb(h2, n, P.PREC_FP64) == best
    assert P.get_tuned_nb(h2, 2160, P.PREC_FP32_IR) == 96
    assert P.get_tuned_nb(h2, 2160, P.PREC_FP64) == P.get_tuned_nb(h, 2160, P.PREC_FP64)
    h2.close()


def test_graph_follows_tuned_width(P, h):
    # a graph captured with one tuned panel width is not replayed after the
    # tuned width changes: each replay equals, bit for bit, a direct call
    # with the width then in force
    torch = _torch()
    w = inputs.subset(inputs.config1(), np.arange(1, 128, 6))
    ref, _ = _oracle_tau(w)
    prob = P.problem_for_workload(h, w)
    n = prob.kk * prob.max_liz
    s = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(s):
        og = P.Opts(0, 0, 0, P.PERSISTENT | P.GRAPH)
        work = torch.empty(P.workspace_size(h, prob, 0, og), dtype=torch.uint8, device="cuda")
        tau = torch.empty(prob.n_inst * 256, dtype=torch.complex128, device="cuda")
        info = torch.empty(prob.n_inst, dtype=torch.int32, device="cuda")
        for nb in (32, 128, 32):
            P.set_tuned_nb(h, n, nb, P.PREC_FP64)
            tau.fill_(0)
            t, i = P.tau00_solve(h, prob, work, og, tau=tau, info=info)
            s.synchronize()
            got = t.cpu().numpy()
            d, di = P.tau00_solve(h, prob, work, P.Opts(0, nb, 0, P.PERSISTENT))
            s.synchronize()
            assert np.all(i.cpu().numpy() == 0) and np.all(di.cpu().numpy() == 0)
            assert np.array_equal(_bits(got), _bits(d.cpu().numpy())), nb
            check_tau(got, ref, w, TOL_TAU, f"graph with tuned nb={nb}")
            out[nb] = got
    assert not np.array_equal(_bits(out[32]), _bits(out[128]))


@pytest.mark.parametrize("max_liz", [300, 1024])
def test_liz_truncation_keeps_nearest(P, h, max_liz):
    # cutoff 4.2a in the 10x10x10 vacancy/noise supercell: about 1200 sites
    # within the cutoff, more than the kernel's LDS candidate store; the rows
    # kept are the max_liz nearest, in the oracle's order
    w = inputs.config4(n_inst=6)
    w.rc = np.full(w.n_inst, 4.2 * inputs.A_LAT)
    liz = P.build_liz(h, w.atom_pos, w.atom_species, w.box, w.centre, w.rc, max_liz, with_atoms=True)
    off = liz["liz_off"].cpu().numpy()
    n = liz["liz_n"].cpu().numpy()
    pos = liz["pos"].cpu().numpy()
    atom = liz["atom"].cpu().numpy()
    for i, (c, rc) in enumerate(zip(w.centre, w.rc)):
        rel, idx = oracle.liz(w.atom_pos, w.box, int(c), float(rc), max_out=8192)
        assert rel.shape[0] > 1024 and n[i] == rel.shape[0]
        a, b = off[i], off[i + 1]
        assert b - a == min(rel.shape[0], max_liz)
        np.testing.assert_array_equal(atom[a:b], idx[:b - a])
        np.testing.assert_array_equal(pos[a:b], rel[:b - a])
