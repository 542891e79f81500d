"""GPU parity of the spin-canted path (build_kkr_spin, tau00_spin_batched,
tau00_spin_solve through the C ABI) against the CPU oracle.

With canted moments the KKR matrix of a LIZ has rank 2 N_LIZ (lmax+1)^2
(paper Sec. 2.1, 2.2): 416 on the tiny systems, 4320 (lmax = 3) and 6750
(lmax = 4, the CoCrFeMnNi rank of the paper's spin-canted benchmark) on the
135-atom LIZ.  Bars as the plain FP64 path: M elementwise within 1e-13 of
max|M|; tau00 rel_F <= 1e-12 per instance, and the scale-free
[M^{-1}]_{00} = tau00 t_0^{-1} elementwise within 1e-12 of its largest entry.
At the full ranks the oracle values come from tests/golden/canted_tau00.npz
(written by make_canted_golden.py beside it, which calls only the oracle).
"""

import dataclasses
import os

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_M = 1e-13
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "canted_tau00.npz")

SX = np.array([[0, 1], [1, 0]], complex)
SY = np.array([[0, -1j], [1j, 0]])
SZ = np.array([[1, 0], [0, -1]], complex)


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


def _canted_cfg1(lmax=3, moments=None, idx=None):
    w1 = inputs.config1()
    up, dn = inputs.spin_phase_shift_tables(w1.energies, lmax)
    mom = inputs.canted_moments(w1.atom_pos.shape[0], 0) if moments is None else moments
    w = dataclasses.replace(w1, lmax=lmax, delta=up, delta_dn=dn, atom_moment=mom)
    return w if idx is None else inputs.subset(w, idx)


def _t0_full(w):
    """t_0 of every instance as the kc x kc matrix (2 x 2 spin block per L)."""
    kk = w.kk
    lv = np.floor(np.sqrt(np.arange(kk)) + 1e-9).astype(int)
    out = np.zeros((w.n_inst, 2 * kk, 2 * kk), complex)
    for i in range(w.n_inst):
        c = int(w.centre[i])
        e = int(w.e_idx[i])
        s = int(w.atom_species[c])
        tu = oracle.tmat(w.lmax, w.energies[e], w.delta[s, e])[lv]
        td = oracle.tmat(w.lmax, w.energies[e], w.delta_dn[s, e])[lv]
        m = w.atom_moment[c]
        for L in range(kk):
            b = 0.5 * (tu[L] + td[L]) * np.eye(2) + 0.5 * (tu[L] - td[L]) * (m[0] * SX + m[1] * SY + m[2] * SZ)
            for a in range(2):
                for bb in range(2):
                    out[i, kk * a + L, kk * bb + L] = b[a, bb]
    return out


def _check(got, ref, w, what, tol=TOL):
    got = np.asarray(got)
    rf = np.linalg.norm((got - ref).reshape(len(ref), -1), axis=1) / np.linalg.norm(ref.reshape(len(ref), -1),
                                                                                      axis=1)
    t0 = _t0_full(w)
    xe = np.zeros(len(ref))
    for i in range(len(ref)):
        xg = np.linalg.solve(t0[i].T, got[i].T).T
        xr = np.linalg.solve(t0[i].T, ref[i].T).T
        xe[i] = np.abs(xg - xr).max() / np.abs(xr).max()
    print(f"{what}: rel_F max {rf.max():.2e}, [M^-1]00 elementwise max {xe.max():.2e}")
    assert rf.max() <= tol, (what, "rel_F", rf.max(), int(np.argmax(rf)))
    assert xe.max() <= tol, (what, "[M^-1]00", xe.max(), int(np.argmax(xe)))


def _build(P, h, w):
    torch = _torch()
    prob = P.problem_for_workload(h, w)
    N = prob.kc * np.diff(prob.liz_off.cpu().numpy())
    m_off = np.concatenate([[0], np.cumsum(N * N)[:-1]]).astype(np.int64)
    moff = torch.as_tensor(m_off, device="cuda")
    M = torch.zeros(int((N * N).sum()), dtype=torch.complex128, device="cuda")
    info = P.build_kkr_spin(h, prob, M, moff)
    torch.cuda.synchronize()
    return prob, M, moff, N, info.cpu().numpy()


def _solve(P, h, w, flags=0, nb=0, chunk=0):
    torch = _torch()
    prob = P.problem_for_workload(h, w)
    opts = P.Opts(0, nb, chunk, flags)
    n_slots = 1 if flags else (prob.n_inst if chunk == 0 else min(chunk, prob.n_inst))
    work = torch.empty(P.spin_workspace_size(h, prob, n_slots, opts), dtype=torch.uint8, device="cuda")
    tau, info = P.tau00_spin_solve(h, prob, work, opts)
    torch.cuda.synchronize()
    return tau.cpu().numpy(), info.cpu().numpy()


# ------------------------------------------------------------------ build
@pytest.mark.parametrize("lmax", [0, 1, 3, 4])
def test_spin_build_matches_oracle(P, h, lmax):
    w = _canted_cfg1(lmax, idx=[0, 17, 40, 127])
    prob, M, moff, N, info = _build(P, h, w)
    assert np.all(info == 0)
    Mg = M.cpu().numpy()
    liz_off, pos, spec = oracle.liz_batch(w)
    mom = oracle.liz_moments(w)
    for i in range(w.n_inst):
        a, b = liz_off[i], liz_off[i + 1]
        e = int(w.e_idx[i])
        ref, st = oracle.build_m_spin(lmax, pos[a:b], spec[a:b], mom[a:b], w.energies[e], w.delta[:, e],
                                      w.delta_dn[:, e])
        assert st == 0 and ref.shape[0] == N[i]
        got = Mg[moff[i].item():moff[i].item() + N[i] * N[i]].reshape(N[i], N[i]).T
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= TOL_M, (lmax, i, err)


# ------------------------------------------------------------------- tau00
def test_spin_batched_config1_all(P, h):
    # all 128 instances, rank 416: three 128-column panels and a ragged tail
    torch = _torch()
    w = _canted_cfg1()
    ref, rinfo = oracle.tau00_spin_workload(w)
    assert np.all(rinfo == 0)
    prob, M, moff, N, binfo = _build(P, h, w)
    assert np.all(binfo == 0)
    work = torch.empty(prob.n_inst * P.BATCHED_WORK_PER_INST, dtype=torch.uint8, device="cuda")
    tau, info = P.tau00_spin_batched(h, prob, M, moff, work=work)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    _check(tau.cpu().numpy(), ref, w, "canted config1 batched")


@pytest.mark.parametrize("flags,nb,chunk", [(1, 0, 0), (0, 48, 7), (0, 16, 0), (1, 96, 0)])
def test_spin_solve_modes(P, h, flags, nb, chunk):
    w = _canted_cfg1(idx=np.arange(0, 128, 5))
    ref, rinfo = oracle.tau00_spin_workload(w)
    tau, info = _solve(P, h, w, flags, nb, chunk)
    assert np.all(info == 0)
    _check(tau, ref, w, f"canted solve flags={flags} nb={nb} chunk={chunk}")


@pytest.mark.parametrize("lmax", [0, 2, 4])
def test_spin_other_lmax(P, h, lmax):
    # rank 26, 234, 650 (kc = 50 at lmax = 4: the Gauss-Jordan block above 32)
    w = _canted_cfg1(lmax, idx=np.arange(3, 128, 11))
    ref, rinfo = oracle.tau00_spin_workload(w)
    tau, info = _solve(P, h, w, flags=1)
    assert np.all(info == 0)
    _check(tau, ref, w, f"canted lmax={lmax}")


def test_spin_collinear_is_two_plain_solves(P, h):
    # every moment along +z: the GPU's canted tau00 is block-diagonal, its
    # blocks the GPU's plain tau00 of the up and the down phase shifts
    n_at = inputs.config1().atom_pos.shape[0]
    w = _canted_cfg1(moments=np.tile([0.0, 0.0, 1.0], (n_at, 1)), idx=np.arange(0, 128, 9))
    tau, info = _solve(P, h, w, flags=1)
    assert np.all(info == 0)
    kk = w.kk
    torch = _torch()
    for blk, delta in ((slice(0, kk), w.delta), (slice(kk, 2 * kk), w.delta_dn)):
        wp = dataclasses.replace(w, delta=delta, delta_dn=None, atom_moment=None)
        prob = P.problem_for_workload(h, wp)
        work = torch.empty(P.workspace_size(h, prob, 1, P.Opts(0, 0, 0, 1)), dtype=torch.uint8, device="cuda")
        plain, pinfo = P.tau00_solve(h, prob, work, P.Opts(0, 0, 0, 1))
        torch.cuda.synchronize()
        plain = plain.cpu().numpy()
        assert np.all(pinfo.cpu().numpy() == 0)
        err = np.abs(tau[:, blk, blk] - plain).max() / np.abs(plain).max()
        assert err <= 1e-12, err
    assert np.all(tau[:, :kk, kk:] == 0) and np.all(tau[:, kk:, :kk] == 0)


def test_spin_global_rotation(P, h):
    # rotating every moment by R rotates tau00 by the matching SU(2) matrix
    ax = np.array([0.3, -0.8, 0.5])
    ax /= np.linalg.norm(ax)
    ang = 1.1
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    R = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
    U = np.cos(ang / 2) * np.eye(2) - 1j * np.sin(ang / 2) * (ax[0] * SX + ax[1] * SY + ax[2] * SZ)
    w = _canted_cfg1(idx=np.arange(2, 128, 13))
    tau, info = _solve(P, h, w, flags=1)
    w2 = dataclasses.replace(w, atom_moment=w.atom_moment @ R.T)
    tau2, info2 = _solve(P, h, w2, flags=1)
    assert np.all(info == 0) and np.all(info2 == 0)
    big = np.kron(U, np.eye(w.kk))
    pred = big @ tau @ big.conj().T
    err = np.abs(tau2 - pred).max() / np.abs(pred).max()
    assert err <= 1e-12, err


def test_spin_argument_errors(P, h):
    torch = _torch()
    w = _canted_cfg1(idx=[0, 1])
    prob = P.problem_for_workload(h, w)
    L = P.lib()
    import ctypes

    ps = prob.struct()
    o = P.Opts()
    sz = ctypes.c_size_t()
    assert L.lsms_spin_workspace_size(h.ptr, ctypes.byref(ps), None, ctypes.byref(o), 1, ctypes.byref(sz)) == -3
    sp = P.lsms._Spin(None, None)
    assert L.lsms_spin_workspace_size(h.ptr, ctypes.byref(ps), ctypes.byref(sp), ctypes.byref(o), 1,
                                      ctypes.byref(sz)) == -3
    spg = prob.spin.struct()
    og = P.Opts(0, 0, 0, P.GRAPH)
    assert L.lsms_spin_workspace_size(h.ptr, ctypes.byref(ps), ctypes.byref(spg), ctypes.byref(og), 1,
                                      ctypes.byref(sz)) == -4
    of = P.Opts(1, 0, 0, 0)
    assert L.lsms_spin_workspace_size(h.ptr, ctypes.byref(ps), ctypes.byref(spg), ctypes.byref(of), 1,
                                      ctypes.byref(sz)) == -4
    assert L.lsms_spin_workspace_size(h.ptr, ctypes.byref(ps), ctypes.byref(spg), ctypes.byref(o), 1,
                                      ctypes.byref(sz)) == 0
    work = torch.empty(16, dtype=torch.uint8, device="cuda")
    tau = torch.empty(2 * 32 * 32, dtype=torch.complex128, device="cuda")
    info = torch.empty(2, dtype=torch.int32, device="cuda")
    rc = L.tau00_spin_solve(h.ptr, ctypes.byref(ps), ctypes.byref(spg), ctypes.byref(o),
                            ctypes.c_void_p(tau.data_ptr()), ctypes.c_void_p(info.data_ptr()),
                            ctypes.c_void_p(work.data_ptr()), 16, None)
    assert rc == -8
    torch.cuda.synchronize()


# ------------------------------------------------------ full spin-canted ranks
def _golden(lmax):
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/canted_tau00.npz not written")
    g = np.load(GOLDEN, allow_pickle=False)
    return g[f"idx_l{lmax}"], g[f"tau_l{lmax}"]


@pytest.mark.parametrize("lmax,flags", [(3, 1), (3, 0), (4, 0)])
def test_spin_full_rank(P, h, lmax, flags):
    # rank 4320 (lmax 3) and 6750 (lmax 4): a Ni and an Au centre at the
    # contour ends, persistent and chunked launches
    idx, ref = _golden(lmax)
    w = inputs.subset(inputs.config_canted(lmax=lmax), idx)
    print(f"canted full rank lmax={lmax}: N={2 * w.kk * 135}, instances {idx.tolist()}", flush=True)
    tau, info = _solve(P, h, w, flags=flags, chunk=0 if flags else 2)
    assert np.all(info == 0)
    _check(tau, ref, w, f"canted rank {2 * w.kk * 135}")
