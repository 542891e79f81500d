"""GPU parity of the block row of tau, ln det M and the contour integrals
(tau_row_batched, lsms_lloyd_idos, lsms_contour_sum through the C ABI)
against the CPU oracle.

tau^{0j} = [M^{-1}]_{0j} t_j (paper Sec. 2.1, eq. Dyson_equation; the blocks
that enter eq. Green_KKR); ln det M is the multiple-scattering term of Lloyd's
formula for the integrated density of states (the energy integral of
eq. Density).

Bars:
  - block row: rel_F <= 1e-12 per instance, and the scale-free block row of
    M^{-1} (tau^{0j} diag(t_j)^{-1}) elementwise within 1e-12 of its largest
    entry (the same FP64 bar as tau00; t_j of the f channel is orders of
    magnitude below the s channel, so the elementwise check sees errors the
    norm hides);
  - ln det M: |d Re| and the wrapped |d Im| at most 1e-10 (absolute, i.e.
    1e-10 relative on det M and on its phase).  Each of the N pivots carries a
    relative rounding error of order cond(M) u, so the sum of their logarithms
    is off by about sqrt(N) cond(M) u: 5e-12 at N = 2160, cond 1e3, with a
    growth margin for the contour ends (cond 1e4);
  - tau00 of this entry point bit-equal to tau00_batched's (same elimination,
    the upper factor only written out in addition);
  - contour sum and Lloyd's integrated DOS: 1e-12 relative to the largest
    entry (sums of 16..32 terms of those inputs).
"""

import numpy as np
import pytest

import inputs
import oracle
from parity import check_tau, l_of, oracle_cached, rel_f

pytestmark = pytest.mark.gpu

TOL_ROW = 1e-12
TOL_LD = 1e-10
TOL_SUM = 1e-12


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint64)


@pytest.fixture(scope="module")
def P():
    _torch()
    import paper_2308_16317_amd as P

    return P


@pytest.fixture(scope="module")
def h(P):
    return P.Handle()


def _build(P, h, w):
    torch = _torch()
    prob = P.problem_for_workload(h, w)
    N = prob.kk * np.diff(prob.liz_off.cpu().numpy())
    m_off = np.concatenate([[0], np.cumsum(N * N)[:-1]]).astype(np.int64)
    moff = torch.as_tensor(m_off, device="cuda")
    M = torch.zeros(int((N * N).sum()), dtype=torch.complex128, device="cuda")
    binfo = P.build_kkr(h, prob, M, moff)
    torch.cuda.synchronize()
    assert np.all(binfo.cpu().numpy() == 0)
    return prob, M, moff, N


def _run_row(P, h, w, nb=0):
    torch = _torch()
    prob, M, moff, N = _build(P, h, w)
    M2 = M.clone()
    rows, roff, ld, tau, info = P.tau_row_batched(h, prob, M, moff, P.Opts(0, nb, 0, 0))
    work = torch.empty(prob.n_inst * P.BATCHED_WORK_PER_INST, dtype=torch.uint8, device="cuda")
    tref, iref = P.tau00_batched(h, prob, M2, moff, P.Opts(0, nb, 0, 0), work=work)
    torch.cuda.synchronize()
    kk = prob.kk
    r = rows.cpu().numpy()
    ro = roff.cpu().numpy()
    blocks = [r[ro[i]:ro[i] + kk * N[i]].reshape(N[i], kk).T for i in range(prob.n_inst)]
    tau = tau.cpu().numpy()
    info = info.cpu().numpy()
    assert np.array_equal(_bits(tau), _bits(tref.cpu().numpy())), "tau00 differs from tau00_batched"
    assert np.array_equal(info, iref.cpu().numpy())
    return blocks, ld.cpu().numpy(), tau, info


def _t_cols(w, i):
    """t_{s(j), l(L')} for every column kk*j + L' of instance i's block row."""
    rel, idx = oracle.liz(w.atom_pos, w.box, int(w.centre[i]), float(w.rc[i]))
    e = int(w.e_idx[i])
    lv = l_of(w.kk)
    spec = w.atom_species[idx]
    return np.concatenate([oracle.tmat(w.lmax, w.energies[e], w.delta[s, e])[lv] for s in spec])


def _check_rows(blocks, ref_blocks, w, what):
    worst_f = worst_x = 0.0
    for i, (g, r) in enumerate(zip(blocks, ref_blocks)):
        assert g.shape == r.shape, (what, i, g.shape, r.shape)
        rf = np.linalg.norm(g - r) / np.linalg.norm(r)
        t = _t_cols(w, i)
        keep = np.abs(t) > 0
        yg = g[:, keep] / t[None, keep]
        yr = r[:, keep] / t[None, keep]
        xe = np.abs(yg - yr).max() / np.abs(yr).max()
        worst_f = max(worst_f, rf)
        worst_x = max(worst_x, xe)
        assert rf <= TOL_ROW, (what, "row rel_F", i, rf)
        assert xe <= TOL_ROW, (what, "[M^-1]_0: elementwise", i, xe)
    print(f"{what}: block row rel_F max {worst_f:.2e}, [M^-1]_0: elementwise max {worst_x:.2e}")


def _check_logdet(ld, ref, what):
    d_re = np.abs(ld.real - ref.real)
    d_im = np.abs(np.angle(np.exp(1j * (ld.imag - ref.imag))))
    print(f"{what}: ln det M |d Re| max {d_re.max():.2e}, |d Im| max {d_im.max():.2e}")
    assert d_re.max() <= TOL_LD, (what, "Re ln det", d_re.max(), int(np.argmax(d_re)))
    assert d_im.max() <= TOL_LD, (what, "Im ln det", d_im.max(), int(np.argmax(d_im)))
    assert np.all(ld.imag > -np.pi) and np.all(ld.imag <= np.pi)


_ROWS = {}


def _oracle_rows(key, w):
    if key not in _ROWS:
        rows, rinfo = oracle.tau_row_workload(w)
        ld, linfo = oracle.logdet_workload(w)
        assert np.all(rinfo == 0) and np.all(linfo == 0)
        _ROWS[key] = (rows, ld)
    return _ROWS[key]


# ------------------------------------------------------------- block row
@pytest.mark.parametrize("nb", [0, 64, 16, 48])
def test_row_logdet_config1_all(P, h, nb):
    # all 128 instances (N = 208: four panels of 48, the last one ragged)
    w = inputs.config1()
    ref_rows, ref_ld = _oracle_rows("cfg1", w)
    ref_tau, _ = oracle_cached("cfg1", w)
    blocks, ld, tau, info = _run_row(P, h, w, nb)
    assert np.all(info == 0)
    check_tau(tau, ref_tau, w, TOL_ROW, f"tau00 of tau_row_batched nb={nb}")
    _check_rows(blocks, ref_rows, w, f"config1 nb={nb}")
    _check_logdet(ld, ref_ld, f"config1 nb={nb}")
    # the central block of the row is tau00 itself
    for i in range(w.n_inst):
        assert np.allclose(blocks[i][:, :w.kk], tau[i], rtol=0, atol=1e-14 * np.abs(tau[i]).max())


@pytest.mark.parametrize("lmax", [0, 1, 2, 4])
def test_row_logdet_other_lmax(P, h, lmax):
    # N = 13, 52, 117, 325 (kk = 25 takes the 32-column solve)
    w = inputs.subset(inputs.config1().with_lmax(lmax), np.arange(0, 128, 9))
    ref_rows, ref_ld = _oracle_rows(f"cfg1-l{lmax}", w)
    blocks, ld, tau, info = _run_row(P, h, w)
    assert np.all(info == 0)
    _check_rows(blocks, ref_rows, w, f"lmax={lmax}")
    _check_logdet(ld, ref_ld, f"lmax={lmax}")


def test_row_logdet_ragged(P, h):
    # eight instances of the ragged workload in one batch (N 1184..2400)
    w = inputs.subset(inputs.config4(n_inst=1024), np.linspace(0, 1023, 8).astype(int))
    ref_rows, ref_ld = _oracle_rows("cfg4-8", w)
    blocks, ld, tau, info = _run_row(P, h, w)
    assert np.all(info == 0)
    _check_rows(blocks, ref_rows, w, "config4 sample")
    _check_logdet(ld, ref_ld, "config4 sample")


def test_row_logdet_full_size(P, h):
    # N = 2160: both contour ends and mid-contour, one Ni and one Au centre
    w2 = inputs.config2()
    ni = int(np.flatnonzero(w2.atom_species == 0)[0])
    au = int(np.flatnonzero(w2.atom_species == 1)[0])
    w = inputs.subset(w2, [ni * 32, ni * 32 + 31, au * 32 + 16, au * 32 + 31])
    ref_rows, ref_ld = _oracle_rows("cfg2-4", w)
    blocks, ld, tau, info = _run_row(P, h, w)
    assert np.all(info == 0)
    _check_rows(blocks, ref_rows, w, "N=2160")
    _check_logdet(ld, ref_ld, "N=2160")


def test_row_logdet_lmax4_full_size(P, h):
    # N = 3375 (the larger leaf register tile and the 32-column solve)
    w = inputs.subset(inputs.config3(), [0, 32 * 7 + 31])
    ref_rows, ref_ld = _oracle_rows("cfg3-2", w)
    blocks, ld, tau, info = _run_row(P, h, w)
    assert np.all(info == 0)
    _check_rows(blocks, ref_rows, w, "N=3375")
    _check_logdet(ld, ref_ld, "N=3375")


# ------------------------------------------------- closed forms, errors
def test_logdet_closed_forms(P, h):
    torch = _torch()
    # dimer at lmax = 0: det M = 1 - t_A t_B g^2, g = -exp(i kappa R) / R
    E = 0.25 + 0.1j
    delta = np.array([[[0.3 + 0.02j]], [[-0.7 + 0.05j]]])
    R = np.array([[0, 0, 0], [2.0, -3.0, 1.5]])
    prob = P.Problem(0, [0, 2], R, [0, 1], [E], [0], delta)
    m_off = torch.zeros(1, dtype=torch.int64, device="cuda")
    M = torch.zeros(4, dtype=torch.complex128, device="cuda")
    P.build_kkr(h, prob, M, m_off)
    _, _, ld, tau, info = P.tau_row_batched(h, prob, M, m_off)
    torch.cuda.synchronize()
    tA = oracle.tmat(0, E, delta[0, 0])[0]
    tB = oracle.tmat(0, E, delta[1, 0])[0]
    r = np.linalg.norm(R[1])
    g = -np.exp(1j * np.sqrt(E) * r) / r
    ref = np.log(1 - tA * tB * g * g)
    assert info.cpu().numpy()[0] == 0
    assert abs(ld.cpu().numpy()[0] - ref) <= 1e-14
    # one-atom LIZ and t = 0: M = I, ln det M = 0 exactly, block row = tau00
    w = inputs.subset(inputs.config1(), [0, 5])
    w0 = inputs.subset(inputs.config1(), [0, 5])
    w0.delta = np.zeros_like(w0.delta)
    for ww in (w0,):
        prob, M, moff, N = _build(P, h, ww)
        rows, roff, ld, tau, info = P.tau_row_batched(h, prob, M, moff)
        torch.cuda.synchronize()
        assert np.all(info.cpu().numpy() == 0)
        assert np.all(ld.cpu().numpy() == 0)
        assert np.all(rows.cpu().numpy() == 0)
    w.rc = np.full(w.n_inst, 0.1)
    prob, M, moff, N = _build(P, h, w)
    assert np.all(N == 16)
    rows, roff, ld, tau, info = P.tau_row_batched(h, prob, M, moff)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0) and np.all(ld.cpu().numpy() == 0)
    t = tau.cpu().numpy()
    assert np.array_equal(rows.cpu().numpy().reshape(2, 16, 16).transpose(0, 2, 1), t)


@pytest.mark.parametrize("step", [1, 300, 2145])
def test_row_zero_pivot(P, h, step):
    # as the tau00 zero-pivot test: M = I with one zero row of M; the row and
    # ln det M are NaN and info names the step
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
    rows, roff, ld, tau, info = P.tau_row_batched(h, prob, Md, torch.zeros(1, dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    assert int(info.cpu().numpy()[0]) == step
    assert np.all(np.isnan(ld.cpu().numpy()))
    assert np.all(np.isnan(rows.cpu().numpy()))
    assert np.all(np.isnan(tau.cpu().numpy()))


def test_row_argument_errors(P, h):
    torch = _torch()
    w = inputs.subset(inputs.config1(), [0, 1])
    prob, M, moff, N = _build(P, h, w)
    L = P.lib()
    ps = prob.struct()
    import ctypes

    tau = torch.empty(2 * 256, dtype=torch.complex128, device="cuda")
    info = torch.empty(2, dtype=torch.int32, device="cuda")
    rows = torch.empty(2 * 16 * 208, dtype=torch.complex128, device="cuda")
    need = P.row_workspace_size(h, prob)
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    o = P.Opts()

    def call(row_off, row, tau_p, work_p, wb, opts=o):
        return L.tau_row_batched(h.ptr, ctypes.byref(ps), ctypes.c_void_p(M.data_ptr()),
                                 ctypes.c_void_p(moff.data_ptr()), ctypes.byref(opts), row_off, row, None,
                                 tau_p, ctypes.c_void_p(info.data_ptr()), work_p, wb, None)

    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert call(None, ptr(rows), ptr(tau), ptr(work), need) == -6
    assert call(None, None, None, ptr(work), need) == -9
    assert call(None, None, ptr(tau), None, need) == -11
    assert call(None, None, ptr(tau), ptr(work), need - 1) == -12
    assert call(None, None, ptr(tau), ptr(work), need, P.Opts(1, 0, 0, 0)) == -5
    torch.cuda.synchronize()


# ------------------------------------------ contour integrals (eq. Density)
def test_lloyd_and_contour_sum(P, h):
    # every energy of the eight config-1 sites: GPU ln det M -> Lloyd's
    # integrated DOS along the contour, GPU tau00 -> its contour integral,
    # against the oracle's functions on the oracle's values
    w = inputs.config1()
    ref_rows, ref_ld = _oracle_rows("cfg1", w)
    ref_tau, _ = oracle_cached("cfg1", w)
    blocks, ld, tau, info = _run_row(P, h, w)
    assert np.all(info == 0)
    torch = _torch()
    n_sites, n_e = 8, 16
    idos = P.lloyd_idos(h, torch.as_tensor(ld).to("cuda"), n_sites, n_e).cpu().numpy()
    ref_idos = np.stack([oracle.lloyd_ms_idos(ref_ld[s * n_e:(s + 1) * n_e]) for s in range(n_sites)])
    err = np.abs(idos - ref_idos).max() / max(np.abs(ref_idos).max(), 1.0)
    print(f"Lloyd integrated DOS: max err {err:.2e} (largest |N| {np.abs(ref_idos).max():.3f})")
    assert err <= TOL_LD
    wts = inputs.contour_weights(n_e)
    got = P.contour_sum(h, wts, torch.as_tensor(np.ascontiguousarray(tau)).to("cuda"), n_sites, n_e).cpu().numpy()
    ref = np.stack([oracle.contour_integral(ref_tau[s * n_e:(s + 1) * n_e], wts) for s in range(n_sites)])
    rf = rel_f(got, ref)
    print(f"contour integral of tau00: rel_F max {rf.max():.2e}")
    assert rf.max() <= TOL_SUM * 10
    # a polynomial in E integrates exactly: sum_k w_k E_k^2 = (E_b^3 - E_a^3) / 3
    Ea, Eb = inputs.contour_ends()
    ek = inputs.contour_energies(n_e)
    vals = torch.as_tensor(np.repeat((ek ** 2)[None, :, None], 3, axis=0).reshape(3 * n_e, 1)).to("cuda")
    s2 = P.contour_sum(h, wts, vals, 3, n_e).cpu().numpy()
    assert np.allclose(s2[:, 0], (Eb ** 3 - Ea ** 3) / 3, rtol=1e-13, atol=0)
