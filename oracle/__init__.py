"""CPU FP64 oracle for the LSMS tau00 path (ctypes over lsms_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The product package never imports it.

Every function follows the definitions cited in lsms_oracle.c (paper Sec. 2.1
eq. Dyson_equation, Sec. 2.2, Sec. 3.2).  Arrays are numpy; complex values are
complex128; matrices are returned with natural [row, column] indexing.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsms_oracle.c")
_LIB = os.path.join(_HERE, "liblsms_oracle.so")
_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int


def build(force: bool = True) -> str:
    """Compile lsms_oracle.c into liblsms_oracle.so beside it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fcx-limited-range", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_liz.restype = _I
        L.orc_liz.argtypes = [_P, _I, _P, _I, ctypes.c_double, _I, _P, _P]
        L.orc_ylm.argtypes = [_I, _P, _P]
        L.orc_gaunt.restype = _I
        L.orc_gaunt.argtypes = [_I, _P]
        L.orc_hankel.argtypes = [_I, _P, _P]
        L.orc_tmat.argtypes = [_I, _P, _P, _P]
        L.orc_structure_constants.argtypes = [_I, _P, _P, _P, _P]
        L.orc_build_m.restype = _I
        L.orc_build_m.argtypes = [_I, _I, _P, _P, _P, _P, _I, _P, _P]
        L.orc_lu_factor.restype = _I
        L.orc_lu_factor.argtypes = [_I, _P, _P]
        L.orc_lu_solve.argtypes = [_I, _P, _P, _I, _P]
        L.orc_tau00_batch.argtypes = [_I, _I, _P, _P, _P, _P, _P, _P, _I, _I, _I, _P, _P]
        L.orc_set_threads.argtypes = [_I]
        L.orc_max_threads.restype = _I
        L.orc_tau00_schur.restype = _I
        L.orc_tau00_schur.argtypes = [_I, _I, _P, _P, _P, _P, _I, _P, _P]
        L.orc_build_m_spin.restype = _I
        L.orc_build_m_spin.argtypes = [_I, _I, _P, _P, _P, _P, _P, _P, _I, _P, _P]
        L.orc_tau00_spin_batch.argtypes = [_I, _I, _P, _P, _P, _P, _P, _P, _P, _P, _I, _I, _I, _P, _P]
        L.orc_tau_row_batch.argtypes = [_I, _I, _P, _P, _P, _P, _P, _P, _I, _I, _I, _P, _P, _P]
        L.orc_logdet_batch.argtypes = [_I, _I, _P, _P, _P, _P, _P, _P, _I, _I, _P, _P]
        _lib = L
    return _lib


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- a1: LIZ
def liz(pos, box, centre: int, rc: float, max_out: int = 4096):
    """LIZ of one centre: (rel [n, 3] relative vectors, idx [n] atom ids), centre first."""
    pos = _c(pos, np.float64)
    box = _c(box, np.float64)
    rel = np.zeros((max_out, 3))
    idx = np.zeros(max_out, np.int32)
    n = lib().orc_liz(_ptr(pos), pos.shape[0], _ptr(box), int(centre), float(rc), max_out, _ptr(rel), _ptr(idx))
    if n > max_out:
        raise ValueError(f"LIZ of {n} atoms exceeds max_out={max_out}")
    return rel[:n].copy(), idx[:n].copy()


def liz_batch(w):
    """LIZs of every instance of a workload: (liz_off [n+1] int64, pos [tot, 3], species [tot])."""
    offs = [0]
    rels, specs = [], []
    for c, r in zip(w.centre, w.rc):
        rel, idx = liz(w.atom_pos, w.box, int(c), float(r))
        rels.append(rel)
        specs.append(w.atom_species[idx])
        offs.append(offs[-1] + rel.shape[0])
    return (np.asarray(offs, np.int64), np.concatenate(rels).astype(np.float64),
            np.concatenate(specs).astype(np.int32))


# ------------------------------------------------------- angular / radial
def ylm(lmax: int, r):
    r = _c(r, np.float64)
    Y = np.zeros((lmax + 1) ** 2)
    lib().orc_ylm(lmax, _ptr(r), _ptr(Y))
    return Y


def gaunt(lmax: int):
    """Real Gaunt table C[L, L', L''] (l, l' <= lmax, l'' <= 2 lmax) and its nonzero count."""
    kk = (lmax + 1) ** 2
    kk2 = (2 * lmax + 1) ** 2
    C = np.zeros((kk, kk, kk2))
    nnz = lib().orc_gaunt(lmax, _ptr(C))
    return C, nnz


def hankel(lmax: int, z: complex):
    zz = np.array([complex(z).real, complex(z).imag])
    h = np.zeros(2 * (lmax + 1))
    lib().orc_hankel(lmax, _ptr(zz), _ptr(h))
    return h[0::2] + 1j * h[1::2]


def tmat(lmax: int, E: complex, delta_l):
    Er = np.array([complex(E).real, complex(E).imag])
    d = _c(delta_l, np.complex128)
    t = np.zeros(lmax + 1, np.complex128)
    lib().orc_tmat(lmax, _ptr(Er), _ptr(d), _ptr(t))
    return t


def structure_constants(lmax: int, kappa: complex, R, C=None):
    """G^{ij}[L, L'] for R = R_i - R_j."""
    if C is None:
        C, _ = gaunt(lmax)
    C = _c(C, np.float64)
    kk = (lmax + 1) ** 2
    k = np.array([complex(kappa).real, complex(kappa).imag])
    R = _c(R, np.float64)
    G = np.zeros((kk, kk), np.complex128, order="F")
    lib().orc_structure_constants(lmax, _ptr(k), _ptr(R), _ptr(C), _ptr(G))
    return G


# --------------------------------------------------------- a2 + a3: M
def build_m(lmax: int, rel, spec, E: complex, delta_e, C=None):
    """M = 1 - t G over one LIZ; delta_e [n_species, lmax + 1] at this energy.
    Returns (M [N, N], status)."""
    if C is None:
        C, _ = gaunt(lmax)
    C = _c(C, np.float64)
    rel = _c(rel, np.float64)
    spec = _c(spec, np.int32)
    d = _c(delta_e, np.complex128)
    n_liz = rel.shape[0]
    N = (lmax + 1) ** 2 * n_liz
    M = np.zeros((N, N), np.complex128, order="F")
    Er = np.array([complex(E).real, complex(E).imag])
    st = lib().orc_build_m(lmax, n_liz, _ptr(rel), _ptr(spec), _ptr(Er), _ptr(d), d.shape[0], _ptr(C), _ptr(M))
    return M, st


# ------------------------------------------------------ a4 + a5: LU, tau00
def lu_factor(A):
    LU = np.array(A, dtype=np.complex128, order="F", copy=True)
    n = LU.shape[0]
    ipiv = np.zeros(n, np.int32)
    info = lib().orc_lu_factor(n, _ptr(LU), _ptr(ipiv))
    return LU, ipiv, info


def lu_solve(LU, ipiv, B):
    X = np.array(B, dtype=np.complex128, order="F", copy=True)
    if X.ndim == 1:
        X = X.reshape(-1, 1, order="F")
    lib().orc_lu_solve(LU.shape[0], _ptr(np.asfortranarray(LU)), _ptr(_c(ipiv, np.int32)), X.shape[1], _ptr(X))
    return X


def tau00_batch(lmax: int, liz_off, pos, species, energies, e_idx, delta, refine: int = 2):
    """tau00 [n_inst, kk, kk] (natural [L, L'] indexing) and info [n_inst]."""
    liz_off = _c(liz_off, np.int64)
    pos = _c(pos, np.float64)
    species = _c(species, np.int32)
    energies = _c(energies, np.complex128)
    e_idx = _c(e_idx, np.int32)
    delta = _c(delta, np.complex128)
    n = e_idx.shape[0]
    kk = (lmax + 1) ** 2
    tau = np.zeros((n, kk, kk), np.complex128)  # [i][L'][L] in memory = column-major per instance
    info = np.zeros(n, np.int32)
    lib().orc_tau00_batch(lmax, n, _ptr(liz_off), _ptr(pos), _ptr(species), _ptr(energies), _ptr(e_idx),
                          _ptr(delta), delta.shape[0], delta.shape[1], int(refine), _ptr(tau), _ptr(info))
    return tau.transpose(0, 2, 1).copy(), info


def tau00_schur(lmax: int, rel, spec, E: complex, delta_e, C=None):
    if C is None:
        C, _ = gaunt(lmax)
    kk = (lmax + 1) ** 2
    rel = _c(rel, np.float64)
    spec = _c(spec, np.int32)
    d = _c(delta_e, np.complex128)
    Er = np.array([complex(E).real, complex(E).imag])
    tau = np.zeros((kk, kk), np.complex128, order="F")
    info = lib().orc_tau00_schur(lmax, rel.shape[0], _ptr(rel), _ptr(spec), _ptr(Er), _ptr(d), d.shape[0],
                                 _ptr(_c(C, np.float64)), _ptr(tau))
    return tau, info


def tau00_workload(w, refine: int = 2):
    """Oracle tau00 for every instance of an inputs.Workload."""
    liz_off, pos, spec = liz_batch(w)
    return tau00_batch(w.lmax, liz_off, pos, spec, w.energies, w.e_idx, w.delta, refine)


# ------------------------------------------------------------- spin canting
def build_m_spin(lmax: int, rel, spec, mom, E: complex, delta_up_e, delta_dn_e, C=None):
    """Spin-canted M over one LIZ (rank 2 kk n_liz, index 2 kk j + kk s + L);
    mom [n_liz, 3] unit moment directions, delta_*_e [n_species, lmax + 1] at
    this energy.  Returns (M, status)."""
    if C is None:
        C, _ = gaunt(lmax)
    rel = _c(rel, np.float64)
    spec = _c(spec, np.int32)
    mom = _c(mom, np.float64)
    du = _c(delta_up_e, np.complex128)
    dd = _c(delta_dn_e, np.complex128)
    n_liz = rel.shape[0]
    N = 2 * (lmax + 1) ** 2 * n_liz
    M = np.zeros((N, N), np.complex128, order="F")
    Er = np.array([complex(E).real, complex(E).imag])
    st = lib().orc_build_m_spin(lmax, n_liz, _ptr(rel), _ptr(spec), _ptr(mom), _ptr(Er), _ptr(du), _ptr(dd),
                                du.shape[0], _ptr(_c(C, np.float64)), _ptr(M))
    return M, st


def tau00_spin_batch(lmax: int, liz_off, pos, species, moment, energies, e_idx, delta_up, delta_dn,
                     refine: int = 2):
    """Spin-canted tau00 [n_inst, 2kk, 2kk] (natural [(s,L), (s',L')] indexing,
    index kk s + L) and info [n_inst]; moment [liz rows, 3] per LIZ row."""
    liz_off = _c(liz_off, np.int64)
    pos = _c(pos, np.float64)
    species = _c(species, np.int32)
    moment = _c(moment, np.float64)
    energies = _c(energies, np.complex128)
    e_idx = _c(e_idx, np.int32)
    du = _c(delta_up, np.complex128)
    dd = _c(delta_dn, np.complex128)
    n = e_idx.shape[0]
    kc = 2 * (lmax + 1) ** 2
    tau = np.zeros((n, kc, kc), np.complex128)
    info = np.zeros(n, np.int32)
    lib().orc_tau00_spin_batch(lmax, n, _ptr(liz_off), _ptr(pos), _ptr(species), _ptr(moment), _ptr(energies),
                               _ptr(e_idx), _ptr(du), _ptr(dd), du.shape[0], du.shape[1], int(refine), _ptr(tau),
                               _ptr(info))
    return tau.transpose(0, 2, 1).copy(), info


def liz_moments(w):
    """Moment direction of every LIZ row of a spin-canted workload, in the
    order of liz_batch."""
    out = []
    for c, r in zip(w.centre, w.rc):
        _, idx = liz(w.atom_pos, w.box, int(c), float(r))
        out.append(w.atom_moment[idx])
    return np.concatenate(out).astype(np.float64)


def tau00_spin_workload(w, refine: int = 2):
    """Oracle spin-canted tau00 for every instance of a spin-canted workload."""
    liz_off, pos, spec = liz_batch(w)
    return tau00_spin_batch(w.lmax, liz_off, pos, spec, liz_moments(w), w.energies, w.e_idx, w.delta, w.delta_dn,
                            refine)


# ------------------------------------------------ block row of tau, ln det M
def tau_row_batch(lmax: int, liz_off, pos, species, energies, e_idx, delta, refine: int = 2):
    """Block rows tau^{0j} = [M^-1]_{0j} t_j of every instance: a list of
    [kk, N_i] arrays (natural [L, column] indexing, column = j*kk + L') and
    info [n_inst]."""
    liz_off = _c(liz_off, np.int64)
    pos = _c(pos, np.float64)
    species = _c(species, np.int32)
    energies = _c(energies, np.complex128)
    e_idx = _c(e_idx, np.int32)
    delta = _c(delta, np.complex128)
    n = e_idx.shape[0]
    kk = (lmax + 1) ** 2
    N = kk * np.diff(liz_off)
    row_off = np.concatenate([[0], np.cumsum(kk * N)[:-1]]).astype(np.int64)
    out = np.zeros(int((kk * N).sum()), np.complex128)
    info = np.zeros(n, np.int32)
    lib().orc_tau_row_batch(lmax, n, _ptr(liz_off), _ptr(pos), _ptr(species), _ptr(energies), _ptr(e_idx),
                            _ptr(delta), delta.shape[0], delta.shape[1], int(refine), _ptr(row_off), _ptr(out),
                            _ptr(info))
    rows = [out[row_off[i]:row_off[i] + kk * N[i]].reshape(N[i], kk).T.copy() for i in range(n)]
    return rows, info


def tau_row_workload(w, refine: int = 2):
    liz_off, pos, spec = liz_batch(w)
    return tau_row_batch(w.lmax, liz_off, pos, spec, w.energies, w.e_idx, w.delta, refine)


def logdet_batch(lmax: int, liz_off, pos, species, energies, e_idx, delta):
    """ln det M of every instance (principal logarithm: imaginary part in
    (-pi, pi]) and info [n_inst]."""
    liz_off = _c(liz_off, np.int64)
    pos = _c(pos, np.float64)
    species = _c(species, np.int32)
    energies = _c(energies, np.complex128)
    e_idx = _c(e_idx, np.int32)
    delta = _c(delta, np.complex128)
    n = e_idx.shape[0]
    ld = np.zeros(n, np.complex128)
    info = np.zeros(n, np.int32)
    lib().orc_logdet_batch(lmax, n, _ptr(liz_off), _ptr(pos), _ptr(species), _ptr(energies), _ptr(e_idx),
                           _ptr(delta), delta.shape[0], delta.shape[1], _ptr(ld), _ptr(info))
    return ld, info


def logdet_workload(w):
    liz_off, pos, spec = liz_batch(w)
    return logdet_batch(w.lmax, liz_off, pos, spec, w.energies, w.e_idx, w.delta)


# ---------------------------------------------------- energy integration
def contour_integral(values, weights):
    """sum_k w_k f(E_k) over the first axis of `values`: the quadrature of
    the contour integral of f along the energy contour whose nodes and
    weights are given (the energy integral of eq. Density taken on a complex
    contour)."""
    v = np.asarray(values)
    w = np.asarray(weights)
    return np.tensordot(w, v, axes=(0, 0))


def lloyd_ms_idos(logdets):
    """Multiple-scattering part of the integrated density of states along a
    contour, from ln det M at its nodes in contour order: Lloyd's formula
    gives N_ms(E) = -(1/pi) Im ln det M(E) with the branch followed
    continuously from the contour's first node, so N_ms(E_k) - N_ms(E_0) =
    -(phi_k - phi_0)/pi, phi the phase of det M unwrapped node by node (each
    step taken as the principal difference, which assumes the phase moves by
    less than pi between neighbouring nodes)."""
    ph = np.asarray(logdets).imag
    steps = np.angle(np.exp(1j * np.diff(ph)))
    phi = np.concatenate([[0.0], np.cumsum(steps)])
    return -phi / np.pi
