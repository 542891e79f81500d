"""ctypes binding of liblsms_tau.so with the entry points' own names.

Argument marshalling only: tensors are allocated with torch on the current
CUDA (HIP) device and passed by data pointer together with the current
stream.  There is no fallback: if the library is missing, `lib()` raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsms_tau.so")
_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32


class _Problem(ctypes.Structure):
    _fields_ = [
        ("lmax", ctypes.c_int32),
        ("n_inst", ctypes.c_int32),
        ("n_species", ctypes.c_int32),
        ("n_energy", ctypes.c_int32),
        ("max_liz", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("liz_off", _P),
        ("pos", _P),
        ("species", _P),
        ("energy", _P),
        ("e_idx", _P),
        ("delta", _P),
    ]


class _Spin(ctypes.Structure):
    _fields_ = [("moment", _P), ("delta_dn", _P)]


class Opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("nb", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("max_refine", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("tol", ctypes.c_double),
    ]


PREC_FP64 = 0
PREC_FP32_IR = 1
INFO_FP64_FALLBACK = 1 << 20
INFO_PIVOT_MASK = (1 << 20) - 1
PERSISTENT = 1
GRAPH = 2


SYMBOLS = ("lsms_create", "lsms_destroy", "lsms_build_liz", "build_kkr", "tau00_batched", "tau00_batched_noalloc",
           "lsms_workspace_size", "tau00_solve", "lsms_autotune", "lsms_set_tuned_nb", "lsms_get_tuned_nb",
           "lsms_autotune_save", "lsms_autotune_load",
           "lsms_mlp_features", "lsms_mlp_cast", "lsms_mlp_forward", "lsms_mlp_backward", "lsms_mlp_mse",
           "lsms_mlp_adamw", "lsms_mlp_seed", "lsms_mlp_targets", "lsms_mlp_norm_stats",
           "lsms_gmres_workspace_size", "tau00_gmres", "lsms_row_workspace_size", "tau_row_batched",
           "lsms_contour_sum", "lsms_lloyd_idos", "lsms_liz_moments", "build_kkr_spin", "tau00_spin_batched",
           "lsms_spin_workspace_size", "tau00_spin_solve", "lsms_large_workspace_size", "tau00_large",
           "tau00_gmres_pc", "lsms_site_blocks", "lsms_large_set_spin_limit")

BATCHED_WORK_PER_INST = 2 * 64 * 64 * 16
MLP_PARAMS = 399616
MLP_ACT = 2560
INFO_ROUTED = 1 << 22
INFO_LU_FALLBACK = 1 << 21


def lib():
    """Load liblsms_tau.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2308_16317_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.lsms_create.argtypes = [ctypes.POINTER(_P), ctypes.c_int]
        L.lsms_destroy.argtypes = [_P]
        L.lsms_build_liz.argtypes = [_P, _P, _P, _I32, _P, _P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P]
        L.build_kkr.argtypes = [_P, ctypes.POINTER(_Problem), _P, _P, _P, _P]
        L.tau00_batched.argtypes = [_P, ctypes.POINTER(_Problem), _P, _P, ctypes.POINTER(Opts), _P, _P, _P,
                                    ctypes.c_size_t, _P]
        L.tau00_batched_noalloc.argtypes = [_P, ctypes.POINTER(_Problem), _P, _P, ctypes.POINTER(Opts), _P, _P, _P]
        L.lsms_row_workspace_size.argtypes = [_P, ctypes.POINTER(_Problem), ctypes.POINTER(ctypes.c_size_t)]
        L.tau_row_batched.argtypes = [_P, ctypes.POINTER(_Problem), _P, _P, ctypes.POINTER(Opts), _P, _P, _P, _P, _P,
                                      _P, ctypes.c_size_t, _P]
        PP = ctypes.POINTER(_Problem)
        SP = ctypes.POINTER(_Spin)
        L.lsms_liz_moments.argtypes = [_P, ctypes.c_int64, _P, _P, _I32, _P, _P]
        L.build_kkr_spin.argtypes = [_P, PP, SP, _P, _P, _P, _P]
        L.tau00_spin_batched.argtypes = [_P, PP, SP, _P, _P, ctypes.POINTER(Opts), _P, _P, _P, ctypes.c_size_t, _P]
        L.lsms_spin_workspace_size.argtypes = [_P, PP, SP, ctypes.POINTER(Opts), _I32,
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.tau00_spin_solve.argtypes = [_P, PP, SP, ctypes.POINTER(Opts), _P, _P, _P, ctypes.c_size_t, _P]
        L.lsms_large_workspace_size.argtypes = [_P, PP, SP, ctypes.POINTER(ctypes.c_size_t)]
        L.lsms_large_set_spin_limit.argtypes = [_P, ctypes.c_int64]
        L.tau00_large.argtypes = [_P, PP, SP, _P, ctypes.POINTER(Opts), _P, _P, _P, ctypes.c_size_t, _P]
        L.lsms_contour_sum.argtypes = [_P, _I32, _I32, _I32, _P, _P, _P, _P]
        L.lsms_lloyd_idos.argtypes = [_P, _I32, _I32, _P, _P, _P]
        L.lsms_workspace_size.argtypes = [_P, ctypes.POINTER(_Problem), ctypes.POINTER(Opts), _I32,
                                          ctypes.POINTER(ctypes.c_size_t)]
        L.tau00_solve.argtypes = [_P, ctypes.POINTER(_Problem), ctypes.POINTER(Opts), _P, _P, _P, ctypes.c_size_t,
                                  _P]
        L.lsms_autotune.argtypes = [_P, ctypes.POINTER(_Problem), ctypes.POINTER(Opts), _P, _P, _P,
                                    ctypes.c_size_t, _P, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_double)]
        L.lsms_set_tuned_nb.argtypes = [_P, _I32, _I32, _I32]
        L.lsms_get_tuned_nb.argtypes = [_P, _I32, _I32, ctypes.POINTER(ctypes.c_int32)]
        L.lsms_autotune_save.argtypes = [_P, ctypes.c_char_p]
        L.lsms_autotune_load.argtypes = [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]
        PP = ctypes.POINTER(_Problem)
        L.lsms_mlp_features.argtypes = [_P, PP, ctypes.c_double, _P, _P]
        L.lsms_mlp_cast.argtypes = [_P, _P, _P, _P]
        L.lsms_mlp_forward.argtypes = [_P, _P, _P, _P, _I32, _P, _P, _P]
        L.lsms_mlp_backward.argtypes = [_P, _P, _P, _P, _P, _I32, _P, _P, _P]
        L.lsms_mlp_mse.argtypes = [_P, _P, _P, ctypes.c_int64, _P, _P, _P]
        L.lsms_mlp_adamw.argtypes = [_P, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, _I32, _P]
        L.lsms_mlp_seed.argtypes = [_P, _P, _P, _P, _I32, _P, _P]
        L.lsms_mlp_targets.argtypes = [_P, PP, _P, _P, _P, _P, _P]
        L.lsms_mlp_norm_stats.argtypes = [_P, _P, _I32, _P, _P, _P]
        L.lsms_gmres_workspace_size.argtypes = [_P, PP, _I32, ctypes.POINTER(ctypes.c_size_t)]
        L.tau00_gmres.argtypes = [_P, PP, _P, _I32, _I32, ctypes.c_double, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.tau00_gmres_pc.argtypes = [_P, PP, _P, _P, _P, _P, _I32, _I32, ctypes.c_double, _P, _P, _P, _P,
                                     ctypes.c_size_t, _P]
        L.lsms_site_blocks.argtypes = [_P, PP, _P, _P, _I32, _P, _P, _P]
        for s in SYMBOLS:
            getattr(L, s).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} returned {rc}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(a, dtype):
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


class Handle:
    """lsms_create / lsms_destroy on the current device."""

    def __init__(self, device: int | None = None):
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        _check(lib().lsms_create(ctypes.byref(h), self.device), "lsms_create")
        self._h = h

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h:
            lib().lsms_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Device-resident lsms_problem: ragged LIZs, energies, phase shifts."""

    def __init__(self, lmax, liz_off, pos, species, energy, e_idx, delta, max_liz=None):
        self.lmax = int(lmax)
        self.liz_off = _dev(liz_off, torch.int64)
        self.pos = _dev(pos, torch.float64)
        self.species = _dev(species, torch.int32)
        self.energy = _dev(energy, torch.complex128)
        self.e_idx = _dev(e_idx, torch.int32)
        self.delta = _dev(delta, torch.complex128)
        self.n_inst = int(self.e_idx.shape[0])
        if max_liz is None:
            sizes = (self.liz_off[1:] - self.liz_off[:-1]) if self.n_inst else torch.zeros(1)
            max_liz = int(sizes.max().item()) if self.n_inst else 1
        self.max_liz = int(max_liz)

    @property
    def kk(self):
        return (self.lmax + 1) ** 2

    @property
    def kc(self):
        """Rows per LIZ site: kk, or 2 kk with spin canting."""
        return self.kk * (2 if self.spin is not None else 1)

    spin = None  # SpinData of a spin-canted problem

    def struct(self) -> _Problem:
        return _Problem(self.lmax, self.n_inst, int(self.delta.shape[0]), int(self.delta.shape[1]), self.max_liz, 0,
                        _ptr(self.liz_off), _ptr(self.pos), _ptr(self.species), _ptr(self.energy), _ptr(self.e_idx),
                        _ptr(self.delta))


class SpinData:
    """Device-resident lsms_spin: per-LIZ-row moment directions and the
    phase shifts of the spin antiparallel to the moment."""

    def __init__(self, moment, delta_dn):
        self.moment = _dev(moment, torch.float64)
        self.delta_dn = _dev(delta_dn, torch.complex128)

    def struct(self) -> _Spin:
        return _Spin(_ptr(self.moment), _ptr(self.delta_dn))


def liz_moments(h: Handle, liz_atom: torch.Tensor, atom_moment) -> torch.Tensor:
    """lsms_liz_moments: the moment of each LIZ row from the supercell's."""
    am = _dev(atom_moment, torch.float64)
    n = int(liz_atom.shape[0])
    out = torch.empty((max(n, 1), 3), dtype=torch.float64, device="cuda")
    _check(lib().lsms_liz_moments(h.ptr, n, _ptr(liz_atom), _ptr(am), int(am.shape[0]), _ptr(out), _stream()),
           "lsms_liz_moments")
    return out[:n]


def build_liz(h: Handle, atom_pos, atom_species, box, centre, rc, max_liz: int, with_atoms: bool = False,
              out: dict | None = None):
    """lsms_build_liz: returns dict(liz_n, liz_off, pos, species[, atom]) of device tensors
    (pos/species are the compact rows liz_off[0]..liz_off[n]).  `out`, a dict
    returned by an earlier call with the same sizes, is reused as the output."""
    ap = _dev(atom_pos, torch.float64)
    asp = _dev(atom_species, torch.int32)
    ce = _dev(centre, torch.int32)
    r = _dev(rc, torch.float64)
    n = int(ce.shape[0])
    box_h = (ctypes.c_double * 3)(*[float(b) for b in box])
    if out is None:
        out = dict(
            liz_n=torch.empty(max(n, 1), dtype=torch.int32, device="cuda"),
            liz_off=torch.empty(n + 1, dtype=torch.int64, device="cuda"),
            pos=torch.empty((max(n, 1) * max_liz, 3), dtype=torch.float64, device="cuda"),
            species=torch.empty(max(n, 1) * max_liz, dtype=torch.int32, device="cuda"),
        )
        if with_atoms:
            out["atom"] = torch.empty(max(n, 1) * max_liz, dtype=torch.int32, device="cuda")
    else:
        out = dict(out)
        out["liz_n"] = out["liz_n_buf"]
    _check(lib().lsms_build_liz(h.ptr, _ptr(ap), _ptr(asp), int(ap.shape[0]), box_h, _ptr(ce), _ptr(r), n,
                                int(max_liz), _ptr(out["liz_n"]), _ptr(out["liz_off"]), _ptr(out["pos"]),
                                _ptr(out["species"]), _ptr(out.get("atom")), _stream()), "lsms_build_liz")
    out["liz_n_buf"] = out["liz_n"]
    out["liz_n"] = out["liz_n"][:n]
    return out


def build_kkr(h: Handle, prob: Problem, M: torch.Tensor, m_off: torch.Tensor) -> torch.Tensor:
    """build_kkr into the complex128 buffer M at offsets m_off; returns info (device)."""
    info = torch.empty(max(prob.n_inst, 1), dtype=torch.int32, device="cuda")
    ps = prob.struct()
    _check(lib().build_kkr(h.ptr, ctypes.byref(ps), _ptr(M), _ptr(m_off), _ptr(info), _stream()), "build_kkr")
    return info[:prob.n_inst]


def _tau_view(tau: torch.Tensor, kk: int) -> torch.Tensor:
    # column-major kk x kk per instance -> natural [i, L, L'] indexing
    return tau.view(-1, kk, kk).transpose(1, 2)


def tau00_batched(h: Handle, prob: Problem, M: torch.Tensor, m_off: torch.Tensor, opts: Opts | None = None,
                  tau=None, info=None, work=None):
    """tau00_batched on caller-built M (overwritten); returns (tau00 [n, kk, kk], info).
    `tau` / `info` may be given as contiguous device buffers of n*kk*kk complex128 / n int32;
    `work` (a device byte buffer of n * BATCHED_WORK_PER_INST bytes) allows panels wider than 64."""
    kk = prob.kk
    if tau is None:
        tau = torch.empty(max(prob.n_inst, 1) * kk * kk, dtype=torch.complex128, device="cuda")
    if info is None:
        info = torch.empty(max(prob.n_inst, 1), dtype=torch.int32, device="cuda")
    assert tau.is_contiguous() and info.is_contiguous()
    ps = prob.struct()
    o = opts if opts is not None else Opts()
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(lib().tau00_batched(h.ptr, ctypes.byref(ps), _ptr(M), _ptr(m_off), ctypes.byref(o), _ptr(tau),
                               _ptr(info), _ptr(work), wb, _stream()), "tau00_batched")
    return _tau_view(tau, kk)[:prob.n_inst], info[:prob.n_inst]


def row_workspace_size(h: Handle, prob: Problem) -> int:
    b = ctypes.c_size_t()
    ps = prob.struct()
    _check(lib().lsms_row_workspace_size(h.ptr, ctypes.byref(ps), ctypes.byref(b)), "lsms_row_workspace_size")
    return int(b.value)


def tau_row_batched(h: Handle, prob: Problem, M: torch.Tensor, m_off: torch.Tensor, opts: Opts | None = None,
                    row: bool = True, logdet: bool = True, work=None):
    """tau_row_batched on caller-built M (overwritten).  Returns (rows, row_off, logdet, tau00, info):
    rows a flat complex128 device buffer, instance i's kk x N_i block row at row_off[i] (column-major,
    ld kk) or None; logdet [n] complex128 or None; tau00 [n, kk, kk]; info [n]."""
    kk = prob.kk
    n = prob.n_inst
    nl = (prob.liz_off[1:] - prob.liz_off[:-1]) if n else torch.zeros(0, dtype=torch.int64, device="cuda")
    sizes = kk * kk * nl
    row_off = torch.cumsum(sizes, 0) - sizes if n else torch.zeros(1, dtype=torch.int64, device="cuda")
    total = int(sizes.sum().item()) if n else 0
    rows = torch.empty(max(total, 1), dtype=torch.complex128, device="cuda") if row else None
    ld = torch.empty(max(n, 1), dtype=torch.complex128, device="cuda") if logdet else None
    tau = torch.empty(max(n, 1) * kk * kk, dtype=torch.complex128, device="cuda")
    info = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    if work is None:
        work = torch.empty(max(row_workspace_size(h, prob), 1), dtype=torch.uint8, device="cuda")
    ps = prob.struct()
    o = opts if opts is not None else Opts()
    row_off = row_off.contiguous()
    _check(lib().tau_row_batched(h.ptr, ctypes.byref(ps), _ptr(M), _ptr(m_off), ctypes.byref(o), _ptr(row_off),
                                 _ptr(rows), _ptr(ld), _ptr(tau), _ptr(info), _ptr(work),
                                 work.numel() * work.element_size(), _stream()), "tau_row_batched")
    return rows, row_off[:n], (ld[:n] if ld is not None else None), _tau_view(tau, kk)[:n], info[:n]


def tau00_large(h: Handle, prob: Problem, M: torch.Tensor, opts: Opts | None = None, work=None):
    """tau00_large: one instance (prob.n_inst == 1) across the whole GPU on caller-built M
    (overwritten); returns (tau00 [1, kc, kc], info [1])."""
    kc = prob.kc
    sp = prob.spin.struct() if prob.spin is not None else None
    ps = prob.struct()
    if work is None:
        b = ctypes.c_size_t()
        _check(lib().lsms_large_workspace_size(h.ptr, ctypes.byref(ps), ctypes.byref(sp) if sp else None,
                                               ctypes.byref(b)), "lsms_large_workspace_size")
        work = torch.empty(int(b.value), dtype=torch.uint8, device="cuda")
    tau = torch.empty(kc * kc, dtype=torch.complex128, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    o = opts if opts is not None else Opts()
    _check(lib().tau00_large(h.ptr, ctypes.byref(ps), ctypes.byref(sp) if sp else None, _ptr(M), ctypes.byref(o),
                             _ptr(tau), _ptr(info), _ptr(work), work.numel() * work.element_size(), _stream()),
           "tau00_large")
    return _tau_view(tau, kc), info


def large_set_spin_limit(h: Handle, polls: int):
    """lsms_large_set_spin_limit (0 = default)."""
    _check(lib().lsms_large_set_spin_limit(h.ptr, int(polls)), "lsms_large_set_spin_limit")


def contour_sum(h: Handle, weights, values: torch.Tensor, n_sites: int, n_energy: int) -> torch.Tensor:
    """lsms_contour_sum: values [n_sites * n_energy, ...] complex128 (instance s * n_energy + k);
    returns [n_sites, ...] = sum_k weights[k] values[s, k]."""
    w = _dev(weights, torch.complex128)
    v = values.contiguous()
    m = v.numel() // max(n_sites * n_energy, 1)
    out = torch.empty((max(n_sites, 1),) + tuple(v.shape[1:]), dtype=torch.complex128, device="cuda")
    _check(lib().lsms_contour_sum(h.ptr, n_sites, n_energy, m, _ptr(w), _ptr(v), _ptr(out), _stream()),
           "lsms_contour_sum")
    return out[:n_sites]


def lloyd_idos(h: Handle, logdet: torch.Tensor, n_sites: int, n_energy: int) -> torch.Tensor:
    """lsms_lloyd_idos: logdet [n_sites * n_energy] complex128 in contour order per site;
    returns [n_sites, n_energy] float64."""
    ld = logdet.contiguous()
    out = torch.empty((max(n_sites, 1), n_energy), dtype=torch.float64, device="cuda")
    _check(lib().lsms_lloyd_idos(h.ptr, n_sites, n_energy, _ptr(ld), _ptr(out), _stream()), "lsms_lloyd_idos")
    return out[:n_sites]


def tau00_batched_noalloc(h: Handle, prob: Problem, M: torch.Tensor, m_off: torch.Tensor, opts: Opts | None = None,
                          tau=None, info=None):
    """tau00_batched_noalloc (no workspace, no allocation in the library): as tau00_batched."""
    kk = prob.kk
    if tau is None:
        tau = torch.empty(max(prob.n_inst, 1) * kk * kk, dtype=torch.complex128, device="cuda")
    if info is None:
        info = torch.empty(max(prob.n_inst, 1), dtype=torch.int32, device="cuda")
    assert tau.is_contiguous() and info.is_contiguous()
    ps = prob.struct()
    o = opts if opts is not None else Opts()
    _check(lib().tau00_batched_noalloc(h.ptr, ctypes.byref(ps), _ptr(M), _ptr(m_off), ctypes.byref(o), _ptr(tau),
                                       _ptr(info), _stream()), "tau00_batched_noalloc")
    return _tau_view(tau, kk)[:prob.n_inst], info[:prob.n_inst]


def workspace_size(h: Handle, prob: Problem, chunk: int, opts: Opts | None = None) -> int:
    b = ctypes.c_size_t()
    ps = prob.struct()
    o = opts if opts is not None else Opts()
    _check(lib().lsms_workspace_size(h.ptr, ctypes.byref(ps), ctypes.byref(o), int(chunk), ctypes.byref(b)),
           "lsms_workspace_size")
    return int(b.value)


def tau00_solve(h: Handle, prob: Problem, work: torch.Tensor, opts: Opts | None = None, tau=None, info=None):
    """Fused build + solve in `work` (a device byte buffer); returns (tau00 [n, kk, kk], info)."""
    kk = prob.kk
    if tau is None:
        tau = torch.empty(max(prob.n_inst, 1) * kk * kk, dtype=torch.complex128, device="cuda")
    if info is None:
        info = torch.empty(max(prob.n_inst, 1), dtype=torch.int32, device="cuda")
    ps = prob.struct()
    o = opts if opts is not None else Opts()
    _check(lib().tau00_solve(h.ptr, ctypes.byref(ps), ctypes.byref(o), _ptr(tau), _ptr(info), _ptr(work),
                             work.numel() * work.element_size(), _stream()), "tau00_solve")
    return _tau_view(tau, kk)[:prob.n_inst], info[:prob.n_inst]


def problem_for_workload(h: Handle, w, max_liz: int = 1024) -> Problem:
    """Upload a workload's inputs (supercell, centres, cutoffs, energies, phase
    shifts) and extract every instance's LIZ with lsms_build_liz.  The
    problem's max_liz is the largest LIZ found (one device-to-host read).  A
    spin-canted workload also gets its per-row moments (lsms_liz_moments) and
    down-spin phase shifts in prob.spin."""
    spin = getattr(w, "atom_moment", None) is not None
    liz = build_liz(h, w.atom_pos, w.atom_species, w.box, w.centre, w.rc, max_liz, with_atoms=spin)
    n_max = int(liz["liz_n"].max().item()) if w.centre.shape[0] else 1
    if n_max > max_liz:
        raise RuntimeError(f"a LIZ has {n_max} sites, above max_liz={max_liz}")
    prob = Problem(w.lmax, liz["liz_off"], liz["pos"], liz["species"], w.energies, w.e_idx, w.delta,
                   max_liz=n_max)
    if spin:
        rows = int(liz["liz_off"][-1].item()) if w.centre.shape[0] else 0
        prob.spin = SpinData(liz_moments(h, liz["atom"][:rows], w.atom_moment), w.delta_dn)
    return prob


def build_kkr_spin(h: Handle, prob: Problem, M: torch.Tensor, m_off: torch.Tensor) -> torch.Tensor:
    """build_kkr_spin into M at offsets m_off; returns info (device)."""
    info = torch.empty(max(prob.n_inst, 1), dtype=torch.int32, device="cuda")
    ps, sp = prob.struct(), prob.spin.struct()
    _check(lib().build_kkr_spin(h.ptr, ctypes.byref(ps), ctypes.byref(sp), _ptr(M), _ptr(m_off), _ptr(info),
                                _stream()), "build_kkr_spin")
    return info[:prob.n_inst]


def tau00_spin_batched(h: Handle, prob: Problem, M: torch.Tensor, m_off: torch.Tensor, opts: Opts | None = None,
                       work=None):
    """tau00_spin_batched on caller-built M (overwritten): (tau00 [n, kc, kc], info)."""
    kc = prob.kc
    tau = torch.empty(max(prob.n_inst, 1) * kc * kc, dtype=torch.complex128, device="cuda")
    info = torch.empty(max(prob.n_inst, 1), dtype=torch.int32, device="cuda")
    ps, sp = prob.struct(), prob.spin.struct()
    o = opts if opts is not None else Opts()
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(lib().tau00_spin_batched(h.ptr, ctypes.byref(ps), ctypes.byref(sp), _ptr(M), _ptr(m_off),
                                    ctypes.byref(o), _ptr(tau), _ptr(info), _ptr(work), wb, _stream()),
           "tau00_spin_batched")
    return _tau_view(tau, kc)[:prob.n_inst], info[:prob.n_inst]


def spin_workspace_size(h: Handle, prob: Problem, chunk: int, opts: Opts | None = None) -> int:
    b = ctypes.c_size_t()
    ps, sp = prob.struct(), prob.spin.struct()
    o = opts if opts is not None else Opts()
    _check(lib().lsms_spin_workspace_size(h.ptr, ctypes.byref(ps), ctypes.byref(sp), ctypes.byref(o), int(chunk),
                                          ctypes.byref(b)), "lsms_spin_workspace_size")
    return int(b.value)


def tau00_spin_solve(h: Handle, prob: Problem, work: torch.Tensor, opts: Opts | None = None, tau=None, info=None):
    """Fused spin-canted build + solve in `work`: (tau00 [n, kc, kc], info)."""
    kc = prob.kc
    if tau is None:
        tau = torch.empty(max(prob.n_inst, 1) * kc * kc, dtype=torch.complex128, device="cuda")
    if info is None:
        info = torch.empty(max(prob.n_inst, 1), dtype=torch.int32, device="cuda")
    ps, sp = prob.struct(), prob.spin.struct()
    o = opts if opts is not None else Opts()
    _check(lib().tau00_spin_solve(h.ptr, ctypes.byref(ps), ctypes.byref(sp), ctypes.byref(o), _ptr(tau), _ptr(info),
                                  _ptr(work), work.numel() * work.element_size(), _stream()), "tau00_spin_solve")
    return _tau_view(tau, kc)[:prob.n_inst], info[:prob.n_inst]


def autotune(h: Handle, prob: Problem, work: torch.Tensor, opts: Opts | None = None):
    """lsms_autotune: returns (best panel width, {nb: ms}) and stores it in the handle."""
    kk = prob.kk
    tau = torch.empty(max(prob.n_inst, 1) * kk * kk, dtype=torch.complex128, device="cuda")
    info = torch.empty(max(prob.n_inst, 1), dtype=torch.int32, device="cuda")
    ps = prob.struct()
    o = opts if opts is not None else Opts()
    best = ctypes.c_int32()
    ms = (ctypes.c_double * 4)()
    _check(lib().lsms_autotune(h.ptr, ctypes.byref(ps), ctypes.byref(o), _ptr(tau), _ptr(info), _ptr(work),
                               work.numel() * work.element_size(), _stream(), ctypes.byref(best), ms),
           "lsms_autotune")
    return int(best.value), dict(zip((32, 64, 96, 128), list(ms)))


def set_tuned_nb(h: Handle, n: int, nb: int, precision: int = PREC_FP64):
    _check(lib().lsms_set_tuned_nb(h.ptr, int(n), int(precision), int(nb)), "lsms_set_tuned_nb")


def get_tuned_nb(h: Handle, n: int, precision: int = PREC_FP64) -> int:
    nb = ctypes.c_int32()
    _check(lib().lsms_get_tuned_nb(h.ptr, int(n), int(precision), ctypes.byref(nb)), "lsms_get_tuned_nb")
    return int(nb.value)


def autotune_save(h: Handle, path: str):
    _check(lib().lsms_autotune_save(h.ptr, os.fsencode(path)), "lsms_autotune_save")


def autotune_load(h: Handle, path: str) -> int:
    n = ctypes.c_int32()
    _check(lib().lsms_autotune_load(h.ptr, os.fsencode(path), ctypes.byref(n)), "lsms_autotune_load")
    return int(n.value)


# ------------------------------------------------------------ learned form

def mlp_features(h: Handle, prob: Problem, a_lat: float) -> torch.Tensor:
    """lsms_mlp_features: [n_inst, 18] float32 features on the device."""
    feat = torch.empty((max(prob.n_inst, 1), 18), dtype=torch.float32, device="cuda")
    ps = prob.struct()
    _check(lib().lsms_mlp_features(h.ptr, ctypes.byref(ps), float(a_lat), _ptr(feat), _stream()),
           "lsms_mlp_features")
    return feat[:prob.n_inst]


def mlp_cast(h: Handle, params: torch.Tensor, w_bf16: torch.Tensor):
    _check(lib().lsms_mlp_cast(h.ptr, _ptr(params), _ptr(w_bf16), _stream()), "lsms_mlp_cast")


def mlp_forward(h: Handle, params: torch.Tensor, w_bf16: torch.Tensor, feat: torch.Tensor, act=None, out=None):
    """lsms_mlp_forward: returns (out [n, 1024], act [n, MLP_ACT])."""
    n = feat.shape[0]
    if act is None:
        act = torch.empty((max(n, 1), MLP_ACT), dtype=torch.float32, device="cuda")
    if out is None:
        out = torch.empty((max(n, 1), 1024), dtype=torch.float32, device="cuda")
    _check(lib().lsms_mlp_forward(h.ptr, _ptr(params), _ptr(w_bf16), _ptr(feat), int(n), _ptr(out), _ptr(act),
                                  _stream()), "lsms_mlp_forward")
    return out[:n], act[:n]


def mlp_backward(h: Handle, w_bf16: torch.Tensor, feat: torch.Tensor, act: torch.Tensor, dout: torch.Tensor,
                 grad=None, work=None) -> torch.Tensor:
    n = feat.shape[0]
    if grad is None:
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    if work is None:
        work = torch.empty((n, 1280), dtype=torch.float32, device="cuda")
    _check(lib().lsms_mlp_backward(h.ptr, _ptr(w_bf16), _ptr(feat), _ptr(act), _ptr(dout), int(n), _ptr(grad),
                                   _ptr(work), _stream()), "lsms_mlp_backward")
    return grad


def mlp_mse(h: Handle, out: torch.Tensor, target: torch.Tensor, dout=None, loss=None):
    """lsms_mlp_mse: returns (dout, loss (device scalar))."""
    if dout is None:
        dout = torch.empty_like(out)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().lsms_mlp_mse(h.ptr, _ptr(out), _ptr(target), int(out.numel()), _ptr(dout), _ptr(loss), _stream()),
           "lsms_mlp_mse")
    return dout, loss


def mlp_adamw(h: Handle, params, w_bf16, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
    _check(lib().lsms_mlp_adamw(h.ptr, _ptr(params), _ptr(w_bf16), _ptr(m), _ptr(v), _ptr(grad), float(lr),
                                float(beta1), float(beta2), float(eps), float(wd), int(step), _stream()),
           "lsms_mlp_adamw")


def mlp_targets(h: Handle, prob: Problem, tau: torch.Tensor, scale=None, shift=None, out=None) -> torch.Tensor:
    """lsms_mlp_targets: [n_inst, 1024] float32 ([tau00 | [M^-1]_00], optionally normalised)."""
    if out is None:
        out = torch.empty((max(prob.n_inst, 1), 1024), dtype=torch.float32, device="cuda")
    ps = prob.struct()
    _check(lib().lsms_mlp_targets(h.ptr, ctypes.byref(ps), _ptr(tau), _ptr(scale), _ptr(shift), _ptr(out),
                                  _stream()), "lsms_mlp_targets")
    return out[:prob.n_inst]


def mlp_norm_stats(h: Handle, target: torch.Tensor):
    scale = torch.empty(1024, dtype=torch.float32, device="cuda")
    shift = torch.empty(1024, dtype=torch.float32, device="cuda")
    _check(lib().lsms_mlp_norm_stats(h.ptr, _ptr(target), int(target.shape[0]), _ptr(scale), _ptr(shift),
                                     _stream()), "lsms_mlp_norm_stats")
    return scale, shift


def mlp_seed(h: Handle, out: torch.Tensor, scale: torch.Tensor, shift: torch.Tensor) -> torch.Tensor:
    """lsms_mlp_seed: [n, 256] complex128 seeds (column-major 16 x 16 each)."""
    n = out.shape[0]
    seed = torch.empty((max(n, 1), 256), dtype=torch.complex128, device="cuda")
    _check(lib().lsms_mlp_seed(h.ptr, _ptr(out), _ptr(scale), _ptr(shift), int(n), _ptr(seed), _stream()),
           "lsms_mlp_seed")
    return seed[:n]


def gmres_workspace_size(h: Handle, prob: Problem, restart: int) -> int:
    b = ctypes.c_size_t()
    ps = prob.struct()
    _check(lib().lsms_gmres_workspace_size(h.ptr, ctypes.byref(ps), int(restart), ctypes.byref(b)),
           "lsms_gmres_workspace_size")
    return int(b.value)


def tau00_gmres(h: Handle, prob: Problem, work: torch.Tensor, seed=None, restart: int = 8, max_cycles: int = 8,
                tol: float = 1e-12, tau=None, info=None, steps=None, precond=None, precond_row=None, route=None):
    """tau00_gmres (tau00_gmres_pc when precond / route are given): returns (tau00 [n, 16, 16], info, steps)."""
    n = max(prob.n_inst, 1)
    if tau is None:
        tau = torch.empty(n * 256, dtype=torch.complex128, device="cuda")
    if info is None:
        info = torch.empty(n, dtype=torch.int32, device="cuda")
    if steps is None:
        steps = torch.empty(n, dtype=torch.int32, device="cuda")
    ps = prob.struct()
    if precond is None and route is None:
        _check(lib().tau00_gmres(h.ptr, ctypes.byref(ps), _ptr(seed), int(restart), int(max_cycles), float(tol),
                                 _ptr(tau), _ptr(info), _ptr(steps), _ptr(work), work.numel() * work.element_size(),
                                 _stream()), "tau00_gmres")
    else:
        _check(lib().tau00_gmres_pc(h.ptr, ctypes.byref(ps), _ptr(seed), _ptr(precond), _ptr(precond_row),
                                    _ptr(route), int(restart), int(max_cycles), float(tol), _ptr(tau), _ptr(info),
                                    _ptr(steps), _ptr(work), work.numel() * work.element_size(), _stream()),
               "tau00_gmres_pc")
    return _tau_view(tau, 16)[:prob.n_inst], info[:prob.n_inst], steps[:prob.n_inst]


def site_blocks(h: Handle, prob: Problem, liz_atom: torch.Tensor, centre, n_atoms: int) -> torch.Tensor:
    """lsms_site_blocks: preconditioner block index of every LIZ row (device int32)."""
    ce = _dev(centre, torch.int32)
    rows = int(prob.liz_off[-1].item()) if prob.n_inst else 0
    out = torch.empty(max(rows, 1), dtype=torch.int32, device="cuda")
    work = torch.empty(max(n_atoms * int(prob.energy.shape[0]), 1), dtype=torch.int32, device="cuda")
    ps = prob.struct()
    _check(lib().lsms_site_blocks(h.ptr, ctypes.byref(ps), _ptr(liz_atom), _ptr(ce), int(n_atoms), _ptr(out),
                                  _ptr(work), _stream()), "lsms_site_blocks")
    return out[:rows]
