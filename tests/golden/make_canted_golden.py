"""Writes canted_tau00.npz: oracle spin-canted tau00 of a few full-size
instances (rank 4320 at lmax = 3 and 6750 at lmax = 4, the 135-atom LIZ of the
spin-canted recipe), for the GPU parity tests, whose per-test time cannot
hold the oracle at these sizes.  Calls only the oracle and the input
recipes.  Run from the repository root:  python tests/golden/make_canted_golden.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402


def instances(w):
    """A Ni and an Au centre at both contour ends (index site * 32 + energy)."""
    ni = int(np.flatnonzero(w.atom_species == 0)[0])
    au = int(np.flatnonzero(w.atom_species == 1)[0])
    return np.array([ni * 32, au * 32 + 31, au * 32, ni * 32 + 31])


def main():
    out = {}
    for lmax, n in ((3, 4), (4, 2)):
        w = inputs.config_canted(lmax=lmax)
        idx = instances(w)[:n]
        tau, info = oracle.tau00_spin_workload(inputs.subset(w, idx))
        assert np.all(info == 0), info
        out[f"idx_l{lmax}"] = idx
        out[f"tau_l{lmax}"] = tau
        print(f"lmax={lmax}: instances {idx.tolist()} done", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "canted_tau00.npz"), **out)


if __name__ == "__main__":
    main()
