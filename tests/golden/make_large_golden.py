"""Writes large_tau00.npz: oracle tau00 of single instances at the paper's
non-canted NiAu rank (N = 6225: lmax = 4 over the 249-atom LIZ of the
large-instance recipe), for the GPU parity test of the whole-GPU elimination,
whose per-test time cannot hold the oracle at this size; with the argument
`canted`, large_canted_tau00.npz: the same at the paper's spin-canted NiAu
rank (2 kk 249 = 12450, canted moments, spin-split wells).  Calls only the
oracle and the input recipes.  Run from the repository root:
    python tests/golden/make_large_golden.py [canted]
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402


def main_canted():
    w = inputs.config_large_canted()
    ni = int(np.flatnonzero(w.atom_species == 0)[0])
    au = int(np.flatnonzero(w.atom_species == 1)[0])
    idx = np.array([ni * 32, au * 32 + 31])
    tau, info = oracle.tau00_spin_workload(inputs.subset(w, idx))
    assert np.all(info == 0), info
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_canted_tau00.npz"),
                        idx=idx, tau=tau)
    print(f"instances {idx.tolist()} done", flush=True)


def main():
    w = inputs.config_large()
    ni = int(np.flatnonzero(w.atom_species == 0)[0])
    au = int(np.flatnonzero(w.atom_species == 1)[0])
    # a Ni centre at the left contour end, an Au centre at the right end
    idx = np.array([ni * 32, au * 32 + 31])
    tau, info = oracle.tau00_workload(inputs.subset(w, idx))
    assert np.all(info == 0), info
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_tau00.npz"), idx=idx,
                        tau=tau)
    print(f"instances {idx.tolist()} done", flush=True)


if __name__ == "__main__":
    main_canted() if sys.argv[1:] == ["canted"] else main()
