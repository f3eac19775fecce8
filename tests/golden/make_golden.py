"""Write the stored oracle trajectories the GPU parity tests hold the library to.

Every value written here comes from the CPU oracle (``oracle/``) run on the
seeded synthetic workloads of ``workloads.py``; nothing is read from the HIP
library.  The files are NumPy archives (no pickled objects):

* ``five_level_tree_fp64_400.npz`` -- the five-level vibronic tree (four Ohmic
  chains of 40 sites, d = D = 20, dt = 0.5 fs, seed 2), all 400 second-order
  TDVP steps: the root reduced density matrix, norm, energy and chain-head
  occupations at t_k = k dt, k = 0..400.
* ``ensemble_subset_fp64_100.npz`` -- instances 0..15 of the 256-tree
  spin-boson ensemble (seed 3), each at its drawn size, all 100 steps, the
  same records per instance.

What the trajectories are (the one-site projector-splitting TDVP of a TTNS,
Lanczos local exponentials, guarded QR) follows the paper's section "TTNS for
vibronic quantum dynamics" and its Methods ("Tensor Network States"); the
oracle's own docstrings cite the passages step by step.

    python tests/golden/make_golden.py five_level   # about 2 h on 8 cores
    python tests/golden/make_golden.py ensemble     # about 40 min on 1 core
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.model import boson_ops, build_tree  # noqa: E402
from oracle.ttns import TTNS  # noqa: E402

ENSEMBLE_SUBSET = 16


def trajectory(model, steps, label):
    """Records of the oracle run at t = 0 .. steps*dt (progress on stderr)."""
    tt = TTNS(build_tree(model), krylov=model.get("krylov", 12))
    heads = tt.tree.heads
    nums = [boson_ops(model["chains"][i]["d"])[2] for i in range(len(heads))]
    rdm, norm, energy, occ = [], [], [], []

    def rec():
        rdm.append(tt.rdm())
        norm.append(tt.norm2())
        energy.append(tt.energy())
        occ.append([tt.local_expectation(h, nums[i]).real for i, h in enumerate(heads)])

    rec()
    t0 = time.perf_counter()
    for k in range(steps):
        tt.step(model["dt"])
        rec()
        if (k + 1) % 10 == 0 or k + 1 == steps:
            print("%s: %d/%d steps, %.0f s" % (label, k + 1, steps, time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    return (np.array(rdm), np.array(norm), np.array(energy), np.array(occ),
            np.array([tt.stats["guarded"], tt.stats["breakdown"]]))


def five_level():
    m = W.vibronic_reference()
    rdm, norm, energy, occ, stats = trajectory(m, m["steps"], "five-level tree")
    out = os.path.join(HERE, "five_level_tree_fp64_400.npz")
    np.savez_compressed(out, rdm=rdm, norm=norm, energy=energy, occ=occ, stats=stats,
                        dt=m["dt"], steps=m["steps"], seed=m["seed"])
    print(out)


def ensemble():
    models = W.ensemble()[:ENSEMBLE_SUBSET]
    cols = {"rdm": [], "norm": [], "energy": [], "occ": [], "stats": []}
    for i, m in enumerate(models):
        r = trajectory(m, m["steps"], "ensemble instance %d" % i)
        for k, v in zip(("rdm", "norm", "energy", "occ", "stats"), r):
            cols[k].append(v)
    out = os.path.join(HERE, "ensemble_subset_fp64_100.npz")
    np.savez_compressed(out, **{k: np.array(v) for k, v in cols.items()},
                        instances=np.arange(ENSEMBLE_SUBSET), dt=models[0]["dt"],
                        steps=models[0]["steps"])
    print(out)


if __name__ == "__main__":
    {"five_level": five_level, "ensemble": ensemble}[sys.argv[1]]()
