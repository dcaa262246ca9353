"""Writes the stored expected values of oracle runs too long to repeat
inside a GPU test.  Calls only oracle/ and the seeded input generators.

    python tests/golden/make_golden.py c3 2      # 8x8 d=4 chi=128, 2 steps
    python tests/golden/make_golden.py c2 200    # 8x8 d=3 chi=64, 200 steps

Output tests/golden/<config>_oracle_<steps>steps.npz with the oracle's GHZ
fidelity and overlap, per-step norm^2, energy and smallest R_kk of the
gauge moves, the root tensor in full, and for every other node 256 entries
at seeded positions (flat index l + D_L (r + D_R p) of T[l, r, p], the
layout the device library exports).  The node tensors are unique (thin QR
gauge with real positive R_kk), so a device run of the same workload must
reproduce these entries.
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ttn_oracle as O            # noqa: E402
from paper_2210_03763_amd import workload as W  # noqa: E402

SAMPLES_PER_NODE = 256


def path_for(name: str, steps: int) -> str:
    return os.path.join(HERE, f"{name}_oracle_{steps}steps.npz")


def sample_positions(n_nodes: int, sizes, seed: int = 2210037699):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for v in range(n_nodes):
        n = sizes[v]
        k = min(n, SAMPLES_PER_NODE)
        out.append(np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64))
    return out


def make(name: str, steps: int) -> str:
    w = W.config(name).copy(precision=0)
    torch.set_num_threads(os.cpu_count() or 1)
    t0 = time.time()
    st, recs = O.run(w, n_steps=steps)
    F, ov = st.ghz_fidelity(w.target_sites)
    tr = st.tree
    flat = [st.T[v].numpy().transpose(2, 1, 0).reshape(-1) for v in range(tr.n_nodes)]
    pos = sample_positions(tr.n_nodes, [f.size for f in flat])
    arrays = dict(
        workload=np.array(w.name), steps=np.array(steps), command=np.array(
            f"python tests/golden/make_golden.py {name} {steps}"),
        seconds=np.array(time.time() - t0), threads=np.array(torch.get_num_threads()),
        F=np.array(F), overlap=np.array(complex(ov)),
        norm2=np.array([r["norm2"] for r in recs]), energy=np.array([r["energy"] for r in recs]),
        min_r_diag=np.array([r["min_r_diag"] for r in recs]),
        root=flat[tr.root], root_index=np.array(tr.root))
    for v in range(tr.n_nodes):
        arrays[f"idx_{v}"] = pos[v]
        arrays[f"val_{v}"] = flat[v][pos[v]]
    out = path_for(name, steps)
    np.savez_compressed(out, **arrays)
    return out


if __name__ == "__main__":
    name, steps = sys.argv[1], int(sys.argv[2])
    print(make(name, steps), flush=True)
