"""Write the oracle's potentials at sampled points of the batching workload.

Calls only the oracle and the seeded input generators. The workload is the 24
independent surface point sets of ``workloads.batch_sets(24)`` (sphere, cube
surface, torus; N log-uniform in [2^12, 2^19]) at p = 6, eps = 1e-6, leaf 64,
with the density ``workloads.uniform_density(N_i, 100 + i)`` on set i, plus 16
right-hand sides ``workloads.uniform_density(N, 7, nrhs=16)`` on the largest
set. For each set it writes 256 seeded sample indices (all points when a set
has fewer) and the FP64 dense-M2L KIFMM potential there; for the largest set
also the 256 x 16 potentials of the 16 right-hand sides.
Output: tests/golden/batch_samples.json.

    python tests/golden/make_batch_samples.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import workloads  # noqa: E402

P, EPS, LEAF, NSAMPLE, NRHS = 6, 1e-6, 64, 256, 16
SEED = workloads.SEED_BASE + 3


def main():
    t0 = time.time()
    sets = workloads.batch_sets(24)
    big = max(range(len(sets)), key=lambda i: sets[i][0].shape[0])
    out = {"p": P, "eps": EPS, "leaf_size": LEAF, "count": len(sets), "big": big, "nrhs": NRHS, "sets": []}
    ops = oracle.build_operators(P, EPS, LEAF, mode="dense")
    for i, (x, name) in enumerate(sets):
        n = x.shape[0]
        rng = np.random.default_rng(SEED + 300 + i)
        sample = np.sort(rng.choice(n, min(NSAMPLE, n), replace=False))
        sig = workloads.uniform_density(n, 100 + i)
        tree = oracle.build_tree(x, LEAF)
        if i == big:
            S = np.concatenate([sig[:, None], workloads.uniform_density(n, 7, nrhs=NRHS)], axis=1)
            phi, _ = oracle.fmm(x, S, P, EPS, LEAF, mode="dense", tree=tree, ops=ops, sample=sample)
            rec = {"phi_dense": phi[:, 0].tolist(), "phi_rhs": phi[:, 1:].tolist()}
        else:
            phi, _ = oracle.fmm(x, sig, P, EPS, LEAF, mode="dense", tree=tree, ops=ops, sample=sample)
            rec = {"phi_dense": phi.tolist()}
        rec.update({"n": n, "name": name, "depth": tree.depth, "sample": sample.tolist()})
        out["sets"].append(rec)
        print(f"set {i} {name} N={n} depth {tree.depth} done {time.time() - t0:.1f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, round(time.time() - t0, 1), "s")


if __name__ == "__main__":
    main()
