"""Write the oracle's potentials at sampled points of the p = 8 precision workloads.

Calls only the oracle and the seeded input generators. For each of the two
2**20-point surfaces - the icosphere centroids of the benchmark and the same
construction with vertices scaled by (2, 1, 0.5) - it writes the sample
indices, the FP64 dense-M2L KIFMM potential (p=8, eps=1e-8, leaf 64) and the
direct sum at 256 seeded sample points, for the density 1 + 0.5 Y_2^0 +
N(0, 0.01) of the polar angle. Output: tests/golden/p8_samples.json.

    python tests/golden/make_p8_samples.py
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

N, P, EPS, LEAF, NSAMPLE = 1 << 20, 8, 1e-8, 64, 256
SEED = workloads.SEED_BASE + 2


def main():
    t0 = time.time()
    out = {"n": N, "p": P, "eps": EPS, "leaf_size": LEAF, "seed": SEED}
    for name, gen in (("sphere", workloads.sphere_points), ("ellipsoid", workloads.ellipsoid_points)):
        x = gen(N, SEED)
        sig = workloads.sphere_density(x, SEED + 100)
        sample = np.sort(np.random.default_rng(SEED + 200).choice(N, NSAMPLE, replace=False))
        tree = oracle.build_tree(x, LEAF)
        phi, info = oracle.fmm(x, sig, P, EPS, LEAF, mode="dense", tree=tree, sample=sample)
        print(name, "dense done", round(time.time() - t0, 1), "s", flush=True)
        out[name] = {"depth": tree.depth, "sample": sample.tolist(), "phi_dense": phi.tolist(),
                     "phi_direct": oracle.direct(x, sig, targets=x[sample]).tolist()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "p8_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, round(time.time() - t0, 1), "s")


if __name__ == "__main__":
    main()
