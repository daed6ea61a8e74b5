"""Write the oracle's potentials at sampled points of the 2**20-point sphere.

Calls only the oracle and the seeded input generators. Output:
tests/golden/sphere1m_p6_samples.json with the sample indices and the FP64
dense-M2L and SVD-M2L KIFMM potentials (p=6, eps=1e-6, leaf 64) and the direct
sum at those points (density 1 + 0.5 Y_2^0 + N(0, 0.01)).

    python tests/golden/make_sphere_samples.py
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

N, P, EPS, LEAF, SEED, NSAMPLE = 1 << 20, 6, 1e-6, 64, workloads.SEED_BASE + 1, 256


def main():
    t0 = time.time()
    x = workloads.sphere_points(N, SEED)
    sig = workloads.sphere_density(x, SEED + 100)
    sample = np.sort(np.random.default_rng(SEED + 200).choice(N, NSAMPLE, replace=False))
    tree = oracle.build_tree(x, LEAF)
    out = {"n": N, "p": P, "eps": EPS, "leaf_size": LEAF, "seed": SEED, "depth": tree.depth,
           "sample": sample.tolist()}
    for mode in ("dense", "svd"):
        phi, info = oracle.fmm(x, sig, P, EPS, LEAF, mode=mode, tree=tree, sample=sample)
        out[f"phi_{mode}"] = phi.tolist()
        out[f"k_{mode}"] = info["ops"].k
        print(mode, "done", round(time.time() - t0, 1), "s", flush=True)
    out["phi_direct"] = oracle.direct(x, sig, targets=x[sample]).tolist()
    # the direct sum skips exact self pairs only through r == 0
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere1m_p6_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, round(time.time() - t0, 1), "s")


if __name__ == "__main__":
    main()
