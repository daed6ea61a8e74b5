"""Write the closed-form charge density of the ellipsoid conductor at sampled
triangle centroids of the BEM meshes.

Calls only the oracle (oracle.bem.conductor_density / conductor_charge: the
closed form of the conductor (2, 1, 3) held at potential 1, Sec. 5.1) and the
seeded mesh generator. For the meshes of 131,072 and 2,097,152 triangles (the
octahedron refined 7 and 9 times) it stores 2048 seeded sample indices, the
density at their centroids and the total charge. Output:
tests/golden/conductor_samples.json.

    python tests/golden/make_conductor_samples.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import workloads  # noqa: E402
from oracle import bem  # noqa: E402

AXES = (2.0, 1.0, 3.0)
NSAMPLE = 2048
SEED = workloads.SEED_BASE + 20


def main():
    out = {"axes": AXES, "potential": 1.0, "charge": bem.conductor_charge(AXES), "levels": {}}
    for level in (7, 9):
        V, F = workloads.ellipsoid_surface_mesh(level, AXES)
        c, _, _ = bem.geometry(V, F)
        idx = np.sort(np.random.default_rng(SEED + level).choice(F.shape[0], NSAMPLE, replace=False))
        out["levels"][str(level)] = {"n": int(F.shape[0]), "sample": idx.tolist(),
                                     "density": bem.conductor_density(c[idx], AXES).tolist()}
        print(level, F.shape[0], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "conductor_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
