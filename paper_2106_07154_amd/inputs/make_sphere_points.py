"""Regenerate the cached relaxed points of the variable-resolution sphere.

    python -m paper_2106_07154_amd.inputs.make_sphere_points

Runs the seeded relaxation of 1.6M points on the sphere (30 Lloyd iterations,
then more until no cell has more than 8 edges; about 15 minutes on one core)
and stores the Morton-ordered points as uint32 fixed-point (longitude,
latitude) in data/.
"""
import os
import time

import numpy as np

from .workloads import DATA, SPH_ITERS, SPH_N, SPH_SEED, _sphere_cache_path, sphere_points


def main(n=SPH_N, seed=SPH_SEED, iters=SPH_ITERS):
    t0 = time.time()
    q = sphere_points(n, seed, iters,
                      progress=lambda it: print(f"lloyd {it + 1} {time.time() - t0:.0f}s", flush=True))
    os.makedirs(DATA, exist_ok=True)
    np.save(_sphere_cache_path(n, seed, iters), q, allow_pickle=False)
    print("wrote", _sphere_cache_path(n, seed, iters), flush=True)


if __name__ == "__main__":
    main()
