"""Regenerate the cached relaxed points of the variable-resolution sphere.

    python -m paper_2106_07154_amd.inputs.make_sphere_points

Runs the seeded 30-iteration Lloyd relaxation of 1.6M points on the sphere
(about 15 minutes on one core), sorts the points along a 3-D Morton curve and
stores them as uint32 fixed-point (longitude, latitude) in data/.
"""
import os
import time

import numpy as np

from . import voronoi_sphere as vs
from .workloads import DATA, SPH_ITERS, SPH_N, SPH_SEED, _sphere_cache_path


def main(n=SPH_N, seed=SPH_SEED, iters=SPH_ITERS):
    t0 = time.time()
    p = vs.cap_points(n, seed, iters,
                      progress=lambda it: print(f"lloyd {it + 1}/{iters} {time.time() - t0:.0f}s",
                                                flush=True))
    p = vs.morton_sort_sphere(p)
    os.makedirs(DATA, exist_ok=True)
    np.save(_sphere_cache_path(n, seed, iters), vs.quantize_lonlat(p), allow_pickle=False)
    print("wrote", _sphere_cache_path(n, seed, iters), flush=True)


if __name__ == "__main__":
    main()
