"""Regenerate the cached relaxed points of the variable-resolution workload.

    python -m paper_2106_07154_amd.inputs.make_vr_points

Runs the seeded 50-iteration Lloyd relaxation (about two minutes for 200,000
points), sorts the points along a Morton curve and stores them as uint32
fixed-point coordinates in data/.
"""
import os
import sys
import time

import numpy as np

from . import voronoi_planar as vp
from .workloads import DATA, VR_ITERS, VR_N, VR_SEED, _vr_cache_path, quantize


def main(n=VR_N, seed=VR_SEED, iters=VR_ITERS):
    t0 = time.time()
    p = vp.vr_points(n, seed, iters,
                     progress=lambda it: print(f"lloyd {it + 1}/{iters} {time.time() - t0:.0f}s",
                                               flush=True))
    p = vp.morton_sort(p, vp.VR_DOMAIN)
    os.makedirs(DATA, exist_ok=True)
    np.save(_vr_cache_path(n, seed, iters), quantize(p, vp.VR_DOMAIN), allow_pickle=False)
    print("wrote", _vr_cache_path(n, seed, iters))


if __name__ == "__main__":
    main(*[int(a) for a in sys.argv[1:]])
