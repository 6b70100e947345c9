"""Regenerate the cached relaxed points of the three-resolution workload.

    python -m paper_2106_07154_amd.inputs.make_vr3_points

Runs the seeded 30-iteration Lloyd relaxation of 800,000 points, sorts them
along a Morton curve and stores them as uint32 fixed-point coordinates in
data/.
"""
import os
import sys
import time

import numpy as np

from . import voronoi_planar as vp
from .workloads import DATA, VR3_ITERS, VR3_N, VR3_SEED, _vr3_cache_path, quantize


def main(n=VR3_N, seed=VR3_SEED, iters=VR3_ITERS):
    t0 = time.time()
    p = vp.vr3_points(n, seed, iters,
                      progress=lambda it: print(f"lloyd {it + 1}/{iters} {time.time() - t0:.0f}s",
                                                flush=True))
    p = vp.morton_sort(p, vp.VR_DOMAIN)
    os.makedirs(DATA, exist_ok=True)
    np.save(_vr3_cache_path(n, seed, iters), quantize(p, vp.VR_DOMAIN), allow_pickle=False)
    print("wrote", _vr3_cache_path(n, seed, iters))


if __name__ == "__main__":
    main(*[int(a) for a in sys.argv[1:]])
