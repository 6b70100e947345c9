"""Cache the relaxed points of the ensemble members listed in ENS_CACHED.

    python -m paper_2106_07154_amd.inputs.make_ensemble_points

Runs each member's seeded Lloyd relaxation (member_points) and stores the
Morton-sorted points as uint32 fixed-point coordinates in data/, followed by
one row holding the number of Lloyd iterations taken.  The members are then
rebuilt from the stored points on every run, so a test can use them without
repeating the relaxation.
"""
import os
import time

import numpy as np

from . import voronoi_planar as vp
from .workloads import (DATA, ENS_CACHED, ENS_SEED, _member_cache_path, ensemble_sizes,
                        member_points, quantize)


def main(members=ENS_CACHED, iters=10, seed=ENS_SEED):
    sizes = ensemble_sizes(64, seed=seed)
    os.makedirs(DATA, exist_ok=True)
    for j in members:
        t0 = time.time()
        p, done = member_points(j, int(sizes[j]), iters, seed)
        q = quantize(p, vp.VR_DOMAIN)
        q = np.concatenate([q, np.array([[done, 0]], np.uint32)])
        path = _member_cache_path(j, int(sizes[j]), iters, seed)
        np.save(path, q, allow_pickle=False)
        print(f"member {j}: {len(p)} points, {done} Lloyd iterations, "
              f"{time.time() - t0:.0f}s -> {path}", flush=True)


if __name__ == "__main__":
    main()
