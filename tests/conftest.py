import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on HIP)")
    config.addinivalue_line("markers", "slow: longer CPU tests")


@pytest.fixture(scope="session")
def hex8():
    from paper_2106_07154_amd.inputs import periodic_hex_mesh
    return periodic_hex_mesh(8, 8, 1.0e4, f0=1.0e-4)


@pytest.fixture(scope="session")
def hex16():
    from paper_2106_07154_amd.inputs import periodic_hex_mesh
    return periodic_hex_mesh(16, 16, 1.0e4, f0=1.0e-4)


@pytest.fixture(scope="session")
def hex64():
    """The 64x64 periodic hexagonal mesh of the inertia-gravity-wave workload."""
    from paper_2106_07154_amd.inputs import periodic_hex_mesh
    return periodic_hex_mesh(64, 64, 1.0e4, f0=1.0e-4)


@pytest.fixture(scope="session")
def irregular():
    """Irregular periodic Voronoi mesh (pentagons/heptagons), random topography."""
    from paper_2106_07154_amd.inputs.voronoi_planar import (
        jittered_hex_points, periodic_voronoi_mesh)
    p, Lx, Ly = jittered_hex_points(16, 16, 1.0e4, 0.6, seed=11)
    m = periodic_voronoi_mesh(p, Lx, Ly, f0=1.0e-4, name="irregular16")
    rng = np.random.default_rng(12)
    m.bottom = 20.0 * rng.standard_normal(m.nCells)
    m.fVertex = 1.0e-4 + 2.0e-5 * rng.standard_normal(m.nVertices)
    return m


@pytest.fixture(scope="session")
def ring_mesh():
    """Periodic Voronoi mesh with one 11-sided cell (a pinned ring of 11
    generators around the domain centre) among hexagons, pentagons and
    heptagons, random topography: cells above 8 edges take the 16-lane
    slot tables of the cell kernels."""
    from paper_2106_07154_amd.inputs.voronoi_planar import (
        periodic_voronoi_mesh, ring_hex_points)
    p, Lx, Ly = ring_hex_points(16, 16, 1.0e4, 11, 1.2, 20)
    m = periodic_voronoi_mesh(p, Lx, Ly, f0=1.0e-4, name="ring11")
    rng = np.random.default_rng(13)
    m.bottom = 20.0 * rng.standard_normal(m.nCells)
    m.fVertex = 1.0e-4 + 2.0e-5 * rng.standard_normal(m.nVertices)
    return m


@pytest.fixture(scope="session")
def lloyd_mesh():
    """Small variable-resolution periodic mesh from the Lloyd generator."""
    from paper_2106_07154_amd.inputs.voronoi_planar import (
        lloyd_step, periodic_voronoi_mesh, sample_points, tanh_spacing)
    L = 4.0e5
    sp = lambda x, y: tanh_spacing(np.hypot(x - L / 2, y - L / 2), 8e3, 3.2e4, 8e4, 2e4)
    p = sample_points(600, L, L, sp, seed=21)
    for _ in range(15):
        p = lloyd_step(p, L, L, lambda x, y: sp(x, y) ** -4.0)
    return periodic_voronoi_mesh(p, L, L, f0=1.0e-4, name="lloyd600")


@pytest.fixture(scope="session")
def sphere_mesh():
    """Small variable-resolution spherical Voronoi mesh (3,000 cells, 20 Lloyd
    iterations, fine cap ratio 4), random topography."""
    from paper_2106_07154_amd.inputs import voronoi_sphere as vs
    P = vs.cap_points(3000, 5, 20)
    m = vs.sphere_voronoi_mesh(vs.morton_sort_sphere(P), name="sphere3000")
    m.bottom = 100.0 * np.random.default_rng(6).standard_normal(m.nCells)
    return m
