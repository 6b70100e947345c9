"""Host checks of the library's multi-level planning (lts_plan_levels, no
GPU): every level's labels in device order form the contiguous class ranges
the passes rely on, each pass's kernel ranges cover its targets, and every
value a pass reads is one that holds a valid stage value when it runs
(Steps 2 and 4 of each level read only its underlined F, interface and
coarse parts; a leaf Step 3 reads nothing outside its level's domain)."""
import numpy as np
import pytest

import oracle as om
from oracle import Oracle
from paper_2106_07154_amd import lts
from paper_2106_07154_amd.inputs import periodic_hex_mesh, strip_fine_mask
from paper_2106_07154_amd.inputs.cases import disk_fine_mask


@pytest.fixture(scope="module")
def lib():
    from paper_2106_07154_amd.build import stale, build_lib
    if stale():
        build_lib()
    return lts.load_library()


def _cases():
    out = []
    m = periodic_hex_mesh(32, 32, 20e3, f0=1e-4)
    out.append((m, [strip_fine_mask(m, 6, 25, 20e3), strip_fine_mask(m, 14, 17, 20e3)]))
    m = periodic_hex_mesh(48, 48, 20e3, f0=1e-4)
    out.append((m, [strip_fine_mask(m, 6, 41, 20e3), strip_fine_mask(m, 14, 33, 20e3),
                    strip_fine_mask(m, 22, 25, 20e3)]))
    from paper_2106_07154_amd.inputs.voronoi_planar import (jittered_hex_points,
                                                            periodic_voronoi_mesh)
    p, Lx, Ly = jittered_hex_points(32, 32, 1.0e4, 0.55, seed=58)
    m = periodic_voronoi_mesh(p, Lx, Ly, f0=1.0e-4, name="irregular32")
    cx, cy = m.Lx / 2, m.Ly / 2
    out.append((m, [disk_fine_mask(m, cx, cy, 1.2e5), disk_fine_mask(m, cx + 1e4, cy, 2.5e4)]))
    return out


def _reads(m, cells, verts):
    rc, re_ = set(), set()
    for i in cells:
        n = m.nEdgesOnCell[i]
        rc.add(i)
        rc.update(m.cellsOnCell[i, :n].tolist())
        re_.update(m.edgesOnCell[i, :n].tolist())
    for v in verts:
        rc.update(m.cellsOnVertex[v].tolist())
        re_.update(m.edgesOnVertex[v].tolist())
    return rc, re_


@pytest.mark.parametrize("k", range(3))
def test_level_classes_and_pass_reads(lib, k):
    m, masks = _cases()[k]
    P = lts.plan_levels(m, masks, 2, 2)
    R = Oracle(m).ml_regions(masks, 2, 2)
    co, eo, vo = P["cell_order"], P["edge_order"], P["vertex_order"]
    assert sorted(co) == list(range(m.nCells)) and sorted(eo) == list(range(m.nEdges))
    assert sorted(vo) == list(range(m.nVertices))
    cpos = np.empty(m.nCells, np.int64)
    cpos[co] = np.arange(m.nCells)
    epos = np.empty(m.nEdges, np.int64)
    epos[eo] = np.arange(m.nEdges)
    nl = len(masks)
    for l in range(nl):
        L = P["levels"][l]
        cb, eb = L["cell_class_start"], L["edge_class_start"]
        creg, ereg = R.cell[l][co], R.edge[l][eo]
        cfb, efb = R.cell_fbar[l][co], R.edge_fbar[l][eo]
        # the level's domain: everything (level 0) or the enclosing fine region
        if l == 0:
            assert cb[7] == m.nCells and eb[5] == m.nEdges
        else:
            O = P["levels"][l - 1]
            assert cb[7] == O["cell_class_start"][3] and eb[5] == O["edge_class_start"][2]
            assert (R.cell[l - 1][co][:cb[7]] == om.F).all()
            assert (R.edge[l - 1][eo][:eb[5]] == om.F).all()
        assert (creg[:cb[3]] == om.F).all() and (creg[cb[3]:cb[4]] == om.I1).all()
        assert (creg[cb[4]:cb[5]] == om.I2).all() and (creg[cb[5]:cb[7]] == om.C).all()
        assert (cfb[cb[1]:cb[3]] == 1).all() and (cfb[:cb[1]] == 0).all()
        assert (ereg[:eb[2]] == om.F).all() and (ereg[eb[2]:eb[3]] == om.I1).all()
        assert (ereg[eb[3]:eb[4]] == om.I2).all() and (ereg[eb[4]:eb[5]] == om.C).all()
        assert (efb[eb[1]:eb[2]] == 1).all() and (efb[:eb[1]] == 0).all()
        # interface and coarse parts are non-empty at every level
        assert 0 <= cb[1] <= cb[3] < cb[4] < cb[5] < cb[7]
        # valid stage values per pass: (min cell pos, min edge pos, max+1 cell, max+1 edge)
        leaf = l == nl - 1
        valid = {"step1": (0, 0, m.nCells, m.nEdges),
                 "step2": (cb[1], eb[1], m.nCells, m.nEdges),
                 "step4": (cb[4], eb[3], m.nCells, m.nEdges),
                 "step3": (0, 0, cb[7], eb[5])}
        for name, pp in L["passes"].items():
            if name == "step3" and not leaf:
                continue
            tc = co[pp["ct_lo"]:pp["ct_hi"]]
            te = eo[pp["et_lo"]:pp["et_hi"]]
            cover = co[pp["c_lo"]:pp["c_hi"]]
            verts = vo[pp["v_lo"]:pp["v_hi"]]
            need = set(tc.tolist()) | set(m.cellsOnEdge[te].reshape(-1).tolist())
            assert need <= set(cover.tolist()), (l, name)
            needv = set()
            for i in cover:
                needv.update(m.verticesOnCell[i, :m.nEdgesOnCell[i]].tolist())
            assert needv <= set(verts.tolist()), (l, name)
            rc, re_ = _reads(m, cover, verts)
            lo_c, lo_e, hi_c, hi_e = valid[name]
            assert cpos[list(rc)].min() >= lo_c and cpos[list(rc)].max() < hi_c, (l, name)
            assert epos[list(re_)].min() >= lo_e and epos[list(re_)].max() < hi_e, (l, name)
            # targets: this level's part plus, for l >= 1, the enclosing interface
            if l > 0 and name != "step3":
                O = P["levels"][l - 1]
                assert pp["ct_hi"] == O["cell_class_start"][5], (l, name)
                assert pp["et_hi"] == O["edge_class_start"][4], (l, name)


def test_nesting_rules(lib):
    m = periodic_hex_mesh(32, 32, 20e3, f0=1e-4)
    outer = strip_fine_mask(m, 6, 25, 20e3)
    # interface rings of the inner strip reach rows 7-8 and 23-24: too close
    with pytest.raises(lts.LTSError) as ei:
        lts.plan_levels(m, [outer, strip_fine_mask(m, 11, 20, 20e3)], 2, 2)
    assert ei.value.status == lts.LTS_ELABEL
    # an inner fine region sticking out of the outer one
    with pytest.raises(lts.LTSError) as ei:
        lts.plan_levels(m, [outer, strip_fine_mask(m, 20, 28, 20e3)], 2, 2)
    assert ei.value.status == lts.LTS_ELABEL
    # one fine level: the two-level plan
    a = lts.plan_levels(m, [outer], 2, 2)
    b = lts.plan(m, outer, 2, 2)
    assert np.array_equal(a["cell_order"], b["cell_order"])
    assert np.array_equal(a["levels"][0]["cell_class_start"], b["cell_class_start"])
