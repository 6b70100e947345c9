// Host runtime of liblts: the C ABI declared in include/lts.h.
//
// Upload: validate the mesh, label the LTS regions (eq:indexSetsCells,
// eq:index_sets_cells, eq:indexSetsEdges), permute cells, edges and vertices so
// that every evaluation set of Algorithm 2.2 is a contiguous range, fold the
// TRiSK coefficients (App. B) into per-cell slot tables, copy to the device.
//
// Cell order: [F minus underlined F | F2 | F1 | I1 | I2 | C1 | rest of C], where
// F1 are fine cells next to I1, F2 the fine cells next to F1, C1 the coarse
// cells next to I2.  Edge order: [edges of F minus underlined F cells |
// underlined-F edges | I1 | I2 | C].  Vertex order: by the smallest position of
// their three cells.  Within a class cells follow a Morton curve of their
// positions when given (input order otherwise); edges and vertices follow
// their cells.
//
// Step: one coarse LTS3 step is a fixed sequence of right-hand-side passes
// (vertex, cell and edge kernels over the ranges of that pass) with the stage
// arithmetic fused into the cell and edge kernels, captured once into a
// hipGraph per (M, dt) and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "lts_host.h"

using namespace lts;


namespace lts {

lts_status fail(lts_ctx* c, lts_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

size_t tsize(const lts_ctx* c) { return c->prec == LTS_FP64 ? 8 : 4; }

lts_status dalloc(lts_ctx* c, void** p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(c, LTS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c->allocs.push_back(*p);
    return LTS_OK;
}


}  // namespace lts

using namespace lts;

namespace {

void free_device(lts_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_kind = -1;
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    c->Qh = c->Qu = nullptr;
    if (c->dm) {
        if (c->prec == LTS_FP64) delete static_cast<DevMesh<double>*>(c->dm);
        else delete static_cast<DevMesh<float>*>(c->dm);
    }
    c->dm = nullptr;
}

// ---------------------------------------------------------------- validation
// Caller's edgesOnEdge / weightsOnEdge tables (optional) against the weights
// of eq:weights derived from the kite areas: w_{e,e'} = -n_{e,i} n_{e',i}
// (R - 1/2), R = kite fractions of cell i summed counter-clockwise from the
// slot of e' to the slot of e (the vertex after slot j is vertices_on_cell[j]).
lts_status check_weights(lts_ctx* c, const lts_mesh* m) {
    const bool any = m->n_edges_on_edge || m->edges_on_edge || m->weights_on_edge;
    if (!any) return LTS_OK;
    if (!m->n_edges_on_edge || !m->edges_on_edge || !m->weights_on_edge || m->max_edges2 < 1)
        return fail(c, LTS_EINVAL, "edges_on_edge tables: give all three with max_edges2 >= 1");
    const int mx = m->max_edges, m2 = m->max_edges2;
    auto kite = [&](int i, int v) {
        for (int k = 0; k < 3; ++k)
            if (m->cells_on_vertex[3 * v + k] == i) return m->kite_areas_on_vertex[3 * v + k];
        return 0.0;
    };
    std::vector<int> ee;
    std::vector<double> wd;
    for (int e = 0; e < m->n_edges; ++e) {
        ee.clear();
        wd.clear();
        for (int s = 0; s < 2; ++s) {
            const int i = m->cells_on_edge[2 * e + s];
            const int n = m->n_edges_on_cell[i];
            const int32_t* eo = m->edges_on_cell + (size_t)i * mx;
            const int32_t* vo = m->vertices_on_cell + (size_t)i * mx;
            int b = 0;
            while (b < n && eo[b] != e) ++b;
            const double ne = m->cells_on_edge[2 * e] == i ? 1.0 : -1.0;
            for (int a = 0; a < n; ++a) {
                if (a == b) continue;
                double R = 0.0;
                for (int j = a; j != b; j = (j + 1) % n) R += kite(i, vo[j]) / m->area_cell[i];
                const double na = m->cells_on_edge[2 * eo[a]] == i ? 1.0 : -1.0;
                ee.push_back(eo[a]);
                wd.push_back(-ne * na * (R - 0.5));
            }
        }
        const int ne_e = m->n_edges_on_edge[e];
        if (ne_e != (int)ee.size() || ne_e > m2)
            return fail(c, LTS_EMESH, "n_edges_on_edge differs from n_i + n_j - 2 at edge " +
                                          std::to_string(e));
        for (int k = 0; k < ne_e; ++k) {
            const int ep = m->edges_on_edge[(size_t)e * m2 + k];
            const double w = m->weights_on_edge[(size_t)e * m2 + k];
            const auto it = std::find(ee.begin(), ee.end(), ep);
            if (it == ee.end())
                return fail(c, LTS_EMESH, "edges_on_edge lists an edge outside EE(e) at edge " +
                                              std::to_string(e));
            const double d = wd[it - ee.begin()];
            if (!(std::fabs(w - d) <= 1e-9 * (1.0 + std::fabs(d))))
                return fail(c, LTS_EMESH, "weights_on_edge differs from the kite-area weights at edge " +
                                              std::to_string(e) + " (given " + std::to_string(w) +
                                              ", derived " + std::to_string(d) + ")");
            ee[it - ee.begin()] = -1;  // each member once
        }
    }
    return LTS_OK;
}

// Caller's sign tables (optional) against the orientation convention:
// n_{e,i} = +1 when i = cells_on_edge[e][0], t_{e,v} = +1 when
// v = vertices_on_edge[e][1].  Runs after the connectivity checks.
lts_status check_signs(lts_ctx* c, const lts_mesh* m) {
    if (m->edge_sign_on_cell)
        for (int i = 0; i < m->n_cells; ++i)
            for (int j = 0; j < m->n_edges_on_cell[i]; ++j) {
                const size_t o = (size_t)i * m->max_edges + j;
                const int e = m->edges_on_cell[o];
                const int want = m->cells_on_edge[2 * e] == i ? 1 : -1;
                if (m->edge_sign_on_cell[o] != want)
                    return fail(c, LTS_EMESH,
                                "edge_sign_on_cell differs from the orientation of cells_on_edge "
                                "at cell " + std::to_string(i));
            }
    if (m->edge_sign_on_vertex)
        for (int v = 0; v < m->n_vertices; ++v)
            for (int k = 0; k < 3; ++k) {
                const int e = m->edges_on_vertex[3 * v + k];
                const int want = m->vertices_on_edge[2 * e + 1] == v ? 1 : -1;
                if (m->edge_sign_on_vertex[3 * v + k] != want)
                    return fail(c, LTS_EMESH,
                                "edge_sign_on_vertex differs from the orientation of "
                                "vertices_on_edge at vertex " + std::to_string(v));
            }
    return LTS_OK;
}

lts_status validate(lts_ctx* c, const lts_mesh* m) {
    const int nC = m->n_cells, nE = m->n_edges, nV = m->n_vertices, mx = m->max_edges;
    if (nC < 3 || nE < 3 || nV < 3 || mx < 3)
        return fail(c, LTS_EMESH, "mesh sizes too small");
    if (mx > LTS_MAX_EDGES) return fail(c, LTS_EMESH, "max_edges exceeds LTS_MAX_EDGES");
    const void* req[] = {m->n_edges_on_cell, m->edges_on_cell, m->cells_on_cell,
                         m->vertices_on_cell, m->cells_on_edge, m->vertices_on_edge,
                         m->edges_on_vertex, m->cells_on_vertex, m->kite_areas_on_vertex,
                         m->area_cell, m->area_triangle, m->dc_edge, m->dv_edge,
                         m->f_vertex, m->bottom};
    for (const void* p : req)
        if (!p) return fail(c, LTS_EINVAL, "NULL mesh array");
    std::vector<int> edge_seen(nE, 0);
    for (int i = 0; i < nC; ++i) {
        const int n = m->n_edges_on_cell[i];
        if (n < 3 || n > mx) return fail(c, LTS_EMESH, "n_edges_on_cell out of range at cell " + std::to_string(i));
        if (!(m->area_cell[i] > 0)) return fail(c, LTS_EMESH, "non-positive area_cell");
        for (int j = 0; j < n; ++j) {
            const int e = m->edges_on_cell[(size_t)i * mx + j];
            const int nb = m->cells_on_cell[(size_t)i * mx + j];
            const int v = m->vertices_on_cell[(size_t)i * mx + j];
            if (e < 0 || e >= nE || nb < 0 || nb >= nC || v < 0 || v >= nV)
                return fail(c, LTS_EMESH, "index out of range at cell " + std::to_string(i));
            const int c0 = m->cells_on_edge[2 * e], c1 = m->cells_on_edge[2 * e + 1];
            if (!((c0 == i && c1 == nb) || (c1 == i && c0 == nb)))
                return fail(c, LTS_EMESH, "edge/cell mismatch at cell " + std::to_string(i));
            const int en = m->edges_on_cell[(size_t)i * mx + (j + 1) % n];
            if (en < 0 || en >= nE) return fail(c, LTS_EMESH, "index out of range");
            const int* ve = m->vertices_on_edge + 2 * e;
            const int* vn = m->vertices_on_edge + 2 * en;
            if (!((ve[0] == v || ve[1] == v) && (vn[0] == v || vn[1] == v)))
                return fail(c, LTS_EMESH, "vertex slot not shared by its edges at cell " + std::to_string(i));
            edge_seen[e]++;
        }
    }
    for (int e = 0; e < nE; ++e) {
        if (edge_seen[e] != 2) return fail(c, LTS_EMESH, "edge not on exactly two cells: " + std::to_string(e));
        if (!(m->dc_edge[e] > 0) || !(m->dv_edge[e] > 0))
            return fail(c, LTS_EMESH, "non-positive edge length");
        for (int s = 0; s < 2; ++s) {
            const int v = m->vertices_on_edge[2 * e + s];
            if (v < 0 || v >= nV) return fail(c, LTS_EMESH, "vertex index out of range");
        }
    }
    for (int v = 0; v < nV; ++v) {
        if (!(m->area_triangle[v] > 0)) return fail(c, LTS_EMESH, "non-positive area_triangle");
        for (int k = 0; k < 3; ++k) {
            const int e = m->edges_on_vertex[3 * v + k];
            const int ci = m->cells_on_vertex[3 * v + k];
            if (e < 0 || e >= nE || ci < 0 || ci >= nC)
                return fail(c, LTS_EMESH, "vertex degree is not 3 or index out of range");
            if (m->vertices_on_edge[2 * e] != v && m->vertices_on_edge[2 * e + 1] != v)
                return fail(c, LTS_EMESH, "edges_on_vertex inconsistent at vertex " + std::to_string(v));
            bool found = false;
            for (int j = 0; j < m->n_edges_on_cell[ci]; ++j)
                if (m->vertices_on_cell[(size_t)ci * mx + j] == v) found = true;
            if (!found) return fail(c, LTS_EMESH, "cells_on_vertex inconsistent at vertex " + std::to_string(v));
            if (!(m->kite_areas_on_vertex[3 * v + k] > 0))
                return fail(c, LTS_EMESH, "non-positive kite area");
        }
    }
    lts_status st = check_signs(c, m);
    return st ? st : check_weights(c, m);
}

// ---------------------------------------------------------------- regions
// Breadth-first rings around the fine set (eq:indexSetsCells with n1 and n2
// rings), F1/F2 (eq:index_sets_cells), edges to the finest adjacent region.
lts_status label_regions(lts_ctx* c, const lts_mesh* m, const uint8_t* fine, int n1, int n2,
                         std::vector<int>& cls, std::vector<int>& ecls) {
    const int nC = m->n_cells, nE = m->n_edges, mx = m->max_edges;
    if (n1 < 1 || n2 < 1) return fail(c, LTS_ELABEL, "interface rings must be >= 1");
    std::vector<int> ring(nC, -1), frontier, next;
    for (int i = 0; i < nC; ++i)
        if (fine[i]) { ring[i] = 0; frontier.push_back(i); }
    if (frontier.empty()) return fail(c, LTS_ELABEL, "empty fine region");
    if ((int)frontier.size() == nC) return fail(c, LTS_ELABEL, "every cell is fine");
    for (int r = 1; r <= n1 + n2; ++r) {
        next.clear();
        for (int i : frontier)
            for (int j = 0; j < m->n_edges_on_cell[i]; ++j) {
                const int nb = m->cells_on_cell[(size_t)i * mx + j];
                if (ring[nb] == -1) { ring[nb] = r; next.push_back(nb); }
            }
        frontier.swap(next);
    }
    c->creg.assign(nC, LTS_C);
    for (int i = 0; i < nC; ++i) {
        if (ring[i] == 0) c->creg[i] = LTS_F;
        else if (ring[i] >= 1 && ring[i] <= n1) c->creg[i] = LTS_I1;
        else if (ring[i] > n1) c->creg[i] = LTS_I2;
    }
    // classes: 0 Fint, 1 F2, 2 F1, 3 I1, 4 I2, 5 C1, 6 Crest
    cls.assign(nC, 6);
    for (int i = 0; i < nC; ++i) {
        if (c->creg[i] == LTS_I1) cls[i] = 3;
        else if (c->creg[i] == LTS_I2) cls[i] = 4;
        else if (c->creg[i] == LTS_F) cls[i] = 0;
    }
    auto touches = [&](int i, auto pred) {
        for (int j = 0; j < m->n_edges_on_cell[i]; ++j)
            if (pred(m->cells_on_cell[(size_t)i * mx + j])) return true;
        return false;
    };
    for (int i = 0; i < nC; ++i)
        if (c->creg[i] == LTS_F && touches(i, [&](int k) { return c->creg[k] == LTS_I1; })) cls[i] = 2;
    for (int i = 0; i < nC; ++i)
        if (cls[i] == 0 && touches(i, [&](int k) { return cls[k] == 2; })) cls[i] = 1;
    for (int i = 0; i < nC; ++i)
        if (c->creg[i] == LTS_C && touches(i, [&](int k) { return c->creg[k] == LTS_I2; })) cls[i] = 5;
    c->cfbar.assign(nC, 0);
    for (int i = 0; i < nC; ++i) c->cfbar[i] = (cls[i] == 1 || cls[i] == 2) ? 1 : 0;
    // edges: 0 Fint, 1 Fbar, 2 I1, 3 I2, 4 C
    ecls.assign(nE, 4);
    c->ereg.assign(nE, LTS_C);
    c->efbar.assign(nE, 0);
    for (int e = 0; e < nE; ++e) {
        const int a = m->cells_on_edge[2 * e], b = m->cells_on_edge[2 * e + 1];
        const int r = std::max(c->creg[a], c->creg[b]);
        c->ereg[e] = (int8_t)r;
        const bool fint = cls[a] == 0 || cls[b] == 0;
        if (r == LTS_F) {
            ecls[e] = fint ? 0 : 1;
            c->efbar[e] = fint ? 0 : 1;
        } else if (r == LTS_I1) ecls[e] = 2;
        else if (r == LTS_I2) ecls[e] = 3;
    }
    return LTS_OK;
}

uint64_t spread3(uint64_t x) {
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

// ---------------------------------------------------------------- typed setup
template <typename T>
std::vector<T> conv(const std::vector<double>& v) {
    return std::vector<T>(v.begin(), v.end());
}

template <typename T>
lts_status upload_vec(lts_ctx* c, const T** dst, const std::vector<T>& v) {
    void* p = nullptr;
    lts_status s = dalloc(c, &p, v.size() * sizeof(T));
    if (s) return s;
    HIPCHK(c, hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *dst = static_cast<const T*>(p);
    return LTS_OK;
}

// Perturbation form: href_i = H_s - b_i rounded to T, beta_i = href_i + b_i - H_s
// (the rounding residue), so the stored eta = h - href is small and
// g(h + b) = g(eta + beta) + g H_s.
template <typename T>
lts_status set_reference(lts_ctx* c, double Hs) {
    const int nC = c->nC;
    std::vector<T> hr(nC), be(nC);
    c->href_host.assign(nC, 0.0);
    for (int i = 0; i < nC; ++i) {
        hr[i] = (T)(Hs - c->bot_perm[i]);
        c->href_host[i] = (double)hr[i];
        be[i] = (T)((double)hr[i] + c->bot_perm[i] - Hs);
    }
    HIPCHK(c, hipMemcpy(c->d_href, hr.data(), nC * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_beta, be.data(), nC * sizeof(T), hipMemcpyHostToDevice));
    return LTS_OK;
}

// Reference surface from a state in device order ([cell][layer]):
// area-weighted mean of h + b over all layers.
double mean_surface(const lts_ctx* c, const std::vector<double>& h) {
    double num = 0.0, den = 0.0;
    for (int i = 0; i < c->nC; ++i)
        for (int l = 0; l < c->L; ++l) {
            num += c->area_perm[i] * (h[(size_t)i * c->L + l] + c->bot_perm[i]);
            den += c->area_perm[i];
        }
    return num / den;
}

template <typename T>
lts_status build_device(lts_ctx* c, const lts_mesh* m) {
    const int nC = c->nC, nE = c->nE, nV = c->nV;
    const int* cinv = c->cinv.data();
    const int* einv = c->einv.data();
    const int* vinv = c->vinv.data();
    // compact slot tables: cell ni's slots start at cso[ni].x
    std::vector<int32_t> nEoC(nC), cso(2 * (size_t)nC);
    size_t nslots = 0;
    for (int ni = 0; ni < nC; ++ni) {
        const int n = m->n_edges_on_cell[c->cperm[ni]];
        nEoC[ni] = n;
        cso[2 * (size_t)ni] = (int32_t)nslots;
        cso[2 * (size_t)ni + 1] = n;
        nslots += n;
    }
    if (nslots > (size_t)INT32_MAX) return fail(c, LTS_EMESH, "more than 2^31 edge slots");
    std::vector<int32_t> eoc(nslots), coc(nslots), voc(nslots);
    std::vector<double> nl(nslots), nd(nslots), kc(nslots), kf(nslots), sb(nslots), sn(nC),
        area(nC), rarea(nC), bot(nC);
    for (int ni = 0; ni < nC; ++ni) {
        const int i = c->cperm[ni];
        const int n = nEoC[ni];
        const size_t o0 = (size_t)cso[2 * (size_t)ni];
        area[ni] = m->area_cell[i];
        bot[ni] = m->bottom[i];
        double S = 0.0;  // counter-clockwise prefix sums of the kite fractions (FP64)
        for (int j = 0; j < n; ++j) {
            const size_t o = o0 + j;
            const int e = m->edges_on_cell[(size_t)i * m->max_edges + j];
            const int v = m->vertices_on_cell[(size_t)i * m->max_edges + j];
            eoc[o] = einv[e];
            coc[o] = cinv[m->cells_on_cell[(size_t)i * m->max_edges + j]];
            voc[o] = vinv[v];
            const double sgn = m->cells_on_edge[2 * e] == i ? 1.0 : -1.0;  // n_{e,i}
            nl[o] = sgn * m->dv_edge[e];
            nd[o] = sgn / m->dc_edge[e];
            kc[o] = m->dv_edge[e] * m->dc_edge[e] / (4.0 * m->area_cell[i]);
            double kite = 0.0;
            for (int k = 0; k < 3; ++k)
                if (m->cells_on_vertex[3 * v + k] == i) kite = m->kite_areas_on_vertex[3 * v + k];
            kf[o] = kite / m->area_cell[i];
            sb[o] = S;
            S += kf[o];
        }
        sn[ni] = S;
        rarea[ni] = 1.0 / m->area_cell[i];
    }
    std::vector<int32_t> eov((size_t)3 * nV), cov((size_t)3 * nV);
    std::vector<double> tdc((size_t)3 * nV), kite((size_t)3 * nV), fA(nV);
    for (int nv = 0; nv < nV; ++nv) {
        const int v = c->vperm[nv];
        fA[nv] = m->f_vertex[v] * m->area_triangle[v];
        for (int k = 0; k < 3; ++k) {
            const size_t o = (size_t)k * nV + nv;
            const int e = m->edges_on_vertex[3 * v + k];
            eov[o] = einv[e];
            const double tsg = m->vertices_on_edge[2 * e + 1] == v ? 1.0 : -1.0;  // t_{e,v}
            tdc[o] = tsg * m->dc_edge[e];
            cov[o] = cinv[m->cells_on_vertex[3 * v + k]];
            kite[o] = m->kite_areas_on_vertex[3 * v + k];
        }
    }
    auto* dm = new DevMesh<T>();
    c->dm = dm;
    dm->nC = nC;
    dm->nE = nE;
    dm->nV = nV;
    dm->maxE = c->maxE;
    lts_status s;
    if ((s = upload_vec<int32_t>(c, &dm->nEoC, nEoC))) return s;
    dm->nwide = (int)c->wide.size();
    dm->wide = nullptr;
    if (dm->nwide && (s = upload_vec<int32_t>(c, &dm->wide, c->wide))) return s;
    {
        const int32_t* p = nullptr;
        if ((s = upload_vec<int32_t>(c, &p, cso))) return s;
        dm->cso = reinterpret_cast<const int2*>(p);
    }
    if ((s = upload_vec<int32_t>(c, &dm->eoc, eoc))) return s;
    if ((s = upload_vec<int32_t>(c, &dm->coc, coc))) return s;
    if ((s = upload_vec<int32_t>(c, &dm->voc, voc))) return s;
    if ((s = upload_vec<T>(c, &dm->nl, conv<T>(nl)))) return s;
    if ((s = upload_vec<T>(c, &dm->nd, conv<T>(nd)))) return s;
    if ((s = upload_vec<T>(c, &dm->kc, conv<T>(kc)))) return s;
    if ((s = upload_vec<T>(c, &dm->kf, conv<T>(kf)))) return s;
    dm->pG = 0;
    dm->peoc = dm->pcoc = dm->pvoc = nullptr;
    dm->pnl = dm->pnd = dm->pkc = dm->pkf = nullptr;
    if (c->L > 1) {  // padded copies for the layered cell kernel
        const int G = padded_slots(c->maxE);
        const size_t np = (size_t)nC * G;
        std::vector<int32_t> pe(np), pc(np), pv(np);
        std::vector<double> pnl(np, 0.0), pnd(np, 0.0), pkc(np, 0.0), pkf(np, 0.0);
        for (int ni = 0; ni < nC; ++ni) {
            const size_t o0 = (size_t)cso[2 * (size_t)ni];
            const int n = nEoC[ni];
            for (int a = 0; a < G; ++a) {
                const size_t o = o0 + std::min(a, n - 1), d = (size_t)ni * G + a;
                pe[d] = eoc[o];
                pc[d] = coc[o];
                pv[d] = voc[o];
                if (a < n) {
                    pnl[d] = nl[o];
                    pnd[d] = nd[o];
                    pkc[d] = kc[o];
                    pkf[d] = kf[o];
                }
            }
        }
        dm->pG = G;
        if ((s = upload_vec<int32_t>(c, &dm->peoc, pe))) return s;
        if ((s = upload_vec<int32_t>(c, &dm->pcoc, pc))) return s;
        if ((s = upload_vec<int32_t>(c, &dm->pvoc, pv))) return s;
        if ((s = upload_vec<T>(c, &dm->pnl, conv<T>(pnl)))) return s;
        if ((s = upload_vec<T>(c, &dm->pnd, conv<T>(pnd)))) return s;
        if ((s = upload_vec<T>(c, &dm->pkc, conv<T>(pkc)))) return s;
        if ((s = upload_vec<T>(c, &dm->pkf, conv<T>(pkf)))) return s;
    }
    if ((s = upload_vec<T>(c, &dm->sb, conv<T>(sb)))) return s;
    if ((s = upload_vec<T>(c, &dm->sn, conv<T>(sn)))) return s;
    if ((s = upload_vec<T>(c, &dm->area, conv<T>(area)))) return s;
    if ((s = upload_vec<T>(c, &dm->rarea, conv<T>(rarea)))) return s;
    if ((s = upload_vec<T>(c, &dm->bot, conv<T>(bot)))) return s;
    c->bot_perm = bot;
    c->area_perm = area;
    c->pert = perturbation_form<T>();
    if (c->pert) {
        void* p = nullptr;
        if ((s = dalloc(c, &p, nC * sizeof(T)))) return s;
        c->d_href = p;
        if ((s = dalloc(c, &p, nC * sizeof(T)))) return s;
        c->d_beta = p;
        dm->href = static_cast<const T*>(c->d_href);
        dm->beta = static_cast<const T*>(c->d_beta);
        if ((s = set_reference<T>(c, 0.0))) return s;
    } else {
        dm->href = nullptr;
        dm->beta = dm->bot;
    }
    if ((s = upload_vec<int32_t>(c, &dm->eov, eov))) return s;
    if ((s = upload_vec<int32_t>(c, &dm->cov, cov))) return s;
    if ((s = upload_vec<T>(c, &dm->tdc, conv<T>(tdc)))) return s;
    if ((s = upload_vec<T>(c, &dm->kite, conv<T>(kite)))) return s;
    if ((s = upload_vec<T>(c, &dm->fA, conv<T>(fA)))) return s;

    // every per-element buffer holds L layers
    const size_t ts = sizeof(T) * (size_t)c->L;
    const int nI1c = c->cb[4] - c->cb[3], nI1e = c->eb[3] - c->eb[2];
    const int nIc = c->cb[5] - c->cb[3], nIe = c->eb[4] - c->eb[2];
    void** bufs[] = {&c->Ah, &c->Bh, &c->Ch};
    for (void** b : bufs) if ((s = dalloc(c, b, nC * ts))) return s;
    void** ubufs[] = {&c->Au, &c->Bu, &c->Cu};
    for (void** b : ubufs) if ((s = dalloc(c, b, nE * ts))) return s;
    if ((s = dalloc(c, &c->x0h, nI1c * ts)) || (s = dalloc(c, &c->x1h, nI1c * ts)) ||
        (s = dalloc(c, &c->x2h, nI1c * ts)) || (s = dalloc(c, &c->x0u, nI1e * ts)) ||
        (s = dalloc(c, &c->x1u, nI1e * ts)) || (s = dalloc(c, &c->x2u, nI1e * ts)) ||
        (s = dalloc(c, &c->acch, nIc * ts)) || (s = dalloc(c, &c->accu, nIe * ts)) ||
        (s = dalloc(c, &c->zs, 2 * (size_t)nE * ts)) || (s = dalloc(c, &c->q, nV * ts)))
        return s;
    // multi-level LTS3: level 0 uses the buffers above, inner levels their own
    for (size_t l = 0; l < c->lv.size(); ++l) {
        LevelData& V = c->lv[l];
        if (l == 0) {
            V.x0h = c->x0h; V.x1h = c->x1h; V.x2h = c->x2h;
            V.x0u = c->x0u; V.x1u = c->x1u; V.x2u = c->x2u;
            V.acch = c->acch; V.accu = c->accu;
            continue;
        }
        const size_t i1c = V.cb[4] - V.cb[3], i1e = V.eb[3] - V.eb[2];
        const size_t ic = V.cb[5] - V.cb[3], ie = V.eb[4] - V.eb[2];
        if ((s = dalloc(c, &V.x0h, i1c * ts)) || (s = dalloc(c, &V.x1h, i1c * ts)) ||
            (s = dalloc(c, &V.x2h, i1c * ts)) || (s = dalloc(c, &V.x0u, i1e * ts)) ||
            (s = dalloc(c, &V.x1u, i1e * ts)) || (s = dalloc(c, &V.x2u, i1e * ts)) ||
            (s = dalloc(c, &V.acch, ic * ts)) || (s = dalloc(c, &V.accu, ie * ts)))
            return s;
    }
    void* fp = nullptr;
    if ((s = dalloc(c, &fp, 64))) return s;
    c->flag = static_cast<int*>(fp);
    const int nblk = diag_blocks(nC * c->L) + diag_blocks(nE * c->L);
    void* pp = nullptr;
    if ((s = dalloc(c, &pp, (size_t)nblk * 8 * sizeof(double)))) return s;
    c->dpart = static_cast<double*>(pp);
    if ((s = dalloc(c, &pp, 8 * sizeof(double)))) return s;
    c->dout = static_cast<double*>(pp);
    // zero every state-sized buffer so ranges that read beyond the evaluated
    // set (never used) see finite numbers
    for (void* b : {c->Ah, c->Bh, c->Ch}) HIPCHK(c, hipMemset(b, 0, nC * ts));
    for (void* b : {c->Au, c->Bu, c->Cu}) HIPCHK(c, hipMemset(b, 0, nE * ts));
    HIPCHK(c, hipMemset(c->zs, 0, 2 * (size_t)nE * ts));
    // interface copies hold n_I1 elements, accumulators n_I1 + n_I2 (each
    // allocation is at least 8 bytes)
    for (void* b : {c->x0h, c->x1h, c->x2h}) HIPCHK(c, hipMemset(b, 0, nI1c * ts));
    for (void* b : {c->x0u, c->x1u, c->x2u}) HIPCHK(c, hipMemset(b, 0, nI1e * ts));
    HIPCHK(c, hipMemset(c->acch, 0, nIc * ts));
    HIPCHK(c, hipMemset(c->accu, 0, nIe * ts));
    HIPCHK(c, hipMemset(c->q, 0, nV * ts));
    HIPCHK(c, hipMemset(c->flag, 0, 64));
    HIPCHK(c, hipDeviceSynchronize());
    return LTS_OK;
}

// ---------------------------------------------------------------- plans
// Kernel ranges of one pass with target cells [ct_lo, ct_hi) and target edges
// [et_lo, et_hi) (device numbering): the cell kernel covers the targets and
// both cells of every target edge, the vertex kernel every vertex of those
// cells; plus the counts of unique elements the kernels gather.
PassPlan plan_cover(const lts_ctx* c, const lts_mesh* m, int ct_lo, int ct_hi, int et_lo,
                    int et_hi) {
    const int nC = c->nC, nE = c->nE;
    PassPlan P;
    P.ct_lo = ct_lo;
    P.ct_hi = ct_hi;
    P.et_lo = et_lo;
    P.et_hi = et_hi;
    int lo = P.ct_lo, hi = P.ct_hi;
    if (P.ct_hi <= P.ct_lo) { lo = nC; hi = 0; }
    for (int ne = P.et_lo; ne < P.et_hi; ++ne) {
        const int e = c->eperm[ne];
        for (int s = 0; s < 2; ++s) {
            const int ci = c->cinv[m->cells_on_edge[2 * e + s]];
            lo = std::min(lo, ci);
            hi = std::max(hi, ci + 1);
        }
    }
    if (hi <= lo) { lo = hi = 0; }
    P.c_lo = lo;
    P.c_hi = hi;
    P.w_lo = (int)(std::lower_bound(c->wide.begin(), c->wide.end(), lo) - c->wide.begin());
    P.w_hi = (int)(std::lower_bound(c->wide.begin(), c->wide.end(), hi) - c->wide.begin());
    int vlo = c->nV, vhi = 0;
    std::vector<char> useu(nE, 0), useh(nC, 0), useq(c->nV, 0);
    long slots = 0;
    for (int ni = lo; ni < hi; ++ni) {
        const int i = c->cperm[ni];
        useh[ni] = 1;
        for (int j = 0; j < m->n_edges_on_cell[i]; ++j) {
            const int v = c->vinv[m->vertices_on_cell[(size_t)i * m->max_edges + j]];
            vlo = std::min(vlo, v);
            vhi = std::max(vhi, v + 1);
            useq[v] = 1;
            useu[c->einv[m->edges_on_cell[(size_t)i * m->max_edges + j]]] = 1;
            useh[c->cinv[m->cells_on_cell[(size_t)i * m->max_edges + j]]] = 1;
            ++slots;
        }
    }
    if (vhi <= vlo) { vlo = vhi = 0; }
    P.v_lo = vlo;
    P.v_hi = vhi;
    P.c_uniq_h = std::count(useh.begin(), useh.end(), 1);
    P.c_uniq_u = std::count(useu.begin(), useu.end(), 1);
    P.c_uniq_q = std::count(useq.begin(), useq.end(), 1);
    P.c_slots = slots;
    std::vector<char> vu(nE, 0), vh(nC, 0);
    for (int nv = vlo; nv < vhi; ++nv) {
        const int v = c->vperm[nv];
        for (int k = 0; k < 3; ++k) {
            vu[c->einv[m->edges_on_vertex[3 * v + k]]] = 1;
            vh[c->cinv[m->cells_on_vertex[3 * v + k]]] = 1;
        }
    }
    P.v_uniq_u = std::count(vu.begin(), vu.end(), 1);
    P.v_uniq_h = std::count(vh.begin(), vh.end(), 1);
    return P;
}

void make_plans(lts_ctx* c, const lts_mesh* m) {
    const int nC = c->nC, nE = c->nE;
    const int* cb = c->cb;
    const int* eb = c->eb;
    struct T4 { int ct_lo, ct_hi, et_lo, et_hi; };
    const T4 targets[P_N] = {
        {0, nC, 0, nE},            // FULL
        {cb[1], nC, eb[1], nE},    // STEP1: underlined F, I, C
        {cb[3], nC, eb[2], nE},    // STEP2: I, C
        {0, cb[5], 0, eb[4]},      // STEP3: F, I (fine edges, I edges)
        {cb[5], nC, eb[4], nE},    // STEP4: C
    };
    for (int p = 0; p < P_N; ++p)
        c->plan[p] = plan_cover(c, m, targets[p].ct_lo, targets[p].ct_hi, targets[p].et_lo,
                                targets[p].et_hi);
    // interface cells and edges only (the surrogate's interface accumulation)
    c->iface_plan = plan_cover(c, m, cb[3], cb[5], eb[2], eb[4]);
    // multi-level LTS3: level 0 is the two-level plan; level l >= 1 adds the
    // enclosing interface (accumulated) to its Steps 1, 2 and 4
    if (!c->lv.empty()) {
        LevelData& V0 = c->lv[0];
        std::copy(cb, cb + 8, V0.cb);
        std::copy(eb, eb + 6, V0.eb);
        V0.p1 = c->plan[P_STEP1];
        V0.p2 = c->plan[P_STEP2];
        V0.p3 = c->plan[P_STEP3];
        V0.p4 = c->plan[P_STEP4];
        for (size_t l = 1; l < c->lv.size(); ++l) {
            LevelData& V = c->lv[l];
            const LevelData& O = c->lv[l - 1];
            V.p1 = plan_cover(c, m, V.cb[1], O.cb[5], V.eb[1], O.eb[4]);
            V.p2 = plan_cover(c, m, V.cb[3], O.cb[5], V.eb[2], O.eb[4]);
            V.p3 = plan_cover(c, m, 0, V.cb[5], 0, V.eb[4]);
            V.p4 = plan_cover(c, m, V.cb[5], O.cb[5], V.eb[4], O.eb[4]);
        }
    }
}

// Enqueue n steps of `scheme`: replayed from a hipGraph captured once per
// (scheme, M, dt), or launched directly with event stamps in timing mode.
template <typename T>
lts_status run_scheme(lts_ctx* c, int scheme, double dt, int M, int n) {
    const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
    Run<T> r{c, dm, c->stream, c->timing};
    if (c->timing) {
        for (int i = 0; i < n; ++i) {
            lts_status st = one_step<T>(r, scheme, dt, M);
            if (st) return st;
        }
        return LTS_OK;
    }
    if (!(c->gexec && c->g_kind == scheme && c->g_M == M && c->g_dt == dt &&
          (scheme != SCH_MLTS3 || c->g_Ms == c->run_Ms))) {
        if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->gexec = nullptr;
        c->graph = nullptr;
        c->g_kind = -1;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        lts_status st = one_step<T>(r, scheme, dt, M);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &gr);
        if (st) {
            if (gr) (void)hipGraphDestroy(gr);
            return st;
        }
        if (e != hipSuccess) return fail(c, LTS_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
        c->graph = gr;
        HIPCHK(c, hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0));
        c->g_kind = scheme;
        c->g_M = M;
        c->g_Ms = c->run_Ms;
        c->g_dt = dt;
    }
    for (int i = 0; i < n; ++i) HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    return LTS_OK;
}

// Host state arrays hold the L layers one after another (layer-major, caller
// numbering); device arrays are [element][layer] in device order.
template <typename T>
void to_device(const lts_ctx* c, const double* h, const double* u, std::vector<T>& hh,
               std::vector<T>& uu) {
    const int nC = c->nC, nE = c->nE, L = c->L;
    hh.resize((size_t)nC * L);
    uu.resize((size_t)nE * L);
    for (int ni = 0; ni < nC; ++ni)
        for (int l = 0; l < L; ++l)
            hh[(size_t)ni * L + l] =
                (T)(h[(size_t)l * nC + c->cperm[ni]] - (c->pert ? c->href_host[ni] : 0.0));
    for (int ne = 0; ne < nE; ++ne)
        for (int l = 0; l < L; ++l) uu[(size_t)ne * L + l] = (T)u[(size_t)l * nE + c->eperm[ne]];
}

template <typename T>
void from_device(const lts_ctx* c, const std::vector<T>& hh, const std::vector<T>& uu, double* h,
                 double* u, bool add_ref) {
    const int nC = c->nC, nE = c->nE, L = c->L;
    if (h)
        for (int ni = 0; ni < nC; ++ni)
            for (int l = 0; l < L; ++l)
                h[(size_t)l * nC + c->cperm[ni]] =
                    (double)hh[(size_t)ni * L + l] + (add_ref && c->pert ? c->href_host[ni] : 0.0);
    if (u)
        for (int ne = 0; ne < nE; ++ne)
            for (int l = 0; l < L; ++l)
                u[(size_t)l * nE + c->eperm[ne]] = (double)uu[(size_t)ne * L + l];
}

template <typename T>
lts_status eval_rhs(lts_ctx* c, const double* h, const double* u, double* dh, double* du) {
    const int nC = c->nC, nE = c->nE;
    const size_t L = c->L;
    std::vector<T> hh, uu;
    to_device<T>(c, h, u, hh, uu);
    HIPCHK(c, hipMemcpyAsync(c->Bh, hh.data(), nC * L * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->Bu, uu.data(), nE * L * sizeof(T), hipMemcpyHostToDevice, c->stream));
    const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
    Run<T> r{c, dm, c->stream, false};
    const Seg<T> none;
    lts_status st = r.pass(P_FULL, (T*)c->Bh, (T*)c->Bu,
                           Run<T>::upd(0, nC, (T*)c->Ch, nullptr, 0, nullptr, 0, 1.0), none,
                           Run<T>::upd(0, nE, (T*)c->Cu, nullptr, 0, nullptr, 0, 1.0), none);
    if (st) return st;
    HIPCHK(c, hipMemcpyAsync(hh.data(), c->Ch, nC * L * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(uu.data(), c->Cu, nE * L * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    from_device<T>(c, hh, uu, dh, du, false);
    // the stage buffers B and C now hold the evaluation's input and output;
    // a captured step graph stays valid, since every step writes them before
    // it reads them
    return LTS_OK;
}

template <typename T>
lts_status set_state(lts_ctx* c, const double* h, const double* u) {
    const size_t L = c->L;
    if (c->pert) {
        std::vector<double> hp((size_t)c->nC * L);
        for (int ni = 0; ni < c->nC; ++ni)
            for (size_t l = 0; l < L; ++l) hp[ni * L + l] = h[l * c->nC + c->cperm[ni]];
        lts_status s = set_reference<T>(c, mean_surface(c, hp));
        if (s) return s;
    }
    std::vector<T> hh, uu;
    to_device<T>(c, h, u, hh, uu);
    HIPCHK(c, hipMemcpyAsync(c->Ah, hh.data(), c->nC * L * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->Au, uu.data(), c->nE * L * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LTS_OK;
}

template <typename T>
lts_status get_state(lts_ctx* c, double* h, double* u) {
    const size_t L = c->L;
    std::vector<T> hh((size_t)c->nC * L), uu((size_t)c->nE * L);
    HIPCHK(c, hipMemcpyAsync(hh.data(), c->Ah, c->nC * L * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(uu.data(), c->Au, c->nE * L * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    from_device<T>(c, hh, uu, h, u, true);
    return LTS_OK;
}

template <typename T>
lts_status diagnostics(lts_ctx* c, double out[8]) {
    const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
    HIPCHK(c, launch_diag<T>(dm, (T*)c->Ah, (T*)c->Au, c->g, c->dpart, diag_blocks(c->nC * c->L),
                             diag_blocks(c->nE * c->L), c->dout, c->stream, c->L));
    int flag = 0;
    HIPCHK(c, hipMemcpyAsync(out, c->dout, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out[6] = flag;
    return LTS_OK;
}

lts_status ready(lts_ctx* c, bool need_state) {
    if (!c) return LTS_EINVAL;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(c, LTS_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    if (!c->has_mesh) return fail(c, LTS_ESTATE, "no mesh uploaded");
    if (need_state && !c->has_state) return fail(c, LTS_ESTATE, "no state initialised");
    return LTS_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

lts_status lts_create(lts_ctx** out, int device, lts_precision prec, void* hip_stream) {
    if (!out) return LTS_EINVAL;
    *out = nullptr;
    if (prec != LTS_FP64 && prec != LTS_FP32) return LTS_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LTS_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return LTS_EDEVICE;
    lts_ctx* c = new lts_ctx();
    c->device = device;
    c->prec = prec;
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return LTS_EDEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return LTS_OK;
}

void lts_destroy(lts_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    free_device(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* lts_last_error(const lts_ctx* c) { return c ? c->err.c_str() : "null context"; }

lts_status lts_set_layers(lts_ctx* c, int n_layers) {
    if (!c) return LTS_EINVAL;
    if (n_layers < 1) return fail(c, LTS_EINVAL, "need n_layers >= 1");
    if (c->has_mesh) return fail(c, LTS_ESTATE, "set the layer count before uploading the mesh");
    c->L = n_layers;
    return LTS_OK;
}

}  // extern "C"

namespace {

// Host-side planning: validation, LTS labels, permutation, pass plans.
lts_status plan_mesh(lts_ctx* c, const lts_mesh* m, const uint8_t* fine, int n1, int n2,
                     double gravity, int nfine = 1) {
    lts_status s = validate(c, m);
    if (s) return s;
    std::vector<int> cls, ecls;
    if ((s = label_regions(c, m, fine, n1, n2, cls, ecls))) return s;
    const int nC = m->n_cells, nE = m->n_edges, nV = m->n_vertices;
    // multi-level LTS3: the classes of every nested level (level 0 above)
    c->lv.clear();
    std::vector<std::vector<int>> lcls(nfine), lecls(nfine);
    lcls[0] = cls;
    lecls[0] = ecls;
    if (nfine > 1) {
        c->lv.resize(nfine);
        for (int l = 1; l < nfine; ++l) {
            lts_ctx tmp;
            if ((s = label_regions(&tmp, m, fine + (size_t)l * nC, n1, n2, lcls[l], lecls[l])))
                return fail(c, s, "level " + std::to_string(l) + ": " + tmp.err);
            LevelData& V = c->lv[l];
            V.creg = tmp.creg;
            V.ereg = tmp.ereg;
            V.cfbar = tmp.cfbar;
            V.efbar = tmp.efbar;
            // nesting: level l's fine and interface cells lie at least four
            // cell rings inside level l-1's fine region (three would do for
            // the method; the fourth keeps level l's coarse cells next to its
            // interface 2 inside level l-1's interior class, so every level's
            // evaluation sets stay contiguous ranges)
            const std::vector<int8_t>& outer = l == 1 ? c->creg : c->lv[l - 1].creg;
            std::vector<int> depth(nC, -1);
            for (int i = 0; i < nC; ++i)
                if (outer[i] != LTS_F) depth[i] = 0;
            for (int r = 1; r <= 3; ++r)
                for (int i = 0; i < nC; ++i) {
                    if (depth[i] != -1) continue;
                    for (int j = 0; j < m->n_edges_on_cell[i]; ++j)
                        if (depth[m->cells_on_cell[(size_t)i * m->max_edges + j]] == r - 1) {
                            depth[i] = r;
                            break;
                        }
                }
            for (int i = 0; i < nC; ++i)
                if (V.creg[i] != LTS_C && depth[i] != -1)
                    return fail(c, LTS_ELABEL,
                                "level " + std::to_string(l) +
                                    ": a fine or interface cell lies fewer than four rings "
                                    "inside the enclosing fine region");
        }
        c->lv[0].creg = c->creg;
        c->lv[0].ereg = c->ereg;
        c->lv[0].cfbar = c->cfbar;
        c->lv[0].efbar = c->efbar;
        // sort keys: level 0's class, then each inner level's class while all
        // enclosing classes are 0 (the interior of their fine region)
        for (int i = 0; i < nC; ++i) {
            int key = 0;
            bool inside = true;
            for (int l = 0; l < nfine; ++l) {
                const int k = inside ? lcls[l][i] : 0;
                key = key * 8 + k;
                inside = inside && lcls[l][i] == 0;
            }
            cls[i] = key;
        }
        for (int e = 0; e < nE; ++e) {
            int key = 0;
            bool inside = true;
            for (int l = 0; l < nfine; ++l) {
                const int k = inside ? lecls[l][e] : 0;
                key = key * 8 + k;
                inside = inside && lecls[l][e] == 0;
            }
            ecls[e] = key;
        }
    }
    c->nC = nC;
    c->nE = nE;
    c->nV = nV;
    // lanes per cell follow the largest cell present, not the declared
    // capacity max_edges (the stride of the caller's arrays)
    c->maxE = 0;
    for (int i = 0; i < nC; ++i) c->maxE = std::max(c->maxE, m->n_edges_on_cell[i]);
    c->g = gravity;
    // cell order: class, then Morton key of the position (or input index)
    std::vector<uint64_t> key(nC, 0);
    if (m->cell_xyz) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int i = 0; i < nC; ++i)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], m->cell_xyz[3 * i + d]);
                hi[d] = std::max(hi[d], m->cell_xyz[3 * i + d]);
            }
        for (int i = 0; i < nC; ++i) {
            uint64_t k = 0;
            for (int d = 0; d < 3; ++d) {
                const double span = hi[d] - lo[d];
                const double f = span > 0 ? (m->cell_xyz[3 * i + d] - lo[d]) / span : 0.0;
                k |= spread3((uint64_t)std::min(2097151.0, f * 2097151.0)) << d;
            }
            key[i] = k;
        }
    }
    c->cperm.resize(nC);
    std::iota(c->cperm.begin(), c->cperm.end(), 0);
    std::stable_sort(c->cperm.begin(), c->cperm.end(), [&](int a, int b) {
        if (cls[a] != cls[b]) return cls[a] < cls[b];
        return key[a] < key[b];
    });
    c->cinv.assign(nC, 0);
    for (int ni = 0; ni < nC; ++ni) c->cinv[c->cperm[ni]] = ni;
    // class starts of level 0, then of every inner level inside the interior
    // of the enclosing fine region
    auto starts = [&](const std::vector<int>& lc, int lo, int hi, int* out, int nk) {
        for (int k = 0; k < nk; ++k) out[k] = hi;
        for (int ni = hi - 1; ni >= lo; --ni) out[lc[ni]] = ni;
        for (int k = nk - 2; k >= 0; --k) out[k] = std::min(out[k], out[k + 1]);
    };
    {
        std::vector<int> lc(nC);
        for (int ni = 0; ni < nC; ++ni) lc[ni] = lcls[0][c->cperm[ni]];
        starts(lc, 0, nC, c->cb, 7);
        c->cb[7] = nC;
        for (int l = 1; l < nfine; ++l) {
            int* ob = l == 1 ? c->cb : c->lv[l - 1].cb;
            for (int ni = 0; ni < nC; ++ni) lc[ni] = lcls[l][c->cperm[ni]];
            starts(lc, 0, ob[1], c->lv[l].cb, 7);
            c->lv[l].cb[7] = ob[3];
        }
    }
    // edges: class, then (min cell position, max cell position)
    c->eperm.resize(nE);
    std::iota(c->eperm.begin(), c->eperm.end(), 0);
    auto emin = [&](int e) { return std::min(c->cinv[m->cells_on_edge[2 * e]], c->cinv[m->cells_on_edge[2 * e + 1]]); };
    auto emax = [&](int e) { return std::max(c->cinv[m->cells_on_edge[2 * e]], c->cinv[m->cells_on_edge[2 * e + 1]]); };
    std::stable_sort(c->eperm.begin(), c->eperm.end(), [&](int a, int b) {
        if (ecls[a] != ecls[b]) return ecls[a] < ecls[b];
        if (emin(a) != emin(b)) return emin(a) < emin(b);
        return emax(a) < emax(b);
    });
    c->einv.assign(nE, 0);
    for (int ne = 0; ne < nE; ++ne) c->einv[c->eperm[ne]] = ne;
    {
        std::vector<int> lc(nE);
        for (int ne = 0; ne < nE; ++ne) lc[ne] = lecls[0][c->eperm[ne]];
        starts(lc, 0, nE, c->eb, 5);
        c->eb[5] = nE;
        for (int l = 1; l < nfine; ++l) {
            int* ob = l == 1 ? c->eb : c->lv[l - 1].eb;
            for (int ne = 0; ne < nE; ++ne) lc[ne] = lecls[l][c->eperm[ne]];
            starts(lc, 0, ob[1], c->lv[l].eb, 5);
            c->lv[l].eb[5] = ob[2];
        }
    }
    // vertices: smallest then largest position of their cells
    std::vector<int> vmin(nV), vmax(nV);
    for (int v = 0; v < nV; ++v) {
        int a = nC, b = -1;
        for (int k = 0; k < 3; ++k) {
            const int ci = c->cinv[m->cells_on_vertex[3 * v + k]];
            a = std::min(a, ci);
            b = std::max(b, ci);
        }
        vmin[v] = a;
        vmax[v] = b;
    }
    c->vperm.resize(nV);
    std::iota(c->vperm.begin(), c->vperm.end(), 0);
    std::stable_sort(c->vperm.begin(), c->vperm.end(), [&](int a, int b) {
        if (vmin[a] != vmin[b]) return vmin[a] < vmin[b];
        return vmax[a] < vmax[b];
    });
    c->vinv.assign(nV, 0);
    for (int nv = 0; nv < nV; ++nv) c->vinv[c->vperm[nv]] = nv;
    c->wide.clear();
    for (int ni = 0; ni < nC; ++ni)
        if (m->n_edges_on_cell[c->cperm[ni]] > 8) c->wide.push_back(ni);
    make_plans(c, m);
    return LTS_OK;
}

}  // namespace

extern "C" {

lts_status lts_upload_mesh(lts_ctx* c, const lts_mesh* m, const uint8_t* fine, int n1, int n2,
                           double gravity) {
    return lts_upload_mesh_levels(c, m, 1, fine, n1, n2, gravity);
}

lts_status lts_upload_mesh_levels(lts_ctx* c, const lts_mesh* m, int nfine, const uint8_t* fine,
                                  int n1, int n2, double gravity) {
    if (!c || !m || !fine) return c ? fail(c, LTS_EINVAL, "NULL argument") : LTS_EINVAL;
    if (nfine < 1 || nfine > LTS_MAX_LEVELS - 1)
        return fail(c, LTS_EINVAL, "n_fine_levels must be 1 .. LTS_MAX_LEVELS - 1");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, LTS_EDEVICE, "hipSetDevice");
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_device(c);
    c->has_mesh = c->has_state = c->nonfinite = false;
    lts_status s = plan_mesh(c, m, fine, n1, n2, gravity, nfine);
    if (s) return s;
    s = c->prec == LTS_FP64 ? build_device<double>(c, m) : build_device<float>(c, m);
    if (s) {
        free_device(c);
        return s;
    }
    c->has_mesh = true;
    return LTS_OK;
}

lts_status lts_plan(const lts_mesh* m, const uint8_t* fine, int n1, int n2, int8_t* cell_region,
                    int8_t* edge_region, uint8_t* cell_fbar, uint8_t* edge_fbar,
                    int32_t* cell_order, int32_t* edge_order, int32_t* vertex_order,
                    int32_t* ranges, char* errbuf, int errlen) {
    if (!m || !fine) return LTS_EINVAL;
    lts_ctx tmp;
    lts_status s = plan_mesh(&tmp, m, fine, n1, n2, 9.81);
    if (s) {
        if (errbuf && errlen > 0) {
            std::strncpy(errbuf, tmp.err.c_str(), errlen - 1);
            errbuf[errlen - 1] = 0;
        }
        return s;
    }
    if (cell_region) std::copy(tmp.creg.begin(), tmp.creg.end(), cell_region);
    if (edge_region) std::copy(tmp.ereg.begin(), tmp.ereg.end(), edge_region);
    if (cell_fbar) std::copy(tmp.cfbar.begin(), tmp.cfbar.end(), cell_fbar);
    if (edge_fbar) std::copy(tmp.efbar.begin(), tmp.efbar.end(), edge_fbar);
    if (cell_order) std::copy(tmp.cperm.begin(), tmp.cperm.end(), cell_order);
    if (edge_order) std::copy(tmp.eperm.begin(), tmp.eperm.end(), edge_order);
    if (vertex_order) std::copy(tmp.vperm.begin(), tmp.vperm.end(), vertex_order);
    if (ranges) {
        int k = 0;
        for (int j = 0; j < 8; ++j) ranges[k++] = tmp.cb[j];
        for (int j = 0; j < 6; ++j) ranges[k++] = tmp.eb[j];
        for (int p = 0; p < P_N; ++p) {
            const PassPlan& P = tmp.plan[p];
            const int v[8] = {P.c_lo, P.c_hi, P.v_lo, P.v_hi, P.ct_lo, P.ct_hi, P.et_lo, P.et_hi};
            for (int j = 0; j < 8; ++j) ranges[k++] = v[j];
        }
    }
    return LTS_OK;
}

lts_status lts_plan_levels(const lts_mesh* m, int nfine, const uint8_t* fine, int n1, int n2,
                           int32_t* cell_order, int32_t* edge_order, int32_t* vertex_order,
                           int32_t* ranges, char* errbuf, int errlen) {
    if (!m || !fine || nfine < 1 || nfine > LTS_MAX_LEVELS - 1) return LTS_EINVAL;
    lts_ctx tmp;
    lts_status s = plan_mesh(&tmp, m, fine, n1, n2, 9.81, nfine);
    if (s) {
        if (errbuf && errlen > 0) {
            std::strncpy(errbuf, tmp.err.c_str(), errlen - 1);
            errbuf[errlen - 1] = 0;
        }
        return s;
    }
    if (cell_order) std::copy(tmp.cperm.begin(), tmp.cperm.end(), cell_order);
    if (edge_order) std::copy(tmp.eperm.begin(), tmp.eperm.end(), edge_order);
    if (vertex_order) std::copy(tmp.vperm.begin(), tmp.vperm.end(), vertex_order);
    if (ranges) {
        int k = 0;
        for (int l = 0; l < nfine; ++l) {
            LevelData V;
            if (tmp.lv.empty()) {  // one fine level: the two-level plan
                std::copy(tmp.cb, tmp.cb + 8, V.cb);
                std::copy(tmp.eb, tmp.eb + 6, V.eb);
                V.p1 = tmp.plan[P_STEP1];
                V.p2 = tmp.plan[P_STEP2];
                V.p3 = tmp.plan[P_STEP3];
                V.p4 = tmp.plan[P_STEP4];
            } else {
                V = tmp.lv[l];
            }
            for (int j = 0; j < 8; ++j) ranges[k++] = V.cb[j];
            for (int j = 0; j < 6; ++j) ranges[k++] = V.eb[j];
            for (const PassPlan* P : {&V.p1, &V.p2, &V.p3, &V.p4}) {
                const int v[8] = {P->c_lo, P->c_hi, P->v_lo, P->v_hi,
                                  P->ct_lo, P->ct_hi, P->et_lo, P->et_hi};
                for (int j = 0; j < 8; ++j) ranges[k++] = v[j];
            }
        }
    }
    return LTS_OK;
}

lts_status lts_get_regions(lts_ctx* c, int8_t* cr, int8_t* er, uint8_t* cf, uint8_t* ef) {
    lts_status s = ready(c, false);
    if (s) return s;
    if (cr) std::copy(c->creg.begin(), c->creg.end(), cr);
    if (er) std::copy(c->ereg.begin(), c->ereg.end(), er);
    if (cf) std::copy(c->cfbar.begin(), c->cfbar.end(), cf);
    if (ef) std::copy(c->efbar.begin(), c->efbar.end(), ef);
    return LTS_OK;
}

lts_status lts_region_counts(lts_ctx* c, int64_t* cells, int64_t* edges, int64_t* fbar) {
    lts_status s = ready(c, false);
    if (s) return s;
    if (cells) {
        cells[LTS_F] = c->cb[3];
        cells[LTS_I1] = c->cb[4] - c->cb[3];
        cells[LTS_I2] = c->cb[5] - c->cb[4];
        cells[LTS_C] = c->nC - c->cb[5];
    }
    if (edges) {
        edges[LTS_F] = c->eb[2];
        edges[LTS_I1] = c->eb[3] - c->eb[2];
        edges[LTS_I2] = c->eb[4] - c->eb[3];
        edges[LTS_C] = c->nE - c->eb[4];
    }
    if (fbar) {
        fbar[0] = c->cb[3] - c->cb[1];
        fbar[1] = c->eb[2] - c->eb[1];
    }
    return LTS_OK;
}

lts_status lts_init_state(lts_ctx* c, const double* h, const double* u, double t0) {
    lts_status s = ready(c, false);
    if (s) return s;
    if (!h || !u) return fail(c, LTS_EINVAL, "NULL state");
    s = c->prec == LTS_FP64 ? set_state<double>(c, h, u) : set_state<float>(c, h, u);
    if (s) return s;
    HIPCHK(c, launch_fill_int(c->flag, 0, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_state = true;
    c->nonfinite = false;
    c->t = t0;
    c->steps = 0;
    c->gate_fallbacks = 0;
    return LTS_OK;
}

lts_status lts_init_state_device(lts_ctx* c, const void* dh, const void* du, double t0) {
    lts_status s = ready(c, false);
    if (s) return s;
    if (!dh || !du) return fail(c, LTS_EINVAL, "NULL state");
    const size_t nh = (size_t)c->nC * c->L, nu = (size_t)c->nE * c->L;
    std::vector<double> h(nh), u(nu);
    if (c->prec == LTS_FP64) {
        HIPCHK(c, hipMemcpy(h.data(), dh, nh * sizeof(double), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(u.data(), du, nu * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::vector<float> hf(nh), uf(nu);
        HIPCHK(c, hipMemcpy(hf.data(), dh, nh * sizeof(float), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(uf.data(), du, nu * sizeof(float), hipMemcpyDeviceToHost));
        std::copy(hf.begin(), hf.end(), h.begin());
        std::copy(uf.begin(), uf.end(), u.begin());
    }
    return lts_init_state(c, h.data(), u.data(), t0);
}

}  // extern "C"

namespace {

lts_status step_scheme(lts_ctx* c, int scheme, double dt, int M, int n) {
    lts_status s = ready(c, true);
    if (s) return s;
    if (scheme >= SCH_SSPRK3 && scheme <= SCH_RK4) M = 1;
    if (!(dt > 0) || M < 1 || n < 0) return fail(c, LTS_EINVAL, "need dt > 0, M >= 1, n >= 0");
    if (c->nonfinite) return fail(c, LTS_ENONFINITE, "state is non-finite; re-initialise");
    if (n == 0) return LTS_OK;
    if (scheme == SCH_RK4 && !c->Qh) {
        const size_t ts = tsize(c) * (size_t)c->L;
        if ((s = dalloc(c, &c->Qh, c->nC * ts)) || (s = dalloc(c, &c->Qu, c->nE * ts))) return s;
        HIPCHK(c, hipMemset(c->Qh, 0, c->nC * ts));
        HIPCHK(c, hipMemset(c->Qu, 0, c->nE * ts));
    }
    s = c->prec == LTS_FP64 ? run_scheme<double>(c, scheme, dt, M, n)
                            : run_scheme<float>(c, scheme, dt, M, n);
    if (s) return s;
    c->t += dt * n;
    c->steps += n;
    return LTS_OK;
}

}  // namespace

extern "C" {

lts_status lts_step_scheme(lts_ctx* c, int scheme, double dt, int M, int n) {
    if (c && (scheme < SCH_LTS3 || scheme > SCH_RK4)) return fail(c, LTS_EINVAL, "unknown scheme");
    return step_scheme(c, scheme, dt, M, n);
}

lts_status lts_step(lts_ctx* c, double dt, int M, int n) {
    return lts_step_scheme(c, SCH_LTS3, dt, M, n);
}

lts_status lts_step_levels(lts_ctx* c, double dt, const int32_t* M, int n) {
    if (!c) return LTS_EINVAL;
    if (!c->has_mesh) return fail(c, LTS_ESTATE, "no mesh");
    if (c->lv.empty()) return fail(c, LTS_EINVAL, "the mesh was uploaded with one fine level");
    if (!M) return fail(c, LTS_EINVAL, "NULL ratios");
    std::vector<int> Ms(c->lv.size());
    for (size_t l = 0; l < Ms.size(); ++l) {
        if (M[l] < 1) return fail(c, LTS_EINVAL, "every ratio must be >= 1");
        Ms[l] = M[l];
    }
    c->run_Ms = Ms;
    return step_scheme(c, SCH_MLTS3, dt, Ms[0], n);
}

lts_status lts_get_level_regions(lts_ctx* c, int level, int8_t* cr, int8_t* er, uint8_t* cf,
                                 uint8_t* ef) {
    lts_status s = ready(c, false);
    if (s) return s;
    if (level == 0) return lts_get_regions(c, cr, er, cf, ef);
    if (level < 0 || level >= (int)c->lv.size())
        return fail(c, LTS_EINVAL, "no such level");
    const LevelData& V = c->lv[level];
    if (cr) std::copy(V.creg.begin(), V.creg.end(), cr);
    if (er) std::copy(V.ereg.begin(), V.ereg.end(), er);
    if (cf) std::copy(V.cfbar.begin(), V.cfbar.end(), cf);
    if (ef) std::copy(V.efbar.begin(), V.efbar.end(), ef);
    return LTS_OK;
}

lts_status lts_step_rk3(lts_ctx* c, double dt, int n) {
    return lts_step_scheme(c, SCH_SSPRK3, dt, 1, n);
}

lts_status lts_eval_rhs(lts_ctx* c, const double* h, const double* u, double* dh, double* du) {
    lts_status s = ready(c, false);
    if (s) return s;
    if (!h || !u || !dh || !du) return fail(c, LTS_EINVAL, "NULL argument");
    return c->prec == LTS_FP64 ? eval_rhs<double>(c, h, u, dh, du)
                               : eval_rhs<float>(c, h, u, dh, du);
}

lts_status lts_diagnostics(lts_ctx* c, lts_diag* out) {
    lts_status s = ready(c, true);
    if (s) return s;
    if (!out) return fail(c, LTS_EINVAL, "NULL output");
    double d[8] = {0};
    s = c->prec == LTS_FP64 ? diagnostics<double>(c, d) : diagnostics<float>(c, d);
    if (s) return s;
    out->t = c->t;
    out->mass = d[0];
    out->energy = d[1];
    out->h_min = d[2];
    out->h_max = d[3];
    out->u_absmax = d[4];
    out->n_nonfinite = (int64_t)d[5];
    out->steps = c->steps;
    out->gate_fallbacks = c->gate_fallbacks;
    if (d[6] != 0 || d[5] != 0) c->nonfinite = true;
    if (c->nonfinite) return fail(c, LTS_ENONFINITE, "a step produced non-finite values");
    return LTS_OK;
}

lts_status lts_get_state(lts_ctx* c, double* h, double* u) {
    lts_status s = ready(c, true);
    if (s) return s;
    return c->prec == LTS_FP64 ? get_state<double>(c, h, u) : get_state<float>(c, h, u);
}

lts_status lts_get_state_device(lts_ctx* c, void* dh, void* du) {
    lts_status s = ready(c, true);
    if (s) return s;
    if (!dh || !du) return fail(c, LTS_EINVAL, "NULL output");
    const size_t nh = (size_t)c->nC * c->L, nu = (size_t)c->nE * c->L;
    std::vector<double> h(nh), u(nu);
    if ((s = lts_get_state(c, h.data(), u.data()))) return s;
    if (c->prec == LTS_FP64) {
        HIPCHK(c, hipMemcpy(dh, h.data(), nh * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(du, u.data(), nu * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> hf(h.begin(), h.end()), uf(u.begin(), u.end());
        HIPCHK(c, hipMemcpy(dh, hf.data(), nh * sizeof(float), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(du, uf.data(), nu * sizeof(float), hipMemcpyHostToDevice));
    }
    return LTS_OK;
}

lts_status lts_set_timing(lts_ctx* c, int enable) {
    if (!c) return LTS_EINVAL;
    c->timing = enable != 0;
    for (int k = 0; k < KC_N; ++k) {
        c->st_launch[k] = 0;
        c->st_ms[k] = 0;
        c->st_bytes[k] = 0;
    }
    return LTS_OK;
}

int lts_kernel_stats(lts_ctx* c, int max_classes, int64_t* launches, double* ms, double* bytes) {
    if (!c) return 0;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto& p : c->pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            c->st_launch[p.cls] += 1;
            c->st_ms[p.cls] += t;
            c->st_bytes[p.cls] += p.bytes;
        }
        c->evpool.push_back(p.a);
        c->evpool.push_back(p.b);
    }
    c->pending.clear();
    const int n = std::min(max_classes, (int)KC_N);
    for (int k = 0; k < n; ++k) {
        if (launches) launches[k] = c->st_launch[k];
        if (ms) ms[k] = c->st_ms[k];
        if (bytes) bytes[k] = c->st_bytes[k];
    }
    return n;
}

}  // extern "C"
