/*
 * FP64 CPU oracle for LTS2/LTS3 on TRiSK shallow water (arXiv 2106.07154).
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use this file.  It shares nothing with the GPU library.
 * Plain loops, no blocking or fusion: each function states the passage of the
 * paper it follows, so it can be read against the paper directly.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Reading of the paper's garbled passages.  0 is the reading this oracle
   defends; the others reproduce the literal printed text and exist only so
   tests can show that the pins reject them:
     1: Step 3.3.3 with the coarse dt instead of dt/M,
     2: Steps 3.3.3 and 4 with 2/3 x^{1st} instead of 2/3 x^{2nd},
     3: eq:weights with V_{i*} collected clockwise (read at om_create); the
        paper allows either direction and the tests show both agree. */
static int g_reading = 0;

/* Threads of the timing build (compiled with OpenMP: the per-element loops of
   the right-hand side and of the stage updates are split over threads; each
   element is still computed by the same operations in the same order, so the
   results are bitwise those of the single-threaded build).  Without OpenMP
   both calls do nothing and report one thread. */
void om_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
int om_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
void om_set_reading(int r) { g_reading = r; }
int om_get_reading(void) { return g_reading; }

struct om_ctx {
    int nC, nE, nV, maxE;
    int32_t *nEoC, *eoc, *coc, *voc, *coe, *voe, *eov, *cov;
    double *kites, *areaC, *areaT, *dc, *dv, *fV, *b;
    double g;
    /* EE(e) lists and TRiSK weights (eq:weights), CSR layout */
    int *ee_start;
    int32_t *ee;
    double *ee_w;
};

static void *dup_mem(const void *p, size_t n) {
    void *q = malloc(n ? n : 1);
    if (q && n) memcpy(q, p, n);
    return q;
}

/* n_{e,i}: +1 when n_e is outward for cell i (Appendix B, sign definitions).
   By convention n_e points from cellsOnEdge[e][0] to cellsOnEdge[e][1]. */
static double n_sign(const om_ctx *c, int e, int i) {
    return c->coe[2 * e] == i ? 1.0 : -1.0;
}

/* t_{e,v}: +1 when v is at the left end of e, i.e. in direction k x n_e. */
static double t_sign(const om_ctx *c, int e, int v) {
    return c->voe[2 * e + 1] == v ? 1.0 : -1.0;
}

/* Kite area A_{i,v}. */
static double kite_area(const om_ctx *c, int i, int v) {
    for (int k = 0; k < 3; ++k)
        if (c->cov[3 * v + k] == i) return c->kites[3 * v + k];
    return 0.0;
}

/* Weight w_{e,e'} of eq:weights.  i* is the cell owning both e and e'.  The
   vertex set V_{i*} is collected counter-clockwise around i* starting after e'
   and ending with v*, the last vertex before e (an endpoint of e). */
static double trisk_weight(const om_ctx *c, int e, int ep, int istar) {
    int n = c->nEoC[istar];
    const int32_t *eo = c->eoc + (size_t)istar * c->maxE;
    const int32_t *vo = c->voc + (size_t)istar * c->maxE;
    int a = -1, bpos = -1;
    for (int j = 0; j < n; ++j) {
        if (eo[j] == ep) a = j;
        if (eo[j] == e) bpos = j;
    }
    double sum = 0.0;
    int vstar = -1;
    if (g_reading == 3) {
        /* clockwise: vertices between edges a-1|a, a-2|a-1, ..., b|b+1 */
        for (int j = (a - 1 + n) % n; ; j = (j - 1 + n) % n) {
            int v = vo[j];
            sum += kite_area(c, istar, v) / c->areaC[istar];
            vstar = v;
            if (j == bpos) break;
        }
        return n_sign(c, ep, istar) * t_sign(c, e, vstar) * (sum - 0.5);
    }
    for (int j = a; j != bpos; j = (j + 1) % n) {
        int v = vo[j]; /* vertex between edge j and edge j+1 */
        sum += kite_area(c, istar, v) / c->areaC[istar];
        vstar = v;
    }
    return n_sign(c, ep, istar) * t_sign(c, e, vstar) * (sum - 0.5);
}

om_ctx *om_create(int nCells, int nEdges, int nVertices, int maxEdges,
                  const int32_t *nEdgesOnCell, const int32_t *edgesOnCell,
                  const int32_t *cellsOnCell, const int32_t *verticesOnCell,
                  const int32_t *cellsOnEdge, const int32_t *verticesOnEdge,
                  const int32_t *edgesOnVertex, const int32_t *cellsOnVertex,
                  const double *kiteAreasOnVertex, const double *areaCell,
                  const double *areaTriangle, const double *dcEdge,
                  const double *dvEdge, const double *fVertex,
                  const double *bottom, double gravity) {
    om_ctx *c = (om_ctx *)calloc(1, sizeof(om_ctx));
    if (!c) return NULL;
    size_t cm = (size_t)nCells * maxEdges;
    c->nC = nCells; c->nE = nEdges; c->nV = nVertices; c->maxE = maxEdges;
    c->nEoC = dup_mem(nEdgesOnCell, sizeof(int32_t) * nCells);
    c->eoc = dup_mem(edgesOnCell, sizeof(int32_t) * cm);
    c->coc = dup_mem(cellsOnCell, sizeof(int32_t) * cm);
    c->voc = dup_mem(verticesOnCell, sizeof(int32_t) * cm);
    c->coe = dup_mem(cellsOnEdge, sizeof(int32_t) * 2 * nEdges);
    c->voe = dup_mem(verticesOnEdge, sizeof(int32_t) * 2 * nEdges);
    c->eov = dup_mem(edgesOnVertex, sizeof(int32_t) * 3 * nVertices);
    c->cov = dup_mem(cellsOnVertex, sizeof(int32_t) * 3 * nVertices);
    c->kites = dup_mem(kiteAreasOnVertex, sizeof(double) * 3 * nVertices);
    c->areaC = dup_mem(areaCell, sizeof(double) * nCells);
    c->areaT = dup_mem(areaTriangle, sizeof(double) * nVertices);
    c->dc = dup_mem(dcEdge, sizeof(double) * nEdges);
    c->dv = dup_mem(dvEdge, sizeof(double) * nEdges);
    c->fV = dup_mem(fVertex, sizeof(double) * nVertices);
    c->b = dup_mem(bottom, sizeof(double) * nCells);
    c->g = gravity;

    /* EE(e): edges owned by the cells of CE(e), other than e (Appendix B). */
    c->ee_start = (int *)malloc(sizeof(int) * (nEdges + 1));
    c->ee_start[0] = 0;
    for (int e = 0; e < nEdges; ++e) {
        int cnt = 0;
        for (int s = 0; s < 2; ++s) cnt += c->nEoC[c->coe[2 * e + s]] - 1;
        c->ee_start[e + 1] = c->ee_start[e] + cnt;
    }
    int tot = c->ee_start[nEdges];
    c->ee = (int32_t *)malloc(sizeof(int32_t) * (tot ? tot : 1));
    c->ee_w = (double *)malloc(sizeof(double) * (tot ? tot : 1));
    for (int e = 0; e < nEdges; ++e) {
        int k = c->ee_start[e];
        for (int s = 0; s < 2; ++s) {
            int istar = c->coe[2 * e + s];
            for (int j = 0; j < c->nEoC[istar]; ++j) {
                int ep = c->eoc[(size_t)istar * maxEdges + j];
                if (ep == e) continue;
                c->ee[k] = ep;
                c->ee_w[k] = trisk_weight(c, e, ep, istar);
                ++k;
            }
        }
    }
    return c;
}

void om_destroy(om_ctx *c) {
    if (!c) return;
    free(c->nEoC); free(c->eoc); free(c->coc); free(c->voc); free(c->coe);
    free(c->voe); free(c->eov); free(c->cov); free(c->kites); free(c->areaC);
    free(c->areaT); free(c->dc); free(c->dv); free(c->fV); free(c->b);
    free(c->ee_start); free(c->ee); free(c->ee_w);
    free(c);
}

int om_n_edges_on_edge(const om_ctx *c, int e) {
    return c->ee_start[e + 1] - c->ee_start[e];
}

int om_weights_on_edge(const om_ctx *c, int e, int32_t *ee, double *w) {
    int n = 0;
    for (int k = c->ee_start[e]; k < c->ee_start[e + 1]; ++k, ++n) {
        ee[n] = c->ee[k];
        w[n] = c->ee_w[k];
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Discrete operators, Appendix B.                                           */

/* [h]_{i->e} = 1/2 sum_{i in CE(e)} h_i;  F_e = [h]_{i->e} u_e. */
static void thickness_flux(const om_ctx *c, const double *h, const double *u,
                           double *F) {
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < c->nE; ++e) {
        double he = 0.5 * (h[c->coe[2 * e]] + h[c->coe[2 * e + 1]]);
        F[e] = he * u[e];
    }
}

/* K_i = 1/(4 A_i) sum_{e in EC(i)} l_e d_e u_e^2. */
static void kinetic_energy(const om_ctx *c, const double *u, double *K) {
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < c->nC; ++i) {
        double s = 0.0;
        for (int j = 0; j < c->nEoC[i]; ++j) {
            int e = c->eoc[(size_t)i * c->maxE + j];
            s += c->dv[e] * c->dc[e] * u[e] * u[e];
        }
        K[i] = s / (4.0 * c->areaC[i]);
    }
}

/* Vertex potential vorticity q_v = (f_v + zeta_v) / h_v, the discrete form of
   q = eta/h (Appendix A).  The paper leaves the vertex discretisation
   implicit; this uses the circulation around the dual triangle
   zeta_v = (1/A_v) sum_{e in EV(v)} t_{e,v} d_e u_e and the kite-weighted
   thickness h_v = (1/A_v) sum_{i in CV(v)} A_{i,v} h_i. */
static void vertex_pv(const om_ctx *c, const double *h, const double *u,
                      double *q, double *zeta) {
    #pragma omp parallel for schedule(static)
    for (int v = 0; v < c->nV; ++v) {
        double circ = 0.0, hv = 0.0;
        for (int k = 0; k < 3; ++k) {
            int e = c->eov[3 * v + k];
            circ += t_sign(c, e, v) * c->dc[e] * u[e];
            hv += c->kites[3 * v + k] * h[c->cov[3 * v + k]];
        }
        double z = circ / c->areaT[v];
        hv /= c->areaT[v];
        if (zeta) zeta[v] = z;
        q[v] = (c->fV[v] + z) / hv;
    }
}

static void rhs_impl(const om_ctx *c, const double *h, const double *u,
                     double *dh, double *du, double *Kout, double *qout,
                     double *zout, double *fperp_out) {
    double *F = (double *)malloc(sizeof(double) * c->nE);
    double *K = (double *)malloc(sizeof(double) * c->nC);
    double *q = (double *)malloc(sizeof(double) * c->nV);
    double *qt = (double *)malloc(sizeof(double) * c->nE);
    thickness_flux(c, h, u, F);
    kinetic_energy(c, u, K);
    vertex_pv(c, h, u, q, zout);
    /* q~_e = 1/2 sum_{v in VE(e)} q_v (eq:discPV) */
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < c->nE; ++e)
        qt[e] = 0.5 * (q[c->voe[2 * e]] + q[c->voe[2 * e + 1]]);

    /* H_i = -[div F]_i = -(1/A_i) sum_{e in EC(i)} n_{e,i} l_e F_e */
    if (dh)
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < c->nC; ++i) {
            double s = 0.0;
            for (int j = 0; j < c->nEoC[i]; ++j) {
                int e = c->eoc[(size_t)i * c->maxE + j];
                s += n_sign(c, e, i) * c->dv[e] * F[e];
            }
            dh[i] = -s / c->areaC[i];
        }

    /* U_e = -F_perp_e[q]_{v->e} - [grad(g(h+b) + K)]_e, with
       F_perp_e[q] = sum_{e' in EE(e)} w_{e,e'} (l_{e'}/d_e) F_{e'} (q~_e+q~_{e'})/2
       (eq:discPV) and [grad phi]_e = (1/d_e) sum_{i in CE(e)} -n_{e,i} phi_i. */
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < c->nE; ++e) {
        double pv = 0.0, fp = 0.0;
        for (int k = c->ee_start[e]; k < c->ee_start[e + 1]; ++k) {
            int ep = c->ee[k];
            double t = c->ee_w[k] * c->dv[ep] / c->dc[e] * F[ep];
            fp += t;
            pv += t * 0.5 * (qt[e] + qt[ep]);
        }
        double grad = 0.0;
        for (int s = 0; s < 2; ++s) {
            int i = c->coe[2 * e + s];
            double phi = c->g * (h[i] + c->b[i]) + K[i];
            grad += -n_sign(c, e, i) * phi;
        }
        grad /= c->dc[e];
        if (du) du[e] = -pv - grad;
        if (fperp_out) fperp_out[e] = fp;
    }
    if (Kout) memcpy(Kout, K, sizeof(double) * c->nC);
    if (qout) memcpy(qout, q, sizeof(double) * c->nV);
    free(F); free(K); free(q); free(qt);
}

void om_rhs(const om_ctx *c, const double *h, const double *u, double *dh,
            double *du) {
    rhs_impl(c, h, u, dh, du, NULL, NULL, NULL, NULL);
}

void om_diag_fields(const om_ctx *c, const double *h, const double *u,
                    double *K, double *q, double *zeta, double *fperp) {
    rhs_impl(c, h, u, NULL, NULL, K, q, zeta, fperp);
}

/* ------------------------------------------------------------------------ */
/* LTS regions: eq:indexSetsCells, eq:index_sets_cells, eq:indexSetsEdges.    */

int om_regions(const om_ctx *c, const uint8_t *fine_mask, int n1, int n2,
               int8_t *cell_region, int8_t *edge_region, uint8_t *cell_fbar,
               uint8_t *edge_fbar) {
    int nC = c->nC, nE = c->nE, nf = 0;
    if (n1 < 1 || n2 < 1) return -1;
    for (int i = 0; i < nC; ++i) {
        cell_region[i] = fine_mask[i] ? OM_F : -1;
        nf += fine_mask[i] != 0;
    }
    if (nf == 0 || nf == nC) return -1;
    /* ring[i]: 0 for F, r for the r-th breadth-first ring, -1 unlabelled */
    int *ring = (int *)malloc(sizeof(int) * nC);
    for (int i = 0; i < nC; ++i) ring[i] = fine_mask[i] ? 0 : -1;
    for (int r = 1; r <= n1 + n2; ++r) {
        for (int i = 0; i < nC; ++i) {
            if (ring[i] != -1) continue;
            for (int j = 0; j < c->nEoC[i]; ++j)
                if (ring[c->coc[(size_t)i * c->maxE + j]] == r - 1) {
                    ring[i] = r;  /* shares an edge with the previous ring */
                    break;
                }
        }
    }
    for (int i = 0; i < nC; ++i) {
        if (ring[i] == 0) continue;
        if (ring[i] >= 1 && ring[i] <= n1) cell_region[i] = OM_I1;
        else if (ring[i] > n1) cell_region[i] = OM_I2;
        else cell_region[i] = OM_C;
    }
    /* F1: fine cells sharing an edge with I1; F2: other fine cells sharing an
       edge with F1; underlined F = F1 u F2. */
    uint8_t *f1 = (uint8_t *)calloc(nC, 1);
    for (int i = 0; i < nC; ++i) {
        cell_fbar[i] = 0;
        if (cell_region[i] != OM_F) continue;
        for (int j = 0; j < c->nEoC[i]; ++j)
            if (cell_region[c->coc[(size_t)i * c->maxE + j]] == OM_I1) f1[i] = 1;
    }
    for (int i = 0; i < nC; ++i) {
        if (cell_region[i] != OM_F) continue;
        if (f1[i]) { cell_fbar[i] = 1; continue; }
        for (int j = 0; j < c->nEoC[i]; ++j)
            if (f1[c->coc[(size_t)i * c->maxE + j]]) cell_fbar[i] = 1;
    }
    /* Edges go to the finest region among their two cells (fine to coarse).
       Underlined-F edges: edges of underlined-F cells that are not edges of
       cells in F minus underlined F. */
    for (int e = 0; e < nE; ++e) {
        int a = c->coe[2 * e], b = c->coe[2 * e + 1];
        int ra = cell_region[a], rb = cell_region[b];
        edge_region[e] = (int8_t)(ra > rb ? ra : rb);
        int touches_fbar = (ra == OM_F && cell_fbar[a]) || (rb == OM_F && cell_fbar[b]);
        int touches_finterior = (ra == OM_F && !cell_fbar[a]) || (rb == OM_F && !cell_fbar[b]);
        edge_fbar[e] = (uint8_t)(touches_fbar && !touches_finterior);
    }
    free(ring);
    free(f1);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Global schemes.                                                           */

/* Algorithm 2.1: SSPRK2 / SSPRK3 in the Shu-Osher stage form. */
void om_ssprk_step(const om_ctx *c, int order, double *h, double *u, double dt) {
    int nC = c->nC, nE = c->nE;
    double w_old = order == 2 ? 0.5 : 0.75, w_1 = order == 2 ? 0.5 : 0.25;
    double *h0 = dup_mem(h, sizeof(double) * nC), *u0 = dup_mem(u, sizeof(double) * nE);
    double *h1 = malloc(sizeof(double) * nC), *u1 = malloc(sizeof(double) * nE);
    double *h2 = malloc(sizeof(double) * nC), *u2 = malloc(sizeof(double) * nE);
    double *dh = malloc(sizeof(double) * nC), *du = malloc(sizeof(double) * nE);
    /* stage 1 */
    om_rhs(c, h0, u0, dh, du);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nC; ++i) h1[i] = h0[i] + dt * dh[i];
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < nE; ++e) u1[e] = u0[e] + dt * du[e];
    /* stage 2 */
    om_rhs(c, h1, u1, dh, du);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nC; ++i) h2[i] = w_old * h0[i] + w_1 * h1[i] + w_1 * dt * dh[i];
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < nE; ++e) u2[e] = w_old * u0[e] + w_1 * u1[e] + w_1 * dt * du[e];
    if (order == 2) {
        memcpy(h, h2, sizeof(double) * nC);
        memcpy(u, u2, sizeof(double) * nE);
    } else {
        /* stage 3 */
        om_rhs(c, h2, u2, dh, du);
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < nC; ++i)
            h[i] = h0[i] / 3.0 + 2.0 / 3.0 * h2[i] + 2.0 / 3.0 * dt * dh[i];
        #pragma omp parallel for schedule(static)
        for (int e = 0; e < nE; ++e)
            u[e] = u0[e] / 3.0 + 2.0 / 3.0 * u2[e] + 2.0 / 3.0 * dt * du[e];
    }
    free(h0); free(u0); free(h1); free(u1); free(h2); free(u2); free(dh); free(du);
}

/* Classical fourth-order Runge-Kutta (the paper's reference solver). */
void om_rk4_step(const om_ctx *c, double *h, double *u, double dt) {
    int nC = c->nC, nE = c->nE;
    double *ht = malloc(sizeof(double) * nC), *ut = malloc(sizeof(double) * nE);
    double *kh[4], *ku[4];
    for (int s = 0; s < 4; ++s) {
        kh[s] = malloc(sizeof(double) * nC);
        ku[s] = malloc(sizeof(double) * nE);
    }
    const double frac[4] = {0.0, 0.5, 0.5, 1.0};
    for (int s = 0; s < 4; ++s) {
        if (s == 0) {
            om_rhs(c, h, u, kh[0], ku[0]);
            continue;
        }
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < nC; ++i) ht[i] = h[i] + frac[s] * dt * kh[s - 1][i];
        #pragma omp parallel for schedule(static)
        for (int e = 0; e < nE; ++e) ut[e] = u[e] + frac[s] * dt * ku[s - 1][e];
        om_rhs(c, ht, ut, kh[s], ku[s]);
    }
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nC; ++i)
        h[i] += dt / 6.0 * (kh[0][i] + 2.0 * kh[1][i] + 2.0 * kh[2][i] + kh[3][i]);
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < nE; ++e)
        u[e] += dt / 6.0 * (ku[0][e] + 2.0 * ku[1][e] + 2.0 * ku[2][e] + ku[3][e]);
    free(ht); free(ut);
    for (int s = 0; s < 4; ++s) { free(kh[s]); free(ku[s]); }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2.2 (LTS2 / LTS3).                                              */

/* Interface-1 prediction (Steps 3.1.1, 3.2.1, 3.3.1):
   x = (1 - a - a~) x_old + (a - a~) x_1st + 2 a~ x_2nd with
   stage 0: a = k/M,          a~ = k^2/M^2            (LTS3; 0 for LTS2)
   stage 1: a = (k+1)/M,      a~ = k(k+2)/M^2         (LTS3; 0 for LTS2)
   stage 2: a = (2k+1)/(2M),  a~ = (2k^2+2k+1)/(2M^2) (LTS3 only). */
void om_lts_predict_coeffs(int order, int stage, int k, int M, double out[3]) {
    double a, at;
    double dk = (double)k, dM = (double)M;
    if (stage == 0) {
        a = dk / dM;
        at = order == 3 ? dk * dk / (dM * dM) : 0.0;
    } else if (stage == 1) {
        a = (dk + 1.0) / dM;
        at = order == 3 ? dk * (dk + 2.0) / (dM * dM) : 0.0;
    } else {
        a = (2.0 * dk + 1.0) / (2.0 * dM);
        at = (2.0 * dk * dk + 2.0 * dk + 1.0) / (2.0 * dM * dM);
    }
    out[0] = 1.0 - a - at;
    out[1] = a - at;
    out[2] = 2.0 * at;
}

void om_lts_step(const om_ctx *c, int order, const int8_t *creg,
                 const int8_t *ereg, const uint8_t *cfbar,
                 const uint8_t *efbar, double *h, double *u, double dt,
                 int M) {
    int nC = c->nC, nE = c->nE;
    size_t bc = sizeof(double) * nC, be = sizeof(double) * nE;
    double w_old = order == 2 ? 0.5 : 0.75, w_1 = order == 2 ? 0.5 : 0.25;
    double th[3];
    if (order == 2) { th[0] = 0.5; th[1] = 0.5; th[2] = 0.0; }
    else { th[0] = 1.0 / 6.0; th[1] = 1.0 / 6.0; th[2] = 2.0 / 3.0; }
    double delta = dt / M;

    /* (h,u)^old, and (h,u)^1st = (h,u)^2nd = (h,u)^old (initialisation) */
    double *h0 = dup_mem(h, bc), *u0 = dup_mem(u, be);
    double *h1 = dup_mem(h, bc), *u1 = dup_mem(u, be);
    double *h2 = dup_mem(h, bc), *u2 = dup_mem(u, be);
    double *dh = malloc(bc), *du = malloc(be);

    /* Step 1: first stage with dt on I1 u I2 u C (and underlined F for LTS3). */
    om_rhs(c, h0, u0, dh, du);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nC; ++i)
        if (creg[i] != OM_F || (order == 3 && cfbar[i])) h1[i] = h0[i] + dt * dh[i];
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < nE; ++e)
        if (ereg[e] != OM_F || (order == 3 && efbar[e])) u1[e] = u0[e] + dt * du[e];

    /* Step 2: second stage with dt on C (LTS2) or I1 u I2 u C (LTS3). */
    om_rhs(c, h1, u1, dh, du);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nC; ++i)
        if (creg[i] == OM_C || (order == 3 && creg[i] != OM_F))
            h2[i] = w_old * h0[i] + w_1 * h1[i] + w_1 * dt * dh[i];
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < nE; ++e)
        if (ereg[e] == OM_C || (order == 3 && ereg[e] != OM_F))
            u2[e] = w_old * u0[e] + w_1 * u1[e] + w_1 * dt * du[e];

    /* Step 3: fine substeps.  The substep states start from the coarse stages;
       cells and edges outside F u I1 keep the coarse stage value of the stage
       being evaluated (old, 1st, 2nd) throughout the loop. */
    double *hk[3] = {dup_mem(h0, bc), dup_mem(h1, bc), dup_mem(h2, bc)};
    double *uk[3] = {dup_mem(u0, be), dup_mem(u1, be), dup_mem(u2, be)};
    double *Hacc[3], *Uacc[3];
    for (int s = 0; s < 3; ++s) {
        Hacc[s] = calloc(nC, sizeof(double));
        Uacc[s] = calloc(nE, sizeof(double));
    }
    int nstage = order == 3 ? 3 : 2;
    /* stage-3 operands: the defended reading uses x^{2nd,k} and dt/M */
    int lit2 = g_reading == 2 ? 1 : 2;
    double dfin = g_reading == 1 ? dt : delta;
    double *h_s3 = g_reading == 2 ? h1 : h2, *u_s3 = g_reading == 2 ? u1 : u2;
    for (int k = 0; k < M; ++k) {
        for (int s = 0; s < nstage; ++s) {
            /* Step 3.s.1: predict interface 1 at this fine stage. */
            double cf[3];
            om_lts_predict_coeffs(order, s, k, M, cf);
            #pragma omp parallel for schedule(static)
            for (int i = 0; i < nC; ++i)
                if (creg[i] == OM_I1)
                    hk[s][i] = cf[0] * h0[i] + cf[1] * h1[i] + cf[2] * h2[i];
            #pragma omp parallel for schedule(static)
            for (int e = 0; e < nE; ++e)
                if (ereg[e] == OM_I1)
                    uk[s][e] = cf[0] * u0[e] + cf[1] * u1[e] + cf[2] * u2[e];
            om_rhs(c, hk[s], uk[s], dh, du);
            /* Step 3.s.2: accumulate correction terms on I1 u I2. */
            #pragma omp parallel for schedule(static)
            for (int i = 0; i < nC; ++i)
                if (creg[i] == OM_I1 || creg[i] == OM_I2) Hacc[s][i] += dh[i];
            #pragma omp parallel for schedule(static)
            for (int e = 0; e < nE; ++e)
                if (ereg[e] == OM_I1 || ereg[e] == OM_I2) Uacc[s][e] += du[e];
            /* Step 3.s.3: SSPRK stage with dt/M on all fine cells and edges. */
            #pragma omp parallel for schedule(static)
            for (int i = 0; i < nC; ++i) {
                if (creg[i] != OM_F) continue;
                if (s == 0)
                    hk[1][i] = hk[0][i] + delta * dh[i];
                else if (s == 1 && order == 3)
                    hk[2][i] = w_old * hk[0][i] + w_1 * hk[1][i] + w_1 * delta * dh[i];
                else if (s == 1) /* LTS2: the second stage gives the new value */
                    hk[0][i] = w_old * hk[0][i] + w_1 * hk[1][i] + w_1 * delta * dh[i];
                else
                    hk[0][i] = hk[0][i] / 3.0 + 2.0 / 3.0 * hk[lit2][i] + 2.0 / 3.0 * dfin * dh[i];
            }
            #pragma omp parallel for schedule(static)
            for (int e = 0; e < nE; ++e) {
                if (ereg[e] != OM_F) continue;
                if (s == 0)
                    uk[1][e] = uk[0][e] + delta * du[e];
                else if (s == 1 && order == 3)
                    uk[2][e] = w_old * uk[0][e] + w_1 * uk[1][e] + w_1 * delta * du[e];
                else if (s == 1)
                    uk[0][e] = w_old * uk[0][e] + w_1 * uk[1][e] + w_1 * delta * du[e];
                else
                    uk[0][e] = uk[0][e] / 3.0 + 2.0 / 3.0 * uk[lit2][e] + 2.0 / 3.0 * dfin * du[e];
            }
        }
    }

    /* Step 4: coarse region (LTS3 third stage, LTS2 takes the second stage). */
    if (order == 3) om_rhs(c, h2, u2, dh, du);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nC; ++i)
        if (creg[i] == OM_C)
            h[i] = order == 3 ? h0[i] / 3.0 + 2.0 / 3.0 * h_s3[i] + 2.0 / 3.0 * dt * dh[i] : h2[i];
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < nE; ++e)
        if (ereg[e] == OM_C)
            u[e] = order == 3 ? u0[e] / 3.0 + 2.0 / 3.0 * u_s3[e] + 2.0 / 3.0 * dt * du[e] : u2[e];

    /* Step 5: interface correction; the fine region takes the last substep. */
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nC; ++i) {
        if (creg[i] == OM_I1 || creg[i] == OM_I2)
            h[i] = h0[i] + delta * (th[0] * Hacc[0][i] + th[1] * Hacc[1][i] + th[2] * Hacc[2][i]);
        else if (creg[i] == OM_F)
            h[i] = hk[0][i];
    }
    #pragma omp parallel for schedule(static)
    for (int e = 0; e < nE; ++e) {
        if (ereg[e] == OM_I1 || ereg[e] == OM_I2)
            u[e] = u0[e] + delta * (th[0] * Uacc[0][e] + th[1] * Uacc[1][e] + th[2] * Uacc[2][e]);
        else if (ereg[e] == OM_F)
            u[e] = uk[0][e];
    }

    free(h0); free(u0); free(h1); free(u1); free(h2); free(u2); free(dh); free(du);
    for (int s = 0; s < 3; ++s) {
        free(hk[s]); free(uk[s]); free(Hacc[s]); free(Uacc[s]);
    }
}

/* ------------------------------------------------------------------------ */
/* More than two LTS levels (Remark 3.1): nested fine regions with an integer */
/* step ratio between neighbouring levels.                                   */
/*
   Level 0 is Algorithm 2.2 (LTS3) on the whole mesh with fine region F_0 and
   ratio M[0].  The fine substeps of level l (size dt_l / M[l]) are not
   SSPRK3 stages but LTS3 steps of level l+1 on the domain D_{l+1} = F_l, with
   fine region F_{l+1} inside F_l and ratio M[l+1]; the deepest level takes
   plain SSPRK3 substeps.  Every level's Steps 1, 2 and 4 evaluate the
   right-hand side on the whole mesh, with the values outside its domain held
   at the enclosing level's stage of the same index (the enclosing interface 1
   predicted, its interface 2 and coarse region at the coarse stage).  Those
   same evaluations give the enclosing level's interface accumulation
   (Steps 3.s.2): near the enclosing interface the domain's cells are coarse
   cells of the inner level, whose three coarse stages are exactly SSPRK3
   stages of the enclosing fine step.  This needs every inner fine and
   interface cell to lie at least three cell rings inside the domain
   (om_mlts_regions checks it).  Labels of level l: creg[l*nC + i],
   ereg[l*nE + e], cfbar, efbar as om_regions gives them for F_l. */

typedef struct {
    int nlev;              /* LTS levels (fine regions + 1) */
    const int8_t *creg, *ereg;
    const uint8_t *cfbar, *efbar;
    const int *M;          /* M[l]: step ratio of level l to level l+1 */
} ml_levels;

static int ml_in_domain_cell(const om_ctx *c, const ml_levels *L, int l, int i) {
    return l == 0 || L->creg[(size_t)(l - 1) * c->nC + i] == OM_F;
}
static int ml_in_domain_edge(const om_ctx *c, const ml_levels *L, int l, int e) {
    return l == 0 || L->ereg[(size_t)(l - 1) * c->nE + e] == OM_F;
}
/* the enclosing level's interface (I1 u I2 of level l-1) */
static int ml_outer_iface_cell(const om_ctx *c, const ml_levels *L, int l, int i) {
    if (l == 0) return 0;
    int r = L->creg[(size_t)(l - 1) * c->nC + i];
    return r == OM_I1 || r == OM_I2;
}
static int ml_outer_iface_edge(const om_ctx *c, const ml_levels *L, int l, int e) {
    if (l == 0) return 0;
    int r = L->ereg[(size_t)(l - 1) * c->nE + e];
    return r == OM_I1 || r == OM_I2;
}

/* One LTS3 step of size dt on level l's domain.  xh[s], xu[s] (s = 0, 1, 2)
   are full-mesh arrays.  On entry xh[0], xu[0] hold the step's start values on
   the domain; outside the domain xh[s], xu[s] hold the enclosing level's
   values at this step's stage s.  On return xh[0], xu[0] hold the end values
   on the domain (xh[1..2], xu[1..2] are overwritten on the domain).  aH[s],
   aU[s] (NULL at level 0): the enclosing level's interface accumulators, to
   which the right-hand side of this step's stage s is added. */
static void ml_step(const om_ctx *c, const ml_levels *L, int l, double dt,
                    double *xh[3], double *xu[3], double *aH[3], double *aU[3]) {
    int nC = c->nC, nE = c->nE, M = L->M[l];
    size_t bc = sizeof(double) * nC, be = sizeof(double) * nE;
    const int8_t *cr = L->creg + (size_t)l * nC, *er = L->ereg + (size_t)l * nE;
    const uint8_t *cf = L->cfbar + (size_t)l * nC, *ef = L->efbar + (size_t)l * nE;
    const double th[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
    double delta = dt / M;
    double *h0 = dup_mem(xh[0], bc), *u0 = dup_mem(xu[0], be);
    double *dh = malloc(bc), *du = malloc(be);

    /* Step 1: first stage with dt on underlined F, I1, I2, C of this level */
    om_rhs(c, xh[0], xu[0], dh, du);
    for (int i = 0; i < nC; ++i) {
        if (aH && ml_outer_iface_cell(c, L, l, i)) aH[0][i] += dh[i];
        if (!ml_in_domain_cell(c, L, l, i)) continue;
        xh[1][i] = (cr[i] != OM_F || cf[i]) ? h0[i] + dt * dh[i] : h0[i];
    }
    for (int e = 0; e < nE; ++e) {
        if (aU && ml_outer_iface_edge(c, L, l, e)) aU[0][e] += du[e];
        if (!ml_in_domain_edge(c, L, l, e)) continue;
        xu[1][e] = (er[e] != OM_F || ef[e]) ? u0[e] + dt * du[e] : u0[e];
    }
    /* Step 2: second stage with dt on I1, I2, C of this level */
    om_rhs(c, xh[1], xu[1], dh, du);
    for (int i = 0; i < nC; ++i) {
        if (aH && ml_outer_iface_cell(c, L, l, i)) aH[1][i] += dh[i];
        if (!ml_in_domain_cell(c, L, l, i)) continue;
        xh[2][i] = cr[i] != OM_F ? 0.75 * h0[i] + 0.25 * xh[1][i] + 0.25 * dt * dh[i] : h0[i];
    }
    for (int e = 0; e < nE; ++e) {
        if (aU && ml_outer_iface_edge(c, L, l, e)) aU[1][e] += du[e];
        if (!ml_in_domain_edge(c, L, l, e)) continue;
        xu[2][e] = er[e] != OM_F ? 0.75 * u0[e] + 0.25 * xu[1][e] + 0.25 * dt * du[e] : u0[e];
    }

    /* Step 3: M substeps on F of this level.  zh[s], zu[s]: the substep stage
       states, starting from the coarse stages (so F starts at the step's
       start values); outside F they keep this level's coarse stage s
       (interface 1 is predicted per substep). */
    double *zh[3], *zu[3], *Hacc[3], *Uacc[3];
    for (int s = 0; s < 3; ++s) {
        zh[s] = dup_mem(xh[s], bc);
        zu[s] = dup_mem(xu[s], be);
        Hacc[s] = calloc(nC, sizeof(double));
        Uacc[s] = calloc(nE, sizeof(double));
    }
    int inner = l + 1 < L->nlev - 1;
    for (int k = 0; k < M; ++k) {
        if (inner) {
            /* interface-1 predictions for the three stages of substep k, then
               one LTS3 step of the next level on F (its Steps 1, 2 and 4 add
               this level's accumulation terms) */
            for (int s = 0; s < 3; ++s) {
                double q[3];
                om_lts_predict_coeffs(3, s, k, M, q);
                for (int i = 0; i < nC; ++i)
                    if (ml_in_domain_cell(c, L, l, i) && cr[i] == OM_I1)
                        zh[s][i] = q[0] * h0[i] + q[1] * xh[1][i] + q[2] * xh[2][i];
                for (int e = 0; e < nE; ++e)
                    if (ml_in_domain_edge(c, L, l, e) && er[e] == OM_I1)
                        zu[s][e] = q[0] * u0[e] + q[1] * xu[1][e] + q[2] * xu[2][e];
            }
            ml_step(c, L, l + 1, delta, zh, zu, Hacc, Uacc);
            continue;
        }
        for (int s = 0; s < 3; ++s) {
            /* Step 3.s.1: predict interface 1 */
            double q[3];
            om_lts_predict_coeffs(3, s, k, M, q);
            for (int i = 0; i < nC; ++i)
                if (ml_in_domain_cell(c, L, l, i) && cr[i] == OM_I1)
                    zh[s][i] = q[0] * h0[i] + q[1] * xh[1][i] + q[2] * xh[2][i];
            for (int e = 0; e < nE; ++e)
                if (ml_in_domain_edge(c, L, l, e) && er[e] == OM_I1)
                    zu[s][e] = q[0] * u0[e] + q[1] * xu[1][e] + q[2] * xu[2][e];
            om_rhs(c, zh[s], zu[s], dh, du);
            /* Step 3.s.2: accumulate on I1 u I2 of this level */
            for (int i = 0; i < nC; ++i)
                if (ml_in_domain_cell(c, L, l, i) && (cr[i] == OM_I1 || cr[i] == OM_I2))
                    Hacc[s][i] += dh[i];
            for (int e = 0; e < nE; ++e)
                if (ml_in_domain_edge(c, L, l, e) && (er[e] == OM_I1 || er[e] == OM_I2))
                    Uacc[s][e] += du[e];
            /* Step 3.s.3: SSPRK3 stage with dt/M on F of this level */
            for (int i = 0; i < nC; ++i) {
                if (cr[i] != OM_F || !ml_in_domain_cell(c, L, l, i)) continue;
                if (s == 0) zh[1][i] = zh[0][i] + delta * dh[i];
                else if (s == 1) zh[2][i] = 0.75 * zh[0][i] + 0.25 * zh[1][i] + 0.25 * delta * dh[i];
                else zh[0][i] = zh[0][i] / 3.0 + 2.0 / 3.0 * zh[2][i] + 2.0 / 3.0 * delta * dh[i];
            }
            for (int e = 0; e < nE; ++e) {
                if (er[e] != OM_F || !ml_in_domain_edge(c, L, l, e)) continue;
                if (s == 0) zu[1][e] = zu[0][e] + delta * du[e];
                else if (s == 1) zu[2][e] = 0.75 * zu[0][e] + 0.25 * zu[1][e] + 0.25 * delta * du[e];
                else zu[0][e] = zu[0][e] / 3.0 + 2.0 / 3.0 * zu[2][e] + 2.0 / 3.0 * delta * du[e];
            }
        }
    }

    /* Step 4: third stage with dt on C of this level */
    om_rhs(c, xh[2], xu[2], dh, du);
    for (int i = 0; i < nC; ++i)
        if (aH && ml_outer_iface_cell(c, L, l, i)) aH[2][i] += dh[i];
    for (int e = 0; e < nE; ++e)
        if (aU && ml_outer_iface_edge(c, L, l, e)) aU[2][e] += du[e];
    /* Step 5 and the new values on the domain */
    for (int i = 0; i < nC; ++i) {
        if (!ml_in_domain_cell(c, L, l, i)) continue;
        if (cr[i] == OM_C)
            xh[0][i] = h0[i] / 3.0 + 2.0 / 3.0 * xh[2][i] + 2.0 / 3.0 * dt * dh[i];
        else if (cr[i] == OM_F)
            xh[0][i] = zh[0][i];
        else
            xh[0][i] = h0[i] + delta * (th[0] * Hacc[0][i] + th[1] * Hacc[1][i] + th[2] * Hacc[2][i]);
    }
    for (int e = 0; e < nE; ++e) {
        if (!ml_in_domain_edge(c, L, l, e)) continue;
        if (er[e] == OM_C)
            xu[0][e] = u0[e] / 3.0 + 2.0 / 3.0 * xu[2][e] + 2.0 / 3.0 * dt * du[e];
        else if (er[e] == OM_F)
            xu[0][e] = zu[0][e];
        else
            xu[0][e] = u0[e] + delta * (th[0] * Uacc[0][e] + th[1] * Uacc[1][e] + th[2] * Uacc[2][e]);
    }
    free(h0); free(u0); free(dh); free(du);
    for (int s = 0; s < 3; ++s) {
        free(zh[s]); free(zu[s]); free(Hacc[s]); free(Uacc[s]);
    }
}

void om_mlts_step(const om_ctx *c, int nlev, const int8_t *creg, const int8_t *ereg,
                  const uint8_t *cfbar, const uint8_t *efbar, const int32_t *M,
                  double *h, double *u, double dt) {
    size_t bc = sizeof(double) * c->nC, be = sizeof(double) * c->nE;
    int Mi[16];
    for (int l = 0; l < nlev - 1 && l < 16; ++l) Mi[l] = M[l];
    ml_levels L = {nlev, creg, ereg, cfbar, efbar, Mi};
    double *xh[3] = {h, dup_mem(h, bc), dup_mem(h, bc)};
    double *xu[3] = {u, dup_mem(u, be), dup_mem(u, be)};
    ml_step(c, &L, 0, dt, xh, xu, NULL, NULL);
    free(xh[1]); free(xh[2]); free(xu[1]); free(xu[2]);
}

int om_mlts_regions(const om_ctx *c, int nlev, const uint8_t *masks, int n1, int n2,
                    int8_t *creg, int8_t *ereg, uint8_t *cfbar, uint8_t *efbar) {
    int nC = c->nC;
    if (nlev < 2 || nlev > 16) return -1;
    for (int l = 0; l < nlev - 1; ++l)
        if (om_regions(c, masks + (size_t)l * nC, n1, n2, creg + (size_t)l * nC,
                       ereg + (size_t)l * c->nE, cfbar + (size_t)l * nC,
                       efbar + (size_t)l * c->nE) != 0)
            return -1;
    /* nesting: the fine, interface-1 and interface-2 cells of level l lie at
       least three rings inside F of level l-1 (depth: ring distance from the
       cells outside it, 0, 1, 2, or -1 for three and more), so every value
       their right-hand side reads lies inside and the two fine rings next to
       the enclosing interface 1 are coarse cells of level l */
    int *depth = (int *)malloc(sizeof(int) * nC);
    int ok = 1;
    for (int l = 1; l < nlev - 1 && ok; ++l) {
        const int8_t *outer = creg + (size_t)(l - 1) * nC, *cr = creg + (size_t)l * nC;
        for (int i = 0; i < nC; ++i) depth[i] = outer[i] == OM_F ? -1 : 0;
        for (int r = 1; r <= 2; ++r)
            for (int i = 0; i < nC; ++i) {
                if (depth[i] != -1) continue;
                for (int j = 0; j < c->nEoC[i]; ++j)
                    if (depth[c->coc[(size_t)i * c->maxE + j]] == r - 1) {
                        depth[i] = r;
                        break;
                    }
            }
        for (int i = 0; i < nC; ++i)
            if (cr[i] != OM_C && depth[i] != -1) ok = 0;
    }
    free(depth);
    return ok ? 0 : -1;
}

/* ------------------------------------------------------------------------ */

static void neumaier_add(double *sum, double *comp, double x) {
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

void om_diagnostics(const om_ctx *c, const double *h, const double *u,
                    double *mass, double *energy) {
    double *K = (double *)malloc(sizeof(double) * c->nC);
    kinetic_energy(c, u, K);
    double ms = 0, mc = 0, es = 0, ec = 0;
    for (int i = 0; i < c->nC; ++i) {
        double A = c->areaC[i];
        neumaier_add(&ms, &mc, A * h[i]);
        neumaier_add(&es, &ec, A * (h[i] * K[i] + c->g * (0.5 * h[i] * h[i] + h[i] * c->b[i])));
    }
    *mass = ms + mc;
    *energy = es + ec;
    free(K);
}
