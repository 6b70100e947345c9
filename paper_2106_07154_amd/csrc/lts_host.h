// Host-side internals of liblts shared by the single-mesh runtime
// (lts_api.cpp) and the ensemble runtime (lts_ensemble.cpp).  Not public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lts_internal.h"

namespace lts {

enum PassKind { P_FULL = 0, P_STEP1, P_STEP2, P_STEP3, P_STEP4, P_N };


struct PassPlan {
    int c_lo = 0, c_hi = 0;    // cell kernel range (targets plus cells of target edges)
    int v_lo = 0, v_hi = 0;    // vertex kernel range
    int w_lo = 0, w_hi = 0;    // cells of the cell range with more than 8 edges (wide list)
    int ct_lo = 0, ct_hi = 0;  // target cells
    int et_lo = 0, et_hi = 0;  // target edges
    // algorithmic bytes of the gathers, per element type (counts of unique
    // elements touched), filled at upload
    long v_uniq_u = 0, v_uniq_h = 0;
    long c_uniq_h = 0, c_uniq_u = 0, c_uniq_q = 0, c_slots = 0;
};

struct TimedLaunch {
    int cls;
    hipEvent_t a, b;
    double bytes;
};

// One level of a multi-level LTS3 (Remark 3.1).  Level 0 is the whole mesh;
// level l >= 1 lives in level l-1's fine region, whose interior cells
// [0, cb_{l-1}[1]) it orders by its own classes (its coarse part then runs on
// through level l-1's underlined-F cells to cb_{l-1}[3]).
struct LevelData {
    int cb[8] = {0};  // cell class starts inside the level's domain, cb[7]: domain end
    int eb[6] = {0};  // edge class starts, eb[5]: domain end
    PassPlan p1, p2, p3, p4;  // Steps 1, 2, 4 (with the enclosing accumulation), Step 3
    void *x0h = nullptr, *x1h = nullptr, *x2h = nullptr;  // interface-1 copies
    void *x0u = nullptr, *x1u = nullptr, *x2u = nullptr;
    void *acch = nullptr, *accu = nullptr;                 // interface accumulators
    std::vector<int8_t> creg, ereg;                        // caller numbering
    std::vector<uint8_t> cfbar, efbar;
};

}  // namespace lts

struct lts_ctx {
    int device = 0;
    lts_precision prec = LTS_FP64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    bool has_mesh = false, has_state = false, nonfinite = false;
    int nC = 0, nE = 0, nV = 0, maxE = 0;
    int L = 1;  // independent layers; per-element device arrays are [element][L]
    double g = 9.81;
    std::vector<int32_t> cperm, cinv, eperm, einv, vperm, vinv;  // perm: new->old, inv: old->new
    std::vector<int32_t> wide;  // device positions of cells with more than 8 edges
    std::vector<int8_t> creg, ereg;                              // caller numbering
    std::vector<uint8_t> cfbar, efbar;
    int cb[8] = {0};  // cell class starts: Fint F2 F1 I1 I2 C1 Crest end
    int eb[6] = {0};  // edge class starts: Fint Fbar I1 I2 C end
    lts::PassPlan plan[lts::P_N];
    lts::PassPlan iface_plan;  // targets I1 u I2 (cells and edges) only
    // multi-level LTS3: levels 0 .. lv.size()-1 (empty for a two-level mesh)
    std::vector<lts::LevelData> lv;
    std::vector<int> run_Ms, g_Ms;  // step ratios of the run / of the cached graph

    // device memory (typed by prec); all owned
    std::vector<void*> allocs;
    void* dm = nullptr;  // DevMesh<T>*
    void *Ah = nullptr, *Au = nullptr, *Bh = nullptr, *Bu = nullptr, *Ch = nullptr, *Cu = nullptr;
    void *x0h = nullptr, *x1h = nullptr, *x2h = nullptr, *x0u = nullptr, *x1u = nullptr,
         *x2u = nullptr;
    void *acch = nullptr, *accu = nullptr, *zs = nullptr, *q = nullptr;
    void *Qh = nullptr, *Qu = nullptr;  // RK4 stage sums (allocated on first use)
    int* flag = nullptr;
    double *dpart = nullptr, *dout = nullptr;

    double t = 0.0;
    int64_t steps = 0;
    int64_t gate_fallbacks = 0;  // surrogate steps rejected by the gate

    // perturbation thickness form (FP32): state holds eta = h - href
    bool pert = false;
    std::vector<double> href_host;           // device order, value of the stored href
    std::vector<double> bot_perm, area_perm; // device order
    void *d_href = nullptr, *d_beta = nullptr;

    // graph cache for one step of one scheme
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int g_kind = -1, g_M = 0;
    double g_dt = 0.0;


    // timing
    bool timing = false;
    std::vector<lts::TimedLaunch> pending;
    std::vector<hipEvent_t> evpool;
    int64_t st_launch[lts::KC_N] = {0};
    double st_ms[lts::KC_N] = {0}, st_bytes[lts::KC_N] = {0};
};

namespace lts {

lts_status fail(lts_ctx* c, lts_status s, const std::string& msg);
size_t tsize(const lts_ctx* c);
lts_status dalloc(lts_ctx* c, void** p, size_t bytes);

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::lts::fail(ctx, LTS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// One right-hand-side pass as recorded instead of launched (the ensemble
// batches the passes of many members into shared launches).
template <typename T>
struct PassRecord {
    PassPlan plan;
    const T* h;
    const T* u;
    Seg<T> cs0, cs1, es0, es1;
    Aux<T> aux, aux2;
};

// ---------------------------------------------------------------- launches
// Algorithmic bytes of one kernel of a pass: every array element the kernel
// needs, read or written once (T-sized state and coefficients, int32 indices).
template <typename T>
double seg_bytes(const Seg<T>& g) {
    if (!g.mode || g.hi <= g.lo) return 0.0;
    const double n = g.hi - g.lo;
    double b = 0.0;
    if (g.mode == 1) {
        b = n * sizeof(T) * (1 + (g.xold ? 1 : 0) + (g.xcur ? 1 : 0));
        if (g.acc) b += n * sizeof(T) * (g.first ? 1 : 2);
        if (g.mhi > g.mlo) b += (g.mhi - g.mlo) * sizeof(T) * ((g.mnew ? 1 : 0) + (g.mcur ? 1 : 0));
    } else {
        b = n * sizeof(T) * (g.first ? 1 : 2);
    }
    return b;
}

// With L layers the mesh tables count once and every state term L times (aux
// counts are already in flat element x layer units).
template <typename T>
double kernel_bytes(const PassPlan& P, int kclass, const Seg<T>& s0, const Seg<T>& s1,
                    const Aux<T>& aux, int L = 1) {
    const double ts = sizeof(T);
    if (kclass == KC_VERTEX)
        return (P.v_hi - P.v_lo) * (3 * 4 * 2 + 7 * ts) +
               L * ((P.v_hi - P.v_lo) * ts + (P.v_uniq_u + P.v_uniq_h) * ts);
    // per cell: the slot record {first entry, n_i} (8 bytes), beta_i and
    // 1/A_i, plus S_n in the single-layer kernel (the layered one sums the
    // kite fractions itself); per real slot: three indices and four
    // coefficients (the tables hold no padding)
    if (kclass == KC_CELL)
        return (P.c_hi - P.c_lo) * (8 + (L > 1 ? 2 : 3) * ts) + P.c_slots * (3 * 4 + 4 * ts) +
               L * (P.c_slots * ts + (P.c_uniq_h + P.c_uniq_u + P.c_uniq_q) * ts +
                    seg_bytes(s0) + seg_bytes(s1));
    return L * ((P.et_hi - P.et_lo) * 2.0 * ts + seg_bytes(s0) + seg_bytes(s1)) +
           (aux.kind == 1 ? 4.0 : aux.kind == 2 ? 3.0 : 0.0) * (aux.nh + aux.nu) * ts;
}

// Enqueues the passes of one step of a scheme for one context: launches them
// on stream s (event-stamped when timed), or, when rec is set, records them so
// the ensemble can batch them with other members' passes.
template <typename T>
struct Run {
    lts_ctx* c;
    const DevMesh<T>& dm;
    hipStream_t s;
    bool timed;
    std::vector<PassRecord<T>>* rec = nullptr;

    // Two events for an event-stamped launch (timing mode only).
    lts_status events(hipEvent_t* a, hipEvent_t* b) {
        *a = *b = nullptr;
        if (!timed) return LTS_OK;
        while (c->evpool.size() < 2) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->evpool.push_back(e);
        }
        *a = c->evpool.back();
        c->evpool.pop_back();
        *b = c->evpool.back();
        c->evpool.pop_back();
        return LTS_OK;
    }
    void done(int cls, hipEvent_t a, hipEvent_t b, double bytes) {
        if (timed) c->pending.push_back({cls, a, b, bytes});
    }

    // One right-hand-side pass of kind p over state (h, u) with epilogues.
    lts_status pass(int p, const T* h, const T* u, const Seg<T>& cs0, const Seg<T>& cs1,
                    const Seg<T>& es0, const Seg<T>& es1, const Aux<T>& aux = Aux<T>()) {
        return pass_plan(c->plan[p], h, u, cs0, cs1, es0, es1, aux);
    }

    // The same with an explicit plan and up to two appended element-wise jobs.
    lts_status pass_plan(const PassPlan& P, const T* h, const T* u, const Seg<T>& cs0,
                         const Seg<T>& cs1, const Seg<T>& es0, const Seg<T>& es1,
                         const Aux<T>& aux, const Aux<T>& aux2 = Aux<T>()) {
        if (rec) {
            rec->push_back(PassRecord<T>{P, h, u, cs0, cs1, es0, es1, aux, aux2});
            return LTS_OK;
        }
        T* q = static_cast<T*>(c->q);
        T* zs = static_cast<T*>(c->zs);
        hipEvent_t e0, e1;
        lts_status st;
        if (c->L > 1) {  // layered: one thread per (element, layer)
            const int L = c->L;
            if ((st = events(&e0, &e1))) return st;
            HIPCHK(c, launch_vertex_l<T>(dm, h, u, q, P.v_lo, P.v_hi, L, s, e0, e1));
            done(KC_VERTEX, e0, e1, kernel_bytes<T>(P, KC_VERTEX, cs0, cs1, aux, L));
            if ((st = events(&e0, &e1))) return st;
            HIPCHK(c, launch_cell_l<T>(dm, h, u, q, zs, P.c_lo, P.c_hi, L, (T)c->g, cs0, cs1,
                                       c->flag, s, e0, e1));
            done(KC_CELL, e0, e1, kernel_bytes<T>(P, KC_CELL, cs0, cs1, aux, L));
            if ((st = events(&e0, &e1))) return st;
            HIPCHK(c, launch_edge_l<T>(zs, c->nE, P.et_lo, P.et_hi, L, es0, es1, aux, c->flag, s,
                                       e0, e1, aux2));
            done(KC_EDGE, e0, e1, kernel_bytes<T>(P, KC_EDGE, es0, es1, aux, L));
            return LTS_OK;
        }
        // vertex PV, then the cell tendency
        if ((st = events(&e0, &e1))) return st;
        HIPCHK(c, launch_vertex<T>(dm, h, u, q, P.v_lo, P.v_hi, s, e0, e1));
        done(KC_VERTEX, e0, e1, kernel_bytes<T>(P, KC_VERTEX, cs0, cs1, aux));
        if ((st = events(&e0, &e1))) return st;
        HIPCHK(c, launch_cell<T>(dm, h, u, q, zs, P.c_lo, P.c_hi, P.w_lo, P.w_hi, (T)c->g, cs0,
                                 cs1, c->flag, s, e0, e1));
        done(KC_CELL, e0, e1, kernel_bytes<T>(P, KC_CELL, cs0, cs1, aux));
        // edge tendency (+ appended element-wise job)
        if ((st = events(&e0, &e1))) return st;
        HIPCHK(c, launch_edge<T>(zs, c->nE, P.et_lo, P.et_hi, es0, es1, aux, c->flag, s, e0, e1,
                                 aux2));
        done(KC_EDGE, e0, e1,
             kernel_bytes<T>(P, KC_EDGE, es0, es1, aux) + kernel_bytes<T>(PassPlan(), KC_EDGE,
                                                                          Seg<T>(), Seg<T>(), aux2));
        return LTS_OK;
    }

    static Seg<T> upd(int lo, int hi, T* out, const T* xold, double a_old, const T* xcur,
                      double a_cur, double a_dt) {
        Seg<T> g;
        g.lo = lo;
        g.hi = hi;
        g.mode = hi > lo ? 1 : 0;
        g.out = out;
        g.xold = xold;
        g.a_old = (T)a_old;
        g.xcur = xcur;
        g.a_cur = (T)a_cur;
        g.a_dt = (T)a_dt;
        g.convex = xold && xcur && a_old + a_cur == 1.0;
        return g;
    }
    static Seg<T> mirror(Seg<T> g, int mlo, int mhi, T* mnew, T* mcur) {
        g.mlo = mlo;
        g.mhi = mhi;
        g.mnew = mnew;
        g.mcur = mcur;
        return g;
    }
    Aux<T> predict_aux(T* xh, T* xu, int stage, int k, int M, int order = 3) {
        Aux<T> x;
        double cf[3];
        predict_coeffs(stage, k, M, cf, order);
        x.kind = 1;
        x.nh = (c->cb[4] - c->cb[3]) * c->L;  // flat element x layer units
        x.nu = (c->eb[3] - c->eb[2]) * c->L;
        x.lo_h = c->cb[3] * c->L;
        x.lo_u = c->eb[2] * c->L;
        x.xh = xh;
        x.xu = xu;
        x.ah = (T*)c->x0h; x.bh = (T*)c->x1h; x.ch = (T*)c->x2h;
        x.au = (T*)c->x0u; x.bu = (T*)c->x1u; x.cu = (T*)c->x2u;
        x.c0 = cf[0]; x.c1 = cf[1]; x.c2 = cf[2];
        return x;
    }
    Aux<T> correct_aux(double delta) {
        Aux<T> x;
        x.kind = 2;
        x.nh = (c->cb[5] - c->cb[3]) * c->L;  // flat element x layer units
        x.nu = (c->eb[4] - c->eb[2]) * c->L;
        x.nbh = (c->cb[4] - c->cb[3]) * c->L;
        x.nbu = (c->eb[3] - c->eb[2]) * c->L;
        x.lo_h = c->cb[3] * c->L;
        x.lo_u = c->eb[2] * c->L;
        x.xh = (T*)c->Ah;
        x.xu = (T*)c->Au;
        x.ah = (T*)c->x0h; x.bh = (T*)c->acch;
        x.au = (T*)c->x0u; x.bu = (T*)c->accu;
        x.c0 = delta;
        return x;
    }
    // Level-l forms of predict_aux / correct_aux (multi-level LTS3).
    Aux<T> predict_aux_level(int l, T* xh, T* xu, int stage, int k, int M) {
        const LevelData& V = c->lv[l];
        Aux<T> x;
        double cf[3];
        predict_coeffs(stage, k, M, cf, 3);
        x.kind = 1;
        x.nh = (V.cb[4] - V.cb[3]) * c->L;  // flat element x layer units
        x.nu = (V.eb[3] - V.eb[2]) * c->L;
        x.lo_h = V.cb[3] * c->L;
        x.lo_u = V.eb[2] * c->L;
        x.xh = xh;
        x.xu = xu;
        x.ah = (T*)V.x0h; x.bh = (T*)V.x1h; x.ch = (T*)V.x2h;
        x.au = (T*)V.x0u; x.bu = (T*)V.x1u; x.cu = (T*)V.x2u;
        x.c0 = cf[0]; x.c1 = cf[1]; x.c2 = cf[2];
        return x;
    }
    Aux<T> correct_aux_level(int l, double delta) {
        const LevelData& V = c->lv[l];
        Aux<T> x;
        x.kind = 2;
        x.nh = (V.cb[5] - V.cb[3]) * c->L;  // flat element x layer units
        x.nu = (V.eb[4] - V.eb[2]) * c->L;
        x.nbh = (V.cb[4] - V.cb[3]) * c->L;
        x.nbu = (V.eb[3] - V.eb[2]) * c->L;
        x.lo_h = V.cb[3] * c->L;
        x.lo_u = V.eb[2] * c->L;
        x.xh = (T*)c->Ah;
        x.xu = (T*)c->Au;
        x.ah = (T*)V.x0h; x.bh = (T*)V.acch;
        x.au = (T*)V.x0u; x.bu = (T*)V.accu;
        x.c0 = delta;
        return x;
    }

    // Multi-level LTS3 (Remark 3.1): one LTS3 step of level l on its domain.
    // Level l's fine substeps are LTS3 steps of level l+1 (the deepest level
    // takes SSPRK3 substeps).  For l >= 1 the step is substep k_out of level
    // l-1: its Steps 1, 2 and 4 also evaluate level l-1's interface (adding
    // theta_s R to its accumulator) and their edge kernels predict level
    // l-1's interface 1 for the next stage (stages 1st and 2nd of substep
    // k_out, then old of substep k_out + 1).
    lts_status level_step(int l, double dt, const int* Ms, int k_out) {
        const LevelData& V = c->lv[l];
        T *Ah = (T*)c->Ah, *Au = (T*)c->Au, *Bh = (T*)c->Bh, *Bu = (T*)c->Bu, *Ch = (T*)c->Ch,
          *Cu = (T*)c->Cu;
        const int M = Ms[l];
        const double delta = dt / M;
        const int endc = V.cb[7], ende = V.eb[5];
        const bool deeper = l + 1 < (int)c->lv.size();
        const double th[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
        const Seg<T> none;
        auto oacc_c = [&](int st) {
            if (l == 0) return none;
            const LevelData& O = c->lv[l - 1];
            return accum(O.cb[3], O.cb[5], (T*)O.acch, th[st], st == 0 && k_out == 0);
        };
        auto oacc_e = [&](int st) {
            if (l == 0) return none;
            const LevelData& O = c->lv[l - 1];
            return accum(O.eb[2], O.eb[4], (T*)O.accu, th[st], st == 0 && k_out == 0);
        };
        auto opred = [&](int st, T* xh, T* xu, int k) {
            if (l == 0) return Aux<T>();
            return predict_aux_level(l - 1, xh, xu, st, k, Ms[l - 1]);
        };
        lts_status st;
        // Step 1
        if ((st = pass_plan(V.p1, Ah, Au,
                            mirror(upd(V.cb[1], endc, Bh, nullptr, 0, Ah, 1, dt), V.cb[3], V.cb[4],
                                   (T*)V.x1h, (T*)V.x0h),
                            oacc_c(0),
                            mirror(upd(V.eb[1], ende, Bu, nullptr, 0, Au, 1, dt), V.eb[2], V.eb[3],
                                   (T*)V.x1u, (T*)V.x0u),
                            oacc_e(0), opred(1, Bh, Bu, k_out))))
            return st;
        // Step 2
        if ((st = pass_plan(V.p2, Bh, Bu,
                            mirror(upd(V.cb[3], endc, Ch, Ah, 0.75, Bh, 0.25, 0.25 * dt), V.cb[3],
                                   V.cb[4], (T*)V.x2h, nullptr),
                            oacc_c(1),
                            mirror(upd(V.eb[2], ende, Cu, Au, 0.75, Bu, 0.25, 0.25 * dt), V.eb[2],
                                   V.eb[3], (T*)V.x2u, nullptr),
                            oacc_e(1), opred(2, Ch, Cu, k_out))))
            return st;
        // Step 3
        for (int k = 0; k < M; ++k) {
            if (deeper) {
                if ((st = level_step(l + 1, delta, Ms, k))) return st;
                continue;
            }
            T* acch = (T*)V.acch;
            T* accu = (T*)V.accu;
            if ((st = pass_plan(V.p3, Ah, Au, upd(0, V.cb[3], Bh, nullptr, 0, Ah, 1, delta),
                                accum(V.cb[3], V.cb[5], acch, th[0], k == 0),
                                upd(0, V.eb[2], Bu, nullptr, 0, Au, 1, delta),
                                accum(V.eb[2], V.eb[4], accu, th[0], k == 0),
                                predict_aux_level(l, Bh, Bu, 1, k, M))))
                return st;
            if ((st = pass_plan(V.p3, Bh, Bu, upd(0, V.cb[3], Ch, Ah, 0.75, Bh, 0.25, 0.25 * delta),
                                accum(V.cb[3], V.cb[5], acch, th[1], false),
                                upd(0, V.eb[2], Cu, Au, 0.75, Bu, 0.25, 0.25 * delta),
                                accum(V.eb[2], V.eb[4], accu, th[1], false),
                                predict_aux_level(l, Ch, Cu, 2, k, M))))
                return st;
            if ((st = pass_plan(V.p3, Ch, Cu,
                                upd(0, V.cb[3], Ah, Ah, 1.0 / 3.0, Ch, 2.0 / 3.0, 2.0 / 3.0 * delta),
                                accum(V.cb[3], V.cb[5], acch, th[2], false),
                                upd(0, V.eb[2], Au, Au, 1.0 / 3.0, Cu, 2.0 / 3.0, 2.0 / 3.0 * delta),
                                accum(V.eb[2], V.eb[4], accu, th[2], false),
                                k + 1 < M ? predict_aux_level(l, Ah, Au, 0, k + 1, M) : Aux<T>())))
                return st;
        }
        // Step 4, with Step 5 of this level and the enclosing level's next
        // stage-old prediction on its edge kernel
        const Aux<T> next = (l > 0 && k_out + 1 < Ms[l - 1]) ? opred(0, Ah, Au, k_out + 1) : Aux<T>();
        return pass_plan(V.p4, Ch, Cu,
                         upd(V.cb[5], endc, Ah, Ah, 1.0 / 3.0, Ch, 2.0 / 3.0, 2.0 / 3.0 * dt),
                         oacc_c(2),
                         upd(V.eb[4], ende, Au, Au, 1.0 / 3.0, Cu, 2.0 / 3.0, 2.0 / 3.0 * dt),
                         oacc_e(2), correct_aux_level(l, delta), next);
    }

    static Seg<T> accum(int lo, int hi, T* acc, double theta, bool first) {
        Seg<T> g;
        g.lo = lo;
        g.hi = hi;
        g.mode = hi > lo ? 2 : 0;
        g.acc = acc;
        g.theta = (T)theta;
        g.first = first ? 1 : 0;
        return g;
    }

    // Algorithm 2.2, order 3: one coarse step on the state in A.  The
    // interface-1 copies of X0, X1, X2 are written by the stage epilogues; each
    // interface-1 prediction and the final interface correction run as extra
    // blocks of the preceding edge kernel (they touch none of its data).
    lts_status lts3_step(double dt, int M) {
        T *Ah = (T*)c->Ah, *Au = (T*)c->Au, *Bh = (T*)c->Bh, *Bu = (T*)c->Bu, *Ch = (T*)c->Ch,
          *Cu = (T*)c->Cu;
        const int* cb = c->cb;
        const int* eb = c->eb;
        const int nC = c->nC, nE = c->nE;
        const double delta = dt / M;
        const Seg<T> none;
        lts_status st;
        // Step 1: first stage with dt on underlined F, I1, I2, C
        if ((st = pass(P_STEP1, Ah, Au,
                       mirror(upd(cb[1], nC, Bh, nullptr, 0, Ah, 1, dt), cb[3], cb[4],
                              (T*)c->x1h, (T*)c->x0h),
                       none,
                       mirror(upd(eb[1], nE, Bu, nullptr, 0, Au, 1, dt), eb[2], eb[3],
                              (T*)c->x1u, (T*)c->x0u),
                       none)))
            return st;
        // Step 2: second stage with dt on I1, I2, C
        if ((st = pass(P_STEP2, Bh, Bu,
                       mirror(upd(cb[3], nC, Ch, Ah, 0.75, Bh, 0.25, 0.25 * dt), cb[3], cb[4],
                              (T*)c->x2h, nullptr),
                       none,
                       mirror(upd(eb[2], nE, Cu, Au, 0.75, Bu, 0.25, 0.25 * dt), eb[2], eb[3],
                              (T*)c->x2u, nullptr),
                       none)))
            return st;
        // Step 3: M fine SSPRK3 substeps on F; I1 predicted, I accumulates.
        // (Stage (old,0) needs no prediction: its coefficients give X0.)
        for (int k = 0; k < M; ++k) {
            // stage (old,k): A holds F at substep k, X0 on I2 and C
            if ((st = pass(P_STEP3, Ah, Au, upd(0, cb[3], Bh, nullptr, 0, Ah, 1, delta),
                           accum(cb[3], cb[5], (T*)c->acch, 1.0 / 6.0, k == 0),
                           upd(0, eb[2], Bu, nullptr, 0, Au, 1, delta),
                           accum(eb[2], eb[4], (T*)c->accu, 1.0 / 6.0, k == 0),
                           predict_aux(Bh, Bu, 1, k, M))))
                return st;
            // stage (1st,k): B holds stage-1 F, X1 on I2 and C
            if ((st = pass(P_STEP3, Bh, Bu, upd(0, cb[3], Ch, Ah, 0.75, Bh, 0.25, 0.25 * delta),
                           accum(cb[3], cb[5], (T*)c->acch, 1.0 / 6.0, false),
                           upd(0, eb[2], Cu, Au, 0.75, Bu, 0.25, 0.25 * delta),
                           accum(eb[2], eb[4], (T*)c->accu, 1.0 / 6.0, false),
                           predict_aux(Ch, Cu, 2, k, M))))
                return st;
            // stage (2nd,k): C holds stage-2 F, X2 on I2 and C; new F into A
            if ((st = pass(P_STEP3, Ch, Cu,
                           upd(0, cb[3], Ah, Ah, 1.0 / 3.0, Ch, 2.0 / 3.0, 2.0 / 3.0 * delta),
                           accum(cb[3], cb[5], (T*)c->acch, 2.0 / 3.0, false),
                           upd(0, eb[2], Au, Au, 1.0 / 3.0, Cu, 2.0 / 3.0, 2.0 / 3.0 * delta),
                           accum(eb[2], eb[4], (T*)c->accu, 2.0 / 3.0, false),
                           k + 1 < M ? predict_aux(Ah, Au, 0, k + 1, M) : Aux<T>())))
                return st;
        }
        // Step 4: third stage with dt on C (reads X2 in C and I2 only); Step 5,
        // the interface correction x = x_old + dt/M * acc on I1 u I2, rides on
        // its edge kernel.
        return pass(P_STEP4, Ch, Cu,
                    upd(cb[5], nC, Ah, Ah, 1.0 / 3.0, Ch, 2.0 / 3.0, 2.0 / 3.0 * dt), none,
                    upd(eb[4], nE, Au, Au, 1.0 / 3.0, Cu, 2.0 / 3.0, 2.0 / 3.0 * dt), none,
                    correct_aux(delta));
    }

    // Algorithm 2.1, SSPRK3, over the whole mesh.
    lts_status rk3_step(double dt) {
        T *Ah = (T*)c->Ah, *Au = (T*)c->Au, *Bh = (T*)c->Bh, *Bu = (T*)c->Bu, *Ch = (T*)c->Ch,
          *Cu = (T*)c->Cu;
        const int nC = c->nC, nE = c->nE;
        const Seg<T> none;
        lts_status st;
        if ((st = pass(P_FULL, Ah, Au, upd(0, nC, Bh, nullptr, 0, Ah, 1, dt), none,
                       upd(0, nE, Bu, nullptr, 0, Au, 1, dt), none)))
            return st;
        if ((st = pass(P_FULL, Bh, Bu, upd(0, nC, Ch, Ah, 0.75, Bh, 0.25, 0.25 * dt), none,
                       upd(0, nE, Cu, Au, 0.75, Bu, 0.25, 0.25 * dt), none)))
            return st;
        return pass(P_FULL, Ch, Cu, upd(0, nC, Ah, Ah, 1.0 / 3.0, Ch, 2.0 / 3.0, 2.0 / 3.0 * dt),
                    none, upd(0, nE, Au, Au, 1.0 / 3.0, Cu, 2.0 / 3.0, 2.0 / 3.0 * dt), none);
    }

    // Algorithm 2.1, SSPRK2, over the whole mesh.
    lts_status ssprk2_step(double dt) {
        T *Ah = (T*)c->Ah, *Au = (T*)c->Au, *Bh = (T*)c->Bh, *Bu = (T*)c->Bu;
        const int nC = c->nC, nE = c->nE;
        const Seg<T> none;
        lts_status st;
        if ((st = pass(P_FULL, Ah, Au, upd(0, nC, Bh, nullptr, 0, Ah, 1, dt), none,
                       upd(0, nE, Bu, nullptr, 0, Au, 1, dt), none)))
            return st;
        return pass(P_FULL, Bh, Bu, upd(0, nC, Ah, Ah, 0.5, Bh, 0.5, 0.5 * dt), none,
                    upd(0, nE, Au, Au, 0.5, Bu, 0.5, 0.5 * dt), none);
    }

    // Classical RK4 over the whole mesh: the stage sum k1 + 2 k2 + 2 k3 is
    // accumulated in Q by the stage epilogues, the last stage adds dt/6 (Q + k4).
    lts_status rk4_step(double dt) {
        T *Ah = (T*)c->Ah, *Au = (T*)c->Au, *Bh = (T*)c->Bh, *Bu = (T*)c->Bu, *Ch = (T*)c->Ch,
          *Cu = (T*)c->Cu, *Qh = (T*)c->Qh, *Qu = (T*)c->Qu;
        const int nC = c->nC, nE = c->nE;
        const Seg<T> none;
        lts_status st;
        auto with_acc = [](Seg<T> g, T* acc, double theta, bool first) {
            g.acc = acc;
            g.theta = (T)theta;
            g.first = first ? 1 : 0;
            return g;
        };
        if ((st = pass(P_FULL, Ah, Au,
                       with_acc(upd(0, nC, Bh, nullptr, 0, Ah, 1, 0.5 * dt), Qh, 1.0, true), none,
                       with_acc(upd(0, nE, Bu, nullptr, 0, Au, 1, 0.5 * dt), Qu, 1.0, true), none)))
            return st;
        if ((st = pass(P_FULL, Bh, Bu,
                       with_acc(upd(0, nC, Ch, nullptr, 0, Ah, 1, 0.5 * dt), Qh, 2.0, false), none,
                       with_acc(upd(0, nE, Cu, nullptr, 0, Au, 1, 0.5 * dt), Qu, 2.0, false), none)))
            return st;
        if ((st = pass(P_FULL, Ch, Cu,
                       with_acc(upd(0, nC, Bh, nullptr, 0, Ah, 1, dt), Qh, 2.0, false), none,
                       with_acc(upd(0, nE, Bu, nullptr, 0, Au, 1, dt), Qu, 2.0, false), none)))
            return st;
        return pass(P_FULL, Bh, Bu, upd(0, nC, Ah, Ah, 1.0, Qh, dt / 6.0, dt / 6.0), none,
                    upd(0, nE, Au, Au, 1.0, Qu, dt / 6.0, dt / 6.0), none);
    }

    // Algorithm 2.2, order 2 (LTS2).  Step 2 (the coarse second stage on C)
    // reads only X0 and X1, and nothing in Step 3 reads its result, so it runs
    // after the substeps, writing the new coarse values straight into A with
    // the interface correction riding on its edge kernel.
    lts_status lts2_step(double dt, int M) {
        T *Ah = (T*)c->Ah, *Au = (T*)c->Au, *Bh = (T*)c->Bh, *Bu = (T*)c->Bu;
        const int* cb = c->cb;
        const int* eb = c->eb;
        const int nC = c->nC, nE = c->nE;
        const double delta = dt / M;
        const Seg<T> none;
        lts_status st;
        // Step 1: first stage with dt on I1, I2, C
        if ((st = pass(P_STEP2, Ah, Au,
                       mirror(upd(cb[3], nC, Bh, nullptr, 0, Ah, 1, dt), cb[3], cb[4],
                              (T*)c->x1h, (T*)c->x0h),
                       none,
                       mirror(upd(eb[2], nE, Bu, nullptr, 0, Au, 1, dt), eb[2], eb[3],
                              (T*)c->x1u, (T*)c->x0u),
                       none)))
            return st;
        for (int k = 0; k < M; ++k) {
            if ((st = pass(P_STEP3, Ah, Au, upd(0, cb[3], Bh, nullptr, 0, Ah, 1, delta),
                           accum(cb[3], cb[5], (T*)c->acch, 0.5, k == 0),
                           upd(0, eb[2], Bu, nullptr, 0, Au, 1, delta),
                           accum(eb[2], eb[4], (T*)c->accu, 0.5, k == 0),
                           predict_aux(Bh, Bu, 1, k, M, 2))))
                return st;
            if ((st = pass(P_STEP3, Bh, Bu,
                           upd(0, cb[3], Ah, Ah, 0.5, Bh, 0.5, 0.5 * delta),
                           accum(cb[3], cb[5], (T*)c->acch, 0.5, false),
                           upd(0, eb[2], Au, Au, 0.5, Bu, 0.5, 0.5 * delta),
                           accum(eb[2], eb[4], (T*)c->accu, 0.5, false),
                           k + 1 < M ? predict_aux(Ah, Au, 0, k + 1, M, 2) : Aux<T>())))
                return st;
        }
        // Step 2 on C: new = 1/2 X0 + 1/2 X1 + 1/2 dt R(X1), into A; Step 5 rides along
        return pass(P_STEP4, Bh, Bu, upd(cb[5], nC, Ah, Ah, 0.5, Bh, 0.5, 0.5 * dt), none,
                    upd(eb[4], nE, Au, Au, 0.5, Bu, 0.5, 0.5 * dt), none, correct_aux(delta));
    }

    // Interface-1 prediction coefficients of Algorithm 2.2 (Steps 3.1.1,
    // 3.2.1, 3.3.1), in FP64: (1 - a - a~, a - a~, 2 a~); a~ = 0 for LTS2.
    static void predict_coeffs(int stage, int k, int M, double out[3], int order = 3) {
        const double dk = k, dM = M;
        double a, at;
        if (stage == 0) {
            a = dk / dM;
            at = order == 3 ? (dk * dk) / (dM * dM) : 0.0;
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
};

enum { SCH_LTS3 = 0, SCH_LTS2 = 1, SCH_SSPRK3 = 2, SCH_SSPRK2 = 3, SCH_RK4 = 4, SCH_MLTS3 = 5 };

template <typename T>
lts_status one_step(Run<T>& r, int scheme, double dt, int M) {
    switch (scheme) {
        case SCH_MLTS3: return r.level_step(0, dt, r.c->run_Ms.data(), 0);
        case SCH_LTS3: return r.lts3_step(dt, M);
        case SCH_LTS2: return r.lts2_step(dt, M);
        case SCH_SSPRK3: return r.rk3_step(dt);
        case SCH_SSPRK2: return r.ssprk2_step(dt);
        default: return r.rk4_step(dt);
    }
}


}  // namespace lts
