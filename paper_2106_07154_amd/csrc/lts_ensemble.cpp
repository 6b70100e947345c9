// Ensemble runtime of liblts: many independent LTS3 runs (members) of uneven
// size advanced together.
//
// Each member is an ordinary context (its own mesh, regions, coefficients and
// state).  A member's coarse step is the sequence of right-hand-side passes of
// Algorithm 2.2 (3 M + 4 passes, each a vertex, a cell and an edge kernel).
// The ensemble runs phase t of every member that has one in shared launches:
// one launch per (phase, kernel class, size class) over a device work list of
// (member, range, epilogue) items, with a persistent grid that strides over the
// list's virtual blocks.  Members fall in three size classes (< 30k cells,
// < 120k, larger), each split by slot count (8 or 16 lanes per cell); each
// class is an independent chain of launches on its own stream, and the whole
// ensemble step is captured once into a hipGraph whose branches run
// concurrently.  An autotuner times block size and grid
// size for every (kernel class, size class) on the members' own data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "lts_host.h"

using namespace lts;

struct lts_ens {
    int device = 0;
    lts_precision prec = LTS_FP64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    static constexpr int NCLS = 6;  // 3 size classes x 2 slot counts
    hipStream_t side[NCLS] = {};
    hipEvent_t fork = nullptr, join[NCLS] = {};
    std::string err;
    std::vector<lts_ctx*> members;
    std::vector<double> dt;
    std::vector<int> M, sclass;
    std::vector<std::vector<int>> Ms;  // multi-level members: ratios per level (else empty)
    bool built = false;
    int n_cu = 256;
    // tuned launch shape per [kernel class][class]: block size, grid factor
    int tune_block[KC_N][NCLS];
    int tune_pf[KC_N][NCLS];
    double tune_us[KC_N][NCLS] = {};
    lts_ens() {
        for (int k = 0; k < KC_N; ++k)
            for (int c = 0; c < NCLS; ++c) {
                tune_block[k][c] = 256;
                tune_pf[k][c] = 4;
            }
    }
    double step_bytes[KC_N] = {0, 0, 0};  // algorithmic bytes of one ensemble step
    struct Launch {
        int sc, kclass, nitems, nvb, block, grid;
        size_t off;    // first item in d_items
        double bytes;  // algorithmic bytes of the launch
    };
    int scheme = SCH_LTS3;  // LTS3, or SSPRK3 in M steps of dt/M per ensemble step
    std::vector<hipEvent_t> evs;  // timing events, two per launch
    // fused step: one cooperative launch per ensemble step
    bool fused = false;
    int spin_limit = 1 << 22;     // polls per bounded barrier wait
    int fused_grid = 0, fused_nphase = 0;
    bool fused_graph = false;     // the launch replays from the captured graph
    void* d_phases = nullptr;
    FusedBarrier* d_bar = nullptr;
    double fused_bytes = 0.0;     // algorithmic bytes of one fused step
    std::vector<Launch> launches;
    void* d_items = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t steps = 0;
};

namespace {

lts_status efail(lts_ens* e, lts_status s, const std::string& msg) {
    if (e) e->err = msg;
    return s;
}

#define EHIP(e, expr)                                                                        \
    do {                                                                                     \
        hipError_t r_ = (expr);                                                              \
        if (r_ != hipSuccess)                                                                \
            return efail(e, LTS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(r_)); \
    } while (0)

// Class of a member: size class (< 30k cells, < 120k, larger) + 3 when its
// cells need 16 lanes (more than 8 edges somewhere).
int member_class(int n_cells, int G) {
    return (n_cells < 30000 ? 0 : n_cells < 120000 ? 1 : 2) + (G > 8 ? 3 : 0);
}
int class_lanes(int cls) { return cls >= 3 ? 16 : 8; }

template <typename T>
struct Builder {
    lts_ens* e;
    std::vector<std::vector<PassRecord<T>>> recs;  // per member, in step order
    int nphase = 0;

    lts_status record() {
        recs.assign(e->members.size(), {});
        nphase = 0;
        for (size_t j = 0; j < e->members.size(); ++j) {
            lts_ctx* c = e->members[j];
            const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
            Run<T> r{c, dm, e->stream, false};
            r.rec = &recs[j];
            lts_status st = LTS_OK;
            if (e->scheme == SCH_LTS3 && !e->Ms[j].empty())
                st = r.level_step(0, e->dt[j], e->Ms[j].data(), 0);
            else if (e->scheme == SCH_LTS3) st = r.lts3_step(e->dt[j], e->M[j]);
            else
                for (int k = 0; k < e->M[j] && !st; ++k) st = r.rk3_step(e->dt[j] / e->M[j]);
            if (st) return efail(e, st, "recording member " + std::to_string(j) + ": " + c->err);
            nphase = std::max(nphase, (int)recs[j].size());
        }
        return LTS_OK;
    }

    // Algorithmic bytes of kernel class k of a recorded pass.
    static double record_bytes(const PassRecord<T>& r, int k) {
        if (k != KC_EDGE) return kernel_bytes<T>(r.plan, k, r.cs0, r.cs1, r.aux);
        return kernel_bytes<T>(r.plan, k, r.es0, r.es1, r.aux) +
               kernel_bytes<T>(PassPlan(), k, Seg<T>(), Seg<T>(), r.aux2);
    }

    // Work items of one launch (sc < 0: members of every class); returns the
    // number of virtual blocks.
    int items(int t, int sc, int kclass, int block, std::vector<Item<T>>& out) const {
        out.clear();
        int first = 0;
        for (size_t j = 0; j < recs.size(); ++j) {
            if ((sc >= 0 && e->sclass[j] != sc) || t >= (int)recs[j].size()) continue;
            lts_ctx* c = e->members[j];
            const PassRecord<T>& r = recs[j][t];
            const PassPlan& P = r.plan;
            Item<T> w;
            w.m = *static_cast<DevMesh<T>*>(c->dm);
            w.h = r.h;
            w.u = r.u;
            w.q = static_cast<T*>(c->q);
            w.zs = static_cast<T*>(c->zs);
            w.flag = c->flag;
            w.g = (T)c->g;
            long n = 0;
            if (kclass == KC_VERTEX) {
                w.lo = P.v_lo;
                w.hi = P.v_hi;
                n = P.v_hi - P.v_lo;
            } else if (kclass == KC_CELL) {
                w.lo = P.c_lo;
                w.hi = P.c_hi;
                w.s0 = r.cs0;
                w.s1 = r.cs1;
                n = (long)(P.c_hi - P.c_lo) * class_lanes(e->sclass[j]);
            } else {
                w.lo = P.et_lo;
                w.hi = P.et_hi;
                w.s0 = r.es0;
                w.s1 = r.es1;
                w.aux = r.aux;
                w.aux2 = r.aux2;
                n = P.et_hi - P.et_lo;
                if (r.aux.kind) w.nblk_aux = (int)((r.aux.nh + r.aux.nu + block - 1) / block);
                if (r.aux2.kind) w.nblk_aux2 = (int)((r.aux2.nh + r.aux2.nu + block - 1) / block);
            }
            w.nblk = (int)((n + block - 1) / block);
            if (w.nblk + w.nblk_aux + w.nblk_aux2 == 0) continue;
            w.first = first;
            first += w.nblk + w.nblk_aux + w.nblk_aux2;
            out.push_back(w);
        }
        return first;
    }

    // Time candidate (block, grid factor) pairs for every (kernel class, size
    // class) on the phase with the most work for it.
    lts_status autotune() {
        const int blocks[3] = {128, 256, 512};
        const int pfs[4] = {1, 2, 4, 8};
        std::vector<Item<T>> it;
        void* dbuf = nullptr;
        size_t dcap = 0;
        hipEvent_t a, b;
        EHIP(e, hipEventCreate(&a));
        EHIP(e, hipEventCreate(&b));
        for (int k = 0; k < KC_N; ++k)
            for (int sc = 0; sc < lts_ens::NCLS; ++sc) {
                int best_t = -1, best_n = 0;
                for (int t = 0; t < nphase; ++t) {
                    const int n = items(t, sc, k, 256, it);
                    if (n > best_n) { best_n = n; best_t = t; }
                }
                if (best_t < 0) continue;
                double best = 1e30;
                for (int bs : blocks) {
                    const int nvb = items(best_t, sc, k, bs, it);
                    const size_t bytes = it.size() * sizeof(Item<T>);
                    if (bytes > dcap) {
                        if (dbuf) (void)hipFree(dbuf);
                        EHIP(e, hipMalloc(&dbuf, bytes));
                        dcap = bytes;
                    }
                    EHIP(e, hipMemcpy(dbuf, it.data(), bytes, hipMemcpyHostToDevice));
                    for (int pf : pfs) {
                        const int grid = std::max(1, std::min(nvb, pf * e->n_cu));
                        const Item<T>* di = static_cast<const Item<T>*>(dbuf);
                        const int G = class_lanes(sc);
                        for (int w = 0; w < 2; ++w)
                            EHIP(e, launch_batch<T>(k, di, (int)it.size(), nvb, bs, grid, G, e->stream));
                        EHIP(e, hipEventRecord(a, e->stream));
                        const int reps = 8;
                        for (int w = 0; w < reps; ++w)
                            EHIP(e, launch_batch<T>(k, di, (int)it.size(), nvb, bs, grid, G, e->stream));
                        EHIP(e, hipEventRecord(b, e->stream));
                        EHIP(e, hipEventSynchronize(b));
                        float ms = 0;
                        EHIP(e, hipEventElapsedTime(&ms, a, b));
                        const double us = 1e3 * ms / reps;
                        if (us < best) {
                            best = us;
                            e->tune_block[k][sc] = bs;
                            e->tune_pf[k][sc] = pf;
                            e->tune_us[k][sc] = us;
                        }
                    }
                }
            }
        if (dbuf) (void)hipFree(dbuf);
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return LTS_OK;
    }

    // Fused step: one item list per (phase, kernel class) over all members,
    // one cooperative launch per step; captured into a graph when the runtime
    // accepts the cooperative launch under capture, else launched directly.
    lts_status finalize_fused() {
        std::vector<Item<T>> all, it;
        std::vector<FusedPhase> ph;
        e->fused_bytes = 0.0;
        for (int k = 0; k < KC_N; ++k) e->fused_bytes += e->step_bytes[k];
        int max_nvb = 1;
        for (int t = 0; t < nphase; ++t)
            for (int k = 0; k < KC_N; ++k) {
                const int nvb = items(t, -1, k, 256, it);
                ph.push_back(FusedPhase{(int)all.size(), (int)it.size(), nvb});
                all.insert(all.end(), it.begin(), it.end());
                max_nvb = std::max(max_nvb, nvb);
            }
        const int per_cu = fused_blocks_per_cu<T>();
        if (per_cu <= 0) return efail(e, LTS_EDEVICE, "fused step: occupancy query failed");
        // one block per CU below the occupancy limit: a margin for co-residency,
        // which every grid barrier relies on (measured 1% slower than the limit)
        e->fused_grid = std::max(1, std::min(max_nvb, std::max(1, per_cu - 1) * e->n_cu));
        e->fused_nphase = nphase;
        EHIP(e, hipMalloc(&e->d_items, std::max<size_t>(all.size(), 1) * sizeof(Item<T>)));
        if (!all.empty())
            EHIP(e, hipMemcpy(e->d_items, all.data(), all.size() * sizeof(Item<T>),
                              hipMemcpyHostToDevice));
        EHIP(e, hipMalloc(&e->d_phases, std::max<size_t>(ph.size(), 1) * sizeof(FusedPhase)));
        if (!ph.empty())
            EHIP(e, hipMemcpy(e->d_phases, ph.data(), ph.size() * sizeof(FusedPhase),
                              hipMemcpyHostToDevice));
        if (!e->d_bar) {
            EHIP(e, hipMalloc(&e->d_bar, sizeof(FusedBarrier)));
            EHIP(e, hipMemset(e->d_bar, 0, sizeof(FusedBarrier)));
        }
        e->fused_graph = false;
        if (hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            hipError_t err = launch_fused<T>(static_cast<const Item<T>*>(e->d_items),
                                             static_cast<const FusedPhase*>(e->d_phases), nphase,
                                             e->d_bar, e->spin_limit, e->fused_grid, e->stream);
            hipGraph_t gr = nullptr;
            hipError_t err2 = hipStreamEndCapture(e->stream, &gr);
            if (err == hipSuccess && err2 == hipSuccess && gr &&
                hipGraphInstantiate(&e->gexec, gr, nullptr, nullptr, 0) == hipSuccess) {
                e->graph = gr;
                e->fused_graph = true;
            } else {
                if (gr) (void)hipGraphDestroy(gr);
                e->gexec = nullptr;
                (void)hipGetLastError();
            }
        }
        return LTS_OK;
    }

    lts_status finalize() {
        std::vector<Item<T>> all, it;
        e->launches.clear();
        for (int k = 0; k < KC_N; ++k) e->step_bytes[k] = 0;
        for (size_t j = 0; j < recs.size(); ++j)
            for (const PassRecord<T>& r : recs[j])
                for (int k = 0; k < KC_N; ++k) e->step_bytes[k] += record_bytes(r, k);
        if (e->fused) return finalize_fused();
        for (int sc = 0; sc < lts_ens::NCLS; ++sc)
            for (int t = 0; t < nphase; ++t)
                for (int k = 0; k < KC_N; ++k) {
                    const int bs = e->tune_block[k][sc];
                    const int nvb = items(t, sc, k, bs, it);
                    if (nvb == 0) continue;
                    lts_ens::Launch L;
                    L.bytes = 0.0;
                    for (size_t j = 0; j < recs.size(); ++j) {
                        if (e->sclass[j] != sc || t >= (int)recs[j].size()) continue;
                        L.bytes += record_bytes(recs[j][t], k);
                    }
                    L.sc = sc;
                    L.kclass = k;
                    L.nitems = (int)it.size();
                    L.nvb = nvb;
                    L.block = bs;
                    L.grid = std::max(1, std::min(nvb, e->tune_pf[k][sc] * e->n_cu));
                    L.off = all.size();
                    all.insert(all.end(), it.begin(), it.end());
                    e->launches.push_back(L);
                }
        const size_t bytes = std::max<size_t>(all.size(), 1) * sizeof(Item<T>);
        EHIP(e, hipMalloc(&e->d_items, bytes));
        if (!all.empty())
            EHIP(e, hipMemcpy(e->d_items, all.data(), all.size() * sizeof(Item<T>),
                              hipMemcpyHostToDevice));
        // capture: fork to one stream per size class, one chain each, join
        EHIP(e, hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipEventRecord(e->fork, e->stream);
        for (int sc = 0; sc < lts_ens::NCLS && err == hipSuccess; ++sc)
            err = hipStreamWaitEvent(e->side[sc], e->fork, 0);
        const Item<T>* base = static_cast<const Item<T>*>(e->d_items);
        for (const auto& L : e->launches) {
            if (err != hipSuccess) break;
            err = launch_batch<T>(L.kclass, base + L.off, L.nitems, L.nvb, L.block, L.grid,
                                  class_lanes(L.sc), e->side[L.sc]);
        }
        for (int sc = 0; sc < lts_ens::NCLS && err == hipSuccess; ++sc) {
            err = hipEventRecord(e->join[sc], e->side[sc]);
            if (err == hipSuccess) err = hipStreamWaitEvent(e->stream, e->join[sc], 0);
        }
        hipGraph_t gr = nullptr;
        hipError_t err2 = hipStreamEndCapture(e->stream, &gr);
        if (err != hipSuccess || err2 != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return efail(e, LTS_EDEVICE, std::string("ensemble capture: ") +
                                             hipGetErrorString(err != hipSuccess ? err : err2));
        }
        e->graph = gr;
        EHIP(e, hipGraphInstantiate(&e->gexec, gr, nullptr, nullptr, 0));
        return LTS_OK;
    }
};

template <typename T>
lts_status build(lts_ens* e, int autotune) {
    Builder<T> b{e};
    lts_status st = b.record();
    if (st) return st;
    if (autotune && !e->fused) {
        // tuning launches advance the members: keep a device copy of every
        // member's state and copy it back afterwards, bit for bit (a round trip
        // through lts_get_state / lts_init_state would re-derive an FP32
        // member's reference thickness and round its perturbation anew)
        const size_t nm = e->members.size();
        std::vector<void*> keep(2 * nm, nullptr);
        auto release = [&]() {
            for (void* p : keep)
                if (p) (void)hipFree(p);
        };
        for (size_t j = 0; j < nm && st == LTS_OK; ++j) {
            lts_ctx* c = e->members[j];
            const size_t bh = (size_t)c->nC * c->L * tsize(c), bu = (size_t)c->nE * c->L * tsize(c);
            if (hipMalloc(&keep[2 * j], bh) != hipSuccess ||
                hipMalloc(&keep[2 * j + 1], bu) != hipSuccess ||
                hipMemcpyAsync(keep[2 * j], c->Ah, bh, hipMemcpyDeviceToDevice, e->stream) !=
                    hipSuccess ||
                hipMemcpyAsync(keep[2 * j + 1], c->Au, bu, hipMemcpyDeviceToDevice, e->stream) !=
                    hipSuccess)
                st = efail(e, LTS_ENOMEM, "autotune: keeping the member states");
        }
        if (st == LTS_OK) st = b.autotune();
        if (st == LTS_OK && hipStreamSynchronize(e->stream) != hipSuccess)
            st = efail(e, LTS_EDEVICE, "autotune: synchronise");
        for (size_t j = 0; j < nm && st == LTS_OK; ++j) {
            lts_ctx* c = e->members[j];
            const size_t bh = (size_t)c->nC * c->L * tsize(c), bu = (size_t)c->nE * c->L * tsize(c);
            if (hipMemcpyAsync(c->Ah, keep[2 * j], bh, hipMemcpyDeviceToDevice, e->stream) !=
                    hipSuccess ||
                hipMemcpyAsync(c->Au, keep[2 * j + 1], bu, hipMemcpyDeviceToDevice, e->stream) !=
                    hipSuccess ||
                launch_fill_int(c->flag, 0, e->stream) != hipSuccess)
                st = efail(e, LTS_EDEVICE, "autotune: restoring the member states");
            c->nonfinite = false;
        }
        if (hipStreamSynchronize(e->stream) != hipSuccess && st == LTS_OK)
            st = efail(e, LTS_EDEVICE, "autotune: synchronise");
        release();
        if (st) return st;
    }
    return b.finalize();
}

// Drop the recorded launches and their graph (the members keep their state).
void unbuild(lts_ens* e) {
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    if (e->d_items) (void)hipFree(e->d_items);
    if (e->d_phases) (void)hipFree(e->d_phases);
    e->gexec = nullptr;
    e->graph = nullptr;
    e->d_items = nullptr;
    e->d_phases = nullptr;
    e->fused_graph = false;
    e->launches.clear();
    e->built = false;
}

// One fused ensemble step without the graph (event-stamped when ev0/ev1).
template <typename T>
hipError_t fused_launch(lts_ens* e, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    return launch_fused<T>(static_cast<const Item<T>*>(e->d_items),
                           static_cast<const FusedPhase*>(e->d_phases), e->fused_nphase, e->d_bar,
                           e->spin_limit, e->fused_grid, e->stream, ev0, ev1);
}

// After fused steps: wait for them and turn a barrier that gave up into
// LTS_EDEVICE (the members' states are then undefined; re-initialise them).
lts_status fused_check(lts_ens* e) {
    EHIP(e, hipStreamSynchronize(e->stream));
    FusedBarrier b;
    EHIP(e, hipMemcpy(&b, e->d_bar, sizeof(b), hipMemcpyDeviceToHost));
    if (fused_barrier_error(b)) {
        EHIP(e, hipMemset(e->d_bar, 0, sizeof(FusedBarrier)));
        for (lts_ctx* c : e->members) c->has_state = false;
        return efail(e, LTS_EDEVICE,
                     "fused step: a grid barrier wait ran out; member states are undefined");
    }
    return LTS_OK;
}

// n ensemble steps with every launch stamped by events, one after another on
// the ensemble's stream (each size class's chain keeps its order).
template <typename T>
lts_status timed_steps(lts_ens* e, int n, int64_t* launches, double* ms, double* bytes) {
    if (e->fused) {
        while (e->evs.size() < 2) {
            hipEvent_t ev;
            EHIP(e, hipEventCreate(&ev));
            e->evs.push_back(ev);
        }
        for (int i = 0; i < n; ++i) {
            EHIP(e, fused_launch<T>(e, e->evs[0], e->evs[1]));
            lts_status st = fused_check(e);
            if (st) return st;
            float t = 0.f;
            EHIP(e, hipEventElapsedTime(&t, e->evs[0], e->evs[1]));
            launches[KC_CELL] += 1;
            ms[KC_CELL] += t;
            bytes[KC_CELL] += e->fused_bytes;
        }
        return LTS_OK;
    }
    const size_t need = 2 * e->launches.size();
    while (e->evs.size() < need) {
        hipEvent_t ev;
        EHIP(e, hipEventCreate(&ev));
        e->evs.push_back(ev);
    }
    const Item<T>* base = static_cast<const Item<T>*>(e->d_items);
    for (int i = 0; i < n; ++i) {
        for (size_t q = 0; q < e->launches.size(); ++q) {
            const auto& L = e->launches[q];
            EHIP(e, launch_batch<T>(L.kclass, base + L.off, L.nitems, L.nvb, L.block, L.grid,
                                    class_lanes(L.sc), e->stream, e->evs[2 * q],
                                    e->evs[2 * q + 1]));
        }
        EHIP(e, hipStreamSynchronize(e->stream));
        for (size_t q = 0; q < e->launches.size(); ++q) {
            float t = 0.f;
            EHIP(e, hipEventElapsedTime(&t, e->evs[2 * q], e->evs[2 * q + 1]));
            const int k = e->launches[q].kclass;
            launches[k] += 1;
            ms[k] += t;
            bytes[k] += e->launches[q].bytes;
        }
    }
    return LTS_OK;
}

lts_status ens_ready(lts_ens* e) {
    if (!e) return LTS_EINVAL;
    if (hipSetDevice(e->device) != hipSuccess) return efail(e, LTS_EDEVICE, "hipSetDevice");
    return LTS_OK;
}

}  // namespace

extern "C" {

lts_status lts_ens_create(lts_ens** out, int device, lts_precision prec, void* hip_stream) {
    if (!out) return LTS_EINVAL;
    *out = nullptr;
    if (prec != LTS_FP64 && prec != LTS_FP32) return LTS_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LTS_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return LTS_EDEVICE;
    lts_ens* e = new lts_ens();
    e->device = device;
    e->prec = prec;
    bool ok = true;
    if (hip_stream) {
        e->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        ok = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) == hipSuccess;
        e->own_stream = ok;
    }
    for (int k = 0; k < lts_ens::NCLS && ok; ++k)
        ok = hipStreamCreateWithFlags(&e->side[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&e->join[k], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&e->fork, hipEventDisableTiming) == hipSuccess;
    hipDeviceProp_t prop;
    if (ok && hipGetDeviceProperties(&prop, device) == hipSuccess) e->n_cu = prop.multiProcessorCount;
    *out = e;
    return ok ? LTS_OK : efail(e, LTS_EDEVICE, "stream/event creation failed");
}

void lts_ens_destroy(lts_ens* e) {
    if (!e) return;
    (void)hipSetDevice(e->device);
    unbuild(e);
    if (e->d_bar) (void)hipFree(e->d_bar);
    for (hipEvent_t ev : e->evs) (void)hipEventDestroy(ev);
    for (lts_ctx* c : e->members) lts_destroy(c);
    for (int k = 0; k < lts_ens::NCLS; ++k) {
        if (e->side[k]) (void)hipStreamDestroy(e->side[k]);
        if (e->join[k]) (void)hipEventDestroy(e->join[k]);
    }
    if (e->fork) (void)hipEventDestroy(e->fork);
    if (e->own_stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

const char* lts_ens_last_error(const lts_ens* e) { return e ? e->err.c_str() : "null ensemble"; }

lts_status lts_ens_add_member(lts_ens* e, const lts_mesh* mesh, const uint8_t* fine_mask,
                              int n_if1_rings, int n_if2_rings, double gravity, double dt_coarse,
                              int M, int* member) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (e->built) return efail(e, LTS_ESTATE, "ensemble already built");
    if (!mesh || !(dt_coarse > 0) || M < 1) return efail(e, LTS_EINVAL, "bad member arguments");
    lts_ctx* c = nullptr;
    if ((s = lts_create(&c, e->device, e->prec, e->stream))) return efail(e, s, "member context");
    if ((s = lts_upload_mesh(c, mesh, fine_mask, n_if1_rings, n_if2_rings, gravity))) {
        const std::string msg = c->err;
        lts_destroy(c);
        return efail(e, s, "member mesh: " + msg);
    }
    e->members.push_back(c);
    e->dt.push_back(dt_coarse);
    e->M.push_back(M);
    e->Ms.emplace_back();
    e->sclass.push_back(member_class(c->nC, padded_slots(c->maxE)));
    if (member) *member = (int)e->members.size() - 1;
    return LTS_OK;
}

lts_status lts_ens_add_member_levels(lts_ens* e, const lts_mesh* mesh, int n_fine_levels,
                                     const uint8_t* fine_masks, int n_if1_rings,
                                     int n_if2_rings, double gravity, double dt_coarse,
                                     const int32_t* M, int* member) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (e->built) return efail(e, LTS_ESTATE, "ensemble already built");
    if (!mesh || !M || !(dt_coarse > 0) || n_fine_levels < 1 ||
        n_fine_levels > LTS_MAX_LEVELS - 1)
        return efail(e, LTS_EINVAL, "bad member arguments");
    long prod = 1;  // the finest level's steps per coarse step
    for (int l = 0; l < n_fine_levels; ++l) {
        if (M[l] < 1) return efail(e, LTS_EINVAL, "bad member arguments: a ratio < 1");
        prod *= M[l];
        if (prod > (1L << 20))
            return efail(e, LTS_EINVAL, "bad member arguments: the ratios multiply beyond 2^20");
    }
    lts_ctx* c = nullptr;
    if ((s = lts_create(&c, e->device, e->prec, e->stream))) return efail(e, s, "member context");
    if ((s = lts_upload_mesh_levels(c, mesh, n_fine_levels, fine_masks, n_if1_rings,
                                    n_if2_rings, gravity))) {
        const std::string msg = c->err;
        lts_destroy(c);
        return efail(e, s, "member mesh: " + msg);
    }
    e->members.push_back(c);
    e->dt.push_back(dt_coarse);
    // the SSPRK3 mode steps a multi-level member at its finest step
    e->M.push_back((int)prod);
    e->Ms.emplace_back(n_fine_levels > 1 ? std::vector<int>(M, M + n_fine_levels)
                                         : std::vector<int>());
    if (n_fine_levels == 1) e->M.back() = M[0];
    e->sclass.push_back(member_class(c->nC, padded_slots(c->maxE)));
    if (member) *member = (int)e->members.size() - 1;
    return LTS_OK;
}

lts_status lts_ens_init_member(lts_ens* e, int member, const double* h, const double* u) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (member < 0 || member >= (int)e->members.size()) return efail(e, LTS_EINVAL, "no such member");
    if ((s = lts_init_state(e->members[member], h, u, 0.0)))
        return efail(e, s, e->members[member]->err);
    return LTS_OK;
}

lts_status lts_ens_build(lts_ens* e, int autotune) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (e->built) return efail(e, LTS_ESTATE, "ensemble already built");
    if (e->members.empty()) return efail(e, LTS_ESTATE, "no members");
    for (lts_ctx* c : e->members)
        if (!c->has_state) return efail(e, LTS_ESTATE, "initialise every member before build");
    s = e->prec == LTS_FP64 ? build<double>(e, autotune) : build<float>(e, autotune);
    if (s) return s;
    e->built = true;
    return LTS_OK;
}

lts_status lts_ens_step(lts_ens* e, int n_steps) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (!e->built) return efail(e, LTS_ESTATE, "build the ensemble first");
    if (n_steps < 0) return efail(e, LTS_EINVAL, "n_steps < 0");
    for (lts_ctx* c : e->members) {
        if (c->nonfinite) return efail(e, LTS_ENONFINITE, "a member is non-finite");
        if (!c->has_state) return efail(e, LTS_ESTATE, "a member has no valid state");
    }
    if (e->fused) {
        for (int i = 0; i < n_steps; ++i) {
            if (e->fused_graph) EHIP(e, hipGraphLaunch(e->gexec, e->stream));
            else if (e->prec == LTS_FP64) EHIP(e, fused_launch<double>(e));
            else EHIP(e, fused_launch<float>(e));
        }
        if ((s = fused_check(e))) return s;
    }
    for (int i = 0; i < n_steps && !e->fused; ++i) EHIP(e, hipGraphLaunch(e->gexec, e->stream));
    for (size_t j = 0; j < e->members.size(); ++j) {
        e->members[j]->t += e->dt[j] * n_steps;
        e->members[j]->steps += n_steps;
    }
    e->steps += n_steps;
    return LTS_OK;
}

lts_status lts_ens_get_member(lts_ens* e, int member, double* h, double* u) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (member < 0 || member >= (int)e->members.size()) return efail(e, LTS_EINVAL, "no such member");
    if ((s = lts_get_state(e->members[member], h, u))) return efail(e, s, e->members[member]->err);
    return LTS_OK;
}

lts_status lts_ens_diagnostics(lts_ens* e, int member, lts_diag* out) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (member < 0 || member >= (int)e->members.size()) return efail(e, LTS_EINVAL, "no such member");
    s = lts_diagnostics(e->members[member], out);
    if (s) return efail(e, s, e->members[member]->err);
    return LTS_OK;
}

lts_status lts_ens_set_scheme(lts_ens* e, int scheme, const double* dt_coarse) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (scheme != SCH_LTS3 && scheme != SCH_SSPRK3) return efail(e, LTS_EINVAL, "unsupported scheme");
    if (dt_coarse)
        for (size_t j = 0; j < e->members.size(); ++j)
            if (!(dt_coarse[j] > 0)) return efail(e, LTS_EINVAL, "dt_coarse must be > 0");
    unbuild(e);
    e->scheme = scheme;
    if (dt_coarse)
        for (size_t j = 0; j < e->members.size(); ++j) e->dt[j] = dt_coarse[j];
    return LTS_OK;
}

lts_status lts_ens_set_fused(lts_ens* e, int enable, int spin_limit) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (spin_limit < 0) return efail(e, LTS_EINVAL, "spin_limit < 0");
    unbuild(e);
    e->fused = enable != 0;
    e->spin_limit = spin_limit > 0 ? spin_limit : (1 << 22);
    return LTS_OK;
}

lts_status lts_ens_kernel_stats(lts_ens* e, int n_steps, int64_t* launches, double* ms,
                                double* bytes) {
    lts_status s = ens_ready(e);
    if (s) return s;
    if (!e->built) return efail(e, LTS_ESTATE, "build the ensemble first");
    if (n_steps < 0 || !launches || !ms || !bytes) return efail(e, LTS_EINVAL, "bad arguments");
    for (int k = 0; k < KC_N; ++k) {
        launches[k] = 0;
        ms[k] = bytes[k] = 0.0;
    }
    for (lts_ctx* c : e->members)
        if (c->nonfinite) return efail(e, LTS_ENONFINITE, "a member is non-finite");
    s = e->prec == LTS_FP64 ? timed_steps<double>(e, n_steps, launches, ms, bytes)
                            : timed_steps<float>(e, n_steps, launches, ms, bytes);
    if (s) return s;
    for (size_t j = 0; j < e->members.size(); ++j) {
        e->members[j]->t += e->dt[j] * n_steps;
        e->members[j]->steps += n_steps;
    }
    e->steps += n_steps;
    return LTS_OK;
}

lts_status lts_ens_info(lts_ens* e, int32_t* tuned, double* tuned_us, int64_t* class_cells,
                        int32_t* n_launches, double* step_bytes) {
    lts_status s = ens_ready(e);
    if (s) return s;
    for (int k = 0; k < KC_N; ++k)
        for (int sc = 0; sc < 3; ++sc) {  // reported for the 8-lane classes
            if (tuned) {
                tuned[(k * 3 + sc) * 2] = e->tune_block[k][sc];
                tuned[(k * 3 + sc) * 2 + 1] = e->tune_pf[k][sc];
            }
            if (tuned_us) tuned_us[k * 3 + sc] = e->tune_us[k][sc];
        }
    if (class_cells) {
        for (int sc = 0; sc < 3; ++sc) class_cells[sc] = 0;
        for (size_t j = 0; j < e->members.size(); ++j) class_cells[e->sclass[j] % 3] += e->members[j]->nC;
    }
    if (n_launches) *n_launches = (int32_t)e->launches.size();
    if (step_bytes)
        for (int k = 0; k < KC_N; ++k) step_bytes[k] = e->step_bytes[k];
    return LTS_OK;
}

}  // extern "C"
