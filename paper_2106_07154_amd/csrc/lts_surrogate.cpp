// Learned fine-region surrogate: training on the solver's own coarse steps
// and the gated surrogate step with plain-LTS3 fallback (C ABI in
// lts_surrogate.h).  The network kernels live in lts_mpnn.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "lts.h"
#include "lts_host.h"
#include "lts_mpnn.h"
#include "lts_surrogate.h"

using namespace lts;

namespace {

constexpr int kLayers = 3;
// parameter offsets (floats)
constexpr int OFF_W0 = 0, OFF_B0 = 16 * 64, OFF_L1 = OFF_B0 + 64;
constexpr int LAYER = 128 * 64 + 64;
constexpr int OFF_WH = OFF_L1 + kLayers * LAYER, OFF_WU = OFF_WH + 64, OFF_BH = OFF_WU + 64;
constexpr int N_PARAMS = OFF_BH + 1;
constexpr int N_WBF = 16 * 64 + kLayers * 128 * 64;
constexpr int RPB = nn::kReduceRows;

inline int off_w(int l) { return l == 0 ? OFF_W0 : OFF_L1 + (l - 1) * LAYER; }
inline int off_b(int l) { return l == 0 ? OFF_B0 : OFF_L1 + (l - 1) * LAYER + 128 * 64; }
inline int off_wbf(int l) { return l == 0 ? 0 : 16 * 64 + (l - 1) * 128 * 64; }

}  // namespace

struct lts_sur {
    lts_ctx* c = nullptr;
    void* dm_at_create = nullptr;
    std::string err;
    hipStream_t s = nullptr;

    int N = 0, nF = 0, nFe = 0, aw = 8, cb1 = 0, cb3 = 0, cb4 = 0;
    int S_cap = 0, S = 0;

    std::vector<void*> allocs;
    int32_t *adj = nullptr, *node_edges = nullptr, *ec0 = nullptr, *ec1 = nullptr;
    float* inv_deg = nullptr;
    float *raw_s = nullptr, *tgt_s = nullptr, *raw = nullptr;
    uint16_t* X = nullptr;
    uint16_t* HC[kLayers] = {nullptr, nullptr, nullptr};
    uint16_t *H3 = nullptr, *dZ = nullptr;
    float *dH = nullptr, *dHn = nullptr;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    int32_t* bf_map = nullptr;
    uint16_t* wbf = nullptr;
    uint16_t* wt[kLayers] = {nullptr, nullptr, nullptr};
    float *out_h = nullptr, *out_u = nullptr, *gh = nullptr, *gu = nullptr;
    float *part = nullptr, *losses = nullptr, *norm = nullptr;
    int loss_cap = 0;
    double* dpart = nullptr;
    double* gout = nullptr;
    double* host4 = nullptr;  // pinned, 6 gate sums
    int* flag = nullptr;
    // state-typed buffers (context precision)
    void *Sh = nullptr, *Su = nullptr, *R0h = nullptr, *R0u = nullptr, *R1h = nullptr,
         *R1u = nullptr, *Ph = nullptr, *Pu = nullptr;
    // interface accumulation: the elements its pass reads (device numbering)
    // with their class (0 fine, 1 interface 1, 2 interface 2 or coarse), and
    // the stage buffers of L = 3M layers (allocated for the M in use)
    int32_t *icidx = nullptr, *ieidx = nullptr;
    int8_t *iccls = nullptr, *iecls = nullptr;
    int nicl = 0, niel = 0;
    int L = 0;
    void *hS = nullptr, *uS = nullptr, *qS = nullptr, *zsS = nullptr, *accH = nullptr,
         *accU = nullptr;
    double* icoef = nullptr;
    // mass fix: 1 / (area of the fine cells), scratch
    double inv_area_f = 0.0;
    double *mpart = nullptr, *mshift = nullptr;

    float norm_host[16] = {0};
    bool has_norm = false;
    int adam_step = 0;
    int skip = 0, backoff = 0;  // gate back-off state

    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    double g_dt = 0.0;
    int g_M = 0;
};

namespace {

lts_status sfail(lts_sur* s, lts_status st, const std::string& msg) {
    if (s) s->err = msg;
    return st;
}

#define SCHK(sur, expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return sfail(sur, LTS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename P>
lts_status salloc(lts_sur* s, P** ptr, size_t bytes) {
    void* q = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return sfail(s, LTS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    s->allocs.push_back(q);
    *ptr = static_cast<P*>(q);
    return LTS_OK;
}

lts_status check(lts_sur* s) {
    if (!s) return LTS_EINVAL;
    if (!s->c->has_mesh || s->c->dm != s->dm_at_create)
        return sfail(s, LTS_EINVAL, "the context's mesh changed since the surrogate was created");
    if (!s->c->has_state) return sfail(s, LTS_EINVAL, "context has no state");
    return LTS_OK;
}

// splitmix64: a counter-based generator for the parameter initialisation
uint64_t splitmix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

std::vector<float> init_params(uint64_t seed) {
    std::vector<float> p(N_PARAMS, 0.f);
    uint64_t ctr = 0;
    auto fill = [&](int off, int n, int fan_in, int fan_out) {
        const double a = std::sqrt(6.0 / (fan_in + fan_out));
        for (int i = 0; i < n; ++i) {
            const double u = (splitmix(seed ^ (0x5851F42D4C957F2Dull * ++ctr)) >> 11) * 0x1.0p-53;
            p[off + i] = (float)((2.0 * u - 1.0) * a);
        }
    };
    fill(OFF_W0, 16 * 64, 16, 64);
    for (int l = 1; l <= kLayers; ++l) fill(off_w(l), 128 * 64, 128, 64);
    fill(OFF_WH, 64, 64, 1);
    fill(OFF_WU, 64, 64, 1);
    return p;
}

// BF16 working copies and transposed halves from the FP32 master weights.
void refresh_bf16(lts_sur* s) {
    nn::to_bf16(s->p + OFF_W0, 16 * 64, s->wbf, s->s);
    for (int l = 1; l <= kLayers; ++l) {
        nn::to_bf16(s->p + off_w(l), 128 * 64, s->wbf + off_wbf(l), s->s);
        nn::transpose_halves(s->wbf + off_wbf(l), s->wt[l - 1], s->s);
    }
}

// Forward pass from X; heads with optional targets (th == nullptr: none).
void forward(lts_sur* s, const float* th, const float* tu, float* loss) {
    const int N = s->N;
    nn::gemm(s->X, nn::kFeat, N, nn::kFeat, s->wbf + off_wbf(0), s->p + off_b(0), 1, s->HC[0], 128,
             nullptr, s->s);
    for (int l = 1; l <= kLayers; ++l) {
        nn::aggregate(s->HC[l - 1], N, s->adj, s->aw, s->inv_deg, s->s);
        uint16_t* out = l < kLayers ? s->HC[l] : s->H3;
        nn::gemm(s->HC[l - 1], 128, N, 128, s->wbf + off_wbf(l), s->p + off_b(l), 1, out,
                 l < kLayers ? 128 : 64, nullptr, s->s);
    }
    nn::heads(s->H3, 64, s->nF, s->nFe, s->ec0, s->ec1, s->p + OFF_WH, s->p + OFF_BH,
              s->p + OFF_WU, th, tu, s->norm_host[10], s->norm_host[11], s->out_h, s->out_u,
              s->gh, s->gu, th ? s->part : nullptr, loss, s->s);
}

// Gradient of the loss of the last forward pass into g.
void backward(lts_sur* s) {
    const int N = s->N;
    nn::heads_back(s->H3, 64, N, s->nF, s->node_edges, s->aw, s->p + OFF_WH, s->p + OFF_WU, s->gh,
                   s->gu, s->dH, s->part, s->g + OFF_WH, s->s);
    for (int l = kLayers; l >= 1; --l) {
        const uint16_t* Hout = l < kLayers ? s->HC[l] : s->H3;
        nn::relu_back(s->dH, Hout, l < kLayers ? 128 : 64, N, s->dZ, s->s);
        nn::gemm_tn(s->HC[l - 1], 128, N, 128, s->dZ, RPB, s->part, s->g + off_w(l), s->s);
        nn::colsum(s->dZ, N, RPB, s->part, s->g + off_b(l), s->s);
        // dHC = dZ Wl^T: self half into dH, neighbour half into dHn
        nn::gemm(s->dZ, 64, N, 64, s->wt[l - 1], nullptr, 0, nullptr, 0, s->dH, s->s);
        nn::gemm(s->dZ, 64, N, 64, s->wt[l - 1] + 4096, nullptr, 0, nullptr, 0, s->dHn, s->s);
        nn::aggregate_back(s->dH, s->dHn, N, s->adj, s->aw, s->inv_deg, s->s);
    }
    nn::relu_back(s->dH, s->HC[0], 128, N, s->dZ, s->s);
    nn::gemm_tn(s->X, nn::kFeat, N, nn::kFeat, s->dZ, RPB, s->part, s->g + off_w(0), s->s);
    nn::colsum(s->dZ, N, RPB, s->part, s->g + off_b(0), s->s);
}

// The cells and edges the interface-only pass reads (its cell range, their
// neighbours and edges, and the cells and edges of its vertex range), with
// the class that decides their stage values.
template <typename T>
lts_status interface_read_set(lts_sur* s) {
    lts_ctx* c = s->c;
    const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
    const PassPlan& P = c->iface_plan;
    const int nC = c->nC, nE = c->nE, nV = c->nV;
    std::vector<int32_t> cso(2 * (size_t)nC);
    SCHK(s, hipMemcpy(cso.data(), dm.cso, cso.size() * 4, hipMemcpyDeviceToHost));
    const size_t nslots = nC ? (size_t)cso[2 * (size_t)(nC - 1)] + cso[2 * (size_t)nC - 1] : 0;
    std::vector<int32_t> eoc(nslots), coc(nslots), eov(3 * (size_t)nV), cov(3 * (size_t)nV);
    SCHK(s, hipMemcpy(eoc.data(), dm.eoc, nslots * 4, hipMemcpyDeviceToHost));
    SCHK(s, hipMemcpy(coc.data(), dm.coc, nslots * 4, hipMemcpyDeviceToHost));
    SCHK(s, hipMemcpy(eov.data(), dm.eov, eov.size() * 4, hipMemcpyDeviceToHost));
    SCHK(s, hipMemcpy(cov.data(), dm.cov, cov.size() * 4, hipMemcpyDeviceToHost));
    std::vector<char> rc(nC, 0), re(nE, 0);
    for (int i = P.c_lo; i < P.c_hi; ++i) {
        rc[i] = 1;
        for (int a = 0; a < cso[2 * (size_t)i + 1]; ++a) {
            const size_t o = (size_t)cso[2 * (size_t)i] + a;
            rc[coc[o]] = 1;
            re[eoc[o]] = 1;
        }
    }
    for (int v = P.v_lo; v < P.v_hi; ++v)
        for (int k = 0; k < 3; ++k) {
            rc[cov[(size_t)k * nV + v]] = 1;
            re[eov[(size_t)k * nV + v]] = 1;
        }
    std::vector<int32_t> ci, ei;
    std::vector<int8_t> cc, ec;
    for (int i = 0; i < nC; ++i)
        if (rc[i]) {
            ci.push_back(i);
            cc.push_back((int8_t)(i < c->cb[3] ? 0 : i < c->cb[4] ? 1 : 2));
        }
    for (int e = 0; e < nE; ++e)
        if (re[e]) {
            ei.push_back(e);
            ec.push_back((int8_t)(e < c->eb[2] ? 0 : e < c->eb[3] ? 1 : 2));
        }
    s->nicl = (int)ci.size();
    s->niel = (int)ei.size();
    lts_status st;
    if ((st = salloc(s, &s->icidx, ci.size() * 4)) || (st = salloc(s, &s->iccls, cc.size())) ||
        (st = salloc(s, &s->ieidx, ei.size() * 4)) || (st = salloc(s, &s->iecls, ec.size())))
        return st;
    SCHK(s, hipMemcpy(s->icidx, ci.data(), ci.size() * 4, hipMemcpyHostToDevice));
    SCHK(s, hipMemcpy(s->iccls, cc.data(), cc.size(), hipMemcpyHostToDevice));
    SCHK(s, hipMemcpy(s->ieidx, ei.data(), ei.size() * 4, hipMemcpyHostToDevice));
    SCHK(s, hipMemcpy(s->iecls, ec.data(), ec.size(), hipMemcpyHostToDevice));
    return LTS_OK;
}

// Stage buffers for L = 3M layers and the per-layer coefficients: tau of the
// fine stage time (SSPRK3 stages at t_k, t_k + dt/M, t_k + dt/(2M)) and the
// interface-1 prediction of Algorithm 2.2 (Steps 3.1.1, 3.2.1, 3.3.1).
template <typename T>
lts_status stage_buffers(lts_sur* s, int M) {
    lts_ctx* c = s->c;
    const int L = 3 * M;
    if (s->L == L) return LTS_OK;
    SCHK(s, hipStreamSynchronize(s->s));
    for (void** b : {&s->hS, &s->uS, &s->qS, &s->zsS, &s->accH, &s->accU,
                     reinterpret_cast<void**>(&s->icoef)}) {
        if (*b) {
            s->allocs.erase(std::find(s->allocs.begin(), s->allocs.end(), *b));
            (void)hipFree(*b);
            *b = nullptr;
        }
    }
    s->L = 0;
    const size_t ts = sizeof(T) * (size_t)L;
    const int nIc = c->cb[5] - c->cb[3], nIe = c->eb[4] - c->eb[2];
    lts_status st;
    if ((st = salloc(s, &s->hS, c->nC * ts)) || (st = salloc(s, &s->uS, c->nE * ts)) ||
        (st = salloc(s, &s->qS, c->nV * ts)) || (st = salloc(s, &s->zsS, 2 * c->nE * ts)) ||
        (st = salloc(s, &s->accH, nIc * ts)) || (st = salloc(s, &s->accU, nIe * ts)) ||
        (st = salloc(s, &s->icoef, (size_t)L * 4 * 8)))
        return st;
    // elements the pass reads but nothing fills stay at zero
    SCHK(s, hipMemset(s->hS, 0, c->nC * ts));
    SCHK(s, hipMemset(s->uS, 0, c->nE * ts));
    std::vector<double> cf(4 * (size_t)L);
    const double frac[3] = {0.0, 1.0, 0.5};
    for (int k = 0; k < M; ++k)
        for (int st3 = 0; st3 < 3; ++st3) {
            double* q = cf.data() + 4 * (3 * k + st3);
            q[0] = (k + frac[st3]) / M;
            Run<double>::predict_coeffs(st3, k, M, q + 1, 3);
        }
    SCHK(s, hipMemcpy(s->icoef, cf.data(), cf.size() * 8, hipMemcpyHostToDevice));
    s->L = L;
    return LTS_OK;
}

template <typename T>
lts_status setup_typed(lts_sur* s) {
    lts_ctx* c = s->c;
    lts_status st;
    const size_t ts = sizeof(T);
    if ((st = salloc(s, &s->Sh, c->nC * ts)) || (st = salloc(s, &s->Su, c->nE * ts)) ||
        (st = salloc(s, &s->R0h, s->nF * ts)) || (st = salloc(s, &s->R0u, s->nFe * ts)) ||
        (st = salloc(s, &s->R1h, s->nF * ts)) || (st = salloc(s, &s->R1u, s->nFe * ts)) ||
        (st = salloc(s, &s->Ph, s->nF * ts)) || (st = salloc(s, &s->Pu, s->nFe * ts)) ||
        (st = salloc(s, &s->mpart, (size_t)nn::mass_fix_parts(c->nC) * 8)) ||
        (st = salloc(s, &s->mshift, 8)))
        return st;
    const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
    if ((st = interface_read_set<T>(s))) return st;
    double af = 0.0;
    for (int i = 0; i < s->nF; ++i) af += (double)(T)c->area_perm[i];
    s->inv_area_f = 1.0 / af;
    SCHK(s, hipMemsetAsync(s->ec0, 0xFF, s->nFe * 4, s->s));
    SCHK(s, hipMemsetAsync(s->ec1, 0xFF, s->nFe * 4, s->s));
    nn::build_graph<T>(dm, s->N, s->nFe, s->adj, s->inv_deg, s->node_edges, s->ec0, s->ec1, s->s);
    SCHK(s, hipGetLastError());
    // every fine edge must have found both of its cells among the nodes
    std::vector<int32_t> e0(s->nFe), e1(s->nFe);
    SCHK(s, hipMemcpyAsync(e0.data(), s->ec0, s->nFe * 4, hipMemcpyDeviceToHost, s->s));
    SCHK(s, hipMemcpyAsync(e1.data(), s->ec1, s->nFe * 4, hipMemcpyDeviceToHost, s->s));
    SCHK(s, hipStreamSynchronize(s->s));
    for (int e = 0; e < s->nFe; ++e)
        if (e0[e] < 0 || e0[e] >= s->N || e1[e] < 0 || e1[e] >= s->N || e0[e] == e1[e])
            return sfail(s, LTS_ELABEL, "a fine edge lacks one of its cells among the nodes");
    return LTS_OK;
}

template <typename T>
void features_of_state(lts_sur* s, float* raw) {
    lts_ctx* c = s->c;
    const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
    nn::features<T>(dm, (const T*)c->Ah, (const T*)c->Au, s->N, s->cb1, s->cb3, s->cb4, raw, s->s);
}

// R(x) on the fine cells and fine edges into (Rh, Ru).
template <typename T>
lts_status fine_rhs(lts_sur* s, const T* h, const T* u, T* Rh, T* Ru, bool timed = false) {
    lts_ctx* c = s->c;
    const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
    Run<T> r{c, dm, s->s, timed};
    const Seg<T> none;
    return r.pass(P_STEP3, h, u, Run<T>::upd(0, c->cb[3], Rh, nullptr, 0, nullptr, 0, 1.0), none,
                  Run<T>::upd(0, c->eb[2], Ru, nullptr, 0, nullptr, 0, 1.0), none);
}

template <typename T>
lts_status record_typed(lts_sur* s, double dt, int M, int n) {
    lts_ctx* c = s->c;
    for (int k = 0; k < n; ++k) {
        features_of_state<T>(s, s->raw_s + (size_t)s->S * s->N * nn::kFeat);
        SCHK(s, hipMemcpyAsync(s->Sh, c->Ah, c->nC * sizeof(T), hipMemcpyDeviceToDevice, s->s));
        SCHK(s, hipMemcpyAsync(s->Su, c->Au, c->nE * sizeof(T), hipMemcpyDeviceToDevice, s->s));
        lts_status st = fine_rhs<T>(s, (const T*)c->Ah, (const T*)c->Au, (T*)s->R0h, (T*)s->R0u);
        if (st) return sfail(s, st, std::string("right-hand side: ") + lts_last_error(c));
        st = lts_step(c, dt, M, 1);
        if (st) return sfail(s, st, std::string("LTS3 step: ") + lts_last_error(c));
        nn::increments<T>((const T*)s->Sh, (const T*)s->Su, (const T*)c->Ah, (const T*)c->Au,
                          (const T*)s->R0h, (const T*)s->R0u, dt, s->nF, s->nFe,
                          s->tgt_s + (size_t)s->S * (s->nF + s->nFe), s->s);
        SCHK(s, hipGetLastError());
        ++s->S;
    }
    SCHK(s, hipStreamSynchronize(s->s));
    return LTS_OK;
}

// The surrogate coarse step up to the gate sums (captured once per dt, M).
// F: the network's prediction.  I1, I2, C: Algorithm 2.2 with the fine
// substeps replaced by the surrogate: Steps 1 and 2 (coarse stages on
// underlined F, I and C), the interface accumulation of Step 3 over all 3M
// fine stages at once (F read linearly in time between x_n and the
// prediction, I1 predicted, I2 and C at the coarse stages), Step 4 on C,
// Step 5 on I.  Then the mass change of the whole step is removed from F as
// a uniform thickness shift, so mass is conserved to rounding.  With timed,
// the right-hand-side passes are event-stamped (the context's timing mode;
// the step is then launched directly, not captured).
template <typename T>
lts_status enqueue_sur_step(lts_sur* s, double dt, int M, bool timed = false) {
    lts_ctx* c = s->c;
    const DevMesh<T>& dm = *static_cast<DevMesh<T>*>(c->dm);
    Run<T> r{c, dm, s->s, timed};
    T *Ah = (T*)c->Ah, *Au = (T*)c->Au, *Bh = (T*)c->Bh, *Bu = (T*)c->Bu, *Ch = (T*)c->Ch,
      *Cu = (T*)c->Cu;
    T *R0h = (T*)s->R0h, *R0u = (T*)s->R0u, *R1h = (T*)s->R1h, *R1u = (T*)s->R1u;
    T *Ph = (T*)s->Ph, *Pu = (T*)s->Pu, *Sh = (T*)s->Sh, *Su = (T*)s->Su;
    const int* cb = c->cb;
    const int* eb = c->eb;
    const int nC = c->nC, nE = c->nE, L = s->L;
    const Seg<T> none;
    lts_status st;
    SCHK(s, hipMemcpyAsync(Sh, Ah, nC * sizeof(T), hipMemcpyDeviceToDevice, s->s));
    SCHK(s, hipMemcpyAsync(Su, Au, nE * sizeof(T), hipMemcpyDeviceToDevice, s->s));
    // R(x_n) on F
    if ((st = fine_rhs<T>(s, Ah, Au, R0h, R0u, timed))) return st;
    // F at t + dt: a forward-Euler step plus the network's correction
    features_of_state<T>(s, s->raw);
    nn::norm_features(s->raw, s->N, s->norm, s->norm + 5, s->X, s->s);
    forward(s, nullptr, nullptr, nullptr);
    nn::apply_increments<T>(Ah, Au, R0h, R0u, dt, s->out_h, s->out_u, s->norm + 12, s->nF, s->nFe,
                            Ph, Pu, s->s);
    // Steps 1 and 2, with the interface-1 copies of X0, X1, X2
    if ((st = r.pass(P_STEP1, Ah, Au,
                     Run<T>::mirror(Run<T>::upd(cb[1], nC, Bh, nullptr, 0, Ah, 1, dt), cb[3],
                                    cb[4], (T*)c->x1h, (T*)c->x0h),
                     none,
                     Run<T>::mirror(Run<T>::upd(eb[1], nE, Bu, nullptr, 0, Au, 1, dt), eb[2],
                                    eb[3], (T*)c->x1u, (T*)c->x0u),
                     none)))
        return st;
    if ((st = r.pass(P_STEP2, Bh, Bu,
                     Run<T>::mirror(Run<T>::upd(cb[3], nC, Ch, Ah, 0.75, Bh, 0.25, 0.25 * dt),
                                    cb[3], cb[4], (T*)c->x2h, nullptr),
                     none,
                     Run<T>::mirror(Run<T>::upd(eb[2], nE, Cu, Au, 0.75, Bu, 0.25, 0.25 * dt),
                                    eb[2], eb[3], (T*)c->x2u, nullptr),
                     none)))
        return st;
    // Step 3 on the interface only: the 3M stage states are all known, so
    // their right-hand sides run as one layered pass (layer 3k + s)
    const nn::IfaceSrc<T> hsrc{Sh, Bh, Ch, Ph, (T*)c->x0h, (T*)c->x1h, (T*)c->x2h};
    const nn::IfaceSrc<T> usrc{Su, Bu, Cu, Pu, (T*)c->x0u, (T*)c->x1u, (T*)c->x2u};
    nn::iface_fill<T>(s->icidx, s->iccls, s->nicl, s->ieidx, s->iecls, s->niel, L, s->icoef, hsrc,
                      usrc, cb[3], eb[2], (T*)s->hS, (T*)s->uS, s->s);
    SCHK(s, hipGetLastError());
    const PassPlan& P = c->iface_plan;
    SCHK(s, launch_vertex_l<T>(dm, (T*)s->hS, (T*)s->uS, (T*)s->qS, P.v_lo, P.v_hi, L, s->s));
    SCHK(s, launch_cell_l<T>(dm, (T*)s->hS, (T*)s->uS, (T*)s->qS, (T*)s->zsS, P.c_lo, P.c_hi, L,
                             (T)c->g, Run<T>::accum(cb[3], cb[5], (T*)s->accH, 1.0, true), none,
                             c->flag, s->s));
    SCHK(s, launch_edge_l<T>((T*)s->zsS, nE, P.et_lo, P.et_hi, L,
                             Run<T>::accum(eb[2], eb[4], (T*)s->accU, 1.0, true), none, Aux<T>(),
                             c->flag, s->s));
    // Step 4 on C (reads X2 on I2 and C only)
    if ((st = r.pass(P_STEP4, Ch, Cu,
                     Run<T>::upd(cb[5], nC, Ah, Ah, 1.0 / 3.0, Ch, 2.0 / 3.0, 2.0 / 3.0 * dt),
                     none,
                     Run<T>::upd(eb[4], nE, Au, Au, 1.0 / 3.0, Cu, 2.0 / 3.0, 2.0 / 3.0 * dt),
                     none)))
        return st;
    // Step 5 on I1 u I2, and F from the surrogate
    nn::iface_combine<T>((T*)s->accH, (T*)s->accU, cb[5] - cb[3], eb[4] - eb[2], L, dt / M, cb[3],
                         eb[2], Sh, Su, Ah, Au, s->s);
    SCHK(s, hipMemcpyAsync(Ah, Ph, s->nF * sizeof(T), hipMemcpyDeviceToDevice, s->s));
    SCHK(s, hipMemcpyAsync(Au, Pu, s->nFe * sizeof(T), hipMemcpyDeviceToDevice, s->s));
    nn::mass_fix<T>(dm.area, Sh, Ah, nC, s->nF, s->inv_area_f, s->mpart, s->mshift, s->s);
    // R(x_new) on F and the residual sums
    if ((st = fine_rhs<T>(s, Ah, Au, R1h, R1u, timed))) return st;
    nn::gate_sums<T>((const T*)Sh, (const T*)Su, Ah, Au, R0h, R0u, R1h, R1u, s->nF, s->nFe, dt,
                     s->dpart, s->gout, s->s);
    return LTS_OK;
}

template <typename T>
lts_status capture_step(lts_sur* s, double dt, int M) {
    lts_ctx* c = s->c;
    if (s->gexec && s->g_dt == dt && s->g_M == M) return LTS_OK;
    lts_status st0 = stage_buffers<T>(s, M);
    if (st0) return st0;
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
    // the surrogate's passes flag non-finite values in the surrogate's own
    // word, so a rejected step leaves the context's flag untouched
    int* saved = c->flag;
    c->flag = s->flag;
    SCHK(s, hipStreamBeginCapture(s->s, hipStreamCaptureModeThreadLocal));
    lts_status st = enqueue_sur_step<T>(s, dt, M);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(s->s, &gr);
    c->flag = saved;
    if (st) {
        if (gr) (void)hipGraphDestroy(gr);
        return sfail(s, st, std::string("surrogate step: ") + c->err);
    }
    if (e != hipSuccess) return sfail(s, LTS_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
    s->graph = gr;
    SCHK(s, hipGraphInstantiate(&s->gexec, gr, nullptr, nullptr, 0));
    s->g_dt = dt;
    s->g_M = M;
    return LTS_OK;
}

template <typename T>
lts_status sur_step_typed(lts_sur* s, double dt, int M, int n, double tau, int max_backoff,
                          int* n_acc, double* resid) {
    lts_ctx* c = s->c;
    lts_status st;
    if ((st = capture_step<T>(s, dt, M))) return st;
    int acc = 0;
    for (int k = 0; k < n; ++k) {
        if (s->skip > 0) {  // backing off after a rejection: plain LTS3
            --s->skip;
            if (resid) resid[k] = -1.0;
            if ((st = lts_step(c, dt, M, 1)))
                return sfail(s, st, std::string("LTS3 step: ") + lts_last_error(c));
            continue;
        }
        if (c->timing) {  // event-stamped passes: the step is launched, not replayed
            int* saved = c->flag;
            c->flag = s->flag;
            st = enqueue_sur_step<T>(s, dt, M, true);
            c->flag = saved;
            if (st) return sfail(s, st, std::string("surrogate step: ") + c->err);
        } else {
            SCHK(s, hipGraphLaunch(s->gexec, s->s));
        }
        SCHK(s, hipMemcpyAsync(s->host4, s->gout, 6 * sizeof(double), hipMemcpyDeviceToHost, s->s));
        SCHK(s, hipStreamSynchronize(s->s));
        const double* o = s->host4;
        // ||defect|| / ((||R(x_n)|| + ||R(x_pred)||) / 2), per field
        auto ratio = [](double num, double d0, double d1) {
            const double den = 0.5 * (std::sqrt(d0) + std::sqrt(d1));
            if (den > 0.0) return std::sqrt(num) / den;
            return num > 0.0 || std::isnan(num) ? std::numeric_limits<double>::infinity() : 0.0;
        };
        double r = std::max(ratio(o[0], o[1], o[2]), ratio(o[3], o[4], o[5]));
        for (int q = 0; q < 6; ++q)
            if (std::isnan(o[q])) r = std::numeric_limits<double>::quiet_NaN();
        if (resid) resid[k] = r;
        if (std::isfinite(r) && r < tau) {
            ++acc;
            c->t += dt;
            c->steps += 1;
            s->backoff = 0;
        } else {
            c->gate_fallbacks += 1;
            s->backoff = std::min(max_backoff, s->backoff ? 2 * s->backoff : 1);
            s->skip = s->backoff;
            SCHK(s, hipMemcpyAsync(c->Ah, s->Sh, c->nC * sizeof(T), hipMemcpyDeviceToDevice, s->s));
            SCHK(s, hipMemcpyAsync(c->Au, s->Su, c->nE * sizeof(T), hipMemcpyDeviceToDevice, s->s));
            // the context stream runs the fallback; order it after the copies
            if (s->s != c->stream) SCHK(s, hipStreamSynchronize(s->s));
            if ((st = lts_step(c, dt, M, 1)))
                return sfail(s, st, std::string("LTS3 fallback: ") + lts_last_error(c));
        }
    }
    if (n_acc) *n_acc = acc;
    SCHK(s, hipStreamSynchronize(c->stream));
    return LTS_OK;
}

lts_status train_iter(lts_sur* s, int k, float* loss_slot) {
    if (k < 0 || k >= s->S) return sfail(s, LTS_EINVAL, "sample index out of range");
    const size_t nT = (size_t)s->nF + s->nFe;
    nn::norm_features(s->raw_s + (size_t)k * s->N * nn::kFeat, s->N, s->norm, s->norm + 5, s->X,
                      s->s);
    const float* th = s->tgt_s + (size_t)k * nT;
    forward(s, th, th + s->nF, loss_slot);
    backward(s);
    return LTS_OK;
}

}  // namespace

extern "C" {

lts_status lts_sur_create(lts_sur** out, lts_ctx* c, int n_layers, int hidden, uint64_t seed,
                          int max_samples) {
    if (!out || !c) return LTS_EINVAL;
    *out = nullptr;
    if (n_layers != kLayers || hidden != nn::kHid || max_samples < 0) {
        c->err = "surrogate: only 3 layers of width 64 are supported";
        return LTS_EINVAL;
    }
    if (!c->has_mesh || !c->has_state) {
        c->err = "surrogate: context needs a mesh and a state";
        return LTS_EINVAL;
    }
    if (c->L != 1) {
        c->err = "surrogate: single-layer contexts only";
        return LTS_EINVAL;
    }
    lts_sur* s = new lts_sur();
    s->c = c;
    s->dm_at_create = c->dm;
    s->s = c->stream;
    s->N = c->cb[5];
    s->nF = c->cb[3];
    s->nFe = c->eb[2];
    s->cb1 = c->cb[1];
    s->cb3 = c->cb[3];
    s->cb4 = c->cb[4];
    s->aw = padded_slots(c->maxE);
    s->S_cap = max_samples;
    if (s->nF <= 0 || s->nFe <= 0) {
        c->err = "surrogate: empty fine region";
        delete s;
        return LTS_EINVAL;
    }
    const size_t N = s->N, nT = (size_t)s->nF + s->nFe;
    const int np_tn = nn::gemm_tn_parts(s->N, RPB);
    const size_t part = std::max<size_t>(
        {(size_t)np_tn * 128 * 64, (size_t)nn::heads_back_parts(s->N) * 129,
         (size_t)nn::heads_parts(s->nF, s->nFe), (size_t)nn::colsum_parts(s->N, RPB) * 64});
    lts_status st;
    auto fail_out = [&](lts_status e) {
        c->err = s->err;
        lts_sur_destroy(s);
        return e;
    };
    if ((st = salloc(s, &s->adj, N * s->aw * 4)) || (st = salloc(s, &s->node_edges, N * s->aw * 4)) ||
        (st = salloc(s, &s->ec0, s->nFe * 4)) || (st = salloc(s, &s->ec1, s->nFe * 4)) ||
        (st = salloc(s, &s->inv_deg, N * 4)) ||
        (st = salloc(s, &s->raw_s, (size_t)max_samples * N * nn::kFeat * 4)) ||
        (st = salloc(s, &s->tgt_s, (size_t)max_samples * nT * 4)) ||
        (st = salloc(s, &s->raw, N * nn::kFeat * 4)) || (st = salloc(s, &s->X, N * nn::kFeat * 2)) ||
        (st = salloc(s, &s->H3, N * 64 * 2)) || (st = salloc(s, &s->dZ, N * 64 * 2)) ||
        (st = salloc(s, &s->dH, N * 64 * 4)) || (st = salloc(s, &s->dHn, N * 64 * 4)) ||
        (st = salloc(s, &s->p, N_PARAMS * 4)) || (st = salloc(s, &s->g, N_PARAMS * 4)) ||
        (st = salloc(s, &s->m, N_PARAMS * 4)) || (st = salloc(s, &s->v, N_PARAMS * 4)) ||
        (st = salloc(s, &s->bf_map, N_PARAMS * 4)) || (st = salloc(s, &s->wbf, N_WBF * 2)) ||
        (st = salloc(s, &s->out_h, s->nF * 4)) || (st = salloc(s, &s->out_u, s->nFe * 4)) ||
        (st = salloc(s, &s->gh, s->nF * 4)) || (st = salloc(s, &s->gu, s->nFe * 4)) ||
        (st = salloc(s, &s->part, part * 4)) || (st = salloc(s, &s->norm, 16 * 4)) ||
        (st = salloc(s, &s->dpart, 256 * 12 * 8)) || (st = salloc(s, &s->gout, 6 * 8)) ||
        (st = salloc(s, &s->flag, 64)))
        return fail_out(st);
    for (int l = 0; l < kLayers; ++l) {
        if ((st = salloc(s, &s->HC[l], N * 128 * 2)) || (st = salloc(s, &s->wt[l], 128 * 64 * 2)))
            return fail_out(st);
    }
    // the gate sums need one partial per 256 fine elements
    const size_t gparts = (nT + 255) / 256;
    if (gparts * 6 > 256 * 12) {
        double* gp = nullptr;
        if ((st = salloc(s, &gp, gparts * 6 * 8))) return fail_out(st);
        s->dpart = gp;
    }
    if (hipHostMalloc((void**)&s->host4, 6 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        s->err = "hipHostMalloc failed";
        return fail_out(LTS_ENOMEM);
    }
    std::vector<int32_t> bmap(N_PARAMS, -1);
    for (int i = 0; i < 16 * 64; ++i) bmap[OFF_W0 + i] = i;
    for (int l = 1; l <= kLayers; ++l)
        for (int i = 0; i < 128 * 64; ++i) bmap[off_w(l) + i] = off_wbf(l) + i;
    std::vector<float> p0 = init_params(seed);
    const float norm0[16] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0};
    memcpy(s->norm_host, norm0, sizeof(norm0));
    if (hipMemcpy(s->bf_map, bmap.data(), N_PARAMS * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->p, p0.data(), N_PARAMS * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->norm, norm0, sizeof(norm0), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->m, 0, N_PARAMS * 4) != hipSuccess ||
        hipMemset(s->v, 0, N_PARAMS * 4) != hipSuccess ||
        hipMemset(s->flag, 0, 64) != hipSuccess) {
        s->err = "surrogate: initial upload failed";
        return fail_out(LTS_EDEVICE);
    }
    st = c->prec == LTS_FP64 ? setup_typed<double>(s) : setup_typed<float>(s);
    if (st) return fail_out(st);
    refresh_bf16(s);
    if (hipStreamSynchronize(s->s) != hipSuccess) {
        s->err = "surrogate: set-up kernels failed";
        return fail_out(LTS_EDEVICE);
    }
    *out = s;
    return LTS_OK;
}

lts_status lts_sur_info(const lts_sur* s, int* n_nodes, int* nF, int* nFe, int* n_params,
                        int* n_samples) {
    if (!s) return LTS_EINVAL;
    if (n_nodes) *n_nodes = s->N;
    if (nF) *nF = s->nF;
    if (nFe) *nFe = s->nFe;
    if (n_params) *n_params = N_PARAMS;
    if (n_samples) *n_samples = s->S;
    return LTS_OK;
}

lts_status lts_sur_node_map(const lts_sur* s, int32_t* node_cell, int32_t* fine_edge) {
    if (!s) return LTS_EINVAL;
    if (s->c->dm != s->dm_at_create) return LTS_EINVAL;
    if (node_cell)
        for (int i = 0; i < s->N; ++i) node_cell[i] = s->c->cperm[i];
    if (fine_edge)
        for (int e = 0; e < s->nFe; ++e) fine_edge[e] = s->c->eperm[e];
    return LTS_OK;
}

lts_status lts_sur_record(lts_sur* s, double dt, int M, int n) {
    lts_status st = check(s);
    if (st) return st;
    if (n < 0 || s->S + n > s->S_cap) return sfail(s, LTS_EINVAL, "sample capacity exceeded");
    if (!(dt > 0) || M < 1) return sfail(s, LTS_EINVAL, "need dt > 0 and M >= 1");
    return s->c->prec == LTS_FP64 ? record_typed<double>(s, dt, M, n)
                                  : record_typed<float>(s, dt, M, n);
}

lts_status lts_sur_normalize(lts_sur* s, int n) {
    if (!s) return LTS_EINVAL;
    if (n < 1 || n > s->S) return sfail(s, LTS_EINVAL, "need 1 <= n_samples <= recorded samples");
    nn::feature_stats(s->raw_s, (long)n * s->N, s->tgt_s, n, s->nF, s->nFe, s->dpart, s->norm, s->s);
    SCHK(s, hipMemcpyAsync(s->norm_host, s->norm, 16 * 4, hipMemcpyDeviceToHost, s->s));
    SCHK(s, hipStreamSynchronize(s->s));
    s->has_norm = true;
    return LTS_OK;
}

lts_status lts_sur_set_norm(lts_sur* s, const float* nrm) {
    if (!s || !nrm) return LTS_EINVAL;
    memcpy(s->norm_host, nrm, 16 * 4);
    SCHK(s, hipMemcpyAsync(s->norm, s->norm_host, 16 * 4, hipMemcpyHostToDevice, s->s));
    SCHK(s, hipStreamSynchronize(s->s));
    s->has_norm = true;
    return LTS_OK;
}

lts_status lts_sur_get_norm(const lts_sur* s, float* nrm) {
    if (!s || !nrm) return LTS_EINVAL;
    memcpy(nrm, s->norm_host, 16 * 4);
    return LTS_OK;
}

lts_status lts_sur_get_params(const lts_sur* s, float* p) {
    if (!s || !p) return LTS_EINVAL;
    if (hipMemcpyAsync(p, s->p, N_PARAMS * 4, hipMemcpyDeviceToHost, s->s) != hipSuccess ||
        hipStreamSynchronize(s->s) != hipSuccess)
        return LTS_EDEVICE;
    return LTS_OK;
}

lts_status lts_sur_set_params(lts_sur* s, const float* p) {
    if (!s || !p) return LTS_EINVAL;
    SCHK(s, hipMemcpyAsync(s->p, p, N_PARAMS * 4, hipMemcpyHostToDevice, s->s));
    SCHK(s, hipMemsetAsync(s->m, 0, N_PARAMS * 4, s->s));
    SCHK(s, hipMemsetAsync(s->v, 0, N_PARAMS * 4, s->s));
    s->adam_step = 0;
    refresh_bf16(s);
    SCHK(s, hipStreamSynchronize(s->s));
    return LTS_OK;
}

// File layout (little-endian): 8-byte tag, int32 n_layers, hidden,
// n_params, has_norm, then float norm[16] and float params[n_params].
static const char kSurTag[8] = {'L', 'T', 'S', 'S', 'U', 'R', '0', '1'};

lts_status lts_sur_save(const lts_sur* s, const char* path) {
    if (!s || !path) return LTS_EINVAL;
    std::vector<float> p(N_PARAMS);
    lts_status st = lts_sur_get_params(s, p.data());
    if (st) return st;
    const int32_t hdr[4] = {kLayers, nn::kHid, N_PARAMS, s->has_norm ? 1 : 0};
    FILE* f = std::fopen(path, "wb");
    if (!f) return LTS_EINVAL;
    bool ok = std::fwrite(kSurTag, 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 &&
              std::fwrite(s->norm_host, 4, 16, f) == 16 &&
              std::fwrite(p.data(), 4, N_PARAMS, f) == (size_t)N_PARAMS;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? LTS_OK : LTS_EINVAL;
}

lts_status lts_sur_load(lts_sur* s, const char* path) {
    if (!s || !path) return LTS_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return sfail(s, LTS_EINVAL, std::string("cannot open ") + path);
    char tag[8];
    int32_t hdr[4];
    float nrm[16];
    std::vector<float> p(N_PARAMS);
    bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, kSurTag, 8) == 0 &&
              std::fread(hdr, 4, 4, f) == 4 && hdr[0] == kLayers && hdr[1] == nn::kHid &&
              hdr[2] == N_PARAMS && std::fread(nrm, 4, 16, f) == 16 &&
              std::fread(p.data(), 4, N_PARAMS, f) == (size_t)N_PARAMS;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the parameters
    std::fclose(f);
    if (!ok) return sfail(s, LTS_EINVAL, std::string("not a surrogate file of this shape: ") + path);
    lts_status st;
    if (hdr[3] && (st = lts_sur_set_norm(s, nrm))) return st;
    return lts_sur_set_params(s, p.data());
}

lts_status lts_sur_train(lts_sur* s, const int32_t* idx, int n, float lr, float* losses) {
    if (!s || (n > 0 && !idx) || n < 0) return LTS_EINVAL;
    if (!s->has_norm) return sfail(s, LTS_EINVAL, "normalisation not set");
    if (n > s->loss_cap) {
        float* l = nullptr;
        lts_status st = salloc(s, &l, (size_t)n * 4);
        if (st) return st;
        s->losses = l;
        s->loss_cap = n;
    }
    for (int i = 0; i < n; ++i) {
        lts_status st = train_iter(s, idx[i], s->losses + i);
        if (st) return st;
        nn::adam(s->p, s->g, s->m, s->v, N_PARAMS, lr, 0.9f, 0.999f, 1e-8f, ++s->adam_step,
                 s->bf_map, s->wbf, s->s);
        for (int l = 1; l <= kLayers; ++l)
            nn::transpose_halves(s->wbf + off_wbf(l), s->wt[l - 1], s->s);
    }
    SCHK(s, hipGetLastError());
    if (losses && n > 0)
        SCHK(s, hipMemcpyAsync(losses, s->losses, (size_t)n * 4, hipMemcpyDeviceToHost, s->s));
    SCHK(s, hipStreamSynchronize(s->s));
    return LTS_OK;
}

lts_status lts_sur_grad(lts_sur* s, int k, float* loss, float* grad) {
    if (!s) return LTS_EINVAL;
    if (!s->has_norm) return sfail(s, LTS_EINVAL, "normalisation not set");
    if (s->loss_cap < 1) {
        float* l = nullptr;
        lts_status st = salloc(s, &l, 4);
        if (st) return st;
        s->losses = l;
        s->loss_cap = 1;
    }
    lts_status st = train_iter(s, k, s->losses);
    if (st) return st;
    SCHK(s, hipGetLastError());
    if (loss) SCHK(s, hipMemcpyAsync(loss, s->losses, 4, hipMemcpyDeviceToHost, s->s));
    if (grad) SCHK(s, hipMemcpyAsync(grad, s->g, N_PARAMS * 4, hipMemcpyDeviceToHost, s->s));
    SCHK(s, hipStreamSynchronize(s->s));
    return LTS_OK;
}

lts_status lts_sur_features(lts_sur* s, float* raw) {
    lts_status st = check(s);
    if (st) return st;
    if (!raw) return LTS_EINVAL;
    if (s->c->prec == LTS_FP64) features_of_state<double>(s, s->raw);
    else features_of_state<float>(s, s->raw);
    SCHK(s, hipGetLastError());
    SCHK(s, hipMemcpyAsync(raw, s->raw, (size_t)s->N * nn::kFeat * 4, hipMemcpyDeviceToHost, s->s));
    SCHK(s, hipStreamSynchronize(s->s));
    return LTS_OK;
}

lts_status lts_sur_predict(lts_sur* s, float* oh, float* ou) {
    lts_status st = check(s);
    if (st) return st;
    if (s->c->prec == LTS_FP64) features_of_state<double>(s, s->raw);
    else features_of_state<float>(s, s->raw);
    nn::norm_features(s->raw, s->N, s->norm, s->norm + 5, s->X, s->s);
    forward(s, nullptr, nullptr, nullptr);
    SCHK(s, hipGetLastError());
    if (oh) SCHK(s, hipMemcpyAsync(oh, s->out_h, (size_t)s->nF * 4, hipMemcpyDeviceToHost, s->s));
    if (ou) SCHK(s, hipMemcpyAsync(ou, s->out_u, (size_t)s->nFe * 4, hipMemcpyDeviceToHost, s->s));
    SCHK(s, hipStreamSynchronize(s->s));
    return LTS_OK;
}

lts_status lts_sur_step(lts_sur* s, double dt, int M, int n, double tau, int max_backoff,
                        int* n_acc, double* resid) {
    lts_status st = check(s);
    if (st) return st;
    if (!(dt > 0) || M < 1 || n < 0) return sfail(s, LTS_EINVAL, "need dt > 0, M >= 1, n >= 0");
    if (!s->has_norm) return sfail(s, LTS_EINVAL, "normalisation not set");
    if (max_backoff < 0) return sfail(s, LTS_EINVAL, "need max_backoff >= 0");
    if (max_backoff == 0) s->skip = s->backoff = 0;
    return s->c->prec == LTS_FP64
               ? sur_step_typed<double>(s, dt, M, n, tau, max_backoff, n_acc, resid)
               : sur_step_typed<float>(s, dt, M, n, tau, max_backoff, n_acc, resid);
}

const char* lts_sur_last_error(const lts_sur* s) { return s ? s->err.c_str() : "null surrogate"; }

void lts_sur_destroy(lts_sur* s) {
    if (!s) return;
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    (void)hipStreamSynchronize(s->s);
    for (void* q : s->allocs) (void)hipFree(q);
    if (s->host4) (void)hipHostFree(s->host4);
    delete s;
}

lts_status lts_nn_gemm_bf16(int device, const uint16_t* A, int N, int K, const uint16_t* W,
                            const float* bias, float* Y) {
    if (!A || !W || !Y || N < 0 || K < 16 || K > 128 || K % 16) return LTS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return LTS_EDEVICE;
    void *dA = nullptr, *dW = nullptr, *dB = nullptr, *dY = nullptr;
    lts_status st = LTS_OK;
    hipStream_t s = nullptr;
    const size_t nA = (size_t)std::max(N, 1) * K;
    if (hipStreamCreate(&s) != hipSuccess || hipMalloc(&dA, nA * 2) != hipSuccess ||
        hipMalloc(&dW, (size_t)K * 64 * 2) != hipSuccess || hipMalloc(&dB, 64 * 4) != hipSuccess ||
        hipMalloc(&dY, (size_t)std::max(N, 1) * 64 * 4) != hipSuccess)
        st = LTS_ENOMEM;
    if (!st && (hipMemcpyAsync(dA, A, (size_t)N * K * 2, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(dW, W, (size_t)K * 64 * 2, hipMemcpyHostToDevice, s) != hipSuccess ||
                (bias && hipMemcpyAsync(dB, bias, 64 * 4, hipMemcpyHostToDevice, s) != hipSuccess)))
        st = LTS_EDEVICE;
    if (!st) {
        nn::gemm((const uint16_t*)dA, K, N, K, (const uint16_t*)dW, bias ? (const float*)dB : nullptr,
                 0, nullptr, 0, (float*)dY, s);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(Y, dY, (size_t)N * 64 * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = LTS_EDEVICE;
    }
    for (void* q : {dA, dW, dB, dY})
        if (q) (void)hipFree(q);
    if (s) (void)hipStreamDestroy(s);
    return st;
}

lts_status lts_nn_gemm_tn_bf16(int device, const uint16_t* A, int N, int K, const uint16_t* D,
                               float* P) {
    if (!A || !D || !P || N < 0 || K < 16 || K > 128 || K % 16) return LTS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return LTS_EDEVICE;
    void *dA = nullptr, *dD = nullptr, *dPart = nullptr, *dP = nullptr;
    lts_status st = LTS_OK;
    hipStream_t s = nullptr;
    const int np = std::max(1, nn::gemm_tn_parts(N, RPB));
    const size_t n1 = (size_t)std::max(N, 1);
    if (hipStreamCreate(&s) != hipSuccess || hipMalloc(&dA, n1 * K * 2) != hipSuccess ||
        hipMalloc(&dD, n1 * 64 * 2) != hipSuccess ||
        hipMalloc(&dPart, (size_t)np * K * 64 * 4) != hipSuccess ||
        hipMalloc(&dP, (size_t)K * 64 * 4) != hipSuccess)
        st = LTS_ENOMEM;
    if (!st && (hipMemcpyAsync(dA, A, (size_t)N * K * 2, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(dD, D, (size_t)N * 64 * 2, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemsetAsync(dP, 0, (size_t)K * 64 * 4, s) != hipSuccess))
        st = LTS_EDEVICE;
    if (!st) {
        nn::gemm_tn((const uint16_t*)dA, K, N, K, (const uint16_t*)dD, RPB, (float*)dPart,
                    (float*)dP, s);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(P, dP, (size_t)K * 64 * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = LTS_EDEVICE;
    }
    for (void* q : {dA, dD, dPart, dP})
        if (q) (void)hipFree(q);
    if (s) (void)hipStreamDestroy(s);
    return st;
}

lts_status lts_nn_gemm_bf16_device(const uint16_t* A, int N, int K, const uint16_t* W,
                                   const float* bias, float* Y_f32, uint16_t* Y_bf16,
                                   void* stream) {
    if (N < 0 || K < 16 || K > 128 || K % 16) return LTS_EINVAL;
    if (N == 0) return LTS_OK;
    if (!A || !W || (!Y_f32 && !Y_bf16)) return LTS_EINVAL;
    // the kernel reads W, A and the bias in 16-byte pieces and writes Y_f32
    // in 16-byte and Y_bf16 in 8-byte pieces
    auto mis = [](const void* p, uintptr_t a) { return p && (uintptr_t)p % a != 0; };
    if (mis(W, 16) || mis(A, 16) || mis(bias, 16) || mis(Y_f32, 16) || mis(Y_bf16, 8))
        return LTS_EINVAL;
    nn::gemm(A, K, N, K, W, bias, 1, Y_bf16, 64, Y_f32, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? LTS_OK : LTS_EDEVICE;
}

}  // extern "C"
