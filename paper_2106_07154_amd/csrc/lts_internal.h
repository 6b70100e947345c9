// Internal declarations shared by the host runtime (lts_api.cpp) and the HIP
// kernels (lts_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lts.h"

namespace lts {

// Thickness storage form of a precision: FP32 contexts store the perturbation
// eta = h - href (see DevMesh::href), FP64 contexts h itself.
template <typename T>
constexpr bool perturbation_form() {
    return sizeof(T) < sizeof(double);
}

// Device mesh, permuted so that every LTS region is a contiguous range.
// Per-cell slot tables are compact: the n_i slots of cell i (counter-
// clockwise) are entries cso[i].x .. cso[i].x + n_i - 1, cells one after
// another in device order, no padding.  The cell kernels give each slot its
// own lane: 8 lanes per cell in the single-range kernel (cells with more
// than 8 edges take appended 16-lane blocks), G = padded_slots(maxE) in the
// batched kernel; lanes past n_i re-read the cell's last entry (a cache line
// already fetched) and zero its coefficients in registers.  A wavefront's
// table reads are one contiguous run of about 6 entries per cell.
template <typename T>
struct DevMesh {
    int nC, nE, nV, maxE;  // maxE: largest n_i of the mesh
    const int32_t* nEoC;   // [nC] n_i
    const int2* cso;       // [nC] {first slot-table entry of cell i, n_i}
    const int32_t* wide;   // [nwide] cells with more than 8 edges, ascending
    int nwide;
    const int32_t* eoc;    // [slots] edge of slot j (ccw)
    const int32_t* coc;    // [slots] cell across edge j
    const int32_t* voc;    // [slots] vertex between edge j and j+1
    const T* nl;           // [slots] n_{e,i} l_e
    const T* nd;           // [slots] n_{e,i} / d_e
    const T* kc;           // [slots] l_e d_e / (4 A_i)
    const T* kf;           // [slots] A_{i,v_j} / A_i (kite fraction of vertex slot j)
    const T* sb;           // [slots] S_j: kite fractions of the slots before j summed
    const T* sn;           // [nC] S_n: all kite fractions of the cell summed
    const T* area;         // [nC] A_i
    const T* rarea;        // [nC] 1 / A_i
    const T* bot;          // [nC] b_i (diagnostics)
    // Thickness storage.  href == nullptr: the state holds h itself and
    // beta = b.  Otherwise the state holds eta = h - href (perturbation form,
    // used in FP32) and beta = href + b - H_s, so g(h + b) = g(eta + beta) +
    // const and the constant drops out of every gradient.
    // href != nullptr exactly when perturbation_form<T>() holds.
    const T* href;         // [nC] or nullptr
    const T* beta;         // [nC]
    const int32_t* eov;    // [3][nV]
    const int32_t* cov;    // [3][nV]
    const T* tdc;          // [3][nV] t_{e,v} d_e
    const T* kite;         // [3][nV] A_{i,v}
    const T* fA;           // [nV] f_v A_v
    // Layered contexts (L > 1) also keep the slot tables the layered cell
    // kernel reads padded to pG = padded_slots(maxE) entries per cell (cell i
    // at i pG; padding entries repeat the last slot's indices with zero
    // coefficients), so its table addresses follow from i alone instead of
    // waiting for cso[i].  Null otherwise.
    int pG;
    const int32_t *peoc, *pcoc, *pvoc;
    const T *pnl, *pnd, *pkc, *pkf;
};

// One epilogue segment: targets [lo, hi) of a tendency kernel.
//   mode 1 (update):     out[j] = a_old*xold[j] + a_cur*xcur[j] + a_dt*G, or,
//                        when a_old + a_cur = 1 (convex), the same as
//                        xold[j] + a_cur*(xcur[j] - xold[j]) + a_dt*G: exact
//                        for xold = xcur whatever the rounding of a_old and
//                        a_cur (in FP32, 1/3 + 2/3 rounds to 1 + 3e-8, which
//                        the first form would apply to the state every step)
//   mode 2 (accumulate): acc[j-lo] = (first ? 0 : acc[j-lo]) + theta*G
//   mode 1 with acc != nullptr also accumulates theta*G into acc (the RK4
//   stage sum).
//   mirror (update only): for j in [mlo, mhi) also store the new value to
//   mnew[j-mlo] and the current value xcur[j] to mcur[j-mlo] (either may be
//   null) -- the interface-1 copies of the coarse stages.
template <typename T>
struct Seg {
    int lo = 0, hi = 0, mode = 0, first = 0;
    T* out = nullptr;
    const T* xold = nullptr;
    const T* xcur = nullptr;
    T a_old = 0, a_cur = 0, a_dt = 0;
    int convex = 0;
    T* acc = nullptr;
    T theta = 0;
    int mlo = 0, mhi = 0;
    T* mnew = nullptr;
    T* mcur = nullptr;
};

// Element-wise work appended to an edge-kernel launch as extra blocks:
//   kind 1 (predict): x[lo+j] = c0 a[j] + c1 b[j] + c2 c[j] in FP64 on the
//                     interface-1 cells (field h) and edges (field u);
//   kind 2 (correct): x[lo+j] = (j < nbase ? base[j] : x[lo+j]) + delta acc[j]
//                     on I1 u I2 cells and edges.
template <typename T>
struct Aux {
    int kind = 0;
    int nh = 0, nu = 0, lo_h = 0, lo_u = 0, nbh = 0, nbu = 0;
    T *xh = nullptr, *xu = nullptr;
    const T *ah = nullptr, *bh = nullptr, *ch = nullptr;
    const T *au = nullptr, *bu = nullptr, *cu = nullptr;
    double c0 = 0, c1 = 0, c2 = 0;
};

enum KernelClass { KC_VERTEX = 0, KC_CELL = 1, KC_EDGE = 2, KC_N = 3 };

// One entry of a batched (ensemble) launch: one member's range for one kernel
// class.  Virtual blocks [first, first + nblk) cover [lo, hi) (G lanes per cell
// for the cell class); for the edge class nblk_aux more blocks run `aux`.
template <typename T>
struct Item {
    DevMesh<T> m;
    const T* h = nullptr;
    const T* u = nullptr;
    T* q = nullptr;
    T* zs = nullptr;
    int* flag = nullptr;
    T g = 0;
    int lo = 0, hi = 0, nblk = 0, nblk_aux = 0, nblk_aux2 = 0, first = 0;
    Seg<T> s0, s1;
    Aux<T> aux, aux2;  // edge items: appended element-wise jobs (blocks after the edges)
};

template <typename T>
hipError_t launch_batch(int kclass, const Item<T>* items, int nitems, int nvb, int block,
                        int grid, int G, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);

// Fused ensemble step (one cooperative launch of 256-thread blocks): phase t,
// kernel class k works on items [off, off + nitems) of the item array with
// nvb virtual blocks; the classes are separated by grid barriers.
struct FusedPhase {
    int off, nitems, nvb;
};
// Grid-barrier workspace in device memory, 128-byte lines of kBarLine words:
// line 0 arrivals of the XCD leaders, 1 generation, 2 error word (non-zero
// once a bounded wait ran out; every block then leaves the kernel), 3 + x
// the number of the launch's blocks running on XCD x (counted at kernel
// start), 19 + x arrivals on XCD x, 35 + x release flag of XCD x (x < 16).
// All zero before the first launch; a completed launch leaves lines 0, 2,
// 3..18 and 19..34 zero again.
constexpr int kBarLine = 32;
constexpr int kBarXcds = 16;
struct FusedBarrier {
    unsigned w[(3 + 3 * kBarXcds) * kBarLine];
};
inline unsigned fused_barrier_error(const FusedBarrier& b) { return b.w[2 * kBarLine]; }
template <typename T>
int fused_blocks_per_cu();  // co-resident 256-thread blocks per CU (0 on error)
template <typename T>
hipError_t launch_fused(const Item<T>* items, const FusedPhase* phases, int nphase,
                        FusedBarrier* bar, int limit, int grid, hipStream_t s,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Launchers (lts_kernels.hip).  All enqueue on `s` and return the launch
// error.  With non-null ev0/ev1 the launch goes through hipExtLaunchKernelGGL,
// which stamps the kernel's own start and end into the two events (timing mode;
// never used while a graph is being captured).
template <typename T>
hipError_t launch_vertex(const DevMesh<T>& m, const T* h, const T* u, T* q, int v_lo,
                         int v_hi, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// Cell kernel over [c_lo, c_hi): 8 lanes per cell; cells with more than 8
// edges (entries [w_lo, w_hi) of m.wide, all inside the range) are taken by
// 16-lane blocks appended to the same launch.
template <typename T>
hipError_t launch_cell(const DevMesh<T>& m, const T* h, const T* u, const T* q, T* zs,
                       int c_lo, int c_hi, int w_lo, int w_hi, T g, const Seg<T>& s0,
                       const Seg<T>& s1, int* flag, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_edge(const T* zs, int nE, int lo, int hi, const Seg<T>& s0,
                       const Seg<T>& s1, const Aux<T>& aux, int* flag, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                       const Aux<T>& aux2 = Aux<T>());
// Lanes per cell in the cell kernel for a mesh whose largest cell has maxE edges.
__host__ __device__ inline int padded_slots(int maxE) { return maxE <= 8 ? 8 : 16; }
// Diagnostics partials per block (mass, energy, h_min, h_max, |u|max, nonfinite)
// then a single-block deterministic reduction into out[8] (doubles).
template <typename T>
hipError_t launch_diag(const DevMesh<T>& m, const T* h, const T* u, double g, double* part,
                       int nblk_cells, int nblk_edges, double* out, hipStream_t s, int L = 1);
// Layered forms (L independent layers, every per-element array [element][L]):
// the same passes with one thread per (element, layer).  Aux counts and
// offsets are given in flat (element x layer) units.
template <typename T>
hipError_t launch_vertex_l(const DevMesh<T>& m, const T* h, const T* u, T* q, int v_lo,
                           int v_hi, int L, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_cell_l(const DevMesh<T>& m, const T* h, const T* u, const T* q, T* zs,
                         int c_lo, int c_hi, int L, T g, const Seg<T>& s0, const Seg<T>& s1,
                         int* flag, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_edge_l(const T* zs, int nE, int lo, int hi, int L, const Seg<T>& s0,
                         const Seg<T>& s1, const Aux<T>& aux, int* flag, hipStream_t s,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                         const Aux<T>& aux2 = Aux<T>());
int diag_blocks(int n);
hipError_t launch_fill_int(int* p, int v, hipStream_t s);

}  // namespace lts
