// Internal declarations shared by the host runtime (lts_api.cpp) and the HIP
// kernels (lts_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lts.h"

namespace lts {

// Device mesh in structure-of-arrays form, permuted so that every LTS region
// is a contiguous range.  Per-cell slot tables are slot-major ([slot][cell]) so
// that a wavefront reading slot j of 64 consecutive cells is coalesced.
template <typename T>
struct DevMesh {
    int nC, nE, nV, maxE;
    const int32_t* nEoC;   // [nC]
    const int32_t* eoc;    // [maxE][nC] edge of slot j (ccw)
    const int32_t* coc;    // [maxE][nC] cell across edge j
    const int32_t* voc;    // [maxE][nC] vertex between edge j and j+1
    const T* nl;           // [maxE][nC] n_{e,i} l_e
    const T* nd;           // [maxE][nC] n_{e,i} / d_e
    const T* kc;           // [maxE][nC] l_e d_e / (4 A_i)
    const T* kf;           // [maxE][nC] A_{i,v_j} / A_i (kite fraction of vertex slot j)
    const T* area;         // [nC] A_i
    const T* bot;          // [nC] b_i
    const int32_t* eov;    // [3][nV]
    const int32_t* cov;    // [3][nV]
    const T* tdc;          // [3][nV] t_{e,v} d_e
    const T* kite;         // [3][nV] A_{i,v}
    const T* fA;           // [nV] f_v A_v
};

// One epilogue segment: targets [lo, hi) of a tendency kernel.
//   mode 1 (update):     out[j] = a_old*xold[j] + a_cur*xcur[j] + a_dt*G
//   mode 2 (accumulate): acc[j-lo] = (first ? 0 : acc[j-lo]) + theta*G
template <typename T>
struct Seg {
    int lo = 0, hi = 0, mode = 0, first = 0;
    T* out = nullptr;
    const T* xold = nullptr;
    const T* xcur = nullptr;
    T a_old = 0, a_cur = 0, a_dt = 0;
    T* acc = nullptr;
    T theta = 0;
};

enum KernelClass { KC_VERTEX = 0, KC_CELL = 1, KC_EDGE = 2, KC_PREDICT = 3,
                   KC_CORRECT = 4, KC_COPY = 5, KC_DIAG = 6, KC_N = 7 };

// Launchers (lts_kernels.hip).  All enqueue on `s` and return the launch error.
template <typename T>
hipError_t launch_vertex(const DevMesh<T>& m, const T* h, const T* u, T* q, int v_lo,
                         int v_hi, hipStream_t s);
template <typename T>
hipError_t launch_cell(const DevMesh<T>& m, const T* h, const T* u, const T* q, T* zs,
                       int c_lo, int c_hi, T g, const Seg<T>& s0, const Seg<T>& s1,
                       int* flag, hipStream_t s);
template <typename T>
hipError_t launch_edge(const T* zs, int nE, int lo, int hi, const Seg<T>& s0,
                       const Seg<T>& s1, int* flag, hipStream_t s);
// x[lo + j] = c0*a[j] + c1*b[j] + c2*c[j] in FP64, j < n, for two fields.
template <typename T>
hipError_t launch_predict(T* xh, const T* ah, const T* bh, const T* ch, int lo_h, int nh,
                          T* xu, const T* au, const T* bu, const T* cu, int lo_u, int nu,
                          double c0, double c1, double c2, hipStream_t s);
// dst[j] = src[lo + j], j < n, for two fields.
template <typename T>
hipError_t launch_copy(T* dh, const T* sh, int lo_h, int nh, T* du, const T* su, int lo_u,
                       int nu, hipStream_t s);
// x[lo+j] = (j < nbase ? base[j] : x[lo+j]) + delta*acc[j], j < n, two fields.
template <typename T>
hipError_t launch_correct(T* xh, const T* baseh, const T* acch, int lo_h, int nh, int nbh,
                          T* xu, const T* baseu, const T* accu, int lo_u, int nu, int nbu,
                          double delta, hipStream_t s);
// Diagnostics partials per block (mass, energy, h_min, h_max, |u|max, nonfinite)
// then a single-block deterministic reduction into out[8] (doubles).
template <typename T>
hipError_t launch_diag(const DevMesh<T>& m, const T* h, const T* u, double g, double* part,
                       int nblk_cells, int nblk_edges, double* out, hipStream_t s);
int diag_blocks(int n);
hipError_t launch_fill_int(int* p, int v, hipStream_t s);

}  // namespace lts
