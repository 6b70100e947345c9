// HIP kernels for the TRiSK right-hand side and the LTS3 stage machinery on
// gfx950 (MI355X).  One thread per target element, 256-thread blocks (four
// wave64s), structure-of-arrays gathers.
//
// The right-hand side of eq:sweTimeStepping is evaluated in three kernels:
//   k_vertex: potential vorticity q_v = (f_v + zeta_v)/h_v at vertices, with
//             zeta_v the circulation over the dual triangle and h_v the
//             kite-weighted thickness (the vertex form of q = eta/h, App. A);
//   k_cell:   per cell i, the thickness fluxes F_e = [h]_{i->e} u_e of its
//             edges, the divergence H_i = -[div F]_i and kinetic energy K_i
//             (App. B), and for every edge b of the cell the cell's share of
//             the edge tendency,
//               Z_i(b) = (n_{b,i}/d_b) [ g(h_i+b_i) + K_i
//                        + sum_{a != b} (R_{ab} - 1/2) n_{a,i} l_a F_a (q~_b+q~_a)/2 ],
//             where R_{ab} sums the kite fractions A_{i,v}/A_i counter-clockwise
//             from edge a to edge b.  This is eq:weights with t_{b,v*} = -n_{b,i}
//             (v* is the vertex before b in counter-clockwise order), so the
//             sum over EE(e) in eq:discPV splits into one sum per cell of CE(e),
//             and the gradient of App. B splits the same way;
//   k_edge:   U_e = Z_{c0}(e) + Z_{c1}(e).
// The per-cell form needs no edgesOnEdge/weightsOnEdge tables: the weights are
// rebuilt in registers from the cell's kite fractions.
//
// Stage arithmetic (Algorithms 2.1 and 2.2) is fused into the cell and edge
// kernels as epilogue segments: an SSPRK stage update, or accumulation of the
// interface correction terms already weighted by theta.
#include <hip/hip_runtime.h>

#include "lts_internal.h"

namespace lts {

namespace {

constexpr int kBlock = 256;

template <typename T>
__device__ __forceinline__ void apply_seg(int j, T G, const Seg<T>& s, int* flag) {
    T v;
    if (s.mode == 1) {
        v = s.a_dt * G;
        if (s.xold) v = s.a_old * s.xold[j] + (s.xcur ? s.a_cur * s.xcur[j] : T(0)) + v;
        else if (s.xcur) v = s.a_cur * s.xcur[j] + v;
        s.out[j] = v;
    } else {
        const int k = j - s.lo;
        v = s.theta * G;
        if (!s.first) v = s.acc[k] + v;
        s.acc[k] = v;
    }
    if (!isfinite(v)) flag[0] = 1;
}

template <typename T>
__device__ __forceinline__ void epilogue(int j, T G, const Seg<T>& s0, const Seg<T>& s1,
                                         int* flag) {
    if (s0.mode && j >= s0.lo && j < s0.hi) apply_seg(j, G, s0, flag);
    else if (s1.mode && j >= s1.lo && j < s1.hi) apply_seg(j, G, s1, flag);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_vertex(DevMesh<T> m, const T* __restrict__ h,
                                                   const T* __restrict__ u, T* __restrict__ q,
                                                   int v_lo, int v_hi) {
    const int v = v_lo + blockIdx.x * kBlock + threadIdx.x;
    if (v >= v_hi) return;
    const int nV = m.nV;
    T circ = 0, hv = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int o = k * nV + v;
        circ += m.tdc[o] * u[m.eov[o]];
        hv += m.kite[o] * h[m.cov[o]];
    }
    q[v] = (m.fA[v] + circ) / hv;
}

template <typename T, int NE>
__global__ __launch_bounds__(kBlock) void k_cell(DevMesh<T> m, const T* __restrict__ h,
                                                 const T* __restrict__ u,
                                                 const T* __restrict__ q, T* __restrict__ zs,
                                                 int c_lo, int c_hi, T g, Seg<T> s0, Seg<T> s1,
                                                 int* flag) {
    const int i = c_lo + blockIdx.x * kBlock + threadIdx.x;
    if (i >= c_hi) return;
    const int nC = m.nC;
    const int n = m.nEoC[i];
    const T hi = h[i];
    T G[NE], qv[NE], S[NE + 1];
    int ed[NE];
    T div = 0, ksum = 0, run = 0, qlast = 0;
    S[0] = 0;
#pragma unroll
    for (int a = 0; a < NE; ++a) {
        G[a] = 0;
        qv[a] = 0;
        ed[a] = 0;
        S[a + 1] = run;
        if (a < n) {
            const size_t o = (size_t)a * nC + i;
            const int e = m.eoc[o];
            const T ue = u[e];
            const T F = T(0.5) * (hi + h[m.coc[o]]) * ue;
            G[a] = m.nl[o] * F;
            div += G[a];
            ksum += m.kc[o] * ue * ue;
            qv[a] = q[m.voc[o]];
            qlast = qv[a];
            run += m.kf[o];
            S[a + 1] = run;
            ed[a] = e;
        }
    }
    const T phi = g * (hi + m.bot[i]) + ksum;
    // q~ of edge a: mean of the vertices before (slot a-1) and after (slot a) it
    T qt[NE];
#pragma unroll
    for (int a = 0; a < NE; ++a) qt[a] = T(0.5) * ((a == 0 ? qlast : qv[a > 0 ? a - 1 : 0]) + qv[a]);
    const size_t nE = (size_t)m.nE;
#pragma unroll
    for (int b = 0; b < NE; ++b) {
        if (b < n) {
            T acc = 0;
#pragma unroll
            for (int a = 0; a < NE; ++a) {
                if (a < n && a != b) {
                    const T R = a < b ? S[b] - S[a] : (run - S[a]) + S[b];
                    acc += (R - T(0.5)) * G[a] * (T(0.5) * (qt[b] + qt[a]));
                }
            }
            const T ndb = m.nd[(size_t)b * nC + i];
            const int side = ndb > T(0) ? 0 : 1;
            zs[side * nE + ed[b]] = ndb * (phi + acc);
        }
    }
    const T H = -div / m.area[i];
    epilogue(i, H, s0, s1, flag);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_edge(const T* __restrict__ zs, int nE, int lo,
                                                 int hi, Seg<T> s0, Seg<T> s1, int* flag) {
    const int e = lo + blockIdx.x * kBlock + threadIdx.x;
    if (e >= hi) return;
    const T U = zs[e] + zs[(size_t)nE + e];
    epilogue(e, U, s0, s1, flag);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_predict(T* xh, const T* ah, const T* bh,
                                                    const T* ch, int lo_h, int nh, T* xu,
                                                    const T* au, const T* bu, const T* cu,
                                                    int lo_u, int nu, double c0, double c1,
                                                    double c2) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < nh) {
        xh[lo_h + j] = T(c0 * (double)ah[j] + c1 * (double)bh[j] + c2 * (double)ch[j]);
    } else if (j < nh + nu) {
        const int k = j - nh;
        xu[lo_u + k] = T(c0 * (double)au[k] + c1 * (double)bu[k] + c2 * (double)cu[k]);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(T* dh, const T* sh, int lo_h, int nh, T* du,
                                                 const T* su, int lo_u, int nu) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < nh) dh[j] = sh[lo_h + j];
    else if (j < nh + nu) du[j - nh] = su[lo_u + j - nh];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_correct(T* xh, const T* baseh, const T* acch,
                                                    int lo_h, int nh, int nbh, T* xu,
                                                    const T* baseu, const T* accu, int lo_u,
                                                    int nu, int nbu, T delta) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < nh) {
        const T b = j < nbh ? baseh[j] : xh[lo_h + j];
        xh[lo_h + j] = b + delta * acch[j];
    } else if (j < nh + nu) {
        const int k = j - nh;
        const T b = k < nbu ? baseu[k] : xu[lo_u + k];
        xu[lo_u + k] = b + delta * accu[k];
    }
}

// Diagnostics: block partials [mass, energy, -h_min, h_max, |u|max, nonfinite]
// as doubles, in a fixed tree order (deterministic).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag_part(DevMesh<T> m, const T* __restrict__ h,
                                                      const T* __restrict__ u, double g,
                                                      double* part, int nblk_cells) {
    __shared__ double red[6][kBlock];
    const int t = threadIdx.x;
    double v[6] = {0.0, 0.0, -1e300, -1e300, 0.0, 0.0};
    if ((int)blockIdx.x < nblk_cells) {
        const int i = blockIdx.x * kBlock + t;
        if (i < m.nC) {
            const double hi = (double)h[i];
            double K = 0.0;
            const int n = m.nEoC[i];
            for (int a = 0; a < n; ++a) {
                const size_t o = (size_t)a * m.nC + i;
                const double ue = (double)u[m.eoc[o]];
                K += (double)m.kc[o] * ue * ue;
            }
            const double A = (double)m.area[i];
            v[0] = A * hi;
            v[1] = A * (hi * K + g * (0.5 * hi * hi + hi * (double)m.bot[i]));
            v[2] = -hi;
            v[3] = hi;
            v[5] = isfinite(hi) ? 0.0 : 1.0;
        }
    } else {
        const int e = (blockIdx.x - nblk_cells) * kBlock + t;
        if (e < m.nE) {
            const double ue = (double)u[e];
            v[4] = fabs(ue);
            v[5] = isfinite(ue) ? 0.0 : 1.0;
        }
    }
    for (int k = 0; k < 6; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] += red[1][t + w];
            red[2][t] = fmax(red[2][t], red[2][t + w]);
            red[3][t] = fmax(red[3][t], red[3][t + w]);
            red[4][t] = fmax(red[4][t], red[4][t + w]);
            red[5][t] += red[5][t + w];
        }
        __syncthreads();
    }
    if (t < 6) part[(size_t)blockIdx.x * 8 + t] = red[t][0];
}

__global__ __launch_bounds__(kBlock) void k_diag_final(const double* part, int nblk,
                                                       double* out) {
    __shared__ double red[6][kBlock];
    const int t = threadIdx.x;
    double v[6] = {0.0, 0.0, -1e300, -1e300, 0.0, 0.0};
    for (int b = t; b < nblk; b += kBlock) {
        const double* p = part + (size_t)b * 8;
        v[0] += p[0];
        v[1] += p[1];
        v[2] = fmax(v[2], p[2]);
        v[3] = fmax(v[3], p[3]);
        v[4] = fmax(v[4], p[4]);
        v[5] += p[5];
    }
    for (int k = 0; k < 6; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] += red[1][t + w];
            red[2][t] = fmax(red[2][t], red[2][t + w]);
            red[3][t] = fmax(red[3][t], red[3][t + w]);
            red[4][t] = fmax(red[4][t], red[4][t + w]);
            red[5][t] += red[5][t + w];
        }
        __syncthreads();
    }
    if (t < 6) out[t] = t == 2 ? -red[2][0] : red[t][0];
}

__global__ void k_fill_int(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[threadIdx.x] = v;
}

inline unsigned nblocks(long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int diag_blocks(int n) { return (int)nblocks(n); }

template <typename T>
hipError_t launch_vertex(const DevMesh<T>& m, const T* h, const T* u, T* q, int v_lo, int v_hi,
                         hipStream_t s) {
    if (v_hi <= v_lo) return hipSuccess;
    hipLaunchKernelGGL(k_vertex<T>, dim3(nblocks(v_hi - v_lo)), dim3(kBlock), 0, s, m, h, u, q,
                       v_lo, v_hi);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cell(const DevMesh<T>& m, const T* h, const T* u, const T* q, T* zs, int c_lo,
                       int c_hi, T g, const Seg<T>& s0, const Seg<T>& s1, int* flag,
                       hipStream_t s) {
    if (c_hi <= c_lo) return hipSuccess;
    const dim3 grid(nblocks(c_hi - c_lo));
    if (m.maxE <= 6)
        hipLaunchKernelGGL((k_cell<T, 6>), grid, dim3(kBlock), 0, s, m, h, u, q, zs, c_lo, c_hi,
                           g, s0, s1, flag);
    else if (m.maxE <= 8)
        hipLaunchKernelGGL((k_cell<T, 8>), grid, dim3(kBlock), 0, s, m, h, u, q, zs, c_lo, c_hi,
                           g, s0, s1, flag);
    else
        hipLaunchKernelGGL((k_cell<T, LTS_MAX_EDGES>), grid, dim3(kBlock), 0, s, m, h, u, q, zs,
                           c_lo, c_hi, g, s0, s1, flag);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_edge(const T* zs, int nE, int lo, int hi, const Seg<T>& s0, const Seg<T>& s1,
                       int* flag, hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    hipLaunchKernelGGL(k_edge<T>, dim3(nblocks(hi - lo)), dim3(kBlock), 0, s, zs, nE, lo, hi, s0,
                       s1, flag);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_predict(T* xh, const T* ah, const T* bh, const T* ch, int lo_h, int nh, T* xu,
                          const T* au, const T* bu, const T* cu, int lo_u, int nu, double c0,
                          double c1, double c2, hipStream_t s) {
    if (nh + nu <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_predict<T>, dim3(nblocks((long)nh + nu)), dim3(kBlock), 0, s, xh, ah,
                       bh, ch, lo_h, nh, xu, au, bu, cu, lo_u, nu, c0, c1, c2);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(T* dh, const T* sh, int lo_h, int nh, T* du, const T* su, int lo_u, int nu,
                       hipStream_t s) {
    if (nh + nu <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy<T>, dim3(nblocks((long)nh + nu)), dim3(kBlock), 0, s, dh, sh, lo_h,
                       nh, du, su, lo_u, nu);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_correct(T* xh, const T* baseh, const T* acch, int lo_h, int nh, int nbh, T* xu,
                          const T* baseu, const T* accu, int lo_u, int nu, int nbu, double delta,
                          hipStream_t s) {
    if (nh + nu <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_correct<T>, dim3(nblocks((long)nh + nu)), dim3(kBlock), 0, s, xh, baseh,
                       acch, lo_h, nh, nbh, xu, baseu, accu, lo_u, nu, nbu, (T)delta);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const DevMesh<T>& m, const T* h, const T* u, double g, double* part,
                       int nblk_cells, int nblk_edges, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_part<T>, dim3(nblk_cells + nblk_edges), dim3(kBlock), 0, s, m, h,
                       u, g, part, nblk_cells);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kBlock), 0, s, part, nblk_cells + nblk_edges,
                       out);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

#define LTS_INSTANTIATE(T)                                                                      \
    template hipError_t launch_vertex<T>(const DevMesh<T>&, const T*, const T*, T*, int, int,    \
                                         hipStream_t);                                          \
    template hipError_t launch_cell<T>(const DevMesh<T>&, const T*, const T*, const T*, T*, int, \
                                       int, T, const Seg<T>&, const Seg<T>&, int*, hipStream_t); \
    template hipError_t launch_edge<T>(const T*, int, int, int, const Seg<T>&, const Seg<T>&,    \
                                       int*, hipStream_t);                                      \
    template hipError_t launch_predict<T>(T*, const T*, const T*, const T*, int, int, T*,        \
                                          const T*, const T*, const T*, int, int, double,       \
                                          double, double, hipStream_t);                         \
    template hipError_t launch_copy<T>(T*, const T*, int, int, T*, const T*, int, int,           \
                                       hipStream_t);                                            \
    template hipError_t launch_correct<T>(T*, const T*, const T*, int, int, int, T*, const T*,   \
                                          const T*, int, int, int, double, hipStream_t);        \
    template hipError_t launch_diag<T>(const DevMesh<T>&, const T*, const T*, double, double*,   \
                                       int, int, double*, hipStream_t);

LTS_INSTANTIATE(double)
LTS_INSTANTIATE(float)

}  // namespace lts
