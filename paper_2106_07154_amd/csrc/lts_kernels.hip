// HIP kernels for the TRiSK right-hand side and the LTS3 stage machinery on
// gfx950 (MI355X).  256-thread blocks (four wave64s), structure-of-arrays
// gathers; one thread per vertex or edge, one lane per edge slot of a cell
// (8 or 16 lanes per cell); the layered forms further down map threads to
// (element, layer).
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
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "lts_internal.h"

namespace lts {

namespace {

constexpr int kBlock = 256;
// Smallest pass (cells) whose FP64 single-range cell kernel takes the shared
// per-cell loads (cell_share_loads).
constexpr int kShareMinCells = 1 << 17;

// Blocks are dispatched round-robin over the 8 XCDs; remap so every XCD works
// on one contiguous chunk of the range and neighbouring blocks share its L2.
__device__ __forceinline__ int xcd_block() {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Epilogue of element j, split in two: epi_loads issues the loads that
// depend only on j (old and current stage values, the accumulator), so their
// latency overlaps the tendency's own gathers; epilogue then combines them
// with the tendency G.  The loads are unconditional and branch-free: an
// operand the owning segment does not have is read from dflt[0] (any valid
// element) and never used.
template <typename T>
struct EpiIn {
    T xo, xc, ac;
    int seg;  // 0 or 1: the segment that owns j; -1: none
};

template <typename T>
__device__ __forceinline__ EpiIn<T> epi_loads(int j, const Seg<T>& s0, const Seg<T>& s1,
                                              const T* dflt) {
    const bool in0 = s0.mode && j >= s0.lo && j < s0.hi;
    const bool in1 = !in0 && s1.mode && j >= s1.lo && j < s1.hi;
    const T* po = in0 && s0.mode == 1 && s0.xold   ? s0.xold + j
                  : in1 && s1.mode == 1 && s1.xold ? s1.xold + j
                                                   : dflt;
    const T* pc = in0 && s0.mode == 1 && s0.xcur   ? s0.xcur + j
                  : in1 && s1.mode == 1 && s1.xcur ? s1.xcur + j
                                                   : dflt;
    // the accumulator is read unless the segment starts it (first) or, in
    // update mode, has none
    const bool a0 = in0 && !s0.first && (s0.mode != 1 || s0.acc);
    const bool a1 = in1 && !s1.first && (s1.mode != 1 || s1.acc);
    const T* pa = a0 ? s0.acc + (j - s0.lo) : a1 ? s1.acc + (j - s1.lo) : dflt;
    return EpiIn<T>{*po, *pc, *pa, in0 ? 0 : in1 ? 1 : -1};
}

// PRE: the operands come from epi_loads (r); otherwise from memory here,
// inside the branches that need them.
template <bool PRE, typename T>
__device__ __forceinline__ void apply_seg(int j, T G, const Seg<T>& s, const EpiIn<T>& r,
                                          int* flag) {
    T v;
    if (s.mode == 1) {
        v = s.a_dt * G;
        if (s.convex) {
            const T xo = PRE ? r.xo : s.xold[j];
            v = xo + s.a_cur * ((PRE ? r.xc : s.xcur[j]) - xo) + v;
        } else if (s.xold) {
            const T xo = PRE ? r.xo : s.xold[j];
            v = s.a_old * xo + (s.xcur ? s.a_cur * (PRE ? r.xc : s.xcur[j]) : T(0)) + v;
        } else if (s.xcur) {
            v = s.a_cur * (PRE ? r.xc : s.xcur[j]) + v;
        }
        s.out[j] = v;
        if (j >= s.mlo && j < s.mhi) {
            if (s.mnew) s.mnew[j - s.mlo] = v;
            if (s.mcur) s.mcur[j - s.mlo] = PRE ? r.xc : s.xcur[j];
        }
        if (s.acc) {
            const int k = j - s.lo;
            const T a = s.theta * G;
            s.acc[k] = s.first ? a : (PRE ? r.ac : s.acc[k]) + a;
        }
    } else {
        const int k = j - s.lo;
        v = s.theta * G;
        if (!s.first) v = (PRE ? r.ac : s.acc[k]) + v;
        s.acc[k] = v;
    }
    if (!isfinite(v)) flag[0] = 1;
}

// Epilogue with the operands of epi_loads.
template <typename T>
__device__ __forceinline__ void epilogue(int j, T G, const Seg<T>& s0, const Seg<T>& s1,
                                         const EpiIn<T>& r, int* flag) {
    if (r.seg == 0) apply_seg<true>(j, G, s0, r, flag);
    else if (r.seg == 1) apply_seg<true>(j, G, s1, r, flag);
}

// Epilogue that loads its operands itself.
template <typename T>
__device__ __forceinline__ void epilogue(int j, T G, const Seg<T>& s0, const Seg<T>& s1,
                                         int* flag) {
    const EpiIn<T> none{};
    if (s0.mode && j >= s0.lo && j < s0.hi) apply_seg<false>(j, G, s0, none, flag);
    else if (s1.mode && j >= s1.lo && j < s1.hi) apply_seg<false>(j, G, s1, none, flag);
}

// Potential vorticity at vertex v: (f_v A_v + circulation) / (A_v h_v) with
// h_v the kite-weighted thickness.
template <typename T>
__device__ __forceinline__ T vertex_q(const DevMesh<T>& m, const T* __restrict__ h,
                                      const T* __restrict__ u, int v, bool hr) {
    const int nV = m.nV;
    T circ = 0, hv = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int o = k * nV + v;
        const int c = m.cov[o];
        circ += m.tdc[o] * u[m.eov[o]];
        hv += m.kite[o] * (hr ? m.href[c] + h[c] : h[c]);
    }
    return (m.fA[v] + circ) / hv;
}

// Optional operand (the reference thickness href): K = 1 present, K = 0
// absent, both known at compile time so the kernel has no branch on it;
// K = -1 tests the pointer at run time.
template <int K>
__device__ __forceinline__ bool present(const void* p) {
    return K < 0 ? p != nullptr : K != 0;
}

template <typename T, int HR>
__device__ __forceinline__ void vertex_body(const DevMesh<T>& m, const T* __restrict__ h,
                                            const T* __restrict__ u, T* __restrict__ q, int v) {
    q[v] = vertex_q(m, h, u, v, present<HR>(m.href));
}

template <typename T, int HR>
__global__ __launch_bounds__(kBlock) void k_vertex(DevMesh<T> m, const T* __restrict__ h,
                                                   const T* __restrict__ u, T* __restrict__ q,
                                                   int v_lo, int v_hi) {
    const int v = v_lo + xcd_block() * kBlock + threadIdx.x;
    if (v < v_hi) vertex_body<T, HR>(m, h, u, q, v);
}

// Cell kernel: one lane per edge slot, G lanes per cell (G = 8 or 16), so a
// wave64 covers 64/G cells and every slot's gathers are issued by its own
// lane.  Slot tables are compact (the cell's n slots from cso[i].x); lanes
// n..G-1 are padding: they re-read slot n-1 (valid indices, so lane G-1
// holds the PV of the vertex before slot 0) with zero coefficients.
//
// The PV part of Z_i(b) is rewritten with prefix sums: with S_a the kite
// fractions summed counter-clockwise before slot a and S_n their total (both
// mesh constants, tabulated at upload),
//   R_ab - 1/2 = (S_b - 1/2) - S_a + S_n [a > b],
// so for any slot quantity X
//   sum_{a != b} (R_ab - 1/2) X_a = (S_b - 1/2)(sum X - X_b)
//                                   - (sum S X - S_b X_b) + S_n sum_{a > b} X_a,
// and the PV sum is (1/2) q~_b P_b(G) + (1/2) P_b(G q~).  Group sums, scans
// and the slot rotation move data between the G lanes of a cell with DPP
// row operations (a cell's lanes lie inside one 16-lane row), not through LDS.
//
// DPP controls (GFX9 encoding): quad_perm [1,0,3,2] = 0xB1 and [2,3,0,1] =
// 0x4E (xor 1, xor 2), row_shl:n = 0x100 + n, row_shr:n = 0x110 + n,
// row_mirror = 0x140, row_half_mirror = 0x141.  Lanes whose source falls
// outside the row read 0 (bound_ctrl).
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

// Sum over the G lanes of the group, the same value in every lane: xor-1 and
// xor-2 pairs give quad sums, the half-row mirror pairs the two quads of an
// 8-lane half, the row mirror the two halves of a row.
template <typename T, int G>
__device__ __forceinline__ T gsum(T x) {
    x += dpp<0xB1>(x);
    x += dpp<0x4E>(x);
    x += dpp<0x141>(x);
    if (G == 16) x += dpp<0x140>(x);
    return x;
}
// Inclusive scan over the group (lane = index within the group).
template <typename T, int G>
__device__ __forceinline__ T gscan(T x, int lane) {
    T y = dpp<0x111>(x);
    x += lane >= 1 ? y : T(0);
    y = dpp<0x112>(x);
    x += lane >= 2 ? y : T(0);
    y = dpp<0x114>(x);
    x += lane >= 4 ? y : T(0);
    if (G == 16) {
        y = dpp<0x118>(x);
        x += lane >= 8 ? y : T(0);
    }
    return x;
}
// Value of the previous lane of the group, cyclically (lane 0 reads lane G-1).
template <typename T, int G>
__device__ __forceinline__ T gprev(T x, int lane) {
    const T a = dpp<0x111>(x);                      // row_shr:1
    const T b = dpp<G == 16 ? 0x10F : 0x107>(x);    // row_shl:(G-1)
    return lane == 0 ? b : a;
}

// Optimisation barrier: x must be available here and may have changed.
template <typename T>
__device__ __forceinline__ void hold(T& x) {
    asm volatile("" : "+v"(x));
}

// The per-cell operands of a wave's 8 cells (h_i, S_n, beta_i, 1/A_i, the
// three epilogue operands and href_i when present, else the FP64 kernel's
// slot record cso[i]) in one vector load:
// lane k reads array k / 8 of the wave's cell k % 8 into lds[threadIdx.x].
// Every lane of a cell needs these values, and read per lane they took
// seven or eight load instructions of the 8-lane layout; the address and data
// units' work grows with the instructions and the bytes each lane requests,
// not with the distinct lines, so one load plus an exchange through LDS
// relieves the units that bound the cell kernel.
template <typename T, int HR>
__device__ __forceinline__ void cell_share_loads(const DevMesh<T>& m, const T* __restrict__ h,
                                                 int c_lo, int c_hi, int t, const Seg<T>& s0,
                                                 const Seg<T>& s1, T* __restrict__ lds) {
    const int k = t & 63;
    const int a = k >> 3;
    int j = c_lo + (t & ~63) / 8 + (k & 7);
    j = j < c_hi ? j : c_hi - 1;  // dead cells shadow a valid one, as in cell_body
    // the epilogue operands' addresses, as epi_loads takes them
    const bool in0 = s0.mode && j >= s0.lo && j < s0.hi;
    const bool in1 = !in0 && s1.mode && j >= s1.lo && j < s1.hi;
    const T* po = in0 && s0.mode == 1 && s0.xold   ? s0.xold + j
                  : in1 && s1.mode == 1 && s1.xold ? s1.xold + j
                                                   : h;
    const T* pc = in0 && s0.mode == 1 && s0.xcur   ? s0.xcur + j
                  : in1 && s1.mode == 1 && s1.xcur ? s1.xcur + j
                                                   : h;
    const bool a0 = in0 && !s0.first && (s0.mode != 1 || s0.acc);
    const bool a1 = in1 && !s1.first && (s1.mode != 1 || s1.acc);
    const T* pa = a0 ? s0.acc + (j - s0.lo) : a1 ? s1.acc + (j - s1.lo) : h;
    const T* p = a == 0   ? h + j
                 : a == 1 ? m.sn + j
                 : a == 2 ? m.beta + j
                 : a == 3 ? m.rarea + j
                 : a == 4 ? po
                 : a == 5 ? pc
                 : a == 6 ? pa
                 : present<HR>(m.href) ? m.href + j
                 // without href the last 8 lanes bring the slot record {first, n}
                 // (8 bytes, the width of a double)
                 : sizeof(T) == sizeof(int2) ? reinterpret_cast<const T*>(m.cso + j)
                                             : h;
    lds[threadIdx.x] = *p;
    // the wave's own LDS writes are visible to its later reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One cell lane between its loads and its arithmetic.
template <typename T>
struct CellLane {
    size_t o;  // slot-table entry
    int i, lane, n, e;
    bool live;
    T nl, kc, sb, sn, nd, hi, hn, hc, ue, bi, ra;
    EpiIn<T> ep;
};

// Loads of lane `lane` of cell i (a valid cell; live: the lane's own cell is
// in the pass range).  HR: presence of m.href (see present).  PRE: the
// epilogue's operands are loaded here too (epi_loads), not after the
// tendency.  SH (8-lane single-range kernel): the per-cell operands come from
// lds as cell_share_loads left them (array a of the cell at a * 8 + the
// cell's place in its wave), the slot record too when it is 8 bytes wide and
// no href is present.
template <typename T, int G, int HR, bool PRE, bool SH = false>
__device__ __forceinline__ CellLane<T> cell_loads(const DevMesh<T>& m, const T* __restrict__ h,
                                                  const T* __restrict__ u, int i, int lane,
                                                  bool live, const Seg<T>& s0, const Seg<T>& s1,
                                                  const T* __restrict__ lds = nullptr) {
    CellLane<T> c;
    const T* __restrict__ href = m.href;
    const bool hr = present<HR>(href);
    int2 so;
    if (SH && sizeof(T) == sizeof(int2) && !present<HR>(href)) {
        const T v = lds[(threadIdx.x & ~63) + ((threadIdx.x & 63) >> 3) + 56];
        __builtin_memcpy(&so, &v, sizeof(so));
    } else {
        so = m.cso[i];
    }
    c.n = so.y;
    // lanes past the cell's last slot re-read that slot, coefficients zeroed
    c.o = (size_t)so.x + min(lane, so.y - 1);
    c.i = i;
    c.lane = lane;
    c.live = live && so.y <= G;  // wider cells: the appended 16-lane blocks
    c.e = m.eoc[c.o];
    const int nb = m.coc[c.o];
    c.nl = lane < so.y ? m.nl[c.o] : T(0);
    c.kc = lane < so.y ? m.kc[c.o] : T(0);
    c.sb = m.sb[c.o];
    c.nd = m.nd[c.o];
    const int wb = (threadIdx.x & ~63) + ((threadIdx.x & 63) >> 3);
    c.sn = SH ? lds[wb + 8] : m.sn[i];
    c.hc = SH ? lds[wb] : h[i];
    c.hi = hr ? (SH ? lds[wb + 56] : href[i]) + c.hc : c.hc;
    c.hn = hr ? href[nb] + h[nb] : h[nb];
    c.ue = u[c.e];
    // every lane of the cell reads its epilogue operands (one address per
    // cell); lane 0 applies the epilogue
    c.ep = EpiIn<T>{};
    if (PRE && !SH) c.ep = epi_loads(i, s0, s1, h);
    if (SH) {
        const bool in0 = s0.mode && i >= s0.lo && i < s0.hi;
        const bool in1 = !in0 && s1.mode && i >= s1.lo && i < s1.hi;
        c.ep = EpiIn<T>{lds[wb + 32], lds[wb + 40], lds[wb + 48], in0 ? 0 : in1 ? 1 : -1};
    }
    c.bi = SH ? lds[wb + 16] : m.beta[i];
    c.ra = SH ? lds[wb + 24] : m.rarea[i];
    return c;
}

// Arithmetic of a cell lane given the PV qv of the vertex after its slot.
template <typename T, int G, bool PRE>
__device__ __forceinline__ void cell_math(const DevMesh<T>& m, CellLane<T> c, T qv,
                                          T* __restrict__ zs, T g, const Seg<T>& s0,
                                          const Seg<T>& s1, int* flag) {
    const int lane = c.lane;
    const T Ga = c.nl * (T(0.5) * (c.hi + c.hn) * c.ue);
    const T K = gsum<T, G>(c.kc * c.ue * c.ue);
    const T Sb = c.sb, Sn = c.sn;  // S_b and S_n from the slot tables
    const T qt = T(0.5) * (gprev<T, G>(qv, lane) + qv);
    const T X1 = Ga, X2 = Ga * qt;
    const T c1 = gscan<T, G>(X1, lane), c2 = gscan<T, G>(X2, lane);
    const T t1 = gsum<T, G>(X1), t2 = gsum<T, G>(X2);  // sums; t1 = sum G
    const T p1 = gsum<T, G>(Sb * X1), p2 = gsum<T, G>(Sb * X2);
    // (S_b - 1/2)(t - X_b) - (p - S_b X_b) + S_n (t - c_b), collected:
    const T w = Sb + Sn - T(0.5);
    const T P1 = w * t1 + T(0.5) * X1 - p1 - Sn * c1;
    const T P2 = w * t2 + T(0.5) * X2 - p2 - Sn * c2;
    if (PRE) {
        // Uses outside the conditional stores below keep these loads with
        // the others at the top; sunk into the stores, each would add a
        // dependent memory round trip.
        hold(c.bi);
        hold(c.ra);
        hold(c.nd);
        hold(c.ep.xo);
        hold(c.ep.xc);
        hold(c.ep.ac);
    }
    const T phi = g * (c.hc + c.bi) + K;
    if (c.live && lane < c.n)
        zs[(c.nd > T(0) ? 0 : (size_t)m.nE) + c.e] =
            c.nd * (phi + T(0.5) * qt * P1 + T(0.5) * P2);
    if (c.live && lane == 0) {
        if (PRE) epilogue(c.i, -t1 * c.ra, s0, s1, c.ep, flag);
        else epilogue(c.i, -t1 * c.ra, s0, s1, flag);
    }
}

// Cell lanes reading q from the vertex pass.  t: thread index within the
// cell range (G lanes per cell, groups aligned).
template <typename T, int G, int HR, bool PRE>
__device__ __forceinline__ void cell_body(const DevMesh<T>& m, const T* __restrict__ h,
                                          const T* __restrict__ u, const T* __restrict__ q,
                                          T* __restrict__ zs, int t, int c_lo, int c_hi, T g,
                                          const Seg<T>& s0, const Seg<T>& s1, int* flag) {
    const int ic = c_lo + t / G;
    const bool live = ic < c_hi;
    const int i = live ? ic : c_hi - 1;  // dead lanes shadow a valid cell
    const CellLane<T> c = cell_loads<T, G, HR, PRE>(m, h, u, i, t & (G - 1), live, s0, s1);
    cell_math<T, G, PRE>(m, c, q[m.voc[c.o]], zs, g, s0, s1, flag);
}

// The cell kernel: 8 lanes per cell over [c_lo, c_hi), blocks spread over
// the 8 XCDs (xcd_block).  SH: the per-cell operands through
// cell_share_loads (launches of many cells; the scalar registers it needs
// would cost a wave per SIMD without the waves-per-EU bound).
template <typename T, int HR, bool SH>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_cell(
    DevMesh<T> m, const T* __restrict__ h, const T* __restrict__ u, const T* __restrict__ q,
    T* __restrict__ zs, int c_lo, int c_hi, T g, Seg<T> s0, Seg<T> s1, int* flag) {
    const int t = xcd_block() * kBlock + threadIdx.x;
    if (!SH) {
        cell_body<T, 8, HR, true>(m, h, u, q, zs, t, c_lo, c_hi, g, s0, s1, flag);
        return;
    }
    __shared__ T lds[kBlock];
    cell_share_loads<T, HR>(m, h, c_lo, c_hi, t, s0, s1, lds);
    const int ic = c_lo + t / 8;
    const bool live = ic < c_hi;
    const int i = live ? ic : c_hi - 1;  // dead lanes shadow a valid cell
    const CellLane<T> c = cell_loads<T, 8, HR, true, true>(m, h, u, i, t & 7, live, s0, s1, lds);
    cell_math<T, 8, true>(m, c, q[m.voc[c.o]], zs, g, s0, s1, flag);
}

// Meshes with cells of more than 8 edges: those cells are not handled by
// their 8-lane groups (their lanes are dead, see cell_loads); nbw blocks
// appended to the launch take them from the mesh's list of such cells
// (entries [w_lo, w_hi)), 16 lanes each, so the other cells keep 8 lanes and
// no extra launch is needed.  The appended branch needs more scalar
// registers (106 against 74, which would cost a wave per SIMD); the
// waves-per-EU bound keeps the kernel at 8 waves per SIMD (a few scalar
// values then live in vector-register lanes).
template <typename T, int HR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_cell_wide(
    DevMesh<T> m, const T* __restrict__ h, const T* __restrict__ u, const T* __restrict__ q,
    T* __restrict__ zs, int c_lo, int c_hi, T g, Seg<T> s0, Seg<T> s1, int* flag, int nbc,
    int w_lo, int w_hi) {
    const int b = blockIdx.x;
    if (b >= nbc) {
        const int t = (b - nbc) * kBlock + threadIdx.x;
        const int p = w_lo + t / 16;
        const bool live = p < w_hi;
        const int i = m.wide[live ? p : w_hi - 1];
        const CellLane<T> c = cell_loads<T, 16, HR, true>(m, h, u, i, t & 15, live, s0, s1);
        cell_math<T, 16, true>(m, c, q[m.voc[c.o]], zs, g, s0, s1, flag);
        return;
    }
    // blocks spread over the 8 XCDs as in xcd_block, over the nbc cell blocks
    const int x = b & 7, k = b >> 3, qq = nbc >> 3, r = nbc & 7;
    const int lb = x < r ? x * (qq + 1) + k : r * (qq + 1) + (x - r) * qq + k;
    cell_body<T, 8, HR, true>(m, h, u, q, zs, lb * kBlock + threadIdx.x, c_lo, c_hi, g, s0, s1,
                              flag);
}

template <typename T>
__device__ void run_aux(const Aux<T>& x, int j) {
    if (x.kind == 1) {
        if (j < x.nh)
            x.xh[x.lo_h + j] = T(x.c0 * (double)x.ah[j] + x.c1 * (double)x.bh[j] +
                                 x.c2 * (double)x.ch[j]);
        else if (j < x.nh + x.nu) {
            const int k = j - x.nh;
            x.xu[x.lo_u + k] = T(x.c0 * (double)x.au[k] + x.c1 * (double)x.bu[k] +
                                 x.c2 * (double)x.cu[k]);
        }
    } else if (x.kind == 2) {
        const T d = (T)x.c0;
        if (j < x.nh) {
            const T base = j < x.nbh ? x.ah[j] : x.xh[x.lo_h + j];
            x.xh[x.lo_h + j] = base + d * x.bh[j];
        } else if (j < x.nh + x.nu) {
            const int k = j - x.nh;
            const T base = k < x.nbu ? x.au[k] : x.xu[x.lo_u + k];
            x.xu[x.lo_u + k] = base + d * x.bu[k];
        }
    }
}

template <typename T>
__device__ __forceinline__ void edge_body(const T* __restrict__ zs, int nE, int e,
                                          const Seg<T>& s0, const Seg<T>& s1, int* flag) {
    epilogue(e, zs[e] + zs[(size_t)nE + e], s0, s1, flag);
}

// Edge tendency U_e = Z_{c0}(e) + Z_{c1}(e) with its epilogue; blocks past the
// edge range run the appended element-wise jobs (nba blocks of aux, then
// aux2; the two touch disjoint elements).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_edge(const T* __restrict__ zs, int nE, int lo,
                                                 int hi, int nbe, Seg<T> s0, Seg<T> s1,
                                                 Aux<T> aux, int nba, Aux<T> aux2, int* flag) {
    if ((int)blockIdx.x >= nbe) {
        const int b = blockIdx.x - nbe;
        if (b < nba) run_aux(aux, b * kBlock + threadIdx.x);
        else run_aux(aux2, (b - nba) * kBlock + threadIdx.x);
        return;
    }
    const int b = blockIdx.x, x = b & 7, k = b >> 3, qq = nbe >> 3, r = nbe & 7;
    const int lb = x < r ? x * (qq + 1) + k : r * (qq + 1) + (x - r) * qq + k;
    const int e = lo + lb * kBlock + threadIdx.x;
    if (e < hi) edge_body(zs, nE, e, s0, s1, flag);
}

// ---------------------------------------------------------------------------
// Batched (ensemble) kernels.  A launch carries a work list: item k covers
// virtual blocks [first_k, first_k + nblk_k + nblk_aux_k + nblk_aux2_k) of one
// member's range.  The grid is persistent (fixed size, chosen by the
// autotuner); each block finds its item by binary search.
//
// Virtual blocks [0, nvb) are split into one contiguous chunk per XCD, sized
// by the XCD's share of the grid (blocks are dispatched round-robin over the
// 8 XCDs), and the XCD's blocks stride over its chunk, so neighbouring cells'
// gathers meet in one L2 (with a plain grid stride every line shared by
// adjacent virtual blocks is fetched into several L2s).  Every virtual block
// is visited once whatever the placement.
struct VbRange {
    int vb, end, step;
};
__device__ __forceinline__ VbRange xcd_range(int nvb) {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
    const int before = x * q + min(x, r);  // blocks on the XCDs before x
    const int mine = q + (x < r ? 1 : 0);  // blocks on XCD x (k < mine)
    const int lo = (int)((long long)nvb * before / nb);
    const int hi = (int)((long long)nvb * (before + mine) / nb);
    return VbRange{lo + k, hi, mine};
}

template <typename T>
__device__ __forceinline__ int find_item(const Item<T>* items, int nitems, int vb) {
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first <= vb) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ __launch_bounds__(512) void kb_vertex(const Item<T>* __restrict__ items, int nitems,
                                                 int nvb) {
    for (VbRange r = xcd_range(nvb); r.vb < r.end; r.vb += r.step) {
        const int vb = r.vb;
        const Item<T>& w = items[find_item(items, nitems, vb)];
        const int v = w.lo + (vb - w.first) * (int)blockDim.x + threadIdx.x;
        if (v < w.hi) vertex_body<T, perturbation_form<T>()>(w.m, w.h, w.u, w.q, v);
    }
}

// Without the up-front loads (PRE = false): with them the persistent batched
// kernel ran 5-10% slower over a 64-member ensemble, while the single-range
// kernel gains up to 10% from them.
template <typename T, int G>
__global__ __launch_bounds__(512) void kb_cell(const Item<T>* __restrict__ items, int nitems,
                                               int nvb) {
    for (VbRange r = xcd_range(nvb); r.vb < r.end; r.vb += r.step) {
        const int vb = r.vb;
        const Item<T>& w = items[find_item(items, nitems, vb)];
        cell_body<T, G, perturbation_form<T>(), false>(w.m, w.h, w.u, w.q, w.zs,
                               (vb - w.first) * (int)blockDim.x + threadIdx.x, w.lo, w.hi, w.g,
                               w.s0, w.s1, w.flag);
    }
}

template <typename T>
__global__ __launch_bounds__(512) void kb_edge(const Item<T>* __restrict__ items, int nitems,
                                               int nvb) {
    for (VbRange r = xcd_range(nvb); r.vb < r.end; r.vb += r.step) {
        const int vb = r.vb;
        const Item<T>& w = items[find_item(items, nitems, vb)];
        const int k = vb - w.first;
        if (k < w.nblk) {
            const int e = w.lo + k * (int)blockDim.x + threadIdx.x;
            if (e < w.hi) edge_body(w.zs, w.m.nE, e, w.s0, w.s1, w.flag);
        } else if (k < w.nblk + w.nblk_aux) {
            run_aux(w.aux, (k - w.nblk) * (int)blockDim.x + threadIdx.x);
        } else {
            run_aux(w.aux2, (k - w.nblk - w.nblk_aux) * (int)blockDim.x + threadIdx.x);
        }
    }
}

// ---------------------------------------------------------------------------
// Fused ensemble step: one persistent cooperative launch runs every phase of
// every member's coarse step, the kernel classes of a phase (vertex, cell,
// edge) separated by grid-wide barriers.  Work lists as for the batched
// kernels above, one per (phase, class), members of every size and lane
// count together.

// Grid barrier.  The 8 XCDs each have their own L2, not coherent with the
// others, so a block's writes become visible to other XCDs only after an L2
// write-back and reads see other XCDs' writes only after an L2 invalidate
// (the agent-scope release and acquire).  Done by every block, the write-back
// serialises on each XCD's L2 and dominates the barrier.  Here one block per
// XCD writes back for all: every block waits for its own stores to reach the
// L2 (s_waitcnt) and arrives on its XCD's counter; the XCD's last arrival
// (its leader) writes the L2 back, arrives on the top counter, waits for the
// generation to advance, invalidates and raises the XCD's flag; the other
// blocks wait for the flag and invalidate (their CU's L1 needs it; the
// invalidate cannot be narrowed to the L1).  Which XCD a block runs on is read
// from the hardware (XCC_ID), and the blocks per XCD are counted at kernel
// start, so no placement is assumed.  Every wait is bounded: after `limit`
// polls the block records the failure in the error word and the barrier
// reports false; every later barrier of the launch then returns false at
// once, so all blocks leave the kernel.
__device__ __forceinline__ unsigned* bar_word(FusedBarrier* bar, int line) {
    return bar->w + line * kBarLine;
}
__device__ __forceinline__ unsigned ld_agent(unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned add_agent(unsigned* p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The value v has arrived (its load or atomic has been performed) before any
// later memory operation issues: a wait on v plus a compiler barrier.  Used
// where two relaxed operations on different words must take effect in order.
__device__ __forceinline__ void arrived(unsigned v) { asm volatile("" ::"v"(v) : "memory"); }
// Poll *p until it differs from old; false (and the error word set) after
// `limit` polls.
__device__ __forceinline__ bool bar_wait(unsigned* p, unsigned old, int limit, unsigned* err) {
    for (int n = 0; ld_agent(p) == old; ++n) {
        if (n >= limit) {
            __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

struct BarCtx {
    int xcd;        // this block's XCD
    unsigned gsz;   // blocks of the launch on that XCD
    unsigned nxcd;  // XCDs holding blocks of the launch
};

// Kernel start: count the blocks per XCD (one barrier on atomics only; no
// data is exchanged through it).
__device__ bool bar_setup(FusedBarrier* bar, int limit, BarCtx& bc) {
    __shared__ int ok;
    __shared__ unsigned sg, sn;
    __shared__ int sx;
    if (threadIdx.x == 0) {
        unsigned* err = bar_word(bar, 2);
        const int x = __builtin_amdgcn_s_getreg(20 | (3 << 11)) & (kBarXcds - 1);  // XCC_ID[3:0]
        int good = ld_agent(err) == 0;
        if (good) {
            arrived(add_agent(bar_word(bar, 3 + x), 1u));
            const unsigned g = ld_agent(bar_word(bar, 1));
            arrived(g);
            if (add_agent(bar_word(bar, 0), 1u) + 1u == gridDim.x) {
                st_agent(bar_word(bar, 0), 0u);
                add_agent(bar_word(bar, 1), 1u);
            } else {
                good = bar_wait(bar_word(bar, 1), g, limit, err);
            }
        }
        unsigned n = 0;
        for (int i = 0; i < kBarXcds; ++i) n += ld_agent(bar_word(bar, 3 + i)) ? 1u : 0u;
        sg = ld_agent(bar_word(bar, 3 + x));
        sn = n;
        sx = x;
        ok = good;
    }
    __syncthreads();
    bc.xcd = sx;
    bc.gsz = sg;
    bc.nxcd = sn;
    return ok != 0;
}

__device__ __forceinline__ bool grid_barrier(FusedBarrier* bar, const BarCtx& bc, int limit) {
    __shared__ int ok;
    __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have reached the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* err = bar_word(bar, 2);
        int good = ld_agent(err) == 0;
        if (good) {
            unsigned* cnt = bar_word(bar, 3 + kBarXcds + bc.xcd);
            unsigned* flag = bar_word(bar, 3 + 2 * kBarXcds + bc.xcd);
            const unsigned f = ld_agent(flag);
            arrived(f);  // read before arriving: the flag cannot move until then
            if (add_agent(cnt, 1u) + 1u == bc.gsz) {
                // leader: the XCD's writes to memory, then the grid-wide arrival
                st_agent(cnt, 0u);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                const unsigned g = ld_agent(bar_word(bar, 1));
                arrived(g);
                if (add_agent(bar_word(bar, 0), 1u) + 1u == bc.nxcd) {
                    st_agent(bar_word(bar, 0), 0u);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    add_agent(bar_word(bar, 1), 1u);
                } else {
                    good = bar_wait(bar_word(bar, 1), g, limit, err);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the XCD's L2 and this L1
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // invalidate done before the flag
                st_agent(flag, f + 1u);
            } else {
                good = bar_wait(flag, f, limit, err);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // this CU's L1 (and the L2)
            }
        }
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

template <typename T>
__global__ __launch_bounds__(256) void kf_step(const Item<T>* __restrict__ items,
                                               const FusedPhase* __restrict__ phases, int nphase,
                                               FusedBarrier* bar, int limit) {
    const unsigned nb = gridDim.x;
    if (nphase <= 0) return;
    BarCtx bc;
    if (!bar_setup(bar, limit, bc)) return;
    for (int t = 0; t < nphase; ++t) {
        for (int k = 0; k < KC_N; ++k) {
            const FusedPhase P = phases[t * KC_N + k];
            const Item<T>* it = items + P.off;
            for (int vb = blockIdx.x; vb < P.nvb; vb += (int)nb) {
                const Item<T>& w = it[find_item(it, P.nitems, vb)];
                const int j = vb - w.first;
                const int lt = j * (int)blockDim.x + threadIdx.x;
                if (k == KC_VERTEX) {
                    const int v = w.lo + lt;
                    if (v < w.hi) vertex_body<T, perturbation_form<T>()>(w.m, w.h, w.u, w.q, v);
                } else if (k == KC_CELL) {
                    if (padded_slots(w.m.maxE) == 8)
                        cell_body<T, 8, perturbation_form<T>(), false>(w.m, w.h, w.u, w.q, w.zs, lt,
                                                                       w.lo, w.hi, w.g, w.s0, w.s1,
                                                                       w.flag);
                    else
                        cell_body<T, 16, perturbation_form<T>(), false>(w.m, w.h, w.u, w.q, w.zs,
                                                                        lt, w.lo, w.hi, w.g, w.s0,
                                                                        w.s1, w.flag);
                } else if (j < w.nblk) {
                    const int e = w.lo + lt;
                    if (e < w.hi) edge_body(w.zs, w.m.nE, e, w.s0, w.s1, w.flag);
                } else if (j < w.nblk + w.nblk_aux) {
                    run_aux(w.aux, (j - w.nblk) * (int)blockDim.x + threadIdx.x);
                } else {
                    run_aux(w.aux2, (j - w.nblk - w.nblk_aux) * (int)blockDim.x + threadIdx.x);
                }
            }
            if (!grid_barrier(bar, bc, limit)) return;
        }
    }
    // every block has passed the last barrier, so the counts are no longer
    // read: clear them for the next launch
    if (blockIdx.x == 0 && threadIdx.x < kBarXcds) st_agent(bar_word(bar, 3 + threadIdx.x), 0u);
}

// Diagnostics: block partials [mass, energy, -h_min, h_max, |u|max, nonfinite]
// as doubles, in a fixed tree order (deterministic).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag_part(DevMesh<T> m, const T* __restrict__ h,
                                                      const T* __restrict__ u, double g,
                                                      double* part, int nblk_cells, int L) {
    __shared__ double red[6][kBlock];
    const int t = threadIdx.x;
    double v[6] = {0.0, 0.0, -1e300, -1e300, 0.0, 0.0};
    if ((int)blockIdx.x < nblk_cells) {
        const long il = (long)blockIdx.x * kBlock + t;
        const int i = (int)(il / L), l = (int)(il % L);
        if (i < m.nC) {
            const double hi = m.href ? (double)m.href[i] + (double)h[il] : (double)h[il];
            double K = 0.0;
            const int2 so = m.cso[i];
            for (int a = 0; a < so.y; ++a) {
                const size_t o = (size_t)so.x + a;
                const double ue = (double)u[(size_t)m.eoc[o] * L + l];
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
        const long e = (long)(blockIdx.x - nblk_cells) * kBlock + t;
        if (e < (long)m.nE * L) {
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

// ---------------------------------------------------------------------------
// Layered kernels: L independent layers on one mesh (the vertical dimension of
// an ocean-like workload).  Every per-element array is [element][layer],
// layer fastest, so consecutive threads are consecutive layers of the same
// element: the mesh tables are read once per element and broadcast to its
// layers, and the state accesses of a wave are contiguous.

// apply_seg for element j, layer l: the same arithmetic on the flat index
// j L + l (segment ranges stay in elements).
template <typename T>
__device__ __forceinline__ void apply_seg_l(int j, int l, int L, T G, const Seg<T>& s,
                                            int* flag) {
    const size_t f = (size_t)j * L + l;
    T v;
    if (s.mode == 1) {
        v = s.a_dt * G;
        if (s.convex) v = s.xold[f] + s.a_cur * (s.xcur[f] - s.xold[f]) + v;
        else if (s.xold) v = s.a_old * s.xold[f] + (s.xcur ? s.a_cur * s.xcur[f] : T(0)) + v;
        else if (s.xcur) v = s.a_cur * s.xcur[f] + v;
        s.out[f] = v;
        if (j >= s.mlo && j < s.mhi) {
            const size_t fm = (size_t)(j - s.mlo) * L + l;
            if (s.mnew) s.mnew[fm] = v;
            if (s.mcur) s.mcur[fm] = s.xcur[f];
        }
        if (s.acc) {
            const size_t k = (size_t)(j - s.lo) * L + l;
            const T a = s.theta * G;
            s.acc[k] = s.first ? a : s.acc[k] + a;
        }
    } else {
        const size_t k = (size_t)(j - s.lo) * L + l;
        v = s.theta * G;
        if (!s.first) v = s.acc[k] + v;
        s.acc[k] = v;
    }
    if (!isfinite(v)) flag[0] = 1;
}

template <typename T>
__device__ __forceinline__ void epilogue_l(int j, int l, int L, T G, const Seg<T>& s0,
                                           const Seg<T>& s1, int* flag) {
    if (s0.mode && j >= s0.lo && j < s0.hi) apply_seg_l(j, l, L, G, s0, flag);
    else if (s1.mode && j >= s1.lo && j < s1.hi) apply_seg_l(j, l, L, G, s1, flag);
}

// Thread-to-(element, layer) maps of the layered vertex and cell kernels.
// W = false: one thread per pair, consecutive threads along the layers.
// W = true: each wave takes one element and a chunk of 64 consecutive layers;
// the element index is wave-uniform, so its mesh-table entries come in
// through scalar loads and the vector memory instructions are the contiguous
// state accesses only.  Lanes past the last layer compute on the last layer
// and store nothing.
template <bool W>
__device__ __forceinline__ void layer_slot(int n_lo, int L, int& k, int& l, bool& act) {
    const long t = (long)xcd_block() * kBlock + threadIdx.x;
    if (!W) {
        k = n_lo + (int)(t / L);
        l = (int)(t % L);
        act = true;
        return;
    }
    const long wv = t >> 6;
    const int nch = (L + 63) >> 6;
    k = __builtin_amdgcn_readfirstlane(n_lo + (int)(wv / nch));
    const int l0 = (int)(wv % nch) * 64 + (int)(threadIdx.x & 63);
    act = l0 < L;
    l = act ? l0 : L - 1;
}

template <typename T, bool W, int HR>
__global__ __launch_bounds__(kBlock) void k_vertex_l(DevMesh<T> m, const T* __restrict__ h,
                                                     const T* __restrict__ u,
                                                     T* __restrict__ q, int v_lo, int v_hi,
                                                     int L) {
    int v, l;
    bool act;
    layer_slot<W>(v_lo, L, v, l, act);
    if (v >= v_hi) return;
    const int nV = m.nV;
    const int32_t* __restrict__ cov = m.cov;
    const int32_t* __restrict__ eov = m.eov;
    const T* __restrict__ tdc = m.tdc;
    const T* __restrict__ kite = m.kite;
    const T* __restrict__ href = m.href;
    T circ = 0, hv = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int o = k * nV + v;
        const int c = cov[o];
        const T hc = h[(size_t)c * L + l];
        circ += tdc[o] * u[(size_t)eov[o] * L + l];
        hv += kite[o] * (present<HR>(href) ? href[c] + hc : hc);
    }
    const T qv = (m.fA[v] + circ) / hv;
    if (act) q[(size_t)v * L + l] = qv;
}

// The cell's slots in a loop, with the same O(n) prefix-sum form of the PV
// share as the single-layer cell kernel.  PAD: the padded slot tables of a
// layered context (addresses from i alone); otherwise the compact ones
// (the surrogate's interface pass on a single-layer context).
template <typename T, int G, bool W, int HR, bool PAD>
__global__ __launch_bounds__(kBlock) void k_cell_l(DevMesh<T> m, const T* __restrict__ h,
                                                   const T* __restrict__ u,
                                                   const T* __restrict__ q,
                                                   T* __restrict__ zs, int c_lo, int c_hi,
                                                   int L, T g, Seg<T> s0, Seg<T> s1,
                                                   int* flag) {
    int i, l;
    bool act;
    layer_slot<W>(c_lo, L, i, l, act);
    if (i >= c_hi) return;
    const int32_t* __restrict__ eoc = PAD ? m.peoc : m.eoc;
    const int32_t* __restrict__ coc = PAD ? m.pcoc : m.coc;
    const int32_t* __restrict__ voc = PAD ? m.pvoc : m.voc;
    const T* __restrict__ nl = PAD ? m.pnl : m.nl;
    const T* __restrict__ nd = PAD ? m.pnd : m.nd;
    const T* __restrict__ kc = PAD ? m.pkc : m.kc;
    const T* __restrict__ kf = PAD ? m.pkf : m.kf;
    const T* __restrict__ href = m.href;
    const int2 so = PAD ? int2{0, m.nEoC[i]} : m.cso[i];
    const int n = so.y;
    const size_t base = PAD ? (size_t)i * G : (size_t)so.x;
    const size_t il = (size_t)i * L + l;
    const bool hr = present<HR>(href);
    const T hi = hr ? href[i] + h[il] : h[il];
    // PV of the last slot's vertex: the predecessor of slot 0
    T qprev = q[(size_t)voc[base + n - 1] * L + l];
    // Every slot up to G, padding included: padding slots re-read the last
    // slot with its coefficients zeroed, so they add exact zeros to the sums
    // and only their stores are skipped.  Without a branch per slot all the
    // slots' loads can be in flight together.
    T X1[G], X2[G], qtA[G], kfA[G];
    T K = 0, S = 0, t1 = 0, t2 = 0, p1 = 0, p2 = 0;
#pragma unroll
    for (int a = 0; a < G; ++a) {
        const bool real = PAD || a < n;  // padded tables hold zero coefficients
        const size_t o = base + (PAD ? a : min(a, n - 1));
        const int e = eoc[o], nb = coc[o];
        const T ue = u[(size_t)e * L + l];
        const T hn0 = h[(size_t)nb * L + l];
        const T hn = hr ? href[nb] + hn0 : hn0;
        const T qa = q[(size_t)voc[o] * L + l];
        const T qt = T(0.5) * (qprev + qa);
        qprev = qa;
        X1[a] = real ? nl[o] * (T(0.5) * (hi + hn) * ue) : T(0);
        X2[a] = X1[a] * qt;
        qtA[a] = qt;
        K += real ? kc[o] * ue * ue : T(0);
        kfA[a] = real ? kf[o] : T(0);
        const T Sb = S;
        S += kfA[a];
        t1 += X1[a];
        t2 += X2[a];
        p1 += Sb * X1[a];
        p2 += Sb * X2[a];
    }
    const T phi = g * (h[il] + m.beta[i]) + K;
    T c1 = 0, c2 = 0, Sr = 0;
#pragma unroll
    for (int a = 0; a < G; ++a) {
        const size_t o = base + (PAD ? a : min(a, n - 1));
        const T Sb = Sr;
        Sr += kfA[a];
        c1 += X1[a];
        c2 += X2[a];
        const T P1 = (Sb - T(0.5)) * (t1 - X1[a]) - (p1 - Sb * X1[a]) + S * (t1 - c1);
        const T P2 = (Sb - T(0.5)) * (t2 - X2[a]) - (p2 - Sb * X2[a]) + S * (t2 - c2);
        const T ndo = nd[o];
        if (act && a < n)
            zs[(ndo > T(0) ? 0 : (size_t)m.nE * L) + (size_t)eoc[o] * L + l] =
                ndo * (phi + T(0.5) * qtA[a] * P1 + T(0.5) * P2);
    }
    if (act) epilogue_l(i, l, L, -t1 / m.area[i], s0, s1, flag);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_edge_l(const T* __restrict__ zs, int nE, int lo,
                                                   int hi, int L, int nbe, Seg<T> s0, Seg<T> s1,
                                                   Aux<T> aux, int nba, Aux<T> aux2, int* flag) {
    if ((int)blockIdx.x >= nbe) {
        const int b = blockIdx.x - nbe;
        if (b < nba) run_aux(aux, b * kBlock + threadIdx.x);
        else run_aux(aux2, (b - nba) * kBlock + threadIdx.x);
        return;
    }
    const int b = blockIdx.x, x = b & 7, k = b >> 3, qq = nbe >> 3, r = nbe & 7;
    const int lb = x < r ? x * (qq + 1) + k : r * (qq + 1) + (x - r) * qq + k;
    const long t = (long)lb * kBlock + threadIdx.x;
    const int e = lo + (int)(t / L), l = (int)(t % L);
    if (e >= hi) return;
    const size_t f = (size_t)e * L + l;
    epilogue_l(e, l, L, zs[f] + zs[(size_t)nE * L + f], s0, s1, flag);
}

inline unsigned nblocks(long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int diag_blocks(int n) { return (int)nblocks(n); }

// Plain launch, or an event-stamped launch in timing mode.
template <typename K, typename... Args>
hipError_t launch(K kernel, dim3 grid, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                  Args... args) {
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, s, ev0, ev1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, s, args...);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_vertex(const DevMesh<T>& m, const T* h, const T* u, T* q, int v_lo, int v_hi,
                         hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (v_hi <= v_lo) return hipSuccess;
    const dim3 grid(nblocks(v_hi - v_lo));
    if (m.href) return launch(k_vertex<T, 1>, grid, s, ev0, ev1, m, h, u, q, v_lo, v_hi);
    return launch(k_vertex<T, 0>, grid, s, ev0, ev1, m, h, u, q, v_lo, v_hi);
}

template <typename T>
hipError_t launch_cell(const DevMesh<T>& m, const T* h, const T* u, const T* q, T* zs, int c_lo,
                       int c_hi, int w_lo, int w_hi, T g, const Seg<T>& s0, const Seg<T>& s1,
                       int* flag, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (c_hi <= c_lo) return hipSuccess;
    const int nbc = (int)nblocks((long)(c_hi - c_lo) * 8);
    const int nbw = w_hi > w_lo ? (int)nblocks((long)(w_hi - w_lo) * 16) : 0;
    if (nbw) {
        const dim3 grid(nbc + nbw);
        if (m.href)
            return launch(k_cell_wide<T, 1>, grid, s, ev0, ev1, m, h, u, q, zs, c_lo, c_hi, g, s0,
                          s1, flag, nbc, w_lo, w_hi);
        return launch(k_cell_wide<T, 0>, grid, s, ev0, ev1, m, h, u, q, zs, c_lo, c_hi, g, s0, s1,
                      flag, nbc, w_lo, w_hi);
    }
    const dim3 grid(nbc);
    // Launches of fewer cells fill the GPU's wave slots at most about twice
    // and are latency bound: there the LDS exchange of the shared per-cell
    // loads lengthens each wave's chain of dependent memory operations
    // (measured 2% slower on a 200k-cell mesh with 62k-cell fine passes).
    // FP32 keeps the per-lane loads: a 4-byte load costs the address and
    // data units half as much, less than the exchange's added work (measured
    // 8% slower on the 1.6M-cell sphere with the shared loads).
    const bool sh = sizeof(T) == 8 && c_hi - c_lo >= kShareMinCells;
    if (m.href)
        return sh ? launch(k_cell<T, 1, true>, grid, s, ev0, ev1, m, h, u, q, zs, c_lo, c_hi, g,
                           s0, s1, flag)
                  : launch(k_cell<T, 1, false>, grid, s, ev0, ev1, m, h, u, q, zs, c_lo, c_hi, g,
                           s0, s1, flag);
    return sh ? launch(k_cell<T, 0, true>, grid, s, ev0, ev1, m, h, u, q, zs, c_lo, c_hi, g, s0,
                       s1, flag)
              : launch(k_cell<T, 0, false>, grid, s, ev0, ev1, m, h, u, q, zs, c_lo, c_hi, g, s0,
                       s1, flag);
}

template <typename T>
hipError_t launch_edge(const T* zs, int nE, int lo, int hi, const Seg<T>& s0, const Seg<T>& s1,
                       const Aux<T>& aux, int* flag, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1, const Aux<T>& aux2) {
    const int nbe = hi > lo ? (int)nblocks(hi - lo) : 0;
    const int nba = aux.kind ? (int)nblocks((long)aux.nh + aux.nu) : 0;
    const int nba2 = aux2.kind ? (int)nblocks((long)aux2.nh + aux2.nu) : 0;
    if (nbe + nba + nba2 == 0) return hipSuccess;
    return launch(k_edge<T>, dim3(nbe + nba + nba2), s, ev0, ev1, zs, nE, lo, hi, nbe, s0, s1, aux,
                  nba, aux2, flag);
}

// The wave-per-element map pays once few lanes of a wave go idle: measured
// on a 200k-cell mesh it is 8% slower per step than one thread per pair at
// 48 layers and 8% faster at 64 (24% at 128); the crossover is near 56.
#ifndef LTS_WAVE_LAYERS_MIN
#define LTS_WAVE_LAYERS_MIN 56
#endif
inline bool wave_layers(int L) { return L >= LTS_WAVE_LAYERS_MIN; }
inline long layer_threads(int n, int L) {
    return wave_layers(L) ? (long)n * ((L + 63) / 64) * 64 : (long)n * L;
}

template <typename T>
hipError_t launch_vertex_l(const DevMesh<T>& m, const T* h, const T* u, T* q, int v_lo, int v_hi,
                           int L, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (v_hi <= v_lo) return hipSuccess;
    const dim3 grid(nblocks(layer_threads(v_hi - v_lo, L)));
#define LTS_VERTEX_L(W, HR) \
    launch(k_vertex_l<T, W, HR>, grid, s, ev0, ev1, m, h, u, q, v_lo, v_hi, L)
    if (wave_layers(L)) return m.href ? LTS_VERTEX_L(true, 1) : LTS_VERTEX_L(true, 0);
    return m.href ? LTS_VERTEX_L(false, 1) : LTS_VERTEX_L(false, 0);
#undef LTS_VERTEX_L
}

template <typename T>
hipError_t launch_cell_l(const DevMesh<T>& m, const T* h, const T* u, const T* q, T* zs,
                         int c_lo, int c_hi, int L, T g, const Seg<T>& s0, const Seg<T>& s1,
                         int* flag, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (c_hi <= c_lo) return hipSuccess;
    const dim3 grid(nblocks(layer_threads(c_hi - c_lo, L)));
    const bool w = wave_layers(L), g8 = padded_slots(m.maxE) == 8;
    const bool pad = m.peoc != nullptr && m.pG == padded_slots(m.maxE);
#define LTS_CELL_L(GG, W, HR, P)                                                                 \
    launch(k_cell_l<T, GG, W, HR, P>, grid, s, ev0, ev1, m, h, u, q, zs, c_lo, c_hi, L, g, s0,   \
           s1, flag)
#define LTS_CELL_LP(GG, W, HR) (pad ? LTS_CELL_L(GG, W, HR, true) : LTS_CELL_L(GG, W, HR, false))
    if (m.href) {
        if (w) return g8 ? LTS_CELL_LP(8, true, 1) : LTS_CELL_LP(16, true, 1);
        return g8 ? LTS_CELL_LP(8, false, 1) : LTS_CELL_LP(16, false, 1);
    }
    if (w) return g8 ? LTS_CELL_LP(8, true, 0) : LTS_CELL_LP(16, true, 0);
    return g8 ? LTS_CELL_LP(8, false, 0) : LTS_CELL_LP(16, false, 0);
#undef LTS_CELL_LP
#undef LTS_CELL_L
}

template <typename T>
hipError_t launch_edge_l(const T* zs, int nE, int lo, int hi, int L, const Seg<T>& s0,
                         const Seg<T>& s1, const Aux<T>& aux, int* flag, hipStream_t s,
                         hipEvent_t ev0, hipEvent_t ev1, const Aux<T>& aux2) {
    const int nbe = hi > lo ? (int)nblocks((long)(hi - lo) * L) : 0;
    const int nba = aux.kind ? (int)nblocks((long)aux.nh + aux.nu) : 0;
    const int nba2 = aux2.kind ? (int)nblocks((long)aux2.nh + aux2.nu) : 0;
    if (nbe + nba + nba2 == 0) return hipSuccess;
    return launch(k_edge_l<T>, dim3(nbe + nba + nba2), s, ev0, ev1, zs, nE, lo, hi, L, nbe, s0, s1,
                  aux, nba, aux2, flag);
}

template <typename T>
hipError_t launch_batch(int kclass, const Item<T>* items, int nitems, int nvb, int block, int grid,
                        int G, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (nvb <= 0) return hipSuccess;
    const dim3 gr(grid), bl(block);
    if (ev0 || ev1) {
        if (kclass == KC_VERTEX)
            hipExtLaunchKernelGGL(kb_vertex<T>, gr, bl, 0, s, ev0, ev1, 0, items, nitems, nvb);
        else if (kclass == KC_CELL && G == 8)
            hipExtLaunchKernelGGL(kb_cell<T, 8>, gr, bl, 0, s, ev0, ev1, 0, items, nitems, nvb);
        else if (kclass == KC_CELL)
            hipExtLaunchKernelGGL(kb_cell<T, 16>, gr, bl, 0, s, ev0, ev1, 0, items, nitems, nvb);
        else
            hipExtLaunchKernelGGL(kb_edge<T>, gr, bl, 0, s, ev0, ev1, 0, items, nitems, nvb);
    } else {
        if (kclass == KC_VERTEX)
            hipLaunchKernelGGL(kb_vertex<T>, gr, bl, 0, s, items, nitems, nvb);
        else if (kclass == KC_CELL && G == 8)
            hipLaunchKernelGGL((kb_cell<T, 8>), gr, bl, 0, s, items, nitems, nvb);
        else if (kclass == KC_CELL)
            hipLaunchKernelGGL((kb_cell<T, 16>), gr, bl, 0, s, items, nitems, nvb);
        else
            hipLaunchKernelGGL(kb_edge<T>, gr, bl, 0, s, items, nitems, nvb);
    }
    return hipGetLastError();
}

template <typename T>
int fused_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kf_step<T>),
                                                     256, 0) != hipSuccess)
        return 0;
    return nb;
}

template <typename T>
hipError_t launch_fused(const Item<T>* items, const FusedPhase* phases, int nphase,
                        FusedBarrier* bar, int limit, int grid, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1) {
    void* args[] = {(void*)&items, (void*)&phases, (void*)&nphase, (void*)&bar, (void*)&limit};
    hipError_t e = hipSuccess;
    if (ev0) e = hipEventRecord(ev0, s);
    if (e == hipSuccess)
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kf_step<T>), dim3(grid),
                                       dim3(256), args, 0, s);
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
    return e;
}

template <typename T>
hipError_t launch_diag(const DevMesh<T>& m, const T* h, const T* u, double g, double* part,
                       int nblk_cells, int nblk_edges, double* out, hipStream_t s, int L) {
    hipLaunchKernelGGL(k_diag_part<T>, dim3(nblk_cells + nblk_edges), dim3(kBlock), 0, s, m, h,
                       u, g, part, nblk_cells, L);
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
                                         hipStream_t, hipEvent_t, hipEvent_t);                  \
    template hipError_t launch_cell<T>(const DevMesh<T>&, const T*, const T*, const T*, T*, int, \
                                       int, int, int, T, const Seg<T>&, const Seg<T>&, int*,     \
                                       hipStream_t, hipEvent_t, hipEvent_t);                    \
    template hipError_t launch_edge<T>(const T*, int, int, int, const Seg<T>&, const Seg<T>&,    \
                                       const Aux<T>&, int*, hipStream_t, hipEvent_t, hipEvent_t, \
                                       const Aux<T>&);                                          \
    template hipError_t launch_batch<T>(int, const Item<T>*, int, int, int, int, int,           \
                                        hipStream_t, hipEvent_t, hipEvent_t);                  \
    template int fused_blocks_per_cu<T>();                                                      \
    template hipError_t launch_fused<T>(const Item<T>*, const FusedPhase*, int, FusedBarrier*,  \
                                        int, int, hipStream_t, hipEvent_t, hipEvent_t);         \
    template hipError_t launch_diag<T>(const DevMesh<T>&, const T*, const T*, double, double*,   \
                                       int, int, double*, hipStream_t, int);                     \
    template hipError_t launch_vertex_l<T>(const DevMesh<T>&, const T*, const T*, T*, int, int,  \
                                           int, hipStream_t, hipEvent_t, hipEvent_t);            \
    template hipError_t launch_cell_l<T>(const DevMesh<T>&, const T*, const T*, const T*, T*,    \
                                         int, int, int, T, const Seg<T>&, const Seg<T>&, int*,   \
                                         hipStream_t, hipEvent_t, hipEvent_t);                   \
    template hipError_t launch_edge_l<T>(const T*, int, int, int, int, const Seg<T>&,            \
                                         const Seg<T>&, const Aux<T>&, int*, hipStream_t,        \
                                         hipEvent_t, hipEvent_t, const Aux<T>&);

LTS_INSTANTIATE(double)
LTS_INSTANTIATE(float)

}  // namespace lts
