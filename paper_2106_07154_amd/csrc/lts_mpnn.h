// Kernels of the message-passing surrogate (lts_mpnn.hip).  Not public ABI.
//
// Matrices are row-major.  BF16 values are stored as uint16_t bit patterns.
// Every launcher enqueues on stream s and returns nothing; launch errors are
// picked up by the caller's next checked HIP call.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lts_internal.h"

namespace lts {
namespace nn {

constexpr int kFeat = 16;    // padded input width (first GEMM K)
constexpr int kHid = 64;     // hidden width
constexpr int kRawFeat = 9;  // used input columns: 5 physical + 4 region one-hot
constexpr int kReduceRows = 512;  // rows per block of the reductions over nodes

// Y = act(A W + bias): A [N x K] BF16 stride lda (K % 16 == 0, K <= 128),
// W [K x 64] BF16; out_bf (stride ldo, relu if relu != 0) and/or out_f
// ([N x 64] FP32, no activation).  Alignment: A, W, bias and out_f 16 bytes
// (lda a multiple of 8), out_bf 8 bytes (ldo a multiple of 4).
void gemm(const uint16_t* A, int lda, int N, int K, const uint16_t* W, const float* bias,
          int relu, uint16_t* out_bf, int ldo, float* out_f, hipStream_t s);

// out[K x 64] = A^T D (A [N x K] BF16 stride lda, D [N x 64] BF16), through
// per-block partials part[gemm_tn_parts(N, rpb)][K x 64].
int gemm_tn_parts(int N, int rows_per_block);
void gemm_tn(const uint16_t* A, int lda, int N, int K, const uint16_t* D, int rows_per_block,
             float* part, float* out, hipStream_t s);

// Wt = the two 64 x 64 blocks (W[0:64,:])^T and (W[64:128,:])^T of W [128 x 64].
void transpose_halves(const uint16_t* W, uint16_t* Wt, hipStream_t s);

// HC[i][64:128] = mean over in-set neighbours of HC[j][0:64] (HC stride 128).
// adj [N][aw]: neighbour node or -1.
void aggregate(uint16_t* HC, int N, const int32_t* adj, int aw, const float* inv_deg,
               hipStream_t s);
// dH[j] += sum over neighbours i of dHn[i] * inv_deg[i] (FP32 [N x 64]).
void aggregate_back(float* dH, const float* dHn, int N, const int32_t* adj, int aw,
                    const float* inv_deg, hipStream_t s);
// dZ = BF16(dH * (H > 0)); H stride ldh.
void relu_back(const float* dH, const uint16_t* H, int ldh, int N, uint16_t* dZ, hipStream_t s);
// out[64] = column sums of D [N x 64] BF16.
int colsum_parts(int N, int rows_per_block);
void colsum(const uint16_t* D, int N, int rows_per_block, float* part, float* out, hipStream_t s);

// Heads on the fine cells (nodes 0..nF-1) and fine edges (ec0 -> ec1):
//   out_h = H.wh + bh,   out_u = (H[ec1] - H[ec0]).wu.
// With targets (th, tu scaled by tsh, tsu): loss = mean(d_h^2) + mean(d_u^2),
// gh, gu = d loss / d out; loss written to *loss.
int heads_parts(int nF, int nFe);
void heads(const uint16_t* H, int ldh, int nF, int nFe, const int32_t* ec0, const int32_t* ec1,
           const float* wh, const float* bh, const float* wu, const float* th, const float* tu,
           float tsh, float tsu, float* out_h, float* out_u, float* gh, float* gu, float* part,
           float* loss, hipStream_t s);
// dH (overwritten) and the head gradients [dwh(64) | dwu(64) | dbh] from gh, gu.
// node_edges [N][aw]: (fine edge << 1 | node is ec1) or -1.
int heads_back_parts(int N);
void heads_back(const uint16_t* H, int ldh, int N, int nF, const int32_t* node_edges, int aw,
                const float* wh, const float* wu, const float* gh, const float* gu, float* dH,
                float* part, float* grads_head, hipStream_t s);

// Adam on FP32 master parameters p (n) with gradient g; parameters with
// bf_map[i] >= 0 also refresh their BF16 working copy wbf[bf_map[i]].
void adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
          float eps, int step, const int32_t* bf_map, uint16_t* wbf, hipStream_t s);
void to_bf16(const float* x, int n, uint16_t* y, hipStream_t s);

// Normalised BF16 features X [N x 16] from raw FP32 features [N x 16]:
// column f < 5: (raw - mu[f]) * inv_sd[f]; columns 5..8 copied; the rest 0.
void norm_features(const float* raw, int N, const float* mu, const float* inv_sd, uint16_t* X,
                   hipStream_t s);
// Column mean / inverse standard deviation of the 5 physical columns over
// S samples of raw features [S][N][16], and inverse RMS of the targets
// [S][nT] (nT = nF + nFe: first nF thickness, then nFe velocity).  FP64 sums.
void feature_stats(const float* raw, long rows, const float* tgt, int S, int nF, int nFe,
                   double* part, float* norm_out, hipStream_t s);

// ------------------------------------------------------------- state side
// Graph tables of the node set (device cells 0..N-1) and fine edges 0..nFe-1.
template <typename T>
void build_graph(const DevMesh<T>& m, int N, int nFe, int32_t* adj, float* inv_deg,
                 int32_t* node_edges, int32_t* ec0, int32_t* ec1, hipStream_t s);
// Raw features of state (h, u) on the nodes: [N][16] FP32, columns
//   0 surface h + b (minus a per-context constant), 1 b, 2 div u, 3 cell
//   relative vorticity (kite-weighted vertex vorticity), 4 K, 5..8 region
//   one-hot (F interior, underlined F, I1, I2); cb = cell class starts.
template <typename T>
void features(const DevMesh<T>& m, const T* h, const T* u, int N, int cb1, int cb3, int cb4,
              float* raw, hipStream_t s);
// Training targets: the part of the step's increment beyond a forward-Euler
// step, tgt[0:nF] = h1 - h0 - dt R0h, tgt[nF:nF+nFe] = u1 - u0 - dt R0u (FP32).
template <typename T>
void increments(const T* h0, const T* u0, const T* h1, const T* u1, const T* R0h, const T* R0u,
                double dt, int nF, int nFe, float* tgt, hipStream_t s);
// xh[i] = h[i] + dt R0h[i] + scale[0] out_h[i] (i < nF),
// xu[e] = u[e] + dt R0u[e] + scale[1] out_u[e] (e < nFe).
template <typename T>
void apply_increments(const T* h, const T* u, const T* R0h, const T* R0u, double dt,
                      const float* out_h, const float* out_u, const float* scale, int nF, int nFe,
                      T* xh, T* xu, hipStream_t s);
// Sources of one field for the interface accumulation's stage states: x0, x1,
// x2 the coarse stages X0, X1, X2 (full arrays, device order), pred the
// surrogate's state at t + dt on the fine elements, i0, i1, i2 the
// interface-1 copies of X0, X1, X2.
template <typename T>
struct IfaceSrc {
    const T *x0, *x1, *x2, *pred, *i0, *i1, *i2;
};
// Stage states [element][L] (L = 3M, layer 3k + s) on the listed elements
// (cells cidx with class ccls, then edges): class 0 fine, linear in time
// between x0 and pred (coef[4 l] = tau); class 1 interface 1, the prediction
// coef[4 l + 1..3] . (i0, i1, i2); class 2 interface 2 or coarse, x_s.
template <typename T>
void iface_fill(const int32_t* cidx, const int8_t* ccls, int ncl, const int32_t* eidx,
                const int8_t* ecls, int nel, int L, const double* coef, const IfaceSrc<T>& h,
                const IfaceSrc<T>& u, int cb3, int eb2, T* hS, T* uS, hipStream_t s);
// x[lo + j] = x0[lo + j] + delta sum_k (acc[j][3k]/6 + acc[j][3k+1]/6 +
// 2 acc[j][3k+2]/3) on the nIc interface cells (lo = cb3) and nIe interface
// edges (lo = eb2), FP64 sums.
template <typename T>
void iface_combine(const T* acch, const T* accu, int nIc, int nIe, int L, double delta, int cb3,
                   int eb2, const T* x0h, const T* x0u, T* xh, T* xu, hipStream_t s);
// Remove the mass change sum_i A_i (h1_i - h0_i) from the fine cells
// 0..nF-1 of h1 as a uniform thickness shift (change * inv_area_f);
// part[mass_fix_parts(nC)], shift[1] device scratch.
int mass_fix_parts(int nC);
template <typename T>
void mass_fix(const T* area, const T* h0, T* h1, int nC, int nF, double inv_area_f, double* part,
              double* shift, hipStream_t s);
// Trapezoid residual sums on the fine region, FP64:
//   out[0] = sum_i ((x1-x0)/dt - (R0+R1)/2)^2 over cells, out[1] = sum R0^2,
//   out[2] = sum R1^2, out[3..5] the same over edges.
template <typename T>
void gate_sums(const T* h0, const T* u0, const T* h1, const T* u1, const T* R0h, const T* R0u,
               const T* R1h, const T* R1u, int nF, int nFe, double dt, double* part, double* out,
               hipStream_t s);

}  // namespace nn
}  // namespace lts
