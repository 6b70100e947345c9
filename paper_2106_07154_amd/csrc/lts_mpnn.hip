// Message-passing surrogate kernels (gfx950): BF16 weights and activations,
// FP32 accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16 for the
// layer products, v_mfma_f32_16x16x16_bf16 where a lane holds 4 values).
//
// Network over the cells of the fine and interface regions (the nodes),
// neighbours = cells sharing an edge within that set:
//   H0 = relu(X W0 + b0)                               X: [N x 16] features
//   Hl = relu([H_{l-1} | mean_nbr H_{l-1}] Wl + bl)   l = 1..3, Wl: [128 x 64]
//   dh_i = H3[i] . wh + bh                             (fine cells)
//   du_e = (H3[c1] - H3[c0]) . wu                      (fine edges; odd in the
//                                                       edge orientation)
// Training: mean squared error against the increments of the solver's own
// coarse step, manual backward, Adam on FP32 master weights with BF16 working
// copies.
//
// MFMA tile layout used by every GEMM (16x16x16, one wave): lane l holds
//   A[m = l % 16][k = 4 (l / 16) + j], B[k = 4 (l / 16) + j][n = l % 16],
//   D[m = 4 (l / 16) + j][n = l % 16], j = 0..3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lts_mpnn.h"

namespace lts {
namespace nn {

namespace {

typedef short sh4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u)  // inf / nan: keep, quiet the nan
        return (uint16_t)((u >> 16) | ((u & 0x007FFFFFu) ? 0x40u : 0u));
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // round to nearest even
}

__device__ __forceinline__ f4 mfma(sh4 a, sh4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// gfx950's double-depth form: 8 BF16 per lane and operand, 32 products per
// output element in one instruction.  Lane group g = l / 16 supplies k-slots
// 8 g .. 8 g + 7 of the instruction in both operands, so any assignment of
// reduction indices to those slots that is the same in A and B gives the
// same sum.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf8 as_bf8(uint4 v) {
    bf8 r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}
__device__ __forceinline__ f4 mfma32(uint4 a, uint4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a), as_bf8(b), c, 0, 0, 0);
}

inline unsigned nblk(long n, int per) { return (unsigned)((n + per - 1) / per); }

// Y[N x 64] = act(A[N x K] W[K x 64] + bias).  4 waves per block, each on
// kGemmTiles tiles of 16 rows (the W staging below is shared by them).
// Each tile is computed as the transposed product D^T = W^T A^T (16 columns
// x 16 rows per MFMA, 4 column tiles), so a lane ends with 4 consecutive
// columns of one row and stores them with one 16-byte (FP32) or 8-byte
// (BF16) store.  The reduction index is permuted, identically in both
// operands (the sum is unchanged): at k-step t the lanes of group
// g = l / 16 take k = g K/4 + 4 t + j, so a lane's A operands over all steps
// are one contiguous run of K/4 elements of its row and its W operands one
// contiguous run of a row of W^T, staged in LDS.  A lane loads its whole A
// run (16-byte pieces, 8-byte for K = 16) before the W staging, so the two
// memory round trips overlap.
constexpr int kGemmTiles = 2;                   // row tiles per wave
constexpr int kGemmRows = 4 * 16 * kGemmTiles;  // rows per block
constexpr int kWtStride = 128 + 8;  // LDS row of W^T (padded, 16-byte multiple: 272 B)

__device__ __forceinline__ sh4 bf4(uint32_t x, uint32_t y) {
    return sh4{(short)(x & 0xFFFFu), (short)(x >> 16), (short)(y & 0xFFFFu), (short)(y >> 16)};
}

template <int K>
__global__ __launch_bounds__(256) void k_gemm(const uint16_t* __restrict__ A, int lda, int N,
                                              const uint16_t* __restrict__ W,
                                              const float* __restrict__ bias, int relu,
                                              uint16_t* __restrict__ out_bf, int ldo,
                                              float* __restrict__ out_f) {
    static_assert(K % 16 == 0 && K <= 128, "K: a multiple of 16 up to 128");
    constexpr int kl = K / 4;                 // run length per lane group
    constexpr bool wide = kl % 8 == 0;        // 16-byte pieces
    constexpr int np = wide ? kl / 8 : kl / 4;  // pieces per run
    __shared__ uint16_t Wt[64 * kWtStride];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kb = (lane >> 4) * kl;  // start of this lane's run
    // loads first, in the order they are needed: this thread's share of W
    // ([K x 64] in 8-column chunks of 16 bytes; chunk i is row i % K, so the
    // lanes of a wave write consecutive k of one W^T row below, free of LDS
    // bank conflicts), its A run, the bias of its columns
    constexpr int nw = (K * 8 + 255) / 256;  // chunks per thread
    uint4 wq[nw];
#pragma unroll
    for (int m = 0; m < nw; ++m) {
        const int i = threadIdx.x + 256 * m;  // blockDim.x == 256
        wq[m] = (K * 8 % 256 == 0 || i < K * 8)
                    ? *reinterpret_cast<const uint4*>(W + (size_t)(i % K) * 64 + (i / K) * 8)
                    : uint4{0u, 0u, 0u, 0u};
    }
    int rows[kGemmTiles];
    uint4 av[kGemmTiles][np];
#pragma unroll
    for (int q = 0; q < kGemmTiles; ++q) {
        rows[q] = (blockIdx.x * 4 * kGemmTiles + wave * kGemmTiles + q) * 16 + (lane & 15);
        const uint16_t* ar = A + (size_t)(rows[q] < N ? rows[q] : 0) * lda + kb;
#pragma unroll
        for (int p = 0; p < np; ++p) {
            if (rows[q] >= N) {
                av[q][p] = uint4{0u, 0u, 0u, 0u};
            } else if (wide) {
                av[q][p] = *reinterpret_cast<const uint4*>(ar + 8 * p);
            } else {
                const uint2 v = *reinterpret_cast<const uint2*>(ar + 4 * p);
                av[q][p] = uint4{v.x, v.y, 0u, 0u};
            }
        }
    }
    float4 bq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        bq[c] = bias ? *reinterpret_cast<const float4*>(bias + c * 16 + 4 * (lane >> 4))
                     : float4{0.f, 0.f, 0.f, 0.f};
    // W written transposed into LDS
#pragma unroll
    for (int m = 0; m < nw; ++m) {
        const int i = threadIdx.x + 256 * m;
        if (K * 8 % 256 != 0 && i >= K * 8) break;
        const int k = i % K, c0 = (i / K) * 8;
        const uint32_t qw[4] = {wq[m].x, wq[m].y, wq[m].z, wq[m].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            Wt[(c0 + 2 * j) * kWtStride + k] = (uint16_t)(qw[j] & 0xFFFFu);
            Wt[(c0 + 2 * j + 1) * kWtStride + k] = (uint16_t)(qw[j] >> 16);
        }
    }
    __syncthreads();
    const uint16_t* __restrict__ wr = Wt + (lane & 15) * kWtStride + kb;
    f4 acc[kGemmTiles][4];
#pragma unroll
    for (int q = 0; q < kGemmTiles; ++q)
        for (int c = 0; c < 4; ++c) acc[q][c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < np; ++p) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (wide) {
                const uint4 wv = *reinterpret_cast<const uint4*>(wr + c * 16 * kWtStride + 8 * p);
#pragma unroll
                for (int q = 0; q < kGemmTiles; ++q) acc[q][c] = mfma32(wv, av[q][p], acc[q][c]);
            } else {
                const uint2 wv = *reinterpret_cast<const uint2*>(wr + c * 16 * kWtStride + 4 * p);
#pragma unroll
                for (int q = 0; q < kGemmTiles; ++q)
                    acc[q][c] = mfma(bf4(wv.x, wv.y), bf4(av[q][p].x, av[q][p].y), acc[q][c]);
            }
        }
    }
    // lane holds Y[row][16 c + 4 (l / 16) + j], j = 0..3, of each tile
#pragma unroll
    for (int q = 0; q < kGemmTiles; ++q) {
        const int row = rows[q];
        if (row >= N) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = c * 16 + 4 * (lane >> 4);
            const float v[4] = {acc[q][c][0] + bq[c].x, acc[q][c][1] + bq[c].y,
                                acc[q][c][2] + bq[c].z, acc[q][c][3] + bq[c].w};
            if (out_f)
                *reinterpret_cast<float4*>(out_f + (size_t)row * 64 + col) =
                    float4{v[0], v[1], v[2], v[3]};
            if (out_bf) {
                uint16_t o[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) o[j] = f2bf(relu ? fmaxf(v[j], 0.f) : v[j]);
                *reinterpret_cast<uint2*>(out_bf + (size_t)row * ldo + col) =
                    uint2{(uint32_t)o[0] | ((uint32_t)o[1] << 16),
                          (uint32_t)o[2] | ((uint32_t)o[3] << 16)};
            }
        }
    }
}

// Partial P_b[K x 64] = sum over the rows of block b of A[row]^T D[row].
// Wave w accumulates k-tiles w and w + 4.
__global__ __launch_bounds__(256) void k_gemm_tn(const uint16_t* __restrict__ A, int lda, int N,
                                                 int K, const uint16_t* __restrict__ D,
                                                 int rows_per_block, float* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nkt = K / 16;
    const int kq = 4 * (lane >> 4);
    const int rb0 = blockIdx.x * rows_per_block;
    const int rb1 = min(N, rb0 + rows_per_block);
    f4 acc[2][4];
    for (int t = 0; t < 2; ++t)
        for (int c = 0; c < 4; ++c) acc[t][c] = f4{0.f, 0.f, 0.f, 0.f};
    for (int rb = rb0; rb < rb1; rb += 16) {
        sh4 b[4];
        for (int c = 0; c < 4; ++c)
            for (int j = 0; j < 4; ++j) {
                const int row = rb + kq + j;
                b[c][j] = row < rb1 ? (short)D[(size_t)row * 64 + c * 16 + (lane & 15)] : (short)0;
            }
        for (int t = 0; t < 2; ++t) {
            const int kt = wave + 4 * t;
            if (kt >= nkt) break;
            sh4 a;
            for (int j = 0; j < 4; ++j) {
                const int row = rb + kq + j;
                a[j] = row < rb1 ? (short)A[(size_t)row * lda + kt * 16 + (lane & 15)] : (short)0;
            }
            for (int c = 0; c < 4; ++c) acc[t][c] = mfma(a, b[c], acc[t][c]);
        }
    }
    float* P = part + (size_t)blockIdx.x * K * 64;
    for (int t = 0; t < 2; ++t) {
        const int kt = wave + 4 * t;
        if (kt >= nkt) break;
        for (int c = 0; c < 4; ++c)
            for (int j = 0; j < 4; ++j)
                P[(kt * 16 + kq + j) * 64 + c * 16 + (lane & 15)] = acc[t][c][j];
    }
}

// out[i] = sum_b part[b][i] in block order, i < n.
__global__ void k_reduce_parts(const float* __restrict__ part, int nparts, int n,
                               float* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int b = 0; b < nparts; ++b) s += part[(size_t)b * n + i];
    out[i] = s;
}

// out[i] = sum_b part[b][i] with one block per output (many parts, few
// outputs); fixed order within each block.
__global__ void k_reduce_cols(const float* __restrict__ part, int nparts, int n,
                              float* __restrict__ out) {
    const int i = blockIdx.x;
    float s = 0.f;
    for (int b = threadIdx.x; b < nparts; b += 256) s += part[(size_t)b * n + i];
    __shared__ float sm[256];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sm[0];
}

// Wt[h][c][k] = W[64 h + k][c] for W [128 x 64]: the operand of dHC = dZ W^T
// split into its two 64-column halves.
__global__ void k_transpose_halves(const uint16_t* __restrict__ W, uint16_t* __restrict__ Wt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 128 * 64) return;
    const int k = i >> 6, c = i & 63;
    Wt[(k >> 6) * 4096 + c * 64 + (k & 63)] = W[i];
}

// HC[i][64 + f] = mean over in-set neighbours j of HC[j][f]; 8 threads per
// node, 8 features (16 bytes) each.
__global__ void k_aggregate(uint16_t* __restrict__ HC, int N, const int32_t* __restrict__ adj,
                            int aw, const float* __restrict__ inv_deg) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int i = t >> 3, f0 = (t & 7) * 8;
    if (i >= N) return;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < aw; ++s) {
        const int j = adj[(size_t)i * aw + s];
        if (j < 0) continue;
        const uint4 v = *reinterpret_cast<const uint4*>(HC + (size_t)j * 128 + f0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        for (int q = 0; q < 4; ++q) {
            acc[2 * q] += __uint_as_float(w[q] << 16);
            acc[2 * q + 1] += __uint_as_float(w[q] & 0xFFFF0000u);
        }
    }
    const float d = inv_deg[i];
    uint32_t w[4];
    for (int q = 0; q < 4; ++q)
        w[q] = (uint32_t)f2bf(acc[2 * q] * d) | ((uint32_t)f2bf(acc[2 * q + 1] * d) << 16);
    *reinterpret_cast<uint4*>(HC + (size_t)i * 128 + 64 + f0) = uint4{w[0], w[1], w[2], w[3]};
}

// dH[j][f] += sum over neighbours i of dHn[i][f] inv_deg[i].  The neighbour
// relation is symmetric, so the transpose of the mean is this gather.
__global__ void k_aggregate_back(float* __restrict__ dH, const float* __restrict__ dHn, int N,
                                 const int32_t* __restrict__ adj, int aw,
                                 const float* __restrict__ inv_deg) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int j = t >> 6, f = t & 63;
    if (j >= N) return;
    float acc = 0.f;
    for (int s = 0; s < aw; ++s) {
        const int i = adj[(size_t)j * aw + s];
        if (i >= 0) acc += dHn[(size_t)i * 64 + f] * inv_deg[i];
    }
    dH[(size_t)j * 64 + f] += acc;
}

__global__ void k_relu_back(const float* __restrict__ dH, const uint16_t* __restrict__ H, int ldh,
                            int N, uint16_t* __restrict__ dZ) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= N * 64) return;
    const int i = t >> 6, f = t & 63;
    dZ[t] = bf2f(H[(size_t)i * ldh + f]) > 0.f ? f2bf(dH[t]) : (uint16_t)0;
}

__global__ void k_colsum(const uint16_t* __restrict__ D, int N, int rows_per_block,
                         float* __restrict__ part) {
    const int f = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int r0 = blockIdx.x * rows_per_block, r1 = min(N, r0 + rows_per_block);
    __shared__ float sm[4][64];
    float s = 0.f;
    for (int r = r0 + g; r < r1; r += 4) s += bf2f(D[(size_t)r * 64 + f]);
    sm[g][f] = s;
    __syncthreads();
    if (g == 0) part[(size_t)blockIdx.x * 64 + f] = sm[0][f] + sm[1][f] + sm[2][f] + sm[3][f];
}

__device__ __forceinline__ float block_sum256(float v, float* sm) {
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    return sm[0];
}

// sum_f row[f] w[f] over a 64-wide BF16 row (16-byte aligned), 8 at a time.
__device__ __forceinline__ float dot_row(const uint16_t* __restrict__ row,
                                         const float* __restrict__ w) {
    float s = 0.f;
    for (int q = 0; q < 8; ++q) {
        const uint4 v = *reinterpret_cast<const uint4*>(row + 8 * q);
        const uint32_t x[4] = {v.x, v.y, v.z, v.w};
        for (int j = 0; j < 4; ++j) {
            s += __uint_as_float(x[j] << 16) * w[8 * q + 2 * j];
            s += __uint_as_float(x[j] & 0xFFFF0000u) * w[8 * q + 2 * j + 1];
        }
    }
    return s;
}

// One thread per fine cell (t < nF) or fine edge (nF <= t < nF + nFe).
__global__ void k_heads(const uint16_t* __restrict__ H, int ldh, int nF, int nFe,
                        const int32_t* __restrict__ ec0, const int32_t* __restrict__ ec1,
                        const float* __restrict__ wh, const float* __restrict__ bh,
                        const float* __restrict__ wu, const float* __restrict__ th,
                        const float* __restrict__ tu, float tsh, float tsu,
                        float* __restrict__ out_h, float* __restrict__ out_u,
                        float* __restrict__ gh, float* __restrict__ gu,
                        float* __restrict__ part) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (t < nF) {
        float s = bh[0] + dot_row(H + (size_t)t * ldh, wh);
        if (out_h) out_h[t] = s;
        if (th) {
            const float d = s - tsh * th[t];
            l = d * d / nF;
            gh[t] = 2.f * d / nF;
        }
    } else if (t < nF + nFe) {
        const int e = t - nF;
        const float s = dot_row(H + (size_t)ec1[e] * ldh, wu) - dot_row(H + (size_t)ec0[e] * ldh, wu);
        if (out_u) out_u[e] = s;
        if (tu) {
            const float d = s - tsu * tu[e];
            l = d * d / nFe;
            gu[e] = 2.f * d / nFe;
        }
    }
    if (!part) return;
    __shared__ float sm[256];
    const float tot = block_sum256(l, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// 64 nodes per block (4 at a time), one thread per feature.
__global__ void k_heads_back(const uint16_t* __restrict__ H, int ldh, int N, int nF,
                             const int32_t* __restrict__ node_edges, int aw,
                             const float* __restrict__ wh, const float* __restrict__ wu,
                             const float* __restrict__ gh, const float* __restrict__ gu,
                             float* __restrict__ dH, float* __restrict__ part) {
    const int f = threadIdx.x & 63, g = threadIdx.x >> 6;
    float pwh = 0.f, pwu = 0.f, pbh = 0.f;
    for (int r = 0; r < 16; ++r) {
        const int i = blockIdx.x * 64 + r * 4 + g;
        if (i >= N) break;
        const float hv = bf2f(H[(size_t)i * ldh + f]);
        float d = 0.f;
        if (i < nF) {
            d += gh[i] * wh[f];
            pwh += gh[i] * hv;
            pbh += gh[i];
        }
        for (int s = 0; s < aw; ++s) {
            const int code = node_edges[(size_t)i * aw + s];
            if (code < 0) continue;
            const float sg = (code & 1) ? gu[code >> 1] : -gu[code >> 1];
            d += sg * wu[f];
            pwu += sg * hv;
        }
        dH[(size_t)i * 64 + f] = d;
    }
    __shared__ float sm[3][4][64];
    sm[0][g][f] = pwh;
    sm[1][g][f] = pwu;
    sm[2][g][f] = pbh;
    __syncthreads();
    if (g == 0) {
        float* P = part + (size_t)blockIdx.x * 129;
        P[f] = sm[0][0][f] + sm[0][1][f] + sm[0][2][f] + sm[0][3][f];
        P[64 + f] = sm[1][0][f] + sm[1][1][f] + sm[1][2][f] + sm[1][3][f];
        if (f == 0) P[128] = sm[2][0][0] + sm[2][1][0] + sm[2][2][0] + sm[2][3][0];
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, const int32_t* __restrict__ bf_map,
                       uint16_t* __restrict__ wbf) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    if (bf_map[i] >= 0) wbf[bf_map[i]] = f2bf(pi);
}

__global__ void k_to_bf16(const float* __restrict__ x, int n, uint16_t* __restrict__ y) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

__global__ void k_norm_features(const float* __restrict__ raw, int N, const float* __restrict__ mu,
                                const float* __restrict__ inv_sd, uint16_t* __restrict__ X) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= N * kFeat) return;
    const int f = t % kFeat;
    float v = 0.f;
    if (f < 5) v = (raw[t] - mu[f]) * inv_sd[f];
    else if (f < kRawFeat) v = raw[t];
    X[t] = f2bf(v);
}

// Per block: [sum x_f (f < 5), sum x_f^2 (f < 5), sum th^2, sum tu^2] in FP64.
__global__ void k_stats(const float* __restrict__ raw, long rows, const float* __restrict__ tgt,
                        int S, int nF, int nFe, double* __restrict__ part) {
    double a[12];
    for (int k = 0; k < 12; ++k) a[k] = 0.0;
    const long stride = (long)gridDim.x * 256;
    for (long r = blockIdx.x * 256L + threadIdx.x; r < rows; r += stride)
        for (int f = 0; f < 5; ++f) {
            const double x = raw[r * kFeat + f];
            a[f] += x;
            a[5 + f] += x * x;
        }
    const long nT = (long)nF + nFe;
    for (long r = blockIdx.x * 256L + threadIdx.x; r < (long)S * nT; r += stride) {
        const double x = tgt[r];
        a[(r % nT) < nF ? 10 : 11] += x * x;
    }
    __shared__ double sm[256];
    for (int k = 0; k < 12; ++k) {
        sm[threadIdx.x] = a[k];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * 12 + k] = sm[0];
        __syncthreads();
    }
}

// norm = [mu(5) | inv_sd(5) | 1/rms_h, 1/rms_u | rms_h, rms_u | 0 0]; a
// column whose variance is below 1e-10 of its mean square is dropped
// (inv_sd = 0), a zero target scale is taken as 1.
__global__ void k_stats_final(const double* __restrict__ part, int nparts, long rows, int S,
                              int nF, int nFe, float* __restrict__ norm) {
    const int k = threadIdx.x;
    __shared__ double tot[12];
    if (k < 12) {
        double s = 0.0;
        for (int b = 0; b < nparts; ++b) s += part[b * 12 + k];
        tot[k] = s;
    }
    __syncthreads();
    if (k < 5) {
        const double n = (double)rows;
        const double mu = tot[k] / n, m2 = tot[5 + k] / n;
        const double var = m2 - mu * mu;
        norm[k] = (float)mu;
        norm[5 + k] = var > 1e-10 * m2 && var > 0.0 ? (float)(1.0 / sqrt(var)) : 0.f;
    } else if (k < 7) {
        const int j = k - 5;
        const double n = (double)S * (j == 0 ? nF : nFe);
        double rms = n > 0 ? sqrt(tot[10 + j] / n) : 0.0;
        if (!(rms > 0.0)) rms = 1.0;
        norm[10 + j] = (float)(1.0 / rms);
        norm[12 + j] = (float)rms;
    } else if (k < 9) {
        norm[7 + k] = 0.f;
    }
}

// ------------------------------------------------------------- state side
template <typename T>
__global__ void k_build_graph(DevMesh<T> m, int N, int nFe, int32_t* __restrict__ adj,
                              float* __restrict__ inv_deg, int32_t* __restrict__ node_edges,
                              int32_t* __restrict__ ec0, int32_t* __restrict__ ec1) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int G = padded_slots(m.maxE);  // adjacency width
    const int2 so = m.cso[i];
    const int n = so.y;
    int deg = 0;
    for (int s = 0; s < G; ++s) {
        int nb = -1, code = -1;
        if (s < n) {
            const size_t o = (size_t)so.x + s;
            const int j = m.coc[o];
            if (j >= 0 && j < N) {
                nb = j;
                ++deg;
            }
            const int e = m.eoc[o];
            if (e < nFe) {
                const int is1 = m.nl[o] < T(0) ? 1 : 0;  // normal points into cell i
                code = (e << 1) | is1;
                (is1 ? ec1 : ec0)[e] = i;
            }
        }
        adj[(size_t)i * G + s] = nb;
        node_edges[(size_t)i * G + s] = code;
    }
    inv_deg[i] = deg ? 1.f / deg : 0.f;
}

template <typename T>
__global__ void k_features(DevMesh<T> m, const T* __restrict__ h, const T* __restrict__ u, int N,
                           int cb1, int cb3, int cb4, float* __restrict__ raw) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int2 so = m.cso[i];
    const int n = so.y;
    const int nV = m.nV;
    T div = 0, K = 0, vort = 0;
    for (int s = 0; s < n; ++s) {
        const size_t o = (size_t)so.x + s;
        const T ue = u[m.eoc[o]];
        div += m.nl[o] * ue;
        K += m.kc[o] * ue * ue;
        const int v = m.voc[o];
        T circ = 0, av = 0;
        for (int k = 0; k < 3; ++k) {
            circ += m.tdc[k * nV + v] * u[m.eov[k * nV + v]];
            av += m.kite[k * nV + v];
        }
        vort += m.kf[o] * (circ / av);
    }
    float* r = raw + (size_t)i * kFeat;
    // h + b: in the perturbation form (href present) the state holds
    // eta = h - href, so h + b = href + eta + b, summed in FP64
    r[0] = m.href ? (float)((double)m.href[i] + (double)h[i] + (double)m.bot[i])
                  : (float)(h[i] + m.beta[i]);
    r[1] = (float)m.bot[i];
    r[2] = (float)(div / m.area[i]);
    r[3] = (float)vort;
    r[4] = (float)K;
    r[5] = i < cb1 ? 1.f : 0.f;
    r[6] = i >= cb1 && i < cb3 ? 1.f : 0.f;
    r[7] = i >= cb3 && i < cb4 ? 1.f : 0.f;
    r[8] = i >= cb4 ? 1.f : 0.f;
    for (int f = kRawFeat; f < kFeat; ++f) r[f] = 0.f;
}

template <typename T>
__global__ void k_increments(const T* __restrict__ h0, const T* __restrict__ u0,
                             const T* __restrict__ h1, const T* __restrict__ u1,
                             const T* __restrict__ R0h, const T* __restrict__ R0u, T dt, int nF,
                             int nFe, float* __restrict__ tgt) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < nF) tgt[t] = (float)(h1[t] - h0[t] - dt * R0h[t]);
    else if (t < nF + nFe) tgt[t] = (float)(u1[t - nF] - u0[t - nF] - dt * R0u[t - nF]);
}

template <typename T>
__global__ void k_apply(const T* __restrict__ h, const T* __restrict__ u,
                        const T* __restrict__ R0h, const T* __restrict__ R0u, T dt,
                        const float* __restrict__ out_h, const float* __restrict__ out_u,
                        const float* __restrict__ scale, int nF, int nFe, T* __restrict__ xh,
                        T* __restrict__ xu) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < nF) xh[t] = h[t] + dt * R0h[t] + (T)(scale[0] * out_h[t]);
    else if (t < nF + nFe) {
        const int e = t - nF;
        xu[e] = u[e] + dt * R0u[e] + (T)(scale[1] * out_u[e]);
    }
}

// Stage states of the interface accumulation, L = 3M layers [element][L]
// (layer l = 3k + s: stage s of fine substep k), on the elements the
// interface pass reads: fine (cls 0) = x_n + tau_l (x_pred - x_n); interface 1
// (cls 1) = c0 X0 + c1 X1 + c2 X2 from its copies of the coarse stages;
// interface 2 and coarse (cls 2) = the coarse stage X_s.  Coefficients are
// FP64 (coef[l] = {tau, c0, c1, c2}); entries past ncl are edges.
template <typename T>
__global__ void k_iface_fill(const int32_t* __restrict__ cidx, const int8_t* __restrict__ ccls,
                             int ncl, const int32_t* __restrict__ eidx,
                             const int8_t* __restrict__ ecls, int nel, int L,
                             const double* __restrict__ coef, IfaceSrc<T> h, IfaceSrc<T> u,
                             int cb3, int eb2, T* __restrict__ hS, T* __restrict__ uS) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const long ent = t / L;
    const int l = (int)(t % L);
    if (ent >= (long)ncl + nel) return;
    const bool cell = ent < ncl;
    const IfaceSrc<T>& x = cell ? h : u;
    const int j = cell ? cidx[ent] : eidx[ent - ncl];
    const int cls = cell ? ccls[ent] : ecls[ent - ncl];
    const int lo = cell ? cb3 : eb2;
    const double* c = coef + 4 * l;
    double v;
    if (cls == 0) {
        const double a = (double)x.x0[j];
        v = a + c[0] * ((double)x.pred[j] - a);
    } else if (cls == 1) {
        const int k = j - lo;
        v = c[1] * (double)x.i0[k] + c[2] * (double)x.i1[k] + c[3] * (double)x.i2[k];
    } else {
        const int st = l % 3;
        v = (double)(st == 0 ? x.x0[j] : st == 1 ? x.x1[j] : x.x2[j]);
    }
    (cell ? hS : uS)[(size_t)j * L + l] = (T)v;
}

// Interface correction from the stage tendencies: x[lo + j] = x_n[lo + j]
// + delta sum_k (G_k0 / 6 + G_k1 / 6 + 2 G_k2 / 3), sums in FP64.
template <typename T>
__global__ void k_iface_combine(const T* __restrict__ acch, const T* __restrict__ accu, int nIc,
                                int nIe, int L, double delta, int cb3, int eb2,
                                const T* __restrict__ x0h, const T* __restrict__ x0u,
                                T* __restrict__ xh, T* __restrict__ xu) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= nIc + nIe) return;
    const bool cell = t < nIc;
    const int k = cell ? t : t - nIc;
    const T* a = (cell ? acch : accu) + (size_t)k * L;
    double sum = 0.0;
    for (int l = 0; l + 2 < L; l += 3)
        sum += (double)a[l] / 6.0 + (double)a[l + 1] / 6.0 + 2.0 * (double)a[l + 2] / 3.0;
    const int j = (cell ? cb3 : eb2) + k;
    if (cell) xh[j] = (T)((double)x0h[j] + delta * sum);
    else xu[j] = (T)((double)x0u[j] + delta * sum);
}

// Mass change sum_i A_i (h1_i - h0_i) over all cells: FP64 block partials in
// a fixed tree order, then one block sums them and stores the thickness
// shift that removes it from the fine cells (the change divided by their
// total area, inv_area_f = 1 / sum over fine cells of A_i).
template <typename T>
__global__ void k_mass_part(const T* __restrict__ area, const T* __restrict__ h0,
                            const T* __restrict__ h1, int nC, double* __restrict__ part) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    __shared__ double sm[256];
    sm[threadIdx.x] = i < nC ? (double)area[i] * ((double)h1[i] - (double)h0[i]) : 0.0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_mass_final(const double* __restrict__ part, int nparts, double inv_area_f,
                             double* __restrict__ shift) {
    __shared__ double sm[256];
    double a = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 256) a += part[b];
    sm[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) shift[0] = sm[0] * inv_area_f;
}

template <typename T>
__global__ void k_mass_apply(T* __restrict__ h, int nF, const double* __restrict__ shift) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < nF) h[i] = (T)((double)h[i] - shift[0]);
}

template <typename T>
__global__ void k_gate(const T* __restrict__ h0, const T* __restrict__ u0,
                       const T* __restrict__ h1, const T* __restrict__ u1,
                       const T* __restrict__ R0h, const T* __restrict__ R0u,
                       const T* __restrict__ R1h, const T* __restrict__ R1u, int nF, int nFe,
                       double dt, double* __restrict__ part) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (t < nF) {
        const double r =
            ((double)h1[t] - (double)h0[t]) / dt - 0.5 * ((double)R0h[t] + (double)R1h[t]);
        a[0] = r * r;
        a[1] = (double)R0h[t] * (double)R0h[t];
        a[2] = (double)R1h[t] * (double)R1h[t];
    } else if (t < nF + nFe) {
        const int e = t - nF;
        const double r =
            ((double)u1[e] - (double)u0[e]) / dt - 0.5 * ((double)R0u[e] + (double)R1u[e]);
        a[3] = r * r;
        a[4] = (double)R0u[e] * (double)R0u[e];
        a[5] = (double)R1u[e] * (double)R1u[e];
    }
    // one fixed-order tree over the block for all six sums
    __shared__ double red[6][256];
    const int i = threadIdx.x;
    for (int k = 0; k < 6; ++k) red[k][i] = a[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (i < w)
            for (int k = 0; k < 6; ++k) red[k][i] += red[k][i + w];
        __syncthreads();
    }
    if (i < 6) part[blockIdx.x * 6 + i] = red[i][0];
}

// Totals of the per-block partials: 256 strided sums, then a tree, all in a
// fixed order (the gate value does not depend on timing).
__global__ __launch_bounds__(256) void k_gate_final(const double* __restrict__ part, int nparts,
                                                    double* __restrict__ out) {
    __shared__ double red[6][256];
    const int i = threadIdx.x;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = i; b < nparts; b += 256)
        for (int k = 0; k < 6; ++k) v[k] += part[(size_t)b * 6 + k];
    for (int k = 0; k < 6; ++k) red[k][i] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (i < w)
            for (int k = 0; k < 6; ++k) red[k][i] += red[k][i + w];
        __syncthreads();
    }
    if (i < 6) out[i] = red[i][0];
}

}  // namespace

// ---------------------------------------------------------------- launchers
void gemm(const uint16_t* A, int lda, int N, int K, const uint16_t* W, const float* bias,
          int relu, uint16_t* out_bf, int ldo, float* out_f, hipStream_t s) {
    if (N <= 0) return;
    const dim3 g(nblk(N, kGemmRows)), b(256);
    switch (K) {
        case 16: hipLaunchKernelGGL(k_gemm<16>, g, b, 0, s, A, lda, N, W, bias, relu, out_bf, ldo, out_f); break;
        case 32: hipLaunchKernelGGL(k_gemm<32>, g, b, 0, s, A, lda, N, W, bias, relu, out_bf, ldo, out_f); break;
        case 48: hipLaunchKernelGGL(k_gemm<48>, g, b, 0, s, A, lda, N, W, bias, relu, out_bf, ldo, out_f); break;
        case 64: hipLaunchKernelGGL(k_gemm<64>, g, b, 0, s, A, lda, N, W, bias, relu, out_bf, ldo, out_f); break;
        case 80: hipLaunchKernelGGL(k_gemm<80>, g, b, 0, s, A, lda, N, W, bias, relu, out_bf, ldo, out_f); break;
        case 96: hipLaunchKernelGGL(k_gemm<96>, g, b, 0, s, A, lda, N, W, bias, relu, out_bf, ldo, out_f); break;
        case 112: hipLaunchKernelGGL(k_gemm<112>, g, b, 0, s, A, lda, N, W, bias, relu, out_bf, ldo, out_f); break;
        case 128: hipLaunchKernelGGL(k_gemm<128>, g, b, 0, s, A, lda, N, W, bias, relu, out_bf, ldo, out_f); break;
        default: break;  // callers pass K % 16 == 0, K <= 128
    }
}

int gemm_tn_parts(int N, int rows_per_block) { return (int)nblk(N, rows_per_block); }

void gemm_tn(const uint16_t* A, int lda, int N, int K, const uint16_t* D, int rows_per_block,
             float* part, float* out, hipStream_t s) {
    const int np = gemm_tn_parts(N, rows_per_block);
    if (np <= 0) return;
    hipLaunchKernelGGL(k_gemm_tn, dim3(np), dim3(256), 0, s, A, lda, N, K, D, rows_per_block, part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(nblk(K * 64, 256)), dim3(256), 0, s, part, np, K * 64,
                       out);
}

void transpose_halves(const uint16_t* W, uint16_t* Wt, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_halves, dim3(32), dim3(256), 0, s, W, Wt);
}

void aggregate(uint16_t* HC, int N, const int32_t* adj, int aw, const float* inv_deg,
               hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL(k_aggregate, dim3(nblk((long)N * 8, 256)), dim3(256), 0, s, HC, N, adj,
                           aw, inv_deg);
}

void aggregate_back(float* dH, const float* dHn, int N, const int32_t* adj, int aw,
                    const float* inv_deg, hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL(k_aggregate_back, dim3(nblk((long)N * 64, 256)), dim3(256), 0, s, dH,
                           dHn, N, adj, aw, inv_deg);
}

void relu_back(const float* dH, const uint16_t* H, int ldh, int N, uint16_t* dZ, hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL(k_relu_back, dim3(nblk((long)N * 64, 256)), dim3(256), 0, s, dH, H, ldh,
                           N, dZ);
}

int colsum_parts(int N, int rows_per_block) { return (int)nblk(N, rows_per_block); }

void colsum(const uint16_t* D, int N, int rows_per_block, float* part, float* out, hipStream_t s) {
    const int np = colsum_parts(N, rows_per_block);
    if (np <= 0) return;
    hipLaunchKernelGGL(k_colsum, dim3(np), dim3(256), 0, s, D, N, rows_per_block, part);
    hipLaunchKernelGGL(k_reduce_cols, dim3(64), dim3(256), 0, s, part, np, 64, out);
}

int heads_parts(int nF, int nFe) { return (int)nblk((long)nF + nFe, 256); }

void heads(const uint16_t* H, int ldh, int nF, int nFe, const int32_t* ec0, const int32_t* ec1,
           const float* wh, const float* bh, const float* wu, const float* th, const float* tu,
           float tsh, float tsu, float* out_h, float* out_u, float* gh, float* gu, float* part,
           float* loss, hipStream_t s) {
    const int n = heads_parts(nF, nFe);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_heads, dim3(n), dim3(256), 0, s, H, ldh, nF, nFe, ec0, ec1, wh, bh, wu,
                       th, tu, tsh, tsu, out_h, out_u, gh, gu, part);
    if (part && loss) hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(256), 0, s, part, n, 1, loss);
}

int heads_back_parts(int N) { return (int)nblk(N, 64); }

void heads_back(const uint16_t* H, int ldh, int N, int nF, const int32_t* node_edges, int aw,
                const float* wh, const float* wu, const float* gh, const float* gu, float* dH,
                float* part, float* grads_head, hipStream_t s) {
    const int n = heads_back_parts(N);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_heads_back, dim3(n), dim3(256), 0, s, H, ldh, N, nF, node_edges, aw, wh,
                       wu, gh, gu, dH, part);
    hipLaunchKernelGGL(k_reduce_cols, dim3(129), dim3(256), 0, s, part, n, 129, grads_head);
}

void adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
          float eps, int step, const int32_t* bf_map, uint16_t* wbf, hipStream_t s) {
    const float c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)step)));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                       c1, c2, bf_map, wbf);
}

void to_bf16(const float* x, int n, uint16_t* y, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n, 256)), dim3(256), 0, s, x, n, y);
}

void norm_features(const float* raw, int N, const float* mu, const float* inv_sd, uint16_t* X,
                   hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL(k_norm_features, dim3(nblk((long)N * kFeat, 256)), dim3(256), 0, s, raw,
                           N, mu, inv_sd, X);
}

void feature_stats(const float* raw, long rows, const float* tgt, int S, int nF, int nFe,
                   double* part, float* norm_out, hipStream_t s) {
    const int np = 256;  // part holds 256 x 12 doubles
    hipLaunchKernelGGL(k_stats, dim3(np), dim3(256), 0, s, raw, rows, tgt, S, nF, nFe, part);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, s, (const double*)part, np, rows, S,
                       nF, nFe, norm_out);
}

template <typename T>
void build_graph(const DevMesh<T>& m, int N, int nFe, int32_t* adj, float* inv_deg,
                 int32_t* node_edges, int32_t* ec0, int32_t* ec1, hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL((k_build_graph<T>), dim3(nblk(N, 256)), dim3(256), 0, s, m, N, nFe, adj,
                           inv_deg, node_edges, ec0, ec1);
}

template <typename T>
void features(const DevMesh<T>& m, const T* h, const T* u, int N, int cb1, int cb3, int cb4,
              float* raw, hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL((k_features<T>), dim3(nblk(N, 256)), dim3(256), 0, s, m, h, u, N, cb1,
                           cb3, cb4, raw);
}

template <typename T>
void increments(const T* h0, const T* u0, const T* h1, const T* u1, const T* R0h, const T* R0u,
                double dt, int nF, int nFe, float* tgt, hipStream_t s) {
    if (nF + nFe > 0)
        hipLaunchKernelGGL((k_increments<T>), dim3(nblk((long)nF + nFe, 256)), dim3(256), 0, s, h0,
                           u0, h1, u1, R0h, R0u, (T)dt, nF, nFe, tgt);
}

template <typename T>
void apply_increments(const T* h, const T* u, const T* R0h, const T* R0u, double dt,
                      const float* out_h, const float* out_u, const float* scale, int nF, int nFe,
                      T* xh, T* xu, hipStream_t s) {
    if (nF + nFe > 0)
        hipLaunchKernelGGL((k_apply<T>), dim3(nblk((long)nF + nFe, 256)), dim3(256), 0, s, h, u,
                           R0h, R0u, (T)dt, out_h, out_u, scale, nF, nFe, xh, xu);
}

template <typename T>
void iface_fill(const int32_t* cidx, const int8_t* ccls, int ncl, const int32_t* eidx,
                const int8_t* ecls, int nel, int L, const double* coef, const IfaceSrc<T>& h,
                const IfaceSrc<T>& u, int cb3, int eb2, T* hS, T* uS, hipStream_t s) {
    const long n = ((long)ncl + nel) * L;
    if (n > 0)
        hipLaunchKernelGGL((k_iface_fill<T>), dim3(nblk(n, 256)), dim3(256), 0, s, cidx, ccls, ncl,
                           eidx, ecls, nel, L, coef, h, u, cb3, eb2, hS, uS);
}

template <typename T>
void iface_combine(const T* acch, const T* accu, int nIc, int nIe, int L, double delta, int cb3,
                   int eb2, const T* x0h, const T* x0u, T* xh, T* xu, hipStream_t s) {
    if (nIc + nIe > 0)
        hipLaunchKernelGGL((k_iface_combine<T>), dim3(nblk((long)nIc + nIe, 256)), dim3(256), 0, s,
                           acch, accu, nIc, nIe, L, delta, cb3, eb2, x0h, x0u, xh, xu);
}

int mass_fix_parts(int nC) { return (int)nblk(nC, 256); }

template <typename T>
void mass_fix(const T* area, const T* h0, T* h1, int nC, int nF, double inv_area_f, double* part,
              double* shift, hipStream_t s) {
    const int np = mass_fix_parts(nC);
    if (np == 0 || nF == 0) return;
    hipLaunchKernelGGL((k_mass_part<T>), dim3(np), dim3(256), 0, s, area, h0, (const T*)h1, nC,
                       part);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(256), 0, s, (const double*)part, np, inv_area_f,
                       shift);
    hipLaunchKernelGGL((k_mass_apply<T>), dim3(nblk(nF, 256)), dim3(256), 0, s, h1, nF,
                       (const double*)shift);
}

template <typename T>
void gate_sums(const T* h0, const T* u0, const T* h1, const T* u1, const T* R0h, const T* R0u,
               const T* R1h, const T* R1u, int nF, int nFe, double dt, double* part, double* out,
               hipStream_t s) {
    const unsigned n = nblk((long)nF + nFe, 256);
    if (n == 0) return;
    hipLaunchKernelGGL((k_gate<T>), dim3(n), dim3(256), 0, s, h0, u0, h1, u1, R0h, R0u, R1h, R1u,
                       nF, nFe, dt, part);
    hipLaunchKernelGGL(k_gate_final, dim3(1), dim3(256), 0, s, (const double*)part, (int)n, out);
}

#define LTS_NN_INSTANTIATE(T)                                                                    \
    template void build_graph<T>(const DevMesh<T>&, int, int, int32_t*, float*, int32_t*,        \
                                 int32_t*, int32_t*, hipStream_t);                               \
    template void features<T>(const DevMesh<T>&, const T*, const T*, int, int, int, int, float*, \
                              hipStream_t);                                                      \
    template void increments<T>(const T*, const T*, const T*, const T*, const T*, const T*,      \
                                double, int, int, float*, hipStream_t);                          \
    template void apply_increments<T>(const T*, const T*, const T*, const T*, double,            \
                                      const float*, const float*, const float*, int, int, T*,    \
                                      T*, hipStream_t);                                          \
    template void iface_fill<T>(const int32_t*, const int8_t*, int, const int32_t*,             \
                                const int8_t*, int, int, const double*, const IfaceSrc<T>&,      \
                                const IfaceSrc<T>&, int, int, T*, T*, hipStream_t);              \
    template void iface_combine<T>(const T*, const T*, int, int, int, double, int, int,          \
                                   const T*, const T*, T*, T*, hipStream_t);                     \
    template void mass_fix<T>(const T*, const T*, T*, int, int, double, double*, double*,        \
                              hipStream_t);                                                      \
    template void gate_sums<T>(const T*, const T*, const T*, const T*, const T*, const T*,       \
                               const T*, const T*, int, int, double, double*, double*,           \
                               hipStream_t);

LTS_NN_INSTANTIATE(double)
LTS_NN_INSTANTIATE(float)

}  // namespace nn
}  // namespace lts
