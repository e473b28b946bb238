// sphx_gnn.hpp -- HIP kernels (gfx950) of the message-passing surrogate on
// the SPH neighbour graph: features from the frozen configuration, BF16 MFMA
// matrix products with FP32 accumulation, edge messages summed per particle,
// the backward pass, Adam and the surrogate's state update.
//
// The network (hidden width 64, 3 layers) predicts each fluid particle's
// mean acceleration and density rate over the next two advection steps:
//   H = relu(F Wn + bn),  E0 = relu(G We + be)
//   layer: P = H Wa + bm, Q = H Wb, R = E0 Wc; m_e = relu(P_i + Q_j + R_e)
//          (a wall edge takes the learned vector qw in place of Q_j);
//          A_i = sum_e m_e;  H <- H + relu([H | A] Wu + bu)
//   Y = relu(H Wo1 + bo1) Wo2 + bo2 = (a_x/g, a_y/g, 1000 Drho h / (rho0 u_ref))
// Node rows are the fluid slots of the batch layout (padding slots carry
// zeros); edge rows are, per particle, its inner then its contact entries in
// list order (CSR by particle). Activations are FP32; every matrix-product
// operand is rounded to bfloat16 (nearest, ties to even) as it is loaded into
// an MFMA fragment, and the products accumulate in FP32. The last product
// (D1 Wo2, 64 -> 3) runs in FP32 on the vector units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sphx_device.hpp"

namespace sphx {
namespace gnn {

constexpr int HID = 64;
constexpr int FPAD = 32;   // padded encoder input width
constexpr int EFEAT = 8;   // edge features used
constexpr int NOUT = 3;
constexpr int WALL_EDGE = -1;  // edst < 0: wall edge, wall index -1 - edst

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

union Frag {
    bf16x8 v;
    uint32_t u[4];
    uint4 q;
};

// Eight consecutive floats rounded into an MFMA operand fragment.
__device__ __forceinline__ bf16x8 frag_from_f32(const float* p, bool ok)
{
    Frag f;
    if (ok) {
        const float4 a = *(const float4*)p;
        const float4 b = *(const float4*)(p + 4);
        f.u[0] = bf16_bits(a.x) | (bf16_bits(a.y) << 16);
        f.u[1] = bf16_bits(a.z) | (bf16_bits(a.w) << 16);
        f.u[2] = bf16_bits(b.x) | (bf16_bits(b.y) << 16);
        f.u[3] = bf16_bits(b.z) | (bf16_bits(b.w) << 16);
    } else {
        f.q = make_uint4(0u, 0u, 0u, 0u);
    }
    return f.v;
}

__device__ __forceinline__ bf16x8 frag_from_bf16(const uint16_t* p)
{
    Frag f;
    f.q = *(const uint4*)p;
    return f.v;
}

// ---------------------------------------------------------------------
// Matrix product with a 64-wide output:
//   C[M x 64] = epi(A[M x K] B),  A FP32 rows of stride lda, B given as
//   Bt = B^T in bf16 [64 x K] (row-major, K contiguous).
// One wavefront computes 16 rows (four 16x16 tiles) with
// v_mfma_f32_16x16x32_bf16: lane l supplies row (l mod 16) of A and column
// (l mod 16) of B at the 8 K positions 8 (l div 16) + 0..7 of each 32-wide K
// step (the same positions for A and B, so the pairing is exact), and holds
// output rows 4 (l div 16) + 0..3 of column (l mod 16).
enum Epi : int {
    EPI_STORE = 0,  // C = acc + bias
    EPI_RELU = 1,   // C = relu(acc + bias)
    EPI_ACCUM = 2,  // C += acc
    EPI_RESID = 3,  // C2 = acc + bias (pre-activation); C += relu(acc + bias)
};

template <int K, int EPI>
__global__ __launch_bounds__(256) void k_gemm64(int M, const float* __restrict__ A, int lda,
                                                const uint16_t* __restrict__ Bt, const float* __restrict__ bias,
                                                float* __restrict__ C, int ldc, float* __restrict__ C2, int ldc2)
{
    static_assert(K % 32 == 0, "K must be a multiple of 32");
    const int lane = threadIdx.x & 63;
    const int m0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (m0 >= M) return;
    const int r = lane & 15, g = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ra = m0 + r;
    const bool ok = ra < M;
#pragma unroll
    for (int ks = 0; ks < K; ks += 32) {
        const bf16x8 a = frag_from_f32(A + (size_t)(ok ? ra : 0) * lda + ks + 8 * g, ok);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bf16x8 b = frag_from_bf16(Bt + (size_t)(16 * t + r) * K + ks + 8 * g);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int col = 16 * t + r;
        const float bv = bias ? bias[col] : 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = m0 + 4 * g + q;
            if (row >= M) continue;
            const float v = acc[t][q];
            float* c = C + (size_t)row * ldc + col;
            if constexpr (EPI == EPI_STORE) {
                *c = v + bv;
            } else if constexpr (EPI == EPI_RELU) {
                *c = fmaxf(v + bv, 0.f);
            } else if constexpr (EPI == EPI_ACCUM) {
                *c = *c + v;
            } else {
                const float z = v + bv;
                C2[(size_t)row * ldc2 + col] = z;
                *c = *c + fmaxf(z, 0.f);
            }
        }
    }
}

// ---------------------------------------------------------------------
// Weight gradient dW[KIN x 64] = X^T dZ over M rows, split over blocks of
// `rows` rows each (partials summed later in a fixed order), and the column
// sums of dZ (bias gradient) in FP32. Each 32-row step stages X and dZ,
// rounded to bf16 and transposed, in LDS; wavefront w computes output column
// tile w for all KIN/16 row tiles.
template <int KIN>
__global__ __launch_bounds__(256) void k_wgrad(int M, int rows, const float* __restrict__ X, int ldx,
                                               const float* __restrict__ dZ, int ldz, float* __restrict__ part,
                                               float* __restrict__ bpart)
{
    constexpr int TM = KIN / 16;
    __shared__ __align__(16) uint16_t Xs[KIN][32 + 8];
    __shared__ __align__(16) uint16_t Zs[HID][32 + 8];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    f32x4 acc[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const int r0 = blockIdx.x * rows;
    const int r1 = min(r0 + rows, M);
    for (int rb = r0; rb < r1; rb += 32) {
        // stage: X chunk 32 x KIN and dZ chunk 32 x 64, transposed
        for (int idx = threadIdx.x; idx < 32 * KIN; idx += 256) {
            const int rr = idx / KIN, k = idx % KIN;
            const int row = rb + rr;
            Xs[k][rr] = (uint16_t)(row < r1 ? bf16_bits(X[(size_t)row * ldx + k]) : 0u);
        }
        for (int idx = threadIdx.x; idx < 32 * HID; idx += 256) {
            const int rr = idx / HID, n = idx % HID;
            const int row = rb + rr;
            const float z = row < r1 ? dZ[(size_t)row * ldz + n] : 0.f;
            Zs[n][rr] = (uint16_t)bf16_bits(z);
        }
        if (threadIdx.x < HID)
            for (int rr = 0; rr < 32 && rb + rr < r1; ++rr) bsum += dZ[(size_t)(rb + rr) * ldz + threadIdx.x];
        __syncthreads();
        Frag fb;
        fb.q = *(const uint4*)&Zs[16 * w + r][8 * g];
#pragma unroll
        for (int t = 0; t < TM; ++t) {
            Frag fa;
            fa.q = *(const uint4*)&Xs[16 * t + r][8 * g];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa.v, fb.v, acc[t], 0, 0, 0);
        }
        __syncthreads();
    }
    float* out = part + (size_t)blockIdx.x * KIN * HID;
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) out[(size_t)(16 * t + 4 * g + q) * HID + 16 * w + r] = acc[t][q];
    if (threadIdx.x < HID) bpart[(size_t)blockIdx.x * HID + threadIdx.x] = bsum;
}

// out[j] (+)= sum over b of part[b][j], b ascending (deterministic).
__global__ __launch_bounds__(256) void k_reduce_parts(int nb, int len, const float* __restrict__ part,
                                                      float* __restrict__ out, int accumulate)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * len + j];
    out[j] = accumulate ? out[j] + s : s;
}

// Column sums of a [M x 64] FP32 matrix in row blocks (partials).
__global__ __launch_bounds__(64) void k_colsum64(int M, int rows, const float* __restrict__ A, int lda,
                                                 float* __restrict__ part)
{
    const int r0 = blockIdx.x * rows, r1 = min(r0 + rows, M);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) s += A[(size_t)r * lda + threadIdx.x];
    part[(size_t)blockIdx.x * HID + threadIdx.x] = s;
}

// ---------------------------------------------------------------------
// Graph: per-slot edge counts, then (after a scan) the CSR edges with their
// features, the reverse of every inner edge, and the node features.

template <typename real>
__global__ __launch_bounds__(BLOCK) void k_gnn_count(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase,
                                                     int ntiles, const int32_t* __restrict__ ncnt,
                                                     const int32_t* __restrict__ wcnt, int32_t* __restrict__ ecount)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    const int i = tile * TILE + (threadIdx.x & 63);
    ecount[i] = i < P.fbase + P.nf ? ncnt[i] + wcnt[i] : 0;
}

__device__ __forceinline__ float wendland_ratio(float q)
{
    const float s = fmaxf(1.f - 0.5f * q, 0.f);
    return s * s * s * s * (1.f + 2.f * q);
}

// One thread per slot. Edge features (x_j - x_i)/h, r/h, (v_j - v_i)/u_ref,
// W(r)/W(0), wall flag, pressure difference (p_j - p_i)/(rho0 |g| h) (for a
// wall the one-sided wall state, p_w - p_i = rho_i g.(x_w - x_i)), taken in
// FP32 from the density deviations before any rounding; node features
// v/u_ref, (rho - rho0)/(0.01 rho0), inner and contact counts / 32 and / 16
// (2D).
//
// G rows hold `ldg` floats: FPAD (zero-padded, for the training path's
// encoder product) or EFEAT (the features alone, for the fused inference
// layer). esrc (may be null) receives each edge's particle; the reverse
// edges (erev, training only: the backward of Q_j) are searched only when
// erev is given.
template <typename real, int T>
__global__ __launch_bounds__(BLOCK) void k_gnn_edges(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, int ntiles, const int32_t* __restrict__ eoff,
    const uint32_t* __restrict__ nbr, const int32_t* __restrict__ ncnt, const uint32_t* __restrict__ wnb,
    const int32_t* __restrict__ wcnt, const R2<real>* __restrict__ geo, const R2<real>* __restrict__ wgeo,
    const R4<real>* __restrict__ st, int32_t* __restrict__ edst, int32_t* __restrict__ erev,
    int32_t* __restrict__ esrc, float* __restrict__ G, int ldg, float* __restrict__ F)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    const int i = tile * TILE + (threadIdx.x & 63);
    float* f = F + (size_t)i * FPAD;
    if (i >= P.fbase + P.nf) {
        for (int k = 0; k < FPAD; ++k) f[k] = 0.f;
        return;
    }
    const float inv_u = (float)(1.0 / P.u_ref);
    const float inv_h = (float)P.inv_h;
    const float gx = (float)P.g[0], gy = (float)P.g[1];
    const float gmag = sqrtf(gx * gx + gy * gy + (float)P.g[2] * (float)P.g[2]);
    const float inv_pscale = 1.f / ((float)P.rho0 * gmag) * inv_h;
    const float c2 = (float)P.c2;
    const R4<real> si = st[i];
    const float devi = (float)si.z;
    const float vix = (float)si.x, viy = (float)si.y;
    const int nin = ncnt[i], nwl = wcnt[i];
    f[0] = vix * inv_u;
    f[1] = viy * inv_u;
    f[2] = (float)si.z / (0.01f * (float)P.rho0);
    f[3] = (float)nin / 32.f;
    f[4] = (float)nwl / 16.f;
    for (int k = 5; k < FPAD; ++k) f[k] = 0.f;
    const R2<real> oi = geo[i];
    int e = eoff[i];
    auto edge = [&](int e_, float dx, float dy, float dvx, float dvy, float wall, float dpres) {
        float* gr = G + (size_t)e_ * ldg;
        if (esrc) esrc[e_] = i;
        const float rr = sqrtf(dx * dx + dy * dy);
        gr[0] = -dx * inv_h;  // x_j - x_i
        gr[1] = -dy * inv_h;
        gr[2] = rr * inv_h;
        gr[3] = dvx * inv_u;
        gr[4] = dvy * inv_u;
        gr[5] = wendland_ratio(rr * inv_h);
        gr[6] = wall;
        gr[7] = dpres * inv_pscale;
        for (int k = EFEAT; k < ldg; ++k) gr[k] = 0.f;
    };
    for (int k = 0; k < nin; ++k, ++e) {
        const uint32_t ent = nbr[ell_at<T>(i, k, P.maxn)];
        const int j = (int)(ent & NBR_MASK);
        const uint32_t code = ent >> NBR_SHIFT;
        const R2<real> oj = geo[j];
        const float dx = (float)((oi.x - oj.x) - (real)((int)(code & 3u) - 1) * P.L[0]);
        const float dy = (float)((oi.y - oj.y) - (real)((int)((code >> 2) & 3u) - 1) * P.L[1]);
        const R4<real> sj = st[j];
        edge(e, dx, dy, (float)sj.x - vix, (float)sj.y - viy, 0.f, c2 * ((float)sj.z - devi));
        edst[e] = j;
        if (erev) {
            // the reverse edge: i in the inner list of j (the lists are symmetric)
            int rv = -1;
            const int nj = ncnt[j];
            for (int kk = 0; kk < nj; ++kk)
                if ((int)(nbr[ell_at<T>(j, kk, P.maxn)] & NBR_MASK) == i) {
                    rv = eoff[j] + kk;
                    break;
                }
            erev[e] = rv;
        }
    }
    for (int k = 0; k < nwl; ++k, ++e) {
        const uint32_t ent = wnb[ell_at<T>(i, k, P.maxw)];
        const int wj = (int)(ent & NBR_MASK);
        const uint32_t code = ent >> NBR_SHIFT;
        const R2<real> ow = wgeo[wj];
        const float dx = (float)((oi.x - ow.x) - (real)((int)(code & 3u) - 1) * P.L[0]);
        const float dy = (float)((oi.y - ow.y) - (real)((int)((code >> 2) & 3u) - 1) * P.L[1]);
        edge(e, dx, dy, -vix, -viy, 1.f, ((float)P.rho0 + devi) * (gx * -dx + gy * -dy));
        edst[e] = -1 - wj;
        if (erev) erev[e] = -1;
    }
}

// ---------------------------------------------------------------------
// Messages: one wavefront per node row, lane = feature.
//   pre_e = P_i + (Q_j | qw) + R_e,  A_i = sum_e relu(pre_e) -> X[i][64 + f]
__global__ __launch_bounds__(256) void k_gnn_msg(int N, const int32_t* __restrict__ eoff,
                                                 const int32_t* __restrict__ edst, const float* __restrict__ P,
                                                 const float* __restrict__ Q, const float* __restrict__ R,
                                                 const float* __restrict__ qw, float* __restrict__ pre_out,
                                                 float* __restrict__ X)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const int f = threadIdx.x & 63;
    const float p = P[(size_t)i * HID + f];
    const float q0 = qw[f];
    float acc = 0.f;
    for (int e = eoff[i]; e < eoff[i + 1]; ++e) {
        const int d = edst[e];
        const float pre = p + (d >= 0 ? Q[(size_t)d * HID + f] : q0) + R[(size_t)e * HID + f];
        if (pre_out) pre_out[(size_t)e * HID + f] = pre;
        acc += fmaxf(pre, 0.f);
    }
    X[(size_t)i * 2 * HID + HID + f] = acc;
}

// One message-passing layer for inference, fused: for every node i, over
// its edges e in CSR order,
//   E0_e = relu(G_e We + be),  R_e = E0_e Wc,
//   m_e  = relu((P_i + (Q_j | qw)) + R_e),  A_i = sum_e m_e -> X[i][64 + f],
// with the edge encoder and the edge product on the matrix cores, so that
// neither E0 nor R nor the messages leave the wavefront (no E x 64 array in
// HBM). Each wavefront takes NPW consecutive nodes and their edges in tiles
// of 16. The products are computed transposed (features as MFMA rows, the
// 16 edges as columns: A = W^T, B = the edge rows), so that each lane then
// holds four consecutive features of one edge and gathers P_i and Q_j with
// 16-byte loads. E0 goes from the accumulator layout to the operand layout
// through LDS, rounded to bf16 as every product operand is; the messages go
// through LDS to one lane per feature, which sums them per node in CSR
// order. G rows hold the EFEAT edge features (the encoder's other inputs
// are zero).
template <int NPW>
__global__ __launch_bounds__(256) void k_gnn_layer_fused(
    int N, const int32_t* __restrict__ eoff, const int32_t* __restrict__ edst, const int32_t* __restrict__ esrc,
    const float* __restrict__ G, const uint16_t* __restrict__ WeT, const float* __restrict__ be,
    const uint16_t* __restrict__ WcT, const float* __restrict__ Pm, const float* __restrict__ Qm,
    const float* __restrict__ qw, float* __restrict__ X)
{
    __shared__ __align__(16) uint16_t Es[4][16][HID + 8];
    __shared__ __align__(16) float Ms[4][16][HID + 4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const int n0 = (blockIdx.x * 4 + wv) * NPW;
    if (n0 >= N) return;
    const int n1 = min(n0 + NPW, N);
    const int e_beg = eoff[n0], e_end = eoff[n1];
    // weight fragments and the encoder bias of this lane, kept for all tiles
    bf16x8 wef[4], wcf[2][4];
    float bev[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        wef[t] = frag_from_bf16(WeT + (size_t)(16 * t + r) * FPAD + 8 * g);
#pragma unroll
        for (int k = 0; k < 2; ++k) wcf[k][t] = frag_from_bf16(WcT + (size_t)(16 * t + r) * HID + 32 * k + 8 * g);
#pragma unroll
        for (int q = 0; q < 4; ++q) bev[t][q] = be[16 * t + 4 * g + q];
    }
    // the reduction: lane = feature, running node `cur` (uniform)
    int cur = n0;
    int cend = eoff[n0 + 1];
    float sum = 0.f;
    for (int eb = e_beg; eb < e_end; eb += 16) {
        const int e = eb + r;
        const bool ok = e < e_end;
        const int src = ok ? esrc[e] : n0;
        const int dst = ok ? edst[e] : -1;
        // E0^T = We^T G^T: lane (r, g) holds edge r, features 16 t + 4 g + q
        const bf16x8 gfr = frag_from_f32(G + (size_t)(ok ? e : e_beg) * EFEAT, ok && g == 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f32x4 a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wef[t], gfr, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            uint2 pk;
            pk.x = bf16_bits(fmaxf(a[0] + bev[t][0], 0.f)) | (bf16_bits(fmaxf(a[1] + bev[t][1], 0.f)) << 16);
            pk.y = bf16_bits(fmaxf(a[2] + bev[t][2], 0.f)) | (bf16_bits(fmaxf(a[3] + bev[t][3], 0.f)) << 16);
            *(uint2*)&Es[wv][r][16 * t + 4 * g] = pk;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // R^T = Wc^T E0^T, two K steps of 32
        f32x4 racc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) racc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const bf16x8 efr = frag_from_bf16(&Es[wv][r][32 * k + 8 * g]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                racc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wcf[k][t], efr, racc[t], 0, 0, 0);
        }
        // messages of edge r, features 16 t + 4 g .. + 3
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int f0 = 16 * t + 4 * g;
            const float4 pv = *(const float4*)(Pm + (size_t)src * HID + f0);
            const float4 qv = dst >= 0 ? *(const float4*)(Qm + (size_t)dst * HID + f0) : *(const float4*)(qw + f0);
            float4 mv;
            mv.x = fmaxf((pv.x + qv.x) + (racc[t][0] + 0.f), 0.f);
            mv.y = fmaxf((pv.y + qv.y) + (racc[t][1] + 0.f), 0.f);
            mv.z = fmaxf((pv.z + qv.z) + (racc[t][2] + 0.f), 0.f);
            mv.w = fmaxf((pv.w + qv.w) + (racc[t][3] + 0.f), 0.f);
            *(float4*)&Ms[wv][r][f0] = mv;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // per-node sums in CSR order (every node of the range, edgeless ones
        // too); the tile's rows are read first, then summed in order
        const int nrow = min(16, e_end - eb);
        float mrow[16];
#pragma unroll
        for (int row = 0; row < 16; ++row) mrow[row] = Ms[wv][row][lane];
#pragma unroll
        for (int row = 0; row < 16; ++row) {
            if (row >= nrow) break;
            const int ee = eb + row;
            while (ee >= cend) {
                X[(size_t)cur * 2 * HID + HID + lane] = sum;
                sum = 0.f;
                ++cur;
                cend = eoff[cur + 1];
            }
            sum += mrow[row];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (; cur < n1; ++cur) {
        X[(size_t)cur * 2 * HID + HID + lane] = sum;
        sum = 0.f;
    }
}

// Backward of the messages: dM_e = dA_i [pre_e > 0]; dP_i = sum_e dM_e;
// wsum_i = sum over wall edges of dM_e (for qw).
__global__ __launch_bounds__(256) void k_gnn_msg_bwd(int N, const int32_t* __restrict__ eoff,
                                                     const int32_t* __restrict__ edst, const float* __restrict__ pre,
                                                     const float* __restrict__ dA, int ldda, float* __restrict__ dM,
                                                     float* __restrict__ dP, float* __restrict__ wsum)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const int f = threadIdx.x & 63;
    const float da = dA[(size_t)i * ldda + f];
    float sp = 0.f, sw = 0.f;
    for (int e = eoff[i]; e < eoff[i + 1]; ++e) {
        const float dm = pre[(size_t)e * HID + f] > 0.f ? da : 0.f;
        dM[(size_t)e * HID + f] = dm;
        sp += dm;
        if (edst[e] < 0) sw += dm;
    }
    dP[(size_t)i * HID + f] = sp;
    wsum[(size_t)i * HID + f] = sw;
}

// dQ_j = sum of dM over the inner edges that end at j, gathered through the
// reverse of j's own inner edges.
__global__ __launch_bounds__(256) void k_gnn_dq(int N, const int32_t* __restrict__ eoff,
                                                const int32_t* __restrict__ edst, const int32_t* __restrict__ erev,
                                                const float* __restrict__ dM, float* __restrict__ dQ)
{
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= N) return;
    const int f = threadIdx.x & 63;
    float s = 0.f;
    for (int e = eoff[j]; e < eoff[j + 1]; ++e) {
        const int rv = erev[e];
        if (edst[e] >= 0 && rv >= 0) s += dM[(size_t)rv * HID + f];
    }
    dQ[(size_t)j * HID + f] = s;
}

// out = src where mask > 0, else 0 (row strides given).
__global__ __launch_bounds__(256) void k_relu_mask(int M, const float* __restrict__ src, int lds,
                                                   const float* __restrict__ mask, int ldm, float* __restrict__ out,
                                                   int ldo)
{
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)M * HID) return;
    const size_t r = idx / HID, c = idx % HID;
    out[r * ldo + c] = mask[r * ldm + c] > 0.f ? src[r * lds + c] : 0.f;
}

// dst[r][c] = src[r][c] for a [M x 64] block (row strides given).
__global__ __launch_bounds__(256) void k_copy64(int M, const float* __restrict__ src, int lds, float* __restrict__ dst,
                                                int ldd)
{
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)M * HID) return;
    const size_t r = idx / HID, c = idx % HID;
    dst[r * ldd + c] = src[r * lds + c];
}

// Decoder output Y = D1 Wo2 + bo2 (FP32), one thread per node.
__global__ __launch_bounds__(256) void k_gnn_out(int N, const float* __restrict__ D1, const float* __restrict__ Wo2,
                                                 const float* __restrict__ bo2, float* __restrict__ Y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float y0 = bo2[0], y1 = bo2[1], y2 = bo2[2];
    const float* d = D1 + (size_t)i * HID;
    for (int k = 0; k < HID; ++k) {
        const float v = d[k];
        y0 += v * Wo2[k * NOUT + 0];
        y1 += v * Wo2[k * NOUT + 1];
        y2 += v * Wo2[k * NOUT + 2];
    }
    Y[(size_t)i * NOUT + 0] = y0;
    Y[(size_t)i * NOUT + 1] = y1;
    Y[(size_t)i * NOUT + 2] = y2;
}

// Loss: mean squared error over the fluid slots (count entries each of 3
// outputs): dY = 2 (Y - T) / (3 count); per-block partial sums of (Y - T)^2.
template <typename real>
__global__ __launch_bounds__(256) void k_gnn_loss(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase,
                                                  int ntiles, double inv_count, const float* __restrict__ Y,
                                                  const float* __restrict__ Tg, float* __restrict__ dY,
                                                  double* __restrict__ part)
{
    __shared__ double sh[4];
    const int tile = wave_tile();
    double s = 0.0;
    if (tile < ntiles) {
        const KP<real>& P = Pt[tcase[tile]];
        const int i = tile * TILE + (threadIdx.x & 63);
        const bool ok = i < P.fbase + P.nf;
        for (int c = 0; c < NOUT; ++c) {
            const float d = ok ? Y[(size_t)i * NOUT + c] - Tg[(size_t)i * NOUT + c] : 0.f;
            dY[(size_t)i * NOUT + c] = (float)(2.0 * (double)d * inv_count);
            s += (double)d * (double)d;
        }
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Decoder backward: dZ1 = (dY Wo2^T) [D1 > 0] (one thread per node and
// feature) ...
__global__ __launch_bounds__(256) void k_gnn_out_bwd(int N, const float* __restrict__ D1, const float* __restrict__ dY,
                                                     const float* __restrict__ Wo2, float* __restrict__ dZ1)
{
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)N * HID) return;
    const size_t i = idx / HID, k = idx % HID;
    const float* dy = dY + i * NOUT;
    const float v = dy[0] * Wo2[k * NOUT + 0] + dy[1] * Wo2[k * NOUT + 1] + dy[2] * Wo2[k * NOUT + 2];
    dZ1[idx] = D1[idx] > 0.f ? v : 0.f;
}

// ... and the partials of dWo2 = D1^T dY (64 x 3) and dbo2 = sum dY, per row
// block (195 values per block).
__global__ __launch_bounds__(256) void k_gnn_out_wgrad(int N, int rows, const float* __restrict__ D1,
                                                       const float* __restrict__ dY, float* __restrict__ part)
{
    const int t = threadIdx.x;
    if (t >= HID * NOUT + NOUT) return;
    const int r0 = blockIdx.x * rows, r1 = min(r0 + rows, N);
    float s = 0.f;
    if (t < HID * NOUT) {
        const int k = t / NOUT, c = t % NOUT;
        for (int r = r0; r < r1; ++r) s += D1[(size_t)r * HID + k] * dY[(size_t)r * NOUT + c];
    } else {
        const int c = t - HID * NOUT;
        for (int r = r0; r < r1; ++r) s += dY[(size_t)r * NOUT + c];
    }
    part[(size_t)blockIdx.x * (HID * NOUT + NOUT) + t] = s;
}

// Adam (FP32 master parameters); c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t).
__global__ __launch_bounds__(256) void k_adam(int n, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// bf16 copies of one weight matrix W [K x 64] (FP32, row-major at src):
// transposed (64 x K, for products with W) and as is (K x 64, for products
// with W^T).
__global__ __launch_bounds__(256) void k_pack_w(int K, const float* __restrict__ W, uint16_t* __restrict__ WT,
                                                uint16_t* __restrict__ WN)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * HID) return;
    const int k = idx / HID, n = idx % HID;
    const uint16_t b = (uint16_t)bf16_bits(W[idx]);
    WT[(size_t)n * K + k] = b;
    WN[idx] = b;
}

// Surrogate state update over dt_c of every accepted case c:
// v' = v + a dt, x' = x + (v + v')/2 dt, rho' = rho + Drho dt; Drho becomes
// the density rate carried into the next half-step.
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_gnn_apply(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase,
                                                     int ntiles, const double* __restrict__ dtc,
                                                     const int32_t* __restrict__ accept, const float* __restrict__ Y,
                                                     double* __restrict__ x0, double* __restrict__ x1,
                                                     R4<real>* __restrict__ st)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    if (!accept[P.case_id]) return;
    const int i = tile * TILE + (threadIdx.x & 63);
    if (i >= P.fbase + P.nf) return;
    const double dt = dtc[P.case_id];
    const double gmag = sqrt((double)P.g[0] * P.g[0] + (double)P.g[1] * P.g[1] + (double)P.g[2] * P.g[2]);
    const double ax = (double)Y[(size_t)i * NOUT + 0] * gmag, ay = (double)Y[(size_t)i * NOUT + 1] * gmag;
    const double drho = (double)Y[(size_t)i * NOUT + 2] * 1e-3 * P.rho0d * P.u_ref / (0.5 * sqrt(P.rc2));
    R4<real> s = st[i];
    const double vx = (double)s.x, vy = (double)s.y;
    const double vx2 = vx + ax * dt, vy2 = vy + ay * dt;
    x0[i] = x0[i] + 0.5 * (vx + vx2) * dt;
    x1[i] = x1[i] + 0.5 * (vy + vy2) * dt;
    s.x = (real)vx2;
    s.y = (real)vy2;
    s.z = (real)((double)s.z + drho * dt);
    s.w = (real)drho;
    st[i] = s;
}

// Largest |rho/rho0 - 1| the surrogate would produce over dt_c, per case:
// per-tile maxima (k_diag_fin-style reduction on the host side of the call).
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_gnn_check(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase,
                                                     int ntiles, const double* __restrict__ dtc,
                                                     const float* __restrict__ Y, const R4<real>* __restrict__ st,
                                                     double* __restrict__ tmax)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    const int i = tile * TILE + (threadIdx.x & 63);
    double v = 0.0;
    if (i < P.fbase + P.nf) {
        const double drho = (double)Y[(size_t)i * NOUT + 2] * 1e-3 * P.rho0d * P.u_ref / (0.5 * sqrt(P.rc2));
        v = fabs(((double)st[i].z + drho * dtc[P.case_id]) / P.rho0d);
        if (v != v) v = 1e300;
    }
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) tmax[tile] = v;
}

// Targets of case c, given in original order (n x 3, FP64), into its slots.
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_gnn_load_target(const KP<real>* __restrict__ Pt, int c,
                                                           const int32_t* __restrict__ id,
                                                           const double* __restrict__ src, float* __restrict__ Tg)
{
    const KP<real>& P = Pt[c];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.nf) return;
    const int i = P.fbase + k;
    const int o = id[i];
    for (int q = 0; q < NOUT; ++q) Tg[(size_t)i * NOUT + q] = (float)src[(size_t)o * NOUT + q];
}

}  // namespace gnn
}  // namespace sphx
