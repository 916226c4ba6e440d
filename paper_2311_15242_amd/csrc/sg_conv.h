// Matrix-core kernels of the learned surrogate: 3x3x3 "valid" convolutions over
// channels-last BF16 grids with FP32 accumulation (v_mfma_f32_32x32x16_bf16), their
// two gradients, the loss and the Adam update. A method addition: the paper has no
// surrogate; the network and its training are defined in the public header.
//
// Every layer is an implicit GEMM. Forward: rows = output nodes, columns = the 32
// (padded) output channels, reduction over 27 taps x input channels; on tiles one
// wavefront computes several 32 x 32 tiles with the layer's weights in LDS, on wide
// grids the weights stay in registers and the input marches through LDS by planes. Input gradient: rows =
// input nodes, columns = input channels, reduction over taps x output channels
// (the transposed weights). Weight gradient: one 32 x 32 tile (input x output
// channels) per tap, reduction over nodes in 256-node chunks staged in LDS
// transposed so every operand fragment is a 16-byte LDS read; partial tiles meet
// in FP32 atomics (the bias gradient rides along in the blocks of one tap).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfd {
namespace sg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

constexpr int NL = 4;                                  // layers
constexpr int CO = 32;                                 // padded output channels of every layer
constexpr int CIN_REAL[NL] = {6, 32, 32, 32};
constexpr int CIN_PAD[NL] = {16, 32, 32, 32};
constexpr int COUT_REAL[NL] = {32, 32, 32, 7};
constexpr int NOUT = 7;                                // network outputs: 3 + 3 flux coefficients, the exchange
constexpr int IN_CH = 16;                              // channels of an input grid (6 used)

__host__ __device__ constexpr long long layer_params(int l) { return 27LL * CIN_REAL[l] * COUT_REAL[l] + COUT_REAL[l]; }
__host__ __device__ constexpr long long n_params()
{
    return layer_params(0) + layer_params(1) + layer_params(2) + layer_params(3);
}

// Round to nearest even; NaN stays NaN.
__device__ __forceinline__ u16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 frag(const u16 *p) { return __builtin_bit_cast(bf16x8, *(const u32x4 *)p); }
__device__ __forceinline__ bf16x8 frag_zero() { return __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u}); }

// Row of the 32 x 32 result held by register r of a lane in lane group kg (the
// column is the lane index mod 32).
__device__ __forceinline__ int acc_row(int r, int kg) { return 8 * (r >> 2) + 4 * kg + (r & 3); }

// Output tiles of 32 nodes per wavefront in the forward layer.
#ifndef LBFD_SG_FWD_NT
#define LBFD_SG_FWD_NT 4
#endif
constexpr int FWD_NT = LBFD_SG_FWD_NT;
constexpr int FWD_NODES = 4 * 32 * FWD_NT;   // output nodes per workgroup

// Forward layer: out[m][o] = act(b[o] + sum_{tap,i} in[m + tap][i] w[tap][o][i]) over the
// M = B (Di-2)(Hi-2)(Wi-2) output nodes. wb: BF16 [27][32][CIN] (input channel fastest).
// out: BF16 [M][32], or with OUTF32 FP32 [M][NOUT] (the first NOUT channels, no activation).
// Each wavefront computes FWD_NT tiles of 32 nodes x 32 channels; every weight
// fragment read from LDS feeds FWD_NT matrix instructions.
template <int CIN, bool RELU, bool OUTF32>
__global__ __launch_bounds__(256) void k_conv_fwd(const u16 *__restrict__ in, const u16 *__restrict__ wb,
                                                 const float *__restrict__ bias, void *__restrict__ out, int Di,
                                                 int Hi, int Wi, long long M)
{
    constexpr int NT = FWD_NT;
    constexpr int LDW = CIN + 8;   // padded LDS row
    __shared__ __attribute__((aligned(16))) u16 sw[27 * CO * LDW];
    for (int i = threadIdx.x; i < 27 * CO * (CIN / 8); i += 256) {
        const int row = i / (CIN / 8), piece = i % (CIN / 8);
        *(u32x4 *)&sw[row * LDW + piece * 8] = *(const u32x4 *)&wb[row * CIN + piece * 8];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mr = lane & 31, kg = lane >> 5;
    const int Do = Di - 2, Ho = Hi - 2, Wo = Wi - 2;
    const long long m0 = ((long long)blockIdx.x * 4 + wave) * (32 * NT);
    const u16 *src[NT];
    bool ok[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const long long m = m0 + 32 * t + mr;
        ok[t] = m < M;
        long long r = ok[t] ? m : 0;
        const int x = (int)(r % Wo);
        r /= Wo;
        const int y = (int)(r % Ho);
        r /= Ho;
        const int z = (int)(r % Do);
        const long long b = r / Do;
        src[t] = in + (((b * Di + z) * Hi + y) * (long long)Wi + x) * CIN + kg * 8;
    }
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int tap = (a * 3 + p) * 3 + q;
                const long long toff = ((long long)(a * Hi + p) * Wi + q) * CIN;
#pragma unroll
                for (int c = 0; c < CIN / 16; ++c) {
                    const bf16x8 B = frag(&sw[(tap * CO + mr) * LDW + c * 16 + kg * 8]);
                    bf16x8 A[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t) A[t] = ok[t] ? frag(src[t] + toff + c * 16) : frag_zero();
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[t], B, acc[t], 0, 0, 0);
                }
            }
    const float bv = bias[mr];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const long long m = m0 + 32 * t + acc_row(r, kg);
            if (m >= M) continue;
            float v = acc[t][r] + bv;
            if constexpr (OUTF32) {
                if (mr < NOUT) ((float *)out)[m * NOUT + mr] = v;
            } else {
                if (RELU) v = fmaxf(v, 0.0f);
                ((u16 *)out)[m * CO + mr] = f2bf(v);
            }
        }
}

// The same layer on wide grids, marching along z. A workgroup owns columns of
// ZX x ZY output nodes (x, y) over zc consecutive output planes; wavefront w computes
// output row y0 + w. The layer's weight fragments stay in registers for the whole
// kernel (27 taps x CIN/16 fragments), so the only operand read per matrix
// instruction is the input fragment, from LDS. Input planes (ZY + 2 rows of 32 nodes)
// rotate through four LDS slots; each plane is fetched into registers two planes
// ahead of the one being computed. The three x-taps share one input fragment: for tap
// q the partial sums P_q[j] = sum in[x0 + j] w_q are kept per input node j of the
// row, and out[x0 + i] = P_0[i] + P_1[i + 1] + P_2[i + 2] (i < ZX = 30): the three
// partial tiles go to a per-wavefront LDS scratch, from which each lane reads 8
// consecutive channels of a node (16-byte stores, hardware BF16 conversion, round to
// nearest even). A persistent grid walks the columns.
constexpr int ZX = 30, ZY = 4;
template <int CIN, bool RELU, bool OUTF32>
__global__ __launch_bounds__(256) void k_conv_fwd_zm(const u16 *__restrict__ in, const u16 *__restrict__ wb,
                                                    const float *__restrict__ bias, void *__restrict__ out, int Di,
                                                    int Hi, int Wi, int nbx, int nby, int nbz, int zc, long long ncol)
{
    constexpr int CP = CIN + 8;                   // node stride in LDS (elements)
    constexpr int PR = ZY + 2;                    // input rows of a plane
    constexpr int PLANE = PR * 32 * CP;           // elements of a plane slot
    constexpr int NC = CIN / 16;                  // reduction fragments per tap
    constexpr int PCS = CIN / 8;                  // 16-byte pieces per node
    constexpr int PIECES = PR * 32 * PCS;         // 16-byte pieces per plane
    constexpr int PPT = (PIECES + 255) / 256;     // pieces per thread
    constexpr int SS = 36;                        // scratch row stride (floats; rows 16-byte aligned)
    __shared__ __attribute__((aligned(16))) u16 ring[4 * PLANE];
    __shared__ __attribute__((aligned(16))) float scr[4][3 * 32 * SS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mr = lane & 31, kg = lane >> 5;
    const int Do = Di - 2, Ho = Hi - 2, Wo = Wi - 2;
    // The last layer (NOUT = 7 outputs) takes 16 x 16 x 32 matrix instructions: 16
    // output columns instead of 32, half the matrix work; every other layer 32 x 32 x 16.
    constexpr bool N16 = OUTF32;
    constexpr int NCB = N16 ? CIN / 32 : NC;      // weight fragments per tap
    const int l16 = lane & 15, k16 = lane >> 4;
    bf16x8 Bw[27][NCB];
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
            Bw[t][c] = N16 ? frag(wb + (t * CO + l16) * CIN + c * 32 + k16 * 8)
                           : frag(wb + (t * CO + mr) * CIN + c * 16 + kg * 8);
    // the epilogue: lane l stores 8 channels (c8 = 8 (l mod 4)) of rows l / 4 and
    // l / 4 + 16, or (last layer) channels 4 (l mod 2) .. of row l / 2
    const int c8 = OUTF32 ? 4 * (lane & 1) : 8 * (lane & 3);
    float *const sw = scr[wave];
    const long long pstride = (long long)Hi * Wi * CIN;   // elements between input planes
    for (long long col = blockIdx.x; col < ncol; col += gridDim.x) {
        long long r = col;
        const int bxi = (int)(r % nbx);
        r /= nbx;
        const int byi = (int)(r % nby);
        r /= nby;
        const int bzi = (int)(r % nbz);
        const long long b = r / nbz;
        const int x0 = bxi * ZX, y0 = byi * ZY, z0 = bzi * zc;
        const int nzo = min(zc, Do - z0);
        // this thread's pieces of a plane: offset from the column's first input node in
        // plane z0 (-1 outside the grid: zeros, which only reach outputs that are not
        // stored) and place in a slot
        const u16 *cbase = in + (((b * Di + z0) * Hi + y0) * (long long)Wi + x0) * CIN;
        int off[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            const int piece = i % PCS, node = i / PCS;
            const bool ok = i < PIECES && x0 + (node & 31) < Wi && y0 + (node >> 5) < Hi;
            off[k] = ok ? ((node >> 5) * Wi + (node & 31)) * CIN + piece * 8 : -1;
        }
        const auto fetch = [&](int pz, u32x4 *v) {
            const bool inz = z0 + pz < Di;
            const u16 *pb = cbase + pz * pstride;
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                v[k] = off[k] >= 0 && inz ? *(const u32x4 *)(pb + off[k]) : u32x4{0u, 0u, 0u, 0u};
        };
        const auto put = [&](int slot, const u32x4 *v) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = (int)threadIdx.x + 256 * k;
                if (i < PIECES) *(u32x4 *)&ring[slot * PLANE + (i / PCS) * CP + (i % PCS) * 8] = v[k];
            }
        };
        // planes 0-2 in slots 0-2; plane 3 in flight in registers (it is stored at the
        // end of plane 0, plane 4 fetched meanwhile)
        u32x4 nx0[PPT], nx1[PPT];
        {
            u32x4 v0[PPT], v1[PPT], v2[PPT];
            fetch(0, v0);
            fetch(1, v1);
            fetch(2, v2);
            if (nzo > 1) fetch(3, nx0);
            put(0, v0);
            put(1, v1);
            put(2, v2);
        }
        __syncthreads();
        const int y = y0 + wave;
        const int lim = min(ZX, Wo - x0);   // output nodes of this row tile
        // output node x0 + i of this wavefront's row at plane z0 + iz is node
        // orow + iz oplane + i; a lane stores rows acc_row(e, kg) of channel mr
        const long long orow = ((b * Do + z0) * Ho + y) * (long long)Wo + x0;
        const long long oplane = (long long)Ho * Wo;
        // one output plane; cur holds plane iz + 3, nxt receives plane iz + 4 (the two
        // register sets swap roles every plane, so the loop below takes planes in pairs)
        const auto plane = [&](int iz, u32x4 *cur, u32x4 *nxt) __attribute__((always_inline)) {
            if (iz + 2 < nzo) fetch(iz + 4, nxt);
            if constexpr (N16) {
                // rows = 16 nodes (two halves of the row tile), k = 32 channels of one tap
                f32x4 acc[3][2];
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int h = 0; h < 2; ++h) acc[q][h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int g = 0; g < 9 * NCB; ++g) {
                    const int a = g / (3 * NCB), p = (g / NCB) % 3, c = g % NCB;
                    const u16 *base = ring + ((iz + a) & 3) * PLANE + ((wave + p) * 32 + l16) * CP + c * 32 + k16 * 8;
                    const bf16x8 A0 = frag(base), A1 = frag(base + 16 * CP);
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, Bw[(a * 3 + p) * 3 + q][c], acc[q][0],
                                                                            0, 0, 0);
                        acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, Bw[(a * 3 + p) * 3 + q][c], acc[q][1],
                                                                            0, 0, 0);
                    }
                }
                // lane l holds column l mod 16, rows 16 h + 4 (l / 16) + r
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int r = 0; r < 4; ++r) sw[(32 * q + 16 * h + 4 * k16 + r) * SS + l16] = acc[q][h][r];
            } else {
                f32x16 acc[3];
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[q][e] = 0.0f;
                // input fragment g = ((a 3 + p) NC + c); the next one is read while the
                // three matrix instructions of the current one run
                const auto afrag = [&](int g) __attribute__((always_inline)) {
                    const int a = g / (3 * NC), p = (g / NC) % 3, c = g % NC;
                    return frag(ring + ((iz + a) & 3) * PLANE + ((wave + p) * 32 + mr) * CP + c * 16 + kg * 8);
                };
                bf16x8 A = afrag(0);
#pragma unroll
                for (int g = 0; g < 9 * NC; ++g) {
                    const bf16x8 An = g + 1 < 9 * NC ? afrag(g + 1) : A;
                    const int ap = g / NC, c = g % NC;
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bw[ap * 3 + q][c], acc[q], 0, 0, 0);
                    A = An;
                }
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int j = acc_row(e, kg);
                    sw[j * SS + mr] = acc[0][e];
                    sw[(32 + j) * SS + mr] = acc[1][e];
                    sw[(64 + j) * SS + mr] = acc[2][e];
                }
            }
            if (iz + 1 < nzo) put((iz + 3) & 3, cur);
            __syncthreads();
            if (y >= Ho) return;
            const long long mrow = orow + iz * oplane;
            // P_0[i] + P_1[i + 1] + P_2[i + 2] + bias of 4 channels at c of row i
            const auto sum4 = [&](int i, int c, float *v) {
                const float4 a = *(const float4 *)&sw[i * SS + c];
                const float4 p = *(const float4 *)&sw[(33 + i) * SS + c];
                const float4 q = *(const float4 *)&sw[(66 + i) * SS + c];
                const float4 bz = *(const float4 *)&bias[c];
                v[0] = a.x + p.x + q.x + bz.x;
                v[1] = a.y + p.y + q.y + bz.y;
                v[2] = a.z + p.z + q.z + bz.z;
                v[3] = a.w + p.w + q.w + bz.w;
            };
            if constexpr (OUTF32) {
                const int i = lane >> 1;
                if (i < lim) {
                    float v[4];
                    sum4(i, c8, v);
                    float *o = (float *)out + (mrow + i) * NOUT + c8;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (c8 + k < NOUT) o[k] = v[k];
                }
            } else {
#pragma unroll
                for (int pass = 0; pass < 2; ++pass) {
                    const int i = (lane >> 2) + 16 * pass;
                    if (i >= lim) continue;
                    float v[8];
                    sum4(i, c8, v);
                    sum4(i, c8 + 4, v + 4);
                    bf16x2 h[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        float lo = v[2 * k], hi = v[2 * k + 1];
                        if (RELU) {
                            lo = fmaxf(lo, 0.0f);
                            hi = fmaxf(hi, 0.0f);
                        }
                        h[k] = bf16x2{(__bf16)lo, (__bf16)hi};
                    }
                    *(u32x4 *)&((u16 *)out)[(mrow + i) * CO + c8] =
                        u32x4{__builtin_bit_cast(uint32_t, h[0]), __builtin_bit_cast(uint32_t, h[1]),
                              __builtin_bit_cast(uint32_t, h[2]), __builtin_bit_cast(uint32_t, h[3])};
                }
            }
        };
        for (int iz = 0; iz < nzo; iz += 2) {
            plane(iz, nx0, nx1);
            if (iz + 1 < nzo) plane(iz + 1, nx1, nx0);
        }
        // every wavefront is past its last read of the slots before the next column fills them
        __syncthreads();
    }
}

// Input gradient of a layer with 32 input channels, with the ReLU of the layer below
// applied: dx[v][i] = [x[v][i] > 0] sum_{tap,o} dy[v - tap][o] w[tap][i][o], over the
// Mi = B Di Hi Wi input nodes. wt: BF16 [27][32 (i)][32 (o)] (output channel fastest).
// x: the layer's input (BF16 [Mi][32]); dy: BF16 [B][Di-2][Hi-2][Wi-2][32].
__global__ __launch_bounds__(256) void k_conv_dgrad(const u16 *__restrict__ dy, const u16 *__restrict__ wt,
                                                   const u16 *__restrict__ x, u16 *__restrict__ dx, int Di, int Hi,
                                                   int Wi, long long Mi)
{
    constexpr int LDW = CO + 8;
    __shared__ __attribute__((aligned(16))) u16 sw[27 * CO * LDW];
    for (int i = threadIdx.x; i < 27 * CO * (CO / 8); i += 256) {
        const int row = i / (CO / 8), piece = i % (CO / 8);
        *(u32x4 *)&sw[row * LDW + piece * 8] = *(const u32x4 *)&wt[row * CO + piece * 8];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mr = lane & 31, kg = lane >> 5;
    const int Do = Di - 2, Ho = Hi - 2, Wo = Wi - 2;
    const long long m0 = ((long long)blockIdx.x * 4 + wave) * 64;
    int xx[2], yy[2], zz[2];
    long long bb[2];
    bool ok[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const long long m = m0 + 32 * t + mr;
        ok[t] = m < Mi;
        long long r = ok[t] ? m : 0;
        xx[t] = (int)(r % Wi);
        r /= Wi;
        yy[t] = (int)(r % Hi);
        r /= Hi;
        zz[t] = (int)(r % Di);
        bb[t] = r / Di;
    }
    f32x16 acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int tap = (a * 3 + p) * 3 + q;
                long long src[2];
                bool in_range[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int z = zz[t] - a, y = yy[t] - p, x = xx[t] - q;
                    in_range[t] = ok[t] && z >= 0 && z < Do && y >= 0 && y < Ho && x >= 0 && x < Wo;
                    src[t] = in_range[t] ? ((((bb[t] * Do + z) * Ho + y) * (long long)Wo + x) * CO + kg * 8) : 0;
                }
#pragma unroll
                for (int c = 0; c < CO / 16; ++c) {
                    const bf16x8 B = frag(&sw[(tap * CO + mr) * LDW + c * 16 + kg * 8]);
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const bf16x8 A = in_range[t] ? frag(dy + src[t] + c * 16) : frag_zero();
                        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[t], 0, 0, 0);
                    }
                }
            }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const long long m = m0 + 32 * t + acc_row(r, kg);
            if (m >= Mi) continue;
            const u16 xv = x[m * CO + mr];
            const bool active = (xv & 0x8000u) == 0 && xv != 0;   // x > 0 (x is a ReLU output)
            dx[m * CO + mr] = active ? f2bf(acc[t][r]) : (u16)0;
        }
}

// Weight gradient of a layer: dw[tap][i][o] += sum_v x[v + tap][i] dy[v][o] over the
// output nodes [v0, v1) of this block's split; grid (27 taps, splits). x: BF16 layer
// input [B][Di][Hi][Wi][CIN]; dy: BF16 [M][32]; dw: FP32 [27][CIN][32]. The blocks of
// tap 0 also add the bias gradient db[o] += sum_v dy[v][o]. Each stage stages 256
// output nodes (input and output gradient transposed to [channel][node] in LDS, so
// every operand fragment is a 16-byte LDS read); each wavefront reduces over 64 of
// them in four matrix instructions; partial tiles meet in FP32 atomics.
template <int CIN>
__global__ __launch_bounds__(256) void k_conv_wgrad(const u16 *__restrict__ x, const u16 *__restrict__ dy,
                                                   float *__restrict__ dw, float *__restrict__ db, int Di, int Hi,
                                                   int Wi, long long M, long long per_split)
{
    constexpr int CH = 256;                 // output nodes per stage
    constexpr int LDV = CH + 8;
    __shared__ __attribute__((aligned(16))) u16 xs[32 * LDV];   // [channel][node]
    __shared__ __attribute__((aligned(16))) u16 ds[32 * LDV];
    __shared__ float red[3][16][64];
    __shared__ float bred[8][32];
    const int tap = blockIdx.x;
    const int a = tap / 9, p = (tap / 3) % 3, q = tap % 3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mr = lane & 31, kg = lane >> 5;
    const uint32_t Do = Di - 2, Ho = Hi - 2, Wo = Wi - 2;
    const long long v_begin = (long long)blockIdx.y * per_split;
    long long v_end = v_begin + per_split;
    if (v_end > M) v_end = M;
    if (CIN < 32)
        for (int i = threadIdx.x; i < (32 - CIN) * LDV; i += 256) xs[CIN * LDV + i] = 0;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    float bsum = 0.0f;                      // tap 0: channel t mod 32 over nodes t/32, t/32 + 8, ...
    const int j = threadIdx.x;              // staging: node j of the stage, every channel
    for (long long v0 = v_begin; v0 < v_end; v0 += CH) {
        const long long m = v0 + j;
        const bool ok = m < v_end;
        u32x4 xv[CIN / 8], dv[4];
#pragma unroll
        for (int k = 0; k < CIN / 8; ++k) xv[k] = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int k = 0; k < 4; ++k) dv[k] = u32x4{0u, 0u, 0u, 0u};
        if (ok) {
            uint32_t r = (uint32_t)m;       // the host keeps M below 2^31
            const uint32_t xo = r % Wo;
            r /= Wo;
            const uint32_t yo = r % Ho;
            r /= Ho;
            const uint32_t zo = r % Do;
            const uint32_t b = r / Do;
            const long long src = ((((long long)b * Di + zo + a) * Hi + yo + p) * (long long)Wi + xo + q) * CIN;
#pragma unroll
            for (int k = 0; k < CIN / 8; ++k) xv[k] = *(const u32x4 *)&x[src + k * 8];
#pragma unroll
            for (int k = 0; k < 4; ++k) dv[k] = *(const u32x4 *)&dy[m * CO + k * 8];
        }
#pragma unroll
        for (int k = 0; k < CIN / 8; ++k) {
            const u16 *xe = (const u16 *)&xv[k];
#pragma unroll
            for (int e = 0; e < 8; ++e) xs[(k * 8 + e) * LDV + j] = xe[e];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u16 *de = (const u16 *)&dv[k];
#pragma unroll
            for (int e = 0; e < 8; ++e) ds[(k * 8 + e) * LDV + j] = de[e];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int col = 64 * wave + 16 * kk + 8 * kg;
            const bf16x8 A = frag(&xs[mr * LDV + col]);
            const bf16x8 B = frag(&ds[mr * LDV + col]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc, 0, 0, 0);
        }
        if (tap == 0) {
            const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
#pragma unroll 8
            for (int n = g; n < CH; n += 8) bsum += bf2f(ds[c * LDV + n]);
        }
        __syncthreads();
    }
    if (wave > 0)
#pragma unroll
        for (int r = 0; r < 16; ++r) red[wave - 1][r][lane] = acc[r];
    if (tap == 0) bred[threadIdx.x >> 5][threadIdx.x & 31] = bsum;
    __syncthreads();
    if (wave == 0)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float s = acc[r] + red[0][r][lane] + red[1][r][lane] + red[2][r][lane];
            const int i = acc_row(r, kg);
            if (i < CIN && s != 0.0f) atomicAdd(&dw[((long long)tap * CIN + i) * CO + mr], s);
        }
    if (tap == 0 && threadIdx.x < 32) {
        float t = 0.0f;
#pragma unroll
        for (int g = 0; g < 8; ++g) t += bred[g][threadIdx.x];
        if (t != 0.0f) atomicAdd(&db[threadIdx.x], t);
    }
}

// Conservative form of the output (the network's 7 channels per node n of a T^3
// tile: flux coefficients f_psi,a, f_phi,a, a = x, y, z, and the exchange s):
//   A_psi[n] = W[n] s[n] - sum_a (Wf_a[n] f_psi,a[n] - Wf_a[n - e_a] f_psi,a[n - e_a])
//   A_phi[n] = -ratio W[n] s[n] - sum_a (Xf_a[n] f_phi,a[n] - Xf_a[n - e_a] f_phi,a[n - e_a])
// with face weights Wf_a[n] = (W[n] + W[n + e_a])/2 (the same for X), on the
// interior nodes [1, T - 2]^3. t holds per node (W dpsi / dpsi_s, X dphi / dphi_s, W, X).
__device__ __forceinline__ void cons_changes(const float *o, const float *t, int T, long long base, int i, int j,
                                             int l, float ratio, float &Ap, float &Af)
{
    const long long n = base + ((long long)l * T + j) * T + i;
    const long long st[3] = {1, T, (long long)T * T};
    const float Wn = t[4 * n + 2], Xn = t[4 * n + 3];
    Ap = Wn * o[NOUT * n + 6];
    Af = -ratio * Wn * o[NOUT * n + 6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long u = n + st[a], d = n - st[a];
        Ap -= 0.5f * (Wn + t[4 * u + 2]) * o[NOUT * n + a];
        Ap += 0.5f * (t[4 * d + 2] + Wn) * o[NOUT * d + a];
        Af -= 0.5f * (Xn + t[4 * u + 3]) * o[NOUT * n + 3 + a];
        Af += 0.5f * (t[4 * d + 3] + Xn) * o[NOUT * d + 3 + a];
    }
}

// Loss of B tiles of T^3 output nodes: squared error of the conservative form
// against the targets, summed into *acc (FP64), and the output gradient dy (BF16
// [M][32], channels NOUT.. zero) of scale/2 times that sum: per node the adjoint
// of the form above, from the residuals g = scale (A - target) of the node and of
// its upper neighbours.
__global__ __launch_bounds__(256) void k_cons_loss(const float *__restrict__ o, const float *__restrict__ t, int T,
                                                  long long M, float ratio, float scale, double *__restrict__ acc,
                                                  u16 *__restrict__ dy)
{
    __shared__ double sh[256];
    double s = 0.0;
    const long long TT = (long long)T * T * T;
    for (long long m = (long long)blockIdx.x * 256 + threadIdx.x; m < M; m += (long long)gridDim.x * 256) {
        const long long b = m / TT, r = m - b * TT, base = b * TT;
        const int i = (int)(r % T), j = (int)((r / T) % T), l = (int)(r / ((long long)T * T));
        const auto inner = [&](int ii, int jj, int ll) {
            return ii >= 1 && jj >= 1 && ll >= 1 && ii <= T - 2 && jj <= T - 2 && ll <= T - 2;
        };
        // residuals at the node (gp0, gf0) and at its upper neighbours along x, y, z
        float gp[4] = {0, 0, 0, 0}, gf[4] = {0, 0, 0, 0};
        const int ci[4] = {i, i + 1, i, i}, cj[4] = {j, j, j + 1, j}, cl[4] = {l, l, l, l + 1};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!inner(ci[c], cj[c], cl[c])) continue;
            float Ap, Af;
            cons_changes(o, t, T, base, ci[c], cj[c], cl[c], ratio, Ap, Af);
            const long long nc = base + ((long long)cl[c] * T + cj[c]) * T + ci[c];
            const float rp = Ap - t[4 * nc], rf = Af - t[4 * nc + 1];
            if (c == 0) s += (double)rp * rp + (double)rf * rf;
            gp[c] = scale * rp;
            gf[c] = scale * rf;
        }
        const long long n = base + r;
        const float Wn = t[4 * n + 2], Xn = t[4 * n + 3];
        float d[8];
        const long long st[3] = {1, T, (long long)T * T};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // face between n and n + e_a: out of n (g at n), into n + e_a (g there)
            const bool up_in = (a == 0 ? i : a == 1 ? j : l) + 1 <= T - 1;
            const float Wf = up_in ? 0.5f * (Wn + t[4 * (n + st[a]) + 2]) : 0.0f;
            const float Xf = up_in ? 0.5f * (Xn + t[4 * (n + st[a]) + 3]) : 0.0f;
            d[a] = Wf * (gp[1 + a] - gp[0]);
            d[3 + a] = Xf * (gf[1 + a] - gf[0]);
        }
        d[6] = Wn * (gp[0] - ratio * gf[0]);
        d[7] = 0.0f;
        u32x4 head = {(uint32_t)f2bf(d[0]) | ((uint32_t)f2bf(d[1]) << 16),
                      (uint32_t)f2bf(d[2]) | ((uint32_t)f2bf(d[3]) << 16),
                      (uint32_t)f2bf(d[4]) | ((uint32_t)f2bf(d[5]) << 16), (uint32_t)f2bf(d[6])};
        u32x4 zero = {0u, 0u, 0u, 0u};
        u32x4 *dd = (u32x4 *)&dy[m * CO];
        dd[0] = head;
        dd[1] = zero;
        dd[2] = zero;
        dd[3] = zero;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(acc, sh[0]);
}

// Device views of the parameters. Master weights in parameter order; gradients and
// the BF16 copies in the padded layouts of the kernels above.
struct Net {
    float *master, *m, *v;      // FP32 [n_params]
    float *gw[NL];              // FP32 [27][CIN_PAD][32] weight gradients
    float *gb[NL];              // FP32 [32] bias gradients
    u16 *wb[NL];                // BF16 [27][32][CIN_PAD] forward weights
    u16 *wt[NL];                // BF16 [27][CIN_PAD][32] transposed weights
    float *bias[NL];            // FP32 [32]
};

// Where parameter index k lives: layer, and either (tap, i, o) of a weight or o of a bias.
__device__ __forceinline__ void param_site(long long k, int &l, int &tap, int &i, int &o, bool &is_bias)
{
    l = 0;
    while (l < NL - 1 && k >= layer_params(l)) k -= layer_params(l++);
    const long long nw = 27LL * CIN_REAL[l] * COUT_REAL[l];
    is_bias = k >= nw;
    if (is_bias) {
        o = (int)(k - nw);
        tap = i = 0;
    } else {
        o = (int)(k % COUT_REAL[l]);
        const long long r = k / COUT_REAL[l];
        i = (int)(r % CIN_REAL[l]);
        tap = (int)(r / CIN_REAL[l]);
    }
}

// Adam step (adam != 0, t = step count after this step) or a plain copy of the master
// weights (adam == 0), then the BF16 copies and FP32 biases the kernels read.
__global__ __launch_bounds__(256) void k_adam_pack(Net net, int adam, float lr, float b1, float b2, float eps,
                                                  float c1, float c2)
{
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= n_params()) return;
    int l, tap, i, o;
    bool is_bias;
    param_site(k, l, tap, i, o, is_bias);
    float w = net.master[k];
    if (adam) {
        const float g = is_bias ? net.gb[l][o] : net.gw[l][((long long)tap * CIN_PAD[l] + i) * CO + o];
        const float m = b1 * net.m[k] + (1.0f - b1) * g;
        const float v = b2 * net.v[k] + (1.0f - b2) * g * g;
        net.m[k] = m;
        net.v[k] = v;
        w -= lr * (m / c1) / (sqrtf(v / c2) + eps);
        net.master[k] = w;
    }
    if (is_bias) {
        net.bias[l][o] = w;
    } else {
        const u16 h = f2bf(w);
        net.wb[l][((long long)tap * CO + o) * CIN_PAD[l] + i] = h;
        net.wt[l][((long long)tap * CIN_PAD[l] + i) * CO + o] = h;
    }
}

// Gradients in parameter order (for export).
__global__ __launch_bounds__(256) void k_grad_flat(Net net, float *out)
{
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= n_params()) return;
    int l, tap, i, o;
    bool is_bias;
    param_site(k, l, tap, i, o, is_bias);
    out[k] = is_bias ? net.gb[l][o] : net.gw[l][((long long)tap * CIN_PAD[l] + i) * CO + o];
}

}  // namespace sg
}  // namespace lbfd
