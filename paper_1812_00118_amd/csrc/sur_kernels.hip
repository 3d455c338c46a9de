// HIP kernels of the convolutional surrogate (gfx950, BF16 MFMA, FP32 accumulation).
//
// Activations are NHWC BF16; gradients FP32.  A 3x3 convolution with circular padding
//   out[p, o] = b[o] + sum_{tap, c} in[p + off(tap), c] w[o, tap, c],  off(tap) = (tap/3 - 1,
//   tap%3 - 1) in (y, x), is an implicit GEMM with M = pixels, N = Cout, K = 9 Cin; the
// K index runs over (tap, channel group of 8).  The same kernel computes the input
// gradient with the weights transposed and the taps mirrored.  The weight gradient is a
// GEMM over pixels (K = B H W) with the tiles transposed through LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sur_internal.hpp"

namespace pfsur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// SiLU z sigmoid(z) and its derivative.  The sigmoid's reciprocal is the hardware
// v_rcp_f32 (1 ulp): the results are rounded to BF16 (or feed BF16 products) anyway, and
// an IEEE division would cost three times the instructions of the whole activation.
__device__ __forceinline__ float sigmoid(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// 8 consecutive input channels at output-resolution pixel (b, y, x), through the layer's
// input mode (same resolution, 2x nearest upsampling, or 2x2 average pooling).  M is the
// mode when the caller fixes it at compile time, -1 to take g.mode.  Pixel indices fit
// 32 bits (at most 2^28 input pixels).
template <int M>
__device__ __forceinline__ bf16x8 gather8(const GatherP& g, int b, int y, int x, int c) {
    const int mode = M >= 0 ? M : g.mode;
    if (mode == MODE_UP) {
        y >>= 1;
        x >>= 1;
    }
    const int cc = g.c0 + c;
    if (mode != MODE_POOL) {
        const uint32_t pix = ((uint32_t)b * (uint32_t)g.Hin + (uint32_t)y) * (uint32_t)g.Win + (uint32_t)x;
        return *reinterpret_cast<const bf16x8*>(g.p + (size_t)pix * g.cs + cc);
    }
    const uint32_t pix =
        ((uint32_t)b * (uint32_t)g.Hin + 2u * (uint32_t)y) * (uint32_t)g.Win + 2u * (uint32_t)x;
    const __bf16* q = g.p + (size_t)pix * g.cs + cc;
    const size_t row = (size_t)g.Win * g.cs;
    const bf16x8 v0 = *reinterpret_cast<const bf16x8*>(q);
    const bf16x8 v1 = *reinterpret_cast<const bf16x8*>(q + g.cs);
    const bf16x8 v2 = *reinterpret_cast<const bf16x8*>(q + row);
    const bf16x8 v3 = *reinterpret_cast<const bf16x8*>(q + row + g.cs);
    bf16x8 r;
    for (int k = 0; k < 8; ++k)
        r[k] = (__bf16)(0.25f * ((((float)v0[k] + (float)v1[k]) + (float)v2[k]) + (float)v3[k]));
    return r;
}

// ---------------------------------------------------------------------------
// Implicit-GEMM 3x3 convolution.  A workgroup of 4 waves covers 256 output pixels x 32
// output channels; a wave covers 64 pixels (4 MFMA row blocks) x 32 channels (2 column
// blocks) with v_mfma_f32_16x16x32_bf16, whose lane l holds A row l%16 / B column l%16
// with K elements 8(l/16)..8(l/16)+7, and C rows 4(l/16)..+3 of column l%16.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_conv3x3(ConvP a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    const int P = a.B * a.H * a.W;
    const int p0 = blockIdx.x * 256 + wave * 64;
    const int co0 = blockIdx.y * 32;
    const int cg_per_tap = a.g.C >> 3;               // channel groups of 8 per tap
    const int nkg = 9 * cg_per_tap;
    // this lane's pixel in each of the 4 row blocks
    int pb[4], py[4], px[4];
    bool pv[4];
    for (int mb = 0; mb < 4; ++mb) {
        const int p = p0 + mb * 16 + r16;
        pv[mb] = p < P;
        const int pp = pv[mb] ? p : 0;
        px[mb] = pp % a.W;
        py[mb] = (pp / a.W) % a.H;
        pb[mb] = pp / (a.W * a.H);
    }
    f32x4 acc[4][2];
    for (int mb = 0; mb < 4; ++mb)
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = (bf16x8){0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; 4 * s < nkg; ++s) {
        const int kg = 4 * s + q;
        const bool kv = kg < nkg;
        const int tap = kv ? kg / cg_per_tap : 0;
        const int cg = kv ? kg - tap * cg_per_tap : 0;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        bf16x8 A[4], Bm[2];
        for (int mb = 0; mb < 4; ++mb)
            A[mb] = (kv && pv[mb]) ? gather8<-1>(a.g, pb[mb], wrap(py[mb] + dy, a.H), wrap(px[mb] + dx, a.W), cg * 8)
                                   : zero8;
        for (int nb = 0; nb < 2; ++nb) {
            const int co = co0 + nb * 16 + r16;
            Bm[nb] = (kv && co < a.Cout)
                         ? *reinterpret_cast<const bf16x8*>(a.w + (size_t)co * 9 * a.g.C + (size_t)kg * 8)
                         : zero8;
        }
        for (int mb = 0; mb < 4; ++mb)
            for (int nb = 0; nb < 2; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mb], Bm[nb], acc[mb][nb], 0, 0, 0);
    }
    // epilogue
    for (int nb = 0; nb < 2; ++nb) {
        const int co = co0 + nb * 16 + r16;
        if (co >= a.Cout) continue;
        const float bias = a.bias ? a.bias[co] : 0.0f;
        for (int mb = 0; mb < 4; ++mb)
            for (int j = 0; j < 4; ++j) {
                const int p = p0 + mb * 16 + 4 * q + j;
                if (p >= P) continue;
                const float v = acc[mb][nb][j] + bias;
                if (a.zout) a.zout[(size_t)p * a.Cout + co] = (__bf16)v;
                if (a.out)
                    a.out[(size_t)p * a.out_cs + a.out_c0 + co] = (__bf16)(a.act ? silu(v) : v);
                if (a.fout) {
                    float* f = a.fout + (size_t)p * a.f_cs + a.f_c0 + co;
                    *f = a.f_accum ? *f + v : v;
                }
            }
    }
}

// ---------------------------------------------------------------------------
// Implicit-GEMM 3x3 convolution staged through LDS, for C and Cout multiples of 32.
// A workgroup (4 waves) computes a 16x16 patch of output pixels of one image x NT
// output channels.  The input channels are processed in chunks of 32: the chunk's
// 18x18 halo patch (wrap, pooling or upsampling applied while loading) and its
// NT x 9 x 32 weights are staged in LDS, and the loads of the next chunk are issued
// into registers before the current chunk is computed.  Wave w owns patch rows
// 4w..4w+3 as two 32-pixel blocks; v_mfma_f32_32x32x16_bf16 takes the weights as A
// (lane l: row l%32 = output channel, K elements 8(l/32)..+7) and the pixels as B
// (column l%32 = pixel, same K), so D[channel][pixel] has lane l on pixel l%32 with
// channels 8(j/4) + 4(l/32) + j%4.  Row strides are padded (40 and 296 BF16) so that 16
// consecutive lanes reading 16 bytes hit distinct banks.
// ---------------------------------------------------------------------------
constexpr int TP = 16;                 // output patch edge
constexpr int HP = TP + 2;             // halo patch edge
constexpr int APAD = 40;               // BF16 per staged pixel (32 channels + pad)
constexpr int BPAD = 9 * 32 + 8;       // BF16 per staged output channel
// Row pitch of the staged halo patch: HP pixels of APAD BF16 plus RPAD BF16, so that a
// row is 112 16-byte units (16 mod 32).  The 32 lanes of a B-operand read cover two patch
// rows of 16 pixels, and gfx950's LDS serves such a 16-byte read in 512-byte groups of
// 32 lanes: with rows HP * APAD apart, two lanes 14 pixels apart in the two rows meet in
// one bank (measured: 1/6 of the LDS cycles of a probe in this pattern were conflict
// stalls, for every APAD); with the pitch at 16 mod 32 units the second row's 16 units
// are exactly the ones the first row leaves free.
constexpr int RPAD = 176;
constexpr int ROWA = HP * APAD + RPAD; // BF16 per staged patch row
constexpr int A_ITEMS = HP * HP * 4;   // 16-byte items of the halo patch
constexpr int A_PER_T = (A_ITEMS + 255) / 256;

// Epilogues of a 16x16-pixel tile.  The MFMAs compute D[channel][pixel] (weights as the
// A operand), so lane l holds pixel l%32 of its 32-pixel row block and, for j = 0..15,
// channel 8(j/4) + 4(l/32) + j%4 of the 32-channel block.
//
// Direct: each lane writes its runs of 4 consecutive channels as one 8-byte (BF16) or
// 16-byte (FP32) store.  Used for 32-channel tiles, where it measured as fast as the
// staged form without its extra barrier.
template <int NB>
__device__ __forceinline__ void tile_epilogue_direct(const ConvP& a, const f32x16 (&acc)[2][NB],
                                                     int b, int y0, int x0, int co0, int wave,
                                                     int l32, int g) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const int y = y0 + 4 * wave + 2 * mb + (l32 >> 4), x = x0 + (l32 & 15);
        if (y >= a.H || x >= a.W) continue;
        const size_t p = ((size_t)b * a.H + y) * a.W + x;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int co = co0 + nb * 32 + 8 * q + 4 * g;   // first of 4 channels
                if (co >= a.Cout) continue;
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    v[e] = acc[mb][nb][4 * q + e] + (a.bias ? a.bias[co + e] : 0.0f);
                if (a.zout) {
                    bf16x4 z;
#pragma unroll
                    for (int e = 0; e < 4; ++e) z[e] = (__bf16)v[e];
                    *reinterpret_cast<bf16x4*>(a.zout + p * a.Cout + co) = z;
                }
                if (a.out) {
                    bf16x4 o;
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[e] = (__bf16)(a.act ? silu(v[e]) : v[e]);
                    *reinterpret_cast<bf16x4*>(a.out + p * a.out_cs + a.out_c0 + co) = o;
                }
                if (a.fout) {
                    float4* f = reinterpret_cast<float4*>(a.fout + p * a.f_cs + a.f_c0 + co);
                    float4 w = make_float4(v[0], v[1], v[2], v[3]);
                    if (a.f_accum) {
                        const float4 o = *f;
                        w.x += o.x; w.y += o.y; w.z += o.z; w.w += o.w;
                    }
                    *f = w;
                }
            }
    }
}

// Staged (64-channel tiles, 8-12% faster there): the BF16 outputs go through LDS, one
// 32-channel block at a time, in the wave's own region of OROW BF16 per pixel (sO: 64
// OROW per wave): each lane writes its 4-channel runs, then reads back 16 bytes (8
// channels) of one pixel so that four consecutive lanes store one pixel's 64 contiguous
// bytes and a store instruction covers 16 pixels instead of 64 scattered 8-byte pieces.
// The FP32 output (input gradients) keeps direct 16-byte stores.  With pout set, the
// staged activations also give their 2x2 averages (the input of the next level's pooling
// layer), so that layer reads a compact quarter-size tensor at its own resolution.
constexpr int OROW = 40;   // BF16 per staged pixel: 32 channels + pad

// LDS accesses of one wave complete in order; the wait and the clobber keep the
// compiler from moving the read-back across the writes (and the next writes across it)
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <int NB>
__device__ __forceinline__ void tile_epilogue_staged(const ConvP& a, const f32x16 (&acc)[2][NB],
                                                     int b, int y0, int x0, int co0, int wave,
                                                     int l32, int g, __bf16* __restrict__ sO) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const int lane = l32 + 32 * g;
    __bf16* so = sO + wave * 64 * OROW;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int cb = co0 + nb * 32;            // first channel of the block
        if (cb >= a.Cout) break;
        // value of channel run q (4 channels), element e, row block mb
        auto val = [&](int mb, int q, int e) {
            return acc[mb][nb][4 * q + e] + (a.bias ? a.bias[cb + 8 * q + 4 * g + e] : 0.0f);
        };
        if (a.fout) {
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int y = y0 + 4 * wave + 2 * mb + (l32 >> 4), x = x0 + (l32 & 15);
                if (y >= a.H || x >= a.W) continue;
                const size_t p = ((size_t)b * a.H + y) * a.W + x;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float4* f = reinterpret_cast<float4*>(a.fout + p * a.f_cs + a.f_c0 + cb +
                                                          8 * q + 4 * g);
                    float4 w = make_float4(val(mb, q, 0), val(mb, q, 1), val(mb, q, 2),
                                           val(mb, q, 3));
                    if (a.f_accum) {
                        const float4 o = *f;
                        w.x += o.x; w.y += o.y; w.z += o.z; w.w += o.w;
                    }
                    *f = w;
                }
            }
        }
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            __bf16* dst = pass == 0 ? a.zout : a.out;
            if (!dst) continue;
            const int cs = pass == 0 ? a.Cout : a.out_cs;
            const int c0 = pass == 0 ? 0 : a.out_c0;
            const bool act = pass == 1 && a.act;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bf16x4 o;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float t = val(mb, q, e);
                        o[e] = (__bf16)(act ? silu(t) : t);
                    }
                    *reinterpret_cast<bf16x4*>(&so[(mb * 32 + l32) * OROW + 8 * q + 4 * g]) = o;
                }
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = lane + 64 * k;                 // 16-byte item: pixel i/4
                const int px = i >> 2, grp = i & 3;
                const int mb = px >> 5, pl = px & 31;
                const int y = y0 + 4 * wave + 2 * mb + (pl >> 4), x = x0 + (pl & 15);
                const bf16x8 val = *reinterpret_cast<const bf16x8*>(&so[px * OROW + 8 * grp]);
                if (y < a.H && x < a.W) {
                    const size_t p = ((size_t)b * a.H + y) * a.W + x;
                    *reinterpret_cast<bf16x8*>(dst + p * cs + c0 + cb + 8 * grp) = val;
                }
            }
            if (pass == 1 && a.pout) {
                // 2x2 average of the stored activations for the next level's pooling
                // layer, added in the pooling gather's order: (y, x), (y, x+1), (y+1, x),
                // (y+1, x+1).  The wave's 4 x 16 pixels give 2 x 8 pooled pixels x 4
                // groups of 8 channels: one item per lane.
                const int pp = lane >> 2, grp = lane & 3;
                const int mb = pp >> 3, pc = pp & 7;
                const int base = mb * 32 + 2 * pc;               // staged pixel (y, x)
                const bf16x8 v00 = *reinterpret_cast<const bf16x8*>(&so[base * OROW + 8 * grp]);
                const bf16x8 v01 = *reinterpret_cast<const bf16x8*>(&so[(base + 1) * OROW + 8 * grp]);
                const bf16x8 v10 = *reinterpret_cast<const bf16x8*>(&so[(base + 16) * OROW + 8 * grp]);
                const bf16x8 v11 = *reinterpret_cast<const bf16x8*>(&so[(base + 17) * OROW + 8 * grp]);
                bf16x8 r;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    r[e] = (__bf16)(0.25f * ((((float)v00[e] + (float)v01[e]) + (float)v10[e]) +
                                             (float)v11[e]));
                const int y = y0 + 4 * wave + 2 * mb, x = x0 + 2 * pc;
                if (y + 1 < a.H && x + 1 < a.W) {
                    const size_t q = ((size_t)b * (a.H >> 1) + (y >> 1)) * (a.W >> 1) + (x >> 1);
                    *reinterpret_cast<bf16x8*>(a.pout + q * a.pout_cs + cb + 8 * grp) = r;
                }
            }
            wave_lds_sync();
        }
    }
}

// Partial sums of the 1x1 head over the 16 channels 8q + 4g + e (q, e = 0..3) of one
// pixel, in that order.  A head output is (half(g = 0) + half(g = 1)) + b: the order
// head_fwd uses and the one the fused epilogue gets, where lanes l and l + 32 of a wave
// hold the two halves of a pixel's 32 channels.
__device__ __forceinline__ void head_half(const float (&v)[16], int g, const float* wh,
                                          float (&p)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                p[k] = fmaf(v[4 * q + e], wh[k * 32 + 8 * q + 4 * g + e], p[k]);
}

// Epilogue of the last 32-channel layer at inference: its activations (rounded to BF16,
// as they would be stored) go straight into the 1x1 head; the layer's activation tensor
// is never written.  sH holds the head's weights and biases.
__device__ __forceinline__ void tile_epilogue_head(const ConvP& a, const f32x16 (&acc)[2][1],
                                                   int b, int y0, int x0, int wave, int l32,
                                                   int g, const float* sH) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const int y = y0 + 4 * wave + 2 * mb + (l32 >> 4), x = x0 + (l32 & 15);
        float v[16];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = 8 * q + 4 * g + e;
                const float t = acc[mb][0][4 * q + e] + (a.bias ? a.bias[co] : 0.0f);
                v[4 * q + e] = (float)(__bf16)(a.act ? silu(t) : t);
            }
        float p[4], o[4];
        head_half(v, g, sH, p);
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = __shfl_xor(p[k], 32);
        if (g == 0 && y < a.H && x < a.W) {
            const size_t px = ((size_t)b * a.H + y) * a.W + x;
            reinterpret_cast<float4*>(a.head_out)[px] =
                make_float4((p[0] + o[0]) + sH[128], (p[1] + o[1]) + sH[129],
                            (p[2] + o[2]) + sH[130], (p[3] + o[3]) + sH[131]);
        }
    }
}

// 32-channel tiles use 50 KB of LDS, so three workgroups fit a CU (160 KB) when the
// registers allow it; 64-channel tiles (69 KB) fit two, and so does the fused-head variant, whose
// head arithmetic needs the registers of two workgroups per CU.
// Epilogue variants: staged (always for 64-channel tiles; for 32-channel tiles only when
// the layer also writes pooled output), direct, or the fused 1x1 head.
enum { EPI_DIRECT = 0, EPI_STAGED = 1, EPI_HEAD = 2 };
template <int NT, int MODE, int EPI>
__global__ void __launch_bounds__(256, (NT == 32 && EPI != EPI_HEAD) ? 3 : 2)
k_conv_tiled(ConvP a, int tiles_per_wg) {
    constexpr int B_ITEMS = NT * 36;             // 16-byte items of the weight tile
    constexpr int B_PER_T = (B_ITEMS + 255) / 256;
    constexpr int NB = NT / 32;
    __shared__ __align__(16) __bf16 sA[HP * ROWA];
    __shared__ __align__(16) __bf16 sB[NT * BPAD];
    static_assert(4 * 64 * OROW <= HP * ROWA, "epilogue staging must fit the patch buffer");
    static_assert((ROWA * 2 / 16) % 32 == 16, "patch rows 16 mod 32 16-byte units apart");
    static_assert(EPI != EPI_HEAD || (NT == 32 && MODE == MODE_SAME), "head fusion: 32 channels");
    __shared__ float sH[EPI == EPI_HEAD ? 4 * 32 + 4 : 1];
    if constexpr (EPI == EPI_HEAD) {   // ordered before use by the first tile's barriers
        for (int i = threadIdx.x; i < 4 * 32 + 4; i += 256)
            sH[i] = i < 128 ? a.head_w[i] : a.head_b[i - 128];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l32 = lane & 31, g = lane >> 5;
    const int tx_n = (a.W + TP - 1) / TP, ty_n = (a.H + TP - 1) / TP;
    const int ntile = a.B * tx_n * ty_n;
    const int t_beg = blockIdx.x * tiles_per_wg;
    const int t_end = min(ntile, t_beg + tiles_per_wg);
    const int co0 = blockIdx.y * NT;
    const int C = a.g.C;
    const int nchunk = C / 32;
    // the (tile, chunk) pairs of this workgroup, in order; with one chunk the weights
    // are staged once
    const int niter = (t_end - t_beg) * nchunk;
    const bf16x8 zero8 = (bf16x8){0, 0, 0, 0, 0, 0, 0, 0};

    auto tile_xy = [&](int t, int& b, int& y0, int& x0) {
        const int tx = t % tx_n;
        t /= tx_n;
        const int ty = t % ty_n;
        b = t / ty_n;
        x0 = tx * TP;
        y0 = ty * TP;
    };

    bf16x8 ra[A_PER_T], rb[B_PER_T];
    auto load_a = [&](int it) {
        int b, y0, x0;
        tile_xy(t_beg + it / nchunk, b, y0, x0);
        const int c0 = (it % nchunk) * 32;
#pragma unroll
        for (int k = 0; k < A_PER_T; ++k) {
            const int i = threadIdx.x + 256 * k;
            if (i < A_ITEMS) {
                const int pi = i >> 2, grp = i & 3;
                const int py = pi / HP, px = pi - py * HP;
                ra[k] = gather8<MODE>(a.g, b, wrap(y0 - 1 + py, a.H), wrap(x0 - 1 + px, a.W),
                                c0 + 8 * grp);
            }
        }
    };
    auto store_a = [&]() {
#pragma unroll
        for (int k = 0; k < A_PER_T; ++k) {
            const int i = threadIdx.x + 256 * k;
            if (i < A_ITEMS) {
                const int pi = i >> 2, py = pi / HP, px = pi - py * HP;
                *reinterpret_cast<bf16x8*>(&sA[py * ROWA + px * APAD + 8 * (i & 3)]) = ra[k];
            }
        }
    };
    auto load_b = [&](int it) {
        const int c0 = (it % nchunk) * 32;
#pragma unroll
        for (int k = 0; k < B_PER_T; ++k) {
            const int i = threadIdx.x + 256 * k;
            const int col = i / 36, rem = i - col * 36;
            const int tap = rem >> 2, grp = rem & 3;
            const int co = co0 + col;
            rb[k] = (i < B_ITEMS && co < a.Cout)
                        ? *reinterpret_cast<const bf16x8*>(a.w + ((size_t)co * 9 + tap) * C +
                                                           c0 + 8 * grp)
                        : zero8;
        }
    };
    auto store_b = [&]() {
#pragma unroll
        for (int k = 0; k < B_PER_T; ++k) {
            const int i = threadIdx.x + 256 * k;
            const int col = i / 36, rem = i - col * 36;
            if (i < B_ITEMS) *reinterpret_cast<bf16x8*>(&sB[col * BPAD + rem * 8]) = rb[k];
        }
    };

    f32x16 acc[2][NB];
    // this lane's pixel in each row block: patch row 4w + 2mb + l32/16, column l32%16
    const int prow = 4 * wave + (l32 >> 4), pcol = l32 & 15;

    if (niter > 0) {
        load_b(0);
        if (MODE != MODE_POOL) load_a(0);
    }
    for (int it = 0; it < niter; ++it) {
        const int ch = it % nchunk;
        if (ch == 0) {
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int j = 0; j < 16; ++j) acc[mb][nb][j] = 0.0f;
        }
        __syncthreads();                         // the previous chunk is consumed
        if (MODE == MODE_POOL) load_a(it);       // pooled gathers average at once
        store_a();
        if (nchunk > 1 || it == 0) store_b();
        __syncthreads();
        if (it + 1 < niter) {
            if (nchunk > 1) load_b(it + 1);
            if (MODE != MODE_POOL) load_a(it + 1);
        }
        // K steps s = 2 tap + h (h: the half of the chunk's 32 channels), the operands of
        // step s + 1 read from LDS ahead of step s's MFMAs, so that the MFMAs cover the
        // reads' latency (the accumulation order is unchanged)
        auto ld = [&](int s, bf16x8 (&A)[2], bf16x8 (&Bm)[NB]) {
            const int tap = s >> 1, h = s & 1;
            const int dy = tap / 3, dx = tap % 3;   // halo coordinates: +1 offset folded in
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
                A[mb] = *reinterpret_cast<const bf16x8*>(
                    &sA[(prow + 2 * mb + dy) * ROWA + (pcol + dx) * APAD + 16 * h + 8 * g]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                Bm[nb] = *reinterpret_cast<const bf16x8*>(
                    &sB[(nb * 32 + l32) * BPAD + tap * 32 + 16 * h + 8 * g]);
        };
        bf16x8 Ac[2], Bc[NB];
        ld(0, Ac, Bc);
#pragma unroll
        for (int s = 0; s < 18; ++s) {
            bf16x8 An[2], Bn[NB];
            if (s + 1 < 18) ld(s + 1, An, Bn);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Bc[nb], Ac[mb],
                                                                         acc[mb][nb], 0, 0, 0);
            if (s + 1 < 18) {
                __builtin_amdgcn_sched_group_barrier(0x100, 2 + NB, 0);   // the next reads,
                __builtin_amdgcn_sched_group_barrier(0x008, 2 * NB, 0);   // then these MFMAs
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) Ac[mb] = An[mb];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) Bc[nb] = Bn[nb];
            }
        }
        if (ch == nchunk - 1) {
            int b, y0, x0;
            tile_xy(t_beg + it / nchunk, b, y0, x0);
            if constexpr (EPI == EPI_STAGED) {
                __syncthreads();                 // every wave is done reading the patch
                tile_epilogue_staged<NB>(a, acc, b, y0, x0, co0, wave, l32, g, sA);
            } else if constexpr (EPI == EPI_HEAD) {
                tile_epilogue_head(a, acc, b, y0, x0, wave, l32, g, sH);
            } else {
                tile_epilogue_direct<NB>(a, acc, b, y0, x0, co0, wave, l32, g);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// First layer (8 input channels, same resolution): the whole K = 9 taps x 8 channels
// fits one stage.  K is ordered (tap, channel) and padded to 10 taps, so each 16-wide
// MFMA K step covers taps 2k (lanes 0-31) and 2k+1 (lanes 32-63).
// ---------------------------------------------------------------------------
constexpr int BPAD1 = 88;   // 10 taps x 8 channels + pad: conflict-free 16-byte reads

__global__ void __launch_bounds__(256, 2) k_conv_first(ConvP a) {
    __shared__ __align__(16) __bf16 sA[HP * HP * 8];
    __shared__ __align__(16) __bf16 sB[32 * BPAD1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l32 = lane & 31, g = lane >> 5;
    const int tx_n = (a.W + TP - 1) / TP, ty_n = (a.H + TP - 1) / TP;
    int blk = blockIdx.x;
    const int tx = blk % tx_n;
    blk /= tx_n;
    const int ty = blk % ty_n;
    const int b = blk / ty_n;
    const int x0 = tx * TP, y0 = ty * TP;
    const int co0 = blockIdx.y * 32;
    const bf16x8 zero8 = (bf16x8){0, 0, 0, 0, 0, 0, 0, 0};
    for (int it = threadIdx.x; it < HP * HP; it += 256) {
        const int py = it / HP, px = it - py * HP;
        *reinterpret_cast<bf16x8*>(&sA[it * 8]) =
            gather8<MODE_SAME>(a.g, b, wrap(y0 - 1 + py, a.H), wrap(x0 - 1 + px, a.W), 0);
    }
    for (int it = threadIdx.x; it < 32 * 10; it += 256) {
        const int col = it / 10, tap = it - col * 10;
        const int co = co0 + col;
        *reinterpret_cast<bf16x8*>(&sB[col * BPAD1 + tap * 8]) =
            (tap < 9 && co < a.Cout)
                ? *reinterpret_cast<const bf16x8*>(a.w + ((size_t)co * 9 + tap) * 8)
                : zero8;
    }
    __syncthreads();
    f32x16 acc[2][1];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[mb][0][j] = 0.0f;
    const int prow = 4 * wave + (l32 >> 4), pcol = l32 & 15;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int tap = 2 * k + g;
        const int dy = tap / 3, dx = tap % 3;
        const bf16x8 Bm = *reinterpret_cast<const bf16x8*>(&sB[l32 * BPAD1 + tap * 8]);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const bf16x8 A =
                tap < 9 ? *reinterpret_cast<const bf16x8*>(
                              &sA[((prow + 2 * mb + dy) * HP + pcol + dx) * 8])
                        : zero8;
            acc[mb][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Bm, A, acc[mb][0], 0, 0, 0);
        }
    }
    tile_epilogue_direct<1>(a, acc, b, y0, x0, co0, wave, l32, g);
}

// ---------------------------------------------------------------------------
// Inference stem: the first layer (8 input channels) computed straight into the second
// layer's staged halo patch.  A workgroup's 16x16 output tile of the second layer needs
// the first layer's activations on its 18x18 halo patch; it computes them from a 20x20
// patch of the input with k_conv_first's MFMA sequence, bias, SiLU and BF16 rounding (so
// they are bitwise the values the first layer would have stored, the periodic wrap
// commuting with the convolution) and writes them where k_conv_tiled stages its input;
// the second layer then runs as k_conv_tiled<32> with the staged epilogue.  Both layers'
// weight operands stay in registers; workgroups walk runs of tiles with the next tile's
// input loads in flight.  The first layer's activations never reach HBM; training keeps
// the two layers apart (its backward pass needs them).  Needs H, W >= 16 (one period of
// wrap covers the patch).  Measured: 151 us at batch 32 against 158 us for the two
// kernels (the pair is bound by its per-tile chain of load, two MFMA phases and stores,
// not by the HBM bytes it saves).
// ---------------------------------------------------------------------------
constexpr int HP2 = HP + 2;                       // input patch edge
constexpr int STEM_PIX = HP * HP;                 // first-layer pixels per tile
constexpr int STEM_BLK = (STEM_PIX + 31) / 32;    // their 32-pixel MFMA blocks

__global__ void __launch_bounds__(256, 2) k_conv_stem(ConvP a0, ConvP a, int tiles_per_wg) {
    __shared__ __align__(16) __bf16 sX[HP2 * HP2 * 8];
    __shared__ __align__(16) __bf16 sA[HP * ROWA];
    static_assert(4 * 64 * OROW <= HP * ROWA, "epilogue staging must fit the patch buffer");
    constexpr int X_PER_T = (HP2 * HP2 + 255) / 256;   // 16-byte input items per thread
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l32 = lane & 31, g = lane >> 5;
    const int tx_n = (a.W + TP - 1) / TP, ty_n = (a.H + TP - 1) / TP;
    const int ntile = a.B * tx_n * ty_n;
    const int t_beg = blockIdx.x * tiles_per_wg;
    const int t_end = min(ntile, t_beg + tiles_per_wg);
    const bf16x8 zero8 = (bf16x8){0, 0, 0, 0, 0, 0, 0, 0};
    auto tile_xy = [&](int t, int& b, int& y0, int& x0) {
        const int tx = t % tx_n;
        t /= tx_n;
        const int ty = t % ty_n;
        b = t / ty_n;
        x0 = tx * TP;
        y0 = ty * TP;
    };
    // a tile's input pixels (y0 - 2 + qy, x0 - 2 + qx), into registers
    bf16x8 rx[X_PER_T];
    auto load_x = [&](int t) {
        int b, y0, x0;
        tile_xy(t, b, y0, x0);
#pragma unroll
        for (int k = 0; k < X_PER_T; ++k) {
            const int it = threadIdx.x + 256 * k;
            if (it < HP2 * HP2) {
                const int qy = it / HP2, qx = it - qy * HP2;
                rx[k] = gather8<MODE_SAME>(a0.g, b, wrap(y0 - 2 + qy, a.H),
                                           wrap(x0 - 2 + qx, a.W), 0);
            }
        }
    };
    // both layers' weight operands, held in registers for the workgroup's life (the
    // values k_conv_first and k_conv_tiled stage in LDS): lane l32 is output channel l32;
    // first layer: taps 2s + g (the tenth zero) of 8 channels; second layer: tap t, input
    // channels 16h + 8g .. + 7
    bf16x8 w0[5], w1[9][2];
#pragma unroll
    for (int s5 = 0; s5 < 5; ++s5) {
        const int tap = 2 * s5 + g;
        w0[s5] = tap < 9 ? *reinterpret_cast<const bf16x8*>(a0.w + ((size_t)l32 * 9 + tap) * 8)
                         : zero8;
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            w1[tap][h] = *reinterpret_cast<const bf16x8*>(a.w + ((size_t)l32 * 9 + tap) * 32 +
                                                          16 * h + 8 * g);
    if (t_beg < t_end) load_x(t_beg);
    for (int t = t_beg; t < t_end; ++t) {
        int b, y0, x0;
        tile_xy(t, b, y0, x0);
        __syncthreads();                           // the previous tile is done with sX, sA
#pragma unroll
        for (int k = 0; k < X_PER_T; ++k) {
            const int it = threadIdx.x + 256 * k;
            if (it < HP2 * HP2) *reinterpret_cast<bf16x8*>(&sX[it * 8]) = rx[k];
        }
        __syncthreads();
        if (t + 1 < t_end) load_x(t + 1);          // in flight while this tile computes
        // the first layer on the 18x18 halo patch, 32 pixels (in row-major patch order) per
        // MFMA block; the last block's spare lanes repeat its last pixel and store nothing
        for (int k = wave; k < STEM_BLK; k += 4) {
            const int p = 32 * k + l32;
            const int pc = p < STEM_PIX ? p : STEM_PIX - 1;
            const int py = pc / HP, px = pc - py * HP;
            f32x16 acc;
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const int tap = 2 * s + g;
                const int dy = tap / 3, dx = tap % 3;
                const bf16x8 Bm = w0[s];
                const bf16x8 A = tap < 9 ? *reinterpret_cast<const bf16x8*>(
                                               &sX[((py + dy) * HP2 + px + dx) * 8])
                                         : zero8;
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Bm, A, acc, 0, 0, 0);
            }
            if (p < STEM_PIX) {
                typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bf16x4 o;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float v =
                            acc[4 * q + e] + (a0.bias ? a0.bias[8 * q + 4 * g + e] : 0.0f);
                        o[e] = (__bf16)(a0.act ? silu(v) : v);
                    }
                    *reinterpret_cast<bf16x4*>(&sA[py * ROWA + px * APAD + 8 * q + 4 * g]) = o;
                }
            }
        }
        __syncthreads();
        // the second layer, as k_conv_tiled<32> over its one input chunk
        f32x16 acc[2][1];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[mb][0][j] = 0.0f;
        const int prow = 4 * wave + (l32 >> 4), pcol = l32 & 15;
        // K steps s = 2 tap + h, the patch operands of step s + 1 read ahead of step s's
        // MFMAs (as in k_conv_tiled; the accumulation order is unchanged)
        auto ld = [&](int s, bf16x8 (&A)[2]) {
            const int tap = s >> 1, h = s & 1;
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
                A[mb] = *reinterpret_cast<const bf16x8*>(
                    &sA[(prow + 2 * mb + dy) * ROWA + (pcol + dx) * APAD + 16 * h + 8 * g]);
        };
        bf16x8 Ac[2];
        ld(0, Ac);
#pragma unroll
        for (int s = 0; s < 18; ++s) {
            bf16x8 An[2];
            if (s + 1 < 18) ld(s + 1, An);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
                acc[mb][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1[s >> 1][s & 1], Ac[mb],
                                                                     acc[mb][0], 0, 0, 0);
            if (s + 1 < 18) {
                __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // the next reads,
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // then these MFMAs
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) Ac[mb] = An[mb];
            }
        }
        __syncthreads();                 // every wave is done reading the patch
        tile_epilogue_staged<1>(a, acc, b, y0, x0, 0, wave, l32, g, sA);
    }
}

// ---------------------------------------------------------------------------
// Weight gradient staged through LDS: dW[o, tap, c] = sum_p dz[p, o] in[p + off(tap), c].
// A workgroup owns 32 output x 32 input channels and all 9 taps, and a contiguous range
// of 16x16 pixel patches (split K).  Per patch, dz is staged transposed ([o][pixel]) and
// the input halo as three copies shifted by dx ([dx][c][halo row][16 pixels]), so every
// MFMA operand (8 consecutive pixels of one channel) is an aligned 16-byte LDS read.
// Wave w reduces over patch rows 4w..4w+3 for all taps; the 4 wave sums are added in a
// fixed order and the workgroup's partial sums go to part[split].
// ---------------------------------------------------------------------------
constexpr int DZ_STRIDE = 264;                 // 256 pixels + pad per output channel
constexpr int XC_STRIDE = HP * 16 + 8;         // 18 halo rows x 16 pixels + pad per channel
constexpr int X_COPY = 32 * XC_STRIDE;         // one dx-shifted copy

template <int MODE>
__global__ void __launch_bounds__(256, 2) k_wgrad_tiled(WgradP a, int patches_per_split,
                                                        int npatch) {
    __shared__ __bf16 sD[32 * DZ_STRIDE];
    __shared__ __bf16 sX[3 * X_COPY];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l32 = lane & 31, g = lane >> 5;
    const int o0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
    const int C = a.g.C;
    const int tx_n = (a.W + TP - 1) / TP, ty_n = (a.H + TP - 1) / TP;
    const int pbeg = blockIdx.z * patches_per_split;
    const int pend = min(npatch, pbeg + patches_per_split);
    const bf16x8 zero8 = (bf16x8){0, 0, 0, 0, 0, 0, 0, 0};

    f32x16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[t][j] = 0.0f;

    bf16x8 rd[4], rx[A_PER_T];
    auto load = [&](int patch) {
        int q = patch;
        const int tx = q % tx_n;
        q /= tx_n;
        const int ty = q % ty_n;
        const int b = q / ty_n;
        const int x0 = tx * TP, y0 = ty * TP;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int it = threadIdx.x + 256 * k;     // 256 pixels x 4 groups of 8 channels
            const int pi = it >> 2, og = it & 3;
            const int y = y0 + (pi >> 4), x = x0 + (pi & 15), o = o0 + 8 * og;
            rd[k] = (y < a.H && x < a.W && o < a.Cout)
                        ? *reinterpret_cast<const bf16x8*>(
                              a.dz + (((size_t)b * a.H + y) * a.W + x) * a.Cout + o)
                        : zero8;
        }
#pragma unroll
        for (int k = 0; k < A_PER_T; ++k) {
            const int it = threadIdx.x + 256 * k;     // 18x18 halo pixels x 4 groups
            if (it < A_ITEMS) {
                const int pi = it >> 2, cg = it & 3;
                const int hy = pi / HP, hx = pi - hy * HP;
                const int c = c0 + 8 * cg;
                rx[k] = c < C ? gather8<MODE>(a.g, b, wrap(y0 - 1 + hy, a.H), wrap(x0 - 1 + hx, a.W), c)
                              : zero8;
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int it = threadIdx.x + 256 * k;
            const int pi = it >> 2, og = it & 3;
#pragma unroll
            for (int e = 0; e < 8; ++e) sD[(8 * og + e) * DZ_STRIDE + pi] = rd[k][e];
        }
#pragma unroll
        for (int k = 0; k < A_PER_T; ++k) {
            const int it = threadIdx.x + 256 * k;
            if (it < A_ITEMS) {
                const int pi = it >> 2, cg = it & 3;
                const int hy = pi / HP, hx = pi - hy * HP;
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int px = hx - dx;
                    if (px >= 0 && px < TP)
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            sX[dx * X_COPY + (8 * cg + e) * XC_STRIDE + hy * 16 + px] = rx[k][e];
                }
            }
        }
    };

    if (pbeg < pend) load(pbeg);
    for (int patch = pbeg; patch < pend; ++patch) {
        __syncthreads();
        store();
        __syncthreads();
        if (patch + 1 < pend) load(patch + 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int py = 4 * wave + r;
            const bf16x8 A = *reinterpret_cast<const bf16x8*>(&sD[l32 * DZ_STRIDE + py * 16 + 8 * g]);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap % 3;
                const bf16x8 Bv = *reinterpret_cast<const bf16x8*>(
                    &sX[dx * X_COPY + l32 * XC_STRIDE + (py + dy) * 16 + 8 * g]);
                acc[tap] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bv, acc[tap], 0, 0, 0);
            }
        }
    }
    // fixed-order sum of the 4 waves, one tap at a time, through the (now free) sX region
    float* red = reinterpret_cast<float*>(sX);       // [4 waves][32 o][33]
    for (int tap = 0; tap < 9; ++tap) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int o = 8 * (j >> 2) + 4 * g + (j & 3);
            red[(wave * 32 + o) * 33 + l32] = acc[tap][j];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < 1024; k += 256) {
            const int o = k >> 5, c = k & 31;
            const float v = ((red[o * 33 + c] + red[(32 + o) * 33 + c]) + red[(64 + o) * 33 + c]) +
                            red[(96 + o) * 33 + c];
            if (o0 + o < a.Cout && c0 + c < C)
                a.part[(size_t)blockIdx.z * a.Cout * 9 * C + ((size_t)(o0 + o) * 9 + tap) * C + c0 + c] = v;
        }
    }
}

// out[i] = sum_s part[s][i] (+ out[i] if accumulate).  A block takes 64 consecutive i;
// its 4 rows of lanes take every 4th split, each with four independent partial sums
// (splits k, k+4, k+8, k+12 of a stride of 16) so that several loads are in flight;
// every combination is in a fixed order, so the result does not depend on scheduling.
__global__ void __launch_bounds__(256) k_reduce_splits(const float* __restrict__ part, int nsplit,
                                                       size_t n, float* __restrict__ out,
                                                       int accumulate) {
    __shared__ float sred[4][65];
    const int ci = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const size_t i = (size_t)blockIdx.x * 64 + ci;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    if (i < n) {
        int k = sl;
        for (; k + 12 < nsplit; k += 16) {
            a0 += part[(size_t)k * n + i];
            a1 += part[(size_t)(k + 4) * n + i];
            a2 += part[(size_t)(k + 8) * n + i];
            a3 += part[(size_t)(k + 12) * n + i];
        }
        for (; k < nsplit; k += 4) a0 += part[(size_t)k * n + i];
    }
    sred[sl][ci] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (sl == 0 && i < n) {
        const float t = ((sred[0][ci] + sred[1][ci]) + sred[2][ci]) + sred[3][ci];
        out[i] = accumulate ? out[i] + t : t;
    }
}

// column sums of a [P][C] BF16 matrix over a pixel range per block: part[blk][C]
__global__ void __launch_bounds__(256) k_colsum(const __bf16* __restrict__ m, int P, int C,
                                                int px_per_block, float* __restrict__ part) {
    __shared__ float s[256];
    const int c = threadIdx.x % 32 + 32 * blockIdx.y;
    const int r = threadIdx.x / 32;                   // 8 row lanes
    const int pb = blockIdx.x * px_per_block, pe = min(P, pb + px_per_block);
    float acc = 0.f;
    if (c < C)
        for (int p = pb + r; p < pe; p += 8) acc += (float)m[(size_t)p * C + c];
    s[threadIdx.x] = acc;
    __syncthreads();
    if (r == 0 && c < C) {
        float t = 0.f;
        for (int k = 0; k < 8; ++k) t += s[k * 32 + threadIdx.x % 32];
        part[(size_t)blockIdx.x * C + c] = t;
    }
}

// dz[p, c] = d_act[p, c0 + c] * silu'(z[p, c]) (BF16), and per block of ppb pixels the
// column sums of dz: part[block][c] (the bias gradient's partial sums)
__global__ void __launch_bounds__(256) k_silu_bwd(const float* __restrict__ dact, int cs, int c0,
                                                  const __bf16* __restrict__ z, int P, int C,
                                                  int ppb, __bf16* __restrict__ dz,
                                                  float* __restrict__ part) {
    __shared__ float sred[8][33];
    const int cl = threadIdx.x & 31, r = threadIdx.x >> 5;
    const int c = blockIdx.y * 32 + cl;
    const int pb = blockIdx.x * ppb, pe = min(P, pb + ppb);
    float acc = 0.f;
    if (c < C)
#pragma unroll 8
        for (int p = pb + r; p < pe; p += 8) {
            const size_t i = (size_t)p * C + c;
            const __bf16 d = (__bf16)(dact[(size_t)p * cs + c0 + c] * silu_grad((float)z[i]));
            dz[i] = d;
            acc += (float)d;
        }
    sred[r][cl] = acc;
    __syncthreads();
    if (r == 0 && c < C) {
        float t = 0.f;
        for (int k = 0; k < 8; ++k) t += sred[k][cl];
        part[(size_t)blockIdx.x * C + c] = t;
    }
}

// grad_hi[b, 2y+i, 2x+j, c0 + c] += dx_lo[b, y, x, c] / 4   (average pooling adjoint)
__global__ void k_unpool_add(const float* __restrict__ dlo, int B, int Hl, int Wl, int C,
                             float* __restrict__ ghi, int cs, int c0) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t n = (size_t)B * 4 * Hl * Wl * C;
    if (i >= n) return;
    const int c = (int)(i % C);
    size_t p = i / C;
    const int x = (int)(p % (2 * Wl));
    p /= 2 * Wl;
    const int y = (int)(p % (2 * Hl));
    const int b = (int)(p / (2 * Hl));
    ghi[(((size_t)b * 2 * Hl + y) * 2 * Wl + x) * cs + c0 + c] +=
        0.25f * dlo[(((size_t)b * Hl + y / 2) * Wl + x / 2) * C + c];
}

// grad_lo[b, y, x, c0 + c] (+)= sum_{i,j} dx_hi[b, 2y+i, 2x+j, c]   (upsampling adjoint)
__global__ void k_sumpool(const float* __restrict__ dhi, int B, int Hl, int Wl, int C,
                          float* __restrict__ glo, int cs, int c0, int acc) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t n = (size_t)B * Hl * Wl * C;
    if (i >= n) return;
    const int c = (int)(i % C);
    const size_t p = i / C;
    const int x = (int)(p % Wl);
    const int y = (int)((p / Wl) % Hl);
    const int b = (int)(p / ((size_t)Wl * Hl));
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            s += dhi[(((size_t)b * 2 * Hl + 2 * y + a) * 2 * Wl + 2 * x + bb) * C + c];
    float* g = glo + p * cs + c0 + c;
    *g = acc ? *g + s : s;
}

// 1x1 head: out[p, o] = bh[o] + sum_c act[p, c] wh[o, c]   (32 -> 4)
__global__ void k_head_fwd(const __bf16* __restrict__ act, int cs, int c0, const float* __restrict__ wh,
                           const float* __restrict__ bh, size_t P, float* __restrict__ out) {
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    float v0[16], v1[16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v0[4 * q + e] = (float)act[p * cs + c0 + 8 * q + e];
            v1[4 * q + e] = (float)act[p * cs + c0 + 8 * q + 4 + e];
        }
    float p0[4], p1[4];
    head_half(v0, 0, wh, p0);
    head_half(v1, 1, wh, p1);
    for (int k = 0; k < 4; ++k) out[p * 4 + k] = (p0[k] + p1[k]) + bh[k];
}

// head backward: dact[p, c] = sum_o dout[p, o] wh[o, c]; per block of HEAD_PPB pixels the
// partial sums part[blk][o * 32 + c] of dwh[o, c] = sum_p dout[p, o] act[p, c] and
// part[blk][128 + o] of dbh[o] = sum_p dout[p, o].  Each thread accumulates its pixels in
// registers; waves reduce by butterfly shuffles, then the 4 wave sums are added in order.
constexpr int HEAD_PPB = 2048;
__global__ void __launch_bounds__(256) k_head_bwd(const __bf16* __restrict__ act, int cs, int c0,
                                                  const float* __restrict__ wh,
                                                  const float* __restrict__ dout, size_t P,
                                                  float* __restrict__ dact, int dcs, int dc0,
                                                  float* __restrict__ part) {
    __shared__ float sred[4][132];
    float acc[132];
#pragma unroll
    for (int k = 0; k < 132; ++k) acc[k] = 0.f;
    const size_t pb = (size_t)blockIdx.x * HEAD_PPB;
    const size_t pe = pb + HEAD_PPB < P ? pb + HEAD_PPB : P;
    for (size_t p = pb + threadIdx.x; p < pe; p += 256) {
        const float4 d4 = reinterpret_cast<const float4*>(dout)[p];
        const float d[4] = {d4.x, d4.y, d4.z, d4.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(act + p * cs + c0 + 8 * q);
            float g[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int c = 8 * q + e;
                const float av = (float)v[e];
                g[e] = d[0] * wh[c] + d[1] * wh[32 + c] + d[2] * wh[64 + c] + d[3] * wh[96 + c];
#pragma unroll
                for (int o = 0; o < 4; ++o) acc[o * 32 + c] += d[o] * av;
            }
            float4* dst = reinterpret_cast<float4*>(dact + p * dcs + dc0 + 8 * q);
            dst[0] = make_float4(g[0], g[1], g[2], g[3]);
            dst[1] = make_float4(g[4], g[5], g[6], g[7]);
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) acc[128 + o] += d[o];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 132; ++k) {
        float v = acc[k];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
        if (lane == 0) sred[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 132)
        part[(size_t)blockIdx.x * 132 + threadIdx.x] =
            ((sred[0][threadIdx.x] + sred[1][threadIdx.x]) + sred[2][threadIdx.x]) +
            sred[3][threadIdx.x];
}

// MSE: per-block partial sums of (out - y)^2 and dout = 2 (out - y) / n
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ out, const float* __restrict__ y,
                                             size_t n, float* __restrict__ dout,
                                             double* __restrict__ part) {
    __shared__ double s[256];
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (i < n) {
        const float d = out[i] - y[i];
        e = (double)d * d;
        if (dout) dout[i] = 2.0f * d / (float)n;
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) k_sum_f64(const double* __restrict__ part, int n,
                                                 double* __restrict__ out) {
    __shared__ double sred[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += part[i];
    sred[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) sred[threadIdx.x] += sred[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sred[0];
}

// Adam (Kingma & Ba) on FP32 masters
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float c1, float c2) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// BF16 copies of one layer's weights: wf [Cout][9][Cin] and, for the input gradient,
// wt [Cin][9][Cout] with the taps mirrored (tap -> 8 - tap)
__global__ void k_weights_bf16(const float* __restrict__ w, int Cout, int Cin, __bf16* __restrict__ wf,
                               __bf16* __restrict__ wt) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t n = (size_t)Cout * 9 * Cin;
    if (i >= n) return;
    const int ci = (int)(i % Cin);
    const int tap = (int)((i / Cin) % 9);
    const int co = (int)(i / (9 * (size_t)Cin));
    wf[i] = (__bf16)w[i];
    if (wt) wt[((size_t)ci * 9 + (8 - tap)) * Cout + co] = (__bf16)w[i];
}

// density of sample b at order parameter phi (clamped: phi overshoots [0, 1] slightly and
// rho must stay positive for the velocity conversion)
__device__ __forceinline__ float dens(const DensTab& d, size_t b, float phi) {
    return fmaf(fminf(fmaxf(phi, 0.0f), 1.0f), d.rd[b], d.rl[b]);
}

// network input from solver fields, sample b = blockIdx.y of the batch:
// x[b, y, x, :] = ((phi - s0) k0, (P - s1) k1, (u_x - s2) k2, (u_y - s3) k3,
// lrr_b lrr_scale, 0, 0, 0) with u = J / rho(phi)
__global__ void k_pack(const float* __restrict__ phi, const float* __restrict__ P,
                       const float* __restrict__ J, DensTab d, Norm nm, size_t HW,
                       __bf16* __restrict__ x) {
    const size_t s = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= HW) return;
    const size_t b = blockIdx.y;
    const size_t i = b * HW + s;
    const float rho = dens(d, b, phi[i]);
    const float f[4] = {phi[i], P[i], J[2 * b * HW + s] / rho, J[(2 * b + 1) * HW + s] / rho};
    bf16x8 v;
    for (int c = 0; c < 4; ++c) v[c] = (__bf16)((f[c] - nm.shift[c]) * nm.scale[c]);
    v[4] = (__bf16)(d.lrr[b] * nm.lrr_scale);
    v[5] = v[6] = v[7] = (__bf16)0.0f;
    *reinterpret_cast<bf16x8*>(x + i * 8) = v;
}

// training target of sample b = blockIdx.y: y[s, c] = (f1_c - f0_c) / out_scale[c] for
// (phi, P, u_x, u_y)
__global__ void k_pack_target(const float* __restrict__ phi0, const float* __restrict__ P0,
                              const float* __restrict__ J0, const float* __restrict__ phi1,
                              const float* __restrict__ P1, const float* __restrict__ J1, DensTab d,
                              Norm nm, size_t HW, float* __restrict__ y) {
    const size_t s = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= HW) return;
    const size_t b = blockIdx.y;
    const size_t i = b * HW + s, jx = 2 * b * HW + s, jy = (2 * b + 1) * HW + s;
    const float r0 = dens(d, b, phi0[i]), r1 = dens(d, b, phi1[i]);
    float4 v;
    v.x = (phi1[i] - phi0[i]) / nm.out_scale[0];
    v.y = (P1[i] - P0[i]) / nm.out_scale[1];
    v.z = (J1[jx] / r1 - J0[jx] / r0) / nm.out_scale[2];
    v.w = (J1[jy] / r1 - J0[jy] / r0) / nm.out_scale[3];
    reinterpret_cast<float4*>(y)[i] = v;
}

// a predicted residual applied to sample b = blockIdx.y in place: phi and P advance by
// out * out_scale, the velocity J / rho(phi) likewise, and J = rho(phi_new) u_new
__global__ void k_apply(const float* __restrict__ out, Norm nm, DensTab d, size_t HW,
                        float* __restrict__ phi, float* __restrict__ P, float* __restrict__ J) {
    const size_t s = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= HW) return;
    const size_t b = blockIdx.y;
    const size_t i = b * HW + s, jx = 2 * b * HW + s, jy = (2 * b + 1) * HW + s;
    const float4 o = reinterpret_cast<const float4*>(out)[i];
    const float r0 = dens(d, b, phi[i]);
    const float ux = J[jx] / r0 + o.z * nm.out_scale[2];
    const float uy = J[jy] / r0 + o.w * nm.out_scale[3];
    const float ph = phi[i] + o.x * nm.out_scale[0];
    const float r1 = dens(d, b, ph);
    phi[i] = ph;
    P[i] += o.y * nm.out_scale[1];
    J[jx] = r1 * ux;
    J[jy] = r1 * uy;
}

// max |a - b| per block for sample blockIdx.y of a batch of fields of n values:
// part[sample][block]; a non-finite difference propagates (fmaxf would drop it)
__global__ void __launch_bounds__(256) k_maxdiff(const float* __restrict__ a, const float* __restrict__ b,
                                                 size_t n, float* __restrict__ part) {
    __shared__ float sred[256];
    const size_t off = (size_t)blockIdx.y * n;
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float d = fabsf(a[off + i] - b[off + i]);
        m = d > m || d != d ? d : m;
    }
    sred[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) {
            const float o = sred[threadIdx.x + w];
            if (o > sred[threadIdx.x] || o != o) sred[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sred[0];
}

// largest hand-over speed |J| / rho'(phi) per block for sample blockIdx.y (see maxspeed):
// part[sample][block]; a non-finite speed propagates
__global__ void __launch_bounds__(256) k_maxspeed(const float* __restrict__ phi,
                                                  const float* __restrict__ J, DensTab d, int H,
                                                  int W, float* __restrict__ part) {
    __shared__ float sred[256];
    const size_t b = blockIdx.y;
    const size_t n = (size_t)H * W;
    const float* ph = phi + b * n;
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int y = (int)(i / W), x = (int)(i - (size_t)y * W);
        const int xm = x == 0 ? W - 1 : x - 1, xp = x == W - 1 ? 0 : x + 1;
        const int ym = y == 0 ? H - 1 : y - 1, yp = y == H - 1 ? 0 : y + 1;
        const float c = ph[i];
        // (2/T) sum_i w_i (phi(x + c_i) - phi(x)), D2Q9 weights 1/9 (axes) and 1/36
        const float ax = (ph[(size_t)y * W + xm] - c) + (ph[(size_t)y * W + xp] - c) +
                         (ph[(size_t)ym * W + x] - c) + (ph[(size_t)yp * W + x] - c);
        const float dg = (ph[(size_t)ym * W + xm] - c) + (ph[(size_t)ym * W + xp] - c) +
                         (ph[(size_t)yp * W + xm] - c) + (ph[(size_t)yp * W + xp] - c);
        const float lap = 6.0f * fmaf(1.0f / 36.0f, dg, (1.0f / 9.0f) * ax);
        const float rho = fmaf(c, d.rd[b], d.rl[b]);
        const float rp = fmaf(d.beta[b] * 0.25f * d.rd[b], lap, rho);
        const float jx = J[2 * b * n + i], jy = J[(2 * b + 1) * n + i];
        const float u = rp > 0.0f ? sqrtf(jx * jx + jy * jy) / rp : INFINITY;
        m = u > m || u != u ? u : m;
    }
    sred[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) {
            const float o = sred[threadIdx.x + w];
            if (o > sred[threadIdx.x] || o != o) sred[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = sred[0];
}

// sum of a float field in float64, per block, for sample blockIdx.y of a batch of
// fields of n values: part[sample][block]
__global__ void __launch_bounds__(256) k_sum_field(const float* __restrict__ a, size_t n,
                                                   double* __restrict__ part) {
    __shared__ double sred[256];
    const size_t off = (size_t)blockIdx.y * n;
    double m = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        m += (double)a[off + i];
    sred[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) sred[threadIdx.x] += sred[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sred[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }

template <int NT>
static hipError_t launch_tiled(const ConvP& a, hipStream_t st) {
    // as many workgroups as are resident at once (3 per CU for 32-channel tiles, 2 for
    // 64-channel tiles and the fused-head variant, as their launch bounds say); each walks
    // a contiguous run of tiles so that the loads of its next tile overlap the MFMAs of
    // the current one
    const int resident = NT == 32 && !a.head_out ? 768 : 512;
    const int ntile = a.B * ((a.H + TP - 1) / TP) * ((a.W + TP - 1) / TP);
    const int nblk_n = (a.Cout + NT - 1) / NT;
    const int per = std::max(1, (ntile * nblk_n + resident - 1) / resident);
    const dim3 grid((ntile + per - 1) / per, nblk_n);
    if (a.pout && (a.H % 2 || a.W % 2 || !a.out || (NT == 32 && a.g.mode != MODE_SAME)))
        return hipErrorInvalidValue;
    constexpr int E = NT == 64 ? EPI_STAGED : EPI_DIRECT;
    if (a.head_out) {
        if constexpr (NT == 32) {
            if (a.Cout != 32 || a.g.mode != MODE_SAME || a.out || a.zout || a.fout || a.pout ||
                !a.head_w || !a.head_b)
                return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_conv_tiled<32, MODE_SAME, EPI_HEAD>), grid, dim3(256), 0, st,
                               a, per);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (a.g.mode == MODE_POOL)
        hipLaunchKernelGGL((k_conv_tiled<NT, MODE_POOL, E>), grid, dim3(256), 0, st, a, per);
    else if (a.g.mode == MODE_UP)
        hipLaunchKernelGGL((k_conv_tiled<NT, MODE_UP, E>), grid, dim3(256), 0, st, a, per);
    else if (NT == 32 && a.pout)
        hipLaunchKernelGGL((k_conv_tiled<NT, MODE_SAME, EPI_STAGED>), grid, dim3(256), 0, st, a,
                           per);
    else
        hipLaunchKernelGGL((k_conv_tiled<NT, MODE_SAME, E>), grid, dim3(256), 0, st, a, per);
    return hipGetLastError();
}

hipError_t conv_stem(const ConvP& a0, const ConvP& a, hipStream_t st) {
    if (a0.g.C != 8 || a0.g.mode != MODE_SAME || a0.Cout != 32 || a.g.C != 32 ||
        a.g.mode != MODE_SAME || a.Cout != 32 || a0.B != a.B || a0.H != a.H || a0.W != a.W ||
        a.H < TP || a.W < TP || !a.out || a.head_out || a.fout || a.zout || a0.zout ||
        (a.pout && (a.H % 2 || a.W % 2)))
        return hipErrorInvalidValue;
    // as many workgroups as are resident at once (2 per CU), each walking a run of tiles
    // with the next tile's input loads in flight during the current tile's work
    const int ntile = a.B * ((a.H + TP - 1) / TP) * ((a.W + TP - 1) / TP);
    const int per = std::max(1, (ntile + 511) / 512);
    hipLaunchKernelGGL(k_conv_stem, dim3((ntile + per - 1) / per), dim3(256), 0, st, a0, a, per);
    return hipGetLastError();
}

hipError_t conv3x3(const ConvP& a, hipStream_t st) {
    if (a.g.C == 8 && a.g.mode == MODE_SAME && a.Cout % 32 == 0) {
        if (a.pout || a.head_out) return hipErrorInvalidValue;
        const dim3 grid(a.B * ((a.H + TP - 1) / TP) * ((a.W + TP - 1) / TP), a.Cout / 32);
        hipLaunchKernelGGL(k_conv_first, grid, dim3(256), 0, st, a);
        return hipGetLastError();
    }
    if (a.g.C % 32 == 0 && a.Cout % 32 == 0)
        return a.Cout % 64 == 0 ? launch_tiled<64>(a, st) : launch_tiled<32>(a, st);
    if (a.pout || a.head_out) return hipErrorInvalidValue;   // only the tiled kernels fuse
    const int P = a.B * a.H * a.W;
    hipLaunchKernelGGL(k_conv3x3, dim3((P + 255) / 256, (a.Cout + 31) / 32), dim3(256), 0, st, a);
    return hipGetLastError();
}

int wgrad_patches(int B, int H, int W) { return B * ((H + TP - 1) / TP) * ((W + TP - 1) / TP); }

// splits of the patch range: about 512 workgroups in all (2 per CU)
int wgrad_nsplit(int B, int H, int W, int Cout, int Cin, int* per_split) {
    const int np = wgrad_patches(B, H, W);
    const int blocks = ((Cout + 31) / 32) * ((Cin + 31) / 32);
    int ns = (512 + blocks - 1) / blocks;
    if (ns > np) ns = np;
    if (ns < 1) ns = 1;
    const int per = (np + ns - 1) / ns;
    *per_split = per;
    return (np + per - 1) / per;
}

hipError_t wgrad(const WgradP& a, hipStream_t st) {
    int per;
    const int ns = wgrad_nsplit(a.B, a.H, a.W, a.Cout, a.g.C, &per);
    const int np = wgrad_patches(a.B, a.H, a.W);
    const dim3 grid((a.Cout + 31) / 32, (a.g.C + 31) / 32, ns);
    if (a.g.mode == MODE_POOL)
        hipLaunchKernelGGL((k_wgrad_tiled<MODE_POOL>), grid, dim3(256), 0, st, a, per, np);
    else if (a.g.mode == MODE_UP)
        hipLaunchKernelGGL((k_wgrad_tiled<MODE_UP>), grid, dim3(256), 0, st, a, per, np);
    else
        hipLaunchKernelGGL((k_wgrad_tiled<MODE_SAME>), grid, dim3(256), 0, st, a, per, np);
    return hipGetLastError();
}

hipError_t reduce_splits(const float* part, int nsplit, size_t n, float* out, int acc,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st, part,
                       nsplit, n, out, acc);
    return hipGetLastError();
}

hipError_t colsum(const __bf16* m, int P, int C, int px_per_block, float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_colsum, dim3((P + px_per_block - 1) / px_per_block, (C + 31) / 32),
                       dim3(256), 0, st, m, P, C, px_per_block, part);
    return hipGetLastError();
}

hipError_t silu_bwd(const float* dact, int cs, int c0, const __bf16* z, int P, int C, int ppb,
                    __bf16* dz, float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_silu_bwd, dim3((P + ppb - 1) / ppb, (C + 31) / 32), dim3(256), 0, st, dact,
                       cs, c0, z, P, C, ppb, dz, part);
    return hipGetLastError();
}

hipError_t unpool_add(const float* dlo, int B, int Hl, int Wl, int C, float* ghi, int cs, int c0,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_unpool_add, dim3(blocks((size_t)B * 4 * Hl * Wl * C)), dim3(256), 0, st,
                       dlo, B, Hl, Wl, C, ghi, cs, c0);
    return hipGetLastError();
}

hipError_t sumpool(const float* dhi, int B, int Hl, int Wl, int C, float* glo, int cs, int c0,
                   int acc, hipStream_t st) {
    hipLaunchKernelGGL(k_sumpool, dim3(blocks((size_t)B * Hl * Wl * C)), dim3(256), 0, st, dhi, B,
                       Hl, Wl, C, glo, cs, c0, acc);
    return hipGetLastError();
}

hipError_t head_fwd(const __bf16* act, int cs, int c0, const float* wh, const float* bh, size_t P,
                    float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_head_fwd, dim3(blocks(P)), dim3(256), 0, st, act, cs, c0, wh, bh, P, out);
    return hipGetLastError();
}

hipError_t head_bwd(const __bf16* act, int cs, int c0, const float* wh, const float* dout, size_t P,
                    float* dact, int dcs, int dc0, float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_head_bwd, dim3(head_blocks(P)), dim3(256), 0, st, act, cs, c0, wh, dout, P, dact,
                       dcs, dc0, part);
    return hipGetLastError();
}

unsigned head_blocks(size_t P) { return (unsigned)((P + HEAD_PPB - 1) / HEAD_PPB); }

hipError_t mse(const float* out, const float* y, size_t n, float* dout, double* part, double* res,
               hipStream_t st) {
    hipLaunchKernelGGL(k_mse, dim3(blocks(n)), dim3(256), 0, st, out, y, n, dout, part);
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, st, part, (int)blocks(n), res);
    return hipGetLastError();
}

unsigned mse_blocks(size_t n) { return blocks(n); }

hipError_t adam(float* w, const float* g, float* m, float* v, size_t n, float lr, int t,
                hipStream_t st) {
    // bias corrections from the exact betas, so that at t = 1 they equal the FP32 (1 - beta)
    // factors of the moment updates and m / c1 = g
    const float c1 = (float)(1.0 - pow(0.9, t)), c2 = (float)(1.0 - pow(0.999, t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(256), 0, st, w, g, m, v, n, lr, c1, c2);
    return hipGetLastError();
}

hipError_t weights_bf16(const float* w, int Cout, int Cin, __bf16* wf, __bf16* wt, hipStream_t st) {
    hipLaunchKernelGGL(k_weights_bf16, dim3(blocks((size_t)Cout * 9 * Cin)), dim3(256), 0, st, w,
                       Cout, Cin, wf, wt);
    return hipGetLastError();
}

hipError_t pack(const float* phi, const float* P, const float* J, const DensTab& d, int B,
                const Norm& nm, size_t HW, __bf16* x, hipStream_t st) {
    if (B < 1 || B > LRR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack, dim3(blocks(HW), B), dim3(256), 0, st, phi, P, J, d, nm, HW, x);
    return hipGetLastError();
}

hipError_t pack_target(const float* phi0, const float* P0, const float* J0, const float* phi1,
                       const float* P1, const float* J1, const DensTab& d, int B, const Norm& nm,
                       size_t HW, float* y, hipStream_t st) {
    if (B < 1 || B > LRR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack_target, dim3(blocks(HW), B), dim3(256), 0, st, phi0, P0, J0, phi1,
                       P1, J1, d, nm, HW, y);
    return hipGetLastError();
}

hipError_t apply(const float* out, const Norm& nm, const DensTab& d, int B, size_t HW, float* phi,
                 float* P, float* J, hipStream_t st) {
    if (B < 1 || B > LRR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_apply, dim3(blocks(HW), B), dim3(256), 0, st, out, nm, d, HW, phi, P, J);
    return hipGetLastError();
}

// grid y is at most 65535: larger batches take several launches
constexpr int MAX_GRID_Y = 65535;

hipError_t maxdiff(const float* a, const float* b, int B, size_t n, float* part, int nblk,
                   hipStream_t st) {
    for (int b0 = 0; b0 < B; b0 += MAX_GRID_Y) {
        const int nb = B - b0 < MAX_GRID_Y ? B - b0 : MAX_GRID_Y;
        hipLaunchKernelGGL(k_maxdiff, dim3(nblk, nb), dim3(256), 0, st, a + b0 * n, b + b0 * n, n,
                           part + (size_t)b0 * nblk);
    }
    return hipGetLastError();
}

hipError_t maxspeed(const float* phi, const float* J, const DensTab& d, int B, int H, int W,
                    float* part, int nblk, hipStream_t st) {
    if (B < 1 || B > LRR_MAX || H < 1 || W < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_maxspeed, dim3(nblk, B), dim3(256), 0, st, phi, J, d, H, W, part);
    return hipGetLastError();
}

hipError_t sum_field(const float* a, int B, size_t n, double* part, int nblk, hipStream_t st) {
    for (int b0 = 0; b0 < B; b0 += MAX_GRID_Y) {
        const int nb = B - b0 < MAX_GRID_Y ? B - b0 : MAX_GRID_Y;
        hipLaunchKernelGGL(k_sum_field, dim3(nblk, nb), dim3(256), 0, st, a + b0 * n, n,
                           part + (size_t)b0 * nblk);
    }
    return hipGetLastError();
}

}  // namespace pfsur
