// Host-side declarations shared by the surrogate's C-ABI layer and its kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pfsur {

// how a convolution reads its input relative to its output resolution
enum { MODE_SAME = 0, MODE_UP = 1, MODE_POOL = 2 };

// channels [c0, c0 + C) of a BF16 NHWC tensor [B][Hin][Win][cs]
struct GatherP {
    const __bf16* p;
    int Hin, Win;
    int cs, c0, C;
    int mode;
};

// out[p, co] for p over B x H x W output pixels, co < Cout; weights [Cout][9][C] BF16.
// Epilogue: v = acc + bias; zout (BF16 [P][Cout]) <- v; out (BF16 at channel stride
// out_cs, offset out_c0) <- act ? silu(v) : v; fout (FP32 at f_cs, f_c0) <- v (or += v);
// pout (BF16 [B][H/2][W/2][pout_cs], channels from 0; needs out and even H, W) <- the 2x2
// average of what out receives, as the pooling gather computes it.  head_out (FP32
// [P][4]; 32-channel same-resolution layers only) <- the 1x1 head (head_w [4][32],
// head_b [4]) applied to the BF16-rounded activations, as head_fwd computes it.
struct ConvP {
    GatherP g;
    int B, H, W;
    const __bf16* w;
    int Cout;
    const float* bias;
    int act;
    __bf16* zout;
    __bf16* out;
    int out_cs, out_c0;
    float* fout;
    int f_cs, f_c0, f_accum;
    __bf16* pout;
    int pout_cs;
    const float* head_w;
    const float* head_b;
    float* head_out;
};

// part[split][Cout][9][C] = sum over the split's pixels of dz[p, co] in[p + off(tap), ci]
// (splits: wgrad_nsplit)
struct WgradP {
    GatherP g;
    int B, H, W;
    const __bf16* dz;
    int Cout;
    float* part;
};

struct Norm {
    float shift[4], scale[4], out_scale[4], lrr_scale;
};

// per-sample densities of one launch over at most LRR_MAX samples: rho(phi) = rl +
// clamp(phi, 0, 1) rd, and lrr = log10(rho_H / rho_L).  The network sees and predicts
// the velocity J / rho(phi) rather than the momentum J, which spans the density ratio.
constexpr int LRR_MAX = 64;
struct DensTab {
    float rl[LRR_MAX], rd[LRR_MAX], lrr[LRR_MAX];
    float beta[LRR_MAX];   // speed check: 1 if the solver uses Eq. 13's modified density
};

hipError_t conv3x3(const ConvP& a, hipStream_t st);
// the first two layers at inference: a0 the first (8 input channels, its outputs not
// stored), a the second (32 -> 32 channels, same resolution)
hipError_t conv_stem(const ConvP& a0, const ConvP& a, hipStream_t st);
hipError_t wgrad(const WgradP& a, hipStream_t st);
int wgrad_nsplit(int B, int H, int W, int Cout, int Cin, int* per_split);
hipError_t reduce_splits(const float* part, int nsplit, size_t n, float* out, int acc,
                         hipStream_t st);
hipError_t colsum(const __bf16* m, int P, int C, int px_per_block, float* part, hipStream_t st);
hipError_t silu_bwd(const float* dact, int cs, int c0, const __bf16* z, int P, int C, int ppb,
                    __bf16* dz, float* part, hipStream_t st);
hipError_t unpool_add(const float* dlo, int B, int Hl, int Wl, int C, float* ghi, int cs, int c0,
                      hipStream_t st);
hipError_t sumpool(const float* dhi, int B, int Hl, int Wl, int C, float* glo, int cs, int c0,
                   int acc, hipStream_t st);
hipError_t head_fwd(const __bf16* act, int cs, int c0, const float* wh, const float* bh, size_t P,
                    float* out, hipStream_t st);
hipError_t head_bwd(const __bf16* act, int cs, int c0, const float* wh, const float* dout, size_t P,
                    float* dact, int dcs, int dc0, float* part, hipStream_t st);
unsigned head_blocks(size_t P);
hipError_t mse(const float* out, const float* y, size_t n, float* dout, double* part, double* res,
               hipStream_t st);
unsigned mse_blocks(size_t n);
hipError_t adam(float* w, const float* g, float* m, float* v, size_t n, float lr, int t,
                hipStream_t st);
hipError_t weights_bf16(const float* w, int Cout, int Cin, __bf16* wf, __bf16* wt, hipStream_t st);
// B <= LRR_MAX samples each (fields per sample: phi, P [HW], J [2][HW])
hipError_t pack(const float* phi, const float* P, const float* J, const DensTab& d, int B,
                const Norm& nm, size_t HW, __bf16* x, hipStream_t st);
hipError_t pack_target(const float* phi0, const float* P0, const float* J0, const float* phi1,
                       const float* P1, const float* J1, const DensTab& d, int B, const Norm& nm,
                       size_t HW, float* y, hipStream_t st);
hipError_t apply(const float* out, const Norm& nm, const DensTab& d, int B, size_t HW, float* phi,
                 float* P, float* J, hipStream_t st);
hipError_t maxdiff(const float* a, const float* b, int B, size_t n, float* part, int nblk,
                   hipStream_t st);
hipError_t sum_field(const float* a, int B, size_t n, double* part, int nblk, hipStream_t st);
// per block, max over sites of the speed a hand-over to a D2Q9 solver would give,
// |J| / rho'(phi) with rho' = rho_L + phi rho_dif + beta rho_dif lap(phi) / 4 (periodic
// central Laplacian; rho' <= 0 counts as infinite), for sample blockIdx.y of
// B <= LRR_MAX (phi [B][H][W], J [B][2][H][W]): part[sample][block]
hipError_t maxspeed(const float* phi, const float* J, const DensTab& d, int B, int H, int W,
                    float* part, int nblk, hipStream_t st);

}  // namespace pfsur
