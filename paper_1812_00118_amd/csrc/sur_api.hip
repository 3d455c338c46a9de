// C-ABI layer of the convolutional surrogate: layer table, workspace planning, forward
// and backward orchestration, Adam, checkpoints, and the guarded hand-over with the
// lattice Boltzmann solver.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/pfsur.h"
#include "pflb_internal.hpp"
#include "sur_internal.hpp"

using namespace pfsur;

namespace {

// Activation buffers, NHWC BF16 at one level (resolution H >> level), with C channels.
// Skip connections share a buffer with the decoder branch they are concatenated with,
// so the concatenation is a channel offset.  POOLk holds the 2x2 averages of an encoder
// output, written by the producing layer's epilogue and read by the next level's pooling
// layer (no gradient buffer: the backward distributes through the pooling explicitly).
enum Buf {
    X, E0A, CAT0, D0A, D0B, E1A, CAT1, D1A, D1B, E2A, CAT2, D2A, D2B, B3A, B3B,
    POOL0, POOL1, POOL2, NBUFS
};
struct BufDef {
    int level, C, grad;
};
constexpr BufDef BUFS[NBUFS] = {{0, 8, 1},   {0, 32, 1},  {0, 64, 1},  {0, 32, 1},  {0, 32, 1},
                            {1, 64, 1},  {1, 128, 1}, {1, 64, 1},  {1, 64, 1},  {2, 128, 1},
                            {2, 256, 1}, {2, 128, 1}, {2, 128, 1}, {3, 256, 1}, {3, 256, 1},
                            {1, 32, 0},  {2, 64, 0},  {3, 128, 0}};

// 3x3 layers in network order; level = output resolution.  pool_out: the buffer that also
// receives the 2x2 average of this layer's output (channels 0..Cout); pool_in: a pooling
// layer reads that buffer at its own resolution instead of pooling its input itself.
struct LayerDef {
    const char* name;
    int in_buf, in_c0, Cin, Cout, level, mode, out_buf, out_c0;
    int pool_out = -1, pool_in = -1;
};
constexpr int NL = 17;
constexpr LayerDef LAYERS[NL] = {
    {"e0a", X, 0, 8, 32, 0, MODE_SAME, E0A, 0},
    {"e0b", E0A, 0, 32, 32, 0, MODE_SAME, CAT0, 0, POOL0},
    {"e1a", CAT0, 0, 32, 64, 1, MODE_POOL, E1A, 0, -1, POOL0},
    {"e1b", E1A, 0, 64, 64, 1, MODE_SAME, CAT1, 0, POOL1},
    {"e2a", CAT1, 0, 64, 128, 2, MODE_POOL, E2A, 0, -1, POOL1},
    {"e2b", E2A, 0, 128, 128, 2, MODE_SAME, CAT2, 0, POOL2},
    {"b3a", CAT2, 0, 128, 256, 3, MODE_POOL, B3A, 0, -1, POOL2},
    {"b3b", B3A, 0, 256, 256, 3, MODE_SAME, B3B, 0},
    {"u2", B3B, 0, 256, 128, 2, MODE_UP, CAT2, 128},
    {"d2a", CAT2, 0, 256, 128, 2, MODE_SAME, D2A, 0},
    {"d2b", D2A, 0, 128, 128, 2, MODE_SAME, D2B, 0},
    {"u1", D2B, 0, 128, 64, 1, MODE_UP, CAT1, 64},
    {"d1a", CAT1, 0, 128, 64, 1, MODE_SAME, D1A, 0},
    {"d1b", D1A, 0, 64, 64, 1, MODE_SAME, D1B, 0},
    {"u0", D1B, 0, 64, 32, 0, MODE_UP, CAT0, 32},
    {"d0a", CAT0, 0, 64, 32, 0, MODE_SAME, D0A, 0},
    {"d0b", D0A, 0, 32, 32, 0, MODE_SAME, D0B, 0},
};
constexpr int HEAD_C = 32;
static_assert(LAYERS[0].Cin == 8 && LAYERS[0].Cout == 32 && LAYERS[0].mode == MODE_SAME &&
                  LAYERS[1].in_buf == LAYERS[0].out_buf && LAYERS[1].Cin == 32 &&
                  LAYERS[1].Cout == 32 && LAYERS[1].mode == MODE_SAME,
              "the first layer is fused into the second at inference");
static_assert(LAYERS[NL - 1].Cout == HEAD_C && LAYERS[NL - 1].mode == MODE_SAME &&
                  LAYERS[NL - 1].pool_out < 0,
              "the head is fused into the last layer at inference");

// a pooled buffer is written whole by one layer at the level above the pooling layer that
// reads it, and holds exactly the channels that layer would pool from its input buffer
constexpr bool pool_links_ok() {
    for (int c = 0; c < NL; ++c) {
        const LayerDef& R = LAYERS[c];
        if (R.pool_in < 0) continue;
        int writers = 0;
        for (int l = 0; l < NL; ++l) {
            const LayerDef& W = LAYERS[l];
            if (W.pool_out != R.pool_in) continue;
            ++writers;
            if (l >= c || W.out_buf != R.in_buf || W.out_c0 != R.in_c0 || W.Cout != R.Cin ||
                W.level + 1 != R.level)
                return false;
        }
        if (writers != 1 || R.mode != MODE_POOL || BUFS[R.pool_in].C != R.Cin ||
            BUFS[R.pool_in].level != R.level || BUFS[R.pool_in].grad)
            return false;
    }
    return true;
}
static_assert(pool_links_ok(), "inconsistent pooled-input links in the layer table");

struct ParamLayout {
    size_t w[NL], b[NL], head, total;
    ParamLayout() {
        size_t o = 0;
        for (int l = 0; l < NL; ++l) {
            w[l] = o;
            o += (size_t)LAYERS[l].Cout * 9 * LAYERS[l].Cin;
            b[l] = o;
            o += LAYERS[l].Cout;
        }
        head = o;
        total = o + PFSUR_OUT_CH * HEAD_C + PFSUR_OUT_CH;
    }
};
const ParamLayout PL;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int COLSUM_PX = 1024;   // pixels per block of the primitive's bias sums
constexpr int SILU_PX = 256;      // pixels per block of the fused SiLU backward

// floats of the partial-sum buffer for one layer's weight and bias gradients
size_t wgrad_part_floats(int B, int H, int W, int Cout, int Cin) {
    int per;
    const int ns = wgrad_nsplit(B, H, W, Cout, Cin, &per);
    const size_t P = (size_t)B * H * W;
    const size_t a = (size_t)ns * Cout * 9 * Cin;
    const size_t b = (P + SILU_PX - 1) / SILU_PX * Cout;
    const size_t c = (P + COLSUM_PX - 1) / COLSUM_PX * Cout;
    return std::max(a, std::max(b, c));
}

// byte offsets into the caller's workspace
struct Plan {
    size_t act[NBUFS], z[NL], dact[NBUFS];
    size_t out, dout, dz, dx, part, mse_part, loss;
    size_t total;
};

Plan make_plan(int H, int W, int B, bool training) {
    Plan p;
    memset(&p, 0, sizeof(p));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes);
        return r;
    };
    auto pix = [&](int level) { return (size_t)B * (H >> level) * (W >> level); };
    for (int k = 1; k < NBUFS; ++k) p.act[k] = take(pix(BUFS[k].level) * BUFS[k].C * 2);
    if (training) {
        for (int l = 0; l < NL; ++l) p.z[l] = take(pix(LAYERS[l].level) * LAYERS[l].Cout * 2);
        for (int k = 1; k < NBUFS; ++k)
            if (BUFS[k].grad) p.dact[k] = take(pix(BUFS[k].level) * BUFS[k].C * 4);
        p.out = take(pix(0) * PFSUR_OUT_CH * 4);
        p.dout = take(pix(0) * PFSUR_OUT_CH * 4);
        size_t dz = 0, dx = 0, part = (size_t)head_blocks(pix(0)) * 132;
        for (int l = 0; l < NL; ++l) {
            const LayerDef& L = LAYERS[l];
            const size_t P = pix(L.level);
            dz = std::max(dz, P * L.Cout);
            if (L.mode != MODE_SAME) dx = std::max(dx, P * L.Cin);
            part = std::max(part, wgrad_part_floats(B, H >> L.level, W >> L.level, L.Cout, L.Cin));
        }
        p.dz = take(dz * 2);
        p.dx = take(dx * 4);
        p.part = take(part * 4);
        p.mse_part = take((size_t)mse_blocks(pix(0) * PFSUR_OUT_CH) * 8);
        p.loss = take(8);
    }
    p.total = o;
    return p;
}

std::string check_cfg(const pfsur_cfg* c) {
    if (!c) return "cfg is NULL";
    if (c->H < 16 || c->W < 16 || c->H % 8 || c->W % 8) return "H and W must be multiples of 8, >= 16";
    if (c->max_batch < 1) return "max_batch must be >= 1";
    if ((double)c->H * c->W * c->max_batch > 67108864.0) return "max_batch * H * W exceeds 2^26";
    for (int k = 0; k < 4; ++k)
        if (!isfinite(c->in_shift[k]) || !isfinite(c->in_scale[k]) || !isfinite(c->out_scale[k]))
            return "normalisation constants must be finite";
    if (!isfinite(c->lrr_scale)) return "lrr_scale must be finite";
    return "";
}

}  // namespace

struct pfsur_ctx {
    pfsur_cfg cfg;
    Norm nm;
    void* mem = nullptr;
    float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    __bf16* wf[NL] = {};
    __bf16* wt[NL] = {};
    int t = 0;
    std::string err;
};

namespace {

int fail(pfsur_ctx* c, int code, const std::string& what) {
    if (c) c->err = what;
    return code;
}

int hip_fail(pfsur_ctx* c, hipError_t e, const char* where) {
    return fail(c, PFLB_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define SUR_TRY(expr, where)                          \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(c, e_, where); \
    } while (0)

hipError_t refresh_bf16(pfsur_ctx* c, hipStream_t st) {
    for (int l = 0; l < NL; ++l) {
        hipError_t e = weights_bf16(c->master + PL.w[l], LAYERS[l].Cout, LAYERS[l].Cin, c->wf[l],
                                    c->wt[l], st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

GatherP gather_of(const LayerDef& L, const char* ws, const Plan& p, const void* x, int H, int W) {
    GatherP g;
    if (L.pool_in >= 0) {   // the pooled input, already averaged, at the layer's resolution
        g.p = reinterpret_cast<const __bf16*>(ws + p.act[L.pool_in]);
        g.Hin = H >> L.level;
        g.Win = W >> L.level;
        g.cs = BUFS[L.pool_in].C;
        g.c0 = 0;
        g.C = L.Cin;
        g.mode = MODE_SAME;
        return g;
    }
    g.p = L.in_buf == X ? static_cast<const __bf16*>(x)
                        : reinterpret_cast<const __bf16*>(ws + p.act[L.in_buf]);
    const int Hl = H >> L.level, Wl = W >> L.level;
    g.Hin = L.mode == MODE_POOL ? 2 * Hl : (L.mode == MODE_UP ? Hl / 2 : Hl);
    g.Win = L.mode == MODE_POOL ? 2 * Wl : (L.mode == MODE_UP ? Wl / 2 : Wl);
    g.cs = BUFS[L.in_buf].C;
    g.c0 = L.in_c0;
    g.C = L.Cin;
    g.mode = L.mode;
    return g;
}

// forward through all layers; training stores the pre-activations z
int run_forward(pfsur_ctx* c, const void* x, float* out, int B, char* ws, bool training,
                hipStream_t st) {
    const int H = c->cfg.H, W = c->cfg.W;
    const Plan p = make_plan(H, W, B, training);
    ConvP a_first;   // inference: the first layer runs inside the second's kernel
    for (int l = 0; l < NL; ++l) {
        const LayerDef& L = LAYERS[l];
        ConvP a;
        memset(&a, 0, sizeof(a));
        a.g = gather_of(L, ws, p, x, H, W);
        a.B = B;
        a.H = H >> L.level;
        a.W = W >> L.level;
        a.w = c->wf[l];
        a.Cout = L.Cout;
        a.bias = c->master + PL.b[l];
        a.act = 1;
        a.zout = training ? reinterpret_cast<__bf16*>(ws + p.z[l]) : nullptr;
        a.out = reinterpret_cast<__bf16*>(ws + p.act[L.out_buf]);
        a.out_cs = BUFS[L.out_buf].C;
        a.out_c0 = L.out_c0;
        if (L.pool_out >= 0) {
            a.pout = reinterpret_cast<__bf16*>(ws + p.act[L.pool_out]);
            a.pout_cs = BUFS[L.pool_out].C;
        }
        if (!training && l == NL - 1) {
            // inference: the head runs in the last layer's epilogue, whose activations
            // are then not stored (training keeps them for the backward pass)
            a.out = nullptr;
            a.head_w = c->master + PL.head;
            a.head_b = c->master + PL.head + PFSUR_OUT_CH * HEAD_C;
            a.head_out = out;
        }
        if (!training && l == 0) {
            a_first = a;
            continue;
        }
        if (!training && l == 1)
            SUR_TRY(conv_stem(a_first, a, st), "conv forward");
        else
            SUR_TRY(conv3x3(a, st), "conv forward");
    }
    if (training) {
        const size_t P0 = (size_t)B * H * W;
        SUR_TRY(head_fwd(reinterpret_cast<const __bf16*>(ws + p.act[D0B]), HEAD_C, 0,
                         c->master + PL.head, c->master + PL.head + PFSUR_OUT_CH * HEAD_C, P0,
                         out, st),
                "head forward");
    }
    return PFLB_OK;
}

// loss and gradients of all parameters into c->grad, after run_forward(training)
int run_backward(pfsur_ctx* c, const void* x, const float* y, int B, char* ws, hipStream_t st) {
    const int H = c->cfg.H, W = c->cfg.W;
    const Plan p = make_plan(H, W, B, true);
    const size_t P0 = (size_t)B * H * W;
    float* out = reinterpret_cast<float*>(ws + p.out);
    float* dout = reinterpret_cast<float*>(ws + p.dout);
    float* part = reinterpret_cast<float*>(ws + p.part);
    __bf16* dz = reinterpret_cast<__bf16*>(ws + p.dz);
    float* dx = reinterpret_cast<float*>(ws + p.dx);
    auto dact = [&](int buf) { return reinterpret_cast<float*>(ws + p.dact[buf]); };
    SUR_TRY(mse(out, y, P0 * PFSUR_OUT_CH, dout, reinterpret_cast<double*>(ws + p.mse_part),
                reinterpret_cast<double*>(ws + p.loss), st),
            "mse");
    SUR_TRY(head_bwd(reinterpret_cast<const __bf16*>(ws + p.act[D0B]), HEAD_C, 0,
                     c->master + PL.head, dout, P0, dact(D0B), HEAD_C, 0, part, st),
            "head backward");
    SUR_TRY(reduce_splits(part, (int)head_blocks(P0), PFSUR_OUT_CH * (HEAD_C + 1),
                          c->grad + PL.head, 0, st),
            "head reduce");
    for (int l = NL - 1; l >= 0; --l) {
        const LayerDef& L = LAYERS[l];
        const int Hl = H >> L.level, Wl = W >> L.level;
        const int P = B * Hl * Wl;
        // dz and the bias gradient's partial sums, then the weight gradient (both use part)
        SUR_TRY(silu_bwd(dact(L.out_buf), BUFS[L.out_buf].C, L.out_c0,
                         reinterpret_cast<const __bf16*>(ws + p.z[l]), P, L.Cout, SILU_PX, dz,
                         part, st),
                "silu backward");
        SUR_TRY(reduce_splits(part, (P + SILU_PX - 1) / SILU_PX, L.Cout, c->grad + PL.b[l], 0, st),
                "bias reduce");
        WgradP wg;
        wg.g = gather_of(L, ws, p, x, H, W);
        wg.B = B;
        wg.H = Hl;
        wg.W = Wl;
        wg.dz = dz;
        wg.Cout = L.Cout;
        int per;
        const int ns = wgrad_nsplit(B, Hl, Wl, L.Cout, L.Cin, &per);
        wg.part = part;
        SUR_TRY(wgrad(wg, st), "wgrad");
        SUR_TRY(reduce_splits(part, ns, (size_t)L.Cout * 9 * L.Cin, c->grad + PL.w[l], 0, st),
                "wgrad reduce");
        if (l == 0) continue;
        ConvP d;
        memset(&d, 0, sizeof(d));
        d.g.p = dz;
        d.g.Hin = Hl;
        d.g.Win = Wl;
        d.g.cs = L.Cout;
        d.g.c0 = 0;
        d.g.C = L.Cout;
        d.g.mode = MODE_SAME;
        d.B = B;
        d.H = Hl;
        d.W = Wl;
        d.w = c->wt[l];
        d.Cout = L.Cin;
        if (L.mode == MODE_SAME) {
            d.fout = dact(L.in_buf);
            d.f_cs = BUFS[L.in_buf].C;
            d.f_c0 = L.in_c0;
        } else {
            d.fout = dx;
            d.f_cs = L.Cin;
            d.f_c0 = 0;
        }
        SUR_TRY(conv3x3(d, st), "dgrad");
        if (L.mode == MODE_POOL)
            SUR_TRY(unpool_add(dx, B, Hl, Wl, L.Cin, dact(L.in_buf), BUFS[L.in_buf].C, L.in_c0, st),
                    "unpool");
        else if (L.mode == MODE_UP)
            SUR_TRY(sumpool(dx, B, Hl / 2, Wl / 2, L.Cin, dact(L.in_buf), BUFS[L.in_buf].C, L.in_c0,
                            0, st),
                    "sumpool");
    }
    return PFLB_OK;
}

int check_batch(pfsur_ctx* c, int batch) {
    if (!c) return PFLB_ERR_PARAM;
    if (batch < 1 || batch > c->cfg.max_batch)
        return fail(c, PFLB_ERR_PARAM, "batch must be in [1, max_batch]");
    return PFLB_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// (rho_L, rho_H) per sample, host array [n][2]: finite and positive
bool dens_ok(const double* rho, int n) {
    for (int k = 0; k < 2 * n; ++k)
        if (!(isfinite(rho[k]) && rho[k] > 0.0)) return false;
    return true;
}

// densities of samples [b0, b0 + nb) for one launch
DensTab dens_tab(const double* rho, int b0, int nb) {
    DensTab d;
    for (int k = 0; k < LRR_MAX; ++k) {
        const double rl = k < nb ? rho[2 * (b0 + k)] : 1.0;
        const double rh = k < nb ? rho[2 * (b0 + k) + 1] : 1.0;
        d.rl[k] = (float)rl;
        d.rd[k] = (float)(rh - rl);
        d.lrr[k] = (float)log10(rh / rl);
        d.beta[k] = 0.0f;
    }
    return d;
}

// forward + backward; *loss (host) = mean squared error of the forward pass
int forward_backward(pfsur_ctx* c, const void* x, const float* y, int batch, float* loss,
                     char* ws, hipStream_t st) {
    const Plan p = make_plan(c->cfg.H, c->cfg.W, batch, true);
    int r = run_forward(c, x, reinterpret_cast<float*>(ws + p.out), batch, ws, true, st);
    if (r) return r;
    r = run_backward(c, x, y, batch, ws, st);
    if (r) return r;
    double sum = 0.0;
    SUR_TRY(hipMemcpyAsync(&sum, ws + p.loss, sizeof(double), hipMemcpyDeviceToHost, st),
            "loss read-back");
    SUR_TRY(hipStreamSynchronize(st), "loss read-back");
    if (loss) *loss = (float)(sum / ((double)batch * c->cfg.H * c->cfg.W * PFSUR_OUT_CH));
    return PFLB_OK;
}

int check_io(pfsur_ctx* c, const void* x, const void* y, const void* ws) {
    if (!x || !y || !ws) return fail(c, PFLB_ERR_PARAM, "NULL input, target or workspace");
    if (!aligned16(x) || ((uintptr_t)ws & 255u))
        return fail(c, PFLB_ERR_ALIGN, "x must be 16-byte and workspace 256-byte aligned");
    return PFLB_OK;
}

struct SurHeader {
    char magic[8];
    int H, W;
    unsigned long long nparams;
    int t;
    int pad;
};

}  // namespace

extern "C" {

size_t pfsur_num_params(void) { return PL.total; }

int pfsur_create(const pfsur_cfg* cfg, pfsur_ctx** out) {
    if (!out) return PFLB_ERR_PARAM;
    *out = nullptr;
    if (!check_cfg(cfg).empty()) return PFLB_ERR_PARAM;
    pfsur_ctx* c = new (std::nothrow) pfsur_ctx();
    if (!c) return PFLB_ERR_NOMEM;
    c->cfg = *cfg;
    for (int k = 0; k < 4; ++k) {
        c->nm.shift[k] = cfg->in_shift[k];
        c->nm.scale[k] = cfg->in_scale[k];
        c->nm.out_scale[k] = cfg->out_scale[k];
    }
    c->nm.lrr_scale = cfg->lrr_scale;
    size_t wbytes = 0;
    for (int l = 0; l < NL; ++l) wbytes += align256((size_t)LAYERS[l].Cout * 9 * LAYERS[l].Cin * 2);
    const size_t fbytes = align256(PL.total * 4);
    const size_t total = 4 * fbytes + 2 * wbytes;
    if (hipMalloc(&c->mem, total) != hipSuccess) {
        delete c;
        return PFLB_ERR_NOMEM;
    }
    char* b = static_cast<char*>(c->mem);
    c->master = reinterpret_cast<float*>(b);
    c->grad = reinterpret_cast<float*>(b + fbytes);
    c->m = reinterpret_cast<float*>(b + 2 * fbytes);
    c->v = reinterpret_cast<float*>(b + 3 * fbytes);
    size_t o = 4 * fbytes;
    for (int l = 0; l < NL; ++l) {
        const size_t n = align256((size_t)LAYERS[l].Cout * 9 * LAYERS[l].Cin * 2);
        c->wf[l] = reinterpret_cast<__bf16*>(b + o);
        c->wt[l] = reinterpret_cast<__bf16*>(b + o + wbytes);
        o += n;
    }
    if (hipMemset(c->mem, 0, total) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->mem);
        delete c;
        return PFLB_ERR_DEVICE;
    }
    *out = c;
    return PFLB_OK;
}

void pfsur_destroy(pfsur_ctx* c) {
    if (!c) return;
    if (c->mem) (void)hipFree(c->mem);
    delete c;
}

const char* pfsur_last_error(const pfsur_ctx* c) {
    if (!c) return "no context (pfsur_create failed or was not called)";
    return c->err.c_str();
}

int pfsur_set_params(pfsur_ctx* c, const float* host) {
    if (!c) return PFLB_ERR_PARAM;
    if (!host) return fail(c, PFLB_ERR_PARAM, "NULL parameter array");
    for (size_t i = 0; i < PL.total; ++i)
        if (!isfinite(host[i])) return fail(c, PFLB_ERR_PARAM, "non-finite parameter");
    SUR_TRY(hipMemcpy(c->master, host, PL.total * 4, hipMemcpyHostToDevice), "parameter upload");
    SUR_TRY(hipMemset(c->m, 0, PL.total * 4), "adam reset");
    SUR_TRY(hipMemset(c->v, 0, PL.total * 4), "adam reset");
    c->t = 0;
    SUR_TRY(refresh_bf16(c, nullptr), "bf16 weights");
    SUR_TRY(hipDeviceSynchronize(), "parameter upload");
    return PFLB_OK;
}

int pfsur_get_params(pfsur_ctx* c, float* host) {
    if (!c) return PFLB_ERR_PARAM;
    if (!host) return fail(c, PFLB_ERR_PARAM, "NULL parameter array");
    SUR_TRY(hipDeviceSynchronize(), "parameter download");
    SUR_TRY(hipMemcpy(host, c->master, PL.total * 4, hipMemcpyDeviceToHost), "parameter download");
    return PFLB_OK;
}

size_t pfsur_workspace_bytes(const pfsur_cfg* cfg, int batch, int training) {
    if (!check_cfg(cfg).empty() || batch < 1 || batch > cfg->max_batch) return 0;
    return make_plan(cfg->H, cfg->W, batch, training != 0).total;
}

int pfsur_layer_io_of(const pfsur_cfg* cfg, int batch, int training, int layer,
                      pfsur_layer_io* out) {
    if (!out || !check_cfg(cfg).empty() || batch < 1 || batch > cfg->max_batch || layer < 0 ||
        layer >= NL)
        return PFLB_ERR_PARAM;
    const Plan p = make_plan(cfg->H, cfg->W, batch, training != 0);
    const LayerDef& L = LAYERS[layer];
    const size_t none = ~(size_t)0;
    memset(out, 0, sizeof(*out));
    if (L.pool_in >= 0) {          // the compact 2x2 averages the producing layer stored
        out->in_off = p.act[L.pool_in];
        out->in_cs = BUFS[L.pool_in].C;
        out->in_c0 = 0;
        out->in_mode = 2;
    } else {
        out->in_off = L.in_buf == X ? none : p.act[L.in_buf];
        out->in_cs = BUFS[L.in_buf].C;
        out->in_c0 = L.in_c0;
        out->in_mode = L.mode == MODE_UP ? 1 : 0;
    }
    out->out_off = p.act[L.out_buf];
    out->out_cs = BUFS[L.out_buf].C;
    out->out_c0 = L.out_c0;
    out->pool_off = L.pool_out >= 0 ? p.act[L.pool_out] : none;
    out->pool_cs = L.pool_out >= 0 ? BUFS[L.pool_out].C : 0;
    out->Cin = L.Cin;
    out->Cout = L.Cout;
    out->level = L.level;
    return PFLB_OK;
}

int pfsur_pack(pfsur_ctx* c, const float* phi, const float* P, const float* J, const double* rho,
               int batch, void* x, void* stream) {
    int r = check_batch(c, batch);
    if (r) return r;
    if (!phi || !P || !J || !rho || !x) return fail(c, PFLB_ERR_PARAM, "NULL pointer");
    if (!aligned16(x)) return fail(c, PFLB_ERR_ALIGN, "x must be 16-byte aligned");
    if (!dens_ok(rho, batch)) return fail(c, PFLB_ERR_PARAM, "densities must be finite and > 0");
    const size_t HW = (size_t)c->cfg.H * c->cfg.W;
    hipStream_t st = (hipStream_t)stream;
    for (int b0 = 0; b0 < batch; b0 += LRR_MAX) {
        const int nb = std::min(LRR_MAX, batch - b0);
        SUR_TRY(pack(phi + b0 * HW, P + b0 * HW, J + 2 * b0 * HW, dens_tab(rho, b0, nb), nb,
                     c->nm, HW, static_cast<__bf16*>(x) + b0 * HW * PFSUR_IN_CH, st),
                "pack");
    }
    return PFLB_OK;
}

int pfsur_pack_target(pfsur_ctx* c, const float* phi0, const float* P0, const float* J0,
                      const float* phi1, const float* P1, const float* J1, const double* rho,
                      int batch, float* y, void* stream) {
    int r = check_batch(c, batch);
    if (r) return r;
    if (!phi0 || !P0 || !J0 || !phi1 || !P1 || !J1 || !rho || !y)
        return fail(c, PFLB_ERR_PARAM, "NULL pointer");
    if (!aligned16(y)) return fail(c, PFLB_ERR_ALIGN, "y must be 16-byte aligned");
    if (!dens_ok(rho, batch)) return fail(c, PFLB_ERR_PARAM, "densities must be finite and > 0");
    const size_t HW = (size_t)c->cfg.H * c->cfg.W;
    hipStream_t st = (hipStream_t)stream;
    for (int b0 = 0; b0 < batch; b0 += LRR_MAX) {
        const int nb = std::min(LRR_MAX, batch - b0);
        SUR_TRY(pack_target(phi0 + b0 * HW, P0 + b0 * HW, J0 + 2 * b0 * HW, phi1 + b0 * HW,
                            P1 + b0 * HW, J1 + 2 * b0 * HW, dens_tab(rho, b0, nb), nb, c->nm, HW,
                            y + b0 * HW * PFSUR_OUT_CH, st),
                "pack target");
    }
    return PFLB_OK;
}

int pfsur_forward(pfsur_ctx* c, const void* x, float* out, int batch, void* workspace,
                  void* stream) {
    int r = check_batch(c, batch);
    if (r) return r;
    r = check_io(c, x, out, workspace);
    if (r) return r;
    return run_forward(c, x, out, batch, static_cast<char*>(workspace), false,
                       (hipStream_t)stream);
}

int pfsur_apply(pfsur_ctx* c, const float* out, float* phi, float* P, float* J,
                const double* rho, int batch, void* stream) {
    int r = check_batch(c, batch);
    if (r) return r;
    if (!out || !phi || !P || !J || !rho) return fail(c, PFLB_ERR_PARAM, "NULL pointer");
    if (!dens_ok(rho, batch)) return fail(c, PFLB_ERR_PARAM, "densities must be finite and > 0");
    const size_t HW = (size_t)c->cfg.H * c->cfg.W;
    for (int b0 = 0; b0 < batch; b0 += LRR_MAX) {
        const int nb = std::min(LRR_MAX, batch - b0);
        SUR_TRY(apply(out + b0 * HW * PFSUR_OUT_CH, c->nm, dens_tab(rho, b0, nb), nb, HW,
                      phi + b0 * HW, P + b0 * HW, J + 2 * b0 * HW, (hipStream_t)stream),
                "apply");
    }
    return PFLB_OK;
}

int pfsur_train_step(pfsur_ctx* c, const void* x, const float* y, int batch, float lr,
                     float* loss, void* workspace, void* stream) {
    int r = check_batch(c, batch);
    if (r) return r;
    r = check_io(c, x, y, workspace);
    if (r) return r;
    if (!(lr >= 0.0f) || !isfinite(lr)) return fail(c, PFLB_ERR_PARAM, "lr must be finite and >= 0");
    hipStream_t st = (hipStream_t)stream;
    r = forward_backward(c, x, y, batch, loss, static_cast<char*>(workspace), st);
    if (r) return r;
    c->t += 1;
    SUR_TRY(adam(c->master, c->grad, c->m, c->v, PL.total, lr, c->t, st), "adam");
    SUR_TRY(refresh_bf16(c, st), "bf16 weights");
    return PFLB_OK;
}

int pfsur_gradients(pfsur_ctx* c, const void* x, const float* y, int batch, float* host_grad,
                    float* loss, void* workspace, void* stream) {
    int r = check_batch(c, batch);
    if (r) return r;
    r = check_io(c, x, y, workspace);
    if (r) return r;
    if (!host_grad) return fail(c, PFLB_ERR_PARAM, "NULL gradient array");
    hipStream_t st = (hipStream_t)stream;
    r = forward_backward(c, x, y, batch, loss, static_cast<char*>(workspace), st);
    if (r) return r;
    SUR_TRY(hipMemcpyAsync(host_grad, c->grad, PL.total * 4, hipMemcpyDeviceToHost, st),
            "gradient read-back");
    SUR_TRY(hipStreamSynchronize(st), "gradient read-back");
    return PFLB_OK;
}

int pfsur_guard_accept(double sum_in, double sum_out, double mass_tol, double speed,
                       double u_max, int checked, double phi_err, double phi_tol) {
    if (!isfinite(sum_in) || !isfinite(sum_out)) return 0;
    if (!(fabs(sum_out - sum_in) <= mass_tol * fabs(sum_in))) return 0;
    if (!(speed <= u_max)) return 0;
    if (checked && !(phi_err <= phi_tol)) return 0;
    return 1;
}

}  // extern "C"

namespace {

constexpr int GUARD_BLOCKS = 256;

struct GuardPlan {
    size_t phi, P, J, phi_lb, x, out, ws, recon, dpart, fpart, upart, total;
};

// dpart holds the per-block sums before and after the prediction ([2][n][blocks]), fpart
// the per-block phi differences of checked windows and upart the per-block largest
// predicted speeds (both [n][blocks]), so that one read-back per window serves every
// decision
GuardPlan guard_plan(const pfsur_cfg* cfg, int n) {
    GuardPlan g;
    const size_t HW = (size_t)cfg->H * cfg->W;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes);
        return r;
    };
    g.phi = take(n * HW * 4);
    g.P = take(n * HW * 4);
    g.J = take(n * 2 * HW * 4);
    g.phi_lb = take(n * HW * 4);
    g.x = take(n * HW * PFSUR_IN_CH * 2);
    g.out = take(n * HW * PFSUR_OUT_CH * 4);
    g.ws = take(make_plan(cfg->H, cfg->W, n, false).total);
    g.recon = take((size_t)std::min(n, pflb::BATCH_MAX) * 2 * 9 * HW * 4);
    g.dpart = take((size_t)2 * n * GUARD_BLOCKS * 8);
    g.fpart = take((size_t)n * GUARD_BLOCKS * 4);
    g.upart = take((size_t)n * GUARD_BLOCKS * 4);
    g.total = o;
    return g;
}

}  // namespace

extern "C" {

size_t pfsur_guard_work_bytes(const pfsur_cfg* cfg, int batch) {
    if (!check_cfg(cfg).empty() || batch < 1 || batch > cfg->max_batch) return 0;
    return guard_plan(cfg, batch).total;
}

int pflb_advance_guarded(pflb_ctx* const* lbs, int n, pfsur_ctx* c, int windows,
                         double mass_tol, double phi_tol, double u_max, int check_every,
                         int* n_fallback, void* work, void* stream) {
    return pflb_advance_guarded_trace(lbs, n, c, windows, mass_tol, phi_tol, u_max,
                                      check_every, n_fallback, nullptr, work, stream);
}

int pflb_advance_guarded_trace(pflb_ctx* const* lbs, int n, pfsur_ctx* c, int windows,
                               double mass_tol, double phi_tol, double u_max, int check_every,
                               int* n_fallback, double* trace, void* work, void* stream) {
    if (!c) return PFLB_ERR_PARAM;
    if (!lbs || !work || !n_fallback) return fail(c, PFLB_ERR_PARAM, "NULL pointer");
    if (n < 1 || n > c->cfg.max_batch) return fail(c, PFLB_ERR_PARAM, "batch must be in [1, max_batch]");
    if (((uintptr_t)work & 255u)) return fail(c, PFLB_ERR_ALIGN, "work must be 256-byte aligned");
    if (windows < 0 || check_every < 0) return fail(c, PFLB_ERR_PARAM, "negative count");
    std::vector<double> rho(2 * (size_t)n);   // (rho_L, rho_H) of each context
    std::vector<float> beta(n);               // 1 where the context uses Eq. 13
    for (int k = 0; k < n; ++k) {
        pflb::CtxInfo info;
        if (!lbs[k] || pflb_ctx_info(lbs[k], &info) != PFLB_OK || !info.bound)
            return fail(c, PFLB_ERR_UNBOUND, "lattice context missing or not bound");
        if (info.q != 9 || info.nx != c->cfg.W || info.ny != c->cfg.H ||
            info.bc[0] != PFLB_BC_PERIODIC || info.bc[1] != PFLB_BC_PERIODIC)
            return fail(c, PFLB_ERR_PARAM, "lattices must be D2Q9, periodic, nx = W, ny = H");
        rho[2 * k] = info.rho_L;
        rho[2 * k + 1] = info.rho_H;
        beta[k] = info.hoc ? 1.0f : 0.0f;
    }
    hipStream_t st = (hipStream_t)stream;
    const GuardPlan g = guard_plan(&c->cfg, n);
    char* w = static_cast<char*>(work);
    const size_t HW = (size_t)c->cfg.H * c->cfg.W;
    float* phi = reinterpret_cast<float*>(w + g.phi);
    float* P = reinterpret_cast<float*>(w + g.P);
    float* J = reinterpret_cast<float*>(w + g.J);
    float* phi_lb = reinterpret_cast<float*>(w + g.phi_lb);
    float* out = reinterpret_cast<float*>(w + g.out);
    double* dpart = reinterpret_cast<double*>(w + g.dpart);
    float* fpart = reinterpret_cast<float*>(w + g.fpart);
    float* upart = reinterpret_cast<float*>(w + g.upart);
    const size_t nb = (size_t)n * GUARD_BLOCKS;
    std::vector<double> hd(2 * nb);
    std::vector<float> hf(nb), hu(nb);
    // per-context field pointers of the batched read-out and hand-over
    std::vector<float*> fphi(n), fP(n), fJ(n), flb(n);
    for (int k = 0; k < n; ++k) {
        fphi[k] = phi + k * HW;
        fP[k] = P + k * HW;
        fJ[k] = J + 2 * k * HW;
        flb[k] = phi_lb + k * HW;
    }
    std::vector<double> s_ref(n, 0.0);        // sum(phi) of each context at the start
    std::vector<pflb_ctx*> acc_ctx, rej_ctx;
    std::vector<const float*> acc_phi, acc_P, acc_J;
    auto lb_fail = [&](int r, pflb_ctx* lc, const char* what) {
        return fail(c, r, std::string(what) + pflb_last_error(lc));
    };
    *n_fallback = 0;
    for (int win = 0; win < windows; ++win) {
        int r;
        if ((r = pflb_read_many(lbs, n, fphi.data(), fP.data(), fJ.data(), st)))
            return lb_fail(r, lbs[0], "lattice read: ");
        SUR_TRY(sum_field(phi, n, HW, dpart, GUARD_BLOCKS, st), "field sum");
        if ((r = pfsur_pack(c, phi, P, J, rho.data(), n, w + g.x, st))) return r;
        if ((r = run_forward(c, w + g.x, out, n, w + g.ws, false, st))) return r;
        if ((r = pfsur_apply(c, out, phi, P, J, rho.data(), n, st))) return r;
        SUR_TRY(sum_field(phi, n, HW, dpart + nb, GUARD_BLOCKS, st), "field sum");
        for (int k0 = 0; k0 < n; k0 += LRR_MAX) {
            // the speed the hand-over would give (u = J / rho', rho' of Eq. 13)
            const int nk = std::min(LRR_MAX, n - k0);
            DensTab d = dens_tab(rho.data(), k0, nk);
            for (int k = 0; k < nk; ++k) d.beta[k] = beta[k0 + k];
            SUR_TRY(maxspeed(phi + k0 * HW, J + 2 * k0 * HW, d, nk, c->cfg.H, c->cfg.W,
                             upart + (size_t)k0 * GUARD_BLOCKS, GUARD_BLOCKS, st),
                    "speed check");
        }
        SUR_TRY(hipMemcpyAsync(hu.data(), upart, nb * 4, hipMemcpyDeviceToHost, st),
                "speed check");
        const bool checked = check_every > 0 && (win + 1) % check_every == 0;
        if (checked) {
            // the plain steps from the same states are the reference; if a prediction
            // is rejected they are the fallback already taken
            if ((r = pflb_step_many(lbs, n, PFSUR_STEPS, st)))
                return lb_fail(r, lbs[0], "lattice steps: ");
            if ((r = pflb_read_many(lbs, n, flb.data(), nullptr, nullptr, st)))
                return lb_fail(r, lbs[0], "lattice read: ");
            SUR_TRY(maxdiff(phi, phi_lb, n, HW, fpart, GUARD_BLOCKS, st), "phi check");
            SUR_TRY(hipMemcpyAsync(hf.data(), fpart, nb * 4, hipMemcpyDeviceToHost, st),
                    "phi check");
        }
        SUR_TRY(hipMemcpyAsync(hd.data(), dpart, 2 * nb * 8, hipMemcpyDeviceToHost, st),
                "field sums");
        SUR_TRY(hipStreamSynchronize(st), "guard read-back");
        // a context whose state is non-finite at the window's start ends the call before
        // any prediction is handed over or any fallback taken; on a checked window every
        // context has already taken the window's plain steps (the reference) by then
        for (int k = 0; k < n; ++k) {
            double s_in = 0.0;
            for (int b = 0; b < GUARD_BLOCKS; ++b) s_in += hd[(size_t)k * GUARD_BLOCKS + b];
            if (!isfinite(s_in))
                return fail(c, PFLB_ERR_NONFINITE,
                            "lattice state of context " + std::to_string(k) + " is non-finite");
            if (win == 0) s_ref[k] = s_in;
        }
        acc_ctx.clear();
        acc_phi.clear();
        acc_P.clear();
        acc_J.clear();
        rej_ctx.clear();
        for (int k = 0; k < n; ++k) {
            // fixed-order host sums of the per-block partials (deterministic)
            double s_in = 0.0, s_out = 0.0, err = 0.0, speed = 0.0;
            for (int b = 0; b < GUARD_BLOCKS; ++b) {
                s_in += hd[(size_t)k * GUARD_BLOCKS + b];
                s_out += hd[nb + (size_t)k * GUARD_BLOCKS + b];
                const float e = hu[(size_t)k * GUARD_BLOCKS + b];
                speed = e > speed || e != e ? e : speed;
            }
            if (speed != speed) speed = INFINITY;
            if (checked) {
                for (int b = 0; b < GUARD_BLOCKS; ++b) {
                    const float e = hf[(size_t)k * GUARD_BLOCKS + b];
                    err = e > err || e != e ? e : err;
                }
                if (err != err) err = INFINITY;
            }
            // the mass test is against the sum at the start of the call, which the method
            // conserves: accepted windows cannot add up to a drift beyond mass_tol
            const int ok =
                pfsur_guard_accept(s_ref[k], s_out, mass_tol, speed, u_max, checked, err, phi_tol);
            if (trace) {
                double* t = trace + ((size_t)win * n + k) * PFSUR_TRACE_FIELDS;
                t[0] = s_ref[k];
                t[1] = s_in;
                t[2] = s_out;
                t[3] = speed;
                t[4] = checked ? err : NAN;
                t[5] = ok;
            }
            if (ok) {
                acc_ctx.push_back(lbs[k]);
                acc_phi.push_back(fphi[k]);
                acc_P.push_back(fP[k]);
                acc_J.push_back(fJ[k]);
            } else {
                *n_fallback += 1;
                if (!checked) rej_ctx.push_back(lbs[k]);
            }
        }
        if (!rej_ctx.empty() &&
            (r = pflb_step_many(rej_ctx.data(), (int)rej_ctx.size(), PFSUR_STEPS, st)))
            return lb_fail(r, rej_ctx[0], "fallback steps: ");
        if (!acc_ctx.empty() &&
            (r = pflb_reconstruct_many(acc_ctx.data(), (int)acc_ctx.size(), acc_phi.data(),
                                             acc_P.data(), acc_J.data(),
                                             reinterpret_cast<float*>(w + g.recon),
                                             checked ? 0 : PFSUR_STEPS, st)))
            return lb_fail(r, acc_ctx[0], "hand-over: ");
    }
    SUR_TRY(hipStreamSynchronize(st), "guarded advance");
    return PFLB_OK;
}

int pfsur_save(pfsur_ctx* c, const char* path) {
    if (!c) return PFLB_ERR_PARAM;
    if (!path) return fail(c, PFLB_ERR_PARAM, "NULL path");
    std::vector<float> host(3 * PL.total);
    SUR_TRY(hipDeviceSynchronize(), "checkpoint");
    SUR_TRY(hipMemcpy(host.data(), c->master, PL.total * 4, hipMemcpyDeviceToHost), "checkpoint");
    SUR_TRY(hipMemcpy(host.data() + PL.total, c->m, PL.total * 4, hipMemcpyDeviceToHost), "checkpoint");
    SUR_TRY(hipMemcpy(host.data() + 2 * PL.total, c->v, PL.total * 4, hipMemcpyDeviceToHost),
            "checkpoint");
    SurHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, "PFSURCK1", 8);
    h.H = c->cfg.H;
    h.W = c->cfg.W;
    h.nparams = PL.total;
    h.t = c->t;
    FILE* f = fopen(path, "wb");
    if (!f) return fail(c, PFLB_ERR_IO, std::string("cannot open ") + path);
    bool ok = fwrite(&h, sizeof(h), 1, f) == 1 &&
              fwrite(host.data(), 4, host.size(), f) == host.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(c, PFLB_ERR_IO, std::string("cannot write ") + path);
    return PFLB_OK;
}

int pfsur_load(pfsur_ctx* c, const char* path) {
    if (!c) return PFLB_ERR_PARAM;
    if (!path) return fail(c, PFLB_ERR_PARAM, "NULL path");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(c, PFLB_ERR_IO, std::string("cannot open ") + path);
    SurHeader h;
    std::vector<float> host(3 * PL.total);
    bool ok = fread(&h, sizeof(h), 1, f) == 1;
    if (ok && (memcmp(h.magic, "PFSURCK1", 8) != 0 || h.nparams != PL.total)) {
        fclose(f);
        return fail(c, PFLB_ERR_PARAM, "not a checkpoint of this network");
    }
    ok = ok && fread(host.data(), 4, host.size(), f) == host.size();
    fclose(f);
    if (!ok) return fail(c, PFLB_ERR_IO, "short checkpoint");
    SUR_TRY(hipMemcpy(c->master, host.data(), PL.total * 4, hipMemcpyHostToDevice), "restore");
    SUR_TRY(hipMemcpy(c->m, host.data() + PL.total, PL.total * 4, hipMemcpyHostToDevice), "restore");
    SUR_TRY(hipMemcpy(c->v, host.data() + 2 * PL.total, PL.total * 4, hipMemcpyHostToDevice),
            "restore");
    c->t = h.t;
    SUR_TRY(refresh_bf16(c, nullptr), "bf16 weights");
    SUR_TRY(hipDeviceSynchronize(), "restore");
    return PFLB_OK;
}

// ----- stateless building blocks -----

static int conv_shape_ok(int batch, int H, int W, int Cin, int Cout, int mode) {
    if (batch < 1 || H < 1 || W < 1 || Cin < 8 || Cin % 8 || Cout < 1) return 0;
    if (mode < MODE_SAME || mode > MODE_POOL) return 0;
    if (mode == MODE_UP && (H % 2 || W % 2)) return 0;
    if ((double)batch * H * W > 67108864.0) return 0;
    return 1;
}

static GatherP plain_gather(const void* x, int H, int W, int Cin, int mode) {
    GatherP g;
    g.p = static_cast<const __bf16*>(x);
    g.Hin = mode == MODE_POOL ? 2 * H : (mode == MODE_UP ? H / 2 : H);
    g.Win = mode == MODE_POOL ? 2 * W : (mode == MODE_UP ? W / 2 : W);
    g.cs = Cin;
    g.c0 = 0;
    g.C = Cin;
    g.mode = mode;
    return g;
}

int pfsur_conv_fwd(const void* x, int batch, int H, int W, int Cin, int Cout, int mode,
                   const void* w, const float* b, int act, float* y_pre, void* y_act,
                   void* stream) {
    if (!conv_shape_ok(batch, H, W, Cin, Cout, mode) || !x || !w) return PFLB_ERR_PARAM;
    if (!aligned16(x) || !aligned16(w)) return PFLB_ERR_ALIGN;
    ConvP a;
    memset(&a, 0, sizeof(a));
    a.g = plain_gather(x, H, W, Cin, mode);
    a.B = batch;
    a.H = H;
    a.W = W;
    a.w = static_cast<const __bf16*>(w);
    a.Cout = Cout;
    a.bias = b;
    a.act = act ? 1 : 0;
    a.out = static_cast<__bf16*>(y_act);
    a.out_cs = Cout;
    a.fout = y_pre;
    a.f_cs = Cout;
    return conv3x3(a, (hipStream_t)stream) == hipSuccess ? PFLB_OK : PFLB_ERR_DEVICE;
}

size_t pfsur_conv_wgrad_work_bytes(int batch, int H, int W, int Cin, int Cout) {
    if (!conv_shape_ok(batch, H, W, Cin, Cout, MODE_SAME)) return 0;
    return wgrad_part_floats(batch, H, W, Cout, Cin) * 4;
}

int pfsur_conv_wgrad(const void* x, const void* dy, int batch, int H, int W, int Cin, int Cout,
                     int mode, float* dw, float* db, void* work, void* stream) {
    if (!conv_shape_ok(batch, H, W, Cin, Cout, mode) || Cout % 8 || !x || !dy || !dw || !work)
        return PFLB_ERR_PARAM;
    if (!aligned16(x) || !aligned16(dy)) return PFLB_ERR_ALIGN;
    hipStream_t st = (hipStream_t)stream;
    const int P = batch * H * W;
    WgradP a;
    a.g = plain_gather(x, H, W, Cin, mode);
    a.B = batch;
    a.H = H;
    a.W = W;
    a.dz = static_cast<const __bf16*>(dy);
    a.Cout = Cout;
    int per;
    const int ns = wgrad_nsplit(batch, H, W, Cout, Cin, &per);
    a.part = static_cast<float*>(work);
    if (wgrad(a, st) != hipSuccess) return PFLB_ERR_DEVICE;
    if (reduce_splits(a.part, ns, (size_t)Cout * 9 * Cin, dw, 0, st) != hipSuccess)
        return PFLB_ERR_DEVICE;
    if (db) {
        if (colsum(a.dz, P, Cout, COLSUM_PX, a.part, st) != hipSuccess) return PFLB_ERR_DEVICE;
        if (reduce_splits(a.part, (P + COLSUM_PX - 1) / COLSUM_PX, Cout, db, 0, st) != hipSuccess)
            return PFLB_ERR_DEVICE;
    }
    return PFLB_OK;
}

}  // extern "C"
