// C-ABI layer of the phase-field lattice Boltzmann library: parameter validation and
// derivation, buffer binding, launch orchestration, read-out, checkpointing.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pflb.h"
#include "pflb_internal.hpp"

using namespace pflb;

struct pflb_ctx {
    pflb_params p;
    int Q = 0, D = 0;
    uint32_t N = 0;
    Launch L{};
    void* buf[PFLB_NBUF] = {nullptr, nullptr, nullptr};
    size_t bytes[PFLB_NBUF] = {0, 0, 0};
    bool bound = false;
    int cur = 0;              // state buffer holding the current state
    long long steps = 0;
    std::string err;
    // pflb_step_graph: instantiated graphs of `graph_n` steps starting from state buffer
    // 0 or 1 (the launches alternate buffers, so the start decides every launch)
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_n = 0;
    void drop_graphs() {
        for (auto& g : graph)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
        graph_n = 0;
    }
    ~pflb_ctx() { drop_graphs(); }
};

namespace {

const double kT = 1.0 / 3.0;

bool finite(double v) { return isfinite(v) != 0; }

// Returns an empty string if p is valid, else the reason.
std::string check_params(const pflb_params* p) {
    if (!p) return "params is NULL";
    if (p->lattice != 9 && p->lattice != 19) return "lattice must be 9 or 19";
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "nx, ny, nz must be >= 1";
    if (p->lattice == 9 && p->nz != 1) return "D2Q9 needs nz = 1";
    const double n = (double)p->nx * p->ny * p->nz;
    // site indices are 32-bit (beyond 2^28 - 64 sites the kernels form 64-bit addresses)
    if (n > 4294967296.0 - 64.0) return "domain larger than 2^32 - 64 sites";
    for (int a = 0; a < 3; ++a)
        if (p->bc[a] != PFLB_BC_PERIODIC && p->bc[a] != PFLB_BC_WALL) return "bc must be 0 or 1";
    if (!(finite(p->rho_L) && p->rho_L > 0) || !(finite(p->rho_H) && p->rho_H > 0))
        return "densities must be finite and > 0";
    if (!(finite(p->nu_L) && p->nu_L > 0) || !(finite(p->nu_H) && p->nu_H > 0))
        return "viscosities must be > 0 (tau = nu/T + 1/2 > 1/2)";
    if (!(finite(p->M) && p->M > 0)) return "mobility M must be > 0";
    if (!(finite(p->W) && p->W > 0)) return "interface thickness W must be > 0";
    if (!(finite(p->sigma) && p->sigma >= 0)) return "sigma must be >= 0";
    if (!(finite(p->eps) && p->eps > 0)) return "eps must be > 0";
    for (int a = 0; a < 3; ++a)
        if (!finite(p->g[a])) return "gravity must be finite";
    if (p->hoc != 0 && p->hoc != 1) return "hoc must be 0 or 1";
    if (!finite(p->dtheta_C)) return "dtheta_C must be finite";
    if (p->storage != PFLB_STORE_FP32 && p->storage != PFLB_STORE_FP16S &&
        p->storage != PFLB_STORE_FP32_INPLACE)
        return "storage must be PFLB_STORE_FP32, PFLB_STORE_FP16S or PFLB_STORE_FP32_INPLACE";
    if (p->storage == PFLB_STORE_FP16S)
        for (int k = 0; k < 2; ++k)
            if (p->scale_log2[k] < -14 || p->scale_log2[k] > 24) return "scale_log2 out of [-14, 24]";
    const int naxes = p->lattice == 9 ? 2 : 3;
    for (int f = 0; f < 6; ++f)
        for (int a = 0; a < 3; ++a) {
            const double v = p->wall_u[f][a];
            if (!finite(v)) return "wall velocities must be finite";
            if (v == 0.0) continue;
            const int axis = f / 2;
            if (axis >= naxes || a >= naxes) return "wall velocity on an axis the lattice does not have";
            if (p->bc[axis] != PFLB_BC_WALL) return "wall velocity given for a face of a periodic axis";
            if (a == axis) return "a wall moves tangentially: its normal velocity must be 0";
        }
    for (int f = 0; f < 6; ++f) {
        const double v = p->wet_cos[f];
        if (!finite(v) || v < -1.0 || v > 1.0) return "wet_cos must be finite and in [-1, 1]";
        if (v == 0.0) continue;
        const int axis = f / 2;
        if (axis >= naxes) return "contact angle on an axis the lattice does not have";
        if (p->bc[axis] != PFLB_BC_WALL) return "contact angle given for a face of a periodic axis";
    }
    bool any_open = false, any_moving = false;
    for (int f = 0; f < 6; ++f)
        for (int a = 0; a < 3; ++a) any_moving = any_moving || p->wall_u[f][a] != 0.0;
    for (int f = 0; f < 6; ++f) {
        if (p->open[f] != 0 && p->open[f] != 1) return "open must be 0 or 1";
        if (!p->open[f]) continue;
        any_open = true;
        const int axis = f / 2;
        if (axis >= naxes) return "open face on an axis the lattice does not have";
        if (p->bc[axis] != PFLB_BC_WALL) return "an open face must be on a wall axis";
        const int len = axis == 0 ? p->nx : (axis == 1 ? p->ny : p->nz);
        if (len < 2) return "an open face needs at least 2 sites along its axis";
        if (!finite(p->open_P[f])) return "open-face pressure must be finite";
        if (p->wet_cos[f] != 0.0) return "a contact angle given for an open face";
    }
    if (any_open && any_moving) return "moving walls and open faces together are not supported";
    if (p->storage == PFLB_STORE_FP32_INPLACE && any_open)
        return "in-place storage has no open faces";
    return "";
}

bool has_open(const pflb_params* p) {
    for (int f = 0; f < 6; ++f)
        if (p->open[f]) return true;
    return false;
}

uint32_t pop_stride(uint32_t N) { return (N + 63u) & ~63u; }

// the pressures of the boundary layers of the open faces: one float per site of a face's
// layer, six layers of stride side_stride (the largest face, rounded up)
uint32_t side_stride(const pflb_params* p) {
    // internal sizes (D2Q9: user (x, y) -> internal (x, z))
    const uint64_t nx = (uint64_t)p->nx, ny = p->lattice == 9 ? 1 : (uint64_t)p->ny,
                   nz = p->lattice == 9 ? (uint64_t)p->ny : (uint64_t)p->nz;
    const uint64_t layer = std::max(ny * nz, std::max(nx * nz, nx * ny));
    return (uint32_t)((layer + 63u) & ~(uint64_t)63u);
}

size_t side_offset(const pflb_params* p, uint32_t N) {
    const size_t b = state_bytes(p->lattice, p->storage == PFLB_STORE_FP16S, pop_stride(N));
    return (b + 255) & ~(size_t)255;
}

size_t set_bytes(const pflb_params* p, uint32_t N) {
    if (!has_open(p))
        return state_bytes(p->lattice, p->storage == PFLB_STORE_FP16S, pop_stride(N));
    return side_offset(p, N) + 6 * (size_t)side_stride(p) * 4;
}

size_t scratch_bytes() {
    const size_t b = mass_scratch_bytes();
    return (b + 65535) & ~(size_t)65535;
}

// in-place storage: the phi field follows the reduction scratch
size_t scratch_bytes(const pflb_params* p, uint32_t N) {
    if (p->storage != PFLB_STORE_FP32_INPLACE) return scratch_bytes();
    return scratch_bytes() + (size_t)pop_stride(N) * 4;
}

bool inplace(const pflb_params* p) { return p->storage == PFLB_STORE_FP32_INPLACE; }

uint32_t sites(const pflb_params* p) { return (uint32_t)p->nx * p->ny * p->nz; }

// Planes per workgroup of the fused step for nctx contexts of one launch.
// D3Q19: a CU runs its share of the B workgroups, each marching bz planes and
// re-gathering two more, so the critical path is ceil(B / CUs) (bz + 2) planes; at least
// two workgroups per CU are needed to hide the gathers' latency.  bz minimises that path
// among the choices that give two per CU (else the most workgroups).  This reproduces
// every measured optimum: 128^3 16 planes (8 and 32 slower), 256x256x128 64 (16, 32
// slower), 256^3 128, and 192^3, where 48 planes (576 workgroups, 2.25 per CU) measured
// 16% slower than 16.  Where even whole columns give more than two workgroups per CU
// (several rounds of workgroups whatever bz), long marches let the running workgroups
// drift apart in z and touch many more pages at once: there 16 planes, which keeps
// them within a few planes of each other.  Measured against the model's choice, FP32
// (FP16S): 1000x1000x268 24% faster, the best of eight plane counts (0.7% slower);
// 512x512x256 2.6% (5.8%) and 384^3 2% faster (3.6% slower); 512^3 11% (4.4%) faster;
// 448^3 8% (9%) slower, where the model's 56 planes were the best of four.  On average
// 7% faster in FP32 and neutral in FP16S; no single count is best everywhere.
// D2Q9 (one-wave workgroups): about 2048 workgroups, at most 4 planes.  Measured: 256x1024
// Rayleigh-Taylor, 2 planes beat 1, 4 and 8 (1.6x over 8); a lone 256x256 domain runs
// best with 1 (small 2-D domains need the parallelism more than they lose to the
// re-gathered planes); 16 256x256 domains in one launch step fastest with 4 (FP32 8%
// faster than 8, 1.9x faster than 32).
int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
        return 256;
    return n;
}

int pick_bz(const Geom& G, int lattice, int nctx) {
    const char* env = getenv("PFLB_BZ");
    if (env && atoi(env) > 0) return atoi(env);
    const long nz = G.nz;
    if (lattice == 19) {
        const long cols = (long)((G.nx + 63) / 64) * ((G.ny + 3) / 4) * nctx;
        const long cus = device_cus();
        if (cols > 2 * cus) return (int)(nz < 16 ? nz : 16);
        long best = nz, best_cost = -1;
        bool best_enough = false;
        long prev_chunks = -1;
        for (long bz = (nz < 8 ? nz : 8); bz <= nz; ++bz) {
            const long chunks = (nz + bz - 1) / bz;
            if (chunks == prev_chunks) continue;           // same split, longer chunks
            prev_chunks = chunks;
            const long B = cols * chunks;
            const bool enough = B >= 2 * cus;
            const long cost = ((B + cus - 1) / cus) * (bz + 2);
            if (best_cost < 0 || (enough && !best_enough) ||
                (enough == best_enough && (enough ? cost < best_cost : false))) {
                best = bz;
                best_cost = cost;
                best_enough = enough;
            }
        }
        return (int)best;
    }
    const long cols = (long)((G.nx + 63) / 64) * nctx;
    long chunks = (2048 + cols - 1) / cols;
    if (chunks < 1) chunks = 1;
    long bz = (nz + chunks - 1) / chunks;
    if (bz < 1) bz = 1;
    if (bz > 4) bz = 4;
    if (bz > nz) bz = nz;
    return (int)bz;
}

void derive(pflb_ctx* c) {
    const pflb_params& p = c->p;
    c->Q = p.lattice;
    c->D = p.lattice == 19 ? 3 : 2;
    c->N = sites(&p);
    Geom& G = c->L.G;
    if (p.lattice == 19) {
        G.nx = p.nx; G.ny = p.ny; G.nz = p.nz;
        G.wx = p.bc[0]; G.wy = p.bc[1]; G.wz = p.bc[2];
    } else {  // user (x, y) -> internal (x, z)
        G.nx = p.nx; G.ny = 1; G.nz = p.ny;
        G.wx = p.bc[0]; G.wy = 0; G.wz = p.bc[1];
    }
    G.S = pop_stride(c->N);
    G.sxy = (uint32_t)G.nx * (uint32_t)G.ny;
    G.open = 0;
    for (int f = 0; f < 6; ++f) {
        const int fi = p.lattice == 19 ? f : (f < 2 ? f : (f < 4 ? f + 2 : -1));
        if (fi >= 0 && p.open[f]) G.open |= 1u << fi;
    }
    G.SL = side_stride(&p);
    G.side_off = side_offset(&p, c->N);
    Model& m = c->L.m;
    const double tau_L = p.nu_L / kT + 0.5, tau_H = p.nu_H / kT + 0.5;
    const double tau_phi = p.M / kT + 0.5;
    m.rho_L = (float)p.rho_L;
    m.rho_dif = (float)(p.rho_H - p.rho_L);
    m.itau_L = (float)(1.0 / tau_L);
    m.itau_dif = (float)(1.0 / tau_H - 1.0 / tau_L);
    m.om_phi = (float)(1.0 / tau_phi);
    m.mu_a = (float)(48.0 * p.sigma / p.W);
    m.mu_b = (float)(1.5 * p.sigma * p.W);
    m.th_a = (float)(p.M / kT / p.W);
    m.dth = (float)(p.dtheta_C * p.M / kT);
    m.eps = (float)p.eps;
    if (p.lattice == 19) {
        m.gx = (float)p.g[0]; m.gy = (float)p.g[1]; m.gz = (float)p.g[2];
    } else {
        m.gx = (float)p.g[0]; m.gy = 0.0f; m.gz = (float)p.g[1];
    }
    m.beta = p.hoc ? 1.0f : 0.0f;
    for (int f = 0; f < 6; ++f) m.Pf[f] = 0.0f;
    for (int f = 0; f < 6; ++f) {
        const int fi = p.lattice == 19 ? f : (f < 2 ? f : (f < 4 ? f + 2 : -1));
        if (fi >= 0 && p.open[f]) m.Pf[fi] = (float)p.open_P[f];
    }
    // wall faces and velocity components in internal axes (D2Q9: user y is internal z)
    m.moving = 0;
    m.wetting = 0;
    for (int f = 0; f < 6; ++f) {
        for (int a = 0; a < 3; ++a) m.uw[f][a] = 0.0f;
        m.wk[f] = 0.0f;
    }
    for (int f = 0; f < 6; ++f) {
        const int fi = p.lattice == 19 ? f : (f < 2 ? f : (f < 4 ? f + 2 : -1));
        if (fi < 0) continue;
        m.wk[fi] = (float)(4.0 * p.wet_cos[f] / p.W);
        if (p.wet_cos[f] != 0.0) m.wetting = 1;
        for (int a = 0; a < 3; ++a) {
            const int ai = p.lattice == 19 ? a : (a == 0 ? 0 : (a == 1 ? 2 : -1));
            if (ai < 0) continue;
            m.uw[fi][ai] = (float)p.wall_u[f][a];
            if (p.wall_u[f][a] != 0.0) m.moving = 1;
        }
    }
    Codec& cd = c->L.cd;
    if (p.storage == PFLB_STORE_FP16S) {
        cd.sh = ldexpf(1.0f, p.scale_log2[0]);
        cd.ish = ldexpf(1.0f, -p.scale_log2[0]);
        cd.sg = ldexpf(1.0f, p.scale_log2[1]);
        cd.isg = ldexpf(1.0f, -p.scale_log2[1]);
    } else {
        cd.sh = cd.ish = cd.sg = cd.isg = 1.0f;
    }
    c->L.q = p.lattice;
    c->L.half = p.storage == PFLB_STORE_FP16S;
    c->L.inplace = p.storage == PFLB_STORE_FP32_INPLACE;
    c->L.tile = 0;
    const char* tenv = getenv("PFLB_TILE");
    if (tenv && atoi(tenv) >= 0 && atoi(tenv) <= 3) c->L.tile = atoi(tenv);
    c->L.bz = pick_bz(G, p.lattice, 1);
    c->L.wide = G.S > (1u << 28) - 64u;
}

int fail(pflb_ctx* c, int code, const std::string& what) {
    if (c) c->err = what;
    return code;
}

int hip_fail(pflb_ctx* c, hipError_t e, const char* where) {
    return fail(c, PFLB_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool aligned(const void* p) { return ((uintptr_t)p & 255u) == 0; }

int need_bound(pflb_ctx* c) {
    if (!c) return PFLB_ERR_PARAM;
    if (!c->bound) return fail(c, PFLB_ERR_UNBOUND, "buffers not bound");
    return PFLB_OK;
}

// In-place storage keeps its state in buffer 0 and `cur` is then its layout (the parity
// of the steps since the state was set).
void* state(pflb_ctx* c) {
    if (c->L.inplace) return c->buf[PFLB_BUF_STATE0];
    return c->buf[c->cur == 0 ? PFLB_BUF_STATE0 : PFLB_BUF_STATE1];
}
// the buffer a pull-storage step writes
void* other(pflb_ctx* c) { return c->buf[c->cur == 0 ? PFLB_BUF_STATE1 : PFLB_BUF_STATE0]; }
float* phi_field(pflb_ctx* c) {
    return reinterpret_cast<float*>(static_cast<char*>(c->buf[PFLB_BUF_SCRATCH]) + scratch_bytes());
}

// one step of context c on stream st from its current buffer or layout `cur`
hipError_t launch_one(pflb_ctx* c, const Launch& a, int cur) {
    if (c->L.inplace) return launch_step_inplace(a, c->buf[PFLB_BUF_STATE0], cur, phi_field(c));
    return launch_step(a, c->buf[cur == 0 ? PFLB_BUF_STATE0 : PFLB_BUF_STATE1],
                       c->buf[cur == 0 ? PFLB_BUF_STATE1 : PFLB_BUF_STATE0]);
}

struct FileHeader {
    char magic[8];
    int lattice, nx, ny, nz, bc[3], storage, scale_log2[2], hoc;
    double rho_L, rho_H, nu_L, nu_H, M, W, sigma, g[3], eps, dtheta_C;
    double wall_u[6][3], wet_cos[6];
    int open[6];
    double open_P[6];
    int layout;               // in-place storage: the layout of the saved state
    long long steps;
    unsigned long long set_bytes;
};

void fill_header(const pflb_ctx* c, FileHeader* h) {
    memset(h, 0, sizeof(*h));
    memcpy(h->magic, "PFLBCK05", 8);
    const pflb_params& p = c->p;
    h->lattice = p.lattice; h->nx = p.nx; h->ny = p.ny; h->nz = p.nz;
    for (int a = 0; a < 3; ++a) { h->bc[a] = p.bc[a]; h->g[a] = p.g[a]; }
    h->storage = p.storage;
    h->scale_log2[0] = p.storage == PFLB_STORE_FP16S ? p.scale_log2[0] : 0;
    h->scale_log2[1] = p.storage == PFLB_STORE_FP16S ? p.scale_log2[1] : 0;
    h->hoc = p.hoc;
    h->rho_L = p.rho_L; h->rho_H = p.rho_H; h->nu_L = p.nu_L; h->nu_H = p.nu_H;
    h->M = p.M; h->W = p.W; h->sigma = p.sigma; h->eps = p.eps; h->dtheta_C = p.dtheta_C;
    for (int f = 0; f < 6; ++f) {
        for (int a = 0; a < 3; ++a) h->wall_u[f][a] = p.wall_u[f][a];
        h->wet_cos[f] = p.wet_cos[f];
        h->open[f] = p.open[f];
        h->open_P[f] = p.open[f] ? p.open_P[f] : 0.0;
    }
    h->layout = c->L.inplace ? c->cur : 0;
    h->steps = c->steps;
    h->set_bytes = set_bytes(&c->p, c->N);
}

}  // namespace

extern "C" {

int pflb_create(const pflb_params* p, pflb_ctx** out) {
    if (!out) return PFLB_ERR_PARAM;
    *out = nullptr;
    if (!check_params(p).empty()) return PFLB_ERR_PARAM;
    pflb_ctx* c = new (std::nothrow) pflb_ctx();
    if (!c) return PFLB_ERR_NOMEM;
    c->p = *p;
    derive(c);
    c->bytes[PFLB_BUF_STATE0] = set_bytes(p, c->N);
    c->bytes[PFLB_BUF_STATE1] = inplace(p) ? 0 : set_bytes(p, c->N);
    c->bytes[PFLB_BUF_SCRATCH] = scratch_bytes(p, c->N);
    *out = c;
    return PFLB_OK;
}

void pflb_destroy(pflb_ctx* ctx) { delete ctx; }

const char* pflb_last_error(const pflb_ctx* ctx) {
    if (!ctx) return "no context (pflb_create failed or was not called)";
    return ctx->err.c_str();
}

size_t pflb_required_bytes(const pflb_params* p, int buffer) {
    if (!check_params(p).empty()) return 0;
    const uint32_t N = sites(p);
    switch (buffer) {
        case PFLB_BUF_STATE0:
            return set_bytes(p, N);
        case PFLB_BUF_STATE1:
            return inplace(p) ? 0 : set_bytes(p, N);
        case PFLB_BUF_SCRATCH:
            return scratch_bytes(p, N);
        default:
            return 0;
    }
}

int pflb_bind(pflb_ctx* c, void* const* dev_ptrs, int n) {
    if (!c) return PFLB_ERR_PARAM;
    if (!dev_ptrs || n != PFLB_NBUF) return fail(c, PFLB_ERR_PARAM, "pflb_bind needs PFLB_NBUF pointers");
    for (int k = 0; k < n; ++k) {
        if (!dev_ptrs[k] && c->bytes[k] == 0) continue;      // a buffer that needs no bytes
        if (!dev_ptrs[k]) return fail(c, PFLB_ERR_PARAM, "NULL buffer pointer");
        if (!aligned(dev_ptrs[k])) return fail(c, PFLB_ERR_ALIGN, "buffer not 256-byte aligned");
    }
    c->drop_graphs();         // captured launches name the previous buffers
    for (int k = 0; k < n; ++k) c->buf[k] = dev_ptrs[k];
    c->bound = true;
    c->cur = 0;
    return PFLB_OK;
}

int pflb_equilibrium(pflb_ctx* c, const float* phi, const float* u, const float* P,
                     float* h_out, float* g_out, void* stream) {
    if (!c) return PFLB_ERR_PARAM;
    if (!phi || !u || !h_out || !g_out) return fail(c, PFLB_ERR_PARAM, "NULL field pointer");
    Launch a = c->L;
    a.stream = (hipStream_t)stream;
    hipError_t e = launch_equilibrium(a, c->N, phi, u, P, h_out, g_out);
    if (e != hipSuccess) return hip_fail(c, e, "equilibrium launch");
    return PFLB_OK;
}

int pflb_set_state(pflb_ctx* c, const float* h, const float* g, void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (!h || !g) return fail(c, PFLB_ERR_PARAM, "NULL distribution pointer");
    Launch a = c->L;
    a.stream = (hipStream_t)stream;
    c->cur = 0;
    hipError_t e = c->L.inplace ? launch_set_state_inplace(a, c->N, h, g, state(c))
                                : launch_set_state(a, c->N, h, g, state(c));
    if (e != hipSuccess) return hip_fail(c, e, "set_state launch");
    c->steps = 0;
    return PFLB_OK;
}

int pflb_get_state(pflb_ctx* c, float* h, float* g, void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (!h || !g) return fail(c, PFLB_ERR_PARAM, "NULL distribution pointer");
    Launch a = c->L;
    a.stream = (hipStream_t)stream;
    hipError_t e = c->L.inplace ? launch_get_state_inplace(a, c->N, state(c), c->cur, h, g)
                                : launch_get_state(a, c->N, state(c), h, g);
    if (e != hipSuccess) return hip_fail(c, e, "get_state launch");
    return PFLB_OK;
}

// In-place storage: layout 0 is the equilibrium kernel's output format with stride S,
// so the equilibria are written straight into the state (no staging, no work buffer).
static int init_inplace(pflb_ctx* c, const float* phi, const float* u, const float* P,
                        void* stream) {
    if (!phi || !u) return fail(c, PFLB_ERR_PARAM, "NULL field pointer");
    Launch a = c->L;
    a.stream = (hipStream_t)stream;
    float* h = static_cast<float*>(state(c));
    float* g = h + (size_t)c->Q * c->L.G.S;
    c->cur = 0;
    hipError_t e = launch_equilibrium(a, c->N, phi, u, P, h, g, c->L.G.S);
    if (e != hipSuccess) return hip_fail(c, e, "equilibrium launch");
    c->steps = 0;
    return PFLB_OK;
}

int pflb_init_fields(pflb_ctx* c, const float* phi, const float* u, const float* P, float* work,
                     void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (c->L.inplace) return init_inplace(c, phi, u, P, stream);
    if (!work) return fail(c, PFLB_ERR_PARAM, "NULL work buffer");
    float* h = work;
    float* g = work + (size_t)c->Q * c->N;
    r = pflb_equilibrium(c, phi, u, P, h, g, stream);
    if (r) return r;
    return pflb_set_state(c, h, g, stream);
}

// ---------------------------------------------------------------------------
// allocation-free start: the equilibria staged between the two kernels of
// pflb_init_fields (2 Q N floats) live in a fixed device array of this library instead
// of caller memory.  Each GPU the library runs on holds its own copy of the array from
// the first use of this code on that GPU until the process ends; its address on each
// device is looked up once, with that device current, and kept.
// ---------------------------------------------------------------------------
}  // extern "C"

static __device__ __align__(256) float scratch[PFLB_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (hipGetSymbolAddress once per device)
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t pflb_noalloc_scratch_bytes(void) { return PFLB_NOALLOC_SCRATCH_BYTES; }

int pflb_init_fields_noalloc(pflb_ctx* c, const float* phi, const float* u, const float* P,
                             void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (!phi || !u) return fail(c, PFLB_ERR_PARAM, "NULL field pointer");
    if (c->L.inplace) return init_inplace(c, phi, u, P, stream);
    const size_t need = (size_t)2 * c->Q * c->N * sizeof(float);
    if (need > (size_t)PFLB_NOALLOC_SCRATCH_BYTES)
        return fail(c, PFLB_ERR_PARAM,
                    "domain too large for the allocation-free start: it stages 2*Q*N floats (" +
                        std::to_string(need) + " bytes) in a fixed array of " +
                        std::to_string((size_t)PFLB_NOALLOC_SCRATCH_BYTES) +
                        " bytes; use pflb_init_fields with a work buffer");
    void* ptr = nullptr;
    hipError_t e = scratch_address(&ptr);
    if (e != hipSuccess) return hip_fail(c, e, "address of the static scratch array");
    // every staged value is written by the equilibrium kernel before the state load
    // reads it, so the array needs no clearing between calls
    float* h = static_cast<float*>(ptr);
    float* g = h + (size_t)c->Q * c->N;
    r = pflb_equilibrium(c, phi, u, P, h, g, stream);
    if (r) return r;
    return pflb_set_state(c, h, g, stream);
}

int pflb_reconstruct(pflb_ctx* c, const float* phi, const float* P, const float* J, float* work,
                     int advance, void* stream) {
    if (!c) return PFLB_ERR_PARAM;
    return pflb_reconstruct_many(&c, 1, &phi, &P, &J, work, advance, (hipStream_t)stream);
}

int pflb_step(pflb_ctx* c, int nsteps, void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (nsteps < 0) return fail(c, PFLB_ERR_PARAM, "nsteps < 0");
    Launch a = c->L;
    a.stream = (hipStream_t)stream;
    for (int s = 0; s < nsteps; ++s) {
        hipError_t e = launch_one(c, a, c->cur);
        if (e != hipSuccess) return hip_fail(c, e, "step launch");
        c->cur ^= 1;
        c->steps += 1;
    }
    return PFLB_OK;
}

int pflb_step_graph(pflb_ctx* c, int nsteps, void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (nsteps < 1) return fail(c, PFLB_ERR_PARAM, "nsteps < 1");
    if (!stream) return fail(c, PFLB_ERR_PARAM, "pflb_step_graph needs a stream other than the null stream");
    hipStream_t st = (hipStream_t)stream;
    if (nsteps != c->graph_n) c->drop_graphs();
    hipGraphExec_t& ex = c->graph[c->cur];
    if (!ex) {
        // capture the launches pflb_step would enqueue, from the current buffer
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(c, e, "graph capture");
        Launch a = c->L;
        a.stream = st;
        int cur = c->cur;
        hipError_t le = hipSuccess;
        for (int k = 0; k < nsteps && le == hipSuccess; ++k) {
            le = launch_one(c, a, cur);
            cur ^= 1;
        }
        e = hipStreamEndCapture(st, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(c, le, "step launch under capture");
        }
        if (e != hipSuccess) return hip_fail(c, e, "graph capture");
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ex = nullptr;
            return hip_fail(c, e, "graph instantiation");
        }
        c->graph_n = nsteps;
    }
    hipError_t e = hipGraphLaunch(ex, st);
    if (e != hipSuccess) return hip_fail(c, e, "graph launch");
    c->cur ^= (nsteps & 1);
    c->steps += nsteps;
    return PFLB_OK;
}

int pflb_read(pflb_ctx* c, float* phi, float* P, float* J, float* u, void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (!phi) return fail(c, PFLB_ERR_PARAM, "phi output is required");
    Launch a = c->L;
    a.stream = (hipStream_t)stream;
    hipError_t e = c->L.inplace ? launch_read_inplace(a, c->N, state(c), c->cur, phi, P, J, u)
                                : launch_read(a, c->N, state(c), phi, P, J, u);
    if (e != hipSuccess) return hip_fail(c, e, "read launch");
    return PFLB_OK;
}

int pflb_mass(pflb_ctx* c, double* sum_phi, int* nonfinite, void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (!sum_phi || !nonfinite) return fail(c, PFLB_ERR_PARAM, "NULL output pointer");
    Launch a = c->L;
    a.stream = (hipStream_t)stream;
    hipError_t e = launch_mass(a, c->N, state(c), c->buf[PFLB_BUF_SCRATCH]);
    if (e != hipSuccess) return hip_fail(c, e, "mass launch");
    const char* base = static_cast<const char*>(c->buf[PFLB_BUF_SCRATCH]);
    double s = 0.0;
    int f = 0;
    e = hipMemcpyAsync(&s, base + mass_result_offset(), sizeof(double), hipMemcpyDeviceToHost,
                       a.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&f, base + mass_flag_offset(), sizeof(int), hipMemcpyDeviceToHost,
                           a.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(a.stream);
    if (e != hipSuccess) return hip_fail(c, e, "mass read-back");
    *sum_phi = s;
    *nonfinite = f;
    if (f) return fail(c, PFLB_ERR_NONFINITE, "non-finite population in the state");
    return PFLB_OK;
}

long long pflb_step_count(const pflb_ctx* c) { return c ? c->steps : -1; }

int pflb_save(pflb_ctx* c, const char* path, void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (!path) return fail(c, PFLB_ERR_PARAM, "NULL path");
    const size_t nb = set_bytes(&c->p, c->N);
    std::vector<char> host;
    try {
        host.resize(nb);
    } catch (...) {
        return fail(c, PFLB_ERR_NOMEM, "host buffer for checkpoint");
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(host.data(), state(c), nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "checkpoint copy");
    FileHeader h;
    fill_header(c, &h);
    FILE* f = fopen(path, "wb");
    if (!f) return fail(c, PFLB_ERR_IO, std::string("cannot open ") + path);
    bool ok = fwrite(&h, sizeof(h), 1, f) == 1 && fwrite(host.data(), 1, nb, f) == nb;
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(c, PFLB_ERR_IO, std::string("cannot write ") + path);
    return PFLB_OK;
}

int pflb_load(pflb_ctx* c, const char* path, void* stream) {
    int r = need_bound(c);
    if (r) return r;
    if (!path) return fail(c, PFLB_ERR_PARAM, "NULL path");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(c, PFLB_ERR_IO, std::string("cannot open ") + path);
    FileHeader h, want;
    fill_header(c, &want);
    if (fread(&h, sizeof(h), 1, f) != 1) {
        fclose(f);
        return fail(c, PFLB_ERR_IO, "short checkpoint header");
    }
    const long long steps = h.steps;
    const int layout = h.layout;
    h.steps = want.steps;
    if (c->L.inplace && (layout == 0 || layout == 1)) h.layout = want.layout;
    if (memcmp(&h, &want, sizeof(h)) != 0) {
        fclose(f);
        return fail(c, PFLB_ERR_PARAM, "checkpoint parameters differ from the context's");
    }
    const size_t nb = set_bytes(&c->p, c->N);
    std::vector<char> host;
    try {
        host.resize(nb);
    } catch (...) {
        fclose(f);
        return fail(c, PFLB_ERR_NOMEM, "host buffer for checkpoint");
    }
    const bool ok = fread(host.data(), 1, nb, f) == nb;
    fclose(f);
    if (!ok) return fail(c, PFLB_ERR_IO, "short checkpoint body");
    c->cur = c->L.inplace ? layout : 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(state(c), host.data(), nb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "checkpoint upload");
    c->steps = steps;
    return PFLB_OK;
}

}  // extern "C"

int pflb_ctx_info(const pflb_ctx* c, CtxInfo* out) {
    if (!c || !out) return PFLB_ERR_PARAM;
    out->q = c->p.lattice;
    out->nx = c->p.nx; out->ny = c->p.ny; out->nz = c->p.nz;
    for (int a = 0; a < 3; ++a) out->bc[a] = c->p.bc[a];
    out->N = c->N;
    out->bound = c->bound;
    out->rho_L = c->p.rho_L;
    out->rho_H = c->p.rho_H;
    out->hoc = c->p.hoc;
    return PFLB_OK;
}

// ---------------------------------------------------------------------------
// batched read-out and hand-over (library-internal, used by the surrogate's guard)
// ---------------------------------------------------------------------------
namespace {

// contexts of one batched launch must be bound and share lattice, storage and geometry
int check_many(pflb_ctx* const* c, int n) {
    if (!c || n < 1 || !c[0]) return PFLB_ERR_PARAM;
    for (int k = 0; k < n; ++k) {
        if (!c[k]) return fail(c[0], PFLB_ERR_PARAM, "NULL context in a batch");
        if (!c[k]->bound) return fail(c[0], PFLB_ERR_UNBOUND, "context in a batch is not bound");
        const Launch& a = c[0]->L;
        const Launch& b = c[k]->L;
        if (b.q != a.q || b.half != a.half || b.inplace != a.inplace || b.G.nx != a.G.nx || b.G.ny != a.G.ny ||
            b.G.nz != a.G.nz || b.G.wx != a.G.wx || b.G.wy != a.G.wy || b.G.wz != a.G.wz)
            return fail(c[0], PFLB_ERR_PARAM,
                        "contexts of a batch must share lattice, storage, sizes and walls");
    }
    return PFLB_OK;
}

}  // namespace

int pflb_read_many(pflb_ctx* const* c, int n, float* const* phi, float* const* P,
                   float* const* J, hipStream_t st) {
    int r = check_many(c, n);
    if (r) return r;
    if (c[0]->L.inplace)
        return fail(c[0], PFLB_ERR_PARAM, "batched read-out takes contexts with pull storage");
    if (!phi) return fail(c[0], PFLB_ERR_PARAM, "phi outputs are required");
    for (int k0 = 0; k0 < n; k0 += BATCH_MAX) {
        const int nb = n - k0 < BATCH_MAX ? n - k0 : BATCH_MAX;
        Batch bt;
        memset(&bt, 0, sizeof(bt));
        bool macro = false;
        for (int j = 0; j < nb; ++j) {
            pflb_ctx* ck = c[k0 + j];
            BatchEnt& e = bt.e[j];
            if (!phi[k0 + j]) return fail(c[0], PFLB_ERR_PARAM, "phi outputs are required");
            e.state = static_cast<char*>(state(ck));
            e.phi = phi[k0 + j];
            e.P = P ? P[k0 + j] : nullptr;
            e.J = J ? J[k0 + j] : nullptr;
            e.m = ck->L.m;
            e.cd = ck->L.cd;
            macro = macro || e.P || e.J;
        }
        Launch a = c[k0]->L;
        a.stream = st;
        hipError_t e = launch_read_batch(a, c[0]->N, bt, nb, macro);
        if (e != hipSuccess) return hip_fail(c[0], e, "batched read launch");
    }
    return PFLB_OK;
}

int pflb_reconstruct_many(pflb_ctx* const* c, int n, const float* const* phi,
                          const float* const* P, const float* const* J, float* work, int advance,
                          hipStream_t st) {
    int r = check_many(c, n);
    if (r) return r;
    if (c[0]->L.inplace)
        return fail(c[0], PFLB_ERR_PARAM, "the hand-over takes contexts with pull storage");
    if (!phi || !J || !work) return fail(c[0], PFLB_ERR_PARAM, "NULL field or work pointer");
    if (advance < 0) return fail(c[0], PFLB_ERR_PARAM, "advance < 0");
    const size_t per = (size_t)2 * c[0]->Q * c[0]->N;   // floats of work per context
    for (int k0 = 0; k0 < n; k0 += BATCH_MAX) {
        const int nb = n - k0 < BATCH_MAX ? n - k0 : BATCH_MAX;
        Batch bt;
        memset(&bt, 0, sizeof(bt));
        for (int j = 0; j < nb; ++j) {
            pflb_ctx* ck = c[k0 + j];
            if (!phi[k0 + j] || !J[k0 + j])
                return fail(c[0], PFLB_ERR_PARAM, "NULL field or work pointer");
            ck->cur = 0;   // the hand-over fills the first state buffer
            BatchEnt& e = bt.e[j];
            e.state = static_cast<char*>(state(ck));
            e.phi = const_cast<float*>(phi[k0 + j]);
            e.P = P ? const_cast<float*>(P[k0 + j]) : nullptr;
            e.J = const_cast<float*>(J[k0 + j]);
            e.work = work + (size_t)j * per;
            e.m = ck->L.m;
            e.cd = ck->L.cd;
        }
        Launch a = c[k0]->L;
        a.stream = st;
        hipError_t e = launch_reconstruct_batch(a, c[0]->N, bt, nb);
        if (e != hipSuccess) return hip_fail(c[0], e, "batched hand-over launch");
        for (int j = 0; j < nb; ++j) c[k0 + j]->steps += advance;
    }
    return PFLB_OK;
}

extern "C" int pflb_step_many(pflb_ctx* const* c, int n, int nsteps, void* stream) {
    int r = check_many(c, n);
    if (r) return r;
    if (nsteps < 0) return fail(c[0], PFLB_ERR_PARAM, "nsteps < 0");
    // a context listed twice would be stepped twice from the same state into the same
    // buffer within one launch
    std::vector<pflb_ctx*> sorted(c, c + n);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(c[0], PFLB_ERR_PARAM, "a context appears twice in a batch");
    // Contexts with moving walls or contact angles take their own launches: the batched
    // kernel has no variant for them, and each context must run the arithmetic its own
    // pflb_step runs (separately compiled kernel variants may contract and round
    // differently).
    std::vector<pflb_ctx*> gr;
    for (int k = 0; k < n; ++k) {
        if (!c[k]->L.m.moving && !c[k]->L.m.wetting && !c[k]->L.wide && !c[k]->L.G.open &&
            !c[k]->L.inplace) {
            gr.push_back(c[k]);
        } else if ((r = pflb_step(c[k], nsteps, stream))) {
            if (c[k] != c[0]) fail(c[0], r, pflb_last_error(c[k]));
            return r;
        }
    }
    const int ng = (int)gr.size();
    for (int k0 = 0; k0 < ng; k0 += BATCH_MAX) {
        const int nb = ng - k0 < BATCH_MAX ? ng - k0 : BATCH_MAX;
        Launch a = gr[k0]->L;
        a.stream = (hipStream_t)stream;
        a.bz = pick_bz(a.G, a.q, nb);
        StepBatch bt;
        memset(&bt, 0, sizeof(bt));
        for (int s = 0; s < nsteps; ++s) {
            for (int j = 0; j < nb; ++j) {
                pflb_ctx* ck = gr[k0 + j];
                StepEnt& e = bt.e[j];
                e.src = static_cast<const char*>(state(ck));
                e.dst = static_cast<char*>(other(ck));
                e.m = ck->L.m;
                e.cd = ck->L.cd;
            }
            hipError_t e = launch_step_batch(a, bt, nb);
            if (e != hipSuccess) return hip_fail(c[0], e, "batched step launch");
            for (int j = 0; j < nb; ++j) {
                gr[k0 + j]->cur ^= 1;
                gr[k0 + j]->steps += 1;
            }
        }
    }
    return PFLB_OK;
}
