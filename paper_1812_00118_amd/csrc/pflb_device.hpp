// Device-side building blocks of the phase-field lattice Boltzmann step (gfx950).
//
// Internal axes: D3Q19 uses (x, y, z).  D2Q9 is laid out in the internal (x, z)
// plane with internal ny = 1, so that one z-marching kernel serves both lattices;
// the user's y axis of a D2Q9 domain is the internal z axis and the site index
// (z*ny + y)*nx + x is unchanged by this relabelling.
//
// Storage of a distribution set ("pull" layout): slot (s, i) holds the post-collision
// population that leaves site s in direction i.  Site x gathers h_i(x) from slot
// (x - c_i, i), or from slot (x, opp(i)) when x - c_i lies beyond a wall (halfway
// bounce-back).  Every slot is read exactly once per step.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

namespace pflb {

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// ---------------------------------------------------------------------------
// lattices (opposite pairs (2k-1, 2k); T = 1/3)
// ---------------------------------------------------------------------------
struct LatD3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr bool USES_Y = true;
    __host__ __device__ static constexpr int cx(int i) {
        constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        return t[i];
    }
    __host__ __device__ static constexpr int cy(int i) {
        constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int cz(int i) {
        constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        return t[i];
    }
    __host__ __device__ static constexpr float w(int i) {
        return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
    }
    // w_i - float(w_i): the float32 weights are 1/18 and 1/36 only to 7.5e-9 relative
    __host__ __device__ static constexpr float w_lo(int i) {
        return i == 0 ? (float)(1.0 / 3.0 - (double)(1.0f / 3.0f))
                      : (i <= 6 ? (float)(1.0 / 18.0 - (double)(1.0f / 18.0f))
                                : (float)(1.0 / 36.0 - (double)(1.0f / 36.0f)));
    }
};

struct LatD2Q9 {  // user (x, y) -> internal (x, z)
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr bool USES_Y = false;
    __host__ __device__ static constexpr int cx(int i) {
        constexpr int t[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int cy(int) { return 0; }
    __host__ __device__ static constexpr int cz(int i) {
        constexpr int t[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
        return t[i];
    }
    __host__ __device__ static constexpr float w(int i) {
        return i == 0 ? 4.0f / 9.0f : (i <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f);
    }
    __host__ __device__ static constexpr float w_lo(int i) {
        return i == 0 ? (float)(4.0 / 9.0 - (double)(4.0f / 9.0f))
                      : (i <= 4 ? (float)(1.0 / 9.0 - (double)(1.0f / 9.0f))
                                : (float)(1.0 / 36.0 - (double)(1.0f / 36.0f)));
    }
};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// 1 - sum_i w_i of the float32 weights (exact in double).  The relaxation towards
// phi w_i adds phi (sum w - 1) per step to every site unless the rest population
// carries phi * kappa.
template <class L>
__host__ __device__ constexpr float kappa() {
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) s += (double)L::w(i);
    return (float)(1.0 - s);
}


// ---------------------------------------------------------------------------
// geometry and model constants passed by value to every kernel
// ---------------------------------------------------------------------------
struct Geom {
    int nx, ny, nz;     // internal sizes
    int wx, wy, wz;     // 1: wall on both faces of the axis, 0: periodic
    uint32_t S;         // population stride of a set, in sites
    uint32_t sxy;       // nx * ny
    uint32_t open;      // open (pressure) faces: bit f for face f (x-, x+, y-, y+, z-, z+)
    uint32_t SL;        // stride of a face's side array, in sites (the largest face, rounded up)
    size_t side_off;    // byte offset of the side arrays in a state buffer
};

struct Model {
    float rho_L, rho_dif;     // rho = rho_L + phi rho_dif
    float itau_L, itau_dif;   // 1/tau_mix = itau_L + phi itau_dif          (Eq. 9)
    float om_phi;             // 1/tau_phi, tau_phi = M/T + 1/2             (Eq. 1)
    float mu_a, mu_b;         // mu = mu_a phi(phi-1)(phi-1/2) - mu_b lap   (Eq. 8)
    float th_a;               // theta = th_a (1 - 4 (phi-1/2)^2)            (Eq. 4)
    float dth;                // C M / T of the Eq. 14 correction (0: off)
    float eps;                // n = grad/(|grad| + eps)
    float gx, gy, gz;         // gravity in internal axes; F = rho g
    float beta;               // 1: Eq. 13 correction and modified velocity
    float uw[6][3];           // wall face velocities, faces x-, x+, y-, y+, z-, z+ (internal)
    int moving;               // 1 if any wall moves
    float wk[6];              // wetting: (4/W) cos(contact angle) per face (internal)
    int wetting;              // 1 if any face has a contact angle other than 90 degrees
    float Pf[6];              // pressure of each open face (x-, x+, y-, y+, z-, z+)
};

struct Codec {                // FP16S: power-of-two scales of the fp16 deviations
    float sh, ish, sg, isg;
};

// One context of a batched launch.  Read-out: phi (and P, J when not NULL) are outputs.
// Hand-over: phi, J and P (NULL: 0) are inputs and work holds the context's equilibria
// (h then g, Q N floats each) between the two kernels.
struct BatchEnt {
    char* state;
    float* phi;
    float* P;
    float* J;
    float* work;
    Model m;
    Codec cd;
};
constexpr int BATCH_MAX = 16;
struct Batch {
    BatchEnt e[BATCH_MAX];
};

// One context of a batched step: its current and next state buffers and its parameters.
struct StepEnt {
    const char* src;
    char* dst;
    Model m;
    Codec cd;
};
struct StepBatch {
    StepEnt e[BATCH_MAX];
};

// ---------------------------------------------------------------------------
// storage codecs.  One state buffer holds both sets.
//   FP32 : [Q][S] float2 (h_i, g_i): one load brings h_i and g_i of a slot.
//   FP16S: [S] float2 (h_0, g_0), the rest populations in float32;
//          [S] uint4, the site's moments word: its pre-collision moments of the step
//          that wrote the buffer, rounded to fp16, as half2 pairs (Phi, Psi),
//          (jh_x, Jg_x), (jh_y, Jg_y), (jh_z, Jg_z) with Phi = sum h, jh = sum c h,
//          Psi = sum g, Jg = sum c g;
//          [Q-1][S] half2 (dev_h, dev_g) for the moving directions i = 1..Q-1.
//   A moving population is stored as an fp16 deviation from a reference that its
//   reader can form on its own: the first-order equilibrium w_i (Phi + 3 c_i . jh) (and
//   w_i (Psi + 3 c_i . Jg) for g) of the reading site's moments.  The writer, which
//   collides the neighbours of the reading site in the same workgroup, takes the same
//   moments from the workgroup's LDS planes, so the reader gathers deviations only (no
//   per-direction reference words), and the deviation is second order in the lattice
//   spacing.  The rest population h_0 is the float32 complement that makes the site's
//   decoded outgoing values sum to its h total.
// ---------------------------------------------------------------------------
struct StoreF32 {
    static constexpr bool HALF = false;
    static constexpr bool INPLACE = false;
    __host__ __device__ static constexpr size_t bytes_per_site(int q) { return (size_t)q * 8; }
};

// FP32 in place (one buffer): Q arrays of h, then Q arrays of g, each of stride S floats
struct StoreF32InPlace {
    static constexpr bool HALF = false;
    static constexpr bool INPLACE = true;
    __host__ __device__ static constexpr size_t bytes_per_site(int q) { return (size_t)q * 8; }
};

struct StoreF16S {
    static constexpr bool HALF = true;
    static constexpr bool INPLACE = false;
    __host__ __device__ static constexpr size_t bytes_per_site(int q) {
        return 8 + 16 + (size_t)(q - 1) * 4;
    }
    // byte offsets of the regions in a buffer of stride S
    __host__ __device__ static constexpr size_t mom_off(uint32_t S) { return (size_t)S * 8; }
    __host__ __device__ static constexpr size_t dev_off(uint32_t S) { return (size_t)S * 24; }
};

// Encode pre-collision values of a slot-site (FP32 state upload).
template <class L>
__device__ __forceinline__ void encode_site_f32(char* __restrict__ b, uint32_t site, uint32_t S,
                                                const float (&h)[L::Q], const float (&g)[L::Q]) {
    float2* o = reinterpret_cast<float2*>(b);
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        o[(size_t)i * S + site] = make_float2(h[i], g[i]);
    });
}

// Streaming stores: the written state is read back only by the next launch, after far
// more data than the caches hold has passed, so the stores bypass cache allocation.
typedef float nt_float2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_uint4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_nt(char* p, float a, float b) {
    nt_float2 v = {a, b};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_float2*>(p));
}

__device__ __forceinline__ void store_nt(char* p, __half2 v) {
    __builtin_nontemporal_store(*reinterpret_cast<uint32_t*>(&v), reinterpret_cast<uint32_t*>(p));
}

__device__ __forceinline__ void store_nt(char* p, uint4 v) {
    nt_uint4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_uint4*>(p));
}

// ----- FP16S moments word and references -----
struct MomF {
    float Phi, Psi, jx, jy, jz, Jx, Jy, Jz;
};

__device__ __forceinline__ uint32_t pack_h2(float a, float b) {
    __half2 v = __halves2half2(__float2half_rn(a), __float2half_rn(b));
    return *reinterpret_cast<uint32_t*>(&v);
}

__device__ __forceinline__ float2 unpack_h2(uint32_t w) {
    return __half22float2(*reinterpret_cast<const __half2*>(&w));
}

__device__ __forceinline__ uint4 pack_mom(float Phi, float Psi, float jx, float jy, float jz,
                                          float Jx, float Jy, float Jz) {
    return make_uint4(pack_h2(Phi, Psi), pack_h2(jx, Jx), pack_h2(jy, Jy), pack_h2(jz, Jz));
}

__device__ __forceinline__ MomF unpack_mom(const uint4& w) {
    MomF m;
    const float2 a = unpack_h2(w.x), bx = unpack_h2(w.y), by = unpack_h2(w.z),
                 bz = unpack_h2(w.w);
    m.Phi = a.x; m.Psi = a.y;
    m.jx = bx.x; m.Jx = bx.y;
    m.jy = by.x; m.Jy = by.y;
    m.jz = bz.x; m.Jz = bz.y;
    return m;
}

// c_I . v as a fixed sum of the components (the same float operations wherever a
// reference is formed, so that writer and reader agree bit for bit)
template <class L, int I>
__device__ __forceinline__ float cdot(float vx, float vy, float vz) {
    constexpr int ex = L::cx(I), ey = L::cy(I), ez = L::cz(I);
    float s = 0.f;
    bool first = true;
    auto add = [&](int e, float v) {
        if (e == 0) return;
        const float t = e > 0 ? v : -v;
        s = first ? t : s + t;
        first = false;
    };
    add(ex, vx);
    add(ey, vy);
    add(ez, vz);
    return s;
}

// FP16S references of the population I (>= 1) a site with moments m reads:
// w_I (Phi + 3 c_I . jh) and w_I (Psi + 3 c_I . Jg)
template <class L, int I>
__device__ __forceinline__ void ref_of(const MomF& m, float& rh, float& rg) {
    constexpr float w = L::w(I);
    rh = w * fmaf(3.0f, cdot<L, I>(m.jx, m.jy, m.jz), m.Phi);
    rg = w * fmaf(3.0f, cdot<L, I>(m.Jx, m.Jy, m.Jz), m.Psi);
}

// moments of a gathered site, accumulated as its populations are decoded
struct MomAcc {
    float S = 0.f;                     // sum of the moving h, in index order
    float jx = 0.f, jy = 0.f, jz = 0.f;
    template <class L, int I>
    __device__ __forceinline__ void add_h(float h) {
        constexpr int ex = L::cx(I), ey = L::cy(I), ez = L::cz(I);
        S = I == 1 ? h : S + h;
        if constexpr (ex > 0) jx += h;
        if constexpr (ex < 0) jx -= h;
        if constexpr (ey > 0) jy += h;
        if constexpr (ey < 0) jy -= h;
        if constexpr (ez > 0) jz += h;
        if constexpr (ez < 0) jz -= h;
    }
};

// c_I . u_w for the population a site with wall bits `solid` (Col.solid | ZRow.solid)
// sends in direction I: u_w is the velocity of the wall face it crosses, the mean at an
// edge or corner, 0 if it crosses none.
template <class L, int I>
__device__ __forceinline__ float wall_cu(const Model& m, uint32_t solid) {
    constexpr int ex = L::cx(I), ey = L::cy(I), ez = L::cz(I);
    float s = 0.f;
    int n = 0;
    auto face = [&](int f) {
        s += (float)ex * m.uw[f][0] + (float)ey * m.uw[f][1] + (float)ez * m.uw[f][2];
        ++n;
    };
    if constexpr (ex > 0) { if (solid & 2u) face(1); }
    if constexpr (ex < 0) { if (solid & 1u) face(0); }
    if constexpr (ey > 0) { if (solid & 8u) face(3); }
    if constexpr (ey < 0) { if (solid & 4u) face(2); }
    if constexpr (ez > 0) { if (solid & 32u) face(5); }
    if constexpr (ez < 0) { if (solid & 16u) face(4); }
    return n == 0 ? 0.f : (n == 1 ? s : (n == 2 ? 0.5f * s : s * (1.0f / 3.0f)));
}

// Writer for the sites of a wave that has wall sites of a moving wall (halfway
// bounce-back with the momentum correction): the population a site sends into a wall
// face is the one it pulls back next step, reduced here by 2 w_I (c_I . u_w)/T times the
// site's phi (h) or rho (g).  `on` is uniform over the wave, so waves away from moving
// walls skip the correction with scalar branches.
template <class L, class W>
struct WallWriter {
    W& w;
    const Model& m;
    uint32_t solid;
    float kh, kg;                 // phi 2/T and rho 2/T
    bool on;
    template <int I>
    __device__ __forceinline__ void put(float h, float g) {
        if constexpr (I != 0) {
            if (on) {
                const float k = L::w(I) * wall_cu<L, I>(m, solid);
                // the h total follows the exact correction (a float product is exact
                // in double): opposite corrections of a tangential pair cancel exactly,
                // and at an edge or corner between walls moving differently, where they
                // need not cancel, the total changes as in the method
                w.shift_h_total(-(double)k * (double)kh);
                h = fmaf(-k, kh, h);
                g = fmaf(-k, kg, g);
            }
        }
        w.template put<I>(h, g);
    }
    __device__ __forceinline__ void finish() { w.finish(); }
};

// ---------------------------------------------------------------------------
// boundary-aware gather
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int map_coord(int v, int n, int wall) {
    // coordinate of the site whose phi a position v stands for: wrap (periodic) or
    // the adjacent fluid site (wall)
    if (wall) return v < 0 ? 0 : (v >= n ? n - 1 : v);
    v %= n;
    return v < 0 ? v + n : v;
}

// Wetting ghost rule: the phi of position (vx, vy, vz) beyond wall faces is
// pm + k pm (1 - pm), pm the value of the site map_coord gives and k the sum, over the
// faces the position lies beyond, of (4/W) cos(contact angle).  Inside the domain, and
// beyond faces of periodic axes (whose coefficients are 0), k = 0 and pm is returned
// unchanged.
__device__ __forceinline__ float wet_ghost(const Geom& G, const Model& m, int vx, int vy,
                                           int vz, float pm) {
    float k = 0.0f;
    if (vx < 0) k += m.wk[0];
    else if (vx >= G.nx) k += m.wk[1];
    if (vy < 0) k += m.wk[2];
    else if (vy >= G.ny) k += m.wk[3];
    if (vz < 0) k += m.wk[4];
    else if (vz >= G.nz) k += m.wk[5];
    return fmaf(k, pm * (1.0f - pm), pm);
}

// Upstream offsets of an (x, y) column: source x - 1 (for c_x = +1) and x + 1 (c_x = -1)
// Site offsets are added modulo 2^32 (a step back is 2^32 - 1): every site index and
// every sum that names a site stays below 2^32.
struct Col {
    uint32_t base;                 // y*nx + x
    uint32_t dxm, dxp, dym, dyp;   // site offsets to the upstream site
    uint32_t solid;                // bit0: x-1 beyond a wall, bit1: x+1, bit2: y-1, bit3: y+1
};
struct ZRow {
    uint32_t base;                 // z*nx*ny
    uint32_t dzm, dzp;
    uint32_t solid;                // bit4: z-1 beyond a wall, bit5: z+1
};

__device__ __forceinline__ Col make_col(const Geom& G, int x, int y) {
    Col c;
    c.base = (uint32_t)y * (uint32_t)G.nx + (uint32_t)x;
    const uint32_t nx = (uint32_t)G.nx, ny = (uint32_t)G.ny;
    c.dxm = (x == 0) ? nx - 1u : 0u - 1u;
    c.dxp = (x == G.nx - 1) ? 0u - (nx - 1u) : 1u;
    c.dym = (y == 0) ? (ny - 1u) * nx : 0u - nx;
    c.dyp = (y == G.ny - 1) ? 0u - (ny - 1u) * nx : nx;
    c.solid = 0;
    if (G.wx) c.solid |= (x == 0 ? 1u : 0u) | (x == G.nx - 1 ? 2u : 0u);
    if (G.wy) c.solid |= (y == 0 ? 4u : 0u) | (y == G.ny - 1 ? 8u : 0u);
    return c;
}

__device__ __forceinline__ ZRow make_zrow(const Geom& G, int z) {
    ZRow r;
    r.base = (uint32_t)z * G.sxy;
    const uint32_t nz = (uint32_t)G.nz;
    r.dzm = (z == 0) ? (nz - 1u) * G.sxy : 0u - G.sxy;
    r.dzp = (z == G.nz - 1) ? 0u - (nz - 1u) * G.sxy : G.sxy;
    r.solid = 0;
    if (G.wz) r.solid = (z == 0 ? 16u : 0u) | (z == G.nz - 1 ? 32u : 0u);
    return r;
}

// Which boundaries a kernel variant handles: walls across x or y (a per-lane test) and
// walls across z (uniform over a plane, so a scalar test in the z-marching kernel).
enum WallSet { WALLS_NONE = 0, WALLS_Z = 1, WALLS_XY = 2, WALLS_XYZ = 3 };
// Added to a kernel's wall set for domains whose slot byte offsets need 64 bits (more
// than 2^28 - 64 sites): addresses are then formed as 64-bit sums per lane instead of
// a uniform base plus a 32-bit lane offset.
constexpr int ADDR64 = 8;

// Upstream slot of direction I for the site (c, r): (site - c_I, I), or (site, opp(I))
// when the upstream site lies beyond a wall (flip = true).
template <class L, int I, int WALLS>
struct Up {
    static constexpr int ex = L::cx(I), ey = L::cy(I), ez = L::cz(I);
    static constexpr uint32_t need_xy = (ex > 0 ? 1u : 0u) | (ex < 0 ? 2u : 0u) |
                                        (ey > 0 ? 4u : 0u) | (ey < 0 ? 8u : 0u);
    static constexpr uint32_t need_z = (ez > 0 ? 16u : 0u) | (ez < 0 ? 32u : 0u);
    static constexpr bool test_xy = (WALLS & WALLS_XY) && need_xy != 0u;
    static constexpr bool test_z = (WALLS & WALLS_Z) && need_z != 0u;
    static constexpr bool MAYFLIP = I != 0 && (test_xy || test_z);
    // the population pair (lo, lo + 1) containing I
    static constexpr int LO = I == 0 ? 0 : ((I & 1) ? I : I - 1);
};

template <class L, int I, int WALLS>
__device__ __forceinline__ void upstream(const Col& c, const ZRow& r, uint32_t& slot_site,
                                         bool& flip) {
    using U = Up<L, I, WALLS>;
    const uint32_t site = c.base + r.base;
    uint32_t off = 0u;
    if constexpr (U::ex > 0) off += c.dxm;
    if constexpr (U::ex < 0) off += c.dxp;
    if constexpr (U::ey > 0) off += c.dym;
    if constexpr (U::ey < 0) off += c.dyp;
    if constexpr (U::ez > 0) off += r.dzm;
    if constexpr (U::ez < 0) off += r.dzp;
    flip = false;
    if constexpr (U::MAYFLIP) {
        bool bb = false;
        if constexpr (U::test_xy) bb = bb || (c.solid & U::need_xy) != 0u;
        if constexpr (U::test_z) bb = bb || (r.solid & U::need_z) != 0u;
        flip = bb;
        slot_site = bb ? site : site + off;
    } else {
        slot_site = site + off;
    }
}

// Address of slot (slot_site, I or opp(I)) in an array of Q populations with stride
// S * esize bytes: a uniform base (kernel argument plus a multiple of the stride) and a
// 32-bit per-lane byte offset, the form the scalar-base loads take.
template <class L, int I, int WALLS, int ESIZE>
__device__ __forceinline__ const char* slot_addr(const char* __restrict__ base0, uint32_t S,
                                                 uint32_t slot_site, bool flip,
                                                 uint32_t& off) {
    using U = Up<L, I, WALLS>;
    const size_t stride = (size_t)S * ESIZE;
    if constexpr ((WALLS & ADDR64) != 0) {
        off = 0u;
        if constexpr (!U::MAYFLIP) {
            return base0 + (size_t)I * stride + (size_t)slot_site * ESIZE;
        } else {
            const bool second = flip ? (I == U::LO) : (I != U::LO);
            return base0 + (size_t)U::LO * stride + (second ? stride : (size_t)0) +
                   (size_t)slot_site * ESIZE;
        }
    } else if constexpr (!U::MAYFLIP) {
        off = slot_site * (uint32_t)ESIZE;
        return base0 + (size_t)I * stride;
    } else {
        // pop = flip ? opp(I) : I; second member of the pair when pop != LO
        const bool second = flip ? (I == U::LO) : (I != U::LO);
        off = slot_site * (uint32_t)ESIZE + (second ? (uint32_t)stride : 0u);
        return base0 + (size_t)U::LO * stride;
    }
}

// byte offset of element `site` of size E: 32-bit (a uniform base plus a lane offset)
// unless the wall set carries ADDR64
template <int WALLS, int E>
__device__ __forceinline__ size_t elem_off(uint32_t site) {
    if constexpr ((WALLS & ADDR64) != 0) return (size_t)site * E;
    else return (size_t)(site * (uint32_t)E);
}

// FP32 storage: slot pair (h, g), or h alone, of direction I.
template <class L, int I, int WALLS>
__device__ __forceinline__ float2 load_pair32(const char* __restrict__ b, uint32_t S,
                                              uint32_t slot_site, bool flip) {
    uint32_t off;
    const char* base = slot_addr<L, I, WALLS, 8>(b, S, slot_site, flip, off);
    return *reinterpret_cast<const float2*>(base + off);
}

template <class L, int I, int WALLS>
__device__ __forceinline__ float load_h32(const char* __restrict__ b, uint32_t S,
                                          uint32_t slot_site, bool flip) {
    uint32_t off;
    const char* base = slot_addr<L, I, WALLS, 8>(b, S, slot_site, flip, off);
    return *reinterpret_cast<const float*>(base + off);
}

// phi of a gathered site with FP32 storage, summed in float64 from the stored values
// and used as hi + lo floats.  The BGK update relaxes h towards phi w_i and the site
// keeps the mass phi: a float32-rounded phi would add that rounding error to the site
// at every step (a random walk of the phase field).
struct PhiAcc {
    double r = 0.0;
    __device__ __forceinline__ double value() const { return r; }
};

// Raw moments of the hydrodynamic set up to second order, sum g, sum c g and sum c c g:
// all that the filtered collision uses of the pre-collision g (Eqs. 10-12: g* depends on
// g only through P, J and Pi), so a site keeps 10 numbers instead of Q populations.
// Each sum runs over the directions in index order.
struct GMom {
    float s = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
    float xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
};

template <class L, int I>
__device__ __forceinline__ void add_moment(GMom& m, float g) {
    constexpr int ex = L::cx(I), ey = L::cy(I), ez = L::cz(I);
    m.s += g;
    if constexpr (ex > 0) m.jx += g;
    if constexpr (ex < 0) m.jx -= g;
    if constexpr (ey > 0) m.jy += g;
    if constexpr (ey < 0) m.jy -= g;
    if constexpr (ez > 0) m.jz += g;
    if constexpr (ez < 0) m.jz -= g;
    if constexpr (ex != 0) m.xx += g;
    if constexpr (ey != 0) m.yy += g;
    if constexpr (ez != 0) m.zz += g;
    if constexpr (ex * ey > 0) m.xy += g;
    if constexpr (ex * ey < 0) m.xy -= g;
    if constexpr (ex * ez > 0) m.xz += g;
    if constexpr (ex * ez < 0) m.xz -= g;
    if constexpr (ey * ez > 0) m.yz += g;
    if constexpr (ey * ez < 0) m.yz -= g;
}

template <class L>
__device__ __forceinline__ GMom g_moments(const float (&g)[L::Q]) {
    GMom m;
    static_for<0, L::Q>([&](auto I) { add_moment<L, decltype(I)::value>(m, g[decltype(I)::value]); });
    return m;
}

// FP16S: decode the populations site (c, r) reads, with its own rest word and moments
// word, calling f(I, h_I, g_I) in index order.  Returns phi = h_0 + (sum of the moving h
// in index order); acc holds that sum and the first moment of h.  The float sums are the
// ones a writer's complement mirrors: over a uniform region the reader's sum and the
// writer's take the same values in the same order, and h_0 = T - S with S within a
// factor two of T is exact (Sterbenz), so phi returns to T exactly there.
template <class L, int WALLS, class F>
__device__ __forceinline__ float gather16(const char* __restrict__ b, const Geom& G,
                                          const Col& c, const ZRow& r, const Codec& cd,
                                          MomAcc& acc, F&& f, MomF* mom_out = nullptr) {
    const uint32_t site = c.base + r.base;
    const float2 rest = reinterpret_cast<const float2*>(b)[site];
    const MomF m =
        unpack_mom(reinterpret_cast<const uint4*>(b + StoreF16S::mom_off(G.S))[site]);
    if (mom_out) *mom_out = m;
    // f(I, h_I, g_I, raw g deviation): the decoded g and its reference are computed only
    // where a caller uses them
    f(std::integral_constant<int, 0>{}, rest.x, rest.y, 0.0f);
    // deviation of population pop >= 1 at dev_off + (pop - 1) S 4
    const char* base0 = b + StoreF16S::dev_off(G.S) - (size_t)G.S * 4;
    static_for<1, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        uint32_t s;
        bool flip;
        upstream<L, i, WALLS>(c, r, s, flip);
        uint32_t off;
        const char* base = slot_addr<L, i, WALLS, 4>(base0, G.S, s, flip, off);
        const float2 q = __half22float2(*reinterpret_cast<const __half2*>(base + off));
        float rh, rg;
        ref_of<L, i>(m, rh, rg);
        const float hv = fmaf(q.x, cd.ish, rh);
        const float gv = fmaf(q.y, cd.isg, rg);
        acc.template add_h<L, i>(hv);
        f(I, hv, gv, q.y);
    });
    return rest.x + acc.S;
}

// Raw moments of the g set of a FP16S site from its moments word and the moments of
// its raw g deviations over the moving directions: the references w_i (Psi + 3 c_i . Jg)
// contribute (1 - w_0) Psi, Jg and Psi/3 per lattice axis (the lattice's second moment
// is 1/3, its first and third vanish), the deviations dg the rest, scaled once.
template <class L>
__device__ __forceinline__ GMom g_moments16(float g0, const MomF& m, const GMom& d,
                                            const Codec& cd) {
    constexpr float wsum = (float)(1.0 - (L::Q == 19 ? 1.0 / 3.0 : 4.0 / 9.0));
    constexpr float third = 1.0f / 3.0f;
    GMom gm;
    gm.s = g0 + fmaf(wsum, m.Psi, cd.isg * d.s);
    gm.jx = fmaf(cd.isg, d.jx, m.Jx);
    gm.jy = L::USES_Y ? fmaf(cd.isg, d.jy, m.Jy) : 0.0f;
    gm.jz = fmaf(cd.isg, d.jz, m.Jz);
    gm.xx = fmaf(third, m.Psi, cd.isg * d.xx);
    gm.yy = L::USES_Y ? fmaf(third, m.Psi, cd.isg * d.yy) : 0.0f;
    gm.zz = fmaf(third, m.Psi, cd.isg * d.zz);
    gm.xy = cd.isg * d.xy;
    gm.xz = cd.isg * d.xz;
    gm.yz = cd.isg * d.yz;
    return gm;
}

// Gather the Q pre-collision populations of both sets of one site and its phi.
template <class L, class ST, int WALLS>
__device__ __forceinline__ double pull_site(const char* __restrict__ b, const Geom& G,
                                            const Col& c, const ZRow& r, const Codec& cd,
                                            float (&h)[L::Q], float (&g)[L::Q]) {
    if constexpr (ST::HALF) {
        MomAcc acc;
        return (double)gather16<L, WALLS>(b, G, c, r, cd, acc,
                                          [&](auto I, float hv, float gv, float) {
            h[decltype(I)::value] = hv;
            g[decltype(I)::value] = gv;
        });
    } else {
        PhiAcc acc;
        static_for<0, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            uint32_t s;
            bool flip;
            upstream<L, i, WALLS>(c, r, s, flip);
            const float2 v = load_pair32<L, i, WALLS>(b, G.S, s, flip);
            acc.r += (double)v.x;
            h[i] = v.x;
            g[i] = v.y;
        });
        return acc.value();
    }
}

// Gather only the h populations of one site and its phi.
template <class L, class ST, int WALLS>
__device__ __forceinline__ double pull_site_h(const char* __restrict__ b, const Geom& G,
                                              const Col& c, const ZRow& r, const Codec& cd,
                                              float (&h)[L::Q]) {
    if constexpr (ST::HALF) {
        MomAcc acc;
        return (double)gather16<L, WALLS>(b, G, c, r, cd, acc,
                                          [&](auto I, float hv, float, float) {
            h[decltype(I)::value] = hv;
        });
    } else {
        PhiAcc acc;
        static_for<0, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            uint32_t s;
            bool flip;
            upstream<L, i, WALLS>(c, r, s, flip);
            h[i] = load_h32<L, i, WALLS>(b, G.S, s, flip);
            acc.r += (double)h[i];
        });
        return acc.value();
    }
}

// Gather the h populations of one site, the raw moments of its g populations and its
// phi: the form the fused step keeps a site in between the gather and the collision
// (FP32 storage).
template <class L, int WALLS>
__device__ __forceinline__ double pull_site_m(const char* __restrict__ b, const Geom& G,
                                              const Col& c, const ZRow& r, float (&h)[L::Q],
                                              GMom& gm) {
    PhiAcc acc;
    gm = GMom{};
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        uint32_t s;
        bool flip;
        upstream<L, i, WALLS>(c, r, s, flip);
        const float2 v = load_pair32<L, i, WALLS>(b, G.S, s, flip);
        acc.r += (double)v.x;
        h[i] = v.x;
        add_moment<L, i>(gm, v.y);
    });
    return acc.value();
}

// The same for FP16S storage, which also returns the site's moments (phi, sum c h,
// sum g, sum c g) as the fp16 moments word the writers of its populations use.
template <class L, int WALLS>
__device__ __forceinline__ float pull_site_m16(const char* __restrict__ b, const Geom& G,
                                               const Col& c, const ZRow& r, const Codec& cd,
                                               float (&h)[L::Q], GMom& gm, uint4& mom) {
    MomAcc acc;
    GMom d;
    float g0 = 0.f;
    MomF m;
    const float phi = gather16<L, WALLS>(b, G, c, r, cd, acc,
                                         [&](auto I, float hv, float gv, float qg) {
        constexpr int i = decltype(I)::value;
        h[i] = hv;
        if constexpr (i == 0) g0 = gv;
        else add_moment<L, i>(d, qg);
    }, &m);
    gm = g_moments16<L>(g0, m, d, cd);
    mom = pack_mom(phi, gm.s, acc.jx, acc.jy, acc.jz, gm.jx, gm.jy, gm.jz);
    return phi;
}

// FP16S: phi and the moments word of a site whose populations are not kept (the halo
// ring and the planes a workgroup only gathers for its neighbours' references).
template <class L, int WALLS>
__device__ __forceinline__ float pull_site_mom16(const char* __restrict__ b, const Geom& G,
                                                 const Col& c, const ZRow& r, const Codec& cd,
                                                 uint4& mom) {
    MomAcc acc;
    float g0 = 0.f, Sg = 0.f, Jx = 0.f, Jy = 0.f, Jz = 0.f;
    MomF m;
    const float phi = gather16<L, WALLS>(b, G, c, r, cd, acc,
                                         [&](auto I, float, float gv, float qg) {
        constexpr int i = decltype(I)::value;
        if constexpr (i == 0) {
            g0 = gv;
        } else {
            Sg += qg;
            if constexpr (L::cx(i) > 0) Jx += qg;
            if constexpr (L::cx(i) < 0) Jx -= qg;
            if constexpr (L::cy(i) > 0) Jy += qg;
            if constexpr (L::cy(i) < 0) Jy -= qg;
            if constexpr (L::cz(i) > 0) Jz += qg;
            if constexpr (L::cz(i) < 0) Jz -= qg;
        }
    }, &m);
    // the moments of the g references as in g_moments16
    constexpr float wsum = (float)(1.0 - (L::Q == 19 ? 1.0 / 3.0 : 4.0 / 9.0));
    Sg = g0 + fmaf(wsum, m.Psi, cd.isg * Sg);
    Jx = fmaf(cd.isg, Jx, m.Jx);
    Jy = L::USES_Y ? fmaf(cd.isg, Jy, m.Jy) : 0.0f;
    Jz = fmaf(cd.isg, Jz, m.Jz);
    mom = pack_mom(phi, Sg, acc.jx, acc.jy, acc.jz, Jx, Jy, Jz);
    return phi;
}

// True if site + c_I lies beyond a wall face, for a site with wall bits `solid`: the
// population it sends in direction I then comes back to itself as opp(I).
template <class L, int I, int WALLS>
__device__ __forceinline__ bool dest_beyond(uint32_t solid) {
    // the upstream site of opp(I) is site + c_I
    using U = Up<L, opp(I), WALLS>;
    bool bb = false;
    if constexpr (U::test_xy) bb = bb || (solid & U::need_xy) != 0u;
    if constexpr (U::test_z) bb = bb || (solid & U::need_z) != 0u;
    return bb;
}

// Streaming writer of one site's post-collision pairs (pairs arrive rest population
// first), FP32 storage.
template <class L, int WALLS>
struct SiteWriter32 {
    char* __restrict__ b;
    uint32_t site;
    uint32_t S;
    template <int I>
    __device__ __forceinline__ void put(float h, float g) {
        char* base = b + (size_t)I * ((size_t)S * 8);
        store_nt(base + elem_off<WALLS, 8>(site), h, g);
    }
    __device__ __forceinline__ void finish() {}
    __device__ __forceinline__ void shift_h_total(double) {}
};

// FP16S writer.  A moving population is stored as the fp16 deviation from the reference
// of its reader, formed from the reader's moments in the workgroup's LDS planes
// (mom(K, DX, DY, DZ) is the moment pair K of site + (DX, DY, DZ)); a population sent
// into a wall face is read back by the site itself as opp(I), with the site's own
// moments and the reference of opp(I).  h_0 is written last as the complement T - (sum
// of the decoded moving values, in index order), so that the decoded values the site
// sends out sum to its h total.  (The site's moments word is written when it is
// gathered.)
template <class L, int WALLS, class MomAt>
struct SiteWriter16 {
    char* __restrict__ b;
    uint32_t site, S;
    const Codec& cd;
    MomAt mom;
    uint32_t solid;
    float T;                       // h total of the site
    float Sout = 0.f, g0 = 0.f;
    float D = 0.f;                 // moving-wall changes of the total (0 where they cancel)
    template <int I>
    __device__ __forceinline__ void put(float h, float g) {
        if constexpr (I == 0) {
            g0 = g;
        } else {
            constexpr int ex = L::cx(I), ey = L::cy(I), ez = L::cz(I);
            const bool back = dest_beyond<L, I, WALLS>(solid);
            // the reader's moments: (Phi, Psi) and the (jh, Jg) pairs of the axes c_I spans
            auto at = [&](int k) { return back ? mom(k, 0, 0, 0) : mom(k, ex, ey, ez); };
            const float2 p0 = at(0);
            const float2 px = ex ? at(1) : make_float2(0.f, 0.f);
            const float2 py = ey ? at(2) : make_float2(0.f, 0.f);
            const float2 pz = ez ? at(3) : make_float2(0.f, 0.f);
            // reference of population I at the reader, or of opp(I) (c = -c_I) at the site
            constexpr float w = L::w(I);
            const float sgn = back ? -3.0f : 3.0f;
            const float rh = w * fmaf(sgn, cdot<L, I>(px.x, py.x, pz.x), p0.x);
            const float rg = w * fmaf(sgn, cdot<L, I>(px.y, py.y, pz.y), p0.y);
            const __half qh = __float2half_rn((h - rh) * cd.sh);
            const __half qg = __float2half_rn((g - rg) * cd.sg);
            const float dec = fmaf(__half2float(qh), cd.ish, rh);
            Sout = I == 1 ? dec : Sout + dec;
            store_nt(b + StoreF16S::dev_off(S) + (size_t)(I - 1) * ((size_t)S * 4) +
                         elem_off<WALLS, 4>(site),
                     __halves2half2(qh, qg));
        }
    }
    // a moving wall changed an h value by d after the total was taken: the stored values
    // must sum to the changed total.  The changes are summed apart and added last: the
    // opposite changes of a tangential pair cancel exactly in D, which leaves T - Sout
    // (exact when Sout is within a factor two of T) untouched
    __device__ __forceinline__ void shift_h_total(double d) { D += (float)d; }
    __device__ __forceinline__ void finish() {
        store_nt(b + elem_off<WALLS, 8>(site), (T - Sout) + D, g0);
    }
};

// ---------------------------------------------------------------------------
// site coordinates and the phi stencil from a phi field (the non-hot kernels)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void site_coords(const Geom& G, uint32_t s, int& x, int& y, int& z) {
    z = (int)(s / G.sxy);
    const uint32_t r = s - (uint32_t)z * G.sxy;
    y = (int)(r / (uint32_t)G.nx);
    x = (int)(r - (uint32_t)y * (uint32_t)G.nx);
}

__device__ __forceinline__ uint32_t site_of(const Geom& G, int x, int y, int z) {
    return (uint32_t)z * G.sxy + (uint32_t)y * (uint32_t)G.nx + (uint32_t)x;
}

// phi(x + c_k) for all k from a phi field, with the ghost rules (mirror, wetting)
template <class L>
__device__ __forceinline__ void phi_stencil(const Geom& G, const Model& m,
                                            const float* __restrict__ phi,
                                            int x, int y, int z, float (&pn)[L::Q]) {
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int vx = x + L::cx(i), vy = y + L::cy(i), vz = z + L::cz(i);
        const int xx = map_coord(vx, G.nx, G.wx);
        const int yy = map_coord(vy, G.ny, G.wy);
        const int zz = map_coord(vz, G.nz, G.wz);
        pn[i] = phi[site_of(G, xx, yy, zz)];
        if (m.wetting) pn[i] = wet_ghost(G, m, vx, vy, vz, pn[i]);
    });
}

// user vector component a (0..D-1) -> internal axis
template <class L>
__device__ __forceinline__ int user_axis(int a) {
    if constexpr (L::USES_Y) return a;
    return a == 0 ? 0 : 2;
}

// float64 phi as hi + lo floats
__device__ __forceinline__ float split_hi_lo(double s, float& lo) {
    const float hi = (float)s;
    lo = (float)(s - (double)hi);
    return hi;
}

// ---------------------------------------------------------------------------
// per-site physics (Section 2, Eqs. 1-13, central differences)
// ---------------------------------------------------------------------------
struct Macro {
    float phi, gx, gy, gz, lap;
    float rho, itau, mu, nx, ny, nz, theta;
    float Fx, Fy, Fz, jx, jy, jz, ux, uy, uz, P;
};

// pn[k] = phi(x + c_k), gm = raw moments of the pre-collision hydrodynamic populations at x
template <class L>
__device__ __forceinline__ Macro macros(const Model& m, const float (&pn)[L::Q],
                                        const GMom& gm) {
    Macro a;
    a.phi = pn[0];
    // grad: pairs i, opp(i) contribute equally -> sum over odd i of w_i c_i (phi+ - phi-)/T
    float gx = 0.f, gy = 0.f, gz = 0.f, ls = 0.f;
    static_for<1, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (i & 1) {
            constexpr float wt = 3.0f * L::w(i);
            const float d = pn[i] - pn[i + 1];
            if constexpr (L::cx(i) != 0) gx = fmaf((float)L::cx(i) * wt, d, gx);
            if constexpr (L::cy(i) != 0) gy = fmaf((float)L::cy(i) * wt, d, gy);
            if constexpr (L::cz(i) != 0) gz = fmaf((float)L::cz(i) * wt, d, gz);
            // differences first: phi_k - phi is exact for neighbouring values
            ls = fmaf(L::w(i), (pn[i] - a.phi) + (pn[i + 1] - a.phi), ls);
        }
    });
    a.gx = gx; a.gy = gy; a.gz = gz;
    a.lap = 6.0f * ls;                                        // (2/T) sum w (phi_k - phi)
    a.rho = fmaf(a.phi, m.rho_dif, m.rho_L);
    a.itau = fmaf(a.phi, m.itau_dif, m.itau_L);
    const float ph = a.phi - 0.5f;
    a.mu = m.mu_a * a.phi * (a.phi - 1.0f) * ph - m.mu_b * a.lap;
    const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
    const float inv = 1.0f / (gn + m.eps);
    a.nx = gx * inv; a.ny = gy * inv; a.nz = gz * inv;
    // Eq. 4's 1 - 4 (phi - 1/2)^2 evaluated as 4 phi (1 - phi): the same value, without
    // the cancellation that leaves it only ~1e-7 / (phi (1 - phi)) accurate in float32
    // in the bulk phases (phi near 0 or 1), where the sharpening flux is then noise
    a.theta = m.th_a * (4.0f * a.phi) * (1.0f - a.phi);
    if (m.dth != 0.0f) {
        const bool dense = fabsf(ph) > 0.35f && ph * a.lap > 0.0f;
        a.theta = fmaf(dense ? -m.dth : 0.0f, gn, a.theta);
    }
    a.Fx = a.rho * m.gx; a.Fy = a.rho * m.gy; a.Fz = a.rho * m.gz;
    const float sg = gm.s;
    a.jx = fmaf(0.5f, fmaf(a.mu, gx, a.Fx), gm.jx);
    a.jy = fmaf(0.5f, fmaf(a.mu, gy, a.Fy), gm.jy);
    a.jz = fmaf(0.5f, fmaf(a.mu, gz, a.Fz), gm.jz);
    const float rho_p = fmaf(m.beta * 0.25f * m.rho_dif, a.lap, a.rho);
    const float irp = 1.0f / rho_p;
    a.ux = a.jx * irp; a.uy = a.jy * irp; a.uz = a.jz * irp;
    const float ug = a.ux * gx + a.uy * gy + a.uz * gz;
    // T sum g with T = 1/3 carried as two floats: float(1/3) alone is 3e-8 too large,
    // a bias the pressure would pick up at every step
    constexpr float third_lo = (float)(1.0 / 3.0 - (double)(1.0f / 3.0f));
    a.P = fmaf(1.0f / 3.0f, sg, third_lo * sg) + (m.rho_dif * (1.0f / 6.0f)) * ug;
    return a;
}

// Equilibria of direction I: Gamma_i = w_i (1 + e_i) (Eq. 3), h^eq (Eq. 2), K (Eq. 7),
// g^eq (Eq. 6 + Eq. 13).  The density terms are arranged so that rho*Gamma - w*rho
// is formed as w*rho*e (no cancellation of O(rho) terms in float32).
struct EqTerms {
    float e15;     // 1.5 u.u
    float ug, uF;  // u.grad(phi), u.F
    float A;       // rho_dif + 3 mu
    float dcoef;   // beta * 0.75 * rho_dif * lap
    float P3;      // 3 P
};

__device__ __forceinline__ EqTerms eq_terms(const Model& m, const Macro& a) {
    EqTerms t;
    t.e15 = 1.5f * (a.ux * a.ux + a.uy * a.uy + a.uz * a.uz);
    t.ug = a.ux * a.gx + a.uy * a.gy + a.uz * a.gz;
    t.uF = a.ux * a.Fx + a.uy * a.Fy + a.uz * a.Fz;
    t.A = fmaf(3.0f, a.mu, m.rho_dif);
    t.dcoef = m.beta * 0.75f * m.rho_dif * a.lap;
    t.P3 = 3.0f * a.P;
    return t;
}

// h^eq_i is returned split as phi w_i + hdev with hdev = w_i (phi e_i + theta c_i.n): in
// float32 the O(u) part e_i would be lost against 1 in w_i (1 + e_i) when |u| ~ 1e-7.
template <class L, int I>
__device__ __forceinline__ void eq_dir(const Macro& a, const EqTerms& t, float& hdev,
                                       float& geq, float& K) {
    constexpr float w = L::w(I);
    constexpr int ex = L::cx(I), ey = L::cy(I), ez = L::cz(I);
    float cu = 0.f, cg = 0.f, cF = 0.f, cn = 0.f;
    if constexpr (ex != 0) { cu += ex * a.ux; cg += ex * a.gx; cF += ex * a.Fx; cn += ex * a.nx; }
    if constexpr (ey != 0) { cu += ey * a.uy; cg += ey * a.gy; cF += ey * a.Fy; cn += ey * a.ny; }
    if constexpr (ez != 0) { cu += ez * a.uz; cg += ez * a.gz; cF += ez * a.Fz; cn += ez * a.nz; }
    const float e = fmaf(cu, fmaf(4.5f, cu, 3.0f), -t.e15);       // 3cu + 4.5cu^2 - 1.5u^2
    const float Gam = w * (1.0f + e);
    hdev = w * fmaf(a.phi, e, a.theta * cn);
    // (Gamma - w) rho_dif + Gamma mu/T = w (e (rho_dif + 3 mu) + 3 mu)
    const float kc = w * fmaf(e, t.A, 3.0f * a.mu);
    K = fmaf(kc, cg - t.ug, 3.0f * Gam * (cF - t.uF));
    // rho Gamma + w (P/T - rho) = w (rho e + 3P); Eq. 13: + w cu (3/4) rho_dif lap
    const float X = fmaf(a.rho, e, t.P3) + cu * t.dcoef;
    geq = fmaf(w, X, fmaf(L::w_lo(I), X, -0.5f * K));
}


// Full collision of one site, h BGK (Eq. 1) and the filtered g update (Eq. 10), with
// each post-collision pair handed to `out` as soon as it is formed.
//
// Pi = sum_l c_l c_l (g_l - g^eq_l) is built from the raw second moment of g and the
// closed form of the equilibrium's: with 4th-order isotropic weights (D2Q9, D3Q19),
//   sum_l c_a c_b g^eq_l = P delta_ab + rho u_a u_b - (1/2) sum_l c_a c_b K_l,
//   sum_l c_a c_b K_l = A [(u_a d_b + u_b d_a)/3 - u_a u_b (u.d)] + (rho_dif/3) delta_ab (u.d)
//                       + (u_a F_b + u_b F_a) - 3 u_a u_b (u.F),
// with d = grad(phi), A = rho_dif + 3 mu (T = 1/3); the delta f^eq term of Eq. 13 is odd
// in c and has no second moment.  Opposite velocities are handled as pairs, sharing
// c.u, c.d, c.F and c.n.  a.phi + phi_lo is the site's phi (see PhiAcc).
template <class L, class Out>
__device__ __forceinline__ void collide_stream(const Model& m, const Macro& a, float phi_lo,
                                               const float (&h)[L::Q], const GMom& gm,
                                               Out& out) {
    constexpr float third = 1.0f / 3.0f;
    const float ux = a.ux, uy = a.uy, uz = a.uz;
    const float E0 = -1.5f * (ux * ux + uy * uy + uz * uz);
    const float ug = ux * a.gx + uy * a.gy + uz * a.gz;
    const float uF = ux * a.Fx + uy * a.Fy + uz * a.Fz;
    const float A = fmaf(3.0f, a.mu, m.rho_dif);
    const float mu3 = 3.0f * a.mu;
    const float dcoef = m.beta * 0.75f * m.rho_dif * a.lap;
    const float P3 = 3.0f * a.P;
    const float om1 = 1.0f - a.itau;
    // raw second moments of g over the lattice's axes
    const float Mxx = gm.xx, Myy = gm.yy, Mzz = gm.zz, Mxy = gm.xy, Mxz = gm.xz, Myz = gm.yz;
    auto pi = [&](float M, float ua, float ub, float da, float db, float Fa, float Fb,
                  bool diag) {
        float sK = A * (fmaf(ua, db, ub * da) * third - ua * ub * ug) + fmaf(ua, Fb, ub * Fa) -
                   3.0f * ua * ub * uF;
        float eq = fmaf(a.rho * ua, ub, -0.5f * sK);
        if (diag) eq += a.P - (0.5f * third) * m.rho_dif * ug;
        return M - eq;
    };
    constexpr bool HX = true, HY = L::USES_Y, HZ = true;
    const float Pxx = HX ? pi(Mxx, ux, ux, a.gx, a.gx, a.Fx, a.Fx, true) : 0.f;
    const float Pyy = HY ? pi(Myy, uy, uy, a.gy, a.gy, a.Fy, a.Fy, true) : 0.f;
    const float Pzz = HZ ? pi(Mzz, uz, uz, a.gz, a.gz, a.Fz, a.Fz, true) : 0.f;
    const float Pxy = HY ? pi(Mxy, ux, uy, a.gx, a.gy, a.Fx, a.Fy, false) : 0.f;
    const float Pxz = pi(Mxz, ux, uz, a.gx, a.gz, a.Fx, a.Fz, false);
    const float Pyz = HY ? pi(Myz, uy, uz, a.gy, a.gz, a.Fy, a.Fz, false) : 0.f;
    const float tr3 = (Pxx + Pyy + Pzz) * third;
    const float hw0 = fmaf(a.phi, L::w(0), -h[0]);
    {   // rest population: c = 0
        constexpr float w = L::w(0), wl = L::w_lo(0);
        const float hdev = fmaf(a.phi, w * E0, a.phi * kappa<L>());
        const float ho = fmaf(m.om_phi, hw0 + fmaf(phi_lo, w, hdev), h[0]);
        const float K = w * (fmaf(E0, A, mu3) * (-ug) + 3.0f * (1.0f + E0) * (-uF));
        const float X = fmaf(a.rho, E0, P3);
        const float go = fmaf(w, X, fmaf(wl, X, fmaf(0.5f, K, om1 * 4.5f * w * (-tr3))));
        out.template put<0>(ho, go);
    }
    static_for<0, (L::Q - 1) / 2>([&](auto K_) {
        constexpr int i = 2 * decltype(K_)::value + 1;          // pair (i, i + 1), c_{i+1} = -c_i
        constexpr int ex = L::cx(i), ey = L::cy(i), ez = L::cz(i);
        constexpr float w = L::w(i), wl = L::w_lo(i);
        float cu = 0.f, cd = 0.f, cF = 0.f, cn = 0.f, ccP = 0.f;
        if constexpr (ex != 0) { cu += ex * ux; cd += ex * a.gx; cF += ex * a.Fx; cn += ex * a.nx; ccP += Pxx; }
        if constexpr (ey != 0) { cu += ey * uy; cd += ey * a.gy; cF += ey * a.Fy; cn += ey * a.ny; ccP += Pyy; }
        if constexpr (ez != 0) { cu += ez * uz; cd += ez * a.gz; cF += ez * a.Fz; cn += ez * a.nz; ccP += Pzz; }
        if constexpr (ex * ey != 0) ccP += (float)(2 * ex * ey) * Pxy;
        if constexpr (ex * ez != 0) ccP += (float)(2 * ex * ez) * Pxz;
        if constexpr (ey * ez != 0) ccP += (float)(2 * ey * ez) * Pyz;
        const float Ee = fmaf(4.5f * cu, cu, E0);                // even part of e
        const float O = 3.0f * cu;                               // odd part of e
        const float ep = Ee + O, em = Ee - O;
        // h: h + (h^eq - h)/tau_phi, h^eq - h = (phi w - h) + w (phi e + theta c.n)
        const float tn = a.theta * cn;
        const float hp = fmaf(m.om_phi, fmaf(a.phi, w, -h[i]) + fmaf(phi_lo, w, w * fmaf(a.phi, ep, tn)), h[i]);
        const float hm = fmaf(m.om_phi, fmaf(a.phi, w, -h[i + 1]) + fmaf(phi_lo, w, w * fmaf(a.phi, em, -tn)), h[i + 1]);
        // K_i = w [(e A + 3 mu)(c.d - u.d) + 3 (1 + e)(c.F - u.F)]             (Eq. 7)
        const float Kp = w * fmaf(fmaf(ep, A, mu3), cd - ug, 3.0f * (1.0f + ep) * (cF - uF));
        const float Km = w * fmaf(fmaf(em, A, mu3), -cd - ug, 3.0f * (1.0f + em) * (-cF - uF));
        // g* = w (rho e + 3P + (c.u) dcoef) + K/2 + (1 - 1/tau) 4.5 w (c c : Pi - tr/3).
        // The equilibrium part takes w as float(w_i) + w_lo: with float(w_i) alone the
        // equilibrium's momentum is rho u (1 + 7.5e-9), a gain that compounds over the
        // steps (after 1000 steps of the droplet impact, 1.9e-5 in phi)
        const float filt = om1 * 4.5f * w * (ccP - tr3);
        const float Xp = fmaf(a.rho, ep, P3) + cu * dcoef;
        const float Xm = fmaf(a.rho, em, P3) - cu * dcoef;
        const float gp = fmaf(w, Xp, fmaf(wl, Xp, fmaf(0.5f, Kp, filt)));
        const float gm = fmaf(w, Xm, fmaf(wl, Xm, fmaf(0.5f, Km, filt)));
        out.template put<i>(hp, gp);
        out.template put<i + 1>(hm, gm);
    });
    out.finish();
}

}  // namespace pflb
