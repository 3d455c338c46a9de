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
    // FP16S reference coefficients: dyadic r_i ~ 4 w_i with sum_i r_i = 4 exactly
    __host__ __device__ static constexpr float r(int i) {
        return i == 0 ? 1398112.0f / 1048576.0f
                      : (i <= 6 ? 233016.0f / 1048576.0f : 116508.0f / 1048576.0f);
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
    __host__ __device__ static constexpr float r(int i) {
        return i == 0 ? 1864144.0f / 1048576.0f
                      : (i <= 4 ? 466032.0f / 1048576.0f : 116508.0f / 1048576.0f);
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

template <class L>
__host__ __device__ constexpr bool dyadic_refs_sum_to_four() {
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) s += (double)L::r(i);
    return s == 4.0;
}

// ---------------------------------------------------------------------------
// geometry and model constants passed by value to every kernel
// ---------------------------------------------------------------------------
struct Geom {
    int nx, ny, nz;     // internal sizes
    int wx, wy, wz;     // 1: wall on both faces of the axis, 0: periodic
    uint32_t S;         // population stride of a set, in sites
    uint32_t sxy;       // nx * ny
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
};

struct Codec {                // FP16S: power-of-two scales of the fp16 deviations
    float sh, ish, sg, isg;
};

// ---------------------------------------------------------------------------
// storage codecs
// ---------------------------------------------------------------------------
struct StoreF32 {
    static constexpr bool HALF = false;
    // raw value of slot (site, pop) of direction I (I fixes the weight ratio only)
    template <class L, int I>
    __device__ __forceinline__ static float load(const char* __restrict__ b, int pop,
                                                 uint32_t site, uint32_t S, float) {
        return reinterpret_cast<const float*>(b)[(size_t)pop * S + site];
    }
};

// FP16S layout of a set: [R: S floats][dev_1..dev_{Q-1}: S halves each].  Slot (s, i)
// decodes to r_i R(s) + dev_i(s)/scale (i >= 1) and the rest slot to r_0 R(s), with the
// dyadic r_i ~ 4 w_i of the lattice (sum r_i = 4): R ~ phi/4 is the site's zeroth-order
// equilibrium level and the fp16 words hold the deviations from it.
struct StoreF16S {
    static constexpr bool HALF = true;
    template <class L, int I>
    __device__ __forceinline__ static float load(const char* __restrict__ b, int pop,
                                                 uint32_t site, uint32_t S, float iscale) {
        const float R = reinterpret_cast<const float*>(b)[site];
        if constexpr (I == 0) {
            return L::r(0) * R;
        } else {
            const __half* dev = reinterpret_cast<const __half*>(b + (size_t)S * 4);
            const float d = __half2float(dev[(size_t)(pop - 1) * S + site]);
            return fmaf(d, iscale, L::r(I) * R);
        }
    }
};

// Write the Q post-collision values of one site.  FP16S: the moving populations are
// rounded as deviations from r_i f_0 / r_0, and R is the complement
// (total - sum of decoded deviations) / 4 (an exact scaling), so that the decoded values
// of the site sum to `total` up to one float32 rounding (sum(phi) conservation).
template <class L, class ST>
__device__ __forceinline__ void store_site(char* __restrict__ b, uint32_t site, uint32_t S,
                                           const float (&f)[L::Q], float total, float total_lo,
                                           float scale, float iscale) {
    if constexpr (!ST::HALF) {
        float* o = reinterpret_cast<float*>(b);
        static_for<0, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            o[(size_t)i * S + site] = f[i];
        });
    } else {
        static_assert(dyadic_refs_sum_to_four<L>(), "reference coefficients must sum to 4");
        __half* dev = reinterpret_cast<__half*>(b + (size_t)S * 4);
        const float R0 = f[0] * (1.0f / L::r(0));
        float dsum = 0.0f;
        static_for<1, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const __half q = __float2half_rn((f[i] - L::r(i) * R0) * scale);
            dsum += __half2float(q) * iscale;
            dev[(size_t)(i - 1) * S + site] = q;
        });
        reinterpret_cast<float*>(b)[site] = 0.25f * ((total - dsum) + total_lo);
    }
}

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

// Upstream offsets of an (x, y) column: source x - 1 (for c_x = +1) and x + 1 (c_x = -1)
struct Col {
    uint32_t base;            // y*nx + x
    int dxm, dxp, dym, dyp;   // site offsets to the upstream site
    uint32_t solid;           // bit0: x-1 beyond a wall, bit1: x+1, bit2: y-1, bit3: y+1
};
struct ZRow {
    uint32_t base;            // z*nx*ny
    int dzm, dzp;
    uint32_t solid;           // bit4: z-1 beyond a wall, bit5: z+1
};

__device__ __forceinline__ Col make_col(const Geom& G, int x, int y) {
    Col c;
    c.base = (uint32_t)y * (uint32_t)G.nx + (uint32_t)x;
    c.dxm = (x == 0) ? G.nx - 1 : -1;
    c.dxp = (x == G.nx - 1) ? -(G.nx - 1) : 1;
    c.dym = (y == 0) ? (G.ny - 1) * G.nx : -G.nx;
    c.dyp = (y == G.ny - 1) ? -(G.ny - 1) * G.nx : G.nx;
    c.solid = 0;
    if (G.wx) c.solid |= (x == 0 ? 1u : 0u) | (x == G.nx - 1 ? 2u : 0u);
    if (G.wy) c.solid |= (y == 0 ? 4u : 0u) | (y == G.ny - 1 ? 8u : 0u);
    return c;
}

__device__ __forceinline__ ZRow make_zrow(const Geom& G, int z) {
    ZRow r;
    r.base = (uint32_t)z * G.sxy;
    r.dzm = (z == 0) ? (int)((G.nz - 1) * G.sxy) : -(int)G.sxy;
    r.dzp = (z == G.nz - 1) ? -(int)((G.nz - 1) * G.sxy) : (int)G.sxy;
    r.solid = 0;
    if (G.wz) r.solid = (z == 0 ? 16u : 0u) | (z == G.nz - 1 ? 32u : 0u);
    return r;
}

// Gather the Q pre-collision populations of one site.
template <class L, class ST, bool WALLS>
__device__ __forceinline__ void pull_site(const char* __restrict__ b, const Geom& G,
                                          const Col& c, const ZRow& r, float iscale,
                                          float (&f)[L::Q]) {
    const uint32_t site = c.base + r.base;
    const uint32_t solid = c.solid | r.solid;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = L::cx(i), ey = L::cy(i), ez = L::cz(i);
        int off = 0;
        if constexpr (ex > 0) off += c.dxm;
        if constexpr (ex < 0) off += c.dxp;
        if constexpr (ey > 0) off += c.dym;
        if constexpr (ey < 0) off += c.dyp;
        if constexpr (ez > 0) off += r.dzm;
        if constexpr (ez < 0) off += r.dzp;
        constexpr uint32_t need = (ex > 0 ? 1u : 0u) | (ex < 0 ? 2u : 0u) | (ey > 0 ? 4u : 0u) |
                                  (ey < 0 ? 8u : 0u) | (ez > 0 ? 16u : 0u) | (ez < 0 ? 32u : 0u);
        if constexpr (i == 0) {
            f[i] = ST::template load<L, i>(b, 0, site, G.S, iscale);
        } else if constexpr (WALLS) {
            const bool bb = (solid & need) != 0u;
            f[i] = ST::template load<L, i>(b, bb ? opp(i) : i, bb ? site : site + off, G.S, iscale);
        } else {
            f[i] = ST::template load<L, i>(b, i, site + off, G.S, iscale);
        }
    });
}

// ---------------------------------------------------------------------------
// per-site physics (Section 2, Eqs. 1-13, central differences)
// ---------------------------------------------------------------------------
struct Macro {
    float phi, gx, gy, gz, lap;
    float rho, itau, mu, nx, ny, nz, theta;
    float Fx, Fy, Fz, jx, jy, jz, ux, uy, uz, P;
};

// pn[k] = phi(x + c_k), g = pre-collision hydrodynamic populations at x
template <class L>
__device__ __forceinline__ Macro macros(const Model& m, const float (&pn)[L::Q],
                                        const float (&g)[L::Q]) {
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
    a.theta = m.th_a * (1.0f - 4.0f * ph * ph);
    if (m.dth != 0.0f) {
        const bool dense = fabsf(ph) > 0.35f && ph * a.lap > 0.0f;
        a.theta = fmaf(dense ? -m.dth : 0.0f, gn, a.theta);
    }
    a.Fx = a.rho * m.gx; a.Fy = a.rho * m.gy; a.Fz = a.rho * m.gz;
    float sg = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        sg += g[i];
        if constexpr (L::cx(i) > 0) jx += g[i];
        if constexpr (L::cx(i) < 0) jx -= g[i];
        if constexpr (L::cy(i) > 0) jy += g[i];
        if constexpr (L::cy(i) < 0) jy -= g[i];
        if constexpr (L::cz(i) > 0) jz += g[i];
        if constexpr (L::cz(i) < 0) jz -= g[i];
    });
    a.jx = fmaf(0.5f, fmaf(a.mu, gx, a.Fx), jx);
    a.jy = fmaf(0.5f, fmaf(a.mu, gy, a.Fy), jy);
    a.jz = fmaf(0.5f, fmaf(a.mu, gz, a.Fz), jz);
    const float rho_p = fmaf(m.beta * 0.25f * m.rho_dif, a.lap, a.rho);
    const float irp = 1.0f / rho_p;
    a.ux = a.jx * irp; a.uy = a.jy * irp; a.uz = a.jz * irp;
    const float ug = a.ux * gx + a.uy * gy + a.uz * gz;
    a.P = (1.0f / 3.0f) * sg + (m.rho_dif * (1.0f / 6.0f)) * ug;
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
    geq = fmaf(w, fmaf(a.rho, e, t.P3) + cu * t.dcoef, -0.5f * K);
}

// phi = sum_i f_i accumulated in float64 and returned as hi + lo floats.  The BGK update
// relaxes h towards phi w_i: with a float32 phi every site would gain or lose the
// rounding error of its own sum at every step (a random walk of the phase field).
template <class L>
__device__ __forceinline__ float phi_sum(const float (&f)[L::Q], float& lo) {
    double s = (double)f[0];
    static_for<1, L::Q>([&](auto I) { s += (double)f[decltype(I)::value]; });
    const float hi = (float)s;
    lo = (float)(s - (double)hi);
    return hi;
}

// Full collision of one site: h BGK (Eq. 1) and the filtered g update (Eq. 10).
// a.phi + phi_lo is the site's phi (see phi_sum).
template <class L>
__device__ __forceinline__ void collide(const Model& m, const Macro& a, float phi_lo,
                                        const float (&h)[L::Q], const float (&g)[L::Q],
                                        float (&ho)[L::Q], float (&go)[L::Q]) {
    const EqTerms t = eq_terms(m, a);
    float pxx = 0.f, pyy = 0.f, pzz = 0.f, pxy = 0.f, pxz = 0.f, pyz = 0.f;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        float hdev, geq, K;
        eq_dir<L, i>(a, t, hdev, geq, K);
        if constexpr (i == 0) hdev = fmaf(a.phi, kappa<L>(), hdev);
        // h + (h^eq - h)/tau_phi with h^eq - h = (phi w_i - h) + hdev
        ho[i] = fmaf(m.om_phi, fmaf(a.phi, L::w(i), -h[i]) + fmaf(phi_lo, L::w(i), hdev), h[i]);
        const float neq = g[i] - geq;
        constexpr int ex = L::cx(i), ey = L::cy(i), ez = L::cz(i);
        if constexpr (ex != 0) pxx += neq;
        if constexpr (ey != 0) pyy += neq;
        if constexpr (ez != 0) pzz += neq;
        if constexpr (ex * ey != 0) pxy += (float)(ex * ey) * neq;
        if constexpr (ex * ez != 0) pxz += (float)(ex * ez) * neq;
        if constexpr (ey * ez != 0) pyz += (float)(ey * ez) * neq;
        go[i] = geq + K;                                          // G^eq = g^eq + K
    });
    const float tr3 = (pxx + pyy + pzz) * (1.0f / 3.0f);
    const float om1 = 1.0f - a.itau;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = L::cx(i), ey = L::cy(i), ez = L::cz(i);
        float ccP = 0.f;                                           // c_i c_i : Pi
        if constexpr (ex != 0) ccP += pxx;
        if constexpr (ey != 0) ccP += pyy;
        if constexpr (ez != 0) ccP += pzz;
        if constexpr (ex * ey != 0) ccP += 2.0f * (float)(ex * ey) * pxy;
        if constexpr (ex * ez != 0) ccP += 2.0f * (float)(ex * ez) * pxz;
        if constexpr (ey * ez != 0) ccP += 2.0f * (float)(ey * ez) * pyz;
        // w_i / (2 T^2) (c_i c_i : Pi - T tr Pi) = 4.5 w_i (ccP - tr/3)
        go[i] = fmaf(om1 * 4.5f * L::w(i), ccP - tr3, go[i]);
    });
}

}  // namespace pflb
