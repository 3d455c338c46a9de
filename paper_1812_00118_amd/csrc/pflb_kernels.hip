// HIP kernels of the phase-field lattice Boltzmann library (gfx950).
//
//   k_step         one fused pull-stream + collide pass for both sets (Eqs. 1, 10)
//   k_equilibrium  pre-collision equilibria from (phi, u, P)
//   k_set_state    pre-collision distributions -> pull storage
//   k_get_state    pull storage -> pre-collision distributions
//   k_phi, k_macro read-out of phi, P, J, u (end of Section 2)
//   k_mass_*       deterministic float64 sum of phi and non-finite flag
#include "pflb_device.hpp"
#include "pflb_internal.hpp"

namespace pflb {

// ---------------------------------------------------------------------------
// Fused step.  A workgroup owns a TX x TY column tile (D2Q9: TX x 1) and marches
// along z over BZ planes.  phi of plane z+1 on the tile plus a one-site ring is
// gathered into a 4-plane rolling LDS buffer (the h values of the tile's own sites
// are kept in registers for the collision of the next plane), then plane z is
// collided with grad(phi) and lap(phi) read from the LDS planes z-1, z, z+1.
// One barrier per plane: plane z+2 is written into the slot plane z-2 used, which
// no thread can still be reading once it has passed the barrier after plane z+1.
// ---------------------------------------------------------------------------
template <class L, class ST, int TX, int TY, bool WALLS>
__global__ void __launch_bounds__(TX * TY)
k_step(Geom G, Model m, Codec cd, int BZ, const char* __restrict__ hs,
       const char* __restrict__ gs, char* __restrict__ hd, char* __restrict__ gd) {
    constexpr int Q = L::Q;
    constexpr int HX = TX + 2;
    constexpr int HY = L::USES_Y ? TY + 2 : 1;
    constexpr int OY = L::USES_Y ? 1 : 0;
    constexpr int NR = L::USES_Y ? 2 * HX + 2 * TY : 2;
    static_assert(L::USES_Y || TY == 1, "D2Q9 tiles are one row high");
    static_assert(NR <= TX * TY, "ring larger than the workgroup");
    __shared__ float sphi[4][HY][HX];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * BZ;
    const int zend = min(z0 + BZ, G.nz);
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < G.nx && y < G.ny;

    const Col own = make_col(G, map_coord(x, G.nx, G.wx), map_coord(y, G.ny, G.wy));
    // ring position of this thread (if any)
    int rhx = 0, rhy = 0;
    const bool has_ring = tid < NR;
    if constexpr (L::USES_Y) {
        if (tid < HX) { rhx = tid; rhy = 0; }
        else if (tid < 2 * HX) { rhx = tid - HX; rhy = HY - 1; }
        else if (tid < 2 * HX + TY) { rhx = 0; rhy = 1 + tid - 2 * HX; }
        else { rhx = HX - 1; rhy = 1 + tid - 2 * HX - TY; }
    } else {
        rhx = (tid == 0) ? 0 : HX - 1;
    }
    const Col ring = make_col(G, map_coord(x0 - 1 + rhx, G.nx, G.wx),
                              L::USES_Y ? map_coord(y0 - 1 + rhy, G.ny, G.wy) : 0);

    auto ring_phi = [&](const ZRow& r) {
        float f[Q], lo;
        pull_site<L, ST, WALLS>(hs, G, ring, r, cd.ish, f);
        return phi_sum<L>(f, lo);
    };

    float hc[Q], lo_c;
    {   // plane z0 - 1 (phi only) and plane z0
        const ZRow rm = make_zrow(G, map_coord(z0 - 1, G.nz, G.wz));
        float f[Q], lo;
        pull_site<L, ST, WALLS>(hs, G, own, rm, cd.ish, f);
        sphi[(z0 - 1) & 3][ty + OY][tx + 1] = phi_sum<L>(f, lo);
        if (has_ring) sphi[(z0 - 1) & 3][rhy][rhx] = ring_phi(rm);
        const ZRow r0 = make_zrow(G, z0);
        pull_site<L, ST, WALLS>(hs, G, own, r0, cd.ish, hc);
        sphi[z0 & 3][ty + OY][tx + 1] = phi_sum<L>(hc, lo_c);
        if (has_ring) sphi[z0 & 3][rhy][rhx] = ring_phi(r0);
    }
    for (int z = z0; z < zend; ++z) {
        // phase A: plane z + 1
        float hn[Q], lo_n;
        const ZRow rn = make_zrow(G, map_coord(z + 1, G.nz, G.wz));
        pull_site<L, ST, WALLS>(hs, G, own, rn, cd.ish, hn);
        sphi[(z + 1) & 3][ty + OY][tx + 1] = phi_sum<L>(hn, lo_n);
        if (has_ring) sphi[(z + 1) & 3][rhy][rhx] = ring_phi(rn);
        __syncthreads();
        // phase B: collide plane z
        if (active) {
            const ZRow r = make_zrow(G, z);
            float gv[Q];
            pull_site<L, ST, WALLS>(gs, G, own, r, cd.isg, gv);
            float pn[Q];
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                pn[i] = sphi[(z + L::cz(i)) & 3][ty + OY + L::cy(i)][tx + 1 + L::cx(i)];
            });
            const Macro a = macros<L>(m, pn, gv);
            float ho[Q], go[Q];
            collide<L>(m, a, lo_c, hc, gv, ho, go);
            const uint32_t site = own.base + r.base;
            store_site<L, ST>(hd, site, G.S, ho, a.phi, lo_c, cd.sh, cd.ish);
            if constexpr (ST::HALF) {
                float glo;
                const float gsum = phi_sum<L>(go, glo);
                store_site<L, ST>(gd, site, G.S, go, gsum, glo, cd.sg, cd.isg);
            } else {
                store_site<L, ST>(gd, site, G.S, go, 0.0f, 0.0f, 1.0f, 1.0f);
            }
        }
        static_for<0, Q>([&](auto I) { hc[decltype(I)::value] = hn[decltype(I)::value]; });
        lo_c = lo_n;
    }
}

// ---------------------------------------------------------------------------
// per-site helpers for the non-hot kernels
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

// phi(x + c_k) for all k from a phi field, with the ghost rule
template <class L>
__device__ __forceinline__ void phi_stencil(const Geom& G, const float* __restrict__ phi,
                                            int x, int y, int z, float (&pn)[L::Q]) {
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int xx = map_coord(x + L::cx(i), G.nx, G.wx);
        const int yy = map_coord(y + L::cy(i), G.ny, G.wy);
        const int zz = map_coord(z + L::cz(i), G.nz, G.wz);
        pn[i] = phi[site_of(G, xx, yy, zz)];
    });
}

// user vector component a (0..D-1) -> internal axis
template <class L>
__device__ __forceinline__ int user_axis(int a) {
    if constexpr (L::USES_Y) return a;
    return a == 0 ? 0 : 2;
}

// ---------------------------------------------------------------------------
// equilibrium start
// ---------------------------------------------------------------------------
template <class L>
__global__ void __launch_bounds__(256)
k_equilibrium(Geom G, Model m, uint32_t N, const float* __restrict__ phi,
              const float* __restrict__ u, const float* __restrict__ P,
              float* __restrict__ h, float* __restrict__ g) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    float pn[L::Q];
    phi_stencil<L>(G, phi, x, y, z, pn);
    // macros with the given u and P: feed a zero g and overwrite J/u/P
    float zero[L::Q];
    static_for<0, L::Q>([&](auto I) { zero[decltype(I)::value] = 0.0f; });
    Macro a = macros<L>(m, pn, zero);
    float uu[3] = {0.f, 0.f, 0.f};
    for (int c = 0; c < L::D; ++c) uu[user_axis<L>(c)] = u[(size_t)c * N + s];
    a.ux = uu[0]; a.uy = uu[1]; a.uz = uu[2];
    a.P = P ? P[s] : 0.0f;
    const EqTerms t = eq_terms(m, a);
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        float hdev, geq, K;
        eq_dir<L, i>(a, t, hdev, geq, K);
        if constexpr (i == 0) hdev = fmaf(a.phi, kappa<L>(), hdev);
        h[(size_t)i * N + s] = fmaf(a.phi, L::w(i), hdev);
        g[(size_t)i * N + s] = geq;
    });
}

// ---------------------------------------------------------------------------
// pre-collision distributions <-> pull storage
// slot (y, j) is gathered by x = y + c_j as population j when x is a fluid site,
// otherwise by y itself as population opp(j)
// ---------------------------------------------------------------------------
template <class L, class ST>
__global__ void __launch_bounds__(256)
k_set_state(Geom G, Codec cd, uint32_t N, const float* __restrict__ h,
            const float* __restrict__ g, char* __restrict__ hb, char* __restrict__ gb) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    float fh[L::Q], fg[L::Q];
    static_for<0, L::Q>([&](auto I) {
        constexpr int j = decltype(I)::value;
        int xx = x + L::cx(j), yy = y + L::cy(j), zz = z + L::cz(j);
        const bool solid = (G.wx && (xx < 0 || xx >= G.nx)) || (G.wy && (yy < 0 || yy >= G.ny)) ||
                           (G.wz && (zz < 0 || zz >= G.nz));
        if (solid) {
            fh[j] = h[(size_t)opp(j) * N + s];
            fg[j] = g[(size_t)opp(j) * N + s];
        } else {
            const uint32_t t = site_of(G, map_coord(xx, G.nx, 0), map_coord(yy, G.ny, 0),
                                       map_coord(zz, G.nz, 0));
            fh[j] = h[(size_t)j * N + t];
            fg[j] = g[(size_t)j * N + t];
        }
    });
    if constexpr (!ST::HALF) {
        store_site<L, ST>(hb, s, G.S, fh, 0.f, 0.f, 1.f, 1.f);
        store_site<L, ST>(gb, s, G.S, fg, 0.f, 0.f, 1.f, 1.f);
    } else {
        // plain encoding: R from the rest population, deviations from r_i R
        auto enc = [&](char* b, const float (&f)[L::Q], float sc) {
            __half* dev = reinterpret_cast<__half*>(b + (size_t)G.S * 4);
            const float R = f[0] / L::r(0);
            reinterpret_cast<float*>(b)[s] = R;
            static_for<1, L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                dev[(size_t)(i - 1) * G.S + s] = __float2half_rn((f[i] - L::r(i) * R) * sc);
            });
        };
        enc(hb, fh, cd.sh);
        enc(gb, fg, cd.sg);
    }
}

template <class L, class ST, bool WALLS>
__global__ void __launch_bounds__(256)
k_get_state(Geom G, Codec cd, uint32_t N, const char* __restrict__ hb,
            const char* __restrict__ gb, float* __restrict__ h, float* __restrict__ g) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    const Col c = make_col(G, x, y);
    const ZRow r = make_zrow(G, z);
    float fh[L::Q], fg[L::Q];
    pull_site<L, ST, WALLS>(hb, G, c, r, cd.ish, fh);
    pull_site<L, ST, WALLS>(gb, G, c, r, cd.isg, fg);
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        h[(size_t)i * N + s] = fh[i];
        g[(size_t)i * N + s] = fg[i];
    });
}

// ---------------------------------------------------------------------------
// read-out
// ---------------------------------------------------------------------------
template <class L, class ST, bool WALLS>
__global__ void __launch_bounds__(256)
k_phi(Geom G, Codec cd, uint32_t N, const char* __restrict__ hb, float* __restrict__ phi) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    float f[L::Q];
    pull_site<L, ST, WALLS>(hb, G, make_col(G, x, y), make_zrow(G, z), cd.ish, f);
    float lo;
    phi[s] = phi_sum<L>(f, lo);
}

template <class L, class ST, bool WALLS>
__global__ void __launch_bounds__(256)
k_macro(Geom G, Model m, Codec cd, uint32_t N, const char* __restrict__ gb,
        const float* __restrict__ phi, float* __restrict__ P, float* __restrict__ J,
        float* __restrict__ U) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    float pn[L::Q], gv[L::Q];
    phi_stencil<L>(G, phi, x, y, z, pn);
    pull_site<L, ST, WALLS>(gb, G, make_col(G, x, y), make_zrow(G, z), cd.isg, gv);
    const Macro a = macros<L>(m, pn, gv);
    if (P) P[s] = a.P;
    const float jv[3] = {a.jx, a.jy, a.jz};
    const float uv[3] = {a.ux, a.uy, a.uz};
    for (int c = 0; c < L::D; ++c) {
        if (J) J[(size_t)c * N + s] = jv[user_axis<L>(c)];
        if (U) U[(size_t)c * N + s] = uv[user_axis<L>(c)];
    }
}

// ---------------------------------------------------------------------------
// sum of phi: every slot is gathered exactly once per step, so sum_x phi(x) is the
// sum of all decoded slots.  Per site in float64, per block by a fixed tree, then
// one block over the partial sums: the result does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int MASS_BLOCKS = 1024;
constexpr int MASS_THREADS = 256;

template <class L, class ST>
__device__ __forceinline__ double slot_sum(const char* b, uint32_t s, uint32_t S, float isc,
                                           bool& bad) {
    double acc = 0.0;
    if constexpr (!ST::HALF) {
        static_for<0, L::Q>([&](auto I) {
            const float v = reinterpret_cast<const float*>(b)[(size_t)decltype(I)::value * S + s];
            bad |= !isfinite(v);
            acc += (double)v;
        });
    } else {
        const float R = reinterpret_cast<const float*>(b)[s];
        bad |= !isfinite(R);
        acc = (double)L::r(0) * (double)R;
        const __half* dev = reinterpret_cast<const __half*>(b + (size_t)S * 4);
        static_for<1, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const float d = __half2float(dev[(size_t)(i - 1) * S + s]);
            bad |= !isfinite(d);
            acc += (double)L::r(i) * (double)R + (double)d * (double)isc;
        });
    }
    return acc;
}

template <class L, class ST>
__global__ void __launch_bounds__(MASS_THREADS)
k_mass_partial(Geom G, Codec cd, uint32_t N, const char* __restrict__ hb,
               const char* __restrict__ gb, double* __restrict__ part, int* __restrict__ flag) {
    __shared__ double sd[MASS_THREADS];
    __shared__ int sb[MASS_THREADS];
    double acc = 0.0;
    bool bad = false;
    for (uint32_t s = blockIdx.x * MASS_THREADS + threadIdx.x; s < N;
         s += MASS_BLOCKS * MASS_THREADS) {
        acc += slot_sum<L, ST>(hb, s, G.S, cd.ish, bad);
        (void)slot_sum<L, ST>(gb, s, G.S, cd.isg, bad);
    }
    sd[threadIdx.x] = acc;
    sb[threadIdx.x] = bad ? 1 : 0;
    __syncthreads();
    for (int w = MASS_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sd[threadIdx.x] += sd[threadIdx.x + w];
            sb[threadIdx.x] |= sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sd[0];
        flag[blockIdx.x] = sb[0];
    }
}

__global__ void __launch_bounds__(MASS_BLOCKS)
k_mass_final(const double* __restrict__ part, const int* __restrict__ flag,
             double* __restrict__ out, int* __restrict__ out_flag) {
    __shared__ double sd[MASS_BLOCKS];
    __shared__ int sb[MASS_BLOCKS];
    sd[threadIdx.x] = part[threadIdx.x];
    sb[threadIdx.x] = flag[threadIdx.x];
    __syncthreads();
    for (int w = MASS_BLOCKS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) {
            sd[threadIdx.x] += sd[threadIdx.x + w];
            sb[threadIdx.x] |= sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sd[0];
        out_flag[0] = sb[0];
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static inline dim3 grid1(uint32_t N) { return dim3((N + 255u) / 256u); }

template <class L, class ST, bool WALLS>
static hipError_t launch_step_t(const Launch& a, const char* hs, const char* gs, char* hd,
                                char* gd) {
    if constexpr (L::USES_Y) {
        constexpr int TX = 64, TY = 4;
        dim3 grid((a.G.nx + TX - 1) / TX, (a.G.ny + TY - 1) / TY, (a.G.nz + a.bz - 1) / a.bz);
        hipLaunchKernelGGL((k_step<L, ST, TX, TY, WALLS>), grid, dim3(TX * TY), 0, a.stream,
                           a.G, a.m, a.cd, a.bz, hs, gs, hd, gd);
    } else {
        constexpr int TX = 64;
        dim3 grid((a.G.nx + TX - 1) / TX, 1, (a.G.nz + a.bz - 1) / a.bz);
        hipLaunchKernelGGL((k_step<L, ST, TX, 1, WALLS>), grid, dim3(TX), 0, a.stream,
                           a.G, a.m, a.cd, a.bz, hs, gs, hd, gd);
    }
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t dispatch_walls(const Launch& a, const char* hs, const char* gs, char* hd,
                                 char* gd) {
    if (a.G.wx || a.G.wy || a.G.wz) return launch_step_t<L, ST, true>(a, hs, gs, hd, gd);
    return launch_step_t<L, ST, false>(a, hs, gs, hd, gd);
}

hipError_t launch_step(const Launch& a, const void* hs, const void* gs, void* hd, void* gd) {
    auto h_s = static_cast<const char*>(hs);
    auto g_s = static_cast<const char*>(gs);
    auto h_d = static_cast<char*>(hd);
    auto g_d = static_cast<char*>(gd);
    if (a.q == 19) {
        if (a.half) return dispatch_walls<LatD3Q19, StoreF16S>(a, h_s, g_s, h_d, g_d);
        return dispatch_walls<LatD3Q19, StoreF32>(a, h_s, g_s, h_d, g_d);
    }
    if (a.half) return dispatch_walls<LatD2Q9, StoreF16S>(a, h_s, g_s, h_d, g_d);
    return dispatch_walls<LatD2Q9, StoreF32>(a, h_s, g_s, h_d, g_d);
}

template <class L>
static hipError_t equilibrium_t(const Launch& a, uint32_t N, const float* phi, const float* u,
                                const float* P, float* h, float* g) {
    hipLaunchKernelGGL((k_equilibrium<L>), grid1(N), dim3(256), 0, a.stream, a.G, a.m, N, phi,
                       u, P, h, g);
    return hipGetLastError();
}

hipError_t launch_equilibrium(const Launch& a, uint32_t N, const float* phi, const float* u,
                              const float* P, float* h, float* g) {
    return a.q == 19 ? equilibrium_t<LatD3Q19>(a, N, phi, u, P, h, g)
                     : equilibrium_t<LatD2Q9>(a, N, phi, u, P, h, g);
}

template <class L, class ST>
static hipError_t set_state_t(const Launch& a, uint32_t N, const float* h, const float* g,
                              void* hb, void* gb) {
    hipLaunchKernelGGL((k_set_state<L, ST>), grid1(N), dim3(256), 0, a.stream, a.G, a.cd, N, h,
                       g, static_cast<char*>(hb), static_cast<char*>(gb));
    return hipGetLastError();
}

hipError_t launch_set_state(const Launch& a, uint32_t N, const float* h, const float* g,
                            void* hb, void* gb) {
    if (a.q == 19)
        return a.half ? set_state_t<LatD3Q19, StoreF16S>(a, N, h, g, hb, gb)
                      : set_state_t<LatD3Q19, StoreF32>(a, N, h, g, hb, gb);
    return a.half ? set_state_t<LatD2Q9, StoreF16S>(a, N, h, g, hb, gb)
                  : set_state_t<LatD2Q9, StoreF32>(a, N, h, g, hb, gb);
}

template <class L, class ST, bool WALLS>
static hipError_t get_state_t(const Launch& a, uint32_t N, const void* hb, const void* gb,
                              float* h, float* g) {
    hipLaunchKernelGGL((k_get_state<L, ST, WALLS>), grid1(N), dim3(256), 0, a.stream, a.G, a.cd,
                       N, static_cast<const char*>(hb), static_cast<const char*>(gb), h, g);
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t get_state_w(const Launch& a, uint32_t N, const void* hb, const void* gb,
                              float* h, float* g) {
    if (a.G.wx || a.G.wy || a.G.wz) return get_state_t<L, ST, true>(a, N, hb, gb, h, g);
    return get_state_t<L, ST, false>(a, N, hb, gb, h, g);
}

hipError_t launch_get_state(const Launch& a, uint32_t N, const void* hb, const void* gb,
                            float* h, float* g) {
    if (a.q == 19)
        return a.half ? get_state_w<LatD3Q19, StoreF16S>(a, N, hb, gb, h, g)
                      : get_state_w<LatD3Q19, StoreF32>(a, N, hb, gb, h, g);
    return a.half ? get_state_w<LatD2Q9, StoreF16S>(a, N, hb, gb, h, g)
                  : get_state_w<LatD2Q9, StoreF32>(a, N, hb, gb, h, g);
}

template <class L, class ST, bool WALLS>
static hipError_t read_t(const Launch& a, uint32_t N, const void* hb, const void* gb,
                         float* phi, float* P, float* J, float* U) {
    hipLaunchKernelGGL((k_phi<L, ST, WALLS>), grid1(N), dim3(256), 0, a.stream, a.G, a.cd, N,
                       static_cast<const char*>(hb), phi);
    if (P || J || U)
        hipLaunchKernelGGL((k_macro<L, ST, WALLS>), grid1(N), dim3(256), 0, a.stream, a.G, a.m,
                           a.cd, N, static_cast<const char*>(gb), phi, P, J, U);
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t read_w(const Launch& a, uint32_t N, const void* hb, const void* gb,
                         float* phi, float* P, float* J, float* U) {
    if (a.G.wx || a.G.wy || a.G.wz) return read_t<L, ST, true>(a, N, hb, gb, phi, P, J, U);
    return read_t<L, ST, false>(a, N, hb, gb, phi, P, J, U);
}

hipError_t launch_read(const Launch& a, uint32_t N, const void* hb, const void* gb, float* phi,
                       float* P, float* J, float* U) {
    if (a.q == 19)
        return a.half ? read_w<LatD3Q19, StoreF16S>(a, N, hb, gb, phi, P, J, U)
                      : read_w<LatD3Q19, StoreF32>(a, N, hb, gb, phi, P, J, U);
    return a.half ? read_w<LatD2Q9, StoreF16S>(a, N, hb, gb, phi, P, J, U)
                  : read_w<LatD2Q9, StoreF32>(a, N, hb, gb, phi, P, J, U);
}

template <class L, class ST>
static hipError_t mass_t(const Launch& a, uint32_t N, const void* hb, const void* gb,
                         void* scratch) {
    double* part = static_cast<double*>(scratch);
    int* flag = reinterpret_cast<int*>(part + MASS_BLOCKS + 1);
    hipLaunchKernelGGL((k_mass_partial<L, ST>), dim3(MASS_BLOCKS), dim3(MASS_THREADS), 0,
                       a.stream, a.G, a.cd, N, static_cast<const char*>(hb),
                       static_cast<const char*>(gb), part, flag);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(MASS_BLOCKS), 0, a.stream, part, flag,
                       part + MASS_BLOCKS, flag + MASS_BLOCKS);
    return hipGetLastError();
}

hipError_t launch_mass(const Launch& a, uint32_t N, const void* hb, const void* gb,
                       void* scratch) {
    if (a.q == 19)
        return a.half ? mass_t<LatD3Q19, StoreF16S>(a, N, hb, gb, scratch)
                      : mass_t<LatD3Q19, StoreF32>(a, N, hb, gb, scratch);
    return a.half ? mass_t<LatD2Q9, StoreF16S>(a, N, hb, gb, scratch)
                  : mass_t<LatD2Q9, StoreF32>(a, N, hb, gb, scratch);
}

size_t mass_scratch_bytes() {
    return (MASS_BLOCKS + 1) * sizeof(double) + (MASS_BLOCKS + 1) * sizeof(int);
}

size_t mass_result_offset() { return MASS_BLOCKS * sizeof(double); }
size_t mass_flag_offset() {
    return (MASS_BLOCKS + 1) * sizeof(double) + MASS_BLOCKS * sizeof(int);
}

}  // namespace pflb
