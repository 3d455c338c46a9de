// In-place storage of the FP32 populations: one state buffer instead of two (half the
// footprint of the pull storage, so about twice the sites per GPU).
//
// Scheme (the "AA" pattern of in-place lattice Boltzmann streaming): two layouts of the
// same Q arrays of h followed by Q arrays of g, each array of stride S floats.
//   layout 0  f_i(x) is in slot (x, i);
//   layout 1  f_i(x) is in slot (x - c_i, opp(i)), or in slot (x, i) where x - c_i lies
//             beyond a wall (halfway bounce-back, Section 2's walls).
// A step from layout 0 reads a site's own slots and writes its post-collision f*_i into
// slot (x, opp(i)); the next step's reader x + c_i then finds it in slot
// ((x + c_i) - c_i, opp(i)): layout 1.  A step from layout 1 reads as layout 1 says and
// writes f*_i into slot (x + c_i, i), or into slot (x, opp(i)) where x + c_i lies beyond a
// wall: layout 0 again.  In either step the slots a site writes are exactly those it
// read, so sites never touch each other's slots and one buffer suffices.
//
// The price is phi: the collision needs phi at the neighbours (central differences,
// Eqs. 2-4 and 9), which other workgroups overwrite in place during the same launch.
// Each step therefore runs two kernels: k_ip_phi writes the phi field (reading only the
// h arrays, 76 B per D3Q19 site, writing 4 B), then k_ip_step collides every site with
// its neighbours' phi from that field (152 B read, 152 B written per site).  That is
// about 1.26x the bytes of the fused pull step, at half its state footprint.
#include "pflb_internal.hpp"

namespace pflb {
namespace {

// byte offset of slot (site, i) of set k (0: h, 1: g)
template <class L>
__device__ __forceinline__ size_t ip_off(uint32_t S, int k, int i, size_t site) {
    return (((size_t)(k * L::Q + i)) * S + site) * 4;
}

// neighbour x + (dx, dy, dz) with the periodic wrap; false where it lies beyond a wall
__device__ __forceinline__ bool ip_neighbour(const Geom& G, int x, int y, int z, int dx, int dy,
                                             int dz, size_t& t) {
    int v[3] = {x + dx, y + dy, z + dz};
    const int n[3] = {G.nx, G.ny, G.nz};
    const int w[3] = {G.wx, G.wy, G.wz};
    for (int a = 0; a < 3; ++a) {
        if (v[a] < 0 || v[a] >= n[a]) {
            if (w[a]) return false;
            v[a] = v[a] < 0 ? v[a] + n[a] : v[a] - n[a];
        }
    }
    t = site_of(G, v[0], v[1], v[2]);
    return true;
}

// (site, direction) of the slot where layout LY holds f_I(x)
template <class L, int I, int LY>
__device__ __forceinline__ size_t ip_src(const Geom& G, int x, int y, int z, size_t s, int& dir) {
    if constexpr (LY == 0 || I == 0) {
        dir = I;
        return s;
    } else {
        size_t t;
        if (!ip_neighbour(G, x, y, z, -L::cx(I), -L::cy(I), -L::cz(I), t)) {
            dir = I;
            return s;
        }
        dir = opp(I);
        return t;
    }
}

// f_i(x) for all i from layout LY; returns phi = sum h in float64, in index order (the
// sum the pull kernels form)
template <class L, int LY>
__device__ __forceinline__ double ip_load(const Geom& G, const char* __restrict__ b, int x, int y,
                                          int z, size_t s, float (&h)[L::Q], float (&g)[L::Q]) {
    double phi = 0.0;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        int dir;
        const size_t t = ip_src<L, i, LY>(G, x, y, z, s, dir);
        h[i] = *reinterpret_cast<const float*>(b + ip_off<L>(G.S, 0, dir, t));
        g[i] = *reinterpret_cast<const float*>(b + ip_off<L>(G.S, 1, dir, t));
        phi += (double)h[i];
    });
    return phi;
}

template <class L, int LY>
__device__ __forceinline__ double ip_phi(const Geom& G, const char* __restrict__ b, int x, int y,
                                         int z, size_t s) {
    double phi = 0.0;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        int dir;
        const size_t t = ip_src<L, i, LY>(G, x, y, z, s, dir);
        phi += (double)*reinterpret_cast<const float*>(b + ip_off<L>(G.S, 0, dir, t));
    });
    return phi;
}

// Writer of a site's post-collision pairs for a step from layout LY
template <class L, int LY>
struct IpWriter {
    char* __restrict__ b;
    const Geom& G;
    int x, y, z;
    size_t s;
    template <int I>
    __device__ __forceinline__ void put(float hv, float gv) {
        int dir = opp(I);
        size_t t = s;
        if constexpr (LY == 1) {
            size_t d;
            if (ip_neighbour(G, x, y, z, L::cx(I), L::cy(I), L::cz(I), d)) {
                dir = I;
                t = d;
            }
        }
        *reinterpret_cast<float*>(b + ip_off<L>(G.S, 0, dir, t)) = hv;
        *reinterpret_cast<float*>(b + ip_off<L>(G.S, 1, dir, t)) = gv;
    }
    __device__ __forceinline__ void finish() {}
    __device__ __forceinline__ void shift_h_total(double) {}
};

template <class L, int LY>
__global__ void __launch_bounds__(256)
k_ip_phi(Geom G, uint32_t N, const char* __restrict__ b, float* __restrict__ phi) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    phi[s] = (float)ip_phi<L, LY>(G, b, x, y, z, s);
}

template <class L, int LY>
__global__ void __launch_bounds__(256)
k_ip_step(Geom G, Model m, uint32_t N, char* __restrict__ b, const float* __restrict__ phi) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    float h[L::Q], g[L::Q];
    float lo;
    const float hi = split_hi_lo(ip_load<L, LY>(G, b, x, y, z, s, h, g), lo);
    float pn[L::Q];
    phi_stencil<L>(G, m, phi, x, y, z, pn);
    pn[0] = hi;      // the same float the phi kernel wrote (the same sum, rounded once)
    const GMom gm = g_moments<L>(g);
    const Macro a = macros<L>(m, pn, gm);
    IpWriter<L, LY> out{b, G, x, y, z, s};
    if (m.moving) {
        // moving walls: the momentum correction of the populations sent into them
        const uint32_t solid = make_col(G, x, y).solid | make_zrow(G, z).solid;
        WallWriter<L, IpWriter<L, LY>> wout{out, m, solid, 6.0f * a.phi, 6.0f * a.rho,
                                            solid != 0u};
        collide_stream<L>(m, a, lo, h, gm, wout);
    } else {
        collide_stream<L>(m, a, lo, h, gm, out);
    }
}

// state upload: pre-collision populations (h, g: Q arrays of N) into layout 0
template <class L>
__global__ void __launch_bounds__(256)
k_ip_set(Geom G, uint32_t N, const float* __restrict__ h, const float* __restrict__ g,
         char* __restrict__ b) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        *reinterpret_cast<float*>(b + ip_off<L>(G.S, 0, i, s)) = h[(size_t)i * N + s];
        *reinterpret_cast<float*>(b + ip_off<L>(G.S, 1, i, s)) = g[(size_t)i * N + s];
    });
}

template <class L, int LY>
__global__ void __launch_bounds__(256)
k_ip_get(Geom G, uint32_t N, const char* __restrict__ b, float* __restrict__ h,
         float* __restrict__ g) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    float fh[L::Q], fg[L::Q];
    ip_load<L, LY>(G, b, x, y, z, s, fh, fg);
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        h[(size_t)i * N + s] = fh[i];
        g[(size_t)i * N + s] = fg[i];
    });
}

// P, J and u (each may be NULL) from the state and its phi field
template <class L, int LY>
__global__ void __launch_bounds__(256)
k_ip_macro(Geom G, Model m, uint32_t N, const char* __restrict__ b, const float* __restrict__ phi,
           float* __restrict__ P, float* __restrict__ J, float* __restrict__ U) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    float pn[L::Q], hv[L::Q], gv[L::Q];
    phi_stencil<L>(G, m, phi, x, y, z, pn);
    ip_load<L, LY>(G, b, x, y, z, s, hv, gv);
    const Macro a = macros<L>(m, pn, g_moments<L>(gv));
    if (P) P[s] = a.P;
    const float jv[3] = {a.jx, a.jy, a.jz};
    const float uv[3] = {a.ux, a.uy, a.uz};
    for (int c = 0; c < L::D; ++c) {
        if (J) J[(size_t)c * N + s] = jv[user_axis<L>(c)];
        if (U) U[(size_t)c * N + s] = uv[user_axis<L>(c)];
    }
}

inline dim3 grid_of(uint32_t N) { return dim3((N + 255u) / 256u); }

template <class L, int LY>
hipError_t step_t(const Launch& a, void* b, float* phi) {
    const uint32_t N = (uint32_t)a.G.nx * a.G.ny * a.G.nz;
    hipLaunchKernelGGL((k_ip_phi<L, LY>), grid_of(N), dim3(256), 0, a.stream, a.G, N,
                       static_cast<const char*>(b), phi);
    hipLaunchKernelGGL((k_ip_step<L, LY>), grid_of(N), dim3(256), 0, a.stream, a.G, a.m, N,
                       static_cast<char*>(b), static_cast<const float*>(phi));
    return hipGetLastError();
}

template <class L>
hipError_t read_t(const Launch& a, uint32_t N, const void* b, int layout, float* phi, float* P,
                  float* J, float* U) {
    const char* c = static_cast<const char*>(b);
    if (layout)
        hipLaunchKernelGGL((k_ip_phi<L, 1>), grid_of(N), dim3(256), 0, a.stream, a.G, N, c, phi);
    else
        hipLaunchKernelGGL((k_ip_phi<L, 0>), grid_of(N), dim3(256), 0, a.stream, a.G, N, c, phi);
    if (P || J || U) {
        if (layout)
            hipLaunchKernelGGL((k_ip_macro<L, 1>), grid_of(N), dim3(256), 0, a.stream, a.G, a.m,
                               N, c, static_cast<const float*>(phi), P, J, U);
        else
            hipLaunchKernelGGL((k_ip_macro<L, 0>), grid_of(N), dim3(256), 0, a.stream, a.G, a.m,
                               N, c, static_cast<const float*>(phi), P, J, U);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step_inplace(const Launch& a, void* b, int layout, float* phi) {
    if (a.q == 19) return layout ? step_t<LatD3Q19, 1>(a, b, phi) : step_t<LatD3Q19, 0>(a, b, phi);
    return layout ? step_t<LatD2Q9, 1>(a, b, phi) : step_t<LatD2Q9, 0>(a, b, phi);
}

hipError_t launch_set_state_inplace(const Launch& a, uint32_t N, const float* h, const float* g,
                                    void* b) {
    char* c = static_cast<char*>(b);
    if (a.q == 19)
        hipLaunchKernelGGL((k_ip_set<LatD3Q19>), grid_of(N), dim3(256), 0, a.stream, a.G, N, h, g, c);
    else
        hipLaunchKernelGGL((k_ip_set<LatD2Q9>), grid_of(N), dim3(256), 0, a.stream, a.G, N, h, g, c);
    return hipGetLastError();
}

hipError_t launch_get_state_inplace(const Launch& a, uint32_t N, const void* b, int layout,
                                    float* h, float* g) {
    const char* c = static_cast<const char*>(b);
    const dim3 gr = grid_of(N);
    if (a.q == 19) {
        if (layout) hipLaunchKernelGGL((k_ip_get<LatD3Q19, 1>), gr, dim3(256), 0, a.stream, a.G, N, c, h, g);
        else hipLaunchKernelGGL((k_ip_get<LatD3Q19, 0>), gr, dim3(256), 0, a.stream, a.G, N, c, h, g);
    } else {
        if (layout) hipLaunchKernelGGL((k_ip_get<LatD2Q9, 1>), gr, dim3(256), 0, a.stream, a.G, N, c, h, g);
        else hipLaunchKernelGGL((k_ip_get<LatD2Q9, 0>), gr, dim3(256), 0, a.stream, a.G, N, c, h, g);
    }
    return hipGetLastError();
}

hipError_t launch_read_inplace(const Launch& a, uint32_t N, const void* b, int layout, float* phi,
                               float* P, float* J, float* U) {
    return a.q == 19 ? read_t<LatD3Q19>(a, N, b, layout, phi, P, J, U)
                     : read_t<LatD2Q9>(a, N, b, layout, phi, P, J, U);
}

}  // namespace pflb
