// HIP kernels of the phase-field lattice Boltzmann library (gfx950).
//
//   k_step         one fused pull-stream + collide pass for both sets (Eqs. 1, 10), for
//                  one context or a batch of contexts
//   k_equilibrium  pre-collision equilibria from (phi, u, P); *_j_b: from (phi, J, P)
//   k_set_state    pre-collision distributions -> pull storage
//   k_get_state    pull storage -> pre-collision distributions
//   k_phi, k_macro read-out of phi, P, J, u (end of Section 2)
//   *_b            the same over a batch of contexts (blockIdx.y = context)
//   k_mass_*       deterministic float64 sum of phi and non-finite flag
#include "pflb_device.hpp"
#include "pflb_internal.hpp"

namespace pflb {

// Workgroup -> tile.  Workgroups are dispatched round-robin over the 8 XCDs (each with
// its own L2); tile t goes to the workgroup that makes each XCD sweep a contiguous run
// of tiles, so the y-neighbours whose halos overlap share an L2 while they run.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
    const int xcd = b & 7, loc = b >> 3, per = nblk >> 3, rem = nblk & 7;
    return xcd < rem ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
}

// Workgroup barrier over LDS traffic only.  Inside the step no thread reads global
// memory that another thread writes (src is read-only, dst write-only), so the global
// stores of a finished plane may stay in flight across it; __syncthreads() would wait
// for them (vmcnt(0)) at every plane.  The memory clobber keeps the compiler from
// moving LDS accesses across it.
// Keeps v computed on every lane at this point: a value used only under a per-lane
// condition is otherwise sunk into that branch, and so are its loads
__device__ __forceinline__ void keep(float v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void keep(const uint4& w) {
    asm volatile("" ::"v"(w.x), "v"(w.y), "v"(w.z), "v"(w.w));
}

__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---------------------------------------------------------------------------
// Fused step.  A workgroup owns a TX x TY column tile (D2Q9: TX x 1) and marches
// along z over BZ planes.  phi of plane z+1 on the tile plus a one-site ring is
// gathered into a 4-plane rolling LDS buffer (the tile's own sites keep their h values
// and the raw moments of their g values in registers for the collision of the next
// plane), then plane z is
// collided with grad(phi) and lap(phi) read from the LDS planes z-1, z, z+1.
// One barrier per plane: plane z+2 is written into the slot plane z-2 used, which
// no thread can still be reading once it has passed the barrier after plane z+1.
// ---------------------------------------------------------------------------
// XBC: the variant for the extra wall conditions, moving walls (momentum-corrected
// bounce-back, WallWriter) and contact angles (the wetting ghost rule), kept apart so
// that the other variants carry none of their registers.
//
// BATCHED: a batch of resting-wall contexts that share lattice, storage and geometry;
// blockIdx.y picks the context, whose buffers and parameters replace src, dst, m and cd.
// (The single-context kernel takes an empty table; the body stays in the kernel itself,
// which compiles to measurably faster code than the same body in an inlined function.)
template <bool BATCHED>
struct StepTable {};
template <>
struct StepTable<true> {
    StepBatch bt;
};

// The FP16S XBC variants are held to two waves per SIMD: they need a few registers
// more than 256 and would otherwise run one wave per SIMD; the spills this costs are
// cheaper (measured: all-wall boxes with contact angles or moving walls 1.7-1.9x faster).
template <class L, class ST, int TX, int TY, int WALLS, bool XBC, bool BATCHED>
__global__ void __launch_bounds__(TX * TY)
__attribute__((amdgpu_waves_per_eu(XBC && ST::HALF ? 2 : 1)))
k_step(Geom G, Model m, Codec cd, int BZ, int ntx, int nty, int nblk,
       const char* __restrict__ src, char* __restrict__ dst, StepTable<BATCHED> tab) {
    static_assert(!(BATCHED && XBC), "contexts with moving walls or contact angles are stepped one by one");
    if constexpr (BATCHED) {
        const StepEnt& e = tab.bt.e[blockIdx.y];
        m = e.m;
        cd = e.cd;
        src = e.src;
        dst = e.dst;
    }
    constexpr int Q = L::Q;
    constexpr int WS = WALLS & WALLS_XYZ;   // the wall set without the addressing flag
    constexpr int HX = TX + 2;
    constexpr int HY = L::USES_Y ? TY + 2 : 1;
    constexpr int OY = L::USES_Y ? 1 : 0;
    constexpr int NR = L::USES_Y ? 2 * HX + 2 * TY : 2;
    static_assert(L::USES_Y || TY == 1, "D2Q9 tiles are one row high");
    static_assert(NR <= TX * TY, "ring larger than the workgroup");
    constexpr bool HALF = ST::HALF;
    __shared__ float sphi[4][HY][HX];
    // FP16S: the moments of the same positions as the writers use them (the fp16 values
    // of each site's moments word, held as floats), one array per pair (Phi, Psi),
    // (jh_x, Jg_x), (jh_y, Jg_y), (jh_z, Jg_z) so that neighbouring lanes read
    // neighbouring words
    __shared__ float2 smom[HALF ? 4 : 1][4][HALF ? HY : 1][HALF ? HX : 1];
    auto put_mom = [&](int zr, int py, int px, const uint4& mw) {
        if constexpr (HALF) {
            smom[zr & 3][0][py][px] = unpack_h2(mw.x);
            smom[zr & 3][1][py][px] = unpack_h2(mw.y);
            smom[zr & 3][2][py][px] = unpack_h2(mw.z);
            smom[zr & 3][3][py][px] = unpack_h2(mw.w);
        }
    };

    const int t = xcd_tile(blockIdx.x, nblk);
    const int bx = t % ntx;
    const int byz = t / ntx;
    const int by = byz % nty;
    const int bzi = byz / nty;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x0 = bx * TX, y0 = by * TY, z0 = bzi * BZ;
    const int zend = min(z0 + BZ, G.nz);
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < G.nx && y < G.ny;

    const Col own = make_col(G, map_coord(x, G.nx, G.wx), map_coord(y, G.ny, G.wy));
    // Without walls across x or y (whose ring gathers take per-lane wall tests) and
    // outside the XBC variants the own and the ring gathers of a plane are issued with no
    // branch between them, so that their loads are in flight together: every thread
    // gathers a ring site (threads past the ring take their wave's first ring position
    // or, in a wave without one, the last, so the duplicates fall in lines their wave or a
    // neighbouring one loads anyway) and only the ring threads store theirs.  Measured:
    // rising bubble FP32 unchanged, FP16S 3% faster, droplet impact 2% and 4.5%; with x/y
    // walls, and in the XBC variants (FP16S moving walls 27% slower), it measured slower.
    constexpr bool TOGETHER = (WS & WALLS_XY) == 0 && !XBC;
    int rhx = 0, rhy = 0;
    const bool has_ring = tid < NR;
    const int rid = (!TOGETHER || tid < NR) ? tid : ((tid & ~63) < NR ? (tid & ~63) : NR - 1);
    if constexpr (L::USES_Y) {
        if (rid < HX) { rhx = rid; rhy = 0; }
        else if (rid < 2 * HX) { rhx = rid - HX; rhy = HY - 1; }
        else if (rid < 2 * HX + TY) { rhx = 0; rhy = 1 + rid - 2 * HX; }
        else { rhx = HX - 1; rhy = 1 + rid - 2 * HX - TY; }
    } else {
        rhx = (rid == 0) ? 0 : HX - 1;
    }
    const Col ring = make_col(G, map_coord(x0 - 1 + rhx, G.nx, G.wx),
                              L::USES_Y ? map_coord(y0 - 1 + rhy, G.ny, G.wy) : 0);

    // contact angles (XBC variant): ghost positions beyond wall faces (the own lanes
    // past a ragged edge, the ring past the domain, the planes below and above it) take
    // the wetting rule
    const int rrx = x0 - 1 + rhx, rry = L::USES_Y ? y0 - 1 + rhy : 0;
    auto wet = [&](float v, int vx, int vy, int vz) {
        if constexpr (WS != WALLS_NONE && XBC) {
            if (m.wetting) return wet_ghost(G, m, vx, vy, vz, v);
        }
        return v;
    };
    // phi (and, FP16S, the moments word) of a site kept only for the neighbours: a ring
    // site, or an own site of a plane this workgroup does not collide
    auto side_site = [&](const Col& cc, const ZRow& r, int zr, int py, int px, int vx, int vy) {
        if constexpr (HALF) {
            uint4 mw;
            const float ph = pull_site_mom16<L, WALLS>(src, G, cc, r, cd, mw);
            sphi[zr & 3][py][px] = wet(ph, vx, vy, zr);
            put_mom(zr, py, px, mw);
        } else {
            float f[Q];
            sphi[zr & 3][py][px] = wet((float)pull_site_h<L, ST, WALLS>(src, G, cc, r, cd, f), vx, vy, zr);
        }
    };
    // an own site that will be collided: its h values and g moments stay in registers
    auto own_site = [&](const ZRow& r, int zr, float (&hv)[Q], GMom& gv, float& lo) {
        if constexpr (HALF) {
            uint4 mw;
            const float ph = pull_site_m16<L, WALLS>(src, G, own, r, cd, hv, gv, mw);
            lo = 0.0f;
            sphi[zr & 3][ty + OY][tx + 1] = wet(ph, x, y, zr);
            put_mom(zr, ty + OY, tx + 1, mw);
            // the site's moments word of this step, read back by the site at the next one
            if (active)
                store_nt(dst + StoreF16S::mom_off(G.S) + elem_off<WALLS, 16>(own.base + r.base),
                         mw);
        } else {
            sphi[zr & 3][ty + OY][tx + 1] =
                wet(split_hi_lo(pull_site_m<L, WALLS>(src, G, own, r, hv, gv), lo), x, y, zr);
        }
    };

    float hA[Q], loA, hB[Q], loB;
    GMom gA, gB;
    if constexpr (!TOGETHER) {   // plane z0 - 1 (for the neighbours only) and plane z0
        const ZRow rm = make_zrow(G, map_coord(z0 - 1, G.nz, G.wz));
        side_site(own, rm, z0 - 1, ty + OY, tx + 1, x, y);
        if (has_ring) side_site(ring, rm, z0 - 1, rhy, rhx, rrx, rry);
        const ZRow r0 = make_zrow(G, z0);
        own_site(r0, z0, hA, gA, loA);
        if (has_ring) side_site(ring, r0, z0, rhy, rhx, rrx, rry);
    } else if constexpr (HALF) {
        // plane z0 - 1 (for the neighbours only) and plane z0, own and ring gathers with no
        // branch between them
        const ZRow rm = make_zrow(G, map_coord(z0 - 1, G.nz, G.wz));
        const ZRow r0 = make_zrow(G, z0);
        uint4 wm, w0, vm, v0;
        const float pm = pull_site_mom16<L, WALLS>(src, G, own, rm, cd, wm);
        const float p0 = pull_site_m16<L, WALLS>(src, G, own, r0, cd, hA, gA, w0);
        const float qm = pull_site_mom16<L, WALLS>(src, G, ring, rm, cd, vm);
        const float q0 = pull_site_mom16<L, WALLS>(src, G, ring, r0, cd, v0);
        keep(qm);
        keep(q0);
        keep(vm);
        keep(v0);
        loA = 0.0f;
        sphi[(z0 - 1) & 3][ty + OY][tx + 1] = wet(pm, x, y, z0 - 1);
        put_mom(z0 - 1, ty + OY, tx + 1, wm);
        sphi[z0 & 3][ty + OY][tx + 1] = wet(p0, x, y, z0);
        put_mom(z0, ty + OY, tx + 1, w0);
        if (active)
            store_nt(dst + StoreF16S::mom_off(G.S) + elem_off<WALLS, 16>(own.base + r0.base), w0);
        if (has_ring) {
            sphi[(z0 - 1) & 3][rhy][rhx] = wet(qm, rrx, rry, z0 - 1);
            put_mom(z0 - 1, rhy, rhx, vm);
            sphi[z0 & 3][rhy][rhx] = wet(q0, rrx, rry, z0);
            put_mom(z0, rhy, rhx, v0);
        }
    } else {
        // FP32: the four gathers with no branch between them; the ring threads store their
        // ring values after
        const ZRow rm = make_zrow(G, map_coord(z0 - 1, G.nz, G.wz));
        const ZRow r0 = make_zrow(G, z0);
        float f[Q];
        const float pm = (float)pull_site_h<L, ST, WALLS>(src, G, own, rm, cd, f);
        const float p0 = split_hi_lo(pull_site_m<L, WALLS>(src, G, own, r0, hA, gA), loA);
        const float qm = (float)pull_site_h<L, ST, WALLS>(src, G, ring, rm, cd, f);
        const float q0 = (float)pull_site_h<L, ST, WALLS>(src, G, ring, r0, cd, f);
        keep(qm);
        keep(q0);
        sphi[(z0 - 1) & 3][ty + OY][tx + 1] = wet(pm, x, y, z0 - 1);
        sphi[z0 & 3][ty + OY][tx + 1] = wet(p0, x, y, z0);
        if (has_ring) {
            sphi[(z0 - 1) & 3][rhy][rhx] = wet(qm, rrx, rry, z0 - 1);
            sphi[z0 & 3][rhy][rhx] = wet(q0, rrx, rry, z0);
        }
    }
    // One plane: gather plane z+1 into (hn, gn), then collide plane z from (hc, gc)
    // (h values and g moments).
    auto plane = [&](int z, const float (&hc)[Q], const GMom& gc, float lo_c,
                     float (&hn)[Q], GMom& gn, float& lo_n) {
        const ZRow rn = make_zrow(G, map_coord(z + 1, G.nz, G.wz));
        // gather phase at raised wave priority, so that the SIMD issues the loads of waves
        // reaching it ahead of other waves' collision arithmetic (measured: 1-3% faster);
        // back to normal after the barrier
        __builtin_amdgcn_s_setprio(2);
        if constexpr (!TOGETHER) {
            if constexpr (HALF) {
                if (z + 1 < zend) {
                    own_site(rn, z + 1, hn, gn, lo_n);
                } else {
                    // the plane above the chunk, for the neighbours only
                    side_site(own, rn, z + 1, ty + OY, tx + 1, x, y);
                }
            } else {
                // (one phi store after either gather: measured faster than one per branch)
                const double pn64 = (z + 1 < zend)
                                        ? pull_site_m<L, WALLS>(src, G, own, rn, hn, gn)
                                        : pull_site_h<L, ST, WALLS>(src, G, own, rn, cd, hn);
                sphi[(z + 1) & 3][ty + OY][tx + 1] = wet(split_hi_lo(pn64, lo_n), x, y, z + 1);
            }
            if (has_ring) side_site(ring, rn, z + 1, rhy, rhx, rrx, rry);
        } else if constexpr (HALF) {
            // the own and the ring gather with no branch between them (the plane above the
            // chunk is gathered like a collided one, its moments word not stored)
            uint4 mw, rmw;
            const float ph = pull_site_m16<L, WALLS>(src, G, own, rn, cd, hn, gn, mw);
            const float rph = pull_site_mom16<L, WALLS>(src, G, ring, rn, cd, rmw);
            keep(rph);
            keep(rmw);
            lo_n = 0.0f;
            sphi[(z + 1) & 3][ty + OY][tx + 1] = wet(ph, x, y, z + 1);
            put_mom(z + 1, ty + OY, tx + 1, mw);
            // the site's moments word of this step, read back by the site at the next one
            if (active && z + 1 < zend)
                store_nt(dst + StoreF16S::mom_off(G.S) + elem_off<WALLS, 16>(own.base + rn.base),
                         mw);
            if (has_ring) {
                sphi[(z + 1) & 3][rhy][rhx] = wet(rph, rrx, rry, z + 1);
                put_mom(z + 1, rhy, rhx, rmw);
            }
        } else {
            // the own and the ring gather with no branch between them, so that their loads
            // are in flight together (the plane above the chunk is gathered as a collided
            // one: the same lines, its g moments unused)
            const double pn64 = pull_site_m<L, WALLS>(src, G, own, rn, hn, gn);
            float f[Q];
            const float qn = (float)pull_site_h<L, ST, WALLS>(src, G, ring, rn, cd, f);
            keep(qn);
            sphi[(z + 1) & 3][ty + OY][tx + 1] = wet(split_hi_lo(pn64, lo_n), x, y, z + 1);
            if (has_ring) sphi[(z + 1) & 3][rhy][rhx] = wet(qn, rrx, rry, z + 1);
        }
        lds_barrier();
        __builtin_amdgcn_s_setprio(0);
        if (active) {
            const ZRow r = make_zrow(G, z);
            float pn[Q];
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                pn[i] = sphi[(z + L::cz(i)) & 3][ty + OY + L::cy(i)][tx + 1 + L::cx(i)];
            });
            const Macro a = macros<L>(m, pn, gc);
            const uint32_t solid = own.solid | r.solid;
            auto collide_to = [&](auto& out) {
                if constexpr (WS == WALLS_NONE || !XBC) {
                    collide_stream<L>(m, a, lo_c, hc, gc, out);
                } else {
                    const bool on =
                        m.moving && __builtin_amdgcn_ballot_w64(solid != 0u) != 0ull;
                    WallWriter<L, std::remove_reference_t<decltype(out)>> wout{
                        out, m, solid, 6.0f * a.phi, 6.0f * a.rho, on};
                    collide_stream<L>(m, a, lo_c, hc, gc, wout);
                }
            };
            if constexpr (HALF) {
                // the moment pair k of site + (dx, dy, dz)
                auto mom_at = [&](int k, int dx, int dy, int dz) -> float2 {
                    return smom[(z + dz) & 3][k][ty + OY + dy][tx + 1 + dx];
                };
                SiteWriter16<L, WALLS, decltype(mom_at)> out{dst, own.base + r.base, G.S, cd,
                                                             mom_at, solid, a.phi};
                collide_to(out);
            } else {
                SiteWriter32<L, WALLS> out{dst, own.base + r.base, G.S};
                collide_to(out);
            }
        }
    };
    for (int z = z0; z < zend; z += 2) {
        plane(z, hA, gA, loA, hB, gB, loB);
        if (z + 1 < zend) plane(z + 1, hB, gB, loB, hA, gA, loA);
    }
}

// D2Q9 FP32 step without contact angles or moving walls, for chunks of one or two rows
// along the second axis (one-wave workgroups of 64 sites along x; small two-dimensional
// domains want many short chunks for their parallelism).  Marching such a chunk row by
// row waits for memory once per row (the gather of row z+1 must land before row z can
// collide); here the own sites of all NB + 2 rows a chunk needs (its rows, the one below
// and the one above) are gathered with no branch between them, so that their loads are in
// flight together, then the two ring sites of every row, and the rows are collided from
// registers.  The per-site arithmetic, the phi values and the stores are the marching
// kernel's (measured bitwise the same; 6-10% faster on 256x1024 and 256x256 domains).
template <class L, int WALLS, bool BATCHED, int NB>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
k_step_rows(Geom G, Model m, int ntx, int nblk, const char* __restrict__ src,
            char* __restrict__ dst, StepTable<BATCHED> tab) {
    static_assert(!L::USES_Y, "rows of a two-dimensional lattice");
    static_assert(NB == 1 || NB == 2, "chunks of one or two rows");
    if constexpr (BATCHED) {
        const StepEnt& e = tab.bt.e[blockIdx.y];
        m = e.m;
        src = e.src;
        dst = e.dst;
    }
    constexpr int Q = L::Q;
    constexpr int TX = 64;
    constexpr int HX = TX + 2;
    constexpr int NP = NB + 2;                 // rows z0 - 1 .. z0 + NB
    __shared__ float sphi[NP][HX];

    const int t = xcd_tile(blockIdx.x, nblk);
    const int bx = t % ntx;
    const int bzi = t / ntx;
    const int tx = threadIdx.x;
    const int x0 = bx * TX, z0 = bzi * NB;
    const int zend = min(z0 + NB, G.nz);
    const int x = x0 + tx;
    const bool active = x < G.nx;
    const Col own = make_col(G, map_coord(x, G.nx, G.wx), 0);
    // ring sites x0 - 1 (lane 0) and x0 + 64 (lane 1); every lane computes the one of its
    // parity, so the ring needs no branch of its own (the compiler moves the ring's loads
    // under the store's condition, lanes 0 and 1: measured faster here than keeping them
    // on every lane), and lanes 0 and 1 store it
    const bool has_ring = tx < 2;
    const int rhx = (tx & 1) ? HX - 1 : 0;
    const Col ring = make_col(G, map_coord(x0 - 1 + rhx, G.nx, G.wx), 0);

    // the rows' addressing first (scalar work with branches of its own); rows past the
    // one above the chunk stand for that row, gathered again and unused
    ZRow rows[NP];
    static_for<0, NP>([&](auto P) {
        constexpr int p = decltype(P)::value;
        const int z = min(z0 - 1 + p, zend);
        rows[p] = make_zrow(G, z < 0 ? (G.wz ? 0 : G.nz - 1)
                                     : (z >= G.nz ? (G.wz ? G.nz - 1 : 0) : z));
    });
    float hv[NB][Q], lo[NB], rphi[NP];
    GMom gv[NB];
    static_for<0, NP>([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (p >= 1 && p <= NB) {
            sphi[p][tx + 1] = split_hi_lo(
                pull_site_m<L, WALLS>(src, G, own, rows[p], hv[p - 1], gv[p - 1]), lo[p - 1]);
        } else {
            float f[Q];
            sphi[p][tx + 1] = (float)pull_site_h<L, StoreF32, WALLS>(src, G, own, rows[p],
                                                                     Codec{}, f);
        }
    });
    static_for<0, NP>([&](auto P) {
        constexpr int p = decltype(P)::value;
        float f[Q];
        rphi[p] = (float)pull_site_h<L, StoreF32, WALLS>(src, G, ring, rows[p], Codec{}, f);
    });
    if (has_ring) {
        static_for<0, NP>([&](auto P) { sphi[decltype(P)::value][rhx] = rphi[decltype(P)::value]; });
    }
    lds_barrier();
    if (!active) return;
    static_for<1, NB + 1>([&](auto P) {
        constexpr int p = decltype(P)::value;
        if (z0 - 1 + p >= zend) return;
        const ZRow& r = rows[p];
        float pn[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            pn[i] = sphi[p + L::cz(i)][tx + 1 + L::cx(i)];
        });
        const Macro a = macros<L>(m, pn, gv[p - 1]);
        SiteWriter32<L, WALLS> out{dst, own.base + r.base, G.S};
        collide_stream<L>(m, a, lo[p - 1], hv[p - 1], gv[p - 1], out);
    });
}

// ---------------------------------------------------------------------------
// equilibrium start and hand-over.  Each kernel body is a per-site function, called by
// a single-context kernel (parameters by value) and by a batched kernel whose
// blockIdx.y picks one context of a Batch (same lattice, storage and geometry).
// ---------------------------------------------------------------------------

// 1 / rho' with rho' = rho + beta rho_dif lap(phi) / 4: the density read-out divides the
// momentum by, so a hand-over of macroscopic fields takes u = J / rho'
template <class L>
__device__ __forceinline__ float inv_rho_prime(const Model& m, const float (&pn)[L::Q]) {
    float ls = 0.f;
    static_for<1, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (i & 1) ls = fmaf(L::w(i), (pn[i] - pn[0]) + (pn[i + 1] - pn[0]), ls);
    });
    const float rho = fmaf(pn[0], m.rho_dif, m.rho_L);
    return 1.0f / fmaf(m.beta * 0.25f * m.rho_dif, 6.0f * ls, rho);
}

// pre-collision equilibria of site s from phi, P (NULL: 0) and the velocity, given as
// u or (u == NULL) as the momentum J; direction i of h and g at i * hs + s
template <class L>
__device__ __forceinline__ void equilibrium_site(const Geom& G, const Model& m, uint32_t N,
                                                 uint32_t s, const float* __restrict__ phi,
                                                 const float* __restrict__ u,
                                                 const float* __restrict__ J,
                                                 const float* __restrict__ P,
                                                 float* __restrict__ h, float* __restrict__ g,
                                                 size_t hs) {
    int x, y, z;
    site_coords(G, s, x, y, z);
    float pn[L::Q];
    phi_stencil<L>(G, m, phi, x, y, z, pn);
    // macros with the given u and P: feed a zero g and overwrite J/u/P
    float zero[L::Q];
    static_for<0, L::Q>([&](auto I) { zero[decltype(I)::value] = 0.0f; });
    Macro a = macros<L>(m, pn, g_moments<L>(zero));
    float uu[3] = {0.f, 0.f, 0.f};
    if (u) {
        for (int c = 0; c < L::D; ++c) uu[user_axis<L>(c)] = u[(size_t)c * N + s];
    } else {
        const float irp = inv_rho_prime<L>(m, pn);
        for (int c = 0; c < L::D; ++c) uu[user_axis<L>(c)] = J[(size_t)c * N + s] * irp;
    }
    a.ux = uu[0]; a.uy = uu[1]; a.uz = uu[2];
    a.P = P ? P[s] : 0.0f;
    const EqTerms t = eq_terms(m, a);
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        float hdev, geq, K;
        eq_dir<L, i>(a, t, hdev, geq, K);
        if constexpr (i == 0) hdev = fmaf(a.phi, kappa<L>(), hdev);
        h[(size_t)i * hs + s] = fmaf(a.phi, L::w(i), hdev);
        g[(size_t)i * hs + s] = geq;
    });
}

template <class L>
__global__ void __launch_bounds__(256)
k_equilibrium(Geom G, Model m, uint32_t N, const float* __restrict__ phi,
              const float* __restrict__ u, const float* __restrict__ P,
              float* __restrict__ h, float* __restrict__ g, size_t hs) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    equilibrium_site<L>(G, m, N, s, phi, u, nullptr, P, h, g, hs);
}

// hand-over: equilibria from (phi, P, J) of context blockIdx.y into its work (h, then g)
template <class L>
__global__ void __launch_bounds__(256) k_equilibrium_j_b(Geom G, uint32_t N, Batch bt) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    const BatchEnt& e = bt.e[blockIdx.y];
    equilibrium_site<L>(G, e.m, N, s, e.phi, nullptr, e.J, e.P, e.work,
                        e.work + (size_t)L::Q * N, N);
}

// ---------------------------------------------------------------------------
// pre-collision distributions <-> pull storage
// slot (y, j) is gathered by x = y + c_j as population j when x is a fluid site,
// otherwise by y itself as population opp(j)
// ---------------------------------------------------------------------------
template <class L, class ST>
__device__ __forceinline__ void set_state_site(const Geom& G, const Codec& cd, uint32_t N,
                                               uint32_t s, const float* __restrict__ h,
                                               const float* __restrict__ g,
                                               char* __restrict__ b) {
    int x, y, z;
    site_coords(G, s, x, y, z);
    if constexpr (!ST::HALF) {
        float fh[L::Q], fg[L::Q];
        static_for<0, L::Q>([&](auto I) {
            constexpr int j = decltype(I)::value;
            const int xx = x + L::cx(j), yy = y + L::cy(j), zz = z + L::cz(j);
            const bool solid = (G.wx && (xx < 0 || xx >= G.nx)) ||
                               (G.wy && (yy < 0 || yy >= G.ny)) ||
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
        encode_site_f32<L>(b, s, G.S, fh, fg);
    } else {
        // FP16S, second pass: each moving slot (s, j) as the deviation from the reference
        // of its reader, whose moments word the first pass wrote
        const uint4* mw = reinterpret_cast<const uint4*>(b + StoreF16S::mom_off(G.S));
        static_for<1, L::Q>([&](auto I) {
            constexpr int j = decltype(I)::value;
            const int xx = x + L::cx(j), yy = y + L::cy(j), zz = z + L::cz(j);
            const bool solid = (G.wx && (xx < 0 || xx >= G.nx)) ||
                               (G.wy && (yy < 0 || yy >= G.ny)) ||
                               (G.wz && (zz < 0 || zz >= G.nz));
            uint32_t t;
            float vh, vg, rh, rg;
            if (solid) {            // read back by s itself as population opp(j)
                t = s;
                vh = h[(size_t)opp(j) * N + s];
                vg = g[(size_t)opp(j) * N + s];
                ref_of<L, opp(j)>(unpack_mom(mw[t]), rh, rg);
            } else {
                t = site_of(G, map_coord(xx, G.nx, 0), map_coord(yy, G.ny, 0),
                            map_coord(zz, G.nz, 0));
                vh = h[(size_t)j * N + t];
                vg = g[(size_t)j * N + t];
                ref_of<L, j>(unpack_mom(mw[t]), rh, rg);
            }
            reinterpret_cast<__half2*>(b + StoreF16S::dev_off(G.S))[(size_t)(j - 1) * G.S + s] =
                __halves2half2(__float2half_rn((vh - rh) * cd.sh), __float2half_rn((vg - rg) * cd.sg));
        });
    }
}

// FP16S, first pass of a state upload: the rest populations and the moments word of
// site s from its pre-collision populations (the same sums a gathered site forms)
template <class L>
__device__ __forceinline__ void set_mom_site(const Geom& G, uint32_t N, uint32_t s,
                                             const float* __restrict__ h,
                                             const float* __restrict__ g,
                                             char* __restrict__ b) {
    MomAcc acc;
    float Sg = 0.f, Jx = 0.f, Jy = 0.f, Jz = 0.f;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const float hv = h[(size_t)i * N + s], gv = g[(size_t)i * N + s];
        if constexpr (i > 0) acc.template add_h<L, i>(hv);
        Sg += gv;
        if constexpr (L::cx(i) > 0) Jx += gv;
        if constexpr (L::cx(i) < 0) Jx -= gv;
        if constexpr (L::cy(i) > 0) Jy += gv;
        if constexpr (L::cy(i) < 0) Jy -= gv;
        if constexpr (L::cz(i) > 0) Jz += gv;
        if constexpr (L::cz(i) < 0) Jz -= gv;
    });
    const float h0 = h[s];
    reinterpret_cast<float2*>(b)[s] = make_float2(h0, g[s]);
    reinterpret_cast<uint4*>(b + StoreF16S::mom_off(G.S))[s] =
        pack_mom(h0 + acc.S, Sg, acc.jx, acc.jy, acc.jz, Jx, Jy, Jz);
}

template <class L>
__global__ void __launch_bounds__(256)
k_set_mom(Geom G, uint32_t N, const float* __restrict__ h, const float* __restrict__ g,
          char* __restrict__ b) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    set_mom_site<L>(G, N, s, h, g, b);
}

template <class L>
__global__ void __launch_bounds__(256) k_set_mom_b(Geom G, uint32_t N, Batch bt) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    const BatchEnt& e = bt.e[blockIdx.y];
    set_mom_site<L>(G, N, s, e.work, e.work + (size_t)L::Q * N, e.state);
}

template <class L, class ST>
__global__ void __launch_bounds__(256)
k_set_state(Geom G, Codec cd, uint32_t N, const float* __restrict__ h,
            const float* __restrict__ g, char* __restrict__ b) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    set_state_site<L, ST>(G, cd, N, s, h, g, b);
}

// hand-over: the work equilibria of context blockIdx.y into its state buffer
template <class L, class ST>
__global__ void __launch_bounds__(256) k_set_state_b(Geom G, uint32_t N, Batch bt) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    const BatchEnt& e = bt.e[blockIdx.y];
    set_state_site<L, ST>(G, e.cd, N, s, e.work, e.work + (size_t)L::Q * N, e.state);
}

template <class L, class ST, int WALLS>
__global__ void __launch_bounds__(256)
k_get_state(Geom G, Codec cd, uint32_t N, const char* __restrict__ b, float* __restrict__ h,
            float* __restrict__ g) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    int x, y, z;
    site_coords(G, s, x, y, z);
    float fh[L::Q], fg[L::Q];
    pull_site<L, ST, WALLS>(b, G, make_col(G, x, y), make_zrow(G, z), cd, fh, fg);
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        h[(size_t)i * N + s] = fh[i];
        g[(size_t)i * N + s] = fg[i];
    });
}

// ---------------------------------------------------------------------------
// read-out
// ---------------------------------------------------------------------------
template <class L, class ST, int WALLS>
__device__ __forceinline__ void phi_site(const Geom& G, const Codec& cd, uint32_t s,
                                         const char* __restrict__ b, float* __restrict__ phi) {
    int x, y, z;
    site_coords(G, s, x, y, z);
    float f[L::Q];
    phi[s] = (float)pull_site_h<L, ST, WALLS>(b, G, make_col(G, x, y), make_zrow(G, z), cd, f);
}

// P, J and u of site s (each output may be NULL) from the state and the phi field
template <class L, class ST, int WALLS>
__device__ __forceinline__ void macro_site(const Geom& G, const Model& m, const Codec& cd,
                                           uint32_t N, uint32_t s, const char* __restrict__ b,
                                           const float* __restrict__ phi, float* __restrict__ P,
                                           float* __restrict__ J, float* __restrict__ U) {
    int x, y, z;
    site_coords(G, s, x, y, z);
    float pn[L::Q], hv[L::Q], gv[L::Q];
    phi_stencil<L>(G, m, phi, x, y, z, pn);
    pull_site<L, ST, WALLS>(b, G, make_col(G, x, y), make_zrow(G, z), cd, hv, gv);
    const Macro a = macros<L>(m, pn, g_moments<L>(gv));
    if (P) P[s] = a.P;
    const float jv[3] = {a.jx, a.jy, a.jz};
    const float uv[3] = {a.ux, a.uy, a.uz};
    for (int c = 0; c < L::D; ++c) {
        if (J) J[(size_t)c * N + s] = jv[user_axis<L>(c)];
        if (U) U[(size_t)c * N + s] = uv[user_axis<L>(c)];
    }
}

template <class L, class ST, int WALLS>
__global__ void __launch_bounds__(256)
k_phi(Geom G, Codec cd, uint32_t N, const char* __restrict__ b, float* __restrict__ phi) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    phi_site<L, ST, WALLS>(G, cd, s, b, phi);
}

template <class L, class ST, int WALLS>
__global__ void __launch_bounds__(256)
k_macro(Geom G, Model m, Codec cd, uint32_t N, const char* __restrict__ b,
        const float* __restrict__ phi, float* __restrict__ P, float* __restrict__ J,
        float* __restrict__ U) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    macro_site<L, ST, WALLS>(G, m, cd, N, s, b, phi, P, J, U);
}

template <class L, class ST, int WALLS>
__global__ void __launch_bounds__(256) k_phi_b(Geom G, uint32_t N, Batch bt) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    const BatchEnt& e = bt.e[blockIdx.y];
    phi_site<L, ST, WALLS>(G, e.cd, s, e.state, e.phi);
}

template <class L, class ST, int WALLS>
__global__ void __launch_bounds__(256) k_macro_b(Geom G, uint32_t N, Batch bt) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= N) return;
    const BatchEnt& e = bt.e[blockIdx.y];
    macro_site<L, ST, WALLS>(G, e.m, e.cd, N, s, e.state, e.phi, e.P, e.J, nullptr);
}

// ---------------------------------------------------------------------------
// sum of phi: every slot is gathered exactly once per step, so sum_x phi(x) is the
// sum of all decoded h slots.  Per site in float64, per block by a fixed tree, then
// one block over the partial sums: the result does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int MASS_BLOCKS = 1024;
constexpr int MASS_THREADS = 256;

template <class L, class ST, int WALLS>
__device__ __forceinline__ double slot_sum(const Geom& G, const char* b, uint32_t s,
                                           const Codec& cd, bool& bad) {
    double acc = 0.0;
    if constexpr (ST::INPLACE) {
        // in-place layouts: every slot is read exactly once by the next step as well
        const float* f = reinterpret_cast<const float*>(b);
        static_for<0, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const float hv = f[(size_t)i * G.S + s], gv = f[(size_t)(L::Q + i) * G.S + s];
            bad |= !isfinite(hv) || !isfinite(gv);
            acc += (double)hv;
        });
    } else if constexpr (!ST::HALF) {
        // FP32: the slots of site s in storage order (each slot is gathered once)
        static_for<0, L::Q>([&](auto I) {
            const float2 v =
                reinterpret_cast<const float2*>(b)[(size_t)decltype(I)::value * G.S + s];
            bad |= !isfinite(v.x) || !isfinite(v.y);
            acc += (double)v.x;
        });
    } else {
        // FP16S: a slot decodes with its reader's reference, so the sum follows the
        // gather: phi of site s as the step forms it
        int x, y, z;
        site_coords(G, s, x, y, z);
        MomAcc ma;
        const float phi = gather16<L, WALLS>(b, G, make_col(G, x, y), make_zrow(G, z), cd, ma,
                                             [&](auto, float hv, float gv, float) {
                                                 bad |= !isfinite(hv) || !isfinite(gv);
                                             });
        bad |= !isfinite(phi);
        acc = (double)phi;
    }
    return acc;
}

template <class L, class ST, int WALLS>
__global__ void __launch_bounds__(MASS_THREADS)
k_mass_partial(Geom G, Codec cd, uint32_t N, const char* __restrict__ b,
               double* __restrict__ part, int* __restrict__ flag) {
    __shared__ double sd[MASS_THREADS];
    __shared__ int sb[MASS_THREADS];
    double acc = 0.0;
    bool bad = false;
    for (uint32_t s = blockIdx.x * MASS_THREADS + threadIdx.x; s < N;
         s += MASS_BLOCKS * MASS_THREADS)
        acc += slot_sum<L, ST, WALLS>(G, b, s, cd, bad);
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
// open (pressure) faces, after a step has written dst.  A population i that enters
// site x through an open face comes from the boundary-layer site s' = x - c_i with its
// out-of-range coordinates put back into the layer, as its post-collision value there,
// and for g plus 2 w_i (P_f - P(s'))/T: the ghost beyond the face copies the layer (zero
// normal gradient of phi and u) with the pressure taken linearly to P_f at the face
// (P(s') from k_open_P; P_f the mean over the open faces crossed at an edge or corner).
// The step stored that value's source slot (s', i), read by the site s' + c_i (inside:
// on every axis the source crossed, s' sits on the boundary and c_i points inwards),
// and treated the faces as walls: x reads the incoming value as the bounce-back of i,
// from its own slot (x, opp(i)), which this kernel overwrites.  A population whose
// source also crosses a closed face keeps its bounce-back.  The kernel reads slots that
// move into the domain and writes slots that leave it through open faces, so no slot is
// both read and written; every slot is still read exactly once by the next step.  A
// population entering through several open faces is written by the first of them.
// One thread per site of a face, blockIdx.y = face (x-, x+, y-, y+, z-, z+).
// ---------------------------------------------------------------------------

// coordinates of site t of face f's layer (the two other axes in increasing order, the
// lower one fastest) and back
__device__ __forceinline__ bool face_site(const Geom& G, int f, uint32_t t, int (&v)[3]) {
    const int n[3] = {G.nx, G.ny, G.nz};
    const int a = f >> 1, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    if (t >= (uint32_t)n[b] * (uint32_t)n[c]) return false;
    v[b] = (int)(t % (uint32_t)n[b]);
    v[c] = (int)(t / (uint32_t)n[b]);
    v[a] = (f & 1) ? n[a] - 1 : 0;
    return true;
}

__device__ __forceinline__ size_t face_index(const Geom& G, int f, const int (&v)[3]) {
    const int n[3] = {G.nx, G.ny, G.nz};
    const int a = f >> 1, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    return (size_t)v[c] * (size_t)n[b] + (size_t)v[b];
}

template <class L, class ST>
__device__ __forceinline__ void open_site(const Geom& G, const Model& m, const Codec& cd,
                                          char* __restrict__ b, const int (&v)[3], int f) {
    const int n[3] = {G.nx, G.ny, G.nz};
    const int w[3] = {G.wx, G.wy, G.wz};
    const int a = f >> 1;
    const int inward = (f & 1) ? -1 : 1;        // c_i[a] of the populations entering
    const size_t S = G.S;
    const size_t xs = site_of(G, v[0], v[1], v[2]);
    const float* Pside = reinterpret_cast<const float*>(b + G.side_off) + (size_t)f * G.SL;
    MomF mx{};
    if constexpr (ST::HALF)
        mx = unpack_mom(reinterpret_cast<const uint4*>(b + StoreF16S::mom_off(G.S))[xs]);
    static_for<1, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int c[3] = {L::cx(i), L::cy(i), L::cz(i)};
        if (c[a] != inward) return;
        // s' = x - c_i, and the site d = s' + c_i that reads slot (s', i): x itself on
        // the axes the source stays inside or wraps across, one site inwards on those
        // it crosses an open face of
        int sp[3], d[3];
        bool closed = false, first = true;
        float Psum = 0.0f;
        int nopen = 0;
        for (int e = 0; e < 3; ++e) {
            sp[e] = v[e] - c[e];
            d[e] = v[e];
            if (sp[e] >= 0 && sp[e] < n[e]) continue;
            if (!w[e]) {                             // periodic: wrap
                sp[e] = sp[e] < 0 ? sp[e] + n[e] : sp[e] - n[e];
                continue;
            }
            const int g = 2 * e + (sp[e] < 0 ? 0 : 1);   // the wall face crossed
            if (!(G.open & (1u << g))) {
                closed = true;
                continue;
            }
            if (g < f) first = false;
            Psum += m.Pf[g];
            ++nopen;
            sp[e] = v[e];                            // back into the layer
            d[e] = v[e] + c[e];
        }
        if (closed || !first) return;
        const float Pf = nopen > 1 ? Psum / (float)nopen : Psum;
        const size_t spi = site_of(G, sp[0], sp[1], sp[2]);
        const float shift = 6.0f * L::w(i) * (Pf - Pside[face_index(G, f, sp)]);
        if constexpr (!ST::HALF) {
            float2 val = reinterpret_cast<const float2*>(b)[(size_t)i * S + spi];
            val.y += shift;
            reinterpret_cast<float2*>(b)[(size_t)opp(i) * S + xs] = val;
        } else {
            // decode with the reference of the slot's reader s' + c_i, encode with the
            // one x applies to its bounce-back of i
            const MomF md = unpack_mom(reinterpret_cast<const uint4*>(
                b + StoreF16S::mom_off(G.S))[site_of(G, d[0], d[1], d[2])]);
            char* dev = b + StoreF16S::dev_off(G.S);
            const float2 q = __half22float2(
                reinterpret_cast<const __half2*>(dev + (size_t)(i - 1) * S * 4)[spi]);
            float rh, rg;
            ref_of<L, i>(md, rh, rg);
            const float hv = fmaf(q.x, cd.ish, rh);
            const float gv = fmaf(q.y, cd.isg, rg) + shift;
            ref_of<L, i>(mx, rh, rg);
            reinterpret_cast<__half2*>(dev + (size_t)(opp(i) - 1) * S * 4)[xs] =
                __halves2half2(__float2half_rn((hv - rh) * cd.sh),
                               __float2half_rn((gv - rg) * cd.sg));
        }
    });
}

// Pressure of the boundary-layer sites of the open faces at the step just taken, from
// the zeroth moments of g before (gathered from src) and after (the slots dst holds) the
// collision: Eq. 6 gives sum g^eq = P/T - sum K/2, the filtered part has no zeroth
// moment, so sum g* = P/T + sum K/2; with P = T sum g + T rho_dif u.grad(phi)/2 and
// sum K = rho_dif u.grad(phi) (Eq. 7; Gamma has moments 1 and u) the two sums average
// to P/T.  One thread per site of a face, blockIdx.y = face.
template <class L, class ST, int WALLS>
__global__ void __launch_bounds__(256) k_open_P(Geom G, Codec cd, const char* __restrict__ src,
                                                char* __restrict__ dst) {
    const int f = blockIdx.y;
    if (!(G.open & (1u << f))) return;
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    int v[3];
    if (!face_site(G, f, t, v)) return;
    const int x = v[0], y = v[1], z = v[2];
    const Col c = make_col(G, x, y);
    const ZRow r = make_zrow(G, z);
    float h[L::Q], g[L::Q];
    pull_site<L, ST, WALLS>(src, G, c, r, cd, h, g);
    double pre = 0.0, post = 0.0;
    static_for<0, L::Q>([&](auto I) { pre += (double)g[decltype(I)::value]; });
    const size_t S = G.S;
    const size_t s = site_of(G, x, y, z);
    if constexpr (!ST::HALF) {
        static_for<0, L::Q>([&](auto I) {
            post += (double)reinterpret_cast<const float2*>(dst)[(size_t)decltype(I)::value * S + s].y;
        });
    } else {
        // each slot decodes with its reader's reference: the site c_I away, or the site
        // itself (reference of opp(I)) where c_I leaves through a wall
        const uint4* mom = reinterpret_cast<const uint4*>(dst + StoreF16S::mom_off(G.S));
        const MomF own = unpack_mom(mom[s]);
        post = (double)reinterpret_cast<const float2*>(dst)[s].y;
        const uint32_t solid = c.solid | r.solid;
        static_for<1, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const float2 q = __half22float2(reinterpret_cast<const __half2*>(
                dst + StoreF16S::dev_off(G.S) + (size_t)(i - 1) * S * 4)[s]);
            float rh, rg;
            if (dest_beyond<L, i, WALLS>(solid)) {
                ref_of<L, opp(i)>(own, rh, rg);
            } else {
                int dx = x + L::cx(i), dy = y + L::cy(i), dz = z + L::cz(i);
                dx = dx < 0 ? dx + G.nx : (dx >= G.nx ? dx - G.nx : dx);
                dy = dy < 0 ? dy + G.ny : (dy >= G.ny ? dy - G.ny : dy);
                dz = dz < 0 ? dz + G.nz : (dz >= G.nz ? dz - G.nz : dz);
                ref_of<L, i>(unpack_mom(mom[site_of(G, dx, dy, dz)]), rh, rg);
            }
            post += (double)fmaf(q.y, cd.isg, rg);
        });
    }
    reinterpret_cast<float*>(dst + G.side_off)[(size_t)f * G.SL + t] =
        (float)((pre + post) * (1.0 / 6.0));
}

template <class L, class ST>
__global__ void __launch_bounds__(256) k_open(Geom G, Model m, Codec cd, char* __restrict__ b) {
    const int f = blockIdx.y;
    if (!(G.open & (1u << f))) return;
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    int v[3];
    if (!face_site(G, f, t, v)) return;
    open_site<L, ST>(G, m, cd, b, v, f);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static inline dim3 grid1(uint32_t N) { return dim3((N + 255u) / 256u); }

// One step of one context (bt == nullptr: buffers s -> d, parameters a.m, a.cd) or of
// the n contexts of a batch (blockIdx.y = context).
struct StepArgs {
    const char* s;
    char* d;
    const StepBatch* bt;
    int n;
};

template <class L, class ST, int WALLS, int TX, int TY, bool XBC = false>
static hipError_t launch_tile(const Launch& a, const StepArgs& x) {
    const int ntx = (a.G.nx + TX - 1) / TX;
    const int nty = (a.G.ny + TY - 1) / TY;
    const int ntz = (a.G.nz + a.bz - 1) / a.bz;
    const int nblk = ntx * nty * ntz;
    if (x.bt) {
        // batches hold contexts without moving walls or contact angles only (the
        // others are stepped one by one)
        if constexpr (XBC) {
            return hipErrorInvalidValue;
        } else {
            StepTable<true> tab;
            tab.bt = *x.bt;
            hipLaunchKernelGGL((k_step<L, ST, TX, TY, WALLS, false, true>), dim3(nblk, x.n),
                               dim3(TX * TY), 0, a.stream, a.G, a.m, a.cd, a.bz, ntx, nty,
                               nblk, (const char*)nullptr, (char*)nullptr, tab);
        }
    } else {
        hipLaunchKernelGGL((k_step<L, ST, TX, TY, WALLS, XBC, false>), dim3(nblk),
                           dim3(TX * TY), 0, a.stream, a.G, a.m, a.cd, a.bz, ntx, nty, nblk,
                           x.s, x.d, StepTable<false>{});
    }
    return hipGetLastError();
}

// D2Q9 FP32 chunks of NB rows (no contact angles or moving walls, 32-bit addressing)
template <class L, int WALLS, int NB>
static hipError_t launch_rows(const Launch& a, const StepArgs& x) {
    const int ntx = (a.G.nx + 63) / 64;
    const int nblk = ntx * ((a.G.nz + NB - 1) / NB);
    if (x.bt) {
        StepTable<true> tab;
        tab.bt = *x.bt;
        hipLaunchKernelGGL((k_step_rows<L, WALLS, true, NB>), dim3(nblk, x.n), dim3(64), 0,
                           a.stream, a.G, a.m, ntx, nblk, (const char*)nullptr, (char*)nullptr,
                           tab);
    } else {
        hipLaunchKernelGGL((k_step_rows<L, WALLS, false, NB>), dim3(nblk), dim3(64), 0,
                           a.stream, a.G, a.m, ntx, nblk, x.s, x.d, StepTable<false>{});
    }
    return hipGetLastError();
}

template <class L, class ST, int WALLS>
static hipError_t launch_step_t(const Launch& a, const StepArgs& x) {
    if constexpr ((WALLS & WALLS_XYZ) != WALLS_NONE) {
        // moving walls or contact angles: one tile shape per lattice
        if (a.m.moving || a.m.wetting) {
            if constexpr (L::USES_Y) return launch_tile<L, ST, WALLS, 64, 4, true>(a, x);
            else return launch_tile<L, ST, WALLS, 64, 1, true>(a, x);
        }
    }
    if constexpr ((WALLS & ADDR64) != 0) {
        // domains beyond 2^28 sites: the default tile only, stepped one context at a time
        if (x.bt) return hipErrorInvalidValue;
        if constexpr (L::USES_Y) return launch_tile<L, ST, WALLS, 64, 4>(a, x);
        else return launch_tile<L, ST, WALLS, 64, 1>(a, x);
    } else if constexpr (L::USES_Y) {
        switch (a.tile) {
            case 1: return launch_tile<L, ST, WALLS, 64, 8>(a, x);
            case 2: return launch_tile<L, ST, WALLS, 32, 8>(a, x);
            case 3: return launch_tile<L, ST, WALLS, 32, 4>(a, x);
            default: return launch_tile<L, ST, WALLS, 64, 4>(a, x);
        }
    } else {
        if constexpr (!ST::HALF) {
            if (a.bz == 1) return launch_rows<L, WALLS, 1>(a, x);
            if (a.bz == 2) return launch_rows<L, WALLS, 2>(a, x);
        }
        return launch_tile<L, ST, WALLS, 64, 1>(a, x);
    }
}

static inline int wallset(const Geom& G) {
    return ((G.wx || G.wy) ? WALLS_XY : 0) | (G.wz ? WALLS_Z : 0);
}

template <class L, class ST>
static hipError_t dispatch_walls(const Launch& a, const StepArgs& x) {
    if (a.wide) {
        switch (wallset(a.G)) {
            case WALLS_XYZ: return launch_step_t<L, ST, WALLS_XYZ | ADDR64>(a, x);
            case WALLS_XY: return launch_step_t<L, ST, WALLS_XY | ADDR64>(a, x);
            case WALLS_Z: return launch_step_t<L, ST, WALLS_Z | ADDR64>(a, x);
            default: return launch_step_t<L, ST, WALLS_NONE | ADDR64>(a, x);
        }
    }
    switch (wallset(a.G)) {
        case WALLS_XYZ: return launch_step_t<L, ST, WALLS_XYZ>(a, x);
        case WALLS_XY: return launch_step_t<L, ST, WALLS_XY>(a, x);
        case WALLS_Z: return launch_step_t<L, ST, WALLS_Z>(a, x);
        default: return launch_step_t<L, ST, WALLS_NONE>(a, x);
    }
}

static hipError_t dispatch_step(const Launch& a, const StepArgs& x) {
    if (a.q == 19) {
        if (a.half) return dispatch_walls<LatD3Q19, StoreF16S>(a, x);
        return dispatch_walls<LatD3Q19, StoreF32>(a, x);
    }
    if (a.half) return dispatch_walls<LatD2Q9, StoreF16S>(a, x);
    return dispatch_walls<LatD2Q9, StoreF32>(a, x);
}

// open faces, after a step src -> dst: the boundary layers' pressures, then the
// populations entering through the faces
template <class L, class ST>
static hipError_t open_t(const Launch& a, const void* src, void* dst) {
    const dim3 grid((a.G.SL + 255u) / 256u, 6);
    const char* s = static_cast<const char*>(src);
    char* d = static_cast<char*>(dst);
    if (a.wide)
        hipLaunchKernelGGL((k_open_P<L, ST, WALLS_XYZ | ADDR64>), grid, dim3(256), 0, a.stream,
                           a.G, a.cd, s, d);
    else
        hipLaunchKernelGGL((k_open_P<L, ST, WALLS_XYZ>), grid, dim3(256), 0, a.stream, a.G, a.cd,
                           s, d);
    hipLaunchKernelGGL((k_open<L, ST>), grid, dim3(256), 0, a.stream, a.G, a.m, a.cd, d);
    return hipGetLastError();
}

hipError_t launch_step(const Launch& a, const void* src, void* dst) {
    const hipError_t e = dispatch_step(
        a, StepArgs{static_cast<const char*>(src), static_cast<char*>(dst), nullptr, 0});
    if (e != hipSuccess || !a.G.open) return e;
    if (a.q == 19)
        return a.half ? open_t<LatD3Q19, StoreF16S>(a, src, dst)
                      : open_t<LatD3Q19, StoreF32>(a, src, dst);
    return a.half ? open_t<LatD2Q9, StoreF16S>(a, src, dst) : open_t<LatD2Q9, StoreF32>(a, src, dst);
}

hipError_t launch_step_batch(const Launch& a, const StepBatch& bt, int n) {
    if (n < 1 || n > BATCH_MAX) return hipErrorInvalidValue;
    return dispatch_step(a, StepArgs{nullptr, nullptr, &bt, n});
}

template <class L>
static hipError_t equilibrium_t(const Launch& a, uint32_t N, const float* phi, const float* u,
                                const float* P, float* h, float* g, size_t hs) {
    hipLaunchKernelGGL((k_equilibrium<L>), grid1(N), dim3(256), 0, a.stream, a.G, a.m, N, phi,
                       u, P, h, g, hs);
    return hipGetLastError();
}

hipError_t launch_equilibrium(const Launch& a, uint32_t N, const float* phi, const float* u,
                              const float* P, float* h, float* g, size_t hs) {
    if (hs == 0) hs = N;
    return a.q == 19 ? equilibrium_t<LatD3Q19>(a, N, phi, u, P, h, g, hs)
                     : equilibrium_t<LatD2Q9>(a, N, phi, u, P, h, g, hs);
}

template <class L, class ST>
static hipError_t reconstruct_batch_t(const Launch& a, uint32_t N, const Batch& bt, int n) {
    const dim3 grid((N + 255u) / 256u, n);
    hipLaunchKernelGGL((k_equilibrium_j_b<L>), grid, dim3(256), 0, a.stream, a.G, N, bt);
    if constexpr (ST::HALF)
        hipLaunchKernelGGL((k_set_mom_b<L>), grid, dim3(256), 0, a.stream, a.G, N, bt);
    hipLaunchKernelGGL((k_set_state_b<L, ST>), grid, dim3(256), 0, a.stream, a.G, N, bt);
    return hipGetLastError();
}

hipError_t launch_reconstruct_batch(const Launch& a, uint32_t N, const Batch& bt, int n) {
    if (n < 1 || n > BATCH_MAX) return hipErrorInvalidValue;
    if (a.q == 19)
        return a.half ? reconstruct_batch_t<LatD3Q19, StoreF16S>(a, N, bt, n)
                      : reconstruct_batch_t<LatD3Q19, StoreF32>(a, N, bt, n);
    return a.half ? reconstruct_batch_t<LatD2Q9, StoreF16S>(a, N, bt, n)
                  : reconstruct_batch_t<LatD2Q9, StoreF32>(a, N, bt, n);
}

template <class L, class ST>
static hipError_t set_state_t(const Launch& a, uint32_t N, const float* h, const float* g,
                              void* b) {
    if constexpr (ST::HALF)
        hipLaunchKernelGGL((k_set_mom<L>), grid1(N), dim3(256), 0, a.stream, a.G, N, h, g,
                           static_cast<char*>(b));
    hipLaunchKernelGGL((k_set_state<L, ST>), grid1(N), dim3(256), 0, a.stream, a.G, a.cd, N, h,
                       g, static_cast<char*>(b));
    return hipGetLastError();
}

hipError_t launch_set_state(const Launch& a, uint32_t N, const float* h, const float* g,
                            void* b) {
    if (a.q == 19)
        return a.half ? set_state_t<LatD3Q19, StoreF16S>(a, N, h, g, b)
                      : set_state_t<LatD3Q19, StoreF32>(a, N, h, g, b);
    return a.half ? set_state_t<LatD2Q9, StoreF16S>(a, N, h, g, b)
                  : set_state_t<LatD2Q9, StoreF32>(a, N, h, g, b);
}

template <class L, class ST, int WALLS>
static hipError_t get_state_t(const Launch& a, uint32_t N, const void* b, float* h, float* g) {
    hipLaunchKernelGGL((k_get_state<L, ST, WALLS>), grid1(N), dim3(256), 0, a.stream, a.G, a.cd,
                       N, static_cast<const char*>(b), h, g);
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t get_state_w(const Launch& a, uint32_t N, const void* b, float* h, float* g) {
    if (a.wide)
        return wallset(a.G) ? get_state_t<L, ST, WALLS_XYZ | ADDR64>(a, N, b, h, g)
                            : get_state_t<L, ST, WALLS_NONE | ADDR64>(a, N, b, h, g);
    if (wallset(a.G)) return get_state_t<L, ST, WALLS_XYZ>(a, N, b, h, g);
    return get_state_t<L, ST, WALLS_NONE>(a, N, b, h, g);
}

hipError_t launch_get_state(const Launch& a, uint32_t N, const void* b, float* h, float* g) {
    if (a.q == 19)
        return a.half ? get_state_w<LatD3Q19, StoreF16S>(a, N, b, h, g)
                      : get_state_w<LatD3Q19, StoreF32>(a, N, b, h, g);
    return a.half ? get_state_w<LatD2Q9, StoreF16S>(a, N, b, h, g)
                  : get_state_w<LatD2Q9, StoreF32>(a, N, b, h, g);
}

template <class L, class ST, int WALLS>
static hipError_t read_t(const Launch& a, uint32_t N, const void* b, float* phi, float* P,
                         float* J, float* U) {
    hipLaunchKernelGGL((k_phi<L, ST, WALLS>), grid1(N), dim3(256), 0, a.stream, a.G, a.cd, N,
                       static_cast<const char*>(b), phi);
    if (P || J || U)
        hipLaunchKernelGGL((k_macro<L, ST, WALLS>), grid1(N), dim3(256), 0, a.stream, a.G, a.m,
                           a.cd, N, static_cast<const char*>(b), phi, P, J, U);
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t read_w(const Launch& a, uint32_t N, const void* b, float* phi, float* P,
                         float* J, float* U) {
    if (a.wide)
        return wallset(a.G) ? read_t<L, ST, WALLS_XYZ | ADDR64>(a, N, b, phi, P, J, U)
                            : read_t<L, ST, WALLS_NONE | ADDR64>(a, N, b, phi, P, J, U);
    if (wallset(a.G)) return read_t<L, ST, WALLS_XYZ>(a, N, b, phi, P, J, U);
    return read_t<L, ST, WALLS_NONE>(a, N, b, phi, P, J, U);
}

hipError_t launch_read(const Launch& a, uint32_t N, const void* b, float* phi, float* P,
                       float* J, float* U) {
    if (a.q == 19)
        return a.half ? read_w<LatD3Q19, StoreF16S>(a, N, b, phi, P, J, U)
                      : read_w<LatD3Q19, StoreF32>(a, N, b, phi, P, J, U);
    return a.half ? read_w<LatD2Q9, StoreF16S>(a, N, b, phi, P, J, U)
                  : read_w<LatD2Q9, StoreF32>(a, N, b, phi, P, J, U);
}

template <class L, class ST, int WALLS>
static hipError_t read_batch_t(const Launch& a, uint32_t N, const Batch& bt, int n, bool macro) {
    const dim3 grid((N + 255u) / 256u, n);
    hipLaunchKernelGGL((k_phi_b<L, ST, WALLS>), grid, dim3(256), 0, a.stream, a.G, N, bt);
    if (macro)
        hipLaunchKernelGGL((k_macro_b<L, ST, WALLS>), grid, dim3(256), 0, a.stream, a.G, N, bt);
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t read_batch_w(const Launch& a, uint32_t N, const Batch& bt, int n, bool macro) {
    if (a.wide) return hipErrorInvalidValue;    // batches hold small domains only
    if (wallset(a.G)) return read_batch_t<L, ST, WALLS_XYZ>(a, N, bt, n, macro);
    return read_batch_t<L, ST, WALLS_NONE>(a, N, bt, n, macro);
}

hipError_t launch_read_batch(const Launch& a, uint32_t N, const Batch& bt, int n, bool macro) {
    if (n < 1 || n > BATCH_MAX) return hipErrorInvalidValue;
    if (a.q == 19)
        return a.half ? read_batch_w<LatD3Q19, StoreF16S>(a, N, bt, n, macro)
                      : read_batch_w<LatD3Q19, StoreF32>(a, N, bt, n, macro);
    return a.half ? read_batch_w<LatD2Q9, StoreF16S>(a, N, bt, n, macro)
                  : read_batch_w<LatD2Q9, StoreF32>(a, N, bt, n, macro);
}

template <class L, class ST>
static hipError_t mass_t(const Launch& a, uint32_t N, const void* b, void* scratch) {
    double* part = static_cast<double*>(scratch);
    int* flag = reinterpret_cast<int*>(part + MASS_BLOCKS + 1);
    if (a.wide)
        hipLaunchKernelGGL((k_mass_partial<L, ST, WALLS_XYZ | ADDR64>), dim3(MASS_BLOCKS),
                           dim3(MASS_THREADS), 0, a.stream, a.G, a.cd, N,
                           static_cast<const char*>(b), part, flag);
    else if (wallset(a.G))
        hipLaunchKernelGGL((k_mass_partial<L, ST, WALLS_XYZ>), dim3(MASS_BLOCKS),
                           dim3(MASS_THREADS), 0, a.stream, a.G, a.cd, N,
                           static_cast<const char*>(b), part, flag);
    else
        hipLaunchKernelGGL((k_mass_partial<L, ST, WALLS_NONE>), dim3(MASS_BLOCKS),
                           dim3(MASS_THREADS), 0, a.stream, a.G, a.cd, N,
                           static_cast<const char*>(b), part, flag);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(MASS_BLOCKS), 0, a.stream, part, flag,
                       part + MASS_BLOCKS, flag + MASS_BLOCKS);
    return hipGetLastError();
}

hipError_t launch_mass(const Launch& a, uint32_t N, const void* b, void* scratch) {
    if (a.inplace)
        return a.q == 19 ? mass_t<LatD3Q19, StoreF32InPlace>(a, N, b, scratch)
                         : mass_t<LatD2Q9, StoreF32InPlace>(a, N, b, scratch);
    if (a.q == 19)
        return a.half ? mass_t<LatD3Q19, StoreF16S>(a, N, b, scratch)
                      : mass_t<LatD3Q19, StoreF32>(a, N, b, scratch);
    return a.half ? mass_t<LatD2Q9, StoreF16S>(a, N, b, scratch)
                  : mass_t<LatD2Q9, StoreF32>(a, N, b, scratch);
}

size_t mass_scratch_bytes() {
    return (MASS_BLOCKS + 1) * sizeof(double) + (MASS_BLOCKS + 1) * sizeof(int);
}

size_t mass_result_offset() { return MASS_BLOCKS * sizeof(double); }
size_t mass_flag_offset() {
    return (MASS_BLOCKS + 1) * sizeof(double) + MASS_BLOCKS * sizeof(int);
}

size_t state_bytes(int q, bool half, uint32_t S) {
    return half ? StoreF16S::bytes_per_site(q) * S : StoreF32::bytes_per_site(q) * S;
}

}  // namespace pflb
