// Host-side declarations shared by the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "pflb_device.hpp"

namespace pflb {

struct Launch {
    int q;              // 9 or 19
    bool half;          // FP16S storage
    int bz;             // planes per workgroup in the fused step
    int tile;           // D3Q19 tile shape: 0: 64x4, 1: 64x8, 2: 32x8, 3: 32x4
    bool wide;          // more than 2^28 - 64 sites: 64-bit slot addresses
    bool inplace;       // FP32 in-place storage: one state buffer, layout by step parity
    Geom G;
    Model m;
    Codec cd;
    hipStream_t stream;
};

hipError_t launch_step(const Launch& a, const void* src, void* dst);
// one step of n <= BATCH_MAX contexts without moving walls or contact angles
// (blockIdx.y = context)
hipError_t launch_step_batch(const Launch& a, const StepBatch& bt, int n);
// h, g: Q arrays of stride hs (0: N) each
hipError_t launch_equilibrium(const Launch& a, uint32_t N, const float* phi, const float* u,
                              const float* P, float* h, float* g, size_t hs = 0);
hipError_t launch_set_state(const Launch& a, uint32_t N, const float* h, const float* g,
                            void* b);
hipError_t launch_get_state(const Launch& a, uint32_t N, const void* b, float* h, float* g);
hipError_t launch_read(const Launch& a, uint32_t N, const void* b, float* phi, float* P,
                       float* J, float* U);
hipError_t launch_mass(const Launch& a, uint32_t N, const void* b, void* scratch);
size_t state_bytes(int q, bool half, uint32_t S);

// In-place storage (one state buffer).  Layout 0 holds f_i(x) in slot (x, i); layout 1
// holds it in slot (x - c_i, opp(i)), or in slot (x, i) where x - c_i lies beyond a wall.
// A step from layout L reads and writes the same slots of each site and leaves layout
// 1 - L; phi (N floats) is the phi field of the state, written by the step's first
// kernel and read by its second.
hipError_t launch_step_inplace(const Launch& a, void* b, int layout, float* phi);
hipError_t launch_set_state_inplace(const Launch& a, uint32_t N, const float* h, const float* g,
                                    void* b);
hipError_t launch_get_state_inplace(const Launch& a, uint32_t N, const void* b, int layout,
                                    float* h, float* g);
hipError_t launch_read_inplace(const Launch& a, uint32_t N, const void* b, int layout, float* phi,
                               float* P, float* J, float* U);

// Batched launches over contexts that share the lattice, the storage and the geometry
// (blockIdx.y = context); per-context pointers and constants go by value in the kernel
// arguments, at most BATCH_MAX contexts per launch.
hipError_t launch_read_batch(const Launch& a, uint32_t N, const Batch& bt, int n, bool macro);
hipError_t launch_reconstruct_batch(const Launch& a, uint32_t N, const Batch& bt, int n);

// shape of a context as the user gave it (nx, ny, nz, bc), for the surrogate hand-over
struct CtxInfo {
    int q, nx, ny, nz;
    int bc[3];
    uint32_t N;
    bool bound;
    double rho_L, rho_H;
    int hoc;
};
size_t mass_scratch_bytes();
size_t mass_result_offset();
size_t mass_flag_offset();

}  // namespace pflb

struct pflb_ctx;
int pflb_ctx_info(const ::pflb_ctx* c, pflb::CtxInfo* out);

// Read-out of n contexts that share lattice, storage, sizes and walls, one launch per
// BATCH_MAX of them: context k writes phi[k] and, where the arrays and entries are not
// NULL, P[k] and J[k] (layouts as pflb_read).  Errors are reported on c[0].
int pflb_read_many(::pflb_ctx* const* c, int n, float* const* phi, float* const* P,
                   float* const* J, hipStream_t st);
// Hand-over of n such contexts from (phi[k], P[k] (NULL: 0), J[k]) as pflb_reconstruct
// does for one; work holds 2 Q N floats for each of min(n, BATCH_MAX) contexts.  Each
// context keeps its step count, increased by advance.
int pflb_reconstruct_many(::pflb_ctx* const* c, int n, const float* const* phi,
                          const float* const* P, const float* const* J, float* work, int advance,
                          hipStream_t st);
