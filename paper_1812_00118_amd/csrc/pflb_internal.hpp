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
    Geom G;
    Model m;
    Codec cd;
    hipStream_t stream;
};

hipError_t launch_step(const Launch& a, const void* hs, const void* gs, void* hd, void* gd);
hipError_t launch_equilibrium(const Launch& a, uint32_t N, const float* phi, const float* u,
                              const float* P, float* h, float* g);
hipError_t launch_set_state(const Launch& a, uint32_t N, const float* h, const float* g,
                            void* hb, void* gb);
hipError_t launch_get_state(const Launch& a, uint32_t N, const void* hb, const void* gb,
                            float* h, float* g);
hipError_t launch_read(const Launch& a, uint32_t N, const void* hb, const void* gb, float* phi,
                       float* P, float* J, float* U);
hipError_t launch_mass(const Launch& a, uint32_t N, const void* hb, const void* gb,
                       void* scratch);
size_t mass_scratch_bytes();
size_t mass_result_offset();
size_t mass_flag_offset();

}  // namespace pflb
