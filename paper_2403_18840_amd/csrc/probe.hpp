// Throughput probes of the roofline denominators (FP32 FMA, hardware 2^x and reciprocal, HBM copy).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmc {

// kind 0: FP32 FMA, 1: 2^x, 2: reciprocal, each `blocks` x 256 lanes x iters x 16 x 8 operations, one value
// per lane to out; kind 3: copy n4 float4 from in to dst
hipError_t launch_probe(int kind, float* out, int blocks, int iters, const float* in, float* dst, int64_t n4,
                        hipStream_t st);

}  // namespace dmc
