// Host stand-ins for the few HIP names used by the register-level op code, so
// the planner's lowered plans can be executed on the CPU in tests.  Test-only.
#pragma once
#include <cmath>
#include <cstdint>
#define __device__
#define __host__
#define __forceinline__ inline
#define __global__
struct float2 {
    float x, y;
};
struct float4 {
    float x, y, z, w;
};
inline double __shfl_xor(double v, int, int) { return v; }
inline void __syncthreads() {}
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
