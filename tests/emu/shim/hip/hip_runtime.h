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
#include <cstring>
inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
