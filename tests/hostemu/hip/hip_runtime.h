// Minimal host stand-in for <hip/hip_runtime.h>: lets the library's device
// collision headers compile as plain host C++ so that tests can run their
// arithmetic on the CPU.  Only what those headers use is defined.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
typedef int hipError_t;
typedef void* hipStream_t;
static inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
static inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
