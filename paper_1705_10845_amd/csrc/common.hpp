// Shared helpers of the XL-BOMD HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace xl {

struct HipError : std::runtime_error {
    explicit HipError(const std::string &m) : std::runtime_error(m) {}
};
struct InvalidArg : std::runtime_error {
    explicit InvalidArg(const std::string &m) : std::runtime_error(m) {}
};
struct NoConv : std::runtime_error {
    explicit NoConv(const std::string &m) : std::runtime_error(m) {}
};
struct Diverged : std::runtime_error {
    explicit Diverged(const std::string &m) : std::runtime_error(m) {}
};
struct NoMem : std::runtime_error {
    explicit NoMem(const std::string &m) : std::runtime_error(m) {}
};
struct StateError : std::runtime_error {   // call not valid in the handle's state
    explicit StateError(const std::string &m) : std::runtime_error(m) {}
};

#define XL_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            throw ::xl::HipError(std::string(#call) + ": " +                  \
                                 hipGetErrorString(e_));                      \
    } while (0)

#define XL_LAUNCH_CHECK() XL_HIP(hipGetLastError())

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sum for blockDim.x a multiple of 64 (<= 1024).  All threads get
// the result.  `sh` must hold 16 doubles.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += sh[i];
    __syncthreads();
    return t;
}

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace xl
