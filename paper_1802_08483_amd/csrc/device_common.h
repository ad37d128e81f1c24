// Device-side helpers shared by the gfx950 kernels.
#pragma once

#include <math.h>

#include "kernels.h"

namespace mapdec {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Pointers into device memory, in the global address space: loads and
// stores through them are global_* instructions, which count only against
// vmcnt (generic pointers give flat_* instructions, which also count against
// lgkmcnt and so make every LDS wait also wait for global memory).
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T *p) {
    return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<const T> to_global(const T *p) {
    return (gptr<const T>)p;
}

// Wave-wide sum delivered to every lane, with DPP moves inside rows of 16
// lanes and four lane reads across rows (no LDS round trips).
__device__ __forceinline__ float dpp_row_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, false));
    return v;
}

__device__ __forceinline__ double dpp_move(double v, int ctrl) {
    const long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    switch (ctrl) {   // the control operand must be a constant
        case 0xB1:
            lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
            break;
        case 0x4E:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
            break;
        case 0x141:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
            break;
        default:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false);
            break;
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double dpp_row_sum(double v) {
    v += dpp_move(v, 0xB1);    // lanes i^1
    v += dpp_move(v, 0x4E);    // lanes i^2
    v += dpp_move(v, 0x141);   // mirror within 8
    v += dpp_move(v, 0x140);   // mirror within 16
    return v;
}

__device__ __forceinline__ float read_lane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T v) {
    v = dpp_row_sum(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Orders LDS traffic inside a single-wave workgroup without waiting for
// outstanding global loads and stores (a workgroup barrier would).
__device__ __forceinline__ void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Sum of one double per thread over the workgroup; every thread gets the
// same value (same summation order everywhere).  red: one double per wave.
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double tot = 0.0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) tot += red[w];
    __syncthreads();
    return tot;
}

// Ends one arm of a wave-uniform branch whose two arms differ only in an
// operand: the empty volatile asm keeps the compiler from merging the arms
// into one with per-lane selects, so the branch stays a scalar branch.
__device__ __forceinline__ void keep_branch() { asm volatile(""); }

// c ? a : b on two register values, written as a bitwise blend so that the
// compiler cannot turn "c ? x[i] : y[i]" over two register arrays into one
// access through a selected array address (which would move both arrays to
// scratch memory).  For a wave-uniform c this is one bitfield-insert.
__device__ __forceinline__ float blend(bool c, float a, float b) {
    const uint32_t m = 0u - (uint32_t)c;
    return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}
__device__ __forceinline__ double blend(bool c, double a, double b) {
    const uint64_t m = 0ull - (uint64_t)c;
    return __longlong_as_double((long long)(((uint64_t)__double_as_longlong(a) & m) |
                                            ((uint64_t)__double_as_longlong(b) & ~m)));
}

}  // namespace mapdec
