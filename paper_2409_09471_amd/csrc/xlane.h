// Cross-lane reductions of doubles inside a wavefront with data-parallel-
// primitive (DPP) moves: register-to-register within a row of 16 lanes, a few
// cycles each, where a shuffle is a round trip through the LDS crossbar.
#pragma once

#include <hip/hip_runtime.h>

namespace ttsg {

// DPP move of a double within a row of 16 lanes (two 32-bit moves).
template <int CTRL> __device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 16 lanes of a row: quad swaps (xor 1, xor 2), then the half-row
// and row mirrors.  Every step adds two partial sums in commuted order on the
// two lanes involved, so all 16 lanes end with bit-identical totals.  Every
// lane of the row must be active.
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return v;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over all 64 lanes (every lane active): row sums, then the four rows
// added in a fixed order as scalars, so every lane gets the same value.
__device__ __forceinline__ double wave_sum64(double v) {
    v = row_sum16(v);
    const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
    const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
    return (r0 + r1) + (r2 + r3);
}

// Keep (v, i) or take (v2, i2): larger value first, lower index on ties.
__device__ __forceinline__ void argmax_take(double& v, int& i, double v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}
template <int CTRL> __device__ __forceinline__ void argmax_dpp(double& v, int& i) {
    const double v2 = dpp_mov<CTRL>(v);
    const int i2 = __builtin_amdgcn_mov_dpp(i, CTRL, 0xf, 0xf, false);
    argmax_take(v, i, v2, i2);
}
// Index of the largest value over all 64 lanes (every lane active; the lowest
// index wins ties); the same on every lane.
__device__ __forceinline__ int wave_argmax64(double v, int i) {
    argmax_dpp<0xB1>(v, i);
    argmax_dpp<0x4E>(v, i);
    argmax_dpp<0x141>(v, i);
    argmax_dpp<0x140>(v, i);
    double bv = readlane_f64(v, 0);
    int bi = __builtin_amdgcn_readlane(i, 0);
    for (int r = 16; r < 64; r += 16) argmax_take(bv, bi, readlane_f64(v, r), __builtin_amdgcn_readlane(i, r));
    return bi;
}

}  // namespace ttsg
