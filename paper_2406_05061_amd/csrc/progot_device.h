// Device helpers shared by the FP32 and BF16 kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pot {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kNegBig = -1.0e30f;  // finite "minus infinity" of running maxima

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

// Loads and stores of global memory through pointers whose address space the
// compiler cannot infer (fields of a job table in device memory).  Without the
// cast they compile to flat instructions, which also count against the LDS
// wait counter, so every LDS wait in a tile loop would also wait for the
// next tile's prefetch.  T must be a scalar or an ext_vector_type.
template <typename T>
__device__ __forceinline__ T ldg(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ void stg(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

// Maximum of v over the lanes l, l ^ 16, l ^ 32 and l ^ 48 (the four lane
// groups that share an MFMA output column) with the cross-row swaps of
// gfx950, which stay in the VALU: v_permlane16_swap of v with itself leaves
// v[l & ~16] in one result and v[l | 16] in the other, v_permlane32_swap the
// same for bit 5.  A __shfl_xor is an LDS round trip (ds_bpermute) on the
// critical path of every tile.  All 64 lanes must be active.
__device__ __forceinline__ float max_lane_groups(float v) {
    const unsigned u = __float_as_uint(v);
    const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    const float m = fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
    const unsigned w = __float_as_uint(m);
    const auto b = __builtin_amdgcn_permlane32_swap(w, w, false, false);
    return fmaxf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// The lane's D/4 features of row `row` of U (zero beyond nu and d).
template <int D>
__device__ __forceinline__ void row_fetch(const float *__restrict__ U, int64_t nu, int d,
                                          int64_t row, int lq, float (&u)[D / 4]) {
    constexpr int KD = D / 4;
    const int c0 = lq * KD;
    if (row < nu && d == D) {
        const f4 *p = reinterpret_cast<const f4 *>(U + row * D + c0);
#pragma unroll
        for (int k = 0; k < KD / 4; ++k) {
            f4 v = ldg(p + k);
            u[4 * k + 0] = v.x; u[4 * k + 1] = v.y; u[4 * k + 2] = v.z; u[4 * k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < KD; ++k)
            u[k] = (row < nu && c0 + k < d) ? ldg(U + row * d + c0 + k) : 0.f;
    }
}

}  // namespace
}  // namespace pot
