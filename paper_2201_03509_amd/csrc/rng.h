// Counter-based normal draws shared by the kernels: Philox4x32-10 (Salmon et
// al., SC'11) and the Box-Muller transform of its four words.  A draw is
// addressed by key = (seed low word, segment) and counter = (k, iteration low,
// iteration high, seed high word); u = (x + 1/2) 2^-32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace c3rng {

// a ^ b ^ c in one instruction (three-input bitwise op, truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // full 32x32 -> 64-bit products: one v_mad_u64_u32 each instead of a
        // separate high and low multiply
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        if (r < 2) {
            // words that are uniform when only the first counter word varies
            // across lanes: plain XORs leave them to the scalar unit
            c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        } else {
            c = make_uint4(xor3(hi1, c.y, k.x), lo1, xor3(hi0, c.w, k.y), lo0);
        }
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// -2 ln u for u = (x + 1/2) 2^-32 with the hardware log2 (FP32 path)
__device__ __forceinline__ float m2log_u(uint32_t x) {
    const float u = ((float)x + 0.5f) * 2.3283064365386963e-10f;
    return -1.3862943611198906f * __builtin_amdgcn_logf(u);  // -2 ln 2 log2(u)
}
__device__ __forceinline__ double m2log_u_d(uint32_t x) {
    return -2.0 * log(((double)x + 0.5) * 2.3283064365386963e-10);
}

template <typename T>
__device__ __forceinline__ void normals4(uint4 w, T *z) {
    if constexpr (sizeof(T) == 4) {
        // -2 ln u >= 2^-32 and q > 0 stay far from denormals: the raw
        // hardware square root needs no range scaling here
        const float r0 = __builtin_amdgcn_sqrtf(m2log_u(w.x)), r1 = __builtin_amdgcn_sqrtf(m2log_u(w.z));
        // hardware sine/cosine take their argument in revolutions: sin(2 pi u)
        const float u1 = ((float)w.y + 0.5f) * 2.3283064365386963e-10f;
        const float u3 = ((float)w.w + 0.5f) * 2.3283064365386963e-10f;
        const float s0 = __builtin_amdgcn_sinf(u1), c0 = __builtin_amdgcn_cosf(u1);
        const float s1 = __builtin_amdgcn_sinf(u3), c1 = __builtin_amdgcn_cosf(u3);
        z[0] = r0 * c0;
        z[1] = r0 * s0;
        z[2] = r1 * c1;
        z[3] = r1 * s1;
    } else {
        double r0 = sqrt(m2log_u_d(w.x)), r1 = sqrt(m2log_u_d(w.z));
        double s0, c0, s1, c1;
        sincospi(((double)w.y + 0.5) * 4.656612873077392578125e-10, &s0, &c0);
        sincospi(((double)w.w + 0.5) * 4.656612873077392578125e-10, &s1, &c1);
        z[0] = r0 * c0;
        z[1] = r0 * s0;
        z[2] = r1 * c1;
        z[3] = r1 * s1;
    }
}

}  // namespace c3rng
