// thermal_noise.h -- the random vector of Brown's thermal field for one cell
// and step (section "Thermal fluctuations"), shared by the field-buffer
// kernel and the fused local Heun pass.
//
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) at counter
// (cell, step mod 2^32, step div 2^32, 0) and key (seed mod 2^32, seed div
// 2^32); 32-bit outputs x -> u = (floor(x / 2^8) + 1/2) / 2^24; Box-Muller:
// eta_x, eta_y = sqrt(-2 ln u0) (cos, sin)(2 pi u1), eta_z = sqrt(-2 ln u2) cos(2 pi u3).
#pragma once

#include <hip/hip_runtime.h>

namespace mm {

struct PhiloxU4 {
    unsigned int x, y, z, w;
};

__device__ inline PhiloxU4 philox4x32_10(PhiloxU4 c, unsigned int k0, unsigned int k1) {
    // round multipliers and the key increments (Weyl sequence)
    constexpr unsigned int MA = 0xD2511F53u, MB = 0xCD9E8D57u;
    constexpr unsigned int WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned int hi0 = __umulhi(MA, c.x), lo0 = MA * c.x;
        const unsigned int hi1 = __umulhi(MB, c.z), lo1 = MB * c.z;
        c = PhiloxU4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += WA;
        k1 += WB;
    }
    return c;
}

__device__ inline float philox_unit24(unsigned int x) { return ((float)(x >> 8) + 0.5f) * 0x1p-24f; }

// sc * eta for cell i at generator step `step`
__device__ inline float3 thermal_eta(long long i, unsigned long long step, unsigned long long seed, float sc) {
    const PhiloxU4 o = philox4x32_10(PhiloxU4{(unsigned int)i, (unsigned int)step, (unsigned int)(step >> 32), 0u},
                                     (unsigned int)seed, (unsigned int)(seed >> 32));
    const float r0 = sqrtf(-2.f * logf(philox_unit24(o.x)));
    const float r2 = sqrtf(-2.f * logf(philox_unit24(o.z)));
    float s1, c1, s3, c3;
    sincospif(2.f * philox_unit24(o.y), &s1, &c1);
    sincospif(2.f * philox_unit24(o.w), &s3, &c3);
    return make_float3(sc * r0 * c1, sc * r0 * s1, sc * r2 * c3);
}

}  // namespace mm
