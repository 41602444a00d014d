// kernels_thermal.hip -- Brown's thermal field (section "Thermal fluctuations").
//
// B_therm = eta sqrt(2 alpha kB T / (Msat gamma_LL dV dt)) per cell, eta three
// independent standard normal numbers drawn anew for every time step and held
// over the stages of the step.  The numbers come from the counter-based
// generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011), so a cell's
// noise of a step is a pure function of (cell, step, seed): nothing is stored
// between steps and any cell can be recomputed alone.
//   counter (cell, step mod 2^32, step div 2^32, 0), key (seed mod 2^32,
//   seed div 2^32); ten rounds; 32-bit outputs x -> u = (floor(x/2^8) + 1/2)/2^24;
//   eta_x, eta_y = sqrt(-2 ln u0) (cos, sin)(2 pi u1), eta_z = sqrt(-2 ln u2) cos(2 pi u3).
#include <hip/hip_runtime.h>

#include "mm_internal.h"

namespace mm {

namespace {

constexpr int NTT = 256;

struct U4 {
    unsigned int x, y, z, w;
};

// Philox4x32 round constants: multipliers and the key increments (Weyl sequence)
__device__ inline U4 philox10(U4 c, unsigned int k0, unsigned int k1) {
    constexpr unsigned int MA = 0xD2511F53u, MB = 0xCD9E8D57u;
    constexpr unsigned int WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned int hi0 = __umulhi(MA, c.x), lo0 = MA * c.x;
        const unsigned int hi1 = __umulhi(MB, c.z), lo1 = MB * c.z;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += WA;
        k1 += WB;
    }
    return c;
}

__device__ inline float unit24(unsigned int x) { return ((float)(x >> 8) + 0.5f) * 0x1p-24f; }

__global__ void __launch_bounds__(NTT) k_thermal(long long ncell, const uint8_t* __restrict__ region,
                                                 const float* __restrict__ sigma, unsigned long long seed,
                                                 const DevState* st, int from_state, unsigned long long step,
                                                 double dt, int check_done, float* __restrict__ bth) {
    if (check_done && st->done) return;
    const long long i = (long long)blockIdx.x * NTT + threadIdx.x;
    if (i >= ncell) return;
    if (from_state) {
        step = st->therm_step;
        dt = st->dt;
    }
    const float sc = sigma[region[i]] * (float)(1.0 / sqrt(dt));
    float ex = 0.f, ey = 0.f, ez = 0.f;
    if (sc != 0.f) {
        const U4 o = philox10(U4{(unsigned int)i, (unsigned int)step, (unsigned int)(step >> 32), 0u},
                              (unsigned int)seed, (unsigned int)(seed >> 32));
        const float r0 = sqrtf(-2.f * logf(unit24(o.x)));
        const float r2 = sqrtf(-2.f * logf(unit24(o.z)));
        float s1, c1, s3, c3;
        sincospif(2.f * unit24(o.y), &s1, &c1);
        sincospif(2.f * unit24(o.w), &s3, &c3);
        ex = sc * r0 * c1;
        ey = sc * r0 * s1;
        ez = sc * r2 * c3;
    }
    bth[i] = ex;
    bth[ncell + i] = ey;
    bth[2 * ncell + i] = ez;
}

__global__ void k_set_therm_step(DevState* st, unsigned long long step) { st->therm_step = step; }

}  // namespace

hipError_t launch_thermal(long long ncell, const uint8_t* region, const float* sigma, unsigned long long seed,
                          const DevState* st, int from_state, unsigned long long step, double dt, int check_done,
                          float* bth, hipStream_t s) {
    hipLaunchKernelGGL(k_thermal, dim3((unsigned)((ncell + NTT - 1) / NTT)), dim3(NTT), 0, s, ncell, region, sigma,
                       seed, st, from_state, step, dt, check_done, bth);
    return hipGetLastError();
}

hipError_t launch_set_therm_step(DevState* st, unsigned long long step, hipStream_t s) {
    hipLaunchKernelGGL(k_set_therm_step, dim3(1), dim3(1), 0, s, st, step);
    return hipGetLastError();
}

}  // namespace mm
