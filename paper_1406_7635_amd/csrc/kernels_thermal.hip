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

#include "extra_field.h"
#include "mm_internal.h"
#include "thermal_noise.h"

namespace mm {

namespace {

constexpr int NTT = 256;

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
    float3 e = make_float3(0.f, 0.f, 0.f);
    if (sc != 0.f) e = thermal_eta(i, step, seed, sc);
    const float ex = e.x, ey = e.y, ez = e.z;
    bth[i] = ex;
    bth[ncell + i] = ey;
    bth[2 * ncell + i] = ez;
}

__global__ void k_set_therm_step(DevState* st, unsigned long long step) { st->therm_step = step; }

__global__ void __launch_bounds__(NTT) k_extra_field(const ExtraArgs e, const DevState* st, double cs,
                                                     int check_done, float* __restrict__ bth) {
    if (check_done && st->done) return;
    const long long i = (long long)blockIdx.x * NTT + threadIdx.x;
    if (i >= e.ncell) return;
    const double dt = st->dt, ts = st->t + cs * dt;
    float3 v = make_float3(0.f, 0.f, 0.f);
    if (e.sigma) {
        const float sc = e.sigma[e.region[i]] * (float)(1.0 / sqrt(dt));
        if (sc != 0.f) v = thermal_eta(i, st->therm_step, e.seed, sc);
    }
#pragma unroll
    for (int k = 0; k < MAX_EXC; ++k) {
        if (k < e.nexc) {
            const float f = (float)(e.exc[k].a + e.exc[k].b * sin(e.exc[k].omega * ts + e.exc[k].phi));
            const float* g = e.exc[k].g;
            v.x += f * g[i];
            v.y += f * g[e.ncell + i];
            v.z += f * g[2 * e.ncell + i];
        }
    }
    bth[i] = v.x;
    bth[e.ncell + i] = v.y;
    bth[2 * e.ncell + i] = v.z;
}

}  // namespace

hipError_t launch_thermal(long long ncell, const uint8_t* region, const float* sigma, unsigned long long seed,
                          const DevState* st, int from_state, unsigned long long step, double dt, int check_done,
                          float* bth, hipStream_t s) {
    hipLaunchKernelGGL(k_thermal, dim3((unsigned)((ncell + NTT - 1) / NTT)), dim3(NTT), 0, s, ncell, region, sigma,
                       seed, st, from_state, step, dt, check_done, bth);
    return hipGetLastError();
}

hipError_t launch_extra_field(const ExtraArgs& e, const DevState* st, double cs, int check_done, float* bth,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_extra_field, dim3((unsigned)((e.ncell + NTT - 1) / NTT)), dim3(NTT), 0, s, e, st, cs,
                       check_done, bth);
    return hipGetLastError();
}

hipError_t launch_set_therm_step(DevState* st, unsigned long long step, hipStream_t s) {
    hipLaunchKernelGGL(k_set_therm_step, dim3(1), dim3(1), 0, s, st, step);
    return hipGetLastError();
}

}  // namespace mm
