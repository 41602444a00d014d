// extra_field.h -- the additive field of a stage: Brown's thermal field of the
// step and the time-dependent excitation terms f_k(t_s) g_k(r) at the stage
// time (kernels_thermal.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mm_internal.h"

namespace mm {

constexpr int MAX_EXC = 4;

// f(t) = a + b sin(omega t + phi) times the profile g ([3][ncell] FP32, T)
struct ExcTerm {
    const float* g;
    double a, b, omega, phi;
};

struct ExtraArgs {
    long long ncell;
    const uint8_t* region;
    const float* sigma;       // thermal prefactors per region; null: no thermal field
    unsigned long long seed;
    int nexc;
    ExcTerm exc[MAX_EXC];
};

// bth <- thermal field of the state's generator step (if sigma) plus
// sum_k f_k(t + cs dt) g_k, with t, dt from the device state
hipError_t launch_extra_field(const ExtraArgs& e, const DevState* st, double cs, int check_done, float* bth,
                              hipStream_t s);

// nsteps fixed Heun steps of uncoupled cells in one launch, then the solver
// state advanced by nsteps accepted steps (kernels_local.hip)
hipError_t launch_heun_uncoupled(const FieldArgs& a, const float* sigma, unsigned long long seed, int nsteps,
                                 int precess, hipStream_t s);

}  // namespace mm
