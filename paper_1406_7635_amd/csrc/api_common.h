// api_common.h -- host helpers shared by the C-ABI entry points: padded
// lengths, HIP error mapping, parameter validation.
#pragma once

#include <math.h>

#include "../../include/mm.h"
#include "mm_internal.h"

namespace mm {

// padded FFT length of an axis of n cells: the power of two >= 2n - 1 (none for n = 1)
inline int pad_len(int n) {
    if (n == 1) return 1;
    int p = 1;
    while (p < 2 * n - 1) p <<= 1;
    return p;
}

inline int map_err(hipError_t e) {
    if (e == hipSuccess) return MM_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MM_ENOMEM;
    return MM_EDEVICE;
}

#define MM_TRY(expr)                      \
    do {                                  \
        const hipError_t e_ = (expr);     \
        if (e_ != hipSuccess) return map_err(e_); \
    } while (0)

#define MM_CHECK(expr)                    \
    do {                                  \
        const int s_ = (expr);            \
        if (s_ != MM_OK) return s_;       \
    } while (0)

inline bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

inline int validate_params(const mm_params* p) {
    if (!p) return MM_EINVAL;
    for (int i = 0; i < NREG; ++i) {
        const double v[5] = {p->msat[i], p->aex[i], p->alpha[i], p->ku1[i], p->ku2[i]};
        for (double x : v)
            if (!isfinite(x)) return MM_EINVAL;
        if (p->msat[i] < 0.0 || p->alpha[i] < 0.0 || p->aex[i] < 0.0) return MM_EINVAL;
        for (int k = 0; k < 3; ++k)
            if (!isfinite(p->anis_u[i][k]) || !isfinite(p->bext[i][k])) return MM_EINVAL;
    }
    for (int i = 0; i < MM_NPAIRS; ++i)
        if (!isfinite(p->exch_scale[i])) return MM_EINVAL;
    if (!isfinite(p->gamma_ll) || p->gamma_ll < 0.0) return MM_EINVAL;
    return MM_OK;
}

}  // namespace mm
