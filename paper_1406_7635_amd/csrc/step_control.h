// step_control.h -- the adaptive step controller of one solver state.
//
// Section "Adaptive time step": eps = dt max|sum (b - b*) k|; accept when
// eps <= MaxErr; next dt = dt * clamp(headroom (MaxErr/eps)^(1/(q+1)), 0.1, 2)
// (2 when eps = 0), clamped to [dt_min, dt_max] and clipped so the run lands
// on t_end.  On accept the last stage derivative becomes the first of the next
// step (first same as last) by swapping the buffer map.
#pragma once

#include <math.h>

#include "mm_internal.h"

namespace mm {

// (Re)start a run: time, step, options; counters and the buffer map optionally.
__device__ inline void set_state(DevState* st, double t, double dt, double t_end, double max_err, double headroom,
                                 double dt_min, double dt_max, int order_low, int reset_counters, int init_perm,
                                 long long target_steps) {
    st->t = t;
    st->dt = dt;
    st->t_end = t_end;
    st->max_err = max_err;
    st->headroom = headroom;
    st->dt_min = dt_min;
    st->dt_max = dt_max;
    st->order_low = order_low;
    st->err_bits = 0u;
    st->tq_bits = 0u;
    st->accepted = 0;
    st->done = 0;
    st->target_steps = target_steps;
    st->sur_num_bits = 0u;
    st->sur_den_bits = 0u;
    st->sur_fail = 0;
    if (reset_counters) {
        st->steps = st->rejects = st->evals = 0;
        st->status = 0;
        st->err = 0.0;
        st->sur_err = 0.0;
        st->sur_fallbacks = 0;
    }
    if (init_perm)
        for (int i = 0; i < 8; ++i) st->perm[i] = i;
}

__device__ inline void controller_update(DevState* st, int last_k, int evals, int check_done) {
    if (check_done && st->done) {
        st->accepted = 0;  // a no-op attempt after the run ended: nothing to finalise
        return;
    }
    if (st->sur_fail) {
        // the surrogate missed its tolerance: reject, keep dt (the host repeats
        // the step on the exact path)
        st->accepted = 0;
        st->err_bits = 0u;
        st->evals += evals;
        return;
    }
    const double emax = (double)__uint_as_float(st->err_bits);
    const double dt = st->dt;
    const double err = dt * emax;
    st->err = err;
    st->err_bits = 0u;
    st->evals += evals;
    if (!isfinite(err)) {
        st->accepted = 0;
        st->rejects += 1;
        st->status = -5;  // MM_ENONFINITE
        st->done = 1;
        return;
    }
    const bool acc = err <= st->max_err;
    double fac = 2.0;
    if (err > 0.0) {
        fac = st->headroom * pow(st->max_err / err, 1.0 / (double)(st->order_low + 1));
        fac = fmin(2.0, fmax(0.1, fac));
    }
    const bool clipped = isfinite(st->t_end) && (st->t + dt >= st->t_end);
    if (acc) {
        st->t = clipped ? st->t_end : st->t + dt;
        st->steps += 1;
        st->therm_step += 1;
        if (last_k > 0) {
            const int tmp = st->perm[0];
            st->perm[0] = st->perm[last_k];
            st->perm[last_k] = tmp;
        }
    } else {
        st->rejects += 1;
    }
    st->accepted = acc ? 1 : 0;
    double dtn = dt * fac;
    if (st->dt_max > 0.0) dtn = fmin(dtn, st->dt_max);
    if (acc && clipped) st->done = 1;
    if (st->target_steps > 0 && st->steps >= st->target_steps) st->done = 1;
    // the step law's proposal below dt_min stops the run, unless the run has
    // just ended (a step clipped to t_end proposes from its short length);
    // clipping the next step to t_end below does not count
    if (!st->done && dtn < st->dt_min) {
        st->status = -6;  // MM_ESTEP
        st->done = 1;
    }
    if (isfinite(st->t_end) && st->t + dtn > st->t_end && st->t < st->t_end) dtn = st->t_end - st->t;
    st->dt = dtn;
}

}  // namespace mm
