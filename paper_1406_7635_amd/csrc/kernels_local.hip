// kernels_local.hip -- table preparation, elementwise field pass without
// demag, stage combine, step controller, finalisation and reductions.
#include <math.h>

#include "../../include/mm.h"
#include "extra_field.h"
#include "field_epilogue.h"
#include "thermal_noise.h"
#include "step_control.h"

namespace mm {

// ---------------------------------------------------------------------------
// Region tables (section "Material Regions") from the FP64 parameters.
// lut: anisotropy prefactors 2 Ku1/Msat and 4 Ku2/Msat (the paper prints
// B_sat; Msat is the reading with units of tesla), torque prefactor
// -gamma/(1+alpha^2).  ptab: for every ordered region pair (i, j), at
// i * NREG + j, the exchange coefficient 2 S(i,j) 2 l_i l_j/(l_i + l_j),
// l = Aex/Msat, of Eq. eqBexch (S from the packed lower triangle
// max(i,j)(max(i,j)+1)/2 + min(i,j); S(i,i) = 1); 0 when either region is
// non-magnetic.  The square layout makes the lookup a shift and an or.
__global__ void k_prepare_tables(const mm_params* __restrict__ p, RegionLut* __restrict__ lut,
                                 float* __restrict__ ptab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double gamma = p->gamma_ll != 0.0 ? p->gamma_ll : GAMMA_DEFAULT;
    if (i < NREG) {
        const double ms = p->msat[i];
        const double inv = ms > 0.0 ? 1.0 / ms : 0.0;
        const double al = p->alpha[i];
        RegionLut L;
        L.a = make_float4((float)ms, (float)(2.0 * p->ku1[i] * inv), (float)(4.0 * p->ku2[i] * inv),
                          (float)al);
        L.b = make_float4((float)p->anis_u[i][0], (float)p->anis_u[i][1], (float)p->anis_u[i][2],
                          (float)(-gamma / (1.0 + al * al)));
        L.c = make_float4((float)p->bext[i][0], (float)p->bext[i][1], (float)p->bext[i][2], 0.f);
        lut[i] = L;
    }
    if (i < NREG * NREG) {
        const int r1 = i / NREG, r2 = i % NREG;
        const int hi = r1 > r2 ? r1 : r2, lo = r1 > r2 ? r2 : r1;
        const double m1 = p->msat[hi], m2 = p->msat[lo];
        double c = 0.0;
        if (m1 > 0.0 && m2 > 0.0) {
            const double l1 = p->aex[hi] / m1, l2 = p->aex[lo] / m2;
            const double s = (hi == lo) ? 1.0 : p->exch_scale[hi * (hi + 1) / 2 + lo];
            if (l1 + l2 > 0.0) c = 2.0 * s * (2.0 * l1 * l2 / (l1 + l2));
        }
        ptab[i] = (float)c;
    }
}

hipError_t launch_prepare_tables(const double* params64, RegionLut* lut, float* ptab, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare_tables, dim3((NREG * NREG + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<const mm_params*>(params64), lut, ptab);
    return hipGetLastError();
}

// FFT twiddles exp(-2 pi i m / pt), evaluated in FP64 and rounded once.
__global__ void k_twiddles(cf* tw, int pt) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < pt) {
        double s, c;
        sincospi(-2.0 * (double)m / (double)pt, &s, &c);
        tw[m] = mkc((float)c, (float)s);
    }
}

hipError_t launch_twiddles(cf* tw, int pt, hipStream_t s) {
    hipLaunchKernelGGL(k_twiddles, dim3((pt + 255) / 256), dim3(256), 0, s, tw, pt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stage combine m_s = m0 + dt sum a_j k_j (used when demag is off; with demag
// the first FFT pass does it on the fly).
__global__ void __launch_bounds__(NT) k_combine(const FieldArgs a) {
    const Resolved rs = resolve(a);
    if ((a.flags & EPI_CHECK_DONE) && rs.done) return;
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= a.ncell) return;
    st3(a.ms, a.ncell, i, stage_state(a, rs, i));
}

hipError_t launch_combine(const FieldArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((a.ncell + NT - 1) / NT)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

// Field pass without the magnetostatic term: one thread per cell.
// Field pass without the convolution: one thread per cell; the magnetostatic
// field is zero, or taken from bd_in (the surrogate's prediction).
__global__ void __launch_bounds__(NT) k_local(const FieldArgs a, const float* __restrict__ bd_in) {
    __shared__ double red[(NT / 64) * 6];
    const Resolved rs = resolve(a);
    if ((a.flags & EPI_CHECK_DONE) && rs.done) return;
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    EpiAcc acc;
    epi_init(acc);
    if (i < a.ncell) {
        const int x = (int)(i % a.nx);
        const long long r = i / a.nx;
        const int y = (int)(r % a.ny), z = (int)(r / a.ny);
        const float* mp = a.sd.nk > 0 ? a.ms : a.m0;
        const float3 bd = bd_in ? ld3(bd_in, a.ncell, i) : make_float3(0.f, 0.f, 0.f);
        epilogue(a, rs, a.lut, mp, i, x, y, z, bd, acc);
    }
    if (a.flags & (EPI_ERR | EPI_MAXTQ | EPI_ENERGY)) epi_reduce<NT>(a, acc, red, blockIdx.x);
}

// One stage of Heun's method without the magnetostatic term, fused: the
// thermal field of the cell is generated in place (no field buffer) and, on
// the second stage (mnew set), the new state m0 + dt (k1 + k2)/2 is formed
// from the first-stage derivative and the torque just computed.
__global__ void __launch_bounds__(NT) k_local_heun(const FieldArgs a, HeunLocal h) {
    __shared__ double red[(NT / 64) * 6];
    const Resolved rs = resolve(a);
    if ((a.flags & EPI_CHECK_DONE) && rs.done) return;
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    EpiAcc acc;
    epi_init(acc);
    if (i < a.ncell) {
        const int x = (int)(i % a.nx);
        const long long r = i / a.nx;
        const int y = (int)(r % a.ny), z = (int)(r / a.ny);
        const float* mp = a.sd.nk > 0 ? a.ms : a.m0;
        float3 bth = make_float3(0.f, 0.f, 0.f);
        if (h.sigma) {
            const float sc = h.sigma[a.region[i]] * (float)(1.0 / sqrt(a.st->dt));
            if (sc != 0.f) bth = thermal_eta(i, a.st->therm_step, h.seed, sc);
        }
        const float3 tq = epilogue(a, rs, a.lut, mp, i, x, y, z, bth, acc);
        if (h.mnew) {
            const float3 m0 = ld3(a.m0, a.ncell, i), k1 = ld3(rs.kin[0], a.ncell, i);
            const float hd = 0.5f * rs.dt;
            st3(h.mnew, a.ncell, i, make_float3(m0.x + hd * (k1.x + tq.x), m0.y + hd * (k1.y + tq.y),
                                                m0.z + hd * (k1.z + tq.z)));
        }
    }
    if (a.flags & (EPI_ERR | EPI_MAXTQ | EPI_ENERGY)) epi_reduce<NT>(a, acc, red, blockIdx.x);
}

// Heun steps of uncoupled cells: no magnetostatic term, no exchange coupling
// (Aex = 0 in every magnetic region), no DMI, no excitation -- the thermal
// switching workload of the paper's figure figSwitch.  Each cell then evolves
// alone, so one launch advances it by nsteps fixed steps with its state in
// registers: per step the thermal field of (cell, step), k1 and k2 from the
// cell's local field (uniaxial and cubic anisotropy, applied field, thermal
// field: the terms of the field epilogue, in its order), the new state
// m0 + dt (k1 + k2)/2 normalised.  The solver state is advanced afterwards by
// k_advance_steps.
__device__ inline float3 uncoupled_torque(const RegionLut& L, const float4* __restrict__ cub, int r, float3 m,
                                          float3 bth, bool precess) {
    const float3 u = make_float3(L.b.x, L.b.y, L.b.z);
    const float um = f3dot(u, m);
    const float3 ban1 = f3scale(L.a.y * um, u);
    const float3 ban2 = f3scale(L.a.z * um * um * um, u);
    const float3 bz = make_float3(L.c.x, L.c.y, L.c.z);
    float3 B = f3add(make_float3(0.f, 0.f, 0.f), f3add(f3add(ban1, ban2), bz));
    B = f3add(B, bth);
    if (cub) {
        const float4 p = cub[3 * r], q = cub[3 * r + 1], w = cub[3 * r + 2];
        const float3 c1 = make_float3(p.x, p.y, p.z), c2 = make_float3(q.x, q.y, q.z),
                     c3 = make_float3(w.x, w.y, w.z);
        const float a1 = f3dot(c1, m), a2 = f3dot(c2, m), a3 = f3dot(c3, m);
        const float s1 = a1 * a1, s2 = a2 * a2, s3 = a3 * a3;
        const float g1 = a1 * (p.w * (s2 + s3) + q.w * s2 * s3 + w.w * s1 * (s2 * s2 + s3 * s3));
        const float g2 = a2 * (p.w * (s1 + s3) + q.w * s1 * s3 + w.w * s2 * (s1 * s1 + s3 * s3));
        const float g3 = a3 * (p.w * (s1 + s2) + q.w * s1 * s2 + w.w * s3 * (s1 * s1 + s2 * s2));
        B = f3add(B, f3add(f3add(f3scale(g1, c1), f3scale(g2, c2)), f3scale(g3, c3)));
    }
    const float3 mxb = f3cross(m, B);
    const float3 mxmxb = f3cross(m, mxb);
    const float alpha = L.a.w;
    return precess ? f3scale(L.b.w, f3add(mxb, f3scale(alpha, mxmxb))) : f3scale(L.b.w * alpha, mxmxb);
}

__global__ void __launch_bounds__(NT) k_heun_uncoupled(const FieldArgs a, const float* __restrict__ sigma,
                                                       unsigned long long seed, int nsteps, int precess) {
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= a.ncell) return;
    const double dtd = a.st->dt;
    const float dt = (float)dtd, hd = 0.5f * dt;
    const unsigned long long step0 = a.st->therm_step;
    const int r = a.region[i];
    const RegionLut L = a.lut[r];
    const float sc = sigma ? sigma[r] * (float)(1.0 / sqrt(dtd)) : 0.f;
    float3 m = ld3(a.m0, a.ncell, i);
    for (int s = 0; s < nsteps; ++s) {
        float3 mn = m;
        if (L.a.x != 0.f) {
            const float3 bth = sc != 0.f ? thermal_eta(i, step0 + (unsigned long long)s, seed, sc)
                                         : make_float3(0.f, 0.f, 0.f);
            const float3 k1 = uncoupled_torque(L, a.cub, r, m, bth, precess != 0);
            const float3 ms = make_float3(m.x + dt * k1.x, m.y + dt * k1.y, m.z + dt * k1.z);
            const float3 k2 = uncoupled_torque(L, a.cub, r, ms, bth, precess != 0);
            mn = make_float3(m.x + hd * (k1.x + k2.x), m.y + hd * (k1.y + k2.y), m.z + hd * (k1.z + k2.z));
        }
        const float n2 = f3dot(mn, mn);
        m = f3scale(n2 > 0.f ? rsqrtf(n2) : 0.f, mn);
    }
    st3(const_cast<float*>(a.m0), a.ncell, i, m);
}

// n accepted fixed steps: time, counters and the thermal generator's step;
// like the controller, the next step is clipped to land on t_end
__global__ void k_advance_steps(DevState* st, int n) {
    for (int s = 0; s < n; ++s) st->t = st->t + st->dt;
    st->steps += n;
    st->therm_step += (unsigned long long)n;
    st->evals += 2LL * n;
    st->accepted = 1;
    if (isfinite(st->t_end) && st->t + st->dt > st->t_end && st->t < st->t_end) st->dt = st->t_end - st->t;
}

hipError_t launch_heun_uncoupled(const FieldArgs& a, const float* sigma, unsigned long long seed, int nsteps,
                                 int precess, hipStream_t s) {
    hipLaunchKernelGGL(k_heun_uncoupled, dim3((unsigned)((a.ncell + NT - 1) / NT)), dim3(NT), 0, s, a, sigma, seed,
                       nsteps, precess);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_advance_steps, dim3(1), dim3(1), 0, s, a.st, nsteps);
    return hipGetLastError();
}

hipError_t launch_local_heun(const FieldArgs& a, const HeunLocal& h, hipStream_t s) {
    hipLaunchKernelGGL(k_local_heun, dim3((unsigned)((a.ncell + NT - 1) / NT)), dim3(NT), 0, s, a, h);
    return hipGetLastError();
}

hipError_t launch_local(const FieldArgs& a, hipStream_t s, int* nblocks_out, const float* bd_in) {
    const int nb = (int)((a.ncell + NT - 1) / NT);
    if (nblocks_out) *nblocks_out = nb;
    hipLaunchKernelGGL(k_local, dim3(nb), dim3(NT), 0, s, a, bd_in);
    return hipGetLastError();
}

// max over cells of |b_sur - b_exact| and of |b_exact| (atomics on the float
// bits of non-negative values)
__global__ void __launch_bounds__(NT) k_sur_check(const float* __restrict__ bs, const float* __restrict__ be,
                                                  long long n, DevState* st) {
    __shared__ float red[2][NT / 64];
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    float dn = 0.f, en = 0.f;
    if (i < n) {
        const float3 s3 = ld3(bs, n, i), e3 = ld3(be, n, i);
        const float3 d = f3sub(s3, e3);
        dn = sqrtf(f3dot(d, d));
        en = sqrtf(f3dot(e3, e3));
        if (!(dn == dn)) dn = INFINITY;  // a NaN prediction fails the check
    }
    dn = wave_max(dn);
    en = wave_max(en);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = dn;
        red[1][wave] = en;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float a = 0.f, b = 0.f;
        for (int w = 0; w < NT / 64; ++w) {
            a = fmaxf(a, red[0][w]);
            b = fmaxf(b, red[1][w]);
        }
        atomicMax(&st->sur_num_bits, __float_as_uint(a));
        atomicMax(&st->sur_den_bits, __float_as_uint(b));
    }
}

hipError_t launch_sur_check(const float* b_sur, const float* b_exact, long long ncell, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_sur_check, dim3((unsigned)((ncell + NT - 1) / NT)), dim3(NT), 0, s, b_sur, b_exact, ncell,
                       st);
    return hipGetLastError();
}

__global__ void k_sur_gate(DevState* st, double tol) {
    const double num = (double)__uint_as_float(st->sur_num_bits);
    const double den = (double)__uint_as_float(st->sur_den_bits);
    st->sur_num_bits = 0u;
    st->sur_den_bits = 0u;
    const double err = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
    st->sur_err = err;
    if (!(err <= tol)) {
        st->sur_fail = 1;
        st->sur_fallbacks += 1;
    }
}

hipError_t launch_sur_gate(DevState* st, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_sur_gate, dim3(1), dim3(1), 0, s, st, tol);
    return hipGetLastError();
}

__global__ void k_sur_clear(DevState* st) { st->sur_fail = 0; }

hipError_t launch_sur_clear(DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_sur_clear, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError();
}

// Torque from a given field (Eq. eqLLG, damping sign).
__global__ void __launch_bounds__(NT) k_llg(const FieldArgs a, const float* __restrict__ beff,
                                            float* __restrict__ tau, int precess) {
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= a.ncell) return;
    const RegionLut L = a.lut[a.region[i]];
    float3 t = make_float3(0.f, 0.f, 0.f);
    if (L.a.x != 0.f) {
        const float3 m = ld3(a.m0, a.ncell, i), B = ld3(beff, a.ncell, i);
        const float3 mxb = f3cross(m, B), mxmxb = f3cross(m, mxb);
        t = precess ? f3scale(L.b.w, f3add(mxb, f3scale(L.a.w, mxmxb))) : f3scale(L.b.w * L.a.w, mxmxb);
    }
    st3(tau, a.ncell, i, t);
}

hipError_t launch_llg(const FieldArgs& a, const float* beff, float* tau, int precess, hipStream_t s) {
    hipLaunchKernelGGL(k_llg, dim3((unsigned)((a.ncell + NT - 1) / NT)), dim3(NT), 0, s, a, beff, tau,
                       precess);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Solver state of one context and its adaptive step controller (the update
// rules are in step_control.h).
__global__ void k_set_state(DevState* st, double t, double dt, double t_end, double max_err,
                            double headroom, double dt_min, double dt_max, int order_low,
                            int reset_counters, int init_perm, long long target_steps) {
    set_state(st, t, dt, t_end, max_err, headroom, dt_min, dt_max, order_low, reset_counters, init_perm,
              target_steps);
}

hipError_t launch_set_state(DevState* st, double t, double dt, double t_end, double max_err,
                            double headroom, double dt_min, double dt_max, int order_low,
                            int reset_counters, int init_perm, long long target_steps,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, s, st, t, dt, t_end, max_err, headroom,
                       dt_min, dt_max, order_low, reset_counters, init_perm, target_steps);
    return hipGetLastError();
}

__global__ void k_reset_accum(DevState* st) {
    st->err_bits = 0u;
    st->tq_bits = 0u;
}

hipError_t launch_reset_accum(DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_accum, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError();
}

__global__ void k_controller(DevState* st, int last_k, int evals, int check_done) {
    controller_update(st, last_k, evals, check_done);
}

hipError_t launch_controller(DevState* st, int last_k, int evals, int check_done, hipStream_t s) {
    hipLaunchKernelGGL(k_controller, dim3(1), dim3(1), 0, s, st, last_k, evals, check_done);
    return hipGetLastError();
}

// After an accepted embedded step: m0 <- m_s / |m_s| (m_s holds the
// higher-order solution, the last stage state).  The caller's array is only
// written when the controller accepted.
__global__ void __launch_bounds__(NT) k_finalize(const FieldArgs a) {
    if (!a.st->accepted) return;
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= a.ncell) return;
    const float3 m = ld3(a.ms, a.ncell, i);
    const float n2 = f3dot(m, m);
    const float inv = n2 > 0.f ? rsqrtf(n2) : 0.f;
    st3(const_cast<float*>(a.m0), a.ncell, i, f3scale(inv, m));
}

hipError_t launch_finalize(const FieldArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((a.ncell + NT - 1) / NT)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

// Fixed-step update m0 <- normalise(m0 + dt sum b_j k_j) (classical RK4).
__global__ void __launch_bounds__(NT) k_final_combine(const FieldArgs a) {
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= a.ncell) return;
    const Resolved rs = resolve(a);
    const float3 m = stage_state(a, rs, i);
    const float n2 = f3dot(m, m);
    const float inv = n2 > 0.f ? rsqrtf(n2) : 0.f;
    st3(const_cast<float*>(a.m0), a.ncell, i, f3scale(inv, m));
}

hipError_t launch_final_combine(const FieldArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_final_combine, dim3((unsigned)((a.ncell + NT - 1) / NT)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

// Deterministic FP64 sum of the per-workgroup energy partials: every thread
// sums a fixed strided subset in order, then a fixed-shape tree.
__global__ void __launch_bounds__(256) k_reduce_energy(const double* __restrict__ partials, int nblocks,
                                                       DevState* st, double cellvol) {
    __shared__ double sh[4][256];
    const int t = threadIdx.x;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = t; b < nblocks; b += 256)
        for (int i = 0; i < 4; ++i) s[i] += partials[(long long)b * 4 + i];
    for (int i = 0; i < 4; ++i) sh[i][t] = s[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int i = 0; i < 4; ++i) sh[i][t] += sh[i][t + w];
        __syncthreads();
    }
    if (t == 0) {
        double tot = 0.0;
        for (int i = 0; i < 4; ++i) {
            st->red[i] = sh[i][0] * cellvol;
            tot += st->red[i];
        }
        st->red[4] = tot;
    }
}

hipError_t launch_reduce_energy(const double* partials, int nblocks, DevState* st, double cellvol,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(256), 0, s, partials, nblocks, st, cellvol);
    return hipGetLastError();
}

// Per-face exchange coefficients as the field kernels gather them.
__global__ void __launch_bounds__(NT) k_exchange_dump(const FieldArgs a, float* __restrict__ out) {
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= a.ncell) return;
    const int x = (int)(i % a.nx);
    const long long rr = i / a.nx;
    const int y = (int)(rr % a.ny), z = (int)(rr / a.ny);
    const int r = a.region[i];
    const long long sxy = (long long)a.nx * a.ny;
    // a face exists inside the grid, or across a periodic boundary of an axis
    // longer than one cell
    const bool wx = (a.pbc & 1) && a.nx > 1, wy = (a.pbc & 2) && a.ny > 1, wz = (a.pbc & 4) && a.nz > 1;
    const bool has[6] = {x > 0 || wx, x < a.nx - 1 || wx, y > 0 || wy, y < a.ny - 1 || wy,
                         z > 0 || wz, z < a.nz - 1 || wz};
    const long long nxl = a.nx;
    const long long off[6] = {x > 0 ? -1 : nxl - 1, x < a.nx - 1 ? 1 : 1 - nxl,
                              y > 0 ? -nxl : sxy - nxl, y < a.ny - 1 ? nxl : nxl - sxy,
                              z > 0 ? -sxy : (a.nz - 1) * sxy, z < a.nz - 1 ? sxy : (1 - a.nz) * sxy};
    const float id2[6] = {a.idx2, a.idx2, a.idy2, a.idy2, a.idz2, a.idz2};
    for (int f = 0; f < 6; ++f) {
        float c = 0.f;
        if (has[f]) c = a.ptab[pair_index(r, a.region[i + off[f]])] * id2[f];
        out[f * a.ncell + i] = c;
    }
}

hipError_t launch_exchange_dump(const FieldArgs& a, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_exchange_dump, dim3((unsigned)((a.ncell + NT - 1) / NT)), dim3(NT), 0, s, a, out);
    return hipGetLastError();
}

}  // namespace mm
