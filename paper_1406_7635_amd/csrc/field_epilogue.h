// field_epilogue.h -- per-cell local field terms, torque and reductions.
//
// Everything a cell needs once its magnetostatic field is known:
//   exchange (Eqs. eqBexch1 / eqBexch: 6 neighbours, harmonic-mean pair
//   coefficients from the packed lower-triangular table, missing or
//   non-magnetic neighbours contribute nothing -- the Neumann rule),
//   uniaxial anisotropy (2 Ku1/Msat (u.m) u + 4 Ku2/Msat (u.m)^3 u),
//   the applied field, the Landau-Lifshitz torque of Eq. eqLLG with the
//   damping sign, the embedded Runge-Kutta error norm and FP64 energies.
#pragma once

#include "mm_internal.h"

namespace mm {

__device__ inline float3 ld3(const float* __restrict__ p, long long n, long long i) {
    return make_float3(p[i], p[n + i], p[2 * n + i]);
}
__device__ inline void st3(float* __restrict__ p, long long n, long long i, float3 v) {
    p[i] = v.x;
    p[n + i] = v.y;
    p[2 * n + i] = v.z;
}
// Loads and stores through a uniform base and a 32-bit byte offset: an array
// of 3 ncell floats (ncell <= 2^28) stays below 2^32 bytes, so every offset
// fits.  They go through a raw buffer resource (base, no stride, 2^32 - 1
// bytes; the third word is the gfx9 family's untyped 32-bit format), so the
// base stays in scalar registers and each lane supplies only its 32-bit
// offset: no 64-bit address arithmetic per lane.  Every base passed here is
// uniform over the workgroup.
__device__ inline __amdgpu_buffer_rsrc_t buffer_of(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)0xffffffffu, 0x00020000);
}
__device__ inline float ldo(const float* base, unsigned int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(buffer_of(base), (int)off, 0, 0));
}
__device__ inline void sto(float* base, unsigned int off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), buffer_of(base), (int)off, 0, 0);
}
// components at byte offsets off, off + n4, off + 2 n4 from one base (n4 =
// 4 ncell; 3 ncell < 2^30 floats): one scalar base per array
__device__ inline float3 ld3o(const float* p, long long n, unsigned int off) {
    const unsigned int n4 = (unsigned int)n << 2;
    return make_float3(ldo(p, off), ldo(p, off + n4), ldo(p, off + 2u * n4));
}
__device__ inline void st3o(float* p, long long n, unsigned int off, float3 v) {
    const unsigned int n4 = (unsigned int)n << 2;
    sto(p, off, v.x);
    sto(p, off + n4, v.y);
    sto(p, off + 2u * n4, v.z);
}

__device__ inline float3 f3add(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline float3 f3sub(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline float3 f3scale(float s, float3 a) { return make_float3(s * a.x, s * a.y, s * a.z); }
__device__ inline float f3dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline float3 f3cross(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// index of the region pair (a, b) in the square exchange-coefficient table
__device__ inline int pair_index(int a, int b) { return (a << 8) | b; }

// Stage-derivative pointers, dt and the done flag, read once per kernel from
// the device-side solver state (the logical-to-physical buffer map changes on
// the device when a step is accepted).  All state words are loaded
// unconditionally first, so they arrive in one round trip, and the pointers
// are then picked with selects; the per-cell loops see no state loads.
struct Resolved {
    const float* kin[6];  // stage-combine inputs, kin[j] for j < sd.nk
    float* kout;          // where the torque goes (a k buffer or the caller's tau)
    const float* ke[7];   // error-norm inputs (null: the torque just computed)
    float dt;
    int done;             // the run already reached its end
};

__device__ inline Resolved resolve(const FieldArgs& a) {
    // the map (entries < 8) is packed 3 bits per entry into one word, so a
    // lookup is a shift rather than an indexed array
    unsigned int pk = 0;
#pragma unroll
    for (int j = 0; j < MAXK; ++j) pk |= ((unsigned int)a.st->perm[j] & 7u) << (3 * j);
    const double dt = a.st->dt;
    const int done = a.st->done;
    auto phys = [&](int logical) { return (int)((pk >> (3 * logical)) & 7u); };
    Resolved r;
    const long long n3 = 3 * a.ncell;
#pragma unroll
    for (int j = 0; j < 6; ++j) r.kin[j] = j < a.sd.nk ? a.kbuf + (long long)phys(a.sd.kidx[j]) * n3 : nullptr;
    r.kout = a.sd.out_k >= 0 ? a.kbuf + (long long)phys(a.sd.out_k) * n3 : a.tau;
#pragma unroll
    for (int j = 0; j < 7; ++j)
        r.ke[j] = (j < a.sd.nerr && a.sd.eidx[j] != a.sd.out_k) ? a.kbuf + (long long)phys(a.sd.eidx[j]) * n3
                                                                 : nullptr;
    r.dt = (float)dt;
    r.done = done;
    return r;
}

// Component c of the stage state m_s = m0 + dt sum_j a_j k_j of one cell (FP32).
// All terms are loaded before any is used so their latencies overlap.
__device__ inline float stage_comp(const FieldArgs& a, const Resolved& r, long long idx) {
    const float m0 = a.m0[idx];
    if (a.sd.nk == 0) return m0;
    float kv[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) kv[j] = j < a.sd.nk ? r.kin[j][idx] : 0.f;
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += a.sd.a[j] * kv[j];
    return m0 + r.dt * acc;
}

// Stage-state components at N positions given as byte offsets off[i] into the
// [3][ncell] arrays: out[i] = m0 + dt sum_{j<NK} a_j k_j at off[i], with NK a
// compile-time count so that every load of the batch is issued before the
// first is used (no data-dependent branches).
template <int NK, int N>
__device__ inline void stage_batch_nk(const FieldArgs& a, const Resolved& r, const unsigned int (&off)[N],
                                      float (&out)[N]) {
    float m0v[N];
    float kv[N][NK > 0 ? NK : 1];
#pragma unroll
    for (int i = 0; i < N; ++i) m0v[i] = ldo(a.m0, off[i]);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < NK; ++j) kv[i][j] = ldo(r.kin[j], off[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < NK; ++j) acc += a.sd.a[j] * kv[i][j];
        out[i] = NK > 0 ? m0v[i] + r.dt * acc : m0v[i];
    }
}

template <int N>
__device__ inline void stage_batch(const FieldArgs& a, const Resolved& r, const unsigned int (&off)[N],
                                   float (&out)[N]) {
    switch (a.sd.nk) {
        case 0: stage_batch_nk<0>(a, r, off, out); break;
        case 1: stage_batch_nk<1>(a, r, off, out); break;
        case 2: stage_batch_nk<2>(a, r, off, out); break;
        case 3: stage_batch_nk<3>(a, r, off, out); break;
        case 4: stage_batch_nk<4>(a, r, off, out); break;
        case 5: stage_batch_nk<5>(a, r, off, out); break;
        default: stage_batch_nk<6>(a, r, off, out); break;
    }
}

__device__ inline float3 stage_state(const FieldArgs& a, const Resolved& r, long long cell) {
    const long long n = a.ncell;
    return make_float3(stage_comp(a, r, cell), stage_comp(a, r, n + cell), stage_comp(a, r, 2 * n + cell));
}

// Exchange field at (x, y, z) from the state array mp.  A neighbour outside
// the grid is replaced by the cell itself (the Neumann rule), which adds
// c (m - m) = 0; so every neighbour is loaded without a branch.  Along a
// periodic axis the grid wraps around instead.  The six
// neighbour slots have fixed positions (x-, x+, y-, y+, z-, z+) so the arrays
// stay in registers; the y and z pairs are skipped (uniformly) for a single
// layer along that axis.
// DMI = false compiles the DMI branch out (the hot x passes of grids without it).
template <bool DMI = true>
__device__ inline float3 exchange_at(const FieldArgs& a, const RegionLut* lut, const float* __restrict__ mp,
                                     long long cell, int x, int y, int z, int r, float3 mc) {
    const long long n = a.ncell;
    const int sxy = a.nx * a.ny;
    const bool use_y = a.ny > 1, use_z = a.nz > 1;
    // wrap-around offsets of the low faces (the high faces take their negatives)
    const int ox = (a.pbc & 1) ? a.nx - 1 : 0;
    const int oy = (a.pbc & 2) ? sxy - a.nx : 0;
    const int oz = (a.pbc & 4) ? (int)(n - sxy) : 0;
    int d[6];  // neighbour - cell, in cells
    d[0] = x > 0 ? -1 : ox;
    d[1] = x < a.nx - 1 ? 1 : -ox;
    d[2] = y > 0 ? -a.nx : oy;
    d[3] = y < a.ny - 1 ? a.nx : -oy;
    d[4] = z > 0 ? -sxy : oz;
    d[5] = z < a.nz - 1 ? sxy : -oz;
    const float id2[3] = {a.idx2, a.idy2, a.idz2};
    const unsigned int c = (unsigned int)cell;
    int rn[6];
    float3 mn[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const bool use = i < 2 || (i < 4 ? use_y : use_z);
        if (use) {
            const unsigned int q = c + (unsigned int)d[i];
            rn[i] = a.region[q];
            mn[i] = ld3o(mp, n, q << 2);
        }
    }
    float3 b = make_float3(0.f, 0.f, 0.f);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const bool use = i < 2 || (i < 4 ? use_y : use_z);
        if (use) b = f3add(b, f3scale(a.ptab[pair_index(r, rn[i])] * id2[i / 2], f3sub(mn[i], mc)));
    }
    if (DMI && a.dmi) {
        // induced DMI (section "Dzyaloshinskii-Moriya interaction"):
        // B = 2D/Msat (dm_z/dx, dm_z/dy, -dm_x/dx - dm_y/dy), central
        // differences; an in-plane neighbour that is missing at the boundary
        // of the magnet (outside an open edge of the grid, or a cell with
        // Msat = 0) is replaced by the ghost
        // m + n Delta dm/di|_b (n = -1 low side, +1 high side) with
        // dm/dx|_b = xi (-m_z, 0, m_x), dm/dy|_b = xi (0, -m_z, m_y), xi = D/(2A);
        // the exchange field then takes 2A/Msat (ghost - m)/Delta^2 from it too.
        const float2 dm = a.dmi[r];
        const float hx = rsqrtf(a.idx2), hy = rsqrtf(a.idy2);
        const float3 gx = make_float3(-dm.y * mc.z, 0.f, dm.y * mc.x);
        const float3 gy = make_float3(0.f, -dm.y * mc.z, dm.y * mc.y);
        const bool wx = a.pbc & 1, wy = a.pbc & 2;
        const bool geo[4] = {x > 0 || wx, x < a.nx - 1 || wx, y > 0 || wy, y < a.ny - 1 || wy};
        const float cs = a.ptab[pair_index(r, r)];
        float3 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool loaded = i < 2 || use_y;
            const int rr = loaded ? rn[i] : r;
            const float3 val = loaded ? mn[i] : mc;
            const bool real = geo[i] && lut[rr].a.x > 0.f;
            const float3 g = i < 2 ? gx : gy;
            const float h = i < 2 ? hx : hy;
            const float3 ghost = f3add(mc, f3scale((i & 1) ? h : -h, g));
            v[i] = real ? val : ghost;
            if (!real) b = f3add(b, f3scale(cs * id2[i / 2], f3sub(ghost, mc)));
        }
        const float ix = 0.5f / hx, iy = 0.5f / hy;
        b = f3add(b, f3scale(dm.x, make_float3((v[1].z - v[0].z) * ix, (v[3].z - v[2].z) * iy,
                                               -(v[1].x - v[0].x) * ix - (v[3].y - v[2].y) * iy)));
    }
    return b;
}

// fmaxf drops a NaN operand, so a NaN norm would vanish from a max reduction:
// it enters as +inf instead (the controller then stops with a non-finite error).
__device__ inline float finite_or_inf(float v) { return v == v ? v : INFINITY; }

// Per-thread accumulators of the reductions.
struct EpiAcc {
    float errmax;
    float tqmax;
    double e[4];  // demag, exchange, anisotropy, Zeeman energy densities (summed)
};

__device__ inline void epi_init(EpiAcc& acc) {
    acc.errmax = 0.f;
    acc.tqmax = 0.f;
    acc.e[0] = acc.e[1] = acc.e[2] = acc.e[3] = 0.0;
}

// Everything after the magnetostatic field for one cell.
// lut: the region table (global memory, or a copy in LDS).  Returns the
// torque (zero in non-magnetic cells; only meaningful with EPI_TORQUE).
template <bool DMI = true>
__device__ inline float3 epilogue(const FieldArgs& a, const Resolved& rs, const RegionLut* lut,
                                const float* __restrict__ mp, long long cell, int x, int y, int z, float3 bd,
                                EpiAcc& acc) {
    const int flags = a.flags;
    const unsigned int c4 = (unsigned int)cell << 2;
    const int r = a.region[(unsigned int)cell];
    const RegionLut L = lut[r];
    const long long n = a.ncell;
    if (flags & EPI_BDEMAG) st3o(a.bdemag, n, c4, bd);
    float3 tq = make_float3(0.f, 0.f, 0.f);
    if (L.a.x == 0.f) {  // non-magnetic cell: no field, no torque
        if (flags & EPI_BEFF) st3o(a.beff, n, c4, tq);
        if (flags & EPI_TORQUE) st3o(rs.kout, n, c4, tq);
        return tq;
    }
    const float3 m = ld3o(mp, n, c4);
    const float3 bex = exchange_at<DMI>(a, lut, mp, cell, x, y, z, r, m);
    const float3 u = make_float3(L.b.x, L.b.y, L.b.z);
    const float um = f3dot(u, m);
    const float3 ban1 = f3scale(L.a.y * um, u);
    const float3 ban2 = f3scale(L.a.z * um * um * um, u);
    const float3 bz = make_float3(L.c.x, L.c.y, L.c.z);
    float3 B = f3add(f3add(bd, bex), f3add(f3add(ban1, ban2), bz));
    if (flags & EPI_THERM) B = f3add(B, ld3o(a.bth, n, c4));
    float ecub = 0.f;  // cubic anisotropy energy density / Msat
    if (a.cub) {
        // cubic anisotropy (section "Magneto-crystalline anisotropy"): with
        // a_i = c_i . m and s_i = a_i^2, B = sum_i g_i c_i where
        // g_i = a_i [k1 (s_j + s_k) + k2 s_j s_k + k3 s_i (s_j^2 + s_k^2)]
        // ({i, j, k} the three axes; k1 = -2 Kc1/Msat, k2 = -2 Kc2/Msat,
        // k3 = -4 Kc3/Msat).  The energy -1/4 M.B(Kc1) - 1/6 M.B(Kc2)
        // - 1/8 M.B(Kc3) uses m.B(Kc1) = 2 k1 (s1 s2 + s1 s3 + s2 s3),
        // m.B(Kc2) = 3 k2 s1 s2 s3, m.B(Kc3) = 2 k3 (s1^2 s2^2 + s1^2 s3^2 + s2^2 s3^2).
        const float4 p = a.cub[3 * r], q = a.cub[3 * r + 1], w = a.cub[3 * r + 2];
        const float3 c1 = make_float3(p.x, p.y, p.z), c2 = make_float3(q.x, q.y, q.z),
                     c3 = make_float3(w.x, w.y, w.z);
        const float a1 = f3dot(c1, m), a2 = f3dot(c2, m), a3 = f3dot(c3, m);
        const float s1 = a1 * a1, s2 = a2 * a2, s3 = a3 * a3;
        const float g1 = a1 * (p.w * (s2 + s3) + q.w * s2 * s3 + w.w * s1 * (s2 * s2 + s3 * s3));
        const float g2 = a2 * (p.w * (s1 + s3) + q.w * s1 * s3 + w.w * s2 * (s1 * s1 + s3 * s3));
        const float g3 = a3 * (p.w * (s1 + s2) + q.w * s1 * s2 + w.w * s3 * (s1 * s1 + s2 * s2));
        B = f3add(B, f3add(f3add(f3scale(g1, c1), f3scale(g2, c2)), f3scale(g3, c3)));
        if (flags & EPI_ENERGY)
            ecub = -(0.5f * p.w * (s1 * s2 + s1 * s3 + s2 * s3) + 0.5f * q.w * s1 * s2 * s3 +
                     0.25f * w.w * (s1 * s1 * s2 * s2 + s1 * s1 * s3 * s3 + s2 * s2 * s3 * s3));
    }
    if (flags & EPI_BEFF) st3o(a.beff, n, c4, B);
    if (flags & (EPI_TORQUE | EPI_MAXTQ | EPI_ERR)) {
        const float3 mxb = f3cross(m, B);
        const float3 mxmxb = f3cross(m, mxb);
        const float alpha = L.a.w;
        tq = (flags & EPI_PRECESS) ? f3scale(L.b.w, f3add(mxb, f3scale(alpha, mxmxb)))
                                   : f3scale(L.b.w * alpha, mxmxb);
        if (flags & EPI_TORQUE) st3o(rs.kout, n, c4, tq);
        if (flags & EPI_MAXTQ) acc.tqmax = fmaxf(acc.tqmax, finite_or_inf(sqrtf(f3dot(tq, tq))));
        if (flags & EPI_ERR) {
            float3 kv[7];
#pragma unroll
            for (int j = 0; j < 7; ++j)
                if (j < a.sd.nerr) kv[j] = rs.ke[j] ? ld3o(rs.ke[j], n, c4) : tq;
            float3 d = make_float3(0.f, 0.f, 0.f);
#pragma unroll
            for (int j = 0; j < 7; ++j)
                if (j < a.sd.nerr) d = f3add(d, f3scale(a.sd.e[j], kv[j]));
            acc.errmax = fmaxf(acc.errmax, finite_or_inf(sqrtf(f3dot(d, d))));
        }
    }
    if (flags & EPI_ENERGY) {
        const double ms = (double)L.a.x;
        const double mx = ms * m.x, my = ms * m.y, mz = ms * m.z;
        auto dot = [&](float3 b) { return mx * (double)b.x + my * (double)b.y + mz * (double)b.z; };
        acc.e[0] += -0.5 * dot(bd);
        acc.e[1] += -0.5 * dot(bex);
        acc.e[2] += -0.5 * dot(ban1) - 0.25 * dot(ban2);
        acc.e[2] += ms * (double)ecub;
        acc.e[3] += -dot(bz);
    }
    return tq;
}

// Workgroup reductions ------------------------------------------------------
__device__ inline float wave_max(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// red: LDS scratch of at least (NTH/64) * 6 doubles; NTH = threads of the workgroup.
template <int NTH>
__device__ inline void epi_reduce(const FieldArgs& a, EpiAcc& acc, double* red, int blk) {
    const int flags = a.flags;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = NTH / 64 > 0 ? NTH / 64 : 1;
    if (flags & (EPI_ERR | EPI_MAXTQ)) {
        const float e = wave_max(acc.errmax), t = wave_max(acc.tqmax);
        if (lane == 0) {
            red[wave * 6 + 4] = e;
            red[wave * 6 + 5] = t;
        }
    }
    if (flags & EPI_ENERGY) {
        for (int i = 0; i < 4; ++i) {
            const double s = wave_sum(acc.e[i]);
            if (lane == 0) red[wave * 6 + i] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (flags & EPI_ERR) {
            float e = 0.f;
#pragma unroll 1
            for (int w = 0; w < NW; ++w) e = fmaxf(e, (float)red[w * 6 + 4]);
            atomicMax(&a.st->err_bits, __float_as_uint(e));
        }
        if (flags & EPI_MAXTQ) {
            float t = 0.f;
#pragma unroll 1
            for (int w = 0; w < NW; ++w) t = fmaxf(t, (float)red[w * 6 + 5]);
            atomicMax(&a.st->tq_bits, __float_as_uint(t));
        }
        if (flags & EPI_ENERGY) {
            for (int i = 0; i < 4; ++i) {
                double s = 0.0;
#pragma unroll 1
                for (int w = 0; w < NW; ++w) s += red[w * 6 + i];
                a.partials[(long long)blk * 4 + i] = s;
            }
        }
    }
}

// Map a dispatch index to a logical tile so that consecutive tiles land on the
// same XCD (workgroups are dealt round-robin over the 8 XCDs), keeping
// neighbouring rows/columns in one L2.
__device__ inline int xcd_remap(int bid, int nblk) {
    constexpr int NX = 8;
    const int per = nblk / NX, rem = nblk % NX;
    const int xcd = bid % NX, slot = bid / NX;
    if (slot >= per) return bid;  // the ragged last round keeps its natural index
    (void)rem;
    return xcd * per + slot;
}

}  // namespace mm
