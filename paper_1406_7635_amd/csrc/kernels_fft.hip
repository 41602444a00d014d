// kernels_fft.hip -- the FP32 magnetostatic convolution passes of one grid:
// the kernels around the device bodies of fft_passes.h, with a workgroup per
// tile (the dispatch index mapped XCD-aware), and their launchers.
#include <hip/hip_ext.h>

#include "fft_passes.h"

namespace mm {


// Tile order of the passes that evaluate the exchange field (x-inverse and
// fused), for grids of several layers: the tiles of one y block over all z
// planes follow each other, so the z neighbours of a row (a plane apart) are
// in tiles that run in the same round and come from L2; in plane-major order
// they are a plane's worth of tiles away and are fetched from HBM again.  A
// bijection on the tiles whenever no tile straddles two planes (else the
// natural order).  Partial sums stay indexed by tile, so results do not change.
__device__ inline int x_tile_order(int t, const FieldArgs& a, int rows_per_tile) {
    if (a.nz <= 1 || a.ny % rows_per_tile) return t;
    const int tpp = a.ny / rows_per_tile;  // tiles per plane
    const int yb = t / a.nz, z = t - yb * a.nz;
    return z * tpp + yb;
}

// FULL: x is a periodic axis transformed at its own length (P = nx).
// W: workgroup width (XCfg): 0 wide, 1 narrow (grids with few rows).
template <int P, bool FULL, int W>
__global__ void __launch_bounds__((XCfg<P, W>::NTH)) k_xfwd(const FieldArgs a) {
    constexpr int GI = XCfg<P, W>::GI, GL = XCfg<P, W>::GL;
    extern __shared__ cf lds[];
    __shared__ long long rbs[2 * GI];
    const Resolved rs = resolve(a);
    if ((a.flags & EPI_CHECK_DONE) && rs.done) return;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    row_bases<GI>(a, blk * GI, rbs, threadIdx.x);
    XLut<P, W> lut;
    lut.load(a, threadIdx.x);
    xfwd_part<P, false, FULL, W>(a, rs, lds, rbs, reinterpret_cast<RegionLut*>(lds + GI * GL), &lut, 0.f, blk,
                                 threadIdx.x);
}

template <int P, bool DMI, bool FULL, int W>
__global__ void __launch_bounds__((XCfg<P, W>::NTH)) __attribute__((amdgpu_waves_per_eu(P >= 4096 ? 4 : 6)))
k_xinv(const FieldArgs a) {
    constexpr int GI = XCfg<P, W>::GI, GL = XCfg<P, W>::GL, NTH = XCfg<P, W>::NTH;
    extern __shared__ cf lds[];
    __shared__ double red[(NTH / 64 > 0 ? NTH / 64 : 1) * 6];
    __shared__ long long rbs[2 * GI];
    const int blk = x_tile_order(xcd_remap(blockIdx.x, gridDim.x), a, 2 * GI);
    row_bases<GI>(a, blk * GI, rbs, threadIdx.x);
    __syncthreads();
    // the solver state only now: its read overlaps the spectrum loads (the
    // finished-run test is inside, after them)
    const Resolved rs = resolve(a);
    xinv_part<P, false, DMI, FULL, W>(a, rs, lds, rbs, reinterpret_cast<RegionLut*>(lds + GI * GL), red, blk,
                                      threadIdx.x);
}

// Fused pass: the x-inverse of stage s (torque k_s, read m_s from ai.ms)
// followed, row pair by row pair, by the x-forward of stage s + 1 (combine
// with k_s from LDS as the last term, m_{s+1} to af.ms, a second buffer since
// other workgroups still read m_s for the exchange field).
// (FULL: every x holds data, so the combine keeps twice the loads in flight;
// its register budget is that of four waves per SIMD instead of six)
template <int P, bool DMI, bool FULL, int W>
__global__ void __launch_bounds__((XCfg<P, W>::NTH)) __attribute__((amdgpu_waves_per_eu(FULL ? 4 : 6)))
k_xrow(const FieldArgs ai, const FieldArgs af, float a_last) {
    constexpr int GI = XCfg<P, W>::GI, GL = XCfg<P, W>::GL, NTH = XCfg<P, W>::NTH;
    extern __shared__ cf lds[];
    __shared__ double red[(NTH / 64 > 0 ? NTH / 64 : 1) * 6];
    __shared__ long long rbs[2 * GI];
    const int blk = x_tile_order(xcd_remap(blockIdx.x, gridDim.x), ai, 2 * GI);
    row_bases<GI>(ai, blk * GI, rbs, threadIdx.x);
    __syncthreads();
    const Resolved rsi = resolve(ai);  // read overlaps the spectrum loads
    RegionLut* lut_l = reinterpret_cast<RegionLut*>(lds + GI * GL);
    if (!xinv_part<P, true, DMI, FULL, W>(ai, rsi, lds, rbs, lut_l, red, blk, threadIdx.x)) return;
    __syncthreads();
    // the next stage's pointers only now (short live ranges across the first part)
    const Resolved rsf = resolve(af);
    xfwd_part<P, true, FULL, W>(af, rsf, lds, rbs, lut_l, nullptr, a_last, blk, threadIdx.x);
}


template <int P, int MODE, int NC, bool CFAST>
__global__ void __launch_bounds__(ColCfg<P>::NTH) k_col(const ColArgs a) {
    extern __shared__ cf lds[];
    col_body<P, MODE, NC, CFAST>(a, xcd_remap(blockIdx.x, gridDim.x), lds, threadIdx.x);
}

template <int P, bool FULL, int W>
__global__ void __launch_bounds__((Col3Cfg<P, W>::NTH), 4) k_col3(const ColArgs a) {
    extern __shared__ cf lds[];
    col3_body<P, FULL, W>(a, xcd_remap(blockIdx.x, gridDim.x), lds, threadIdx.x);
}

// two workgroups per CU for the two-layer case (the z step of more layers
// needs the registers of one)
template <int PY, int PZ>
__global__ void __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(PZ == 4 ? 6 : 1))) k_yz(const ColArgs a) {
    extern __shared__ cf lds[];
    yz_body<PY, PZ>(a, xcd_remap(blockIdx.x, gridDim.x), lds, threadIdx.x);
}


// ---------------------------------------------------------------------------
// Launch helpers: dispatch the run-time padded length to a template instance.


template <int P, int W>
static int x_blocks_w(int nrows) {
    const int npairs = (nrows + 1) / 2;
    return (npairs + XCfg<P, W>::GI - 1) / XCfg<P, W>::GI;
}

// Narrow x workgroups when the wide ones would not give every CU two
// (and the narrow form actually holds fewer row pairs).
constexpr int NARROW_BELOW = 512;
template <int P>
static int x_width(int nrows) {
    return (XCfg<P, 1>::GI < XCfg<P, 0>::GI && x_blocks_w<P, 0>(nrows) < NARROW_BELOW) ? 1 : 0;
}
template <int P>
static int x_blocks(int nrows) {
    return x_width<P>(nrows) ? x_blocks_w<P, 1>(nrows) : x_blocks_w<P, 0>(nrows);
}

template <int P, int W>
static hipError_t xfwd_pw(const FieldArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const size_t lds = x_lds<P, W>();
    const dim3 g(x_blocks_w<P, W>(a.nrows)), b(XCfg<P, W>::NTH);
    if (a.full_x)
        hipExtLaunchKernelGGL((k_xfwd<P, true, W>), g, b, (uint32_t)lds, s, e0, e1, 0, a);
    else
        hipExtLaunchKernelGGL((k_xfwd<P, false, W>), g, b, (uint32_t)lds, s, e0, e1, 0, a);
    return hipGetLastError();
}
template <int P>
static hipError_t xfwd_p(const FieldArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return x_width<P>(a.nrows) ? xfwd_pw<P, 1>(a, s, e0, e1) : xfwd_pw<P, 0>(a, s, e0, e1);
}

template <int P, int W>
static hipError_t xinv_pw(const FieldArgs& a, hipStream_t s, int* nb_out, hipEvent_t e0, hipEvent_t e1) {
    const size_t lds = x_lds<P, W>();
    const int nb = x_blocks_w<P, W>(a.nrows);
    if (nb_out) *nb_out = nb;
#define MM_XI(D, F) \
    hipExtLaunchKernelGGL((k_xinv<P, D, F, W>), dim3(nb), dim3(XCfg<P, W>::NTH), (uint32_t)lds, s, e0, e1, 0, a)
    if (a.dmi) {
        if (a.full_x)
            MM_XI(true, true);
        else
            MM_XI(true, false);
    } else {
        if (a.full_x)
            MM_XI(false, true);
        else
            MM_XI(false, false);
    }
#undef MM_XI
    return hipGetLastError();
}
template <int P>
static hipError_t xinv_p(const FieldArgs& a, hipStream_t s, int* nb_out, hipEvent_t e0, hipEvent_t e1) {
    return x_width<P>(a.nrows) ? xinv_pw<P, 1>(a, s, nb_out, e0, e1) : xinv_pw<P, 0>(a, s, nb_out, e0, e1);
}

template <int P, int W>
static hipError_t xrow_pw(const FieldArgs& ai, const FieldArgs& af, float a_last, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1) {
    const size_t lds = x_lds<P, W>();
    const dim3 g(x_blocks_w<P, W>(ai.nrows)), b(XCfg<P, W>::NTH);
#define MM_XR(D, F) \
    hipExtLaunchKernelGGL((k_xrow<P, D, F, W>), g, b, (uint32_t)lds, s, e0, e1, 0, ai, af, a_last)
    if (ai.dmi) {
        if (ai.full_x)
            MM_XR(true, true);
        else
            MM_XR(true, false);
    } else {
        if (ai.full_x)
            MM_XR(false, true);
        else
            MM_XR(false, false);
    }
#undef MM_XR
    return hipGetLastError();
}
template <int P>
static hipError_t xrow_p(const FieldArgs& ai, const FieldArgs& af, float a_last, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
    return x_width<P>(ai.nrows) ? xrow_pw<P, 1>(ai, af, a_last, s, e0, e1) : xrow_pw<P, 0>(ai, af, a_last, s, e0, e1);
}

template <int P, int MODE, int NC, bool CFAST>
static hipError_t col_p(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const size_t lds = col_lds<P, MODE, NC, CFAST>();
    const long long nb = (long long)col_ntile<P, MODE, NC>(a.ncol) * a.nouter;
    hipExtLaunchKernelGGL((k_col<P, MODE, NC, CFAST>), dim3((unsigned)nb), dim3(ColCfg<P>::NTH), (uint32_t)lds, s,
                          e0, e1, 0, a);
    return hipGetLastError();
}

template <int PY, int PZ>
static hipError_t yz_p(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int nb = (a.ncol + YzCfg<PY, PZ>::T - 1) / YzCfg<PY, PZ>::T;
    hipExtLaunchKernelGGL((k_yz<PY, PZ>), dim3(nb), dim3(YzCfg<PY, PZ>::NTH), (uint32_t)yz_lds<PY, PZ>(), s, e0, e1,
                          0, a);
    return hipGetLastError();
}

template <int P, int W>
static hipError_t col3_pw(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const long long nb = (a.ncol + Col3Cfg<P, W>::T - 1) / Col3Cfg<P, W>::T;
    const dim3 g((unsigned)nb), b(Col3Cfg<P, W>::NTH);
    if (a.full)
        hipExtLaunchKernelGGL((k_col3<P, true, W>), g, b, (uint32_t)col3_lds<P, W>(), s, e0, e1, 0, a);
    else
        hipExtLaunchKernelGGL((k_col3<P, false, W>), g, b, (uint32_t)col3_lds<P, W>(), s, e0, e1, 0, a);
    return hipGetLastError();
}
// narrow (about one wave) column workgroups when the wide ones would not
// give every CU two
template <int P>
static hipError_t col3_p(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const long long nb_wide = (a.ncol + Col3Cfg<P, 0>::T - 1) / Col3Cfg<P, 0>::T;
    if (Col3Cfg<P, 1>::T < Col3Cfg<P, 0>::T && nb_wide < NARROW_BELOW) return col3_pw<P, 1>(a, s, e0, e1);
    return col3_pw<P, 0>(a, s, e0, e1);
}

#define MM_CASES(M) M(1) M(2) M(4) M(8) M(16) M(32) M(64) M(128) M(256) M(512) M(1024) M(2048) M(4096)

template <int P>
static hipError_t allow_lds(const void* f, size_t bytes) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int P, int W>
static hipError_t configure_xw(void) {
    constexpr size_t L = x_lds<P, W>();
    hipError_t e = allow_lds<P>((const void*)k_xfwd<P, false, W>, L);
    if (e == hipSuccess) e = allow_lds<P>((const void*)k_xfwd<P, true, W>, L);
    if (e == hipSuccess) e = allow_lds<P>((const void*)k_xinv<P, false, false, W>, L);
    if (e == hipSuccess) e = allow_lds<P>((const void*)k_xinv<P, true, false, W>, L);
    if (e == hipSuccess) e = allow_lds<P>((const void*)k_xinv<P, false, true, W>, L);
    if (e == hipSuccess) e = allow_lds<P>((const void*)k_xinv<P, true, true, W>, L);
    if constexpr (P >= 8) {
        if (e == hipSuccess) e = allow_lds<P>((const void*)k_xrow<P, false, false, W>, L);
        if (e == hipSuccess) e = allow_lds<P>((const void*)k_xrow<P, true, false, W>, L);
        if (e == hipSuccess) e = allow_lds<P>((const void*)k_xrow<P, false, true, W>, L);
        if (e == hipSuccess) e = allow_lds<P>((const void*)k_xrow<P, true, true, W>, L);
    }
    return e;
}

template <int P>
static hipError_t configure_x(void) {
    hipError_t e = configure_xw<P, 0>();
    if (e == hipSuccess) e = configure_xw<P, 1>();
    return e;
}

// Dispatch (py, pz) of the thin-grid convolution to f.template operator()<PY, PZ>();
// returns hipErrorInvalidValue for pairs it does not serve.
template <class F>
static hipError_t yz_dispatch(int py, int pz, const F& f) {
    switch (pz) {
#define MZ(pzv)                                                                 \
    case pzv:                                                                   \
        switch (py) {                                                           \
            MM_CASES(MY##pzv)                                                   \
            default:                                                            \
                return hipErrorInvalidValue;                                    \
        }
#define MYB(q, pzv)                                                             \
    case q:                                                                     \
        if constexpr (use_yz<q, pzv>()) return f.template operator()<q, pzv>(); \
        return hipErrorInvalidValue;
#define MY4(q) MYB(q, 4)
#define MY8(q) MYB(q, 8)
        MZ(4)
        MZ(8)
#undef MY4
#undef MY8
#undef MYB
#undef MZ
        default:
            return hipErrorInvalidValue;
    }
}

__global__ void k_zkernel(const float* __restrict__ khat, float* __restrict__ zk, long long rows, int pz) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const int kzh = pz / 2 + 1;
    const float* K = khat + i * kzh * 6;
    float* G = zk + i * zkernel_len(pz);
    for (int d = 0; d < pz / 2; ++d) {
        double e[4] = {0.0, 0.0, 0.0, 0.0}, o[2] = {0.0, 0.0};
        for (int kz = 0; kz < pz; ++kz) {
            const bool fq = 2 * kz > pz;
            const int kh = fq ? pz - kz : kz;
            double sn, cs;
            sincospi(2.0 * (double)(kz * d) / (double)pz, &sn, &cs);
            for (int q = 0; q < 4; ++q) e[q] += (double)K[kh * 6 + q] * cs;
            // xz and yz are odd in z
            for (int q = 0; q < 2; ++q) o[q] += (fq ? -1.0 : 1.0) * (double)K[kh * 6 + 4 + q] * sn;
        }
        float* out = G + (d == 0 ? 0 : 4 + 6 * (d - 1));
        for (int q = 0; q < 4; ++q) out[q] = (float)e[q];
        if (d > 0) {
            out[4] = (float)o[0];
            out[5] = (float)o[1];
        }
    }
}

int zkernel_floats(int pz) { return zkernel_len(pz); }

hipError_t launch_zkernel(const float* khat, float* zker, long long rows, int pz, hipStream_t s) {
    hipLaunchKernelGGL(k_zkernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, khat, zker, rows, pz);
    return hipGetLastError();
}

struct YzNop {
    template <int PY, int PZ>
    hipError_t operator()() const {
        return hipSuccess;
    }
};
struct YzLaunch {
    const ColArgs& a;
    hipStream_t s;
    hipEvent_t e0, e1;
    template <int PY, int PZ>
    hipError_t operator()() const {
        return yz_p<PY, PZ>(a, s, e0, e1);
    }
};
struct YzConfigure {
    template <int PY, int PZ>
    hipError_t operator()() const {
        return hipFuncSetAttribute((const void*)k_yz<PY, PZ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)yz_lds<PY, PZ>());
    }
};

bool yz_supported(int py, int pz) { return yz_dispatch(py, pz, YzNop{}) == hipSuccess; }

hipError_t launch_yz(int py, int pz, const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return yz_dispatch(py, pz, YzLaunch{a, s, e0, e1});
}

template <int P>
static hipError_t configure_col(bool three_d) {
    if (!three_d) {
        if constexpr (use_col3<P>()) {
            hipError_t e = allow_lds<P>((const void*)k_col3<P, false, 0>, col3_lds<P, 0>());
            if (e == hipSuccess) e = allow_lds<P>((const void*)k_col3<P, true, 0>, col3_lds<P, 0>());
            if (e == hipSuccess) e = allow_lds<P>((const void*)k_col3<P, false, 1>, col3_lds<P, 1>());
            if (e == hipSuccess) e = allow_lds<P>((const void*)k_col3<P, true, 1>, col3_lds<P, 1>());
            return e;
        }
        return allow_lds<P>((const void*)k_col<P, COL_CONV, 4, false>, col_lds<P, COL_CONV, 4>());
    }
    hipError_t e = allow_lds<P>((const void*)k_col<P, COL_FWD, 4, false>, col_lds<P, COL_FWD, 4>());
    if (e == hipSuccess) e = allow_lds<P>((const void*)k_col<P, COL_INV, 4, false>, col_lds<P, COL_INV, 4>());
    return e;
}

template <int P>
static hipError_t configure_zconv(void) {
    return allow_lds<P>((const void*)k_col<P, COL_CONV, 6, true>, col_lds<P, COL_CONV, 6, true>());
}

hipError_t configure_field_kernels(int px, int py, int pz) {
    hipError_t e = hipErrorInvalidValue;
    switch (px) {
#define M(p)                 \
    case p:                  \
        e = configure_x<p>(); \
        break;
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    switch (py) {
#define M(p)                         \
    case p:                          \
        e = configure_col<p>(pz > 1); \
        break;
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
    if (e != hipSuccess || pz == 1) return e;
    if (yz_supported(py, pz)) return yz_dispatch(py, pz, YzConfigure{});
    switch (pz) {
#define M(p)                    \
    case p:                     \
        e = configure_zconv<p>(); \
        break;
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
    return e;
}

int xinv_blocks(int px, int nrows) {
    switch (px) {
#define M(p) \
    case p:  \
        return x_blocks<p>(nrows);
        MM_CASES(M)
#undef M
        default:
            return 0;
    }
}

hipError_t launch_xfwd(int px, const FieldArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (px) {
#define M(p) \
    case p:  \
        return xfwd_p<p>(a, s, e0, e1);
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_xrow(int px, const FieldArgs& ai, const FieldArgs& af, float a_last, hipStream_t s,
                       hipEvent_t e0, hipEvent_t e1) {
    switch (px) {
#define M(p)                                                                       \
    case p:                                                                        \
        if constexpr (p >= 8) return xrow_p<p>(ai, af, a_last, s, e0, e1);          \
        return hipErrorInvalidValue;
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_xinv(int px, const FieldArgs& a, hipStream_t s, int* nb_out, hipEvent_t e0, hipEvent_t e1) {
    switch (px) {
#define M(p) \
    case p:  \
        return xinv_p<p>(a, s, nb_out, e0, e1);
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_col(int p, int mode, const ColArgs& a, int ncomp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (mode == COL_FWD) {
        switch (p) {
#define M(q) \
    case q:  \
        return col_p<q, COL_FWD, 4, false>(a, s, e0, e1);
            MM_CASES(M)
#undef M
            default:
                return hipErrorInvalidValue;
        }
    }
    if (mode == COL_INV) {
        switch (p) {
#define M(q) \
    case q:  \
        return col_p<q, COL_INV, 4, false>(a, s, e0, e1);
            MM_CASES(M)
#undef M
            default:
                return hipErrorInvalidValue;
        }
    }
    if (ncomp == 4) {
        switch (p) {
#define M(q)                                          \
    case q:                                           \
        if constexpr (use_col3<q>()) return col3_p<q>(a, s, e0, e1); \
        return col_p<q, COL_CONV, 4, false>(a, s, e0, e1);
            MM_CASES(M)
#undef M
            default:
                return hipErrorInvalidValue;
        }
    }
    switch (p) {
#define M(q) \
    case q:  \
        return col_p<q, COL_CONV, 6, true>(a, s, e0, e1);
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace mm
