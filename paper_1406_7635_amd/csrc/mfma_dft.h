// mfma_dft.h -- split-precision DFT matrices on the matrix cores (gfx950).
//
// A batch of R-point DFTs (R = 16, or two 8-point DFTs side by side) is one
// real 16 x 16 x 32 GEMM per output part: Re Y = [Re F | -Im F] [Re x; Im x],
// Im Y = [Im F | Re F] [Re x; Im x].  Operands are split x = x_hi + x_lo in
// BF16 or FP16 (hi = round(x), lo = round(x - hi)); a product keeps
// hi hi + hi lo + lo hi with FP32 accumulation.  The DFT matrices are split
// once per context from FP64 values (k_dft_tables).
#pragma once

#include "../../include/mm.h"
#include "field_epilogue.h"

namespace mm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int PREC>
struct Low;

template <>
struct Low<MM_PREC_BF16> {
    using T = __bf16;
    using T8 = bf16x8;
    static constexpr bool SCALE = false;
    __device__ static f32x4 mfma(T8 a, T8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

template <>
struct Low<MM_PREC_FP16> {
    using T = _Float16;
    using T8 = f16x8;
    static constexpr bool SCALE = true;
    __device__ static f32x4 mfma(T8 a, T8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

// hi = round(x), lo = round(x - hi)
template <int PREC>
__device__ inline void split8(const float (&x)[8], typename Low<PREC>::T8& hi, typename Low<PREC>::T8& lo) {
    using T = typename Low<PREC>::T;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const T h = (T)x[e];
        hi[e] = h;
        lo[e] = (T)(x[e] - (float)h);
    }
}

// The split DFT matrices, one entry per lane of a wave (rows l % 16, K block
// 8 (l / 16) ... + 7): table [mode][inverse][lane] of {re_hi, re_lo, im_hi,
// im_lo}, 8 values each; mode 0: 16-point DFT, mode 1: two 8-point DFTs
// (block-diagonal).  Built once per context in FP64 by k_dft_tables.
template <int PREC>
struct DftEntry {
    typename Low<PREC>::T8 re_hi, re_lo, im_hi, im_lo;
};
static_assert(sizeof(DftEntry<MM_PREC_BF16>) * 256 == DFT_TABLE_BYTES, "DFT table size");
static_assert(sizeof(DftEntry<MM_PREC_FP16>) * 256 == DFT_TABLE_BYTES, "DFT table size");

template <int PREC>
__global__ void k_dft_tables(DftEntry<PREC>* tab) {
    const int lane = threadIdx.x & 63, which = blockIdx.x;  // which = 2 mode + inverse
    const int mode = which >> 1;
    const bool inv = (which & 1) != 0;
    const int row = lane & 15, g = lane >> 4, part = g >> 1;
    float ar[8], ai[8];
    for (int e = 0; e < 8; ++e) {
        bool on = true;
        int num, den;  // angle 2 pi num / den
        if (mode == 0) {
            num = row * (8 * (g & 1) + e);
            den = 16;
        } else {
            on = (row >> 3) == (g & 1);
            num = (row & 7) * e;
            den = 8;
        }
        double sn, cn;
        sincospi(2.0 * (double)(num % den) / (double)den, &sn, &cn);
        const double fr = cn, fi = inv ? sn : -sn;  // F = exp(-+ 2 pi i num / den)
        // Re Y = Fr Re x - Fi Im x ; Im Y = Fi Re x + Fr Im x
        ar[e] = on ? (float)(part == 0 ? fr : -fi) : 0.f;
        ai[e] = on ? (float)(part == 0 ? fi : fr) : 0.f;
    }
    DftEntry<PREC> d;
    split8<PREC>(ar, d.re_hi, d.re_lo);
    split8<PREC>(ai, d.im_hi, d.im_lo);
    tab[which * 64 + lane] = d;
}


template <int PREC>
__device__ inline const DftEntry<PREC>* a_tab(const ColArgs& a) {
    return reinterpret_cast<const DftEntry<PREC>*>(a.dft_tab);
}

// the six split products of one 16 x 16 x 32 tile: Re and Im outputs
template <int PREC>
__device__ inline void dft_mfma(const DftEntry<PREC>& A, const typename Low<PREC>::T8& bh,
                                const typename Low<PREC>::T8& bl, f32x4& yr, f32x4& yi) {
    using L = Low<PREC>;
    yr = f32x4{0.f, 0.f, 0.f, 0.f};
    yi = f32x4{0.f, 0.f, 0.f, 0.f};
    yr = L::mfma(A.re_hi, bh, yr);
    yr = L::mfma(A.re_hi, bl, yr);
    yr = L::mfma(A.re_lo, bh, yr);
    yi = L::mfma(A.im_hi, bh, yi);
    yi = L::mfma(A.im_hi, bl, yi);
    yi = L::mfma(A.im_lo, bh, yi);
}

// power of two 2^-e with 2^e >= m / target (1 for m == 0): FP16 operand scaling
__device__ inline float pow2_scale(float m, float target) {
    if (!(m > 0.f)) return 1.f;
    int e;
    (void)frexpf(m / target, &e);
    return ldexpf(1.f, -e);
}

}  // namespace mm
