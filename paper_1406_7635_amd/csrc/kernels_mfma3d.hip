// kernels_mfma3d.hip -- the column passes of 3D grids (y forward, z
// convolution with K^, y inverse) with their DFT stages on the matrix cores
// (BF16 or FP16 split-precision products, FP32 accumulation).
//
// A workgroup holds G columns of the pass (three field components each, so
// 3 G sequences of length P) as separate real / imaginary planes in LDS and
// runs the transform as steps of R-point DFTs, R = 16 or 8, in place:
// step l works inside blocks of B_l points (B_1 = P, B_{l+1} = B_l / R_l) on
// the vectors (block b, offset r < S_l = B_l / R_l) with points
// b B_l + d S_l + r, d < R_l.  Forward (decimation in frequency): the DFT
// over d, then the twiddle exp(-2 pi i r k / B_l) on output k; the spectrum
// ends digit-reversed (position p holds k = sum_l k_l R_1 ... R_(l-1), with
// k_l the digit of p at stride S_l).  The inverse runs the steps backwards
// with conjugate matrices and returns natural order; the conjugate twiddle
// of step l is applied to the outputs of inverse step l + 1 (those are the
// inputs of step l, and both parts of a value sit in one lane there).
// Twiddles are FP32 from the context's table exp(-2 pi i m / PT).
//
// A tile is 16 GEMM columns: 16 vectors for R = 16, 32 for R = 8 (two
// vectors per column, block-diagonal matrix), the vectors numbered over all
// sequences of the workgroup.  FP16 operands are scaled by a power of two
// per workgroup (inputs to |x| <= 1/16, so the P-point sums stay in range).
#include <hip/hip_ext.h>

#include "mfma_dft.h"

namespace mm {

// LDS plane index: one spare float every 32
__device__ inline int ppos(int n) { return n + (n >> 5); }

// factorisation of P into steps of 16 and 8 (at most 3 steps)
template <int P>
struct Fac {
    static constexpr int NS = P == 64 ? 2 : P == 128 ? 2 : P == 256 ? 2 : P == 512 ? 3 : P == 1024 ? 3 : 0;
    static constexpr int R(int l) {
        return P == 64 ? 8 : P == 128 ? (l == 0 ? 16 : 8) : P == 256 ? 16 : P == 512 ? 8 : (l == 0 ? 16 : 8);
    }
    static constexpr int B(int l) { return l == 0 ? P : B(l - 1) / R(l - 1); }
    static constexpr int S(int l) { return B(l) / R(l); }
    static constexpr int PL = P + P / 32;  // floats per plane
};

template <int P>
struct M3Cfg {
    static constexpr int G = 2048 / P;           // columns per workgroup
    static constexpr int NSEQ = 3 * G;           // sequences (component planes pairs)
    static constexpr int NTH = 256;
    static constexpr int TILES = NSEQ * P / 256;  // GEMM tiles per step
    static constexpr size_t LDS = (size_t)NSEQ * 2 * Fac<P>::PL * sizeof(float);
};

template <int P, int NTH>
__device__ inline float block_absmax3(float v, float* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_max(fabsf(v));
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float m = 0.f;
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w) m = fmaxf(m, red[w]);
    return m;
}

// exponent e (of exp(-+2 pi i e / B_l)) of the twiddle of step l at position p
template <int P>
__device__ inline int tw_exp(int l, int p) {
    using F = Fac<P>;
    int B = P, S = P / F::R(0);
#pragma unroll
    for (int j = 0; j < 3; ++j)
        if (j < l) {
            B = B / F::R(j);
            S = B / F::R(j + 1 < F::NS ? j + 1 : j);
        }
    const int rem = p & (B - 1);
    const int d = rem / S, r = rem & (S - 1);
    return (r * d) & (B - 1);
}

// One step (index l) over all tiles of the workgroup.  INV: conjugate
// matrix; the twiddle applied to the outputs is the forward one of step l
// (forward), or the conjugate one of step l - 1 (inverse, none after step 0).
template <int P, int PREC, bool INV>
__device__ inline void mstep(int l, float* planes, const DftEntry<PREC>& A16, const DftEntry<PREC>& A8,
                             const cf* __restrict__ tw, int twshift, int wave, int lane, float scale) {
    using F = Fac<P>;
    constexpr int PL = F::PL, NW = M3Cfg<P>::NTH / 64;
    const int R = F::R(l), B = F::B(l), S = F::S(l);
    const int NV = P / R;  // vectors per sequence
    const int c = lane & 15, g = lane >> 4, part = g >> 1, half = g & 1;
    const bool r16 = R == 16;
    const DftEntry<PREC>& A = r16 ? A16 : A8;
    // twiddle of the outputs: forward step l (none for the last), inverse step l - 1
    const int tl = INV ? l - 1 : l;
    const bool twid = INV ? l > 0 : l + 1 < F::NS;
    int tB = P;
#pragma unroll
    for (int j = 0; j < 3; ++j)
        if (j < tl) tB /= F::R(j);
    const int tsh = twshift - ilog2_rt(tB);  // table stride of the twiddles of step tl
    for (int u = wave; u < M3Cfg<P>::TILES; u += NW) {
        // the lane's input vector and its points
        const int V = r16 ? u * 16 + c : u * 32 + 16 * half + c;
        const int seq = V / NV, v = V - seq * NV;
        const int b = v / S, r = v - b * S;
        const int base = b * B + r;
        const float* src = planes + (2 * seq + part) * PL;
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int d = r16 ? 8 * half + e : e;
            const float val = src[ppos(base + d * S)];
            x[e] = Low<PREC>::SCALE ? val * scale : val;
        }
        typename Low<PREC>::T8 bh, bl;
        split8<PREC>(x, bh, bl);
        f32x4 yr, yi;
        dft_mfma<PREC>(A, bh, bl, yr, yi);
        // outputs: rows 4 g + q of column c -> (vector, digit)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 4 * g + q;
            const int Vo = r16 ? u * 16 + c : u * 32 + 16 * (row >> 3) + c;
            const int k = r16 ? row : (row & 7);
            const int so = Vo / NV, vo = Vo - so * NV;
            const int bo = vo / S, ro = vo - bo * S;
            const int p = bo * B + k * S + ro;
            float vr = yr[q], vi = yi[q];
            if (twid) {
                const int m = INV ? tw_exp<P>(tl, p) : (ro * k) & (B - 1);
                cf w = tw[m << tsh];
                if (INV) w = cconj(w);
                const float tr = vr * w.x - vi * w.y;
                vi = vr * w.y + vi * w.x;
                vr = tr;
            }
            float* dst = planes + 2 * so * PL;
            dst[ppos(p)] = vr;
            dst[PL + ppos(p)] = vi;
        }
    }
}

// frequency index of digit-reversed position p
template <int P>
__device__ inline int freq_of(int p) {
    using F = Fac<P>;
    int k = 0, mul = 1;
#pragma unroll
    for (int l = 0; l < 3; ++l)
        if (l < F::NS) {
            const int d = (p / F::S(l)) % F::R(l);
            k += d * mul;
            mul *= F::R(l);
        }
    return k;
}

// position of natural frequency k in the digit-reversed order
template <int P>
__device__ inline int pos_of(int k) {
    using F = Fac<P>;
    int p = 0, rest = k;
#pragma unroll
    for (int l = 0; l < 3; ++l)
        if (l < F::NS) {
            const int d = rest % F::R(l);
            rest /= F::R(l);
            p += d * F::S(l);
        }
    return p;
}

// MODE: COL_FWD (inputs q < n_in, all P outputs), COL_INV (P inputs, outputs
// q < n_out), COL_CONV (the 3D z convolution: forward, K^, inverse).
template <int P, int MODE, int PREC>
__global__ void __launch_bounds__(256) k_colm3d(const ColArgs a) {
    using F = Fac<P>;
    using C = M3Cfg<P>;
    constexpr int G = C::G, NSEQ = C::NSEQ, NTH = C::NTH, PL = F::PL;
    extern __shared__ float planes[];
    __shared__ float red[NTH / 64];
    if (a.check_done && a.st->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ntile = (a.ncol + G - 1) / G;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int o = blk / ntile, c0 = (blk - o * ntile) * G;
    cf* sbase = a.spec + (long long)o * a.outer_stride;
    const int nin = MODE == COL_INV ? P : a.n_in;
    // ---- load: element (column g, position q, component k); zero padding above nin
    float amax = 0.f;
    for (int i = tid; i < G * P * 3; i += NTH) {
        int g, q, k;
        if (MODE == COL_CONV) {  // adjacent columns are adjacent in memory: (q, g, k)
            q = i / (3 * G);
            const int rem = i - q * 3 * G;
            g = rem / 3;
            k = rem - 3 * g;
        } else {  // positions of one column are adjacent: (g, q, k)
            g = i / (3 * P);
            const int rem = i - g * 3 * P;
            q = rem / 3;
            k = rem - 3 * q;
        }
        const int col = c0 + g;
        cf x = mkc(0.f, 0.f);
        if (col < a.ncol && q < nin) x = sbase[(long long)col * a.col_stride + (long long)q * a.pos_stride + k];
        // the inverse pass takes a natural-order spectrum into the digit-reversed
        // positions its steps expect
        const int pq = ppos(MODE == COL_INV ? pos_of<P>(q) : q);
        float* pl = planes + 2 * (3 * g + k) * PL;
        pl[pq] = x.x;
        pl[PL + pq] = x.y;
        amax = fmaxf(amax, fmaxf(fabsf(x.x), fabsf(x.y)));
    }
    float s_in = 1.f;
    if (Low<PREC>::SCALE) s_in = pow2_scale(block_absmax3<P, NTH>(amax, red), 1.f / 16);
    __syncthreads();
    const DftEntry<PREC>* tab = a_tab<PREC>(a);
    float out_scale = 1.f / s_in;  // undoes the input scaling at the store
    if (MODE != COL_INV) {
        const DftEntry<PREC> A16 = tab[0 * 64 + lane], A8 = tab[2 * 64 + lane];
#pragma unroll
        for (int l = 0; l < F::NS; ++l) {
            mstep<P, PREC, false>(l, planes, A16, A8, a.tw, a.twshift, wave, lane, l == 0 ? s_in : 1.f);
            __syncthreads();
        }
    }
    if (MODE == COL_CONV) {
        // B^ = K^ M^ on the digit-reversed spectrum; column c0 + g is ky, the
        // transform axis is z; K^[kx][ky_h][kz_h][xx, yy, zz, xy, xz, yz], xy odd
        // in y, xz odd in z, yz odd in both
        float bmax = 0.f;
        const float inv_in = 1.f / s_in;
        for (int i = tid; i < G * P; i += NTH) {
            const int g = i / P, p = i - g * P;
            const int ky = c0 + g;
            if (ky >= a.ncol) continue;
            const int kz = freq_of<P>(p);
            const bool fa = 2 * ky > a.pa, fq = 2 * kz > P;
            const int kyh = fa ? a.pa - ky : ky, kzh = fq ? P - kz : kz;
            const float* K = a.khat + (((long long)o * a.kyh + kyh) * a.kzh + kzh) * 6;
            const float kxx = K[0], kyy = K[1], kzz = K[2];
            const float kxy = fa ? -K[3] : K[3];
            const float kxz = fq ? -K[4] : K[4];
            const float kyz = (fa != fq) ? -K[5] : K[5];
            float* p0 = planes + 2 * (3 * g) * PL;
            float* p1 = p0 + 2 * PL;
            float* p2 = p1 + 2 * PL;
            const int q = ppos(p);
            const float m0r = p0[q], m0i = p0[PL + q], m1r = p1[q], m1i = p1[PL + q], m2r = p2[q], m2i = p2[PL + q];
            const float b0r = inv_in * (kxx * m0r + kxy * m1r + kxz * m2r);
            const float b0i = inv_in * (kxx * m0i + kxy * m1i + kxz * m2i);
            const float b1r = inv_in * (kxy * m0r + kyy * m1r + kyz * m2r);
            const float b1i = inv_in * (kxy * m0i + kyy * m1i + kyz * m2i);
            const float b2r = inv_in * (kxz * m0r + kyz * m1r + kzz * m2r);
            const float b2i = inv_in * (kxz * m0i + kyz * m1i + kzz * m2i);
            p0[q] = b0r;
            p0[PL + q] = b0i;
            p1[q] = b1r;
            p1[PL + q] = b1i;
            p2[q] = b2r;
            p2[PL + q] = b2i;
            bmax = fmaxf(bmax, fmaxf(fmaxf(fmaxf(fabsf(b0r), fabsf(b0i)), fmaxf(fabsf(b1r), fabsf(b1i))),
                                     fmaxf(fabsf(b2r), fabsf(b2i))));
        }
        float s_mid = 1.f;
        if (Low<PREC>::SCALE) s_mid = pow2_scale(block_absmax3<P, NTH>(bmax, red), 1.f / 16);
        __syncthreads();
        s_in = s_mid;
        out_scale = 1.f / s_mid;
    }
    if (MODE != COL_FWD) {
        const DftEntry<PREC> A16 = tab[1 * 64 + lane], A8 = tab[3 * 64 + lane];
#pragma unroll
        for (int l = F::NS - 1; l >= 0; --l) {
            mstep<P, PREC, true>(l, planes, A16, A8, a.tw, a.twshift, wave, lane, l == F::NS - 1 ? s_in : 1.f);
            __syncthreads();
        }
    }
    // ---- store (same element order as the load)
    const int nout = MODE == COL_FWD ? P : a.n_out;
    for (int i = tid; i < G * P * 3; i += NTH) {
        int g, q, k;
        if (MODE == COL_CONV) {
            q = i / (3 * G);
            const int rem = i - q * 3 * G;
            g = rem / 3;
            k = rem - 3 * g;
        } else {
            g = i / (3 * P);
            const int rem = i - g * 3 * P;
            q = rem / 3;
            k = rem - 3 * q;
        }
        const int col = c0 + g;
        if (col >= a.ncol || q >= nout) continue;
        const float* pl = planes + 2 * (3 * g + k) * PL;
        // the forward pass leaves digit-reversed positions: natural order out
        const int pq = ppos(MODE == COL_FWD ? pos_of<P>(q) : q);
        const float vr = pl[pq], vi = pl[PL + pq];
        sbase[(long long)col * a.col_stride + (long long)q * a.pos_stride + k] = mkc(out_scale * vr, out_scale * vi);
    }
}

template <int P>
static hipError_t colm3d_p(int mode, int prec, const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const long long nb = (long long)((a.ncol + M3Cfg<P>::G - 1) / M3Cfg<P>::G) * a.nouter;
    const size_t lds = M3Cfg<P>::LDS;
    const dim3 grid((unsigned)nb), blk(M3Cfg<P>::NTH);
#define MM_M3(MD, PR)                                                                                        \
    if (mode == MD && prec == PR) {                                                                          \
        hipExtLaunchKernelGGL((k_colm3d<P, MD, PR>), grid, blk, (uint32_t)lds, s, e0, e1, 0, a);             \
        return hipGetLastError();                                                                            \
    }
    MM_M3(COL_FWD, MM_PREC_BF16)
    MM_M3(COL_INV, MM_PREC_BF16)
    MM_M3(COL_CONV, MM_PREC_BF16)
    MM_M3(COL_FWD, MM_PREC_FP16)
    MM_M3(COL_INV, MM_PREC_FP16)
    MM_M3(COL_CONV, MM_PREC_FP16)
#undef MM_M3
    return hipErrorInvalidValue;
}

bool colm3d_supported(int p) { return p == 64 || p == 128 || p == 256 || p == 512 || p == 1024; }

hipError_t launch_colm3d(int p, int mode, int prec, const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    ColArgs b = a;
    if (prec == MM_PREC_FP16) b.dft_tab = reinterpret_cast<const char*>(a.dft_tab) + DFT_TABLE_BYTES;
    switch (p) {
        case 64: return colm3d_p<64>(mode, prec, b, s, e0, e1);
        case 128: return colm3d_p<128>(mode, prec, b, s, e0, e1);
        case 256: return colm3d_p<256>(mode, prec, b, s, e0, e1);
        case 512: return colm3d_p<512>(mode, prec, b, s, e0, e1);
        case 1024: return colm3d_p<1024>(mode, prec, b, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t allow3(void) {
    const int lds = (int)M3Cfg<P>::LDS;
    const void* fs[6] = {(const void*)k_colm3d<P, COL_FWD, MM_PREC_BF16>, (const void*)k_colm3d<P, COL_INV, MM_PREC_BF16>,
                         (const void*)k_colm3d<P, COL_CONV, MM_PREC_BF16>, (const void*)k_colm3d<P, COL_FWD, MM_PREC_FP16>,
                         (const void*)k_colm3d<P, COL_INV, MM_PREC_FP16>, (const void*)k_colm3d<P, COL_CONV, MM_PREC_FP16>};
    for (const void* f : fs) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t configure_colm3d(void) {
    hipError_t e = allow3<64>();
    if (e == hipSuccess) e = allow3<128>();
    if (e == hipSuccess) e = allow3<256>();
    if (e == hipSuccess) e = allow3<512>();
    if (e == hipSuccess) e = allow3<1024>();
    return e;
}

}  // namespace mm
