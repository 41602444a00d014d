// kernels_mfma.hip -- the 2D y convolution with its DFT stages on the matrix
// cores (BF16 or FP16 split-precision products, FP32 accumulation).
//
// Per column (one workgroup, the three field components), the length-2048
// transform is factored 2048 = 16 x 16 x 8.  With n = 128 n1 + 8 n2 + n3 and
// k = k1 + 16 k2 + 256 k3 (w = exp(-2 pi i / 2048)):
//   step 1: A1[k1][n2][n3] = sum_n1 x[n] w16^(n1 k1),        times w^((8 n2 + n3) k1)
//   step 2: A2[k1][k2][n3] = sum_n2 A1 w16^(n2 k2),           times w^(16 n3 k2)
//   step 3: X[k]           = sum_n3 A2 w8^(n3 k3)
// Every step is in place in LDS: a step reads the digits it transforms from
// the positions its outputs go to, so the spectrum ends up in digit-reversed
// order, position (k1 16 + k2) 8 + k3.  The inverse runs the steps backwards
// (conjugate matrices and twiddles) and returns natural order, so the K^
// product works on the digit-reversed spectrum.
//
// A DFT step over 16 vectors of 16 points is one 16 x 16 x 32 real GEMM per
// output part: Re Y = [Re F | -Im F] [Re x; Im x], Im Y = [Im F | Re F] [Re x;
// Im x].  The 8-point step takes two vectors per GEMM column with a
// block-diagonal matrix.  Inputs and the DFT matrix are split x = x_hi + x_lo
// in the low precision (hi = round(x), lo = round(x - hi)); the product keeps
// hi hi + hi lo + lo hi with FP32 accumulation.  Twiddles are applied in FP32
// to the GEMM outputs (the inverse applies its twiddles to the outputs of the
// step before, where both parts of a value sit in one lane).  FP16 inputs are
// scaled per column by powers of two so that every value stays in range.
#include <hip/hip_ext.h>

#include "mfma_dft.h"

namespace mm {

// LDS plane addressing: one spare float every 32 (bank spreading)
__device__ inline int pidx(int n) { return n + (n >> 5); }
constexpr int MPL = 2048 + 64;  // floats per plane

struct ColmCfg {
    static constexpr int P = 2048;
    static constexpr int NTH = 512;
    static constexpr int KHP = P / 2 + 1;
    // three components x (re, im) planes, then the K^ rows of the column
    static constexpr size_t LDS = 6 * MPL * sizeof(float) + KHP * sizeof(float4);
};

// One 16-vector tile of a DFT step for component planes (re, im).
// STEP 1 / 2: 16-point DFT over digit n1 / n2 (vectors q / (k1, n3));
// STEP 3: 8-point DFTs over n3 for 32 vectors V = (k1, k2).
// Forward: output twiddles of steps 1, 2.  Inverse: output twiddles of steps
// 3 and 2 (the ones the following inverse step needs), natural output of
// step 1 restricted to n1 < 8 (rows y < 1024).  ZERO_HI: inputs with digit
// n1 >= 8 are zero (zero padding), skip reading them.
template <int PREC, bool INV, int STEP, bool ZERO_HI>
__device__ inline void dft_tile(float* re, float* im, int tile, const DftEntry<PREC>& A, const cf* __restrict__ tw,
                                int twsh, int lane, float scale) {
    const int c = lane & 15, g = lane >> 4, part = g >> 1, half = g & 1;
    const float* src = part ? im : re;
    // output positions and twiddles of this lane's rows 4 g + r of column c;
    // the twiddle loads go out first so their latency overlaps the GEMMs
    constexpr bool TWID = STEP != (INV ? 1 : 3);
    int pos[4];
    cf wv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 4 * g + r;
        int m = 0;  // twiddle exponent of w = exp(-2 pi i / 2048)
        if (STEP == 1) {
            const int q = tile * 16 + c;
            pos[r] = pidx(128 * row + q);
            m = q * row;
        } else if (STEP == 2) {
            const int v = tile * 16 + c, k1 = v >> 3, n3 = v & 7;
            pos[r] = pidx(k1 * 128 + 8 * row + n3);
            // forward: w^(16 n3 k2), k2 = row; inverse (before step 1'): w^-((8 n2 + n3) k1), n2 = row
            m = INV ? (8 * row + n3) * k1 : 16 * n3 * row;
        } else {
            const int p = row >> 3, d = row & 7;
            const int V = tile * 32 + 16 * p + c;
            pos[r] = pidx(V * 8 + d);
            // inverse (before step 2'): w^-(16 n3 k2), n3 = d, k2 = V % 16
            m = 16 * d * (V & 15);
        }
        if (TWID) wv[r] = tw[(m & 2047) << twsh];
    }
    // vector of this lane's column and the address of its digit d
    auto addr = [&](int d) -> int {
        if (STEP == 1) return pidx(128 * d + tile * 16 + c);
        if (STEP == 2) {
            const int v = tile * 16 + c;
            return pidx((v >> 3) * 128 + 8 * d + (v & 7));
        }
        return 0;
    };
    float x[8];
    if (STEP == 3) {
        const int V = tile * 32 + 16 * half + c;
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = Low<PREC>::SCALE ? src[pidx(V * 8 + e)] * scale : src[pidx(V * 8 + e)];
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int d = 8 * half + e;
            const float v = (ZERO_HI && half) ? 0.f : src[addr(d)];
            x[e] = Low<PREC>::SCALE ? v * scale : v;
        }
    }
    typename Low<PREC>::T8 bh, bl;
    split8<PREC>(x, bh, bl);
    using L = Low<PREC>;
    f32x4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
    yr = L::mfma(A.re_hi, bh, yr);
    yr = L::mfma(A.re_hi, bl, yr);
    yr = L::mfma(A.re_lo, bh, yr);
    yi = L::mfma(A.im_hi, bh, yi);
    yi = L::mfma(A.im_hi, bl, yi);
    yi = L::mfma(A.im_lo, bh, yi);
    // lane holds output rows 4 g + r of column c
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float vr = yr[r], vi = yi[r];
        if (TWID) {
            const cf w = INV ? cconj(wv[r]) : wv[r];
            const float tr = vr * w.x - vi * w.y;
            vi = vr * w.y + vi * w.x;
            vr = tr;
        }
        if (INV && STEP == 1 && 4 * g + r >= 8) continue;  // rows y >= 1024 are cropped
        re[pos[r]] = vr;
        im[pos[r]] = vi;
    }
}

// Block-wide maximum of |v| (FP16 scaling), through LDS.
__device__ inline float block_absmax(float v, float* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_max(fabsf(v));
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float m = 0.f;
#pragma unroll
    for (int w = 0; w < ColmCfg::NTH / 64; ++w) m = fmaxf(m, red[w]);
    return m;
}

template <int PREC>
__global__ void __launch_bounds__(ColmCfg::NTH) k_colm(const ColArgs a) {
    constexpr int P = ColmCfg::P, NTH = ColmCfg::NTH, KHP = ColmCfg::KHP;
    extern __shared__ float slds[];
    __shared__ float red[NTH / 64];
    if (a.check_done && a.st->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int col = blk;  // one column per workgroup
    const bool packed = a.pack_col > 0 && col == 0;
    float* plane = slds;  // component k: re at 2k MPL, im at (2k+1) MPL
    const float4* lk = reinterpret_cast<const float4*>(slds + 6 * MPL);
    // ---- load the column (rows y < ny; the rest is zero padding) and K^
    const cf* base = a.spec + (long long)col * a.col_stride;
    const cf* baseN = a.spec + (long long)a.pack_col * a.col_stride;
    // rows y >= P/2 are zero padding (ny <= P/2): each thread loads its rows
    // y = tid + NTH j, j < P/(2 NTH), all loads first
    constexpr int NJ = P / (2 * NTH), NJZ = P / NTH;
    constexpr int NK = (KHP + NTH - 1) / NTH;
    cf v[NJ][3];
    float4 kt[NK];
    {
        const float4* kh = reinterpret_cast<const float4*>(a.khat) + (long long)col * KHP;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int y = tid + NTH * j;
            const bool in = y < a.n_in;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cf x = in ? base[3LL * y + k] : mkc(0.f, 0.f);
                if (packed) x = mkc(x.x, in ? baseN[3LL * y + k].x : 0.f);
                v[j][k] = x;
            }
        }
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const int r = tid + NTH * i;
            kt[i] = r < KHP ? kh[r] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    float amax = 0.f;
#pragma unroll
    for (int j = 0; j < NJZ; ++j) {
        const int y = tid + NTH * j;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const cf x = j < NJ ? v[j < NJ ? j : 0][k] : mkc(0.f, 0.f);
            plane[2 * k * MPL + pidx(y)] = x.x;
            plane[(2 * k + 1) * MPL + pidx(y)] = x.y;
            amax = fmaxf(amax, fmaxf(fabsf(x.x), fabsf(x.y)));
        }
    }
    {
        float4* lkw = reinterpret_cast<float4*>(slds + 6 * MPL);
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const int r = tid + NTH * i;
            if (r < KHP) lkw[r] = kt[i];
        }
    }
    // FP16: inputs scaled so that |x| <= 1/16 (the 2048-point sums stay below 2^7)
    float s_in = 1.f;
    if (Low<PREC>::SCALE) s_in = pow2_scale(block_absmax(amax, red), 1.f / 16);
    __syncthreads();
    const int twshift = a.twshift - 11;  // table exp(-2 pi i m / PT), PT = 2^twshift >= 2048

    // ---- forward transform of the three components
    {
        const DftEntry<PREC> A16 = a_tab<PREC>(a)[0 * 64 + lane], A8 = a_tab<PREC>(a)[2 * 64 + lane];
        // step 1: 8 tiles of 16 vectors per component, the upper 8 inputs are zero
        for (int u = wave; u < 24; u += NTH / 64)
            dft_tile<PREC, false, 1, true>(plane + 2 * (u >> 3) * MPL, plane + (2 * (u >> 3) + 1) * MPL, u & 7, A16,
                                           a.tw, twshift, lane, s_in);
        __syncthreads();
        for (int u = wave; u < 24; u += NTH / 64)
            dft_tile<PREC, false, 2, false>(plane + 2 * (u >> 3) * MPL, plane + (2 * (u >> 3) + 1) * MPL, u & 7, A16,
                                            a.tw, twshift, lane, 1.f);
        __syncthreads();
        for (int u = wave; u < 24; u += NTH / 64)
            dft_tile<PREC, false, 3, false>(plane + 2 * (u >> 3) * MPL, plane + (2 * (u >> 3) + 1) * MPL, u & 7, A8,
                                            a.tw, twshift, lane, 1.f);
        __syncthreads();
    }

    // ---- B^ = K^ M^ on the digit-reversed spectrum, position p <-> k = k1 + 16 k2 + 256 k3
    auto kof = [](int p) {
        const int V = p >> 3;
        return (V >> 4) + 16 * (V & 15) + 256 * (p & 7);
    };
    auto pof = [](int k) { return ((k & 15) * 16 + ((k >> 4) & 15)) * 8 + (k >> 8); };
    auto krow = [&](int k, float& kxx, float& kyy, float& kzz, float& kxy) {
        const bool f = 2 * k > P;
        const float4 k4 = lk[f ? P - k : k];
        kxx = k4.x;
        kyy = k4.y;
        kzz = k4.z;
        kxy = f ? -k4.w : k4.w;
    };
    float bmax = 0.f;
    if (!packed) {
        for (int p = tid; p < P; p += NTH) {
            const int k = kof(p), q = pidx(p);
            float kxx, kyy, kzz, kxy;
            krow(k, kxx, kyy, kzz, kxy);
            const float mxr = plane[q], mxi = plane[MPL + q];
            const float myr = plane[2 * MPL + q], myi = plane[3 * MPL + q];
            const float mzr = plane[4 * MPL + q], mzi = plane[5 * MPL + q];
            const float s = 1.f / s_in;
            const float bxr = s * (kxx * mxr + kxy * myr), bxi = s * (kxx * mxi + kxy * myi);
            const float byr = s * (kxy * mxr + kyy * myr), byi = s * (kxy * mxi + kyy * myi);
            const float bzr = s * kzz * mzr, bzi = s * kzz * mzi;
            plane[q] = bxr;
            plane[MPL + q] = bxi;
            plane[2 * MPL + q] = byr;
            plane[3 * MPL + q] = byi;
            plane[4 * MPL + q] = bzr;
            plane[5 * MPL + q] = bzi;
            bmax = fmaxf(bmax, fmaxf(fmaxf(fabsf(bxr), fabsf(bxi)), fmaxf(fmaxf(fabsf(byr), fabsf(byi)),
                                                                          fmaxf(fabsf(bzr), fabsf(bzi)))));
        }
    } else {
        // Z = A0 + i AN (kx = 0 and kx = px/2, both real along y):
        // B(k) = Kp(k) Z(k) + Km(k) conj Z(-k), Kp = (K0 + KN)/2, Km = (K0 - KN)/2;
        // one thread per pair (k, P - k)
        const float4* khN = reinterpret_cast<const float4*>(a.khat) + (long long)a.pack_col * KHP;
        auto kpm = [&](int k, float (&kp)[4], float (&km)[4]) {
            const bool f = 2 * k > P;
            const int kk = f ? P - k : k;
            float4 k0 = lk[kk], kn = khN[kk];
            if (f) {
                k0.w = -k0.w;
                kn.w = -kn.w;
            }
            const float a0[4] = {k0.x, k0.y, k0.z, k0.w}, an[4] = {kn.x, kn.y, kn.z, kn.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                kp[i] = 0.5f * (a0[i] + an[i]);
                km[i] = 0.5f * (a0[i] - an[i]);
            }
        };
        for (int k = tid; 2 * k <= P; k += NTH) {
            const int kn = (P - k) & (P - 1);
            const int q1 = pidx(pof(k)), q2 = pidx(pof(kn));
            float z1r[3], z1i[3], z2r[3], z2i[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                z1r[c] = plane[2 * c * MPL + q1];
                z1i[c] = plane[(2 * c + 1) * MPL + q1];
                z2r[c] = plane[2 * c * MPL + q2];
                z2i[c] = plane[(2 * c + 1) * MPL + q2];
            }
            float kp1[4], km1[4], kp2[4], km2[4];
            kpm(k, kp1, km1);
            kpm(kn, kp2, km2);
            // B = Kp Z + Km conj(Z'), K = [[xx, xy, 0], [xy, yy, 0], [0, 0, zz]]
            auto apply = [&](const float (&kp)[4], const float (&km)[4], const float (&zr)[3], const float (&zi)[3],
                             const float (&wr)[3], const float (&wi)[3], float (&br)[3], float (&bi)[3]) {
                // conj(W): (wr, -wi)
                br[0] = kp[0] * zr[0] + kp[3] * zr[1] + km[0] * wr[0] + km[3] * wr[1];
                bi[0] = kp[0] * zi[0] + kp[3] * zi[1] - km[0] * wi[0] - km[3] * wi[1];
                br[1] = kp[3] * zr[0] + kp[1] * zr[1] + km[3] * wr[0] + km[1] * wr[1];
                bi[1] = kp[3] * zi[0] + kp[1] * zi[1] - km[3] * wi[0] - km[1] * wi[1];
                br[2] = kp[2] * zr[2] + km[2] * wr[2];
                bi[2] = kp[2] * zi[2] - km[2] * wi[2];
            };
            float b1r[3], b1i[3], b2r[3], b2i[3];
            apply(kp1, km1, z1r, z1i, z2r, z2i, b1r, b1i);
            apply(kp2, km2, z2r, z2i, z1r, z1i, b2r, b2i);
            const float s = 1.f / s_in;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                plane[2 * c * MPL + q1] = s * b1r[c];
                plane[(2 * c + 1) * MPL + q1] = s * b1i[c];
                plane[2 * c * MPL + q2] = s * b2r[c];
                plane[(2 * c + 1) * MPL + q2] = s * b2i[c];
                bmax = fmaxf(bmax, fmaxf(fabsf(s * b1r[c]), fabsf(s * b1i[c])));
                bmax = fmaxf(bmax, fmaxf(fabsf(s * b2r[c]), fabsf(s * b2i[c])));
            }
        }
    }
    float s_out = 1.f;
    if (Low<PREC>::SCALE) s_out = pow2_scale(block_absmax(bmax, red), 1.f / 16);
    __syncthreads();

    // ---- inverse transform (steps 3', 2', 1'), natural order, rows y < 1024
    {
        const DftEntry<PREC> A16 = a_tab<PREC>(a)[1 * 64 + lane], A8 = a_tab<PREC>(a)[3 * 64 + lane];
        for (int u = wave; u < 24; u += NTH / 64)
            dft_tile<PREC, true, 3, false>(plane + 2 * (u >> 3) * MPL, plane + (2 * (u >> 3) + 1) * MPL, u & 7, A8,
                                           a.tw, twshift, lane, s_out);
        __syncthreads();
        for (int u = wave; u < 24; u += NTH / 64)
            dft_tile<PREC, true, 2, false>(plane + 2 * (u >> 3) * MPL, plane + (2 * (u >> 3) + 1) * MPL, u & 7, A16,
                                           a.tw, twshift, lane, 1.f);
        __syncthreads();
        for (int u = wave; u < 24; u += NTH / 64)
            dft_tile<PREC, true, 1, false>(plane + 2 * (u >> 3) * MPL, plane + (2 * (u >> 3) + 1) * MPL, u & 7, A16,
                                           a.tw, twshift, lane, 1.f);
        __syncthreads();
    }

    // ---- store rows y < ny
    cf* out = a.spec + (long long)col * a.col_stride;
    cf* outN = a.spec + (long long)a.pack_col * a.col_stride;
    const float inv = 1.f / s_out;
    for (int y = tid; y < a.n_out; y += NTH) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float vr = inv * plane[2 * k * MPL + pidx(y)], vi = inv * plane[(2 * k + 1) * MPL + pidx(y)];
            if (!packed) {
                out[3LL * y + k] = mkc(vr, vi);
            } else {
                out[3LL * y + k] = mkc(vr, 0.f);
                outN[3LL * y + k] = mkc(vi, 0.f);
            }
        }
    }
}

hipError_t launch_colm(int p, int prec, const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (p != ColmCfg::P) return hipErrorInvalidValue;
    const int nb = a.ncol;
    ColArgs b = a;
    if (prec == MM_PREC_FP16) b.dft_tab = reinterpret_cast<const char*>(a.dft_tab) + DFT_TABLE_BYTES;
    if (prec == MM_PREC_BF16)
        hipExtLaunchKernelGGL((k_colm<MM_PREC_BF16>), dim3(nb), dim3(ColmCfg::NTH), (uint32_t)ColmCfg::LDS, s, e0, e1,
                              0, b);
    else if (prec == MM_PREC_FP16)
        hipExtLaunchKernelGGL((k_colm<MM_PREC_FP16>), dim3(nb), dim3(ColmCfg::NTH), (uint32_t)ColmCfg::LDS, s, e0, e1,
                              0, b);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// The DFT tables of both precisions (DFT_TABLE_BYTES each, BF16 first).
hipError_t launch_dft_tables(void* tab, hipStream_t s) {
    hipLaunchKernelGGL(k_dft_tables<MM_PREC_BF16>, dim3(4), dim3(64), 0, s,
                       reinterpret_cast<DftEntry<MM_PREC_BF16>*>(tab));
    hipLaunchKernelGGL(k_dft_tables<MM_PREC_FP16>, dim3(4), dim3(64), 0, s,
                       reinterpret_cast<DftEntry<MM_PREC_FP16>*>(reinterpret_cast<char*>(tab) + DFT_TABLE_BYTES));
    return hipGetLastError();
}

hipError_t configure_colm(void) {
    hipError_t e = hipFuncSetAttribute((const void*)k_colm<MM_PREC_BF16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)ColmCfg::LDS);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_colm<MM_PREC_FP16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)ColmCfg::LDS);
    return e;
}

}  // namespace mm
