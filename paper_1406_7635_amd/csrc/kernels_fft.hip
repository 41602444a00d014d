// kernels_fft.hip -- the FP32 magnetostatic convolution passes.
//
// Section "Magnetostatic field": B_demag = K * M evaluated with the
// convolution theorem on a grid zero-padded to px x py x pz.  The passes:
//   x-forward  : per pair of x-rows, stage combine m_s = m0 + dt sum a k,
//                M = Msat[region] m_s, zero padding in LDS, real-to-complex
//                FFT along x (two real rows packed per complex transform),
//                written as 3 interleaved complex components per (row, kx);
//   column     : FFT along y (and z) of T adjacent kx columns; in the last
//                axis the pointwise B^ = K^ M^ (K^ real symmetric, stored as
//                one octant with mirror signs) and the inverse transform;
//   x-inverse  : complex-to-real along x (two real rows per transform), crop
//                to the physical cells, then the per-cell epilogue (exchange,
//                anisotropy, Zeeman, torque, error norm, energies).
// The 1/(px py pz) normalisation and -mu0 are folded into K^.
#include <algorithm>

#include "field_epilogue.h"

namespace mm {

// rows of the x passes per workgroup: H rows = 3H/2 complex transforms
constexpr int rows_per_wg(int P) { return P >= 2048 ? 2 : (P >= 256 ? 4096 / P : 16); }
// adjacent kx columns per workgroup in the column passes
constexpr int cols_per_wg(int P) { return P >= 2048 ? 1 : (P >= 128 ? 2048 / P : 16); }

__device__ inline long long row_offset(const FieldArgs& a, int row) {
    const int z = row / a.ny, y = row - z * a.ny;
    return (long long)z * a.zstride + (long long)y * a.rowstride;
}

// ---------------------------------------------------------------------------
template <int P, int H>
__global__ void __launch_bounds__(NT) k_xfwd(const FieldArgs a) {
    constexpr int F = 3 * H / 2;
    constexpr int SEQ = seq_len(P);
    constexpr int KX = P / 2 + 1;
    extern __shared__ cf lds[];
    if ((a.flags & EPI_CHECK_DONE) && a.st->done) return;
    const int tid = threadIdx.x;
    const int row0 = xcd_remap(blockIdx.x, gridDim.x) * H;
    const float dt = (float)a.st->dt;
    const bool write_ms = a.sd.nk > 0;

    // load, combine, scale by Msat; pack rows (a, b) as Mx_a + i My_a,
    // Mx_b + i My_b and Mz_a + i Mz_b
    for (int idx = tid; idx < H * P; idx += NT) {
        const int rr = idx / P, x = idx - rr * P;
        const int row = row0 + rr;
        float3 M = make_float3(0.f, 0.f, 0.f);
        if (x < a.nx && row < a.nrows) {
            const long long cell = (long long)row * a.nx + x;
            const float3 m = stage_state(a, cell, dt);
            if (write_ms) st3(a.ms, a.ncell, cell, m);
            M = f3scale(a.lut[a.region[cell]].a.x, m);
        }
        const int p = rr >> 1;
        cf* s01 = lds + (3 * p + (rr & 1)) * SEQ;
        cf* s2 = lds + (3 * p + 2) * SEQ;
        const int px = lds_pad(x);
        s01[px] = mkc(M.x, M.y);
        if (rr & 1)
            s2[px].y = M.z;
        else
            s2[px].x = M.z;
    }
    __syncthreads();
    Fft<P, 1, F, NT, false>::run(lds, a.tw, a.twshift, tid);

    // unpack the half spectra: X = (Z[k] + conj Z[P-k])/2, Y = (Z[k] - conj Z[P-k])/(2i)
    for (int idx = tid; idx < (H / 2) * KX; idx += NT) {
        const int p = idx / KX, k = idx - p * KX;
        const int kn = (P - k) & (P - 1);
        const int ra = row0 + 2 * p, rb = ra + 1;
        const cf* s0 = lds + (3 * p) * SEQ;
        cf X[3], Y[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const cf z = s0[s * SEQ + lds_pad(k)];
            const cf w = cconj(s0[s * SEQ + lds_pad(kn)]);
            const cf d = z - w;
            X[s] = 0.5f * (z + w);
            Y[s] = mkc(0.5f * d.y, -0.5f * d.x);
        }
        // slot 0 -> row a (x, y), slot 1 -> row b (x, y), slot 2 -> (z of a, z of b)
        if (ra < a.nrows) {
            cf* d = a.spec + row_offset(a, ra) + 3LL * k;
            d[0] = X[0];
            d[1] = Y[0];
            d[2] = X[2];
        }
        if (rb < a.nrows) {
            cf* d = a.spec + row_offset(a, rb) + 3LL * k;
            d[0] = X[1];
            d[1] = Y[1];
            d[2] = Y[2];
        }
    }
}

// ---------------------------------------------------------------------------
template <int P, int T, int MODE, int NC>
__global__ void __launch_bounds__(NT) k_col(const ColArgs a) {
    constexpr int F = 3 * T;
    constexpr int SEQ = seq_len(P);
    constexpr int W = 3 * T;
    extern __shared__ cf lds[];
    if (a.check_done && a.st->done) return;
    const int tid = threadIdx.x;
    const int ntile = (a.ncolx + T - 1) / T;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int o = blk / ntile, tile = blk - o * ntile;
    const int kx0 = tile * T;
    const int wv = 3 * min(T, a.ncolx - kx0);
    cf* base = a.spec + (long long)o * a.outer_stride + 3LL * kx0;

    for (int idx = tid; idx < P * W; idx += NT) {
        const int q = idx / W, tc = idx - q * W;
        cf v = mkc(0.f, 0.f);
        if (q < a.n_in && tc < wv) v = base[(long long)q * a.stride + tc];
        lds[tc * SEQ + lds_pad(q)] = v;
    }
    __syncthreads();
    if (MODE == COL_INV)
        Fft<P, 1, F, NT, true>::run(lds, a.tw, a.twshift, tid);
    else
        Fft<P, 1, F, NT, false>::run(lds, a.tw, a.twshift, tid);

    if (MODE == COL_CONV) {
        // outer index o is ky in 3D (parity of xy, yz in y), 0 in 2D
        int ah = o;
        bool fa = false;
        if (a.pa > 1 && 2 * o > a.pa) {
            ah = a.pa - o;
            fa = true;
        }
        for (int idx = tid; idx < P * T; idx += NT) {
            const int t = idx / P, q = idx - t * P;
            if (3 * t >= wv) continue;
            int qh = q;
            bool fq = false;
            if (2 * q > P) {
                qh = P - q;
                fq = true;
            }
            const float* K = a.khat + (((long long)ah * a.ncolx + kx0 + t) * a.khq + qh) * NC;
            const float kxx = K[0], kyy = K[1], kzz = K[2];
            float kxy = K[3], kxz = 0.f, kyz = 0.f;
            if (NC == 6) {
                kxz = K[4];
                kyz = K[5];
                if (fq) {  // conv axis z: xz and yz are odd in z
                    kxz = -kxz;
                    kyz = -kyz;
                }
                if (fa) {  // outer axis y: xy and yz are odd in y
                    kxy = -kxy;
                    kyz = -kyz;
                }
            } else if (fq) {  // conv axis y: xy is odd in y
                kxy = -kxy;
            }
            cf* sx = lds + (3 * t) * SEQ + lds_pad(q);
            cf* sy = sx + SEQ;
            cf* sz = sy + SEQ;
            const cf mx = *sx, my = *sy, mz = *sz;
            *sx = kxx * mx + kxy * my + kxz * mz;
            *sy = kxy * mx + kyy * my + kyz * mz;
            *sz = kxz * mx + kyz * my + kzz * mz;
        }
        __syncthreads();
        Fft<P, 1, F, NT, true>::run(lds, a.tw, a.twshift, tid);
    }

    for (int idx = tid; idx < a.n_out * W; idx += NT) {
        const int q = idx / W, tc = idx - q * W;
        if (tc < wv) base[(long long)q * a.stride + tc] = lds[tc * SEQ + lds_pad(q)];
    }
}

// ---------------------------------------------------------------------------
template <int P, int H>
__global__ void __launch_bounds__(NT) k_xinv(const FieldArgs a) {
    constexpr int F = 3 * H / 2;
    constexpr int SEQ = seq_len(P);
    constexpr int KX = P / 2 + 1;
    extern __shared__ cf lds[];
    __shared__ double red[(NT / 64) * 6];
    if ((a.flags & EPI_CHECK_DONE) && a.st->done) return;
    const int tid = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int row0 = blk * H;

    // Hermitian extension: slot[k] = X[k] + i Y[k], slot[P-k] = conj X[k] + i conj Y[k]
    for (int idx = tid; idx < (H / 2) * KX; idx += NT) {
        const int p = idx / KX, k = idx - p * KX;
        const int ra = row0 + 2 * p, rb = ra + 1;
        cf A[3] = {mkc(0.f, 0.f), mkc(0.f, 0.f), mkc(0.f, 0.f)};
        cf B[3] = {mkc(0.f, 0.f), mkc(0.f, 0.f), mkc(0.f, 0.f)};
        if (ra < a.nrows) {
            const cf* s = a.spec + row_offset(a, ra) + 3LL * k;
            A[0] = s[0];
            A[1] = s[1];
            A[2] = s[2];
        }
        if (rb < a.nrows) {
            const cf* s = a.spec + row_offset(a, rb) + 3LL * k;
            B[0] = s[0];
            B[1] = s[1];
            B[2] = s[2];
        }
        const bool edge = (k == 0) || (2 * k == P);
        if (edge) {  // DC and Nyquist bins of a real signal are real
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                A[s].y = 0.f;
                B[s].y = 0.f;
            }
        }
        cf* s0 = lds + (3 * p) * SEQ;
        const cf u[3] = {A[0], B[0], A[2]};
        const cf v[3] = {A[1], B[1], B[2]};
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            s0[s * SEQ + lds_pad(k)] = mkc(u[s].x - v[s].y, u[s].y + v[s].x);
            if (!edge) s0[s * SEQ + lds_pad(P - k)] = mkc(u[s].x + v[s].y, v[s].x - u[s].y);
        }
    }
    __syncthreads();
    Fft<P, 1, F, NT, true>::run(lds, a.tw, a.twshift, tid);

    EpiAcc acc;
    epi_init(acc);
    const float* mp = a.sd.nk > 0 ? a.ms : a.m0;
    for (int idx = tid; idx < H * a.nx; idx += NT) {
        const int rr = idx / a.nx, x = idx - rr * a.nx;
        const int row = row0 + rr;
        if (row >= a.nrows) continue;
        const cf* s0 = lds + (3 * (rr >> 1)) * SEQ;
        const cf v = s0[(rr & 1) * SEQ + lds_pad(x)];
        const cf w = s0[2 * SEQ + lds_pad(x)];
        const float3 bd = make_float3(v.x, v.y, (rr & 1) ? w.y : w.x);
        const int z = row / a.ny, y = row - z * a.ny;
        epilogue(a, mp, (long long)row * a.nx + x, x, y, z, bd, acc);
    }
    if (a.flags & (EPI_ERR | EPI_MAXTQ | EPI_ENERGY)) epi_reduce(a, acc, red, blk);
}

// ---------------------------------------------------------------------------
// Launch helpers: dispatch the run-time padded length to a template instance.

template <int P>
static hipError_t xfwd_p(const FieldArgs& a, hipStream_t s) {
    constexpr int H = rows_per_wg(P);
    const size_t lds = (size_t)(3 * H / 2) * seq_len(P) * sizeof(cf);
    const int nb = (a.nrows + H - 1) / H;
    hipFuncSetAttribute((const void*)k_xfwd<P, H>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_xfwd<P, H>), dim3(nb), dim3(NT), lds, s, a);
    return hipGetLastError();
}

template <int P>
static hipError_t xinv_p(const FieldArgs& a, hipStream_t s, int* nb_out) {
    constexpr int H = rows_per_wg(P);
    const size_t lds = (size_t)(3 * H / 2) * seq_len(P) * sizeof(cf);
    const int nb = (a.nrows + H - 1) / H;
    if (nb_out) *nb_out = nb;
    hipFuncSetAttribute((const void*)k_xinv<P, H>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_xinv<P, H>), dim3(nb), dim3(NT), lds, s, a);
    return hipGetLastError();
}

template <int P, int MODE, int NC>
static hipError_t col_p(const ColArgs& a, hipStream_t s) {
    constexpr int T = cols_per_wg(P);
    const size_t lds = (size_t)(3 * T) * seq_len(P) * sizeof(cf);
    const int ntile = (a.ncolx + T - 1) / T;
    const long long nb = (long long)ntile * a.nouter;
    hipFuncSetAttribute((const void*)k_col<P, T, MODE, NC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    hipLaunchKernelGGL((k_col<P, T, MODE, NC>), dim3((unsigned)nb), dim3(NT), lds, s, a);
    return hipGetLastError();
}

int xinv_blocks(int px, int nrows) {
    int H = 16;
    if (px >= 2048) H = 2;
    else if (px >= 256) H = 4096 / px;
    return (nrows + H - 1) / H;
}

#define MM_CASES(M)                                                                        \
    M(1) M(2) M(4) M(8) M(16) M(32) M(64) M(128) M(256) M(512) M(1024) M(2048) M(4096)

hipError_t launch_xfwd(int px, const FieldArgs& a, hipStream_t s) {
    switch (px) {
#define M(p) \
    case p:  \
        return xfwd_p<p>(a, s);
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_xinv(int px, const FieldArgs& a, hipStream_t s, int* nb_out) {
    switch (px) {
#define M(p) \
    case p:  \
        return xinv_p<p>(a, s, nb_out);
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_col(int p, int mode, const ColArgs& a, int ncomp, hipStream_t s) {
    if (mode == COL_FWD) {
        switch (p) {
#define M(q) \
    case q:  \
        return col_p<q, COL_FWD, 4>(a, s);
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
        return col_p<q, COL_INV, 4>(a, s);
            MM_CASES(M)
#undef M
            default:
                return hipErrorInvalidValue;
        }
    }
    if (ncomp == 4) {
        switch (p) {
#define M(q) \
    case q:  \
        return col_p<q, COL_CONV, 4>(a, s);
            MM_CASES(M)
#undef M
            default:
                return hipErrorInvalidValue;
        }
    }
    switch (p) {
#define M(q) \
    case q:  \
        return col_p<q, COL_CONV, 6>(a, s);
        MM_CASES(M)
#undef M
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace mm
