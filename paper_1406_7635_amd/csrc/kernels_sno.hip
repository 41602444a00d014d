// kernels_sno.hip -- forward pass of the spectral neural operator that can
// stand in for the magnetostatic convolution at the inner Runge-Kutta stages.
//
// The network (32 channels, kept modes kx = 0..15, ky = -8..7, four layers):
//   lift      h_c = sum_j P[c][j] m_j + p[c]
//   layer     hhat_c(k) = sum_{x,y} h_c(x, y) exp(-2 pi i (kx x/nx + ky y/ny))
//             ghat_o(k) = sum_c R[ky + 8][kx][o][c] hhat_c(k)
//             g_o = Re sum_k w_kx ghat_o(k) exp(+2 pi i (...)) / (nx ny), w_0 = 1, else 2
//             h_o <- GELU(g_o + sum_c W[o][c] h_c + b[o])   (exact erf form)
//   project   B_j = scale (sum_c Q[j][c] h_c + q[j])
// Weights are stored as BF16 and widened to FP32; all arithmetic and
// accumulation is FP32.  Activations are FP32 [32][ny][nx].
//
// Per layer: x transform of every row (kept kx only) -> y transform of every
// kept column -> mode mixing -> inverse y transform -> inverse x transform
// fused with the pointwise branch and GELU.
#include <hip/hip_runtime.h>

#include "sno_internal.h"

namespace mm {

namespace {

__device__ inline float bf16f(uint16_t v) { return __uint_as_float((unsigned int)v << 16); }

// exp(-2 pi i m / n), m < n, evaluated in FP64 and rounded once
__global__ void k_sno_twiddles(float2* tw, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) {
        double s, c;
        sincospi(-2.0 * (double)m / (double)n, &s, &c);
        tw[m] = make_float2((float)c, (float)s);
    }
}

__global__ void __launch_bounds__(256) k_sno_lift(const SnoArgs a, const float* __restrict__ m, float* __restrict__ h) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n) return;
    const float m0 = m[p], m1 = m[a.n + p], m2 = m[2 * a.n + p];
#pragma unroll 4
    for (int c = 0; c < SNO_C; ++c) {
        const uint16_t* P = a.lift + 3 * c;
        h[(long long)c * a.n + p] = bf16f(P[0]) * m0 + bf16f(P[1]) * m1 + bf16f(P[2]) * m2 + bf16f(a.lift_b[c]);
    }
}

// H1[c][y][kx] = sum_x h[c][y][x] exp(-2 pi i kx x / nx): a workgroup takes 16
// rows of one channel, thread (row, kx).
__global__ void __launch_bounds__(256) k_sno_dftx(const SnoArgs a, const float* __restrict__ h,
                                                  float2* __restrict__ H1) {
    extern __shared__ float sx[];  // 16 rows x nx, then nx twiddles (float2)
    const int nx = a.nx, ny = a.ny;
    const int rows_per_c = (ny + 15) / 16;
    const int c = blockIdx.x / rows_per_c, y0 = (blockIdx.x - c * rows_per_c) * 16;
    float2* tw = reinterpret_cast<float2*>(sx + 16 * nx);
    for (int i = threadIdx.x; i < 16 * nx; i += 256) {
        const int r = i / nx, x = i - r * nx;
        sx[i] = y0 + r < ny ? h[((long long)c * ny + y0 + r) * nx + x] : 0.f;
    }
    for (int i = threadIdx.x; i < nx; i += 256) tw[i] = a.twx[i];
    __syncthreads();
    const int r = threadIdx.x >> 4, kx = threadIdx.x & 15;
    if (y0 + r >= ny) return;
    const float* row = sx + r * nx;
    float re = 0.f, im = 0.f;
    int idx = 0;  // kx x mod nx
    for (int x = 0; x < nx; ++x) {
        const float v = row[x];
        const float2 w = tw[idx];
        re += v * w.x;
        im += v * w.y;
        idx += kx;
        if (idx >= nx) idx -= nx;
    }
    H1[((long long)c * ny + y0 + r) * SNO_KX + kx] = make_float2(re, im);
}

// Hhat[c][j][kx] = sum_y H1[c][y][kx] exp(-2 pi i ky y / ny), ky = j - 8:
// a workgroup per channel (its kept columns and the y twiddles staged in
// LDS), thread (j, kx).
__global__ void __launch_bounds__(256) k_sno_dfty(const SnoArgs a, const float2* __restrict__ H1,
                                                  float2* __restrict__ Hh) {
    extern __shared__ float2 sy[];  // ny x 16 columns, then ny twiddles
    const int c = blockIdx.x;
    const int ny = a.ny;
    float2* tw = sy + ny * SNO_KX;
    const float2* src = H1 + (long long)c * ny * SNO_KX;
    for (int i = threadIdx.x; i < ny * SNO_KX; i += 256) sy[i] = src[i];
    for (int i = threadIdx.x; i < ny; i += 256) tw[i] = a.twy[i];
    __syncthreads();
    const int j = threadIdx.x >> 4, kx = threadIdx.x & 15;
    const int ky = j - SNO_KY / 2;
    const int step = ky >= 0 ? ky : ky + ny;  // ky mod ny
    float2 acc = make_float2(0.f, 0.f);
    int idx = 0;
    for (int y = 0; y < ny; ++y) {
        const float2 v = sy[y * SNO_KX + kx];
        const float2 w = tw[idx];
        acc.x += v.x * w.x - v.y * w.y;
        acc.y += v.x * w.y + v.y * w.x;
        idx += step;
        if (idx >= ny) idx -= ny;
    }
    Hh[((long long)c * SNO_KY + j) * SNO_KX + kx] = acc;
}

// Ghat[o][j][kx] = sum_c R[j][kx][o][c] Hhat[c][j][kx]: a workgroup per mode,
// thread o.
__global__ void __launch_bounds__(SNO_C) k_sno_mix(const SnoArgs a, const uint16_t* __restrict__ R,
                                                   const float2* __restrict__ Hh, float2* __restrict__ Gh) {
    __shared__ float2 hm[SNO_C];
    const int mode = blockIdx.x;  // j * 16 + kx
    const int o = threadIdx.x;
    hm[o] = Hh[(long long)o * SNO_KY * SNO_KX + mode];
    __syncthreads();
    const uint16_t* r = R + ((long long)mode * SNO_C + o) * SNO_C * 2;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int c = 0; c < SNO_C; ++c) {
        const float2 w = make_float2(bf16f(r[2 * c]), bf16f(r[2 * c + 1]));
        const float2 v = hm[c];
        acc.x += w.x * v.x - w.y * v.y;
        acc.y += w.x * v.y + w.y * v.x;
    }
    Gh[(long long)o * SNO_KY * SNO_KX + mode] = acc;
}

// G1[o][y][kx] = sum_j Ghat[o][j][kx] exp(+2 pi i ky y / ny): thread per (o, y, kx).
__global__ void __launch_bounds__(256) k_sno_invy(const SnoArgs a, const float2* __restrict__ Gh,
                                                  float2* __restrict__ G1) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const int ny = a.ny;
    if (t >= (long long)SNO_C * ny * SNO_KX) return;
    const int kx = (int)(t % SNO_KX);
    const long long oy = t / SNO_KX;
    const int y = (int)(oy % ny), o = (int)(oy / ny);
    float2 acc = make_float2(0.f, 0.f);
    const float2* g = Gh + (long long)o * SNO_KY * SNO_KX + kx;
#pragma unroll
    for (int j = 0; j < SNO_KY; ++j) {
        const int ky = j - SNO_KY / 2;
        long long e = ((long long)ky * y) % ny;
        if (e < 0) e += ny;
        const float2 w = a.twy[e];  // exp(-2 pi i ky y / ny); conjugated below
        const float2 v = g[j * SNO_KX];
        acc.x += v.x * w.x + v.y * w.y;
        acc.y += v.y * w.x - v.x * w.y;
    }
    G1[t] = acc;
}

// h_new[o][y][x] = GELU(sum_kx w_kx Re(G1[o][y][kx] exp(+2 pi i kx x/nx)) / (nx ny)
//                       + sum_c W[o][c] h[c][y][x] + b[o]): a workgroup per row.
__global__ void __launch_bounds__(256) k_sno_invx(const SnoArgs a, const uint16_t* __restrict__ W,
                                                  const uint16_t* __restrict__ b, const float* __restrict__ h,
                                                  const float2* __restrict__ G1, float* __restrict__ hn) {
    __shared__ float2 g[SNO_C * SNO_KX];
    __shared__ float wl[SNO_C * SNO_C];
    __shared__ float bl[SNO_C];
    const int y = blockIdx.x;
    const int nx = a.nx, ny = a.ny;
    const float inv_n = 1.f / ((float)nx * (float)ny);
    for (int i = threadIdx.x; i < SNO_C * SNO_KX; i += 256) {
        const int o = i / SNO_KX, kx = i - o * SNO_KX;
        const float2 v = G1[((long long)o * ny + y) * SNO_KX + kx];
        const float s = (kx == 0 ? 1.f : 2.f) * inv_n;
        g[i] = make_float2(s * v.x, s * v.y);
    }
    for (int i = threadIdx.x; i < SNO_C * SNO_C; i += 256) wl[i] = bf16f(W[i]);
    if (threadIdx.x < SNO_C) bl[threadIdx.x] = bf16f(b[threadIdx.x]);
    __syncthreads();
    for (int x = threadIdx.x; x < nx; x += 256) {
        float hv[SNO_C];
#pragma unroll
        for (int c = 0; c < SNO_C; ++c) hv[c] = h[((long long)c * ny + y) * nx + x];
        float2 e[SNO_KX];  // exp(-2 pi i kx x / nx); the inverse uses the conjugate
        int idx = 0;
#pragma unroll
        for (int kx = 0; kx < SNO_KX; ++kx) {
            e[kx] = a.twx[idx];
            idx += x;
            if (idx >= nx) idx -= nx;
        }
        for (int o = 0; o < SNO_C; ++o) {
            float acc = bl[o];
#pragma unroll
            for (int c = 0; c < SNO_C; ++c) acc += wl[o * SNO_C + c] * hv[c];
#pragma unroll
            for (int kx = 0; kx < SNO_KX; ++kx) {
                const float2 v = g[o * SNO_KX + kx];
                acc += v.x * e[kx].x + v.y * e[kx].y;  // Re(v conj(e))
            }
            hn[((long long)o * ny + y) * nx + x] = 0.5f * acc * (1.f + erff(acc * 0.70710678118654752f));
        }
    }
}

__global__ void __launch_bounds__(256) k_sno_project(const SnoArgs a, const float* __restrict__ h,
                                                     float* __restrict__ out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n) return;
    float acc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[j] = bf16f(a.proj_b[j]);
    for (int c = 0; c < SNO_C; ++c) {
        const float v = h[(long long)c * a.n + p];
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[j] += bf16f(a.proj[j * SNO_C + c]) * v;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) out[(long long)j * a.n + p] = a.scale * acc[j];
}

}  // namespace

hipError_t sno_twiddles(float2* tw, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_sno_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, tw, n);
    return hipGetLastError();
}

size_t sno_dfty_lds(int ny);

hipError_t sno_forward(const SnoArgs& a, const float* m, float* out, hipStream_t s) {
    const unsigned pix = (unsigned)((a.n + 255) / 256);
    hipLaunchKernelGGL(k_sno_lift, dim3(pix), dim3(256), 0, s, a, m, a.h0);
    float* h = a.h0;
    float* hn = a.h1;
    const int rows_per_c = (a.ny + 15) / 16;
    const size_t xlds = (size_t)16 * a.nx * sizeof(float) + (size_t)a.nx * sizeof(float2);
    for (int l = 0; l < SNO_LAYERS; ++l) {
        hipLaunchKernelGGL(k_sno_dftx, dim3(SNO_C * rows_per_c), dim3(256), xlds, s, a, h, a.H1);
        hipLaunchKernelGGL(k_sno_dfty, dim3(SNO_C), dim3(256), sno_dfty_lds(a.ny), s, a, a.H1, a.Hh);
        hipLaunchKernelGGL(k_sno_mix, dim3(SNO_KY * SNO_KX), dim3(SNO_C), 0, s, a, a.spec[l], a.Hh, a.Gh);
        const long long ninv = (long long)SNO_C * a.ny * SNO_KX;
        hipLaunchKernelGGL(k_sno_invy, dim3((unsigned)((ninv + 255) / 256)), dim3(256), 0, s, a, a.Gh, a.G1);
        hipLaunchKernelGGL(k_sno_invx, dim3(a.ny), dim3(256), 0, s, a, a.pw[l], a.pw_b[l], h, a.G1, hn);
        float* t = h;
        h = hn;
        hn = t;
    }
    hipLaunchKernelGGL(k_sno_project, dim3(pix), dim3(256), 0, s, a, h, out);
    return hipGetLastError();
}

size_t sno_dftx_lds(int nx) { return (size_t)16 * nx * sizeof(float) + (size_t)nx * sizeof(float2); }
size_t sno_dfty_lds(int ny) { return (size_t)(SNO_KX + 1) * ny * sizeof(float2); }

hipError_t configure_sno(int ny) {
    return hipFuncSetAttribute((const void*)k_sno_dfty, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sno_dfty_lds(ny));
}

}  // namespace mm
