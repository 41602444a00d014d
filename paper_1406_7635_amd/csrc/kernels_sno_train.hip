// kernels_sno_train.hip -- training of the spectral neural operator that can
// stand in for the magnetostatic convolution: batched forward pass that keeps
// the activations, backward pass, Adam.
//
// The network is the one of kernels_sno.hip (lift 3 -> 32 channels, four
// layers of kept-mode transform -> per-mode complex 32 x 32 mixing -> inverse
// plus a pointwise 32 x 32 branch and exact-erf GELU, projection 32 -> 3),
// here with FP32 weights (the master copy; inference rounds them to BF16) and
// a batch of B samples.  Loss: the mean over the batch of the relative L2
// error ||y - t|| / ||t|| of each sample.
//
// Backward of one layer, z = g + W h + b, h' = GELU(z), g = inverse(R . H),
// H(k) = sum_r h(r) exp(-i k.r) over the kept modes, with the complex
// gradient convention Xbar = dL/dRe X + i dL/dIm X:
//   dz      = dh' GELU'(z),  GELU'(z) = Phi(z) + z phi(z)
//   dW      = sum dz h^T,  db = sum dz,  dh = W^T dz + (spectral part)
//   Gbar(k) = (w_kx / N) sum_r dz(r) exp(-i k.r)     (the forward transform of dz)
//   Rbar(k) = sum_b Gbar(k) conj(H(k))^T,  Hbar(k) = R(k)^H Gbar(k)
//   dh(r)  += Re sum_k Hbar(k) exp(+i k.r)           (inverse without w_kx / N)
// with w_0 = 1 and w_kx = 2 otherwise, N = nx ny.
//
// Layouts: fields [B][channels][ny][nx] (x fastest), kept modes
// [B][C][ky + 8][kx], weights in the flat order of include/mm.h.  Sums over
// pixels (dW, db, dQ, dq, dP, dp) go through per-workgroup partials reduced
// by a second kernel, so results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sno_internal.h"

namespace mm {

namespace {

constexpr int C = SNO_C;
constexpr int NM = SNO_KY * SNO_KX;  // kept modes
constexpr int TP = 128;              // pixels per tile of the tiled reductions
constexpr int TILES = 4;             // tiles per workgroup

__device__ inline float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_d(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// lift: h0[b][c][p] = sum_j P[c][j] m[b][j][p] + p[c]
__global__ void __launch_bounds__(256) k_tr_lift(const SnoTrainArgs a, const float* __restrict__ m,
                                                 float* __restrict__ h0) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long tot = (long long)a.batch * a.n;
    if (i >= tot) return;
    const int b = (int)(i / a.n), p = (int)(i - (long long)b * a.n);
    const float* mb = m + (long long)b * 3 * a.n;
    const float m0 = mb[p], m1 = mb[a.n + p], m2 = mb[2 * a.n + p];
    const float* P = a.w + SNO_OFF_P;
    const float* pb = a.w + SNO_OFF_PB;
    float* hb = h0 + (long long)b * C * a.n;
#pragma unroll 4
    for (int c = 0; c < C; ++c) hb[(long long)c * a.n + p] = P[3 * c] * m0 + P[3 * c + 1] * m1 + P[3 * c + 2] * m2 + pb[c];
}

// H1[q][y][kx] = sum_x src[q][y][x] exp(-2 pi i kx x / nx) for q < nq (sample x
// channel): a workgroup takes 16 rows of one q, thread (row, kx).
__global__ void __launch_bounds__(256) k_tr_dftx(const SnoTrainArgs a, const float* __restrict__ src,
                                                 float2* __restrict__ H1, int nq) {
    extern __shared__ float sx[];  // 16 rows x nx, then nx twiddles (float2)
    const int nx = a.nx, ny = a.ny;
    const int rows_per_q = (ny + 15) / 16;
    const int q = blockIdx.x / rows_per_q, y0 = (blockIdx.x - q * rows_per_q) * 16;
    if (q >= nq) return;
    float2* tw = reinterpret_cast<float2*>(sx + 16 * nx);
    for (int i = threadIdx.x; i < 16 * nx; i += 256) {
        const int r = i / nx, x = i - r * nx;
        sx[i] = y0 + r < ny ? src[((long long)q * ny + y0 + r) * nx + x] : 0.f;
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
    H1[((long long)q * ny + y0 + r) * SNO_KX + kx] = make_float2(re, im);
}

// Hh[q][j][kx] = s(kx) sum_y H1[q][y][kx] exp(-2 pi i ky y / ny), ky = j - 8,
// s = 1, or (scaled) w_kx / (nx ny): a workgroup per q, thread (j, kx).
__global__ void __launch_bounds__(256) k_tr_dfty(const SnoTrainArgs a, const float2* __restrict__ H1,
                                                 float2* __restrict__ Hh, int scaled) {
    extern __shared__ float2 sy[];  // ny x 16 columns, then ny twiddles
    const int q = blockIdx.x;
    const int ny = a.ny;
    float2* tw = sy + ny * SNO_KX;
    const float2* src = H1 + (long long)q * ny * SNO_KX;
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
    if (scaled) {
        const float s = (kx == 0 ? 1.f : 2.f) / ((float)a.nx * (float)ny);
        acc.x *= s;
        acc.y *= s;
    }
    Hh[(long long)q * NM + j * SNO_KX + kx] = acc;
}

// Gh[b][o][k] = sum_c R[k][o][c] Hh[b][c][k]: workgroup (mode, sample), thread o.
__global__ void __launch_bounds__(C) k_tr_mix(const SnoTrainArgs a, int layer, const float2* __restrict__ Hh,
                                              float2* __restrict__ Gh) {
    __shared__ float2 hm[C];
    const int mode = blockIdx.x, b = blockIdx.y;
    const int o = threadIdx.x;
    hm[o] = Hh[((long long)b * C + o) * NM + mode];
    __syncthreads();
    const float* r = a.w + SNO_OFF_R(layer) + ((long long)mode * C + o) * C * 2;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int c = 0; c < C; ++c) {
        const float wr = r[2 * c], wi = r[2 * c + 1];
        const float2 v = hm[c];
        acc.x += wr * v.x - wi * v.y;
        acc.y += wr * v.y + wi * v.x;
    }
    Gh[((long long)b * C + o) * NM + mode] = acc;
}

// Hbar[b][c][k] = sum_o conj(R[k][o][c]) Gbar[b][o][k]: workgroup (mode,
// sample), thread c.
__global__ void __launch_bounds__(C) k_tr_hbar(const SnoTrainArgs a, int layer, const float2* __restrict__ Gb,
                                               float2* __restrict__ Hb) {
    __shared__ float2 gm[C];
    const int mode = blockIdx.x, b = blockIdx.y;
    const int c = threadIdx.x;
    gm[c] = Gb[((long long)b * C + c) * NM + mode];
    __syncthreads();
    const float* r = a.w + SNO_OFF_R(layer) + (long long)mode * C * C * 2;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int o = 0; o < C; ++o) {
        const float wr = r[(o * C + c) * 2], wi = r[(o * C + c) * 2 + 1];
        const float2 v = gm[o];
        acc.x += wr * v.x + wi * v.y;  // conj(w) v
        acc.y += wr * v.y - wi * v.x;
    }
    Hb[((long long)b * C + c) * NM + mode] = acc;
}

// Rbar[k][o][c] = sum_b Gbar[b][o][k] conj(H[b][c][k]) into the gradient:
// workgroup per mode, thread (o, c).
__global__ void __launch_bounds__(C * C) k_tr_rgrad(const SnoTrainArgs a, int layer, const float2* __restrict__ Gb,
                                                    const float2* __restrict__ H) {
    const int mode = blockIdx.x;
    const int o = threadIdx.x / C, c = threadIdx.x % C;
    float2 acc = make_float2(0.f, 0.f);
    for (int b = 0; b < a.batch; ++b) {
        const float2 g = Gb[((long long)b * C + o) * NM + mode];
        const float2 h = H[((long long)b * C + c) * NM + mode];
        acc.x += g.x * h.x + g.y * h.y;  // g conj(h)
        acc.y += g.y * h.x - g.x * h.y;
    }
    float* out = a.g + SNO_OFF_R(layer) + (((long long)mode * C + o) * C + c) * 2;
    out[0] = acc.x;
    out[1] = acc.y;
}

// G1[q][y][kx] = sum_j Gh[q][j][kx] exp(+2 pi i ky y / ny): thread per (q, y, kx).
__global__ void __launch_bounds__(256) k_tr_invy(const SnoTrainArgs a, const float2* __restrict__ Gh,
                                                 float2* __restrict__ G1, int nq) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const int ny = a.ny;
    if (t >= (long long)nq * ny * SNO_KX) return;
    const int kx = (int)(t % SNO_KX);
    const long long qy = t / SNO_KX;
    const int y = (int)(qy % ny);
    const long long q = qy / ny;
    float2 acc = make_float2(0.f, 0.f);
    const float2* g = Gh + q * NM + kx;
#pragma unroll
    for (int j = 0; j < SNO_KY; ++j) {
        const int ky = j - SNO_KY / 2;
        int e = (int)(((long long)ky * y) % ny);
        if (e < 0) e += ny;
        const float2 w = a.twy[e];  // exp(-2 pi i ky y / ny), conjugated below
        const float2 v = g[j * SNO_KX];
        acc.x += v.x * w.x + v.y * w.y;
        acc.y += v.y * w.x - v.x * w.y;
    }
    G1[t] = acc;
}

// forward pointwise part of layer l, per row (b, y):
// z_o = sum_kx (w_kx/N) Re(G1[b][o][y][kx] exp(+2 pi i kx x/nx)) + sum_c W[o][c] h_c + b_o,
// h'_o = GELU(z_o); z and h' are kept.
__global__ void __launch_bounds__(256) k_tr_invx_fwd(const SnoTrainArgs a, int layer, const float* __restrict__ h,
                                                     const float2* __restrict__ G1, float* __restrict__ z,
                                                     float* __restrict__ hn) {
    __shared__ float2 g[C * SNO_KX];
    __shared__ float wl[C * C];
    __shared__ float bl[C];
    const int b = blockIdx.x / a.ny, y = blockIdx.x - b * a.ny;
    const int nx = a.nx, ny = a.ny;
    const float inv_n = 1.f / ((float)nx * (float)ny);
    for (int i = threadIdx.x; i < C * SNO_KX; i += 256) {
        const int o = i / SNO_KX, kx = i - o * SNO_KX;
        const float2 v = G1[(((long long)b * C + o) * ny + y) * SNO_KX + kx];
        const float s = (kx == 0 ? 1.f : 2.f) * inv_n;
        g[i] = make_float2(s * v.x, s * v.y);
    }
    for (int i = threadIdx.x; i < C * C; i += 256) wl[i] = a.w[SNO_OFF_W(layer) + i];
    if (threadIdx.x < C) bl[threadIdx.x] = a.w[SNO_OFF_B(layer) + threadIdx.x];
    __syncthreads();
    const long long rowbase = (long long)b * C * a.n + (long long)y * nx;
    for (int x = threadIdx.x; x < nx; x += 256) {
        float hv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) hv[c] = h[rowbase + (long long)c * a.n + x];
        float2 e[SNO_KX];
        int idx = 0;
#pragma unroll
        for (int kx = 0; kx < SNO_KX; ++kx) {
            e[kx] = a.twx[idx];
            idx += x;
            if (idx >= nx) idx -= nx;
        }
        for (int o = 0; o < C; ++o) {
            float acc = bl[o];
#pragma unroll
            for (int c = 0; c < C; ++c) acc += wl[o * C + c] * hv[c];
#pragma unroll
            for (int kx = 0; kx < SNO_KX; ++kx) {
                const float2 v = g[o * SNO_KX + kx];
                acc += v.x * e[kx].x + v.y * e[kx].y;  // Re(v conj(e))
            }
            z[rowbase + (long long)o * a.n + x] = acc;
            hn[rowbase + (long long)o * a.n + x] = gelu(acc);
        }
    }
}

// backward pointwise part, per row (b, y):
// dh_c = sum_o W[o][c] dz_o + Re sum_kx Hb1[b][c][y][kx] exp(+2 pi i kx x/nx)
__global__ void __launch_bounds__(256) k_tr_invx_bwd(const SnoTrainArgs a, int layer, const float* __restrict__ dz,
                                                     const float2* __restrict__ Hb1, float* __restrict__ dh) {
    __shared__ float2 g[C * SNO_KX];
    __shared__ float wl[C * C];
    const int b = blockIdx.x / a.ny, y = blockIdx.x - b * a.ny;
    const int nx = a.nx, ny = a.ny;
    for (int i = threadIdx.x; i < C * SNO_KX; i += 256) {
        const int c = i / SNO_KX, kx = i - c * SNO_KX;
        g[i] = Hb1[(((long long)b * C + c) * ny + y) * SNO_KX + kx];
    }
    for (int i = threadIdx.x; i < C * C; i += 256) wl[i] = a.w[SNO_OFF_W(layer) + i];
    __syncthreads();
    const long long rowbase = (long long)b * C * a.n + (long long)y * nx;
    for (int x = threadIdx.x; x < nx; x += 256) {
        float dv[C];
#pragma unroll
        for (int o = 0; o < C; ++o) dv[o] = dz[rowbase + (long long)o * a.n + x];
        float2 e[SNO_KX];
        int idx = 0;
#pragma unroll
        for (int kx = 0; kx < SNO_KX; ++kx) {
            e[kx] = a.twx[idx];
            idx += x;
            if (idx >= nx) idx -= nx;
        }
        for (int c = 0; c < C; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int o = 0; o < C; ++o) acc += wl[o * C + c] * dv[o];
#pragma unroll
            for (int kx = 0; kx < SNO_KX; ++kx) {
                const float2 v = g[c * SNO_KX + kx];
                acc += v.x * e[kx].x + v.y * e[kx].y;
            }
            dh[rowbase + (long long)c * a.n + x] = acc;
        }
    }
}

// projection: y[b][j][p] = sum_c Q[j][c] h[b][c][p] + q[j]
__global__ void __launch_bounds__(256) k_tr_project(const SnoTrainArgs a, const float* __restrict__ h,
                                                    float* __restrict__ y) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)a.batch * a.n) return;
    const int b = (int)(i / a.n), p = (int)(i - (long long)b * a.n);
    const float* Q = a.w + SNO_OFF_Q;
    const float* q = a.w + SNO_OFF_QB;
    float acc[3] = {q[0], q[1], q[2]};
    const float* hb = h + (long long)b * C * a.n + p;
    for (int c = 0; c < C; ++c) {
        const float v = hb[(long long)c * a.n];
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[j] += Q[j * C + c] * v;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) y[((long long)b * 3 + j) * a.n + p] = acc[j];
}

// per (sample, chunk): sum (y - t)^2 and sum t^2 in FP64
constexpr int LOSS_CHUNKS = 64;
__global__ void __launch_bounds__(256) k_tr_loss_part(const SnoTrainArgs a, const float* __restrict__ y,
                                                      const float* __restrict__ t, double* __restrict__ part) {
    __shared__ double red[2][4];
    const int b = blockIdx.y, ch = blockIdx.x;
    const long long len = 3LL * a.n;
    const long long per = (len + LOSS_CHUNKS - 1) / LOSS_CHUNKS;
    const long long i0 = ch * per, i1 = i0 + per < len ? i0 + per : len;
    const float* yb = y + (long long)b * len;
    const float* tb = t + (long long)b * len;
    double dd = 0.0, tt = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += 256) {
        const double d = (double)yb[i] - (double)tb[i];
        dd += d * d;
        tt += (double)tb[i] * (double)tb[i];
    }
    for (int off = 32; off > 0; off >>= 1) {
        dd += __shfl_xor(dd, off, 64);
        tt += __shfl_xor(tt, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = dd;
        red[1][wv] = tt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[((long long)b * LOSS_CHUNKS + ch) * 2] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        part[((long long)b * LOSS_CHUNKS + ch) * 2 + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// scale[b] = 1 / (||d_b|| ||t_b|| B) (0 when d_b = 0 or t_b = 0), loss = mean ||d_b|| / ||t_b||
__global__ void k_tr_loss_final(const SnoTrainArgs a, const double* __restrict__ part, float* __restrict__ scale,
                                double* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double l = 0.0;
    for (int b = 0; b < a.batch; ++b) {
        double dd = 0.0, tt = 0.0;
        for (int ch = 0; ch < LOSS_CHUNKS; ++ch) {
            dd += part[((long long)b * LOSS_CHUNKS + ch) * 2];
            tt += part[((long long)b * LOSS_CHUNKS + ch) * 2 + 1];
        }
        const double nd = sqrt(dd), nt = sqrt(tt);
        scale[b] = (nd > 0.0 && nt > 0.0) ? (float)(1.0 / (nd * nt * a.batch)) : 0.f;
        l += nt > 0.0 ? nd / nt : 0.0;
    }
    *loss = l / a.batch;
}

// Tiled pixel sums: a workgroup takes TILES tiles of TP pixels of the
// flattened (sample, pixel) index; per tile the per-pixel vectors go to LDS
// and thread k < K accumulates output k over the tile; the workgroup writes
// its K sums to part[blockIdx.x][K].
__device__ inline void pixel_of(const SnoTrainArgs& a, long long i, int& b, int& p) {
    b = (int)(i / a.n);
    p = (int)(i - (long long)b * a.n);
}

// projection backward: dy = scale_b (y - t); dh_c = sum_j Q[j][c] dy_j;
// sums dQ[j][c] = dy_j h_c (96), dq[j] = dy_j (3)
constexpr int KPROJ = 3 * C + 3;
__global__ void __launch_bounds__(256) k_tr_project_bwd(const SnoTrainArgs a, const float* __restrict__ y,
                                                        const float* __restrict__ t, const float* __restrict__ scale,
                                                        const float* __restrict__ h, float* __restrict__ dh,
                                                        float* __restrict__ part) {
    __shared__ float sdy[3][TP + 1];  // rows padded by one: the threads of a wave read 32 rows at one column
    __shared__ float sh[C][TP + 1];
    const long long tot = (long long)a.batch * a.n;
    const float* Q = a.w + SNO_OFF_Q;
    const int k = threadIdx.x;
    float acc = 0.f;
    for (int tile = 0; tile < TILES; ++tile) {
        const long long i0 = ((long long)blockIdx.x * TILES + tile) * TP;
        __syncthreads();
        if (threadIdx.x < TP) {
            const long long i = i0 + threadIdx.x;
            float dy[3] = {0.f, 0.f, 0.f};
            if (i < tot) {
                int b, p;
                pixel_of(a, i, b, p);
                const float s = scale[b];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const long long o = ((long long)b * 3 + j) * a.n + p;
                    dy[j] = s * (y[o] - t[o]);
                }
                const long long hb = (long long)b * C * a.n + p;
                for (int c = 0; c < C; ++c) {
                    const float hv = h[hb + (long long)c * a.n];
                    sh[c][threadIdx.x] = hv;
                    dh[hb + (long long)c * a.n] = Q[c] * dy[0] + Q[C + c] * dy[1] + Q[2 * C + c] * dy[2];
                }
            } else {
                for (int c = 0; c < C; ++c) sh[c][threadIdx.x] = 0.f;
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) sdy[j][threadIdx.x] = dy[j];
        }
        __syncthreads();
        if (k < 3 * C) {
            const int j = k / C, c = k - j * C;
            for (int u = 0; u < TP; ++u) acc += sdy[j][u] * sh[c][u];
        } else if (k < KPROJ) {
            const int j = k - 3 * C;
            for (int u = 0; u < TP; ++u) acc += sdy[j][u];
        }
    }
    if (k < KPROJ) part[(long long)blockIdx.x * KPROJ + k] = acc;
}

// GELU backward of layer l: dz = dh GELU'(z) (written), sums dW[o][c] =
// dz_o h_c (1024) and db[o] = dz_o (32) with h the layer's input
constexpr int KLAYER = C * C + C;
__global__ void __launch_bounds__(256) k_tr_gelu_bwd(const SnoTrainArgs a, const float* __restrict__ z,
                                                     const float* __restrict__ dh, const float* __restrict__ h,
                                                     float* __restrict__ dz, float* __restrict__ part) {
    __shared__ float sdz[C][TP + 1];
    __shared__ float sh[C][TP + 1];
    const long long tot = (long long)a.batch * a.n;
    float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // outputs threadIdx.x + 256 r
    for (int tile = 0; tile < TILES; ++tile) {
        const long long i0 = ((long long)blockIdx.x * TILES + tile) * TP;
        __syncthreads();
        {
            // 256 threads fill 2 x 32 x 128 values: thread (half, pixel)
            const int u = threadIdx.x & (TP - 1), half = threadIdx.x / TP;
            const long long i = i0 + u;
            if (i < tot) {
                int b, p;
                pixel_of(a, i, b, p);
                const long long base = (long long)b * C * a.n + p;
                for (int c = half * (C / 2); c < (half + 1) * (C / 2); ++c) {
                    const long long o = base + (long long)c * a.n;
                    const float d = dh[o] * gelu_d(z[o]);
                    dz[o] = d;
                    sdz[c][u] = d;
                    sh[c][u] = h[o];
                }
            } else {
                for (int c = half * (C / 2); c < (half + 1) * (C / 2); ++c) {
                    sdz[c][u] = 0.f;
                    sh[c][u] = 0.f;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const int k = threadIdx.x + 256 * r;
            if (k < C * C) {
                const int o = k / C, c = k - o * C;
                float s = 0.f;
                for (int u = 0; u < TP; ++u) s += sdz[o][u] * sh[c][u];
                acc[r] += s;
            } else if (k < KLAYER) {
                const int o = k - C * C;
                float s = 0.f;
                for (int u = 0; u < TP; ++u) s += sdz[o][u];
                acc[r] += s;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        const int k = threadIdx.x + 256 * r;
        if (k < KLAYER) part[(long long)blockIdx.x * KLAYER + k] = acc[r];
    }
}

// lift backward: sums dP[c][j] = dh0_c m_j (96), dp[c] = dh0_c (32)
constexpr int KLIFT = 3 * C + C;
__global__ void __launch_bounds__(256) k_tr_lift_bwd(const SnoTrainArgs a, const float* __restrict__ m,
                                                     const float* __restrict__ dh0, float* __restrict__ part) {
    __shared__ float sd[C][TP + 1];
    __shared__ float sm[3][TP + 1];
    const long long tot = (long long)a.batch * a.n;
    const int k = threadIdx.x;
    float acc = 0.f;
    for (int tile = 0; tile < TILES; ++tile) {
        const long long i0 = ((long long)blockIdx.x * TILES + tile) * TP;
        __syncthreads();
        if (threadIdx.x < TP) {
            const long long i = i0 + threadIdx.x;
            if (i < tot) {
                int b, p;
                pixel_of(a, i, b, p);
                const long long hb = (long long)b * C * a.n + p;
                for (int c = 0; c < C; ++c) sd[c][threadIdx.x] = dh0[hb + (long long)c * a.n];
                for (int j = 0; j < 3; ++j) sm[j][threadIdx.x] = m[((long long)b * 3 + j) * a.n + p];
            } else {
                for (int c = 0; c < C; ++c) sd[c][threadIdx.x] = 0.f;
                for (int j = 0; j < 3; ++j) sm[j][threadIdx.x] = 0.f;
            }
        }
        __syncthreads();
        if (k < 3 * C) {
            const int c = k / 3, j = k - 3 * c;
            for (int u = 0; u < TP; ++u) acc += sd[c][u] * sm[j][u];
        } else if (k < KLIFT) {
            const int c = k - 3 * C;
            for (int u = 0; u < TP; ++u) acc += sd[c][u];
        }
    }
    if (k < KLIFT) part[(long long)blockIdx.x * KLIFT + k] = acc;
}

// out[k] = sum_r part[r][k] (FP64 accumulation), k < K
__global__ void __launch_bounds__(256) k_tr_reduce(const float* __restrict__ part, int nrows, int K,
                                                   float* __restrict__ out) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int r = 0;
    for (; r + 3 < nrows; r += 4) {
        s0 += part[(long long)r * K + k];
        s1 += part[(long long)(r + 1) * K + k];
        s2 += part[(long long)(r + 2) * K + k];
        s3 += part[(long long)(r + 3) * K + k];
    }
    for (; r < nrows; ++r) s0 += part[(long long)r * K + k];
    out[k] = (float)((s0 + s1) + (s2 + s3));
}

// Adam (Kingma and Ba): m1 <- b1 m1 + (1 - b1) g, m2 <- b2 m2 + (1 - b2) g^2,
// w <- w - lr (m1 / c1) / (sqrt(m2 / c2) + eps), c = 1 - beta^t
__global__ void __launch_bounds__(256) k_tr_adam(float* __restrict__ w, const float* __restrict__ g,
                                                 float* __restrict__ m1, float* __restrict__ m2, long long n,
                                                 float lr, float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    w[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

unsigned nblk(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

size_t sno_train_dfty_lds(int ny) { return (size_t)(SNO_KX + 1) * ny * sizeof(float2); }

hipError_t configure_sno_train(int ny) {
    return hipFuncSetAttribute((const void*)k_tr_dfty, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sno_train_dfty_lds(ny));
}

int sno_train_tiles(long long pixels) { return (int)((pixels + TP * TILES - 1) / (TP * TILES)); }

// forward pass with the activations kept, loss, backward pass into a.g
hipError_t sno_train_grad(const SnoTrainArgs& a, const SnoTrainBufs& s, const float* m, const float* t,
                          hipStream_t st) {
    const long long pix = (long long)a.batch * a.n;
    const int nq = a.batch * C;
    const unsigned pixb = nblk(pix, 256);
    const size_t xlds = (size_t)16 * a.nx * sizeof(float) + (size_t)a.nx * sizeof(float2);
    const size_t ylds = sno_train_dfty_lds(a.ny);
    const unsigned xgrid = (unsigned)(nq * ((a.ny + 15) / 16));
    const unsigned invgrid = nblk((long long)nq * a.ny * SNO_KX, 256);
    const unsigned rows = (unsigned)(a.batch * a.ny);
    // forward
    hipLaunchKernelGGL(k_tr_lift, dim3(pixb), dim3(256), 0, st, a, m, s.h[0]);
    for (int l = 0; l < SNO_LAYERS; ++l) {
        hipLaunchKernelGGL(k_tr_dftx, dim3(xgrid), dim3(256), xlds, st, a, s.h[l], s.line, nq);
        hipLaunchKernelGGL(k_tr_dfty, dim3(nq), dim3(256), ylds, st, a, s.line, s.H[l], 0);
        hipLaunchKernelGGL(k_tr_mix, dim3(NM, a.batch), dim3(C), 0, st, a, l, s.H[l], s.modes);
        hipLaunchKernelGGL(k_tr_invy, dim3(invgrid), dim3(256), 0, st, a, s.modes, s.line, nq);
        hipLaunchKernelGGL(k_tr_invx_fwd, dim3(rows), dim3(256), 0, st, a, l, s.h[l], s.line, s.z[l], s.h[l + 1]);
    }
    hipLaunchKernelGGL(k_tr_project, dim3(pixb), dim3(256), 0, st, a, s.h[SNO_LAYERS], s.y);
    hipLaunchKernelGGL(k_tr_loss_part, dim3(LOSS_CHUNKS, a.batch), dim3(256), 0, st, a, s.y, t, s.lpart);
    hipLaunchKernelGGL(k_tr_loss_final, dim3(1), dim3(64), 0, st, a, s.lpart, s.scale, s.loss);
    // backward
    const unsigned tiles = (unsigned)sno_train_tiles(pix);
    float* dh = s.dh[0];
    float* dhp = s.dh[1];
    hipLaunchKernelGGL(k_tr_project_bwd, dim3(tiles), dim3(256), 0, st, a, s.y, t, s.scale, s.h[SNO_LAYERS], dh,
                       s.part);
    hipLaunchKernelGGL(k_tr_reduce, dim3(nblk(KPROJ, 256)), dim3(256), 0, st, s.part, (int)tiles, KPROJ,
                       a.g + SNO_OFF_Q);
    for (int l = SNO_LAYERS - 1; l >= 0; --l) {
        hipLaunchKernelGGL(k_tr_gelu_bwd, dim3(tiles), dim3(256), 0, st, a, s.z[l], dh, s.h[l], s.dz, s.part);
        hipLaunchKernelGGL(k_tr_reduce, dim3(nblk(KLAYER, 256)), dim3(256), 0, st, s.part, (int)tiles, KLAYER,
                           a.g + SNO_OFF_W(l));
        hipLaunchKernelGGL(k_tr_dftx, dim3(xgrid), dim3(256), xlds, st, a, s.dz, s.line, nq);
        hipLaunchKernelGGL(k_tr_dfty, dim3(nq), dim3(256), ylds, st, a, s.line, s.modes, 1);
        hipLaunchKernelGGL(k_tr_rgrad, dim3(NM), dim3(C * C), 0, st, a, l, s.modes, s.H[l]);
        hipLaunchKernelGGL(k_tr_hbar, dim3(NM, a.batch), dim3(C), 0, st, a, l, s.modes, s.modes2);
        hipLaunchKernelGGL(k_tr_invy, dim3(invgrid), dim3(256), 0, st, a, s.modes2, s.line, nq);
        hipLaunchKernelGGL(k_tr_invx_bwd, dim3(rows), dim3(256), 0, st, a, l, s.dz, s.line, dhp);
        float* tmp = dh;
        dh = dhp;
        dhp = tmp;
    }
    hipLaunchKernelGGL(k_tr_lift_bwd, dim3(tiles), dim3(256), 0, st, a, m, dh, s.part);
    hipLaunchKernelGGL(k_tr_reduce, dim3(nblk(KLIFT, 256)), dim3(256), 0, st, s.part, (int)tiles, KLIFT,
                       a.g + SNO_OFF_P);
    return hipGetLastError();
}

hipError_t sno_train_adam(float* w, const float* g, float* m1, float* m2, long long n, float lr, float b1, float b2,
                          float eps, long long step, hipStream_t st) {
    const float c1 = (float)(1.0 - pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)step));
    hipLaunchKernelGGL(k_tr_adam, dim3(nblk(n, 256)), dim3(256), 0, st, w, g, m1, m2, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace mm
