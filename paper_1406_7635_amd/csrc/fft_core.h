// fft_core.h -- in-LDS Stockham FFT building blocks (FP32) for gfx950.
//
// A workgroup holds F independent sequences of power-of-two length P in LDS,
// sequence f at buf[f * seq_len(P) + lds_pad(i)].  The transform runs as a
// chain of radix-R Stockham stages (autosort, no bit reversal): stage (R, L)
// reads inputs j + r P/R, applies twiddles w^(r k) with w = exp(-+2 pi i/(L R))
// and k = j mod L, does an R-point DFT and writes the outputs to
// (j - k) R + k + r L.  The first stage takes radix 2 or 4 when log2 P is not
// a multiple of 3; every later stage is radix 8.  Every stage first reads all
// of its inputs into registers, then (after a barrier) writes, so one LDS
// buffer suffices.  Forward uses exp(-2 pi i n k / P), inverse exp(+...),
// both unnormalised.
//
// The read and write halves of a stage are separate __host__ __device__
// functions so that a host program can emulate a whole workgroup and check
// the index arithmetic against a reference DFT without a GPU.
#pragma once

#include <hip/hip_runtime.h>

namespace mm {

struct cf {
    float x, y;
};

__host__ __device__ inline cf mkc(float x, float y) { cf r; r.x = x; r.y = y; return r; }
__host__ __device__ inline cf operator+(cf a, cf b) { return mkc(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cf operator-(cf a, cf b) { return mkc(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cf operator*(float s, cf a) { return mkc(s * a.x, s * a.y); }
__host__ __device__ inline cf cmul(cf a, cf b) {
    return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cf cconj(cf a) { return mkc(a.x, -a.y); }

// multiply by exp(+-i pi/2): forward (INV=false) by -i, inverse by +i
template <bool INV>
__host__ __device__ inline cf rot90(cf a) {
    return INV ? mkc(-a.y, a.x) : mkc(a.y, -a.x);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// one spare element every 8 spreads stride-8 Stockham writes over the LDS banks
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int seq_len(int P) { return P + (P >> 3); }

// R-point DFTs in registers -------------------------------------------------
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
    __host__ __device__ static void run(cf*) {}
};

template <bool INV>
struct Dft<2, INV> {
    __host__ __device__ static void run(cf* v) {
        cf a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <bool INV>
struct Dft<4, INV> {
    __host__ __device__ static void run(cf* v) {
        cf a0 = v[0] + v[2], a1 = v[0] - v[2];
        cf a2 = v[1] + v[3], a3 = rot90<INV>(v[1] - v[3]);
        v[0] = a0 + a2;
        v[2] = a0 - a2;
        v[1] = a1 + a3;
        v[3] = a1 - a3;
    }
};

template <bool INV>
struct Dft<8, INV> {
    __host__ __device__ static void run(cf* v) {
        const float h = 0.70710678118654752f;  // 1/sqrt(2)
        cf e[4] = {v[0], v[2], v[4], v[6]};
        cf o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, INV>::run(e);
        Dft<4, INV>::run(o);
        // o[k] *= w8^k with w8 = exp(-+ i pi/4)
        cf o1 = o[1], o3 = o[3];
        o[1] = INV ? mkc(h * (o1.x - o1.y), h * (o1.x + o1.y)) : mkc(h * (o1.x + o1.y), h * (o1.y - o1.x));
        o[2] = rot90<INV>(o[2]);
        o[3] = INV ? mkc(-h * (o3.x + o3.y), h * (o3.x - o3.y)) : mkc(h * (o3.y - o3.x), -h * (o3.x + o3.y));
        for (int k = 0; k < 4; ++k) {
            v[k] = e[k] + o[k];
            v[k + 4] = e[k] - o[k];
        }
    }
};

// radix of the stage that starts at span L (the first stage absorbs log2 P mod 3)
__host__ __device__ constexpr int stage_radix(int P, int L) {
    return (L == 1 && (ilog2(P) % 3) != 0) ? (1 << (ilog2(P) % 3)) : 8;
}

// Stage read half: gather, twiddle and transform the butterflies of thread tid.
// tw: table exp(-2 pi i m / PT), m < PT; twshift = log2(PT).
template <int P, int R, int L, int F, int NT, bool INV>
struct Stage {
    static constexpr int NBF = P / R;          // butterflies per sequence
    static constexpr int TOT = F * NBF;
    static constexpr int NB = (TOT + NT - 1) / NT;
    static constexpr int SEQ = seq_len(P);
    static constexpr int TWL = ilog2(L * R);

    __host__ __device__ static void read(const cf* buf, const cf* __restrict__ tw, int twshift,
                                         int tid, cf (&v)[NB][R]) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int b = tid + q * NT;
            if ((TOT % NT) == 0 || b < TOT) {
                const int f = b / NBF;
                const int j = b - f * NBF;
                const int k = j & (L - 1);
                const cf* src = buf + f * SEQ;
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = src[lds_pad(j + r * NBF)];
                if (L > 1) {
                    const int sh = twshift - TWL;
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        cf w = tw[(r * k) << sh];
                        if (INV) w = cconj(w);
                        v[q][r] = cmul(v[q][r], w);
                    }
                }
                Dft<R, INV>::run(v[q]);
            }
        }
    }

    __host__ __device__ static void write(cf* buf, int tid, const cf (&v)[NB][R]) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int b = tid + q * NT;
            if ((TOT % NT) == 0 || b < TOT) {
                const int f = b / NBF;
                const int j = b - f * NBF;
                const int k = j & (L - 1);
                cf* dst = buf + f * SEQ;
                const int base = (j - k) * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) dst[lds_pad(base + r * L)] = v[q][r];
            }
        }
    }
};

// Whole transform on the device: stages chained at compile time.
template <int P, int L, int F, int NT, bool INV>
struct Fft {
    static constexpr int R = stage_radix(P, L);
    __device__ static void run(cf* buf, const cf* __restrict__ tw, int twshift, int tid) {
        using S = Stage<P, R, L, F, NT, INV>;
        cf v[S::NB][R];
        S::read(buf, tw, twshift, tid, v);
        __syncthreads();
        S::write(buf, tid, v);
        __syncthreads();
        Fft<P, L * R, F, NT, INV>::run(buf, tw, twshift, tid);
    }
};

template <int P, int F, int NT, bool INV>
struct Fft<P, P, F, NT, INV> {
    __device__ static void run(cf*, const cf* __restrict__, int, int) {}
};

}  // namespace mm
