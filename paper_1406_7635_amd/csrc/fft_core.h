// fft_core.h -- register-resident FP32 FFT building blocks for gfx950.
//
// Power-of-two transforms in Stockham (autosort) form: stage (R, L) reads
// inputs j + r P/R, multiplies them by w^(r k) with w = exp(-+2 pi i/(L R)) and
// k = j mod L, does an R-point DFT and writes the outputs to (j - k) R + k + r L.
// Forward uses exp(-2 pi i n k / P), inverse exp(+...), both unnormalised.
// Each thread keeps its points in registers; LDS is only the exchange medium
// between stages.
#pragma once

#include <hip/hip_runtime.h>

namespace mm {

struct alignas(8) cf {
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

// Complex load and store through a raw buffer resource: uniform base in
// scalar registers, 32-bit byte offset per lane (no 64-bit address
// arithmetic); the third resource word is the gfx9 family's untyped format.
// Device code only (declared in both compilation passes, as device code
// that the host pass parses refers to them).
__device__ inline __amdgpu_buffer_rsrc_t cf_buffer(const cf* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<cf*>(base), (short)0, (int)0xffffffffu, 0x00020000);
}
__device__ inline cf ld_cf(const cf* base, unsigned int byte_off) {
    return __builtin_bit_cast(cf, __builtin_amdgcn_raw_buffer_load_b64(cf_buffer(base), (int)byte_off, 0, 0));
}
__device__ inline void st_cf(cf* base, unsigned int byte_off, cf v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), cf_buffer(base), (int)byte_off, 0, 0);
}

// multiply by exp(+-i pi/2): forward (INV=false) by -i, inverse by +i
template <bool INV>
__host__ __device__ inline cf rot90(cf a) {
    return INV ? mkc(-a.y, a.x) : mkc(a.y, -a.x);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int ilog2_floor(int n) { return n <= 1 ? 0 : 1 + ilog2_floor(n / 2); }
__host__ __device__ inline int ilog2_rt(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// LDS position of sequence element i outside the transforms (staging,
// separation, crop): three spare elements after every 32, so contiguous wave
// accesses meet at most one spare run; being additive over 32-aligned
// offsets, the per-register offsets fold into the instructions' immediate
// offsets.  The exchanges inside a transform use their own padding
// (RegFft::xpad), at most one spare per 8 elements.
__host__ __device__ constexpr int lds_pad(int i) { return i + 3 * (i >> 5); }
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

template <bool INV>
struct Dft<16, INV> {
    // 16 = 4 x 4: DFT-4 over n1 for each n2, twiddle w16^(n2 k1), DFT-4 over n2
    __host__ __device__ static void run(cf* v) {
        const float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
        const float cs[10][2] = {{1.f, 0.f}, {c1, s1}, {h, h}, {s1, c1}, {0.f, 1.f},
                                 {-s1, c1}, {-h, h}, {-c1, s1}, {-1.f, 0.f}, {-c1, -s1}};
        cf a[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            cf t[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
            Dft<4, INV>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) {
                const int m = n2 * k1;
                const cf w = mkc(cs[m][0], INV ? cs[m][1] : -cs[m][1]);
                a[n2][k1] = (m == 0) ? t[k1] : cmul(t[k1], w);
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cf t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            Dft<4, INV>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
        }
    }
};

// exp(-+2 pi i m / 16) x for a compile-time m (after unrolling): the
// multiplications by 0 and +-1 are spelled out, since the compiler may not
// drop them itself (signed zeros)
template <bool INV>
__host__ __device__ inline cf twist16(cf x, int m) {
    const float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
    m &= 15;
    if (m == 0) return x;
    if (m == 4) return rot90<INV>(x);
    if (m == 8) return mkc(-x.x, -x.y);
    if (m == 12) return rot90<!INV>(x);
    const float cs[16][2] = {{1.f, 0.f}, {c1, s1}, {h, h}, {s1, c1}, {0.f, 1.f}, {-s1, c1}, {-h, h}, {-c1, s1},
                             {-1.f, 0.f}, {-c1, -s1}, {-h, -h}, {-s1, -c1}, {0.f, -1.f}, {s1, -c1}, {h, -h}, {c1, -s1}};
    const float wr = cs[m][0], wi = INV ? cs[m][1] : -cs[m][1];
    if ((m & 3) == 2) {  // +-h (1 +- i): two products instead of four
        const float hr = wr, hi = wi;  // |hr| = |hi| = h
        return (hr == hi) ? mkc(hr * (x.x - x.y), hr * (x.x + x.y)) : mkc(hr * (x.x + x.y), hr * (x.y - x.x));
    }
    return cmul(x, mkc(wr, wi));
}

// R-point DFT of a sequence whose upper R/2 inputs are zero (zero padding):
// the even outputs are the R/2-point DFT of the inputs, the odd outputs that
// of the inputs twisted by w_R^n.  Inputs in v[0..R/2), outputs in v[0..R).
template <int R, bool INV>
struct DftHalf {
    __host__ __device__ static void run(cf* v) {
        constexpr int H = R / 2;
        cf y[H], z[H];
#pragma unroll
        for (int n = 0; n < H; ++n) {
            y[n] = v[n];
            z[n] = twist16<INV>(v[n], n * (16 / R));
        }
        Dft<H, INV>::run(y);
        Dft<H, INV>::run(z);
#pragma unroll
        for (int j = 0; j < H; ++j) {
            v[2 * j] = y[j];
            v[2 * j + 1] = z[j];
        }
    }
};

// ---------------------------------------------------------------------------
// Register-resident transform.  A group of TPF threads owns NF sequences of
// length P; thread t keeps PPT = P/TPF points of each in registers, in
// natural order v[f][m] = x[t + TPF m] on entry and X[t + TPF m] on exit.
// Stage 0 has radix R0 (the remainder of log2 P modulo log2 PPT, else PPT) and
// runs on the loaded registers; every later stage has radix PPT and gets its
// inputs through one LDS exchange (write the previous stage's outputs at their
// Stockham positions, barrier, read j + r TPF).  The NF sequences go through a
// single LDS sequence one after the other, so a group needs seq_len(P)
// elements of LDS.  The exchange halves are separate __host__ __device__
// functions so a host program can emulate a group without a GPU.
// HIN: the inputs x[n], n >= P/2, are zero (zero padding) and the registers
// holding them are ignored; stage 0 then runs the half-input butterflies.
template <int P, int TPF, int NF, bool INV, bool HIN = false>
struct RegFft {
    static constexpr int PPT = P / TPF;
    static constexpr int LP = ilog2(P);
    static constexpr int LA = ilog2(PPT);
    static constexpr int REM = LA == 0 ? 0 : LP % LA;
    static constexpr int R0 = LA == 0 ? 1 : (REM ? (1 << REM) : PPT);
    static constexpr int NS = LA == 0 ? 0 : (REM ? 1 : 0) + LP / LA;
    static constexpr int SEQ = seq_len(P);

    // span of stage s (product of the radices before it)
    __host__ __device__ static int span(int s) { return s == 0 ? 1 : R0 << (LA * (s - 1)); }

    // natural order -> stage-0 order, then the stage-0 butterflies (no twiddles).
    // Input r of butterfly u is x[t + TPF u + r P/R0], zero for r >= R0/2 under HIN.
    __host__ __device__ static void stage0(cf (&v)[NF][PPT]) {
        constexpr bool HALF = HIN && R0 >= 2;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cf w[PPT];
#pragma unroll
            for (int u = 0; u < PPT / R0; ++u)
#pragma unroll
                for (int r = 0; r < R0; ++r) w[u * R0 + r] = v[f][u + r * (PPT / R0)];
#pragma unroll
            for (int u = 0; u < PPT / R0; ++u) {
                if constexpr (HALF)
                    DftHalf<R0, INV>::run(w + u * R0);
                else
                    Dft<R0, INV>::run(w + u * R0);
            }
#pragma unroll
            for (int i = 0; i < PPT; ++i) v[f][i] = w[i];
        }
    }

    // twiddles w^(r k), r < PPT, of thread t in stage s >= 1: the powers
    // w^(2^i k) come from the table (exp(-2 pi i m / PT) rounded once), the
    // others are products of at most log2(PPT) - 1 of them
    __host__ __device__ static void twiddles(int s, int t, const cf* __restrict__ tw, int twshift, cf (&wt)[PPT]) {
        const int L = span(s);
        int k = t & (L - 1);
#ifdef __HIP_DEVICE_COMPILE__
        asm volatile("" : "+v"(k));  // keep the table loads at their stage (short live ranges)
#endif
        const int sh = twshift - ilog2_rt(L * PPT);
        wt[0] = mkc(1.f, 0.f);
#pragma unroll
        for (int b = 1; b < PPT; b <<= 1) {
#ifdef __HIP_DEVICE_COMPILE__
            const cf w = ld_cf(tw, (unsigned int)((b * k) << sh) * 8u);
#else
            const cf w = tw[(b * k) << sh];
#endif
            wt[b] = INV ? cconj(w) : w;
        }
#pragma unroll
        for (int r = 3; r < PPT; ++r) {
            if ((r & (r - 1)) == 0) continue;
            const int hb = 1 << ilog2_floor(r);
            wt[r] = cmul(wt[hb], wt[r - hb]);
        }
    }

    // LDS position of element i in the exchange whose writes have radix RP
    // and span lp (the exchange that feeds a stage).  Each wave writes its 16-lane
    // groups (8 bytes a lane, 128 bytes a group) so that no two lanes share a
    // bank: span 1 writes lanes RP elements apart, which one spare per 16
    // elements spreads over all banks; spans 2 ... 8 write runs of lp elements
    // RP lp apart, which lp spares per RP lp elements stagger; from span 16 on the
    // runs are contiguous and need none.  Every form is additive over the
    // thread's register offsets (r lp, r TPF for TPF a multiple of 8 lp), so
    // they fold into immediate offsets, and stays below P + P/8.
    __host__ __device__ static int xpad(int rp, int lp, int i) {
        if (lp == 1) return i + (i >> 4);
        if (lp < 16) {
            const int sh = ilog2_rt(rp * lp), sl = ilog2_rt(lp);
            return i + ((i >> sh) << sl);
        }
        return i;
    }
    // radix and span of the writes of the exchange that feeds stage s (>= 1)
    __host__ __device__ static int xrp(int s) { return s == 1 ? R0 : PPT; }
    __host__ __device__ static int xlp(int s) { return s == 1 ? 1 : span(s - 1); }

    // write the outputs of stage s-1 of sequence f at their positions
    template <int RP>
    __host__ __device__ static void write_r(int lp, const cf (&v)[NF][PPT], int f, cf* buf, int t) {
#pragma unroll
        for (int uu = 0; uu < PPT / RP; ++uu) {
            const int j = t + TPF * uu;
            const int k = j & (lp - 1);
            const int base = (j - k) * RP + k;
#pragma unroll
            for (int r = 0; r < RP; ++r) buf[xpad(RP, lp, base + r * lp)] = v[f][uu * RP + r];
        }
    }
    __host__ __device__ static void write(int s, const cf (&v)[NF][PPT], int f, cf* buf, int t) {
        if (s == 1)
            write_r<R0>(1, v, f, buf, t);
        else
            write_r<PPT>(span(s - 1), v, f, buf, t);
    }

    // read the inputs of stage s (>= 1) for sequence f
    __host__ __device__ static void read(int s, cf (&v)[NF][PPT], int f, const cf* buf, int t) {
        const int rp = xrp(s), lp = xlp(s);
#pragma unroll
        for (int r = 0; r < PPT; ++r) v[f][r] = buf[xpad(rp, lp, t + r * TPF)];
    }
    // twiddle and butterfly of stage s (>= 1) for sequence f
    __host__ __device__ static void compute(cf (&v)[NF][PPT], int f, const cf (&wt)[PPT]) {
#pragma unroll
        for (int r = 1; r < PPT; ++r) v[f][r] = cmul(v[f][r], wt[r]);
        Dft<PPT, INV>::run(v[f]);
    }
    __host__ __device__ static void read_compute(int s, cf (&v)[NF][PPT], int f, const cf* buf, int t,
                                                 const cf (&wt)[PPT]) {
        read(s, v, f, buf, t);
        compute(v, f, wt);
    }

    // stage order of the last stage -> natural order
    __host__ __device__ static void finish(cf (&v)[NF][PPT]) {
        constexpr int RL = NS == 1 ? R0 : PPT;
        if (RL == 1) return;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cf w[PPT];
#pragma unroll
            for (int u = 0; u < PPT / RL; ++u)
#pragma unroll
                for (int r = 0; r < RL; ++r) w[u + r * (PPT / RL)] = v[f][u * RL + r];
#pragma unroll
            for (int i = 0; i < PPT; ++i) v[f][i] = w[i];
        }
    }

    // With NF > 1 the butterfly of sequence f - 1 runs between the LDS writes
    // of sequence f and the barrier that publishes them, so it covers their
    // latency and the wait at the barrier.
    __device__ static void run(cf (&v)[NF][PPT], cf* buf, const cf* __restrict__ tw, int twshift, int t) {
        if (NS == 0) return;
        stage0(v);
#pragma unroll
        for (int s = 1; s < NS; ++s) {
            cf wt[PPT];
            twiddles(s, t, tw, twshift, wt);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                __syncthreads();
                if (s == 1)
                    write_r<R0>(1, v, f, buf, t);
                else
                    write_r<PPT>(span(s - 1), v, f, buf, t);
                if (f > 0) compute(v, f - 1, wt);
                __syncthreads();
                read(s, v, f, buf, t);
            }
            compute(v, NF - 1, wt);
        }
        finish(v);
    }
};

}  // namespace mm
