// fft_passes.h -- the device bodies of the FP32 convolution passes.
//
// Section "Magnetostatic field": B_demag = K * M evaluated with the
// convolution theorem on a grid zero-padded to px x py x pz.
//
// Spectrum layout (complex64): element (z, kx, y, c) at
//   z * zstride + kx * colstride + y * 3 + c,  zstride = 3 * ycount,
//   colstride = nz * zstride (kx-major: the planes of one kx are adjacent),
// ycount = py in 3D grids whose y transforms run in place, else ny.  Every
// column along y is contiguous, so the column passes read and write whole
// columns.
//
// The three real components of two x-rows a, b travel as three complex
// "slots": slot 0 = Mx_a + i My_a, slot 1 = Mx_b + i My_b, slot 2 = Mz_a + i Mz_b.
// Each thread owns one slot (or one component in the column passes), so a
// row pair or a column is spread over three thread groups.
//
// Passes:
//   x-forward : one slot of one row pair per thread group: stage combine
//               m_s = m0 + dt sum a k, M = Msat[region] m_s, FFT along x of
//               the zero-padded rows, separation of the two real transforms
//               X = (Z[k] + conj Z[P-k])/2, Y = (Z[k] - conj Z[P-k])/(2i);
//   column    : per column, one thread group per component: FFT along y (3D:
//               forward and inverse around the z pass), or forward FFT,
//               B^_i = sum_j K^_ij M^_j through LDS (K^ real symmetric, one
//               octant stored, mirror signs applied), inverse FFT.  In 2D the
//               DC and Nyquist columns (both real along y) share one complex
//               column;
//   x-inverse : the three slots of a row pair: Hermitian extension, inverse
//               FFT, crop, then the per-cell epilogue (exchange, anisotropy,
//               Zeeman, torque, error norm, energies).
// The 1/(px py pz) normalisation and -mu0 are folded into K^.
#pragma once

#include "field_epilogue.h"

namespace mm {

template <int P>
struct Cfg {
    static constexpr int PPT = P < 8 ? P : (P >= 4096 ? 16 : 8);  // points per thread
    static constexpr int TPF = P / PPT;                           // threads per sequence
    static constexpr int G = TPF >= 256 ? 1 : 256 / TPF;          // sequences per 256 threads
};

// x passes: the 3 slots of GI row pairs per workgroup.  GL = LDS elements per
// row pair: the three exchange sequences, reused afterwards as the staging
// area [kx][row][component] through which the spectrum is written / read in
// contiguous runs (rows a, b are adjacent in the spectrum when a is even).
// W = 0: wide workgroups (768 threads for P <= 2048); W = 1: narrow ones of
// about 192 threads, for grids with too few rows to give every CU two wide
// workgroups.
template <int P, int W = 0>
struct XCfg {
    static constexpr int TPF = Cfg<P>::TPF;
    static constexpr int GIW = TPF >= 256 ? 1 : (TPF >= 128 ? 2 : 256 / TPF);
    static constexpr int GIN = TPF >= 64 ? 1 : 64 / TPF;
    static constexpr int GI = (W && GIN < GIW) ? GIN : GIW;
    static constexpr int NTH = 3 * GI * Cfg<P>::TPF;
    static constexpr int KH = P / 2 + 1;
    static constexpr int GL = 3 * seq_len(P) > 6 * KH ? 3 * seq_len(P) : 6 * KH;
};

// columns: the 3 components of T columns per workgroup
template <int P>
struct ColCfg {
    static constexpr int T = Cfg<P>::TPF >= 256 ? 1 : (Cfg<P>::TPF >= 128 ? 2 : 256 / Cfg<P>::TPF);
    static constexpr int NTH = 3 * T * Cfg<P>::TPF;
};

// 2D convolution: the K^ octant rows (xx, yy, zz, xy) of the workgroup's T
// columns, staged in LDS after the exchange buffers (bytes)
template <int P>
constexpr size_t khat_lds() {
    return (size_t)ColCfg<P>::T * (P / 2 + 1) * sizeof(float4);
}

__device__ inline long long row_base(const FieldArgs& a, int row) {
    const int z = row / a.ny, y = row - z * a.ny;
    return (long long)z * a.zstride + 3LL * y;
}

// Spectrum offsets of the 2 GI rows of a workgroup (-1 past the grid), into
// LDS by the first threads; the cooperative copies read them after a barrier.
template <int GI>
__device__ inline void row_bases(const FieldArgs& a, int pair0, long long* rbs, int tid) {
    if (tid < 2 * GI) {
        const int row = 2 * pair0 + tid;
        rbs[tid] = row < a.nrows ? row_base(a, row) : -1;
    }
}

// Cooperative copy between a workgroup's staged half spectra
// [pair][kx][row][component] (6 complex per kx) in LDS and the spectrum:
// thread tid handles the elements u = tid + NTH i.  NTH is a multiple of 6, so
// the (row, component) of a thread's elements is fixed and kx advances by
// NTH/6 per step; offsets need no division per element.
template <int P, int W = 0>
struct Staged {
    static constexpr int GI = XCfg<P, W>::GI, NTH = XCfg<P, W>::NTH, KH = XCfg<P, W>::KH, GL = XCfg<P, W>::GL;
    static constexpr int TOT = GI * KH * 6, NIT = (TOT + NTH - 1) / NTH, KS = NTH / 6;
    static_assert(NTH % 6 == 0, "workgroup size must be a multiple of 6");
    int comp, h, kq0;
    __device__ explicit Staged(int tid) {
        const int rc = tid % 6;
        h = rc >= 3 ? 1 : 0;
        comp = rc - 3 * h;
        kq0 = tid / 6;
    }
    // element i of the thread: LDS index, and spectrum offset (-1: no element,
    // or its row is past the grid)
    __device__ void at(const FieldArgs& a, const long long* rbs, int i, int& lidx, long long& off) const {
        const int kq = kq0 + KS * i;
        const int gg = GI == 1 ? 0 : kq / KH;
        const int k = kq - gg * KH;
        lidx = gg * GL + 6 * k + 3 * h + comp;
        const bool in = i < NIT - 1 || kq < GI * KH;
        const long long rb = rbs[2 * gg + h];
        off = (in && rb >= 0) ? rb + (long long)k * a.colstride + comp : -1;
    }
};

// ---------------------------------------------------------------------------
// x passes.  Both stage the region table in LDS after the row-pair area.
template <int P, int W = 0>
struct XLut {
    static constexpr int NTH = XCfg<P, W>::NTH;
    static constexpr int NL4 = NREG * (int)(sizeof(RegionLut) / sizeof(float4));
    static constexpr int NLI = (NL4 + NTH - 1) / NTH;
    float4 lt[NLI];
    __device__ void load(const FieldArgs& a, int tid) {
#pragma unroll
        for (int i = 0; i < NLI; ++i)
            lt[i] = tid + NTH * i < NL4 ? reinterpret_cast<const float4*>(a.lut)[tid + NTH * i]
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __device__ void store(RegionLut* lut_l, int tid) const {
#pragma unroll
        for (int i = 0; i < NLI; ++i)
            if (tid + NTH * i < NL4) reinterpret_cast<float4*>(lut_l)[tid + NTH * i] = lt[i];
    }
};

// In the fused pass the torque of the finished stage is handed to the next
// stage's combine through LDS.  Padded x: component c of a row pair's two rows
// ([row][x], floats) in the upper half of slot buffer c, which the x-inverse
// results (x < nx <= P/2, the lower half) leave free.  Unpadded periodic x
// (FULL: nx = P, no free half): in place of the cell's own x-inverse result,
// which only that cell's epilogue reads (components x, y of row rr in slot
// rr; z of both rows in slot 2, row rr in its float rr).  Needs P >= 2.
template <int P>
__device__ inline float* ks_stage(cf* gbuf, int c) {
    return reinterpret_cast<float*>(gbuf + c * seq_len(P) + seq_len(P) / 2);
}
template <int P, bool FULL>
__device__ inline float* k_slot(cf* gbuf, int c, int rr, int x, int nx) {
    if constexpr (FULL) {
        if (c < 2) return reinterpret_cast<float*>(gbuf + rr * seq_len(P) + lds_pad(x)) + c;
        return reinterpret_cast<float*>(gbuf + 2 * seq_len(P) + lds_pad(x)) + rr;
    } else {
        return ks_stage<P>(gbuf, c) + rr * nx + x;
    }
}

// Forward x pass of one workgroup: stage combine m_s = m0 + dt sum a k (FUSED:
// plus dt a_last k_last, k_last from LDS), M = Msat[region] m_s, FFT of the
// zero-padded rows, separation of the two real transforms, staged coalesced
// spectrum write.  The region table is in LDS at lut_l once the first barrier
// has passed (the non-fused pass writes it from lut after issuing its loads).
template <int P, bool FUSED, bool FULL = false, int XW = 0>
__device__ inline void xfwd_part(const FieldArgs& a, const Resolved& rs, cf* lds, const long long* rbs,
                                 RegionLut* lut_l, const XLut<P, XW>* lut, float a_last, int blk, int tid) {
    constexpr int PPT = Cfg<P>::PPT, TPF = Cfg<P>::TPF, GI = XCfg<P, XW>::GI;
    constexpr int SEQ = seq_len(P), GL = XCfg<P, XW>::GL;
    constexpr int MH = PPT / 2 + 1;
    // in the fused pass, derive every index afresh here (nothing of the first
    // part stays live across the boundary)
    if constexpr (FUSED) asm volatile("" : "+v"(tid)::"memory");
    const int t = tid % TPF, slot = (tid / TPF) % 3, g = tid / (3 * TPF);
    const int pair0 = blk * GI;
    const int pair = pair0 + g;
    const int ra = 2 * pair, rb = ra + 1;
    const bool va = ra < a.nrows, vb = rb < a.nrows;
    cf* gbuf = lds + g * GL;
    cf* buf = gbuf + slot * SEQ;
    const long long n = a.ncell;

    // slot 0: (x, y) of row a, slot 1: (x, y) of row b, slot 2: z of rows a and b
    const int r0 = slot == 1 ? rb : ra;
    const bool v0 = slot == 1 ? vb : va;
    const int c0 = slot == 2 ? 2 : 0;
    const int r1 = slot == 0 ? ra : rb;
    const bool v1 = slot == 0 ? va : vb;
    const int c1 = slot == 2 ? 2 : 1;
    const int rr0 = slot == 1 ? 1 : 0, rr1 = slot == 0 ? 0 : 1;  // rows within the pair

    // Only x < P/2 can hold cells (P >= 2 nx - 1), except along an unpadded
    // periodic axis (FULL: P = nx); rows and columns past the grid are clamped
    // for the loads and masked afterwards, so every load of the thread is
    // issued before the first one is used.
    constexpr int MV = FULL ? PPT : (PPT > 1 ? PPT / 2 : 1);
    const int r0c = v0 ? r0 : 0, r1c = v1 ? r1 : 0;
    cf v[1][PPT];
#pragma unroll
    for (int m = MV; m < PPT; ++m) v[0][m] = mkc(0.f, 0.f);
    unsigned int idx0[MV], idx1[MV];  // byte offsets into the [3][ncell] arrays
    int g0[MV], g1[MV];
#pragma unroll
    for (int m = 0; m < MV; ++m) {
        const int x = t + TPF * m;
        const int xc = x < a.nx ? x : a.nx - 1;
        const unsigned int cell0 = (unsigned int)(r0c * a.nx + xc), cell1 = (unsigned int)(r1c * a.nx + xc);
        idx0[m] = (c0 * (unsigned int)n + cell0) << 2;
        idx1[m] = (c1 * (unsigned int)n + cell1) << 2;
        g0[m] = a.region[cell0];
        g1[m] = a.region[cell1];
    }
    // two batches (one per component) bound the loads in flight per thread
    float sv[2 * MV];
    {
        float s0[MV], s1[MV];
        stage_batch(a, rs, idx0, s0);
        stage_batch(a, rs, idx1, s1);
#pragma unroll
        for (int m = 0; m < MV; ++m) {
            sv[m] = s0[m];
            sv[MV + m] = s1[m];
        }
    }
    if constexpr (FUSED) {
        // the last term of the combine, k of the stage the x-inverse part of
        // this workgroup just finished (after the barrier that published it)
        const float w = rs.dt * a_last;
#pragma unroll
        for (int m = 0; m < MV; ++m) {
            const int x = t + TPF * m;
            const int xc = x < a.nx ? x : a.nx - 1;
            sv[m] += w * *k_slot<P, FULL>(gbuf, c0, rr0, xc, a.nx);
            sv[MV + m] += w * *k_slot<P, FULL>(gbuf, c1, rr1, xc, a.nx);
        }
    } else {
        lut->store(lut_l, tid);
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < MV; ++m) {
        const int x = t + TPF * m;
        const bool in = x < a.nx;
        if (a.sd.nk > 0 || FUSED) {
            if (in && v0) sto(a.ms, idx0[m], sv[m]);
            if (in && v1) sto(a.ms, idx1[m], sv[MV + m]);
        }
        const float re = (in && v0) ? lut_l[g0[m]].a.x * sv[m] : 0.f;
        const float im = (in && v1) ? lut_l[g1[m]].a.x * sv[MV + m] : 0.f;
        v[0][m] = mkc(re, im);
    }
    // x >= nx is zero padding (nx <= P/2) unless the axis is unpadded
    RegFft<P, TPF, 1, false, (P >= 2 && !FULL)>::run(v, buf, a.tw, a.twshift, t);

    // separate the two real transforms of this slot
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PPT; ++m) buf[lds_pad(t + TPF * m)] = v[0][m];
    __syncthreads();
    cf X[MH], Y[MH];
#pragma unroll
    for (int m = 0; m < MH; ++m) {
        const int k = t + TPF * m;
        const cf z = v[0][m < PPT ? m : 0];
        const cf w = cconj(buf[lds_pad((P - k) & (P - 1))]);
        const cf d = z - w;
        X[m] = 0.5f * (z + w);
        Y[m] = mkc(0.5f * d.y, -0.5f * d.x);
    }
    __syncthreads();
    // stage [kx][row][component] and write the runs of 6 complex per kx
#pragma unroll
    for (int m = 0; m < MH; ++m) {
        const int k = t + TPF * m;
        if (2 * k > P) continue;
        if (slot == 2) {
            gbuf[k * 6 + 2] = X[m];
            gbuf[k * 6 + 5] = Y[m];
        } else {
            gbuf[k * 6 + slot * 3] = X[m];
            gbuf[k * 6 + slot * 3 + 1] = Y[m];
        }
    }
    __syncthreads();
    const Staged<P, XW> sc(tid);
#pragma unroll
    for (int i = 0; i < Staged<P, XW>::NIT; ++i) {
        int li;
        long long off;
        sc.at(a, rbs, i, li, off);
        if (off >= 0) a.spec[off] = lds[li];
    }
}

// Inverse x pass of one workgroup: staged coalesced spectrum read, Hermitian
// extension, inverse FFT, crop, per-cell epilogue (FUSED: the torque also to
// LDS for the next stage's combine), reductions.  The region table goes to
// LDS at lut_l.  A run that already reached its end (EPI_CHECK_DONE) stops
// once the staged spectrum is in LDS, before anything is written to global
// memory, and the call returns false: the solver-state read behind the test
// then overlaps the spectrum loads instead of preceding them.
template <int P, bool FUSED, bool DMI = false, bool FULL = false, int XW = 0>
__device__ inline bool xinv_part(const FieldArgs& a, const Resolved& rs, cf* lds, const long long* rbs,
                                 RegionLut* lut_l, double* red, int blk, int tid) {
    constexpr int PPT = Cfg<P>::PPT, TPF = Cfg<P>::TPF, GI = XCfg<P, XW>::GI, NTH = XCfg<P, XW>::NTH;
    constexpr int SEQ = seq_len(P), GL = XCfg<P, XW>::GL;
    constexpr int MH = PPT / 2 + 1;
    const int t = tid % TPF, slot = (tid / TPF) % 3, g = tid / (3 * TPF);
    const int pair0 = blk * GI;
    cf* gbuf = lds + g * GL;
    cf* buf = gbuf + slot * SEQ;

    XLut<P, XW> lut;
    lut.load(a, tid);
    // read the half spectra of the row pairs in contiguous runs into
    // [kx][row][component]: every load of the thread first, then the LDS writes
    const Staged<P, XW> sc(tid);
    constexpr int NIT = Staged<P, XW>::NIT;
    cf tmp[NIT];
    int li[NIT];
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        long long off;
        sc.at(a, rbs, i, li[i], off);
        tmp[i] = off >= 0 ? a.spec[off] : mkc(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < NIT; ++i)
        if (i < NIT - 1 || sc.kq0 + Staged<P, XW>::KS * i < Staged<P, XW>::GI * XCfg<P, XW>::KH) lds[li[i]] = tmp[i];
    lut.store(lut_l, tid);
    __syncthreads();
    if ((a.flags & EPI_CHECK_DONE) && rs.done) return false;
    // slot s = u + i w (slot 0: x, y of row a; slot 1: x, y of row b; slot 2: z of
    // rows a and b); the DC and Nyquist bins of a real signal are real
    const int iu = slot == 2 ? 2 : slot * 3, iw = slot == 2 ? 5 : slot * 3 + 1;
    cf U[MH], W[MH];
#pragma unroll
    for (int m = 0; m < MH; ++m) {
        const int k = t + TPF * m;
        const int kc = 2 * k <= P ? k : 0;
        U[m] = gbuf[kc * 6 + iu];
        W[m] = gbuf[kc * 6 + iw];
        if (k == 0 || 2 * k == P) {
            U[m].y = 0.f;
            W[m].y = 0.f;
        }
    }
    __syncthreads();
    // Hermitian extension: Z[k] = u + i w, Z[P-k] = conj u + i conj w for k <= P/2
#pragma unroll
    for (int m = 0; m < MH; ++m) {
        const int k = t + TPF * m;
        if (2 * k > P) continue;
        const cf u = U[m], w = W[m];
        buf[lds_pad(k)] = mkc(u.x - w.y, u.y + w.x);
        if (k != 0 && 2 * k != P) buf[lds_pad(P - k)] = mkc(u.x + w.y, w.x - u.y);
    }
    __syncthreads();
    cf v[1][PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) v[0][m] = buf[lds_pad(t + TPF * m)];
    RegFft<P, TPF, 1, true>::run(v, buf, a.tw, a.twshift, t);
    // only x < nx <= P/2 is kept (every x along an unpadded periodic axis)
    constexpr int MOUT = (P >= 2 && !FULL) ? PPT / 2 : PPT;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MOUT; ++m) buf[lds_pad(t + TPF * m)] = v[0][m];
    __syncthreads();

    // per-cell epilogue over the 2 GI rows of this workgroup
    EpiAcc acc;
    epi_init(acc);
    const float* mp = a.sd.nk > 0 || FUSED ? a.ms : a.m0;
    // one cell of row rr at x; rows past the grid are skipped
    auto cell = [&](int rr, int x, int y, int z) {
        cf* b3 = lds + (rr >> 1) * GL;
        const cf v01 = b3[(rr & 1) * SEQ + lds_pad(x)];
        const cf v2 = b3[2 * SEQ + lds_pad(x)];
        const int row = 2 * pair0 + rr;
        const float3 tq = epilogue<DMI>(a, rs, lut_l, mp, (long long)row * a.nx + x, x, y, z,
                                   make_float3(v01.x, v01.y, (rr & 1) ? v2.y : v2.x), acc);
        if constexpr (FUSED) {
            *k_slot<P, FULL>(b3, 0, rr & 1, x, a.nx) = tq.x;
            *k_slot<P, FULL>(b3, 1, rr & 1, x, a.nx) = tq.y;
            *k_slot<P, FULL>(b3, 2, rr & 1, x, a.nx) = tq.z;
        }
    };
    constexpr int NROW = 2 * GI;
    if constexpr (NTH % NROW == 0) {
        // NTH / NROW threads per row: the row (and its y, z) is fixed per
        // thread, x advances by a compile-time stride
        constexpr int TR = NTH / NROW;
        const int rr = tid / TR, x0 = tid - rr * TR;
        const int row = 2 * pair0 + rr;
        if (row < a.nrows) {
            const int z = row / a.ny, y = row - z * a.ny;
            for (int x = x0; x < a.nx; x += TR) cell(rr, x, y, z);
        }
    } else {
        for (int idx = tid; idx < NROW * a.nx; idx += NTH) {
            const int rr = idx / a.nx, x = idx - rr * a.nx;
            const int row = 2 * pair0 + rr;
            if (row >= a.nrows) continue;
            const int z = row / a.ny, y = row - z * a.ny;
            cell(rr, x, y, z);
        }
    }
    // the fused pass serves inner stages only (no error norm, no reductions)
    if constexpr (!FUSED)
        if (a.flags & (EPI_ERR | EPI_MAXTQ | EPI_ENERGY)) epi_reduce<NTH>(a, acc, red, blk);
    return true;
}

// ---------------------------------------------------------------------------
// Column pass.  Threads: (column ci < T, component s < 3, t < TPF); with
// CFAST the column index varies fastest over the lanes (strided columns, so
// neighbouring lanes read neighbouring columns), else t does (contiguous
// columns).
// LDS elements per sequence of the column pass.  With CFAST the lanes of a
// wave walk different sequences at the same position, so the sequence stride
// is made odd: consecutive sequences then start in different LDS banks (an
// even stride such as 144 would put every other lane on the same banks).
template <int P, bool CFAST>
constexpr int col_seq() {
    return CFAST ? (seq_len(P) | 1) : seq_len(P);
}

// The 3D z convolution pairs the columns ky and py - ky in one tile (the
// first half of the tile's columns take kyh = ky <= py/2, the second half
// their mirrors), so each K^ block is loaded once; kyh = 0 and py/2 have no
// distinct mirror.  Tiles per outer index:
template <int P, int MODE, int NC>
constexpr bool col_pairs() {
    return MODE == COL_CONV && NC == 6 && ColCfg<P>::T >= 2;
}
template <int P, int MODE, int NC>
__host__ __device__ constexpr int col_ntile(int ncol) {
    constexpr int T = ColCfg<P>::T;
    return col_pairs<P, MODE, NC>() ? (ncol / 2 + T / 2) / (T / 2) : (ncol + T - 1) / T;
}

template <int P, int MODE, int NC, bool CFAST>
__device__ inline void col_body(const ColArgs& a, int blk, cf* lds, int tid) {
    constexpr int PPT = Cfg<P>::PPT, TPF = Cfg<P>::TPF, T = ColCfg<P>::T;
    constexpr int SEQ = col_seq<P, CFAST>();
    constexpr bool PAIR = col_pairs<P, MODE, NC>();
    constexpr int TH = PAIR ? T / 2 : T;  // K^ blocks per tile
    // a finished run is tested after the forward transform (nothing is
    // written before), so the state read overlaps the column loads
    const int done = a.check_done ? a.st->done : 0;
    int ci, s, t;
    if (CFAST) {
        s = tid % 3;
        ci = (tid / 3) % T;
        t = tid / (3 * T);
    } else {
        t = tid % TPF;
        s = (tid / TPF) % 3;
        ci = tid / (3 * TPF);
    }
    const int ntile = col_ntile<P, MODE, NC>(a.ncol);
    const int o = blk / ntile, tile = blk - o * ntile;
    int c;
    bool valid;
    if constexpr (PAIR) {
        const int kh = tile * TH + (ci % TH);
        const bool mir = ci >= TH;
        c = mir ? a.ncol - kh : kh;
        valid = 2 * kh <= a.ncol && !(mir && (kh == 0 || 2 * kh == a.ncol));
    } else {
        c = tile * T + ci;
        valid = c < a.ncol;
    }
    // 2D convolution: column 0 carries kx = 0 (real part) and kx = px/2 (imaginary part)
    const bool packed = MODE == COL_CONV && NC == 4 && a.pack_col > 0 && c == 0;
    // the workgroup's outer slab (uniform) and 32-bit element offsets within
    // it: a slab of the spectrum (at most 2048 x 4096 x 3 complex for the
    // largest grids) stays far below 2^32 bytes
    cf* obase = a.spec + (long long)o * a.outer_stride;
    const unsigned int coff = (unsigned int)(valid ? c : 0) * (unsigned int)a.col_stride;
    const unsigned int noff = (unsigned int)a.pack_col * (unsigned int)a.col_stride;  // from a.spec
    cf* bufs = lds + ci * 3 * SEQ;
    cf* buf = bufs + s * SEQ;

    // A padded axis has P >= 2 n: the forward transforms read only q < P/2
    // (the rest is zero padding) and the cropped outputs are q < P/2.
    constexpr bool HIN = MODE != COL_INV && P >= 2;
    constexpr int MIN = HIN ? PPT / 2 : PPT;
    constexpr int MOUT = (MODE != COL_FWD && P >= 2) ? PPT / 2 : PPT;
    cf v[1][PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int q = t + TPF * m;
        const bool ld = m < MIN && valid && q < a.n_in;
        const unsigned int off = (unsigned int)q * (unsigned int)a.pos_stride + (unsigned int)s;
        cf x = ld ? ld_cf(obase, (coff + off) * 8u) : mkc(0.f, 0.f);
        if (packed) x = mkc(x.x, ld ? ld_cf(a.spec, (noff + off) * 8u).x : 0.f);
        v[0][m] = x;
    }
    // 2D convolution: the K^ rows of the workgroup's columns go to LDS now, so
    // their latency overlaps that of the column loads (K^ column kx is
    // contiguous: (P/2 + 1) rows of 4 floats)
    constexpr int KHP = P / 2 + 1;
    float4* lk = reinterpret_cast<float4*>(lds + T * 3 * SEQ);
    if constexpr (MODE == COL_CONV && NC == 4) {
        constexpr int TOT = T * KHP, NTH = ColCfg<P>::NTH, NIT = (TOT + NTH - 1) / NTH;
        const float4* kh = reinterpret_cast<const float4*>(a.khat);
        const int c0 = (blk - o * ntile) * T;
        float4 kt[NIT];
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int e = tid + NTH * i;
            const int ce = e / KHP, r = e - ce * KHP;
            const bool in = (i < NIT - 1 || e < TOT) && c0 + ce < a.ncol;
            kt[i] = in ? kh[(long long)(c0 + ce) * KHP + r] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int e = tid + NTH * i;
            if (i < NIT - 1 || e < TOT) lk[e] = kt[i];
        }
    }
    // 3D z convolution: the K^ blocks of the tile's (kx, ky) columns (all kz,
    // 6 components, contiguous per column) go to LDS the same way
    float* lk6 = reinterpret_cast<float*>(lds + T * 3 * SEQ);
    if constexpr (MODE == COL_CONV && NC == 6) {
        constexpr int BL = KHP * 3;  // float2 per column block
        constexpr int TOT = TH * BL, NTH = ColCfg<P>::NTH, NIT = (TOT + NTH - 1) / NTH;
        // the kx slab of K^ (uniform) and 32-bit offsets within it
        const cf* kslab = reinterpret_cast<const cf*>(a.khat + (long long)o * a.kyh * (KHP * 6));
        float2 kt[NIT];
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int e = tid + NTH * i;
            const int ce = e / BL, r = e - ce * BL;
            int kyh;
            bool in;
            if constexpr (PAIR) {
                kyh = tile * TH + ce;
                in = (i < NIT - 1 || e < TOT) && 2 * kyh <= a.pa;
            } else {
                const int cy = tile * T + ce;
                in = (i < NIT - 1 || e < TOT) && cy < a.ncol;
                kyh = 2 * cy > a.pa ? a.pa - cy : cy;
            }
            const cf kv = in ? ld_cf(kslab, (unsigned int)(kyh * BL + r) * 8u) : mkc(0.f, 0.f);
            kt[i] = make_float2(kv.x, kv.y);
        }
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int e = tid + NTH * i;
            if (i < NIT - 1 || e < TOT) reinterpret_cast<float2*>(lk6)[e] = kt[i];
        }
    }
    RegFft<P, TPF, 1, MODE == COL_INV, HIN>::run(v, buf, a.tw, a.twshift, t);
    if (done) return;

    if (MODE == COL_CONV) {
        // all three components of this column through LDS
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PPT; ++m) buf[lds_pad(t + TPF * m)] = v[0][m];
        __syncthreads();
        // 2D: column c is kx and the transform runs along y.
        // 3D: outer o is kx, column c is ky, the transform runs along z.
        int kx = NC == 6 ? o : c;
        asm volatile("" : "+v"(kx));  // load K^ here, not before the forward transform
        int kyh = 0;
        bool fa = false;
        if (NC == 6) {
            kyh = c;
            if (2 * c > a.pa) {
                kyh = a.pa - c;
                fa = true;
            }
        }
        if constexpr (NC == 6) {
            // 3D: row s of the symmetric K^ (from the tile's blocks in LDS): s = 0
            // (xx, xy, xz), 1 (xy, yy, yz), 2 (xz, yz, zz); xy is odd in y, xz
            // odd in z, yz odd in both
            const int j0 = s == 0 ? 0 : (s == 1 ? 3 : 4);
            const int j1 = s == 0 ? 3 : (s == 1 ? 1 : 5);
            const int j2 = s == 0 ? 4 : (s == 1 ? 5 : 2);
            auto odd_y = [](int j) { return j == 3 || j == 5; };
            auto odd_z = [](int j) { return j == 4 || j == 5; };
            const float* Kb = lk6 + (ci % TH) * KHP * 6;
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                const int q = t + TPF * m;
                const bool fq = 2 * q > P;
                const float* K = Kb + (fq ? P - q : q) * 6;
                const float s0 = ((fa && odd_y(j0)) != (fq && odd_z(j0))) ? -1.f : 1.f;
                const float s1 = ((fa && odd_y(j1)) != (fq && odd_z(j1))) ? -1.f : 1.f;
                const float s2 = ((fa && odd_y(j2)) != (fq && odd_z(j2))) ? -1.f : 1.f;
                const cf m0 = bufs[lds_pad(q)], m1 = bufs[SEQ + lds_pad(q)], m2 = bufs[2 * SEQ + lds_pad(q)];
                const cf b = (s0 * K[j0]) * m0 + (s1 * K[j1]) * m1 + (s2 * K[j2]) * m2;
                v[0][m] = valid ? b : mkc(0.f, 0.f);
            }
        } else {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            const int q = t + TPF * m;
            int qh = q;
            bool fq = false;
            if (2 * q > P) {
                qh = P - q;
                fq = true;
            }
            // row s of the symmetric K^ at (kxx, ky, q), with the mirror signs
            // (2D: column kxx == c of this thread is staged in LDS)
            auto krow = [&](int kxx) {
                float3 r = make_float3(0.f, 0.f, 0.f);
                if (!valid) return r;
                float k0, k1, k2, kxy, kxz = 0.f, kyz = 0.f;
                if (NC == 4 && kxx == c) {
                    const float4 k4 = lk[ci * KHP + qh];
                    k0 = k4.x;
                    k1 = k4.y;
                    k2 = k4.z;
                    kxy = k4.w;
                } else if (NC == 6) {
                    const float* K = lk6 + ((ci % TH) * KHP + qh) * 6;
                    k0 = K[0];
                    k1 = K[1];
                    k2 = K[2];
                    kxy = K[3];
                    kxz = K[4];
                    kyz = K[5];
                } else {
                    const float* K = a.khat + (((long long)kxx * a.kyh + kyh) * a.kzh + qh) * NC;
                    k0 = K[0];
                    k1 = K[1];
                    k2 = K[2];
                    kxy = K[3];
                    if (NC == 6) {
                        kxz = K[4];
                        kyz = K[5];
                    }
                }
                if (NC == 6) {
                    if (fq) {  // z: xz and yz are odd in z
                        kxz = -kxz;
                        kyz = -kyz;
                    }
                    if (fa) {  // y: xy and yz are odd in y
                        kxy = -kxy;
                        kyz = -kyz;
                    }
                } else if (fq) {  // y: xy is odd in y
                    kxy = -kxy;
                }
                if (s == 0)
                    r = make_float3(k0, kxy, kxz);
                else if (s == 1)
                    r = make_float3(kxy, k1, kyz);
                else
                    r = make_float3(kxz, kyz, k2);
                return r;
            };
            const cf m0 = bufs[lds_pad(q)], m1 = bufs[SEQ + lds_pad(q)], m2 = bufs[2 * SEQ + lds_pad(q)];
            if (!packed) {
                const float3 K = krow(kx);
                v[0][m] = K.x * m0 + K.y * m1 + K.z * m2;
            } else {
                // Z = A0 + i AN with A0, AN real along y: A0^(k) = (Z(k) + conj Z(-k))/2,
                // AN^(k) = (Z(k) - conj Z(-k))/(2i); both field columns stay real, so
                // B0^ + i BN^ recombines them.
                const int qn = (P - q) & (P - 1);
                const cf n0 = cconj(bufs[lds_pad(qn)]), n1 = cconj(bufs[SEQ + lds_pad(qn)]),
                         n2 = cconj(bufs[2 * SEQ + lds_pad(qn)]);
                const cf a00 = 0.5f * (m0 + n0), a01 = 0.5f * (m1 + n1), a02 = 0.5f * (m2 + n2);
                const cf d0 = m0 - n0, d1 = m1 - n1, d2 = m2 - n2;
                const cf an0 = mkc(0.5f * d0.y, -0.5f * d0.x), an1 = mkc(0.5f * d1.y, -0.5f * d1.x),
                         an2 = mkc(0.5f * d2.y, -0.5f * d2.x);
                const float3 K0 = krow(0), KN = krow(a.pack_col);
                const cf b0 = K0.x * a00 + K0.y * a01 + K0.z * a02;
                const cf bn = KN.x * an0 + KN.y * an1 + KN.z * an2;
                v[0][m] = mkc(b0.x - bn.y, b0.y + bn.x);
            }
        }
        }
        RegFft<P, TPF, 1, true>::run(v, buf, a.tw, a.twshift, t);
    }

    int t2 = t;
    asm volatile("" : "+v"(t2));  // form the store addresses here, not at load time
#pragma unroll
    for (int m = 0; m < MOUT; ++m) {
        const int q = t2 + TPF * m;
        if (valid && q < a.n_out) {
            const unsigned int off = (unsigned int)q * (unsigned int)a.pos_stride + (unsigned int)s;
            if (!packed) {
                st_cf(obase, (coff + off) * 8u, v[0][m]);
            } else {
                st_cf(obase, (coff + off) * 8u, mkc(v[0][m].x, 0.f));
                st_cf(a.spec, (noff + off) * 8u, mkc(v[0][m].y, 0.f));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 3D convolution of a thin grid (a few layers) in one pass per kx column:
// forward FFT along y of the three components of every z plane (the nz
// planes' sequences side by side in LDS), then for each ky the convolution
// along the short z axis done directly in real space, B(z') = sum_z
// G(z' - z) M(z), and the inverse FFT along y.  G(d) = sum_kz K^(kz)
// exp(+2 pi i kz d / PZ) is the kernel spectrum transformed back along z
// (zkernel_table below): real and even in d for xx, yy, zz, xy; imaginary and
// odd in d for xz, yz.  The spectrum keeps ny rows per column (ycount = ny);
// the padded y and z lengths live only on chip.
//
// Threads: for each of T kx columns, 3 PZ/2 thread groups (plane z, component
// c; planes z >= nz idle) of TPF threads.  Serves PZ in {4, 8} (nz from 2 to
// 4) and PY PZ <= 4096: the workgroup is 768 threads and its exchange LDS
// 55 KB for every such pair.  (More layers keep the three-pass path.)
template <int PY, int PZ>
struct YzCfg {
    static constexpr int TPF = Cfg<PY>::TPF, PPT = Cfg<PY>::PPT;
    static constexpr int NZM = PZ / 2;           // planes a thread group set can hold
    static constexpr int G = 3 * NZM;            // thread groups per column
    static constexpr int TK = G * TPF;           // threads per column
    static constexpr int T = 768 / TK;           // columns per workgroup
    static constexpr int NTH = T * TK;
    static constexpr int SEQ = seq_len(PY);
};

template <int PY, int PZ>
constexpr bool use_yz() {
    return (PZ == 4 || PZ == 8) && PY >= 16 && PY * PZ <= 4096;
}

template <int PY, int PZ>
constexpr size_t yz_lds() {
    return (size_t)YzCfg<PY, PZ>::T * YzCfg<PY, PZ>::G * YzCfg<PY, PZ>::SEQ * sizeof(cf);
}

// floats of the z-space kernel per (kx, ky_h): d = 0: xx, yy, zz, xy; each
// d = 1 .. PZ/2 - 1: xx, yy, zz, xy, Im xz, Im yz
constexpr int zkernel_len(int pz) { return 4 + 6 * (pz / 2 - 1); }

// a: spec, col_stride (between kx columns), outer_stride (between z planes),
// ncol (= kx count), nouter (= nz), n_in (= ny), khat (the z-space kernel
// [kx][ky_h][zkernel_len(PZ)]), kyh (= PY/2 + 1).
template <int PY, int PZ>
__device__ inline void yz_body(const ColArgs& a, int blk, cf* lds, int tid) {
    using C = YzCfg<PY, PZ>;
    constexpr int TPF = C::TPF, PPT = C::PPT, NZM = C::NZM, G = C::G, TK = C::TK, T = C::T, SEQ = C::SEQ;
    constexpr int MH = PPT / 2, NG = zkernel_len(PZ);
    static_assert(use_yz<PY, PZ>() && C::NTH == 768, "thin-grid convolution shape");
    if (a.check_done && a.st->done) return;
    const int kc = tid / TK, r = tid - kc * TK;
    const int g = r / TPF, t = r - g * TPF;
    const int z = g / 3, c = g - 3 * z;
    const int nz = a.nouter;
    const int kx = blk * T + kc;
    const bool valid = kx < a.ncol && z < nz;
    cf* col = a.spec + (long long)(kx < a.ncol ? kx : 0) * a.col_stride + (long long)(z < nz ? z : 0) * a.outer_stride + c;
    cf* buf = lds + (kc * G + g) * SEQ;

    // forward y transform of plane z, component c (rows y < ny <= PY/2)
    cf v[1][PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int q = t + TPF * m;
        v[0][m] = (m < MH && valid && q < a.n_in) ? col[3LL * q] : mkc(0.f, 0.f);
    }
    RegFft<PY, TPF, 1, false, true>::run(v, buf, a.tw, a.twshift, t);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PPT; ++m) buf[lds_pad(t + TPF * m)] = v[0][m];
    __syncthreads();

    // along z, one ky at a time: B(z') = sum_z G(z' - z) M(z)
    if (kx < a.ncol) {
        cf* cb = lds + kc * G * SEQ;
        for (int ky = r; ky < PY; ky += TK) {
            const bool fa = 2 * ky > PY;
            const float sy = fa ? -1.f : 1.f;  // xy and yz are odd in y
            const float* Gr = a.khat + ((long long)kx * a.kyh + (fa ? PY - ky : ky)) * NG;
            float gk[NG];
#pragma unroll
            for (int i = 0; i < NG; ++i) gk[i] = Gr[i];
            cf X[3][NZM];
#pragma unroll
            for (int zz = 0; zz < NZM; ++zz)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    X[cc][zz] = zz < nz ? cb[(3 * zz + cc) * SEQ + lds_pad(ky)] : mkc(0.f, 0.f);
#pragma unroll
            for (int zo = 0; zo < NZM; ++zo) {
                cf B0 = mkc(0.f, 0.f), B1 = mkc(0.f, 0.f), B2 = mkc(0.f, 0.f);
#pragma unroll
                for (int zi = 0; zi < NZM; ++zi) {
                    const int d = zo - zi, ad = d < 0 ? -d : d;
                    const float* e = gk + (ad == 0 ? 0 : 4 + 6 * (ad - 1));
                    const float kxx = e[0], kyy = e[1], kzz = e[2], kxy = sy * e[3];
                    const cf x0 = X[0][zi], x1 = X[1][zi], x2 = X[2][zi];
                    B0 = B0 + kxx * x0 + kxy * x1;
                    B1 = B1 + kxy * x0 + kyy * x1;
                    B2 = B2 + kzz * x2;
                    if (ad > 0) {
                        // i g: i (a + i b) = (-b, a)
                        const float sd = d > 0 ? 1.f : -1.f;
                        const float gxz = sd * e[4], gyz = sd * sy * e[5];
                        B0 = B0 + gxz * mkc(-x2.y, x2.x);
                        B1 = B1 + gyz * mkc(-x2.y, x2.x);
                        B2 = B2 + gxz * mkc(-x0.y, x0.x) + gyz * mkc(-x1.y, x1.x);
                    }
                }
                if (zo < nz) {
                    cb[(3 * zo) * SEQ + lds_pad(ky)] = B0;
                    cb[(3 * zo + 1) * SEQ + lds_pad(ky)] = B1;
                    cb[(3 * zo + 2) * SEQ + lds_pad(ky)] = B2;
                }
            }
        }
    }
    __syncthreads();

    // inverse y transform; rows y < ny are kept
#pragma unroll
    for (int m = 0; m < PPT; ++m) v[0][m] = buf[lds_pad(t + TPF * m)];
    RegFft<PY, TPF, 1, true>::run(v, buf, a.tw, a.twshift, t);
    int t2 = t;
    asm volatile("" : "+v"(t2));  // form the store addresses here, not at load time
#pragma unroll
    for (int m = 0; m < MH; ++m) {
        const int q = t2 + TPF * m;
        if (valid && q < a.n_in) col[3LL * q] = v[0][m];
    }
}

// ---------------------------------------------------------------------------
// 2D convolution, one thread group per column carrying all three components
// (three sequences through one LDS exchange buffer).  The K^ product is then
// local to the thread, and the twiddles and exchange addresses of a stage
// serve all three components.  Workgroup: T columns of TPF threads; LDS per
// column: the exchange buffer and a second one that only the workgroup of the
// packed DC/Nyquist column uses.  The K^ rows come straight from global
// memory (L2 / MALL) at the product: staging them in LDS before the forward
// transforms made every workgroup wait for them before its first butterfly.
template <int P, int W = 0>
struct Col3Cfg {
    static constexpr int TPF = Cfg<P>::TPF;
    // W = 0: 256-thread workgroups; W = 1: about one wave, for grids with too
    // few columns to give every CU two wide workgroups
    static constexpr int T = W ? (TPF >= 64 ? 1 : 64 / TPF) : (TPF >= 256 ? 1 : 256 / TPF);
    static constexpr int NTH = T * TPF;
    static constexpr int SEQ = seq_len(P);
    static constexpr int KHP = P / 2 + 1;
    static constexpr int CL = 2 * SEQ;  // complex elements per column
};

// the three-components-per-thread 2D convolution serves 64 <= P <= 2048
template <int P>
constexpr bool use_col3() {
    return P >= 64 && P <= 2048;
}

template <int P, int W = 0>
constexpr size_t col3_lds() {
    return (size_t)Col3Cfg<P, W>::T * Col3Cfg<P, W>::CL * sizeof(cf);
}

// FULL: the y axis is periodic and unpadded (P = ny): every row holds data
// and every row is kept.
template <int P, bool FULL = false, int W = 0>
__device__ inline void col3_body(const ColArgs& a, int blk, cf* lds, int tid) {
    constexpr int PPT = Cfg<P>::PPT, TPF = Cfg<P>::TPF, T = Col3Cfg<P, W>::T;
    constexpr int SEQ = Col3Cfg<P, W>::SEQ, KHP = Col3Cfg<P, W>::KHP, CL = Col3Cfg<P, W>::CL;
    constexpr int MH = FULL ? PPT : PPT / 2;  // registers that load and store rows
    // a finished run is tested once the column is loaded and transformed
    // (nothing is written before), so the state read overlaps the loads
    const int done = a.check_done ? a.st->done : 0;
    const int t = tid % TPF, ci = tid / TPF;
    const int c = blk * T + ci;
    const bool valid = c < a.ncol;
    const bool wg_packed = a.pack_col > 0 && blk == 0;  // uniform over the workgroup
    const bool packed = wg_packed && ci == 0;
    cf* buf = lds + ci * CL;
    cf* reg2 = buf + SEQ;
    const cf* base = a.spec + (long long)(valid ? c : 0) * a.col_stride;
    const cf* baseN = a.spec + (long long)a.pack_col * a.col_stride;
    const float4* kh = reinterpret_cast<const float4*>(a.khat);

    // rows y < ny <= P/2 hold data, the rest is zero padding (all P rows with FULL)
    // (two loops, so no load waits on another: a select of the packed
    // column's second half inside one loop makes every load wait for the last)
    cf v[3][PPT];
    if (!packed) {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            const int q = t + TPF * m;
            const bool ld = m < MH && valid && q < a.n_in;
#pragma unroll
            for (int k = 0; k < 3; ++k) v[k][m] = ld ? base[3LL * q + k] : mkc(0.f, 0.f);
        }
    } else {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            const int q = t + TPF * m;
            const bool ld = m < MH && valid && q < a.n_in;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                v[k][m] = ld ? mkc(base[3LL * q + k].x, baseN[3LL * q + k].x) : mkc(0.f, 0.f);
        }
    }
    RegFft<P, TPF, 3, false, !FULL>::run(v, buf, a.tw, a.twshift, t);
    if (done) return;

    // B^ = K^ M^ (2D: K^ = [[xx, xy, 0], [xy, yy, 0], [0, 0, zz]], xy odd in y);
    // row q of column kx is (xx, yy, zz, xy) at K^[kx][min(q, P - q)]
    if (!wg_packed) {
        int cq = valid ? c : 0;
        asm volatile("" : "+v"(cq));  // the K^ loads go out here, not during the transform
        const float4* kc = kh + (long long)cq * KHP;
        float4 kg[PPT];
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            const int q = t + TPF * m;
            kg[m] = kc[2 * q > P ? P - q : q];
        }
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            const int q = t + TPF * m;
            const bool fq = 2 * q > P;
            const float4 k4 = kg[m];
            const float kxy = fq ? -k4.w : k4.w;
            const cf mx = v[0][m], my = v[1][m];
            v[0][m] = k4.x * mx + kxy * my;
            v[1][m] = kxy * mx + k4.y * my;
            v[2][m] = k4.z * v[2][m];
        }
    } else {
        // Packed column Z = A0 + i AN (A0: kx = 0, AN: kx = px/2, both real along
        // y): B = K0 A0 + i KN AN = Kp Z(q) + Km conj Z(-q), Kp = (K0 + KN)/2,
        // Km = (K0 - KN)/2.  Z(-q) comes through LDS: z first (one buffer), then
        // x and y together (two buffers).  The other columns of this workgroup
        // (T > 1) take the plain product.
        auto kpm = [&](int q, float4& kp, float4& km) {
            const bool fq = 2 * q > P;
            const int qh = fq ? P - q : q;
            float4 k0 = kh[qh];
            float4 kn = kh[(long long)a.pack_col * KHP + qh];
            if (fq) {
                k0.w = -k0.w;
                kn.w = -kn.w;
            }
            kp = make_float4(0.5f * (k0.x + kn.x), 0.5f * (k0.y + kn.y), 0.5f * (k0.z + kn.z), 0.5f * (k0.w + kn.w));
            km = make_float4(0.5f * (k0.x - kn.x), 0.5f * (k0.y - kn.y), 0.5f * (k0.z - kn.z), 0.5f * (k0.w - kn.w));
        };
        __syncthreads();
        if (packed) {
#pragma unroll
            for (int m = 0; m < PPT; ++m) buf[lds_pad(t + TPF * m)] = v[2][m];
        }
        __syncthreads();
        if (packed) {
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                const int q = t + TPF * m;
                float4 kp, km;
                kpm(q, kp, km);
                const cf zr = cconj(buf[lds_pad((P - q) & (P - 1))]);
                v[2][m] = kp.z * v[2][m] + km.z * zr;
            }
        }
        __syncthreads();
        if (packed) {
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                buf[lds_pad(t + TPF * m)] = v[0][m];
                reg2[lds_pad(t + TPF * m)] = v[1][m];
            }
        }
        __syncthreads();
        if (packed) {
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                const int q = t + TPF * m;
                const int qn = (P - q) & (P - 1);
                float4 kp, km;
                kpm(q, kp, km);
                const cf xr = cconj(buf[lds_pad(qn)]), yr = cconj(reg2[lds_pad(qn)]);
                const cf zx = v[0][m], zy = v[1][m];
                v[0][m] = kp.x * zx + kp.w * zy + km.x * xr + km.w * yr;
                v[1][m] = kp.w * zx + kp.y * zy + km.w * xr + km.y * yr;
            }
        } else {
            const float4* kc = kh + (long long)(valid ? c : 0) * KHP;
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                const int q = t + TPF * m;
                const bool fq = 2 * q > P;
                const float4 k4 = kc[fq ? P - q : q];
                const float kxy = fq ? -k4.w : k4.w;
                const cf mx = v[0][m], my = v[1][m];
                v[0][m] = k4.x * mx + kxy * my;
                v[1][m] = kxy * mx + k4.y * my;
                v[2][m] = k4.z * v[2][m];
            }
        }
    }
    // the inverse transform derives its exchange addresses afresh (nothing of
    // the forward one stays live across the product)
    int ti = t;
    asm volatile("" : "+v"(ti));
    RegFft<P, TPF, 3, true>::run(v, buf, a.tw, a.twshift, ti);

    // rows y < ny (<= P/2 unless FULL) are kept; one component after the other
    cf* out = a.spec + (long long)(valid ? c : 0) * a.col_stride;
    cf* outN = a.spec + (long long)a.pack_col * a.col_stride;
    int t2 = t;
    asm volatile("" : "+v"(t2));  // form the store addresses here, not at load time
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int m = 0; m < MH; ++m) {
            const int q = t2 + TPF * m;
            if (valid && q < a.n_out) {
                if (!packed) {
                    out[3LL * q + k] = v[k][m];
                } else {
                    out[3LL * q + k] = mkc(v[k][m].x, 0.f);
                    outN[3LL * q + k] = mkc(v[k][m].y, 0.f);
                }
            }
        }
    }
}

// Dynamic LDS of each pass (bytes per workgroup).
template <int P, int W = 0>
constexpr size_t x_lds() {
    return (size_t)XCfg<P, W>::GI * XCfg<P, W>::GL * sizeof(cf) + NREG * sizeof(RegionLut);
}
template <int P, int MODE, int NC, bool CFAST = false>
constexpr size_t col_lds() {
    return (size_t)ColCfg<P>::T * 3 * col_seq<P, CFAST>() * sizeof(cf) +
           (MODE == COL_CONV && NC == 4 ? khat_lds<P>() : 0) +
           (MODE == COL_CONV && NC == 6
                ? (size_t)(col_pairs<P, MODE, NC>() ? ColCfg<P>::T / 2 : ColCfg<P>::T) * (P / 2 + 1) * 6 * sizeof(float)
                : 0);
}

}  // namespace mm
