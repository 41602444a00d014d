// kernels_batch.hip -- an ensemble of independent grids advanced together.
//
// Every pass of a Runge-Kutta stage is one persistent launch over a work list
// of (member, tile) items covering all members: a workgroup takes items in
// turn and runs, for each, the same device body the single-grid passes use
// (fft_passes.h), instantiated for the member's padded length.  The x passes
// and the 3D column passes of every padded length 64 ... 1024 have 768 threads
// and 55 KB of exchange LDS, the 2D column pass 256 threads and 36 KB, so one
// launch shape serves every member.  The x passes and the 2D column pass also
// come in a narrow tile shape (a quarter of the row pairs or columns per item:
// 192 and 64 threads) for ensembles whose padded lengths are all <= 512; the
// host picks the shape per pass.
//
// Items are dealt XCD-aware: the work list is cut into 8 contiguous chunks,
// and the workgroups of XCD x (dispatch index = x mod 8) walk chunk x, so the
// tiles of one member share an L2.  The number of persistent workgroups is a
// launch parameter (tuned by the host).
//
// A member's record and the current item are read through the constant
// address space: they are uniform over the workgroup, so they arrive in
// scalar registers; the member's pointers are the kernel arguments' base
// pointers plus its offsets.
#include "fft_passes.h"
#include "step_control.h"

namespace mm {

namespace {

constexpr int BX_NTH = 768;   // x passes and the 3D column passes
constexpr int BC3_NTH = 256;  // 2D column pass
constexpr int XMAX_GI = XCfg<64>::GI;
// narrow tile shape (TILE_NARROW) of the x passes and the 2D column pass:
// lengths up to 512
constexpr int BXN_NTH = 192;
constexpr int BC3N_NTH = 64;
constexpr int NARROW_MAX = 512;
template <int TILE>
constexpr int bx_nth() { return TILE == TILE_NARROW ? BXN_NTH : BX_NTH; }
template <int TILE>
constexpr int bc3_nth() { return TILE == TILE_NARROW ? BC3N_NTH : BC3_NTH; }
// lengths a tile shape serves
template <int P, int TILE>
constexpr bool tile_serves() { return TILE == TILE_WIDE || P <= NARROW_MAX; }

#define MB_XCASES(M) M(64) M(128) M(256) M(512) M(1024)
#define MB_ZCASES(M) M(4) M(8) M(16)

#define M(p)                                                                        \
    static_assert(XCfg<p>::NTH == BX_NTH && ColCfg<p>::NTH == BX_NTH, "x / y shape"); \
    static_assert(Col3Cfg<p>::NTH == BC3_NTH && use_col3<p>(), "2D column shape");    \
    static_assert(XCfg<p>::GI <= XMAX_GI, "row-pair table");                          \
    static_assert(p > NARROW_MAX || (XCfg<p, 1>::NTH == BXN_NTH && Col3Cfg<p, 1>::NTH == BC3N_NTH), "narrow");
MB_XCASES(M)
#undef M
#define M(p) static_assert(ColCfg<p>::NTH == BX_NTH, "z shape");
MB_ZCASES(M)
#undef M
#define M(p)                                                                                     \
    static_assert(!use_yz<p, 4>() || (YzCfg<p, 4>::NTH == BX_NTH && yz_lds<p, 4>() == yz_lds<64, 4>()), "yz");  \
    static_assert(!use_yz<p, 8>() || (YzCfg<p, 8>::NTH == BX_NTH && yz_lds<p, 8>() == yz_lds<64, 8>()), "yz");
MB_XCASES(M)
#undef M

template <class T>
using const_as = const __attribute__((address_space(4))) T;

template <class T>
__device__ inline T uload(const T* p) {
#if __HIP_DEVICE_COMPILE__
    return *(const_as<T>*)p;
#else
    return *p;
#endif
}


// The thread index, opaque to the compiler: the per-length index arithmetic of
// an item is then formed inside the loop, not hoisted out of it for every
// length at once (which would keep all of it live across the loop).
__device__ inline int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

struct ItemRange {
    int it, end, step;
};

// Items of this workgroup: chunk (dispatch index mod 8) of the list, strided
// by the workgroups of that XCD.
__device__ inline ItemRange item_range(int nitems) {
    const int w = blockIdx.x, g = gridDim.x;
    const int x = w & 7;
    ItemRange r;
    r.it = (int)(((long long)nitems * x) >> 3) + (w >> 3);
    r.end = (int)(((long long)nitems * (x + 1)) >> 3);
    r.step = g >> 3;
    return r;
}

// The field arguments of member i from the ensemble's base arguments.
__device__ inline FieldArgs member_field(const FieldArgs& b, const BMember& mb, int i) {
    FieldArgs a = b;
    a.nx = mb.nx;
    a.ny = mb.ny;
    a.nz = mb.nz;
    a.nrows = mb.nrows;
    a.ncell = (long long)mb.nx * mb.ny * mb.nz;
    a.pbc = 0;                // ensemble members have open boundaries
    a.flags &= ~EPI_THERM;    // and no thermal field
    a.cub = nullptr;          // nor cubic anisotropy
    a.dmi = nullptr;          // nor DMI
    const long long c = mb.cell_off, c3 = 3 * c;
    a.m0 = b.m0 + c3;
    a.ms = b.ms + c3;
    a.region = b.region + c;
    a.lut = b.lut + (long long)i * NREG;
    a.ptab = b.ptab + (long long)i * NREG * NREG;
    a.idx2 = mb.idx2;
    a.idy2 = mb.idy2;
    a.idz2 = mb.idz2;
    a.kbuf = b.kbuf + MAXK * c3;
    a.st = b.st + i;
    a.spec = b.spec + mb.spec_off;
    a.colstride = mb.colstride;
    a.zstride = mb.zstride;
    a.beff = b.beff ? b.beff + c3 : nullptr;
    a.bdemag = b.bdemag ? b.bdemag + c3 : nullptr;
    a.tau = b.tau ? b.tau + c3 : nullptr;
    a.partials = nullptr;
    a.cellvol = mb.cellvol;
    return a;
}

// The column arguments of member i for column pass `kind`.
__device__ inline ColArgs member_col(const ColArgs& b, const BMember& mb, int i, int kind) {
    ColArgs a = b;
    a.spec = b.spec + mb.spec_off;
    a.khat = b.khat + mb.khat_off;
    a.st = b.st + i;
    a.kyh = mb.py / 2 + 1;
    a.kzh = mb.pz / 2 + 1;
    a.pa = mb.py;
    a.pack_col = 0;
    if (kind == BC_YZ) {
        // thin 3D member: y FFT, z convolution with the z-space kernel, inverse y FFT per kx column
        a.khat = b.zker + mb.zker_off;
        a.pos_stride = 3;
        a.col_stride = mb.colstride;
        a.ncol = mb.kx;
        a.outer_stride = mb.zstride;
        a.nouter = mb.nz;
        a.n_in = mb.ny;
        a.n_out = mb.ny;
    } else if (kind == BC_ZCONV) {
        // z convolution of every (kx, ky) column; tiles of adjacent ky
        a.pos_stride = mb.zstride;
        a.col_stride = 3;
        a.ncol = mb.py;
        a.outer_stride = mb.colstride;
        a.nouter = mb.kx;
        a.n_in = mb.nz;
        a.n_out = mb.nz;
    } else if (kind == BC_YFWD || kind == BC_YINV) {
        // y transforms of every (kx, z) column, in place (ny rows <-> py rows);
        // tiles of adjacent planes of one kx
        a.pos_stride = 3;
        a.col_stride = mb.zstride;
        a.ncol = mb.nz;
        a.outer_stride = mb.colstride;
        a.nouter = mb.kx;
        a.n_in = kind == BC_YFWD ? mb.ny : mb.py;
        a.n_out = kind == BC_YFWD ? mb.py : mb.ny;
    } else {
        // 2D y convolution of every kx column; DC and Nyquist share column 0
        a.pos_stride = 3;
        a.col_stride = mb.colstride;
        a.ncol = mb.px / 2;
        a.pack_col = mb.px / 2;
        a.outer_stride = 0;
        a.nouter = 1;
        a.n_in = mb.ny;
        a.n_out = mb.ny;
    }
    return a;
}

// One x-pass item: row-pair tile blk of member i (tile shape TILE: row pairs
// per item as in the single-grid pass of that width).
template <int P, int KIND, int TILE>
__device__ inline void bx_item(const FieldArgs& fi, const FieldArgs& ff, float a_last, const BMember& mb, int i,
                               int blk, int tid, cf* lds, long long* rbs, double* red) {
    constexpr int XW = TILE == TILE_NARROW ? 1 : 0;
    constexpr int GI = XCfg<P, XW>::GI, GL = XCfg<P, XW>::GL;
    RegionLut* lut_l = reinterpret_cast<RegionLut*>(lds + GI * GL);
    const FieldArgs a = member_field(fi, mb, i);
    const Resolved rs = resolve(a);
    if ((a.flags & EPI_CHECK_DONE) && rs.done) return;
    row_bases<GI>(a, blk * GI, rbs, tid);
    if constexpr (KIND == BX_FWD) {
        XLut<P, XW> lut;
        lut.load(a, tid);
        xfwd_part<P, false, false, XW>(a, rs, lds, rbs, lut_l, &lut, 0.f, blk, tid);
    } else if constexpr (KIND == BX_INV) {
        __syncthreads();
        xinv_part<P, false, false, false, XW>(a, rs, lds, rbs, lut_l, red, blk, tid);
    } else {
        __syncthreads();
        if (!xinv_part<P, true, false, false, XW>(a, rs, lds, rbs, lut_l, red, blk, tid)) return;
        __syncthreads();
        const FieldArgs af = member_field(ff, mb, i);
        const Resolved rsf = resolve(af);
        xfwd_part<P, true, false, XW>(af, rsf, lds, rbs, lut_l, nullptr, a_last, blk, tid);
    }
}

template <int KIND, int TILE>
__global__ void __launch_bounds__(bx_nth<TILE>()) __attribute__((amdgpu_waves_per_eu(6)))
k_bx(const BatchList l, const FieldArgs fi, const FieldArgs ff, float a_last) {
    extern __shared__ cf lds[];
    __shared__ long long rbs[2 * XMAX_GI];
    __shared__ double red[(bx_nth<TILE>() / 64) * 6];
    const ItemRange r = item_range(l.nitems);
    for (int it = r.it; it < r.end; it += r.step) {
        const unsigned int item = uload(l.items + it);
        const int i = (int)(item >> 16), blk = (int)(item & 0xffffu);
        const BMember mb = uload(l.mem + i);
        __syncthreads();  // the previous item is done with LDS
        const int tid = opaque_tid();
        switch (mb.px) {
#define M(p)                                                                       \
    case p:                                                                        \
        if constexpr (tile_serves<p, TILE>())                                      \
            bx_item<p, KIND, TILE>(fi, ff, a_last, mb, i, blk, tid, lds, rbs, red);  \
        break;
            MB_XCASES(M)
#undef M
            default:
                break;
        }
    }
}

template <int TILE>
__global__ void __launch_bounds__(bc3_nth<TILE>(), 3) k_bcol3(const BatchList l, const ColArgs b) {
    constexpr int W = TILE == TILE_NARROW ? 1 : 0;
    extern __shared__ cf lds[];
    const ItemRange r = item_range(l.nitems);
    for (int it = r.it; it < r.end; it += r.step) {
        const unsigned int item = uload(l.items + it);
        const int i = (int)(item >> 16), blk = (int)(item & 0xffffu);
        const BMember mb = uload(l.mem + i);
        const ColArgs a = member_col(b, mb, i, BC_CONV2);
        __syncthreads();
        const int tid = opaque_tid();
        switch (mb.py) {
#define M(p)                                                                    \
    case p:                                                                     \
        if constexpr (tile_serves<p, TILE>()) col3_body<p, false, W>(a, blk, lds, tid);  \
        break;
            MB_XCASES(M)
#undef M
            default:
                break;
        }
    }
}

// y transforms of the 3D members
template <int KIND>
__global__ void __launch_bounds__(BX_NTH) k_bcoly(const BatchList l, const ColArgs b) {
    extern __shared__ cf lds[];
    const ItemRange r = item_range(l.nitems);
    for (int it = r.it; it < r.end; it += r.step) {
        const unsigned int item = uload(l.items + it);
        const int i = (int)(item >> 16), blk = (int)(item & 0xffffu);
        const BMember mb = uload(l.mem + i);
        const ColArgs a = member_col(b, mb, i, KIND);
        __syncthreads();
        const int tid = opaque_tid();
        switch (mb.py) {
#define M(q)                                                                             \
    case q:                                                                              \
        col_body<q, KIND == BC_YFWD ? COL_FWD : COL_INV, 4, false>(a, blk, lds, tid);  \
        break;
            MB_XCASES(M)
#undef M
            default:
                break;
        }
    }
}

// z convolution of the 3D members of one padded z length (a launch per length:
// the short transforms differ too much in register needs to share a kernel)
template <int PZ>
__global__ void __launch_bounds__(BX_NTH) k_bzconv(const BatchList l, const ColArgs b) {
    extern __shared__ cf lds[];
    const ItemRange r = item_range(l.nitems);
    for (int it = r.it; it < r.end; it += r.step) {
        const unsigned int item = uload(l.items + it);
        const int i = (int)(item >> 16), blk = (int)(item & 0xffffu);
        const BMember mb = uload(l.mem + i);
        const ColArgs a = member_col(b, mb, i, BC_ZCONV);
        __syncthreads();
        col_body<PZ, COL_CONV, 6, true>(a, blk, lds, opaque_tid());
    }
}

// thin 3D members of one padded z length (y FFT, z DFT with K^, inverse y FFT)
template <int PZ>
__global__ void __launch_bounds__(BX_NTH) __attribute__((amdgpu_waves_per_eu(PZ == 4 ? 6 : 1)))
k_byz(const BatchList l, const ColArgs b) {
    extern __shared__ cf lds[];
    const ItemRange r = item_range(l.nitems);
    for (int it = r.it; it < r.end; it += r.step) {
        const unsigned int item = uload(l.items + it);
        const int i = (int)(item >> 16), blk = (int)(item & 0xffffu);
        const BMember mb = uload(l.mem + i);
        const ColArgs a = member_col(b, mb, i, BC_YZ);
        __syncthreads();
        const int tid = opaque_tid();
        switch (mb.py) {
#define M(q)                                                   \
    case q:                                                    \
        if constexpr (use_yz<q, PZ>()) yz_body<q, PZ>(a, blk, lds, tid); \
        break;
            MB_XCASES(M)
#undef M
            default:
                break;
        }
    }
}

// After the controllers: members whose step was accepted take m0 <- m_s/|m_s|.
__global__ void __launch_bounds__(NT) k_bfinalize(const BatchList l, const float* __restrict__ ms,
                                                  float* __restrict__ m, const DevState* __restrict__ st) {
    const ItemRange r = item_range(l.nitems);
    for (int it = r.it; it < r.end; it += r.step) {
        const unsigned int item = uload(l.items + it);
        const int i = (int)(item >> 16), blk = (int)(item & 0xffffu);
        if (!st[i].accepted) continue;
        const BMember mb = uload(l.mem + i);
        const long long n = (long long)mb.nx * mb.ny * mb.nz;
        const long long cell = (long long)blk * NT + threadIdx.x;
        if (cell >= n) continue;
        const long long c3 = 3 * mb.cell_off;
        const float3 v = ld3(ms + c3, n, cell);
        const float n2 = f3dot(v, v);
        const float inv = n2 > 0.f ? rsqrtf(n2) : 0.f;
        st3(m + c3, n, cell, f3scale(inv, v));
    }
}

// The step controllers of every member, then the number of members still
// running (for the host's stopping test).
__global__ void __launch_bounds__(1024) k_bcontroller(DevState* st, int n, int last_k, int evals, int check_done,
                                                      int* active) {
    __shared__ int cnt[1024 / 64];
    int live = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        controller_update(st + i, last_k, evals, check_done);
        live += st[i].done ? 0 : 1;
    }
    for (int off = 32; off > 0; off >>= 1) live += __shfl_xor(live, off, 64);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = live;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += cnt[w];
        *active = tot;
    }
}

__global__ void k_bset_state(DevState* st, int n, double t, double dt, double t_end, double max_err,
                             double headroom, double dt_min, double dt_max, int order_low, int reset_counters,
                             int init_perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        set_state(st + i, t, dt, t_end, max_err, headroom, dt_min, dt_max, order_low, reset_counters, init_perm,
                  0);
}

// dynamic LDS of the batched passes: the largest over the served lengths
constexpr size_t max2(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t BX_LDS = max2(max2(max2(x_lds<64>(), x_lds<128>()), max2(x_lds<256>(), x_lds<512>())), x_lds<1024>());
constexpr size_t BC3_LDS =
    max2(max2(max2(col3_lds<64>(), col3_lds<128>()), max2(col3_lds<256>(), col3_lds<512>())), col3_lds<1024>());
constexpr size_t BXN_LDS = max2(max2(x_lds<64, 1>(), x_lds<128, 1>()), max2(x_lds<256, 1>(), x_lds<512, 1>()));
constexpr size_t BC3N_LDS =
    max2(max2(col3_lds<64, 1>(), col3_lds<128, 1>()), max2(col3_lds<256, 1>(), col3_lds<512, 1>()));
constexpr size_t BY_LDS = max2(max2(max2(col_lds<64, COL_FWD, 4>(), col_lds<128, COL_FWD, 4>()),
                                    max2(col_lds<256, COL_FWD, 4>(), col_lds<512, COL_FWD, 4>())),
                               col_lds<1024, COL_FWD, 4>());

// host-side tile counts per padded length (0: a length the shape does not serve)
int x_gi(int p, int tile = TILE_WIDE) {
    switch (p) {
#define M(q) \
    case q:  \
        return tile == TILE_WIDE ? XCfg<q>::GI : (q <= NARROW_MAX ? XCfg<q, 1>::GI : 0);
        MB_XCASES(M)
#undef M
        default:
            return 0;
    }
}
int col3_t(int p, int tile = TILE_WIDE) {
    switch (p) {
#define M(q) \
    case q:  \
        return tile == TILE_WIDE ? Col3Cfg<q>::T : (q <= NARROW_MAX ? Col3Cfg<q, 1>::T : 0);
        MB_XCASES(M)
#undef M
        default:
            return 0;
    }
}
int col_t(int p) {
    switch (p) {
#define M(q) \
    case q:  \
        return ColCfg<q>::T;
        MB_XCASES(M) MB_ZCASES(M)
#undef M
        default:
            return 0;
    }
}

// kx columns per workgroup of the thin-grid pass
int yz_t(int py, int pz) {
    switch (pz) {
#define MT(pzv)                                                           \
    case pzv:                                                             \
        switch (py) {                                                     \
            MB_XCASES(MT##pzv)                                            \
            default:                                                      \
                return 0;                                                 \
        }
#define MTB(q, pzv)                                                       \
    case q:                                                               \
        if constexpr (use_yz<q, pzv>()) return YzCfg<q, pzv>::T;          \
        return 0;
#define MT4(q) MTB(q, 4)
#define MT8(q) MTB(q, 8)
        MT(4)
        MT(8)
#undef MT4
#undef MT8
#undef MTB
#undef MT
        default:
            return 0;
    }
}

int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// kernel, block size and dynamic LDS of each batched pass
struct PassShape {
    const void* fn;
    int nth;
    size_t lds;
};

PassShape pass_shape(int pass, int tile = TILE_WIDE) {
    const bool nar = tile == TILE_NARROW;
    switch (pass) {
        case BP_X:
            return nar ? PassShape{(const void*)k_bx<BX_ROW, TILE_NARROW>, BXN_NTH, BXN_LDS}
                       : PassShape{(const void*)k_bx<BX_ROW, TILE_WIDE>, BX_NTH, BX_LDS};
        case BP_C3:
            return nar ? PassShape{(const void*)k_bcol3<TILE_NARROW>, BC3N_NTH, BC3N_LDS}
                       : PassShape{(const void*)k_bcol3<TILE_WIDE>, BC3_NTH, BC3_LDS};
        case BP_Y:
            return {(const void*)k_bcoly<BC_YFWD>, BX_NTH, BY_LDS};
        case BP_Z4:
            return {(const void*)k_bzconv<4>, BX_NTH, col_lds<4, COL_CONV, 6, true>()};
        case BP_Z8:
            return {(const void*)k_bzconv<8>, BX_NTH, col_lds<8, COL_CONV, 6, true>()};
        case BP_Z16:
            return {(const void*)k_bzconv<16>, BX_NTH, col_lds<16, COL_CONV, 6, true>()};
        case BP_YZ4:
            return {(const void*)k_byz<4>, BX_NTH, yz_lds<64, 4>()};
        case BP_YZ8:
            return {(const void*)k_byz<8>, BX_NTH, yz_lds<64, 8>()};
        case BP_F:
            return {(const void*)k_bfinalize, NT, 0};
        default:
            return {nullptr, 0, 0};
    }
}

hipError_t check_grid(const BatchList& l, int grid) {
    return (grid <= 0 || grid % 8) ? hipErrorInvalidValue : hipSuccess;
}

}  // namespace

bool batch_supported(int px, int py, int pz) {
    return x_gi(px) > 0 && x_gi(py) > 0 && (pz == 1 || pz == 4 || pz == 8 || pz == 16);
}

bool batch_tile_serves(int pass, int tile, const BMember& m) {
    if (tile == TILE_WIDE) return true;
    if (tile != TILE_NARROW) return false;
    if (pass == BP_X) return x_gi(m.px, tile) > 0;
    if (pass == BP_C3) return m.pz != 1 || col3_t(m.py, tile) > 0;
    return false;
}

int batch_tiles(int pass, const BMember& m, int tile) {
    if (!batch_tile_serves(pass, tile, m)) return 0;
    switch (pass) {
        case BP_X:
            return cdiv((m.nrows + 1) / 2, x_gi(m.px, tile));
        case BP_C3:
            return m.pz == 1 ? cdiv(m.px / 2, col3_t(m.py, tile)) : 0;
        case BP_Y:
            return m.pz > 1 && !yz_supported(m.py, m.pz) ? cdiv(m.nz, col_t(m.py)) * m.kx : 0;
        case BP_Z4:
            return m.pz == 4 && !yz_supported(m.py, m.pz) ? col_ntile<4, COL_CONV, 6>(m.py) * m.kx : 0;
        case BP_Z8:
            return m.pz == 8 && !yz_supported(m.py, m.pz) ? col_ntile<8, COL_CONV, 6>(m.py) * m.kx : 0;
        case BP_Z16:
            return m.pz == 16 && !yz_supported(m.py, m.pz) ? col_ntile<16, COL_CONV, 6>(m.py) * m.kx : 0;
        case BP_YZ4:
        case BP_YZ8: {
            const int pz = pass == BP_YZ4 ? 4 : 8;
            return m.pz == pz && yz_supported(m.py, m.pz) ? cdiv(m.kx, yz_t(m.py, pz)) : 0;
        }
        case BP_F:
            return cdiv((long long)m.nx * m.ny * m.nz, NT);
        default:
            return 0;
    }
}

hipError_t batch_resident(int pass, int tile, int* per_cu) {
    const PassShape ps = pass_shape(pass, tile);
    if (!ps.fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, ps.fn, ps.nth, ps.lds);
}

hipError_t configure_batch_kernels(void) {
    const PassShape extra[] = {{(const void*)k_bx<BX_FWD, TILE_WIDE>, BX_NTH, BX_LDS},
                               {(const void*)k_bx<BX_INV, TILE_WIDE>, BX_NTH, BX_LDS},
                               {(const void*)k_bx<BX_FWD, TILE_NARROW>, BXN_NTH, BXN_LDS},
                               {(const void*)k_bx<BX_INV, TILE_NARROW>, BXN_NTH, BXN_LDS},
                               {(const void*)k_bcoly<BC_YINV>, BX_NTH, BY_LDS}};
    for (int p = 0; p < BP_N; ++p) {
        for (int tile : {TILE_WIDE, TILE_NARROW}) {
            if (tile == TILE_NARROW && p != BP_X && p != BP_C3) continue;
            const PassShape ps = pass_shape(p, tile);
            if (ps.lds == 0) continue;
            const hipError_t e = hipFuncSetAttribute(ps.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ps.lds);
            if (e != hipSuccess) return e;
        }
    }
    for (const PassShape& ps : extra) {
        const hipError_t e = hipFuncSetAttribute(ps.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ps.lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int TILE>
static hipError_t launch_bx_t(int kind, const BatchList& l, int grid, const FieldArgs& fi, const FieldArgs& ff,
                              float a_last, hipStream_t s) {
    constexpr int NTH = bx_nth<TILE>();
    constexpr size_t LDS = TILE == TILE_NARROW ? BXN_LDS : BX_LDS;
    switch (kind) {
        case BX_FWD:
            hipLaunchKernelGGL((k_bx<BX_FWD, TILE>), dim3(grid), dim3(NTH), LDS, s, l, fi, ff, a_last);
            break;
        case BX_ROW:
            hipLaunchKernelGGL((k_bx<BX_ROW, TILE>), dim3(grid), dim3(NTH), LDS, s, l, fi, ff, a_last);
            break;
        case BX_INV:
            hipLaunchKernelGGL((k_bx<BX_INV, TILE>), dim3(grid), dim3(NTH), LDS, s, l, fi, ff, a_last);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bx(int kind, const BatchList& l, int grid, const FieldArgs& fi, const FieldArgs& ff, float a_last,
                     hipStream_t s, int tile) {
    if (l.nitems <= 0) return hipSuccess;
    if (check_grid(l, grid) != hipSuccess) return hipErrorInvalidValue;
    if (tile == TILE_NARROW) return launch_bx_t<TILE_NARROW>(kind, l, grid, fi, ff, a_last, s);
    if (tile == TILE_WIDE) return launch_bx_t<TILE_WIDE>(kind, l, grid, fi, ff, a_last, s);
    return hipErrorInvalidValue;
}

hipError_t launch_bcol3(const BatchList& l, int grid, const ColArgs& base, hipStream_t s, int tile) {
    if (l.nitems <= 0) return hipSuccess;
    if (check_grid(l, grid) != hipSuccess) return hipErrorInvalidValue;
    if (tile == TILE_NARROW)
        hipLaunchKernelGGL(k_bcol3<TILE_NARROW>, dim3(grid), dim3(BC3N_NTH), BC3N_LDS, s, l, base);
    else if (tile == TILE_WIDE)
        hipLaunchKernelGGL(k_bcol3<TILE_WIDE>, dim3(grid), dim3(BC3_NTH), BC3_LDS, s, l, base);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_bcoly(int inverse, const BatchList& l, int grid, const ColArgs& base, hipStream_t s) {
    if (l.nitems <= 0) return hipSuccess;
    if (check_grid(l, grid) != hipSuccess) return hipErrorInvalidValue;
    if (inverse)
        hipLaunchKernelGGL(k_bcoly<BC_YINV>, dim3(grid), dim3(BX_NTH), BY_LDS, s, l, base);
    else
        hipLaunchKernelGGL(k_bcoly<BC_YFWD>, dim3(grid), dim3(BX_NTH), BY_LDS, s, l, base);
    return hipGetLastError();
}

hipError_t launch_bzconv(int pass, const BatchList& l, int grid, const ColArgs& base, hipStream_t s) {
    if (l.nitems <= 0) return hipSuccess;
    if (check_grid(l, grid) != hipSuccess) return hipErrorInvalidValue;
    const PassShape ps = pass_shape(pass);
    switch (pass) {
        case BP_Z4:
            hipLaunchKernelGGL(k_bzconv<4>, dim3(grid), dim3(BX_NTH), ps.lds, s, l, base);
            break;
        case BP_Z8:
            hipLaunchKernelGGL(k_bzconv<8>, dim3(grid), dim3(BX_NTH), ps.lds, s, l, base);
            break;
        case BP_Z16:
            hipLaunchKernelGGL(k_bzconv<16>, dim3(grid), dim3(BX_NTH), ps.lds, s, l, base);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_byz(int pass, const BatchList& l, int grid, const ColArgs& base, hipStream_t s) {
    if (l.nitems <= 0) return hipSuccess;
    if (check_grid(l, grid) != hipSuccess) return hipErrorInvalidValue;
    const PassShape ps = pass_shape(pass);
    switch (pass) {
        case BP_YZ4:
            hipLaunchKernelGGL(k_byz<4>, dim3(grid), dim3(BX_NTH), ps.lds, s, l, base);
            break;
        case BP_YZ8:
            hipLaunchKernelGGL(k_byz<8>, dim3(grid), dim3(BX_NTH), ps.lds, s, l, base);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bfinalize(const BatchList& l, int grid, const float* ms, float* m, const DevState* st,
                            hipStream_t s) {
    if (l.nitems <= 0) return hipSuccess;
    if (check_grid(l, grid) != hipSuccess) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bfinalize, dim3(grid), dim3(NT), 0, s, l, ms, m, st);
    return hipGetLastError();
}

hipError_t launch_bcontroller(DevState* st, int n, int last_k, int evals, int check_done, int* active,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_bcontroller, dim3(1), dim3(1024), 0, s, st, n, last_k, evals, check_done, active);
    return hipGetLastError();
}

hipError_t launch_bset_state(DevState* st, int n, double t, double dt, double t_end, double max_err,
                             double headroom, double dt_min, double dt_max, int order_low, int reset_counters,
                             int init_perm, hipStream_t s) {
    hipLaunchKernelGGL(k_bset_state, dim3((n + 255) / 256), dim3(256), 0, s, st, n, t, dt, t_end, max_err,
                       headroom, dt_min, dt_max, order_low, reset_counters, init_perm);
    return hipGetLastError();
}

}  // namespace mm
