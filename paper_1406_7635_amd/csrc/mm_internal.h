// mm_internal.h -- device-side structures and launch interfaces of libmm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mm.h"
#include "fft_core.h"

namespace mm {

constexpr int NREG = 256;
constexpr int NPAIR = NREG * (NREG + 1) / 2;
static_assert(NREG == 256, "the square exchange table index packs a region in 8 bits");
constexpr int NT = 256;            // threads per workgroup of every field kernel
constexpr int MAXK = 7;            // stage-derivative buffers (Dormand-Prince needs 7)
constexpr double MU0 = 4.0e-7 * 3.14159265358979323846;
constexpr double GAMMA_DEFAULT = 1.7595e11;

// Per-region FP32 table derived on the device from the FP64 parameters.
struct RegionLut {
    float4 a;  // msat, 2 Ku1/Msat, 4 Ku2/Msat, alpha
    float4 b;  // anisotropy axis u (x, y, z), -gamma/(1+alpha^2)
    float4 c;  // B_ext (x, y, z), 0
};

// Solver state that lives on the device so steps need no host round trip.
struct DevState {
    double t, dt, t_end;
    double max_err, headroom, dt_min, dt_max;
    double err;                 // error estimate of the last attempt
    unsigned int err_bits;      // max over cells of |sum e_j k_j| (float bits, atomicMax)
    unsigned int tq_bits;       // max over cells of |tau| (float bits, atomicMax)
    int perm[8];                // logical stage derivative -> physical k buffer
    int accepted, done, status, order_low;
    long long steps, rejects, evals;
    long long target_steps;     // > 0: the run is done once steps reaches it
    double red[8];              // results of FP64 reductions (energies)
    // surrogate check of an attempt whose inner stages used the surrogate:
    // max |B_sur - B_exact| and max |B_exact| over cells at the new state
    unsigned int sur_num_bits, sur_den_bits;
    double sur_err;             // their ratio for the last checked attempt
    int sur_fail;               // the last attempt exceeded the tolerance: rejected, dt kept
    long long sur_fallbacks;
    // steps accepted since the thermal generator was seeded: the step index of
    // its counter (not reset by set_state)
    unsigned long long therm_step;
};

// One torque evaluation inside a Runge-Kutta step.
struct StageDesc {
    int nk;          // stage state m_s = m0 + dt sum_j a[j] k[kidx[j]]; nk = 0: m_s = m0
    int kidx[6];
    float a[6];
    int out_k;       // logical index of the derivative written, -1 = none
    int nerr;        // error norm |sum_j e[j] k[eidx[j]]| accumulated when > 0
    int eidx[7];
    float e[7];
};

enum EpiFlags {
    EPI_TORQUE = 1,      // compute the torque (to k[out_k] or tau)
    EPI_BEFF = 2,        // write B_eff
    EPI_BDEMAG = 4,      // write B_demag
    EPI_ERR = 8,         // accumulate the embedded error norm
    EPI_MAXTQ = 16,      // accumulate max |tau|
    EPI_ENERGY = 32,     // per-workgroup FP64 energy partial sums
    EPI_PRECESS = 64,    // keep the m x B term of the torque
    EPI_HAS_DEMAG = 128, // the pass carries a demag field (else B_demag = 0)
    EPI_CHECK_DONE = 256, // device-controlled run: skip the work once the run is done
    EPI_THERM = 512       // add the thermal field of the step (bth) to B_eff
};

struct FieldArgs {
    int nx, ny, nz, nrows;        // nrows = ny * nz
    long long ncell;
    const float* m0;              // committed state (or the caller's m)
    float* ms;                    // stage state (written by the first pass when sd.nk > 0)
    const uint8_t* region;
    const RegionLut* lut;
    const float* ptab;            // exchange pair coefficients, packed lower triangle
    float idx2, idy2, idz2;       // 1/dx^2, 1/dy^2, 1/dz^2
    float* kbuf;                  // [MAXK][3][ncell]
    DevState* st;
    StageDesc sd;
    cf* spec;                     // spectrum, element (z, kx, y, c) at z*zstride + kx*colstride + 3y + c
    long long colstride, zstride; // in complex elements
    const cf* tw;                 // exp(-2 pi i m / PT)
    int twshift;                  // log2 PT
    float* beff;
    float* bdemag;
    float* tau;                   // explicit torque output when sd.out_k < 0
    double* partials;             // [blocks][4] energy partial sums
    float cellvol;
    int flags;
    int pbc;                      // periodic axes: bit 0 x, bit 1 y, bit 2 z (exchange wraps around)
    const float* bth;             // thermal field of the current step [3][ncell] (EPI_THERM)
    // cubic anisotropy per region (null: none): 3 float4 per region,
    // (c1, -2 Kc1/Msat), (c2, -2 Kc2/Msat), (c3, -4 Kc3/Msat)
    const float4* cub;
    // induced DMI per region (null: none): (2 D/Msat, D/(2 A))
    const float2* dmi;
    int full_x;                   // x is periodic and transformed unpadded (px = nx)
};

struct ColArgs {
    cf* spec;
    int n_in, n_out;              // non-zero input length, kept output length along the transform
    long long pos_stride;         // complex elements between consecutive transform positions
    long long col_stride;         // between adjacent columns of a workgroup tile
    int ncol;                     // columns along the tile direction
    long long outer_stride;       // between outer indices
    int nouter;
    int pa;                       // 3D convolution: padded y length (ky folding)
    const float* khat;            // convolution only: [kx][ky_h][kz_h][ncomp]
    int kyh, kzh;                 // folded lengths py/2+1, pz/2+1
    int pack_col;                 // 2D convolution: > 0 when column 0 also carries kx = pack_col (Nyquist)
    const cf* tw;
    int twshift;
    const DevState* st;
    int check_done;
    const void* dft_tab;          // matrix-core variant: split DFT matrices of its precision
    const float* zker;            // ensembles: base of the members' z-space kernels (thin grids)
    int full;                     // 2D convolution: y periodic and unpadded (py = ny)
};

// ---- launchers (kernels_fft.hip) -------------------------------------------
// e0 / e1 (optional) are recorded by the dispatch itself at the start / end of
// the kernel, so their elapsed time is the kernel's own duration.
hipError_t launch_xfwd(int px, const FieldArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
hipError_t launch_xinv(int px, const FieldArgs& a, hipStream_t s, int* nblocks_out, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
hipError_t launch_col(int p, int mode, const ColArgs& a, int ncomp, hipStream_t s, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
// Matrix-core y convolution (2D, P = 2048) with split-precision DFT stages;
// prec MM_PREC_BF16 / MM_PREC_FP16.  launch_dft_tables fills the per-context
// table of split DFT matrices (2 x DFT_TABLE_BYTES).
constexpr int DFT_TABLE_BYTES = 256 * 64;
hipError_t launch_colm(int p, int prec, const ColArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
hipError_t launch_dft_tables(void* tab, hipStream_t s);
hipError_t configure_colm(void);
// Matrix-core column passes of 3D grids (y forward / inverse, z convolution)
// for padded lengths 64 ... 1024; mode COL_FWD, COL_INV or COL_CONV.
bool colm3d_supported(int p);
hipError_t launch_colm3d(int p, int mode, int prec, const ColArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
hipError_t configure_colm3d(void);

// Fused x-inverse of one stage and x-forward of the next (px >= 8): ai is the
// finishing stage (reads m_s from ai.ms), af the next one (its combine holds
// every term but the last, a_last k_s, which comes from the finishing stage;
// m_{s+1} goes to af.ms, which must differ from ai.ms).
hipError_t launch_xrow(int px, const FieldArgs& ai, const FieldArgs& af, float a_last, hipStream_t s,
                       hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Thin-grid 3D convolution (y FFT, z DFT with the K^ product, inverse y FFT
// in one pass per kx column; the spectrum keeps ny rows): padded lengths
// (py, pz) with pz in {4, 8}, py >= 16 and py pz <= 4096.
bool yz_supported(int py, int pz);
hipError_t launch_yz(int py, int pz, const ColArgs& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// The thin-grid pass's kernel in z space, G(d) = sum_kz K^(kz) exp(+2 pi i kz d/pz),
// from the K^ octant [kx][ky_h][kz_h][6] (rows = kx (py/2 + 1)); FP64 sums.
int zkernel_floats(int pz);
hipError_t launch_zkernel(const float* khat, float* zker, long long rows, int pz, hipStream_t s);
int xinv_blocks(int px, int nrows);
// Raise the dynamic-LDS limit of every pass a grid of padded size px x py x pz
// launches (once per context, on the current device).
hipError_t configure_field_kernels(int px, int py, int pz);
enum ColMode { COL_FWD = 0, COL_INV = 1, COL_CONV = 2 };

// ---- batched ensemble (kernels_batch.hip) ----------------------------------
// An ensemble of independent grids shares one work list per pass.  The
// ensemble's arrays are the members' arrays back to back; BMember locates
// member i in them (its [3][ncell] vector fields at 3 cell_off floats, its
// region map at cell_off bytes, its stage derivatives at MAXK 3 cell_off
// floats, its spectrum at spec_off and kernel spectrum at khat_off elements,
// its region tables at i NREG entries, its pair table at i NREG^2 floats, its
// solver state at entry i).  The kernels take the base pointers and stage
// descriptor in FieldArgs / ColArgs and derive each member's arguments.
struct BMember {
    int nx, ny, nz, nrows;
    int px, py, pz, kx;
    long long cell_off;
    long long spec_off;
    long long khat_off;
    long long zker_off;           // z-space kernel floats before this member's (thin 3D members)
    long long colstride, zstride;
    float idx2, idy2, idz2, cellvol;
};
// Work list of one batched pass: item = (member << 16) | tile.
struct BatchList {
    const BMember* mem;
    const unsigned int* items;
    int nitems;
};
enum BatchPass {
    BP_X = 0,     // x passes
    BP_C3 = 1,    // 2D y convolution
    BP_Y = 2,     // 3D y transforms (members without the thin-grid pass)
    BP_Z4 = 3,    // 3D z convolution, padded z length 4 / 8 / 16
    BP_Z8 = 4,
    BP_Z16 = 5,
    BP_YZ4 = 6,   // thin-grid 3D convolution, padded z length 4 / 8
    BP_YZ8 = 7,
    BP_F = 8,     // finalisation
    BP_N = 9
};
enum BatchXKind { BX_FWD = 0, BX_ROW = 1, BX_INV = 2 };
enum BatchColKind { BC_CONV2 = 0, BC_YFWD = 1, BC_YINV = 2, BC_ZCONV = 3, BC_YZ = 4 };
// Tile shapes of the x passes and the 2D column pass: wide (the single-grid
// wide workgroups: 768 / 256 threads) or narrow (192 / 64 threads, a quarter
// of the row pairs or columns per item; padded lengths <= 512 only).
enum BatchTile { TILE_WIDE = 0, TILE_NARROW = 1 };
// Padded lengths the batched passes serve: 64 <= px, py <= 1024, pz in {1, 4, 8, 16}.
bool batch_supported(int px, int py, int pz);
// Whether tile shape `tile` of pass p serves member m (every shape but the
// narrow x / 2D column shapes serves every member).
bool batch_tile_serves(int pass, int tile, const BMember& m);
// Tiles (work items) of member m in pass p with tile shape `tile`; 0 when the
// pass does not apply to it (or the shape does not serve it).
int batch_tiles(int pass, const BMember& m, int tile = TILE_WIDE);
// Workgroups of pass p (tile shape `tile`) that fit on one compute unit at once.
hipError_t batch_resident(int pass, int tile, int* per_cu);
hipError_t configure_batch_kernels(void);
// Every launcher takes the pass's work list and its number of persistent
// workgroups (a multiple of 8).  x passes: fi (and ff for the fused pass)
// hold the base pointers, stage descriptor and flags; the work list must be
// the one built for the tile shape.
hipError_t launch_bx(int kind, const BatchList& l, int grid, const FieldArgs& fi, const FieldArgs& ff, float a_last,
                     hipStream_t s, int tile);
// Column passes; base holds the spectrum, kernel and state base pointers, the
// twiddles and check_done.  2D y convolution of the members with nz = 1:
hipError_t launch_bcol3(const BatchList& l, int grid, const ColArgs& base, hipStream_t s, int tile);
// y transforms (forward, or inverse) of the members with nz > 1:
hipError_t launch_bcoly(int inverse, const BatchList& l, int grid, const ColArgs& base, hipStream_t s);
// z convolution of the members of one padded z length (pass BP_Z4 / BP_Z8 / BP_Z16):
hipError_t launch_bzconv(int pass, const BatchList& l, int grid, const ColArgs& base, hipStream_t s);
// thin-grid 3D convolution of the members of one padded z length (pass BP_YZ4 / BP_YZ8):
hipError_t launch_byz(int pass, const BatchList& l, int grid, const ColArgs& base, hipStream_t s);
hipError_t launch_bfinalize(const BatchList& l, int grid, const float* ms, float* m, const DevState* st,
                            hipStream_t s);
hipError_t launch_bcontroller(DevState* st, int n, int last_k, int evals, int check_done, int* active,
                              hipStream_t s);
hipError_t launch_bset_state(DevState* st, int n, double t, double dt, double t_end, double max_err,
                             double headroom, double dt_min, double dt_max, int order_low, int reset_counters,
                             int init_perm, hipStream_t s);

// ---- launchers (kernels_local.hip) -----------------------------------------
hipError_t launch_prepare_tables(const double* params64, RegionLut* lut, float* ptab,
                                 hipStream_t s);
hipError_t launch_twiddles(cf* tw, int pt, hipStream_t s);
hipError_t launch_combine(const FieldArgs& a, hipStream_t s);
// bd_in (optional): a magnetostatic field [3][ncell] to use instead of none
hipError_t launch_local(const FieldArgs& a, hipStream_t s, int* nblocks_out, const float* bd_in = nullptr);
// Surrogate check: accumulate max |b_sur - b_exact| and max |b_exact| (cell
// vectors) into st, then (gate) their ratio; above tol (or not finite) the
// attempt is marked failed.  sur_clear resets the failure flag.
hipError_t launch_sur_check(const float* b_sur, const float* b_exact, long long ncell, DevState* st, hipStream_t s);
hipError_t launch_sur_gate(DevState* st, double tol, hipStream_t s);
hipError_t launch_sur_clear(DevState* st, hipStream_t s);
hipError_t launch_llg(const FieldArgs& a, const float* beff, float* tau, int precess,
                      hipStream_t s);
hipError_t launch_set_state(DevState* st, double t, double dt, double t_end, double max_err,
                            double headroom, double dt_min, double dt_max, int order_low,
                            int reset_counters, int init_perm, long long target_steps,
                            hipStream_t s);
hipError_t launch_reset_accum(DevState* st, hipStream_t s);
hipError_t launch_controller(DevState* st, int last_k, int evals, int check_done, hipStream_t s);
hipError_t launch_finalize(const FieldArgs& a, hipStream_t s);
hipError_t launch_final_combine(const FieldArgs& a, hipStream_t s);
// thermal field (kernels_thermal.hip): bth = eta sigma[r] / sqrt(dt) for the
// generator step `step` and time step dt, or (from_state) for the state's
// therm_step and dt; sigma[256] = sqrt(2 alpha kB T / (Msat gamma dV)) (FP32)
hipError_t launch_thermal(long long ncell, const uint8_t* region, const float* sigma, unsigned long long seed,
                          const DevState* st, int from_state, unsigned long long step, double dt, int check_done,
                          float* bth, hipStream_t s);
hipError_t launch_set_therm_step(DevState* st, unsigned long long step, hipStream_t s);
// fused Heun stage without the magnetostatic term (kernels_local.hip)
struct HeunLocal {
    const float* sigma;       // thermal prefactors per region, null at 0 K
    unsigned long long seed;
    float* mnew;              // second stage: new state m0 + dt (k1 + k2)/2 written here
};
hipError_t launch_local_heun(const FieldArgs& a, const HeunLocal& h, hipStream_t s);
hipError_t launch_reduce_energy(const double* partials, int nblocks, DevState* st, double cellvol,
                                hipStream_t s);
hipError_t launch_exchange_dump(const FieldArgs& a, float* out, hipStream_t s);

// ---- demag kernel construction (kernels_demag.hip) -------------------------
hipError_t demag_tensor_octant(int nx, int ny, int nz, double dx, double dy, double dz,
                               double* out, hipStream_t s);
// periodic images: oct[c][k][j][i] = sum over the images of the box
// displacement (i, j, k) of the window tensor win[c][|dk|][|dj|][|di|], the
// negative displacements by parity (win: lengths w[3] = n P or n)
hipError_t demag_fold_images(int nx, int ny, int nz, const int* w, const int* pbc, const double* win,
                             double* oct, hipStream_t s);
hipError_t demag_kernel_spectrum(int nx, int ny, int nz, int px, int py, int pz,
                                 const double* octant, double2* work, float* khat, int ncomp,
                                 int kx, hipStream_t s);

}  // namespace mm
