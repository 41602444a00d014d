// mm_api.cpp -- the C ABI of include/mm.h: context, validation, solver
// drivers (Runge-Kutta stage sequencing, device-side step control, relax).
#include <algorithm>
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/mm.h"
#include "extra_field.h"
#include "mm_internal.h"
#include "api_common.h"
#include "sno_internal.h"
#include "tableau.h"

using namespace mm;

namespace {

// Event pairs are created when timing is enabled (not in the launch path) and
// handed out in order; `used` of them hold launches.
struct TimingClass {
    bool enabled = false;
    size_t used = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
constexpr size_t TIMING_POOL = 4096;
// launch classes: 0 x-forward, 1 column passes, 2 x-inverse, 3 fused x-inverse + x-forward
constexpr int NTIMING = 4;

// Spectrum of mm_beff_noalloc: one fixed array per GPU, alive until the
// process ends.  In host code `scratch` is only a stand-in for the symbol; its
// device address on each GPU comes from hipGetSymbolAddress (static_scratch).
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)MM_STATIC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device `dev`, resolved once
// per device (the first mm_create on it).
hipError_t static_scratch(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

}  // namespace

struct mm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int nx = 0, ny = 0, nz = 0, nrows = 0;
    double dx = 0, dy = 0, dz = 0;
    int px = 1, py = 1, pz = 1, kx = 1, ncomp = 4;
    bool yz = false;  // thin 3D grid: y FFT, z DFT with K^ and inverse y FFT in one pass
    long long ncell = 0, colstride = 0, zstride = 0, spec_elems = 0, khat_elems = 0;
    int pt = 1, twshift = 0;
    bool demag_on = true, khat_ready = false;
    int pbc[3] = {0, 0, 0};  // images per side (0: open boundary)
    // periodic axes transformed at their own length (no zero padding): x of
    // any grid, y of 2D grids whose column pass holds whole columns
    bool full_x = false, full_y = false;
    int win[3] = {1, 1, 1};  // tensor window per axis: n P, or n
    uint8_t* region = nullptr;
    double* params64 = nullptr;
    RegionLut* lut = nullptr;
    float* ptab = nullptr;
    cf* tw = nullptr;
    cf* spec = nullptr;
    float* khat = nullptr;
    float* kbuf = nullptr;
    float* ms = nullptr;   // stage state
    float* ms2 = nullptr;  // second stage-state buffer of the fused passes
    void* dft_tab = nullptr;  // split DFT matrices of the matrix-core y convolution
    float* zker = nullptr;    // thin 3D grids: the kernel transformed back along z
    int conv_prec = MM_PREC_FP32;
    DevState* st = nullptr;
    double* partials = nullptr;
    DevState* hst = nullptr;  // pinned host mirror of st
    long long dev_bytes = 0;
    bool fsal_valid = false;
    const float* fsal_m = nullptr;
    int fsal_precess = -1;
    int fsal_solver = 0;
    TimingClass timing[NTIMING];
    // surrogate of the magnetostatic field at the inner Dormand-Prince stages
    const mm_sno* sno = nullptr;
    double sur_tol = 1e-4;
    bool sur_active = false;  // this run still uses it (cleared by a fallback)
    float* bsur = nullptr;    // its prediction [3][ncell]
    float* bexact = nullptr;  // the exact B_demag of the last stage [3][ncell]
    long long sur_steps = 0;  // accepted steps taken with surrogate stages
    // thermal field (section "Thermal fluctuations")
    double temp[NREG] = {};   // temperature per region (K)
    bool therm_on = false;    // some magnetic region has T > 0
    unsigned long long seed = 0;
    float* sigma = nullptr;   // [256] sqrt(2 alpha kB T / (Msat gamma dV)), FP32
    float* bth = nullptr;     // thermal field of the current step [3][ncell]
    mm_params* hparams = nullptr;  // host copy of the parameters
    // cubic anisotropy (section "Magneto-crystalline anisotropy")
    bool cub_on = false;
    float4* cub = nullptr;    // [256][3] device table
    double hkc[NREG][3] = {}, hc1[NREG][3] = {}, hc2[NREG][3] = {};
    // induced DMI (section "Dzyaloshinskii-Moriya interaction")
    bool dmi_on = false;
    float2* dmi = nullptr;    // [256] (2 D/Msat, D/(2 A))
    double hdind[NREG] = {};
    // mm_run replays one captured attempt as a HIP graph on a stream of its own
    // (opt-in: measured slower than direct launches on this stack)
    bool run_graphs = false;
    hipStream_t gstream = nullptr;
    hipEvent_t ev_user = nullptr, ev_graph = nullptr;
    // time-dependent excitation terms f_k(t) g_k(r) (caller-owned profiles)
    ExcTerm exc[MAX_EXC] = {};
    bool relaxing = false;    // relax runs without excitations
    void* scratch = nullptr;  // this device's static spectrum array (mm_beff_noalloc)
};

namespace {

hipError_t dalloc(mm_ctx* c, void** p, size_t bytes) {
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) c->dev_bytes += (long long)bytes;
    return e;
}

void free_all(mm_ctx* c) {
    void* ptrs[] = {c->region, c->params64, c->lut,      c->ptab,    c->tw,   c->spec,   c->khat, c->kbuf,
                    c->ms,     c->ms2,      c->st,       c->partials, c->dft_tab, c->bsur, c->bexact, c->zker,
                    c->sigma,  c->bth,      c->cub,      c->dmi};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete c->hparams;
    if (c->ev_user) (void)hipEventDestroy(c->ev_user);
    if (c->ev_graph) (void)hipEventDestroy(c->ev_graph);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->hst) (void)hipHostFree(c->hst);
    for (auto& t : c->timing)
        for (auto& pr : t.ev) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
}

FieldArgs base_args(mm_ctx* c, const float* m0) {
    FieldArgs a;
    memset(&a, 0, sizeof(a));
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.nrows = c->nrows;
    a.ncell = c->ncell;
    a.m0 = m0;
    a.ms = c->ms;
    a.region = c->region;
    a.lut = c->lut;
    a.ptab = c->ptab;
    a.idx2 = (float)(1.0 / (c->dx * c->dx));
    a.idy2 = (float)(1.0 / (c->dy * c->dy));
    a.idz2 = (float)(1.0 / (c->dz * c->dz));
    a.kbuf = c->kbuf;
    a.st = c->st;
    a.sd.out_k = -1;
    a.spec = c->spec;
    a.colstride = c->colstride;
    a.zstride = c->zstride;
    a.tw = c->tw;
    a.twshift = c->twshift;
    a.partials = c->partials;
    a.cellvol = (float)(c->dx * c->dy * c->dz);
    a.pbc = (c->pbc[0] > 0 ? 1 : 0) | (c->pbc[1] > 0 ? 2 : 0) | (c->pbc[2] > 0 ? 4 : 0);
    a.cub = c->cub_on ? c->cub : nullptr;
    a.dmi = c->dmi_on ? c->dmi : nullptr;
    a.full_x = c->full_x ? 1 : 0;
    return a;
}

// Per-launch timing of one launch class: the events are handed to the
// launches (start on the first kernel of the class, stop on the last), which
// record them at the kernels' own start and end.
struct Timed {
    mm_ctx* c;
    int which;
    hipEvent_t e1 = nullptr, e2 = nullptr;
    Timed(mm_ctx* c_, int w, bool on = true) : c(c_), which(w) {
        TimingClass& t = c->timing[which];
        if (!on || !t.enabled) return;
        if (t.used == t.ev.size()) {
            hipEvent_t a = nullptr, b = nullptr;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return;
            }
            t.ev.emplace_back(a, b);
        }
        e1 = t.ev[t.used].first;
        e2 = t.ev[t.used].second;
        ++t.used;
    }
};

// The column (y / z) passes between the two x passes of a field evaluation.
int run_cols(mm_ctx* c, bool check_done, cf* spec, bool timed = true) {
    hipStream_t s = c->stream;
    ColArgs ca;
    memset(&ca, 0, sizeof(ca));
    ca.spec = spec;
    ca.tw = c->tw;
    ca.twshift = c->twshift;
    ca.st = c->st;
    ca.check_done = check_done ? 1 : 0;
    ca.khat = c->khat;
    ca.full = c->full_y ? 1 : 0;
    ca.kyh = c->py / 2 + 1;
    ca.kzh = c->pz / 2 + 1;
    ca.pa = c->py;
    Timed t(c, 1, timed);
    if (c->yz) {
        // thin 3D grid: one pass per kx column over all planes
        ca.pos_stride = 3;
        ca.col_stride = c->colstride;
        ca.ncol = c->kx;
        ca.outer_stride = c->zstride;
        ca.nouter = c->nz;
        ca.n_in = c->ny;
        ca.n_out = c->ny;
        ca.khat = c->zker;
        MM_TRY(launch_yz(c->py, c->pz, ca, s, t.e1, t.e2));
    } else if (c->pz > 1) {
        // y transforms of every (kx, z) column, in place (ny rows -> py rows);
        // tiles of adjacent z planes of one kx
        ca.pos_stride = 3;
        ca.col_stride = c->zstride;
        ca.ncol = c->nz;
        ca.outer_stride = c->colstride;
        ca.nouter = c->kx;
        const bool ypass = c->py > 1;
        // matrix-core DFT stages (BF16 / FP16 split products) when selected
        const bool mc = c->conv_prec != MM_PREC_FP32;
        if (mc) ca.dft_tab = c->dft_tab;
        if (ypass) {
            ca.n_in = c->ny;
            ca.n_out = c->py;
            if (mc)
                MM_TRY(launch_colm3d(c->py, COL_FWD, c->conv_prec, ca, s, t.e1, nullptr));
            else
                MM_TRY(launch_col(c->py, COL_FWD, ca, 6, s, t.e1, nullptr));
        }
        // z convolution of every (kx, ky) column; tiles of adjacent ky
        ca.pos_stride = c->zstride;
        ca.col_stride = 3;
        ca.ncol = c->py;
        ca.outer_stride = c->colstride;
        ca.nouter = c->kx;
        ca.n_in = c->nz;
        ca.n_out = c->nz;
        if (mc)
            MM_TRY(launch_colm3d(c->pz, COL_CONV, c->conv_prec, ca, s, ypass ? nullptr : t.e1, ypass ? nullptr : t.e2));
        else
            MM_TRY(launch_col(c->pz, COL_CONV, ca, 6, s, ypass ? nullptr : t.e1, ypass ? nullptr : t.e2));
        if (ypass) {
            ca.pos_stride = 3;
            ca.col_stride = c->zstride;
            ca.ncol = c->nz;
            ca.outer_stride = c->colstride;
            ca.nouter = c->kx;
            ca.n_in = c->py;
            ca.n_out = c->ny;
            if (mc)
                MM_TRY(launch_colm3d(c->py, COL_INV, c->conv_prec, ca, s, nullptr, t.e2));
            else
                MM_TRY(launch_col(c->py, COL_INV, ca, 6, s, nullptr, t.e2));
        }
    } else {
        // 2D: y convolution of every kx column; the DC and Nyquist columns
        // (both real along y) share the first workgroup
        ca.pos_stride = 3;
        ca.col_stride = c->colstride;
        ca.ncol = c->px >= 2 ? c->px / 2 : 1;
        ca.pack_col = c->px >= 2 ? c->px / 2 : 0;
        ca.outer_stride = 0;
        ca.nouter = 1;
        ca.n_in = c->ny;
        ca.n_out = c->ny;
        if (c->conv_prec != MM_PREC_FP32) {
            ca.dft_tab = c->dft_tab;
            MM_TRY(launch_colm(c->py, c->conv_prec, ca, s, t.e1, t.e2));
        } else {
            MM_TRY(launch_col(c->py, COL_CONV, ca, 4, s, t.e1, t.e2));
        }
    }
    return MM_OK;
}

int run_xfwd(mm_ctx* c, const FieldArgs& a, bool timed = true) {
    Timed t(c, 0, timed);
    MM_TRY(launch_xfwd(c->px, a, c->stream, t.e1, t.e2));
    return MM_OK;
}

int run_xinv(mm_ctx* c, const FieldArgs& a, int* nblocks_out, bool timed = true) {
    Timed t(c, 2, timed);
    MM_TRY(launch_xinv(c->px, a, c->stream, nblocks_out, t.e1, t.e2));
    return MM_OK;
}

// One field evaluation (section "Landau-Lifshitz torque": B_eff and torque).
// Per-region prefactor of the thermal field, sqrt(2 alpha kB T / (Msat gamma dV))
// (section "Thermal fluctuations", with B_sat = mu0 Msat), in FP64, stored FP32.
int upload_sigma(mm_ctx* c) {
    const double kb = 1.380649e-23;
    const double gamma = c->hparams->gamma_ll != 0.0 ? c->hparams->gamma_ll : GAMMA_DEFAULT;
    const double vol = c->dx * c->dy * c->dz;
    float sig[NREG];
    bool on = false;
    for (int r = 0; r < NREG; ++r) {
        const double ms = c->hparams->msat[r], al = c->hparams->alpha[r], t = c->temp[r];
        const double v = (ms > 0.0 && t > 0.0) ? sqrt(2.0 * al * kb * t / (ms * gamma * vol)) : 0.0;
        sig[r] = (float)v;
        on = on || sig[r] != 0.f;
    }
    c->therm_on = on;
    MM_TRY(hipMemcpyAsync(c->sigma, sig, sizeof(sig), hipMemcpyHostToDevice, c->stream));
    MM_TRY(hipStreamSynchronize(c->stream));
    return MM_OK;
}

// Cubic anisotropy table: c1, c2 normalised, c3 = c1 x c2, coefficients
// -2 Kc1/Msat, -2 Kc2/Msat, -4 Kc3/Msat (FP64, stored FP32); zero for
// non-magnetic regions.
int upload_cubic(mm_ctx* c) {
    float4 tab[NREG * 3];
    bool on = false;
    for (int r = 0; r < NREG; ++r) {
        const double ms = c->hparams->msat[r];
        double u[3], v[3], w[3];
        const double nu = sqrt(c->hc1[r][0] * c->hc1[r][0] + c->hc1[r][1] * c->hc1[r][1] + c->hc1[r][2] * c->hc1[r][2]);
        const double nv = sqrt(c->hc2[r][0] * c->hc2[r][0] + c->hc2[r][1] * c->hc2[r][1] + c->hc2[r][2] * c->hc2[r][2]);
        for (int i = 0; i < 3; ++i) {
            u[i] = nu > 0.0 ? c->hc1[r][i] / nu : 0.0;
            v[i] = nv > 0.0 ? c->hc2[r][i] / nv : 0.0;
        }
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
        const double inv = ms > 0.0 ? 1.0 / ms : 0.0;
        const double k1 = -2.0 * c->hkc[r][0] * inv, k2 = -2.0 * c->hkc[r][1] * inv, k3 = -4.0 * c->hkc[r][2] * inv;
        tab[3 * r] = make_float4((float)u[0], (float)u[1], (float)u[2], (float)k1);
        tab[3 * r + 1] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)k2);
        tab[3 * r + 2] = make_float4((float)w[0], (float)w[1], (float)w[2], (float)k3);
        on = on || k1 != 0.0 || k2 != 0.0 || k3 != 0.0;
    }
    c->cub_on = on;
    MM_TRY(hipMemcpyAsync(c->cub, tab, sizeof(tab), hipMemcpyHostToDevice, c->stream));
    MM_TRY(hipStreamSynchronize(c->stream));
    return MM_OK;
}

// DMI table: 2 D/Msat and D/(2 A) per region in FP64, stored FP32 (0 for
// non-magnetic regions; D/(2A) = 0 where A = 0).
int upload_dmi(mm_ctx* c) {
    float2 tab[NREG];
    bool on = false;
    for (int r = 0; r < NREG; ++r) {
        const double ms = c->hparams->msat[r], aex = c->hparams->aex[r], d = c->hdind[r];
        const double pre = ms > 0.0 ? 2.0 * d / ms : 0.0;
        const double xi = (ms > 0.0 && aex > 0.0) ? d / (2.0 * aex) : 0.0;
        tab[r] = make_float2((float)pre, (float)xi);
        on = on || pre != 0.0;
    }
    c->dmi_on = on;
    MM_TRY(hipMemcpyAsync(c->dmi, tab, sizeof(tab), hipMemcpyHostToDevice, c->stream));
    MM_TRY(hipStreamSynchronize(c->stream));
    return MM_OK;
}

int run_field(mm_ctx* c, FieldArgs& a, int* nblocks_out, bool timed = true) {
    hipStream_t s = c->stream;
    if (c->demag_on) {
        if (!c->khat_ready) return MM_ESTATE;
        a.flags |= EPI_HAS_DEMAG;
        MM_CHECK(run_xfwd(c, a, timed));
        MM_CHECK(run_cols(c, (a.flags & EPI_CHECK_DONE) != 0, a.spec, timed));
        MM_CHECK(run_xinv(c, a, nblocks_out, timed));
    } else {
        if (a.sd.nk > 0) MM_TRY(launch_combine(a, s));
        MM_TRY(launch_local(a, s, nblocks_out));
    }
    return MM_OK;
}

int sync_state(mm_ctx* c) {
    MM_TRY(hipMemcpyAsync(c->hst, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    MM_TRY(hipStreamSynchronize(c->stream));
    return MM_OK;
}

struct Opts {
    double max_err, headroom, dt_min, dt_max;
    int precess;
};

Opts get_opts(const mm_solver_opts* o) {
    Opts r{1e-5, 0.8, 0.0, 0.0, 1};
    if (o) {
        if (o->max_err > 0.0) r.max_err = o->max_err;
        if (o->headroom > 0.0) r.headroom = o->headroom;
        if (o->dt_min > 0.0) r.dt_min = o->dt_min;
        if (o->dt_max > 0.0) r.dt_max = o->dt_max;
        r.precess = o->precess ? 1 : 0;
    }
    return r;
}

// Cells that do not interact: no magnetostatic term, no exchange (Aex = 0 in
// every magnetic region), no DMI, no excitation.
bool uncoupled(const mm_ctx* c) {
    if (c->demag_on || c->dmi_on) return false;
    for (const auto& e : c->exc)
        if (e.g) return false;
    for (int r = 0; r < NREG; ++r)
        if (c->hparams->msat[r] > 0.0 && c->hparams->aex[r] != 0.0) return false;
    return true;
}

int n_exc(const mm_ctx* c) {
    int n = 0;
    for (const auto& e : c->exc) n += e.g != nullptr;
    return n;
}

// Stage time fraction c_s of tableau tb: the row sum of a.
double stage_c(const Tableau& tb, int s) {
    double v = 0.0;
    for (int j = 0; j < s; ++j) v += tb.a[s][j];
    return v;
}

// The additive field of a field evaluation at t + cs dt (t, dt on the device):
// the thermal field of the step when `thermal` (Heun stages) and the
// excitation terms (not during relax), into the field buffer the pass adds.
int prep_extra(mm_ctx* c, FieldArgs& a, double cs, bool thermal, bool check_done) {
    const bool th = thermal && c->therm_on;
    const int nx = c->relaxing ? 0 : n_exc(c);
    if (!th && nx == 0) return MM_OK;
    ExtraArgs e{};
    e.ncell = c->ncell;
    e.region = c->region;
    e.sigma = th ? c->sigma : nullptr;
    e.seed = c->seed;
    e.nexc = 0;
    if (nx > 0)
        for (const auto& t : c->exc)
            if (t.g) e.exc[e.nexc++] = t;
    MM_TRY(launch_extra_field(e, c->st, cs, check_done ? 1 : 0, c->bth, c->stream));
    a.flags |= EPI_THERM;
    a.bth = c->bth;
    return MM_OK;
}

// Torque of the committed state into logical derivative 0 (first stage).
int eval_first(mm_ctx* c, const float* m, int precess) {
    FieldArgs a = base_args(c, m);
    a.sd.nk = 0;
    a.sd.out_k = 0;
    a.flags = EPI_TORQUE | (precess ? EPI_PRECESS : 0);
    MM_CHECK(prep_extra(c, a, 0.0, false, false));
    return run_field(c, a, nullptr);
}

// Field arguments of stage s of tableau tb: combine over the non-zero a_sj,
// torque into logical derivative s, error norm on the last stage.
FieldArgs stage_args(mm_ctx* c, float* m, const Tableau& tb, int s, int precess, bool check_done) {
    FieldArgs a = base_args(c, m);
    const bool last = fill_stage(tb, s, a.sd);
    a.flags = EPI_TORQUE | (precess ? EPI_PRECESS : 0) | (check_done ? EPI_CHECK_DONE : 0);
    if (last) a.flags |= EPI_ERR;
    return a;
}

// One Dormand-Prince attempt whose inner stages 2..S-1 take the magnetostatic
// field from the surrogate (stage combine, surrogate, local terms and torque);
// the last stage, at the new state, is exact and also writes B_demag, which
// the surrogate's prediction at the same state is checked against before the
// controller (a miss rejects the attempt with dt kept).
int attempt_surrogate(mm_ctx* c, float* m, const Tableau& tb, int precess, bool check_done) {
    const int S = tb.stages;
    hipStream_t s = c->stream;
    for (int st = 1; st < S - 1; ++st) {
        FieldArgs a = stage_args(c, m, tb, st, precess, check_done);
        a.flags |= EPI_HAS_DEMAG;
        MM_TRY(launch_combine(a, s));
        MM_TRY(sno_run(c->sno, c->ms, c->bsur, s));
        MM_TRY(launch_local(a, s, nullptr, c->bsur));
    }
    FieldArgs al = stage_args(c, m, tb, S - 1, precess, check_done);
    al.flags |= EPI_BDEMAG;
    al.bdemag = c->bexact;
    MM_CHECK(run_field(c, al, nullptr));
    MM_TRY(sno_run(c->sno, c->ms, c->bsur, s));
    MM_TRY(launch_sur_check(c->bsur, c->bexact, c->ncell, c->st, s));
    MM_TRY(launch_sur_gate(c->st, c->sur_tol, s));
    MM_TRY(launch_controller(c->st, S - 1, S - 1, check_done ? 1 : 0, s));
    FieldArgs f = base_args(c, m);
    MM_TRY(launch_finalize(f, s));
    return MM_OK;
}

// One attempt of an embedded pair: stages 2..S, controller, finalisation.
// With the magnetostatic term (and px >= 8) the x-inverse pass of every inner
// stage and the x-forward pass of the next one run as one fused pass; the
// stage state then alternates between two buffers.
int attempt(mm_ctx* c, float* m, const Tableau& tb, int precess, bool check_done) {
    const int S = tb.stages;
    if (c->sur_active && c->demag_on && S == 7 && n_exc(c) == 0) {
        if (!c->khat_ready) return MM_ESTATE;
        return attempt_surrogate(c, m, tb, precess, check_done);
    }
    float* fin_ms = c->ms;
    // (an unpadded periodic x of 4096 points keeps the separate passes: its
    // fused form would hold 16 points of both parts per thread)
    if (c->demag_on && c->px >= 8 && S > 2 && !(c->full_x && c->px >= 4096)) {
        if (!c->khat_ready) return MM_ESTATE;
        float* buf[2] = {c->ms, c->ms2};
        int cur = 0;
        FieldArgs a = stage_args(c, m, tb, 1, precess, check_done);
        a.flags |= EPI_HAS_DEMAG;
        a.ms = buf[cur];
        MM_CHECK(run_xfwd(c, a));
        MM_CHECK(run_cols(c, check_done, c->spec));
        for (int s = 1; s < S - 1; ++s) {
            FieldArgs ai = stage_args(c, m, tb, s, precess, check_done);
            ai.flags |= EPI_HAS_DEMAG;
            ai.ms = buf[cur];
            FieldArgs af = stage_args(c, m, tb, s + 1, precess, check_done);
            af.flags |= EPI_HAS_DEMAG;
            af.ms = buf[cur ^ 1];
            // the k_s term (always the last one listed) comes from the fused pass
            float a_last = 0.f;
            if (af.sd.nk > 0 && af.sd.kidx[af.sd.nk - 1] == s) {
                a_last = af.sd.a[af.sd.nk - 1];
                --af.sd.nk;
            }
            MM_CHECK(prep_extra(c, ai, stage_c(tb, s), false, check_done));
            {
                Timed t(c, 3);
                MM_TRY(launch_xrow(c->px, ai, af, a_last, c->stream, t.e1, t.e2));
            }
            cur ^= 1;
            MM_CHECK(run_cols(c, check_done, c->spec));
        }
        FieldArgs al = stage_args(c, m, tb, S - 1, precess, check_done);
        al.flags |= EPI_HAS_DEMAG;
        al.ms = buf[cur];
        MM_CHECK(prep_extra(c, al, stage_c(tb, S - 1), false, check_done));
        MM_CHECK(run_xinv(c, al, nullptr));
        fin_ms = buf[cur];
    } else {
        for (int s = 1; s < S; ++s) {
            FieldArgs a = stage_args(c, m, tb, s, precess, check_done);
            MM_CHECK(prep_extra(c, a, stage_c(tb, s), false, check_done));
            MM_CHECK(run_field(c, a, nullptr));
        }
    }
    MM_TRY(launch_controller(c->st, S - 1, S - 1, check_done ? 1 : 0, c->stream));
    FieldArgs f = base_args(c, m);
    f.ms = fin_ms;
    MM_TRY(launch_finalize(f, c->stream));
    return MM_OK;
}

// One Heun (RK12) attempt (section "Dynamics"; with the thermal field,
// section "Thermal fluctuations"): the thermal field of the step, k1 at m0, k2
// at m0 + dt k1 with the Euler error estimate, the new state
// m0 + dt (k1 + k2)/2 into the stage buffer (before the controller changes
// dt), the controller, and the commit of an accepted state.  The thermal
// field is held over both stages; its generator step advances per accepted
// step.
int heun_attempt(mm_ctx* c, float* m, int precess, bool check_done) {
    hipStream_t s = c->stream;
    const bool th = c->therm_on;
    if (!c->demag_on && n_exc(c) == 0) {
        // no convolution: two fused local passes (noise generated in place,
        // the new state formed by the second), the stage combine between them
        HeunLocal h{th ? c->sigma : nullptr, c->seed, nullptr};
        FieldArgs a0 = base_args(c, m);
        a0.sd.nk = 0;
        a0.sd.out_k = 0;
        a0.flags = EPI_TORQUE | (precess ? EPI_PRECESS : 0) | (check_done ? EPI_CHECK_DONE : 0);
        MM_TRY(launch_local_heun(a0, h, s));
        FieldArgs a1 = stage_args(c, m, RK12, 1, precess, check_done);
        MM_TRY(launch_combine(a1, s));
        h.mnew = c->ms2;
        MM_TRY(launch_local_heun(a1, h, s));
        MM_TRY(launch_controller(c->st, 0, 2, check_done ? 1 : 0, s));
        FieldArgs fin = base_args(c, m);
        fin.ms = c->ms2;
        MM_TRY(launch_finalize(fin, s));
        return MM_OK;
    }
    FieldArgs a0 = base_args(c, m);
    a0.sd.nk = 0;
    a0.sd.out_k = 0;
    a0.flags = EPI_TORQUE | (precess ? EPI_PRECESS : 0) | (check_done ? EPI_CHECK_DONE : 0);
    MM_CHECK(prep_extra(c, a0, 0.0, true, check_done));
    MM_CHECK(run_field(c, a0, nullptr));
    FieldArgs a1 = stage_args(c, m, RK12, 1, precess, check_done);
    MM_CHECK(prep_extra(c, a1, 1.0, true, check_done));
    MM_CHECK(run_field(c, a1, nullptr));
    FieldArgs f = base_args(c, m);
    f.sd.nk = 2;
    f.sd.kidx[0] = 0;
    f.sd.kidx[1] = 1;
    f.sd.a[0] = 0.5f;
    f.sd.a[1] = 0.5f;
    f.flags = check_done ? EPI_CHECK_DONE : 0;
    MM_TRY(launch_combine(f, s));
    MM_TRY(launch_controller(c->st, 0, 2, check_done ? 1 : 0, s));
    FieldArgs fin = base_args(c, m);
    MM_TRY(launch_finalize(fin, s));
    return MM_OK;
}

bool timing_any(const mm_ctx* c) {
    for (const auto& t : c->timing)
        if (t.enabled) return true;
    return false;
}

// One mm_run attempt captured as a graph.  Every kernel argument is fixed for
// the run (buffers, solver, flags); what changes per attempt -- t, dt, the
// stage map, the generator step -- lives in the device-side solver state, so
// replays are the same launches.  The capture runs on the context's own
// stream (default priority); on failure the caller launches directly.
int capture_attempt(mm_ctx* c, float* m, const Tableau& tb, bool heun, int precess, hipGraphExec_t* out) {
    *out = nullptr;
    if (!c->gstream) {
        MM_TRY(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        MM_TRY(hipEventCreateWithFlags(&c->ev_user, hipEventDisableTiming));
        MM_TRY(hipEventCreateWithFlags(&c->ev_graph, hipEventDisableTiming));
    }
    hipStream_t user = c->stream;
    c->stream = c->gstream;
    hipError_t e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        c->stream = user;
        return map_err(e);
    }
    const int st = heun ? heun_attempt(c, m, precess, true) : attempt(c, m, tb, precess, true);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->gstream, &g);
    c->stream = user;
    if (st != MM_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return st != MM_OK ? st : map_err(e);
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) *out = nullptr;
    return map_err(e);
}

bool need_first(mm_ctx* c, const float* m, int precess, int solver) {
    return !(c->fsal_valid && c->fsal_m == m && c->fsal_precess == precess && c->fsal_solver == solver);
}

int embedded_step(mm_ctx* c, float* m, const Tableau& tb, int solver, double* t, double* dt,
                  const mm_solver_opts* o, int32_t* accepted, double* err) {
    if (!c || !m || !t || !dt) return MM_EINVAL;
    if (!(isfinite(*t) && finite_pos(*dt))) return MM_EINVAL;
    if (c->therm_on) return MM_EUNSUPPORTED;  // the thermal field needs Heun's fixed step
    const Opts op = get_opts(o);
    const bool first = need_first(c, m, op.precess, solver);
    MM_TRY(launch_set_state(c->st, *t, *dt, INFINITY, op.max_err, op.headroom, op.dt_min, op.dt_max,
                            tb.order_low, 1, first ? 1 : 0, 0, c->stream));
    if (first) {
        c->fsal_valid = false;
        MM_CHECK(eval_first(c, m, op.precess));
    }
    MM_CHECK(attempt(c, m, tb, op.precess, false));
    MM_CHECK(sync_state(c));
    c->fsal_valid = true;
    c->fsal_m = m;
    c->fsal_precess = op.precess;
    c->fsal_solver = solver;
    if (accepted) *accepted = c->hst->accepted;
    if (err) *err = c->hst->err;
    *t = c->hst->t;
    *dt = c->hst->dt;
    if (c->hst->status != 0) return c->hst->status;
    return MM_OK;
}

int energy_pass(mm_ctx* c, const float* m, double* out5) {
    FieldArgs a = base_args(c, m);
    a.flags = EPI_ENERGY;
    MM_CHECK(prep_extra(c, a, 0.0, false, false));
    int nb = 0;
    MM_CHECK(run_field(c, a, &nb));
    MM_TRY(launch_reduce_energy(c->partials, nb, c->st, c->dx * c->dy * c->dz, c->stream));
    MM_CHECK(sync_state(c));
    for (int i = 0; i < 5; ++i) out5[i] = c->hst->red[i];
    return MM_OK;
}

int maxtorque_pass(mm_ctx* c, const float* m, int precess, double* out) {
    MM_TRY(launch_reset_accum(c->st, c->stream));
    FieldArgs a = base_args(c, m);
    a.flags = EPI_MAXTQ | (precess ? EPI_PRECESS : 0);
    MM_CHECK(prep_extra(c, a, 0.0, false, false));
    MM_CHECK(run_field(c, a, nullptr));
    MM_CHECK(sync_state(c));
    unsigned int bits = c->hst->tq_bits;
    float f;
    memcpy(&f, &bits, sizeof(f));
    *out = (double)f;
    return MM_OK;
}

}  // namespace

extern "C" {

const char* mm_strerror(int status) {
    switch (status) {
        case MM_OK: return "ok";
        case MM_EINVAL: return "invalid argument";
        case MM_ENOMEM: return "device memory allocation failed";
        case MM_EDEVICE: return "HIP runtime error";
        case MM_EUNSUPPORTED: return "unsupported configuration (size, image window or feature)";
        case MM_ENONFINITE: return "non-finite error estimate";
        case MM_ESTEP: return "time step fell below dt_min";
        case MM_ENOTCONVERGED: return "relax did not reach the MaxErr floor within max_steps";
        case MM_ESTATE: return "call order: demag kernel not initialised";
        case MM_ESCRATCH: return "grid too large for the static spectrum of mm_beff_noalloc";
        default: return "unknown status";
    }
}

int mm_create(mm_ctx** out, const mm_grid* g, const mm_params* p, const uint8_t* region_dev,
              void* hip_stream) {
    if (!out || !g || !p || !region_dev) return MM_EINVAL;
    *out = nullptr;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return MM_EINVAL;
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz)) return MM_EINVAL;
    if (g->pbc[0] < 0 || g->pbc[1] < 0 || g->pbc[2] < 0) return MM_EINVAL;
    if (g->nx > 2048 || g->ny > 2048 || g->nz > 2048) return MM_EUNSUPPORTED;
    // image window: n P displacements (0 .. n P - 1) along a periodic axis
    long long win[3];
    const int nn[3] = {g->nx, g->ny, g->nz};
    for (int ax = 0; ax < 3; ++ax) {
        if (g->pbc[ax] > (1 << 20)) return MM_EUNSUPPORTED;
        win[ax] = g->pbc[ax] > 0 ? (long long)nn[ax] * g->pbc[ax] : nn[ax];
    }
    if (win[0] * win[1] * win[2] > (1LL << 26)) return MM_EUNSUPPORTED;
    // one component array must stay below 2^30 bytes (32-bit offsets in the kernels)
    if ((long long)g->nx * g->ny * g->nz > (1LL << 28)) return MM_EUNSUPPORTED;
    MM_CHECK(validate_params(p));
    mm_ctx* c = new (std::nothrow) mm_ctx();
    if (!c) return MM_ENOMEM;
    c->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&c->device);
    c->nx = g->nx;
    c->ny = g->ny;
    c->nz = g->nz;
    c->dx = g->dx;
    c->dy = g->dy;
    c->dz = g->dz;
    c->nrows = g->ny * g->nz;
    c->ncell = (long long)g->nx * g->ny * g->nz;
    for (int ax = 0; ax < 3; ++ax) {
        c->pbc[ax] = g->pbc[ax];
        c->win[ax] = (int)win[ax];
    }
    // A periodic axis needs no zero padding (the convolution along it is
    // cyclic): one whose length is a power of two is transformed at that length
    auto pow2 = [](int n) { return n >= 2 && (n & (n - 1)) == 0; };
    c->full_x = g->pbc[0] > 0 && pow2(g->nx);
    c->full_y = g->pbc[1] > 0 && g->nz == 1 && pow2(g->ny) && g->ny >= 64 && g->ny <= 2048;
    c->px = c->full_x ? g->nx : pad_len(g->nx);
    c->py = c->full_y ? g->ny : pad_len(g->ny);
    c->pz = pad_len(g->nz);
    if (c->px > 4096 || c->py > 4096 || c->pz > 4096) {
        delete c;
        return MM_EUNSUPPORTED;
    }
    c->kx = c->px / 2 + 1;
    c->ncomp = (c->pz > 1) ? 6 : 4;
    c->yz = c->pz > 1 && yz_supported(c->py, c->pz);
    // rows per spectrum column: py when the y transforms run in place, else ny
    const long long ycount = (c->pz > 1 && !c->yz) ? c->py : c->ny;
    // kx-major: the nz planes of one kx are adjacent, so the z transforms read
    // rows a plane apart within one kx block
    c->zstride = 3LL * ycount;
    c->colstride = c->zstride * c->nz;
    c->spec_elems = c->colstride * c->kx;
    c->khat_elems = (long long)c->kx * (c->py / 2 + 1) * (c->pz / 2 + 1) * c->ncomp;
    c->pt = c->px;
    if (c->py > c->pt) c->pt = c->py;
    if (c->pz > c->pt) c->pt = c->pz;
    c->twshift = ilog2(c->pt);
    const int maxblk_x = xinv_blocks(c->px, c->nrows);
    const long long maxblk_l = (c->ncell + NT - 1) / NT;
    const long long maxblk = maxblk_x > maxblk_l ? maxblk_x : maxblk_l;

    int st = MM_OK;
    auto A = [&](void** ptr, size_t bytes) {
        if (st != MM_OK) return;
        const hipError_t e = dalloc(c, ptr, bytes);
        if (e != hipSuccess) st = map_err(e);
    };
    A((void**)&c->region, (size_t)c->ncell);
    A((void**)&c->params64, sizeof(mm_params));
    A((void**)&c->lut, NREG * sizeof(RegionLut));
    A((void**)&c->ptab, (size_t)NREG * NREG * sizeof(float));
    A((void**)&c->tw, (size_t)c->pt * sizeof(cf));
    A((void**)&c->spec, (size_t)c->spec_elems * sizeof(cf));
    A((void**)&c->khat, (size_t)c->khat_elems * sizeof(float));
    A((void**)&c->kbuf, (size_t)MAXK * 3 * c->ncell * sizeof(float));
    A((void**)&c->ms, (size_t)3 * c->ncell * sizeof(float));
    A((void**)&c->ms2, (size_t)3 * c->ncell * sizeof(float));
    A((void**)&c->dft_tab, (size_t)2 * DFT_TABLE_BYTES);
    if (c->yz) A((void**)&c->zker, (size_t)c->kx * (c->py / 2 + 1) * zkernel_floats(c->pz) * sizeof(float));
    A((void**)&c->st, sizeof(DevState));
    A((void**)&c->partials, (size_t)maxblk * 4 * sizeof(double));
    if (st == MM_OK && hipHostMalloc((void**)&c->hst, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
        st = MM_ENOMEM;
    if (st == MM_OK) st = map_err(static_scratch(c->device, &c->scratch));
    if (st == MM_OK) {
        hipError_t e = hipMemcpyAsync(c->region, region_dev, (size_t)c->ncell, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(c->params64, p, sizeof(mm_params), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = launch_prepare_tables(c->params64, c->lut, c->ptab, c->stream);
        if (e == hipSuccess) e = launch_twiddles(c->tw, c->pt, c->stream);
        if (e == hipSuccess) e = configure_field_kernels(c->px, c->py, c->pz);
        if (e == hipSuccess) e = launch_dft_tables(c->dft_tab, c->stream);
        if (e == hipSuccess) e = configure_colm();
        if (e == hipSuccess) e = configure_colm3d();
        if (e == hipSuccess)
            e = launch_set_state(c->st, 0.0, 1e-14, INFINITY, 1e-5, 0.8, 0.0, 0.0, 4, 1, 1, 0, c->stream);
        if (e == hipSuccess) e = launch_set_therm_step(c->st, 0, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        st = map_err(e);
    }
    if (st == MM_OK) {
        c->hparams = new (std::nothrow) mm_params(*p);
        if (!c->hparams) st = MM_ENOMEM;
    }
    if (st != MM_OK) {
        free_all(c);
        delete c;
        return st;
    }
    *out = c;
    return MM_OK;
}

int mm_demag_kernel_init(mm_ctx* c) {
    if (!c) return MM_EINVAL;
    double* oct = nullptr;
    double* win = nullptr;  // the tensor over the image window (periodic grids)
    double2* work = nullptr;
    const bool periodic = c->pbc[0] > 0 || c->pbc[1] > 0 || c->pbc[2] > 0;
    hipError_t e = hipMalloc((void**)&oct, (size_t)6 * c->ncell * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc((void**)&work, (size_t)c->px * c->py * c->pz * sizeof(double2));
    if (e == hipSuccess && periodic)
        e = hipMalloc((void**)&win, (size_t)6 * c->win[0] * c->win[1] * c->win[2] * sizeof(double));
    if (e == hipSuccess && periodic) {
        e = demag_tensor_octant(c->win[0], c->win[1], c->win[2], c->dx, c->dy, c->dz, win, c->stream);
        if (e == hipSuccess) e = demag_fold_images(c->nx, c->ny, c->nz, c->win, c->pbc, win, oct, c->stream);
    } else if (e == hipSuccess) {
        e = demag_tensor_octant(c->nx, c->ny, c->nz, c->dx, c->dy, c->dz, oct, c->stream);
    }
    if (e == hipSuccess)
        e = demag_kernel_spectrum(c->nx, c->ny, c->nz, c->px, c->py, c->pz, oct, work, c->khat, c->ncomp,
                                  c->kx, c->stream);
    if (e == hipSuccess && c->yz) e = launch_zkernel(c->khat, c->zker, (long long)c->kx * (c->py / 2 + 1), c->pz, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (oct) (void)hipFree(oct);
    if (win) (void)hipFree(win);
    if (work) (void)hipFree(work);
    if (e != hipSuccess) return map_err(e);
    c->khat_ready = true;
    c->fsal_valid = false;
    return MM_OK;
}

int mm_set_params(mm_ctx* c, const mm_params* p) {
    if (!c) return MM_EINVAL;
    MM_CHECK(validate_params(p));
    MM_TRY(hipMemcpyAsync(c->params64, p, sizeof(mm_params), hipMemcpyHostToDevice, c->stream));
    MM_TRY(launch_prepare_tables(c->params64, c->lut, c->ptab, c->stream));
    MM_TRY(hipStreamSynchronize(c->stream));
    *c->hparams = *p;
    if (c->sigma) MM_CHECK(upload_sigma(c));
    if (c->cub) MM_CHECK(upload_cubic(c));
    if (c->dmi) MM_CHECK(upload_dmi(c));
    c->fsal_valid = false;
    return MM_OK;
}

int mm_set_temperature(mm_ctx* c, const double* temp_k, uint64_t seed) {
    if (!c) return MM_EINVAL;
    if (temp_k)
        for (int r = 0; r < NREG; ++r)
            if (!(temp_k[r] >= 0.0) || !isfinite(temp_k[r])) return MM_EINVAL;
    for (int r = 0; r < NREG; ++r) c->temp[r] = temp_k ? temp_k[r] : 0.0;
    c->seed = seed;
    if (!c->sigma) {
        MM_TRY(dalloc(c, (void**)&c->sigma, NREG * sizeof(float)));
        MM_TRY(dalloc(c, (void**)&c->bth, (size_t)3 * c->ncell * sizeof(float)));
    }
    MM_CHECK(upload_sigma(c));
    MM_TRY(launch_set_therm_step(c->st, 0, c->stream));
    MM_TRY(hipStreamSynchronize(c->stream));
    return MM_OK;
}

int mm_set_cubic_anisotropy(mm_ctx* c, const double* kc, const double* c1, const double* c2) {
    if (!c) return MM_EINVAL;
    if (kc && (!c1 || !c2)) return MM_EINVAL;
    for (int r = 0; r < NREG; ++r)
        for (int i = 0; i < 3; ++i) {
            c->hkc[r][i] = kc ? kc[3 * r + i] : 0.0;
            c->hc1[r][i] = kc ? c1[3 * r + i] : 0.0;
            c->hc2[r][i] = kc ? c2[3 * r + i] : 0.0;
            if (!isfinite(c->hkc[r][i]) || !isfinite(c->hc1[r][i]) || !isfinite(c->hc2[r][i])) return MM_EINVAL;
        }
    if (!c->cub) MM_TRY(dalloc(c, (void**)&c->cub, (size_t)NREG * 3 * sizeof(float4)));
    MM_CHECK(upload_cubic(c));
    c->fsal_valid = false;
    return MM_OK;
}

int mm_set_dmi(mm_ctx* c, const double* dind) {
    if (!c) return MM_EINVAL;
    for (int r = 0; r < NREG; ++r) {
        c->hdind[r] = dind ? dind[r] : 0.0;
        if (!isfinite(c->hdind[r])) return MM_EINVAL;
    }
    if (!c->dmi) MM_TRY(dalloc(c, (void**)&c->dmi, (size_t)NREG * sizeof(float2)));
    MM_CHECK(upload_dmi(c));
    c->fsal_valid = false;
    return MM_OK;
}

int mm_set_excitation(mm_ctx* c, int32_t slot, const float* g_dev, double a, double b, double omega, double phi) {
    if (!c || slot < 0 || slot >= MAX_EXC) return MM_EINVAL;
    if (g_dev && !(isfinite(a) && isfinite(b) && isfinite(omega) && isfinite(phi))) return MM_EINVAL;
    if (g_dev && !c->bth) MM_TRY(dalloc(c, (void**)&c->bth, (size_t)3 * c->ncell * sizeof(float)));
    c->exc[slot] = ExcTerm{g_dev, a, b, omega, phi};
    c->fsal_valid = false;
    return MM_OK;
}

int mm_set_run_graphs(mm_ctx* c, int32_t enable) {
    if (!c) return MM_EINVAL;
    c->run_graphs = enable != 0;
    return MM_OK;
}

int mm_thermal_field(mm_ctx* c, double dt, uint64_t step, float* out_dev) {
    if (!c || !out_dev || !finite_pos(dt)) return MM_EINVAL;
    if (!c->sigma) return MM_ESTATE;
    return map_err(launch_thermal(c->ncell, c->region, c->sigma, c->seed, c->st, 0, step, dt, 0, out_dev,
                                  c->stream));
}

int mm_set_demag(mm_ctx* c, int32_t enable) {
    if (!c) return MM_EINVAL;
    c->demag_on = enable != 0;
    c->fsal_valid = false;
    return MM_OK;
}

int mm_beff(mm_ctx* c, const float* m_dev, float* beff_dev, float* bdemag_dev) {
    if (!c || !m_dev || !beff_dev) return MM_EINVAL;
    FieldArgs a = base_args(c, m_dev);
    a.beff = beff_dev;
    a.bdemag = bdemag_dev;
    a.flags = EPI_BEFF | (bdemag_dev ? EPI_BDEMAG : 0);
    MM_CHECK(prep_extra(c, a, 0.0, false, false));
    return run_field(c, a, nullptr);
}

int mm_beff_noalloc(mm_ctx* c, const float* m_dev, float* beff_dev, float* bdemag_dev) {
    if (!c || !m_dev || !beff_dev) return MM_EINVAL;
    if (c->demag_on && (unsigned long long)c->spec_elems * sizeof(cf) > STATIC_SCRATCH_BYTES) return MM_ESCRATCH;
    if (!c->scratch) return MM_EDEVICE;
    FieldArgs a = base_args(c, m_dev);
    a.spec = static_cast<cf*>(c->scratch);
    a.beff = beff_dev;
    a.bdemag = bdemag_dev;
    a.flags = EPI_BEFF | (bdemag_dev ? EPI_BDEMAG : 0);
    MM_CHECK(prep_extra(c, a, 0.0, false, false));
    return run_field(c, a, nullptr, false);
}

int mm_llg_torque(mm_ctx* c, const float* m_dev, const float* beff_dev, float* tau_dev, int32_t precess) {
    if (!c || !m_dev || !beff_dev || !tau_dev) return MM_EINVAL;
    FieldArgs a = base_args(c, m_dev);
    return map_err(launch_llg(a, beff_dev, tau_dev, precess ? 1 : 0, c->stream));
}

int mm_torque(mm_ctx* c, const float* m_dev, float* tau_dev, int32_t precess) {
    if (!c || !m_dev || !tau_dev) return MM_EINVAL;
    FieldArgs a = base_args(c, m_dev);
    a.tau = tau_dev;
    a.flags = EPI_TORQUE | (precess ? EPI_PRECESS : 0);
    MM_CHECK(prep_extra(c, a, 0.0, false, false));
    return run_field(c, a, nullptr);
}

int mm_rk4_step(mm_ctx* c, float* m_dev, double dt, int32_t precess) {
    if (!c || !m_dev || !finite_pos(dt)) return MM_EINVAL;
    if (n_exc(c) > 0) return MM_EUNSUPPORTED;  // no time argument for the excitations
    c->fsal_valid = false;
    MM_TRY(launch_set_state(c->st, 0.0, dt, INFINITY, 1e-5, 0.8, 0.0, 0.0, 4, 0, 1, 0, c->stream));
    const int pf = precess ? EPI_PRECESS : 0;
    const float half = 0.5f;
    for (int s = 0; s < 4; ++s) {
        FieldArgs a = base_args(c, m_dev);
        a.sd.nk = s == 0 ? 0 : 1;
        a.sd.kidx[0] = s - 1;
        a.sd.a[0] = (s == 3) ? 1.0f : half;
        a.sd.out_k = s;
        a.flags = EPI_TORQUE | pf;
        MM_CHECK(run_field(c, a, nullptr));
    }
    FieldArgs f = base_args(c, m_dev);
    f.sd.nk = 4;
    const float b[4] = {1.0f / 6, 1.0f / 3, 1.0f / 3, 1.0f / 6};
    for (int j = 0; j < 4; ++j) {
        f.sd.kidx[j] = j;
        f.sd.a[j] = b[j];
    }
    MM_TRY(launch_final_combine(f, c->stream));
    return MM_OK;
}

int mm_rk45_step(mm_ctx* c, float* m_dev, double* t, double* dt, const mm_solver_opts* o, int32_t* accepted,
                 double* err) {
    return embedded_step(c, m_dev, DP45, 45, t, dt, o, accepted, err);
}

int mm_rk23_step(mm_ctx* c, float* m_dev, double* t, double* dt, const mm_solver_opts* o, int32_t* accepted,
                 double* err) {
    return embedded_step(c, m_dev, BS23, 23, t, dt, o, accepted, err);
}

int mm_run(mm_ctx* c, float* m_dev, int32_t solver, double t_end, int64_t max_attempts, double* t, double* dt,
           const mm_solver_opts* o, mm_run_stats* stats) {
    if (!c || !m_dev || !t || !dt || max_attempts < 0) return MM_EINVAL;
    if (solver != 45 && solver != 23 && solver != 12) return MM_EINVAL;
    if (!(isfinite(*t) && finite_pos(*dt)) || isnan(t_end)) return MM_EINVAL;
    // with the thermal field only Heun runs, at a fixed step
    if (c->therm_on && solver != 12) return MM_EUNSUPPORTED;
    const bool heun = solver == 12;
    const Tableau& tb = solver == 45 ? DP45 : (solver == 23 ? BS23 : RK12);
    Opts op = get_opts(o);
    double dt0 = *dt;
    if (isfinite(t_end) && *t + dt0 > t_end) dt0 = t_end - *t;
    if (!(dt0 > 0.0)) {  // nothing to do
        if (stats) memset(stats, 0, sizeof(*stats));
        return MM_OK;
    }
    if (heun && c->therm_on) {  // every step accepted, dt kept
        op.max_err = INFINITY;
        op.dt_min = 0.0;
        op.dt_max = dt0;
    }
    const bool first = !heun && need_first(c, m_dev, op.precess, solver);
    MM_TRY(launch_set_state(c->st, *t, dt0, t_end, op.max_err, op.headroom, op.dt_min, op.dt_max, tb.order_low,
                            1, first ? 1 : 0, 0, c->stream));
    long long extra = 0;
    if (first) {
        c->fsal_valid = false;
        MM_CHECK(eval_first(c, m_dev, op.precess));
        extra = 1;
    }
    long long per = (long long)(3e7 / (double)c->ncell);
    if (per < 4) per = 4;
    if (per > 64) per = 64;
    // with the surrogate every attempt is checked on the host: after a miss the
    // rest of the run takes the exact path
    c->sur_active = c->sno != nullptr && solver == 45 && c->demag_on;
    // Heun at finite temperature on uncoupled cells: whole chunks of fixed
    // steps in one launch each (every cell alone, its state in registers); the
    // last, clipped step of a run takes the general path
    if (heun && c->therm_on && uncoupled(c)) {
        MM_CHECK(sync_state(c));
        long long done_attempts = 0;
        while (done_attempts < max_attempts && !c->hst->done) {
            const long long cap = std::min<long long>(max_attempts - done_attempts, 4096);
            double tt = c->hst->t;
            long long n = 0;
            while (n < cap && !(isfinite(t_end) && tt + dt0 >= t_end)) {
                tt += dt0;
                ++n;
            }
            const long long before = c->hst->steps + c->hst->rejects;
            if (n > 0)
                MM_TRY(launch_heun_uncoupled(base_args(c, m_dev), c->sigma, c->seed, (int)n, op.precess, c->stream));
            else
                MM_CHECK(heun_attempt(c, m_dev, op.precess, true));
            done_attempts += n > 0 ? n : 1;
            MM_CHECK(sync_state(c));
            // every attempt either ends the run or counts a step or a reject
            if (!c->hst->done && c->hst->steps + c->hst->rejects == before) return MM_EDEVICE;
        }
        c->fsal_valid = false;
        *t = c->hst->t;
        *dt = c->hst->dt;
        if (stats) {
            stats->steps = c->hst->steps;
            stats->rejects = c->hst->rejects;
            stats->evals = c->hst->evals;
            stats->t = c->hst->t;
            stats->dt = c->hst->dt;
            stats->err = c->hst->err;
        }
        return c->hst->status != 0 ? c->hst->status : MM_OK;
    }
    // many attempts: replay one captured attempt (fewer host launches)
    hipGraphExec_t ge = nullptr;
    if (c->run_graphs && !c->sur_active && !timing_any(c) && max_attempts >= 16) {
        if (capture_attempt(c, m_dev, tb, heun, op.precess, &ge) != MM_OK) ge = nullptr;
    }
    long long done_attempts = 0;
    int rst = MM_OK;
    MM_CHECK(sync_state(c));
    while (done_attempts < max_attempts) {
        const long long before = c->hst->steps + c->hst->rejects;
        long long nb = max_attempts - done_attempts;
        if (nb > per) nb = per;
        if (c->sur_active) nb = 1;
        if (ge) {
            hipError_t e = hipEventRecord(c->ev_user, c->stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(c->gstream, c->ev_user, 0);
            for (long long i = 0; i < nb && e == hipSuccess; ++i) e = hipGraphLaunch(ge, c->gstream);
            if (e == hipSuccess) e = hipEventRecord(c->ev_graph, c->gstream);
            if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->ev_graph, 0);
            if (e != hipSuccess) {
                rst = map_err(e);
                break;
            }
        } else {
            for (long long i = 0; i < nb && rst == MM_OK; ++i)
                rst = heun ? heun_attempt(c, m_dev, op.precess, true) : attempt(c, m_dev, tb, op.precess, true);
            if (rst != MM_OK) break;
        }
        done_attempts += nb;
        rst = sync_state(c);
        if (rst != MM_OK) break;
        // every attempt either ends the run or counts a step or a reject (a
        // surrogate miss counts neither: it repeats the step on the exact path)
        if (!c->sur_active && !c->hst->done && c->hst->steps + c->hst->rejects == before) {
            rst = MM_EDEVICE;
            break;
        }
        if (c->sur_active) {
            if (c->hst->sur_fail) {
                c->sur_active = false;
                MM_TRY(launch_sur_clear(c->st, c->stream));
            } else if (c->hst->accepted) {
                ++c->sur_steps;
            }
        }
        if (c->hst->done) break;
    }
    if (ge) (void)hipGraphExecDestroy(ge);
    if (rst != MM_OK) return rst;
    c->sur_active = false;
    c->fsal_valid = !heun;  // Heun leaves no first-stage torque of the new state
    c->fsal_m = m_dev;
    c->fsal_precess = op.precess;
    c->fsal_solver = solver;
    *t = c->hst->t;
    *dt = c->hst->dt;
    if (stats) {
        stats->steps = c->hst->steps;
        stats->rejects = c->hst->rejects;
        stats->evals = c->hst->evals + extra;
        stats->t = c->hst->t;
        stats->dt = c->hst->dt;
        stats->err = c->hst->err;
    }
    return c->hst->status != 0 ? c->hst->status : MM_OK;
}

int mm_energy(mm_ctx* c, const float* m_dev, double* e_terms5) {
    if (!c || !m_dev || !e_terms5) return MM_EINVAL;
    return energy_pass(c, m_dev, e_terms5);
}

int mm_max_torque(mm_ctx* c, const float* m_dev, int32_t precess, double* out) {
    if (!c || !m_dev || !out) return MM_EINVAL;
    return maxtorque_pass(c, m_dev, precess ? 1 : 0, out);
}

static int relax_impl(mm_ctx* c, float* m_dev, const mm_solver_opts* o, double min_max_err, int64_t max_steps,
                      double* energy_out, double* max_torque_out, int64_t* steps_out) {
    Opts op = get_opts(o);
    op.precess = 0;
    if (!(min_max_err > 0.0)) min_max_err = 1e-9;
    const Tableau& tb = BS23;
    double max_err = op.max_err;
    MM_TRY(launch_set_state(c->st, 0.0, 1e-14, INFINITY, max_err, op.headroom, op.dt_min, op.dt_max, tb.order_low,
                            1, 1, 0, c->stream));
    c->fsal_valid = false;
    MM_CHECK(eval_first(c, m_dev, 0));
    c->fsal_valid = true;
    c->fsal_m = m_dev;
    c->fsal_precess = 0;
    c->fsal_solver = 23;
    MM_CHECK(sync_state(c));
    long long steps = 0, attempts = 0;
    double t = 0.0, dt = 1e-14;
    bool hit_cap = false;
    // advance by `block` accepted steps (device-controlled), at most max_steps attempts overall
    auto advance = [&](int block) -> int {
        MM_TRY(launch_set_state(c->st, t, dt, INFINITY, max_err, op.headroom, op.dt_min, op.dt_max, tb.order_low,
                                0, 0, steps + block, c->stream));
        while (!hit_cap) {
            long long nb = 4;
            if (attempts + nb > max_steps) nb = max_steps - attempts;
            if (nb <= 0) {
                hit_cap = true;
                break;
            }
            for (long long i = 0; i < nb; ++i) MM_CHECK(attempt(c, m_dev, tb, 0, true));
            MM_CHECK(sync_state(c));
            attempts = c->hst->steps + c->hst->rejects;
            steps = c->hst->steps;
            t = c->hst->t;
            dt = c->hst->dt;
            if (c->hst->status != 0) return c->hst->status;
            if (c->hst->done) break;
        }
        return MM_OK;
    };
    double e5[5];
    MM_CHECK(energy_pass(c, m_dev, e5));
    double e0 = e5[4];
    while (!hit_cap) {
        MM_CHECK(advance(3));
        MM_CHECK(energy_pass(c, m_dev, e5));
        if (e5[4] >= e0) break;
        e0 = e5[4];
    }
    double t0 = 0.0;
    MM_CHECK(maxtorque_pass(c, m_dev, 0, &t0));
    while (max_err >= min_max_err && !hit_cap) {
        while (!hit_cap) {
            MM_CHECK(advance(3));
            double t1 = 0.0;
            MM_CHECK(maxtorque_pass(c, m_dev, 0, &t1));
            if (t1 >= t0) break;
            t0 = t1;
        }
        max_err *= 0.5;
    }
    MM_CHECK(energy_pass(c, m_dev, e5));
    double tq = 0.0;
    MM_CHECK(maxtorque_pass(c, m_dev, 0, &tq));
    if (energy_out) *energy_out = e5[4];
    if (max_torque_out) *max_torque_out = tq;
    if (steps_out) *steps_out = steps;
    return hit_cap ? MM_ENOTCONVERGED : MM_OK;
}

// relax minimises the energy of the static problem: no excitations, 0 K
int mm_relax(mm_ctx* c, float* m_dev, const mm_solver_opts* o, double min_max_err, int64_t max_steps,
             double* energy_out, double* max_torque_out, int64_t* steps_out) {
    if (!c || !m_dev || max_steps < 0) return MM_EINVAL;
    c->relaxing = true;
    const int r = relax_impl(c, m_dev, o, min_max_err, max_steps, energy_out, max_torque_out, steps_out);
    c->relaxing = false;
    return r;
}

int mm_solver_reset(mm_ctx* c) {
    if (!c) return MM_EINVAL;
    c->fsal_valid = false;
    return MM_OK;
}

int mm_get_info(mm_ctx* c, mm_info* info) {
    if (!c || !info) return MM_EINVAL;
    memset(info, 0, sizeof(*info));
    info->px = c->px;
    info->py = c->py;
    info->pz = c->pz;
    info->kx = c->kx;
    info->ncomp = c->ncomp;
    info->ncell = c->ncell;
    info->khat_elems = c->khat_elems;
    info->device_bytes = c->dev_bytes;
    return MM_OK;
}

// Saved solver state: header, the device-side solver record, and (when the
// FSAL derivative is valid) the first-stage derivative of the next step.
namespace {
struct StateHeader {
    uint32_t magic, version;
    int32_t nx, ny, nz, devstate_bytes;
    int32_t fsal_valid, fsal_precess, fsal_solver, reserved;
    uint64_t seed;
};
constexpr uint32_t STATE_MAGIC = 0x4d4d5354u;  // "MMST"
long long state_bytes(const mm_ctx* c, bool with_k) {
    return (long long)sizeof(StateHeader) + (long long)sizeof(DevState) +
           (with_k ? 3LL * c->ncell * (long long)sizeof(float) : 0LL);
}
}  // namespace

int mm_state_size(mm_ctx* c, int64_t* bytes) {
    if (!c || !bytes) return MM_EINVAL;
    *bytes = state_bytes(c, true);
    return MM_OK;
}

int mm_state_save(mm_ctx* c, void* host_buf, int64_t bytes) {
    if (!c || !host_buf || bytes < state_bytes(c, c->fsal_valid)) return MM_EINVAL;
    MM_CHECK(sync_state(c));
    StateHeader h;
    memset(&h, 0, sizeof(h));
    h.magic = STATE_MAGIC;
    h.version = 1;
    h.nx = c->nx;
    h.ny = c->ny;
    h.nz = c->nz;
    h.devstate_bytes = (int32_t)sizeof(DevState);
    h.fsal_valid = c->fsal_valid ? 1 : 0;
    h.fsal_precess = c->fsal_precess;
    h.fsal_solver = c->fsal_solver;
    h.seed = c->seed;
    char* out = static_cast<char*>(host_buf);
    memcpy(out, &h, sizeof(h));
    memcpy(out + sizeof(h), c->hst, sizeof(DevState));
    if (c->fsal_valid) {
        // logical derivative 0 (the next step's first stage) lives in the
        // physical buffer the device-side map names
        const int phys = c->hst->perm[0] & 7;
        MM_TRY(hipMemcpyAsync(out + sizeof(h) + sizeof(DevState), c->kbuf + (long long)phys * 3 * c->ncell,
                              (size_t)3 * c->ncell * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        MM_TRY(hipStreamSynchronize(c->stream));
    }
    return MM_OK;
}

int mm_state_load(mm_ctx* c, const void* host_buf, int64_t bytes, const float* m_dev) {
    if (!c || !host_buf || !m_dev || bytes < (int64_t)sizeof(StateHeader)) return MM_EINVAL;
    StateHeader h;
    memcpy(&h, host_buf, sizeof(h));
    if (h.magic != STATE_MAGIC || h.version != 1 || h.devstate_bytes != (int32_t)sizeof(DevState)) return MM_EINVAL;
    if (h.nx != c->nx || h.ny != c->ny || h.nz != c->nz) return MM_EINVAL;
    if (bytes < state_bytes(c, h.fsal_valid != 0)) return MM_EINVAL;
    const char* in = static_cast<const char*>(host_buf);
    DevState ds;
    memcpy(&ds, in + sizeof(h), sizeof(DevState));
    for (int i = 0; i < 8; ++i)
        if (ds.perm[i] < 0 || ds.perm[i] > 7) return MM_EINVAL;
    MM_TRY(hipMemcpyAsync(c->st, &ds, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
    if (h.fsal_valid) {
        const int phys = ds.perm[0];
        MM_TRY(hipMemcpyAsync(c->kbuf + (long long)phys * 3 * c->ncell, in + sizeof(h) + sizeof(DevState),
                              (size_t)3 * c->ncell * sizeof(float), hipMemcpyHostToDevice, c->stream));
    }
    MM_TRY(hipStreamSynchronize(c->stream));
    c->seed = h.seed;
    c->fsal_valid = h.fsal_valid != 0;
    c->fsal_m = m_dev;
    c->fsal_precess = h.fsal_precess;
    c->fsal_solver = h.fsal_solver;
    return MM_OK;
}

int mm_demag_tensor_dump(mm_ctx* c, double* out_dev) {
    if (!c || !out_dev) return MM_EINVAL;
    if (c->pbc[0] == 0 && c->pbc[1] == 0 && c->pbc[2] == 0)
        return map_err(demag_tensor_octant(c->nx, c->ny, c->nz, c->dx, c->dy, c->dz, out_dev, c->stream));
    double* win = nullptr;
    hipError_t e = hipMalloc((void**)&win, (size_t)6 * c->win[0] * c->win[1] * c->win[2] * sizeof(double));
    if (e == hipSuccess) e = demag_tensor_octant(c->win[0], c->win[1], c->win[2], c->dx, c->dy, c->dz, win, c->stream);
    if (e == hipSuccess) e = demag_fold_images(c->nx, c->ny, c->nz, c->win, c->pbc, win, out_dev, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (win) (void)hipFree(win);
    return map_err(e);
}

int mm_demag_kernel_dump(mm_ctx* c, float* out_dev) {
    if (!c || !out_dev) return MM_EINVAL;
    if (!c->khat_ready) return MM_ESTATE;
    MM_TRY(hipMemcpyAsync(out_dev, c->khat, (size_t)c->khat_elems * sizeof(float), hipMemcpyDeviceToDevice,
                          c->stream));
    return MM_OK;
}

int mm_exchange_dump(mm_ctx* c, float* out_dev) {
    if (!c || !out_dev) return MM_EINVAL;
    FieldArgs a = base_args(c, nullptr);
    return map_err(launch_exchange_dump(a, out_dev, c->stream));
}

int mm_set_conv_precision(mm_ctx* c, int32_t prec) {
    if (!c) return MM_EINVAL;
    if (prec != MM_PREC_FP32 && prec != MM_PREC_BF16 && prec != MM_PREC_FP16) return MM_EINVAL;
    if (prec != MM_PREC_FP32) {
        // 2D: the y convolution at padded y length 2048; 3D (the three-pass
        // column path): padded y and z lengths the matrix-core passes serve
        const bool film = c->pz == 1 && c->py == 2048 && c->px >= 2 && !c->full_y;
        const bool vol = c->pz > 1 && !c->yz && (c->py == 1 || colm3d_supported(c->py)) && colm3d_supported(c->pz);
        if (!film && !vol) return MM_EUNSUPPORTED;
    }
    MM_TRY(hipStreamSynchronize(c->stream));
    c->conv_prec = prec;
    c->fsal_valid = false;
    return MM_OK;
}

int mm_set_surrogate(mm_ctx* c, const mm_sno* s, double tol) {
    if (!c) return MM_EINVAL;
    if (!s) {
        c->sno = nullptr;
        return MM_OK;
    }
    if (!(tol > 0.0)) return MM_EINVAL;
    int nx = 0, ny = 0;
    sno_grid(s, &nx, &ny);
    if (c->nz != 1 || nx != c->nx || ny != c->ny) return MM_EUNSUPPORTED;
    if (c->pbc[0] > 0 || c->pbc[1] > 0 || c->pbc[2] > 0) return MM_EUNSUPPORTED;
    if (!c->bsur) {
        MM_TRY(dalloc(c, (void**)&c->bsur, (size_t)3 * c->ncell * sizeof(float)));
        MM_TRY(dalloc(c, (void**)&c->bexact, (size_t)3 * c->ncell * sizeof(float)));
    }
    MM_TRY(hipStreamSynchronize(c->stream));
    c->sno = s;
    c->sur_tol = tol;
    c->sur_steps = 0;
    c->fsal_valid = false;
    return MM_OK;
}

int mm_surrogate_stats(mm_ctx* c, int64_t* sur_steps, int64_t* fallbacks, double* last_err) {
    if (!c) return MM_EINVAL;
    MM_CHECK(sync_state(c));
    if (sur_steps) *sur_steps = c->sur_steps;
    if (fallbacks) *fallbacks = c->hst->sur_fallbacks;
    if (last_err) *last_err = c->hst->sur_err;
    return MM_OK;
}

int mm_timing_enable(mm_ctx* c, int32_t which, int32_t enable) {
    if (!c || which < 0 || which >= NTIMING) return MM_EINVAL;
    TimingClass& t = c->timing[which];
    MM_TRY(hipStreamSynchronize(c->stream));
    t.used = 0;
    t.enabled = enable != 0;
    if (!t.enabled) {
        for (auto& pr : t.ev) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        t.ev.clear();
        return MM_OK;
    }
    while (t.ev.size() < TIMING_POOL) {
        hipEvent_t a = nullptr, b = nullptr;
        MM_TRY(hipEventCreate(&a));
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return MM_EDEVICE;
        }
        t.ev.emplace_back(a, b);
    }
    return MM_OK;
}

int mm_timing_read(mm_ctx* c, int32_t which, int64_t* launches, double* total_ms) {
    if (!c || which < 0 || which >= NTIMING || !launches || !total_ms) return MM_EINVAL;
    MM_TRY(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    const TimingClass& t = c->timing[which];
    for (size_t i = 0; i < t.used; ++i) {
        float ms = 0.f;
        MM_TRY(hipEventElapsedTime(&ms, t.ev[i].first, t.ev[i].second));
        tot += ms;
    }
    *launches = (int64_t)t.used;
    *total_ms = tot;
    return MM_OK;
}

void mm_destroy(mm_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

}  // extern "C"
