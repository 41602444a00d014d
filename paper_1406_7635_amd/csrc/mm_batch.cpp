// mm_batch.cpp -- the ensemble entry points of include/mm.h: member layout,
// work lists, the batched Runge-Kutta attempt (launched directly or replayed
// as a captured HIP graph) and the tuning of the persistent grid sizes.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/mm.h"
#include "api_common.h"
#include "mm_internal.h"
#include "tableau.h"

using namespace mm;

struct mm_batch {
    int device = 0;
    int ncu = 0;
    hipStream_t user = nullptr;    // the caller's stream
    hipStream_t stream = nullptr;  // the ensemble's own (capturable) stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int n = 0;
    std::vector<BMember> hmem;
    std::vector<mm_grid> hgrid;
    long long ncell = 0, spec_elems = 0, khat_elems = 0, zker_elems = 0;
    bool has2d = false;
    int pt = 1, twshift = 0;
    // device buffers
    BMember* mem = nullptr;
    // work lists per pass and tile shape (TILE_WIDE, TILE_NARROW); a narrow
    // list exists only for the x passes and the 2D column pass, and only when
    // the narrow shape serves every member
    unsigned int* items[BP_N][2] = {};
    int nitems[BP_N][2] = {};
    bool tile_ok[BP_N][2] = {};
    int tile[BP_N] = {};  // the shape in use
    int grid[BP_N] = {};
    uint8_t* region = nullptr;
    double* params64 = nullptr;
    RegionLut* lut = nullptr;
    float* ptab = nullptr;
    cf* tw = nullptr;
    cf* spec = nullptr;
    float* khat = nullptr;
    float* zker = nullptr;  // thin 3D members: kernels transformed back along z
    float* kbuf = nullptr;
    float* ms = nullptr;
    float* ms2 = nullptr;
    DevState* st = nullptr;
    int* active = nullptr;
    // pinned host mirrors
    DevState* hst = nullptr;
    int* hactive = nullptr;
    bool khat_ready = false;
    // solver
    const Tableau* tb = &DP45;
    int solver = 45;
    int precess = 1;
    bool started = false;
    bool fsal_valid = false;
    const float* fsal_m = nullptr;
    // graph of one attempt
    bool use_graph = true;
    hipGraphExec_t graph = nullptr;
    const float* graph_m = nullptr;
    int graph_solver = 0, graph_precess = -1;
};

namespace {

void free_batch(mm_batch* b) {
    void* ptrs[] = {b->mem, b->region, b->params64, b->lut, b->ptab, b->tw,     b->spec,
                    b->khat, b->zker, b->kbuf,  b->ms,       b->ms2, b->st, b->active};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& pl : b->items)
        for (unsigned int* p : pl)
            if (p) (void)hipFree(p);
    if (b->hst) (void)hipHostFree(b->hst);
    if (b->hactive) (void)hipHostFree(b->hactive);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

// Order the ensemble's stream after the caller's work, and the caller's
// stream after the ensemble's.
int enter(mm_batch* b) {
    MM_TRY(hipEventRecord(b->ev_in, b->user));
    MM_TRY(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    return MM_OK;
}
int leave(mm_batch* b) {
    MM_TRY(hipEventRecord(b->ev_out, b->stream));
    MM_TRY(hipStreamWaitEvent(b->user, b->ev_out, 0));
    return MM_OK;
}

// work items of pass p in its current tile shape (0: no member uses the pass)
int nitems_of(const mm_batch* b, int pass) { return b->nitems[pass][b->tile[pass]]; }

BatchList list(const mm_batch* b, int pass) {
    BatchList l;
    l.mem = b->mem;
    l.items = b->items[pass][b->tile[pass]];
    l.nitems = nitems_of(b, pass);
    return l;
}

// one workgroup per tile, rounded up to the XCD count
int full_grid(int nitems) { return ((nitems + 7) / 8) * 8; }

int grid_of(const mm_batch* b, int pass) {
    return b->grid[pass] > 0 ? b->grid[pass] : full_grid(nitems_of(b, pass));
}

// Base field arguments: the ensemble's buffers; the kernels add each member's offsets.
FieldArgs base_field(const mm_batch* b, const float* m) {
    FieldArgs a;
    memset(&a, 0, sizeof(a));
    a.m0 = m;
    a.ms = b->ms;
    a.region = b->region;
    a.lut = b->lut;
    a.ptab = b->ptab;
    a.kbuf = b->kbuf;
    a.st = b->st;
    a.sd.out_k = -1;
    a.spec = b->spec;
    a.tw = b->tw;
    a.twshift = b->twshift;
    return a;
}

ColArgs base_col(const mm_batch* b, bool check_done) {
    ColArgs c;
    memset(&c, 0, sizeof(c));
    c.spec = b->spec;
    c.khat = b->khat;
    c.zker = b->zker;
    c.tw = b->tw;
    c.twshift = b->twshift;
    c.st = b->st;
    c.check_done = check_done ? 1 : 0;
    return c;
}

// The column passes between the x passes of a field evaluation.
int run_cols(mm_batch* b, bool check_done) {
    const ColArgs c = base_col(b, check_done);
    hipStream_t s = b->stream;
    if (b->has2d) MM_TRY(launch_bcol3(list(b, BP_C3), grid_of(b, BP_C3), c, s, b->tile[BP_C3]));
    for (int p : {BP_YZ4, BP_YZ8})
        if (nitems_of(b, p) > 0) MM_TRY(launch_byz(p, list(b, p), grid_of(b, p), c, s));
    if (nitems_of(b, BP_Y) > 0) {
        MM_TRY(launch_bcoly(0, list(b, BP_Y), grid_of(b, BP_Y), c, s));
        for (int p : {BP_Z4, BP_Z8, BP_Z16})
            if (nitems_of(b, p) > 0) MM_TRY(launch_bzconv(p, list(b, p), grid_of(b, p), c, s));
        MM_TRY(launch_bcoly(1, list(b, BP_Y), grid_of(b, BP_Y), c, s));
    }
    return MM_OK;
}

// One field evaluation of every member (non-fused passes).
int run_field(mm_batch* b, FieldArgs& a) {
    if (!b->khat_ready) return MM_ESTATE;
    a.flags |= EPI_HAS_DEMAG;
    const bool cd = (a.flags & EPI_CHECK_DONE) != 0;
    const int tx = b->tile[BP_X];
    MM_TRY(launch_bx(BX_FWD, list(b, BP_X), grid_of(b, BP_X), a, a, 0.f, b->stream, tx));
    MM_CHECK(run_cols(b, cd));
    MM_TRY(launch_bx(BX_INV, list(b, BP_X), grid_of(b, BP_X), a, a, 0.f, b->stream, tx));
    return MM_OK;
}

FieldArgs stage_field(const mm_batch* b, const float* m, int s) {
    FieldArgs a = base_field(b, m);
    const bool last = fill_stage(*b->tb, s, a.sd);
    a.flags = EPI_TORQUE | EPI_HAS_DEMAG | EPI_CHECK_DONE | (b->precess ? EPI_PRECESS : 0);
    if (last) a.flags |= EPI_ERR;
    return a;
}

// One attempt of the embedded pair for every running member: the x-inverse
// of each inner stage fused with the x-forward of the next (stage states
// alternate between two buffers), then the controllers and finalisation.
int enqueue_attempt(mm_batch* b, float* m) {
    const Tableau& tb = *b->tb;
    const int S = tb.stages;
    hipStream_t s = b->stream;
    const BatchList lx = list(b, BP_X);
    const int gx = grid_of(b, BP_X), tx = b->tile[BP_X];
    float* buf[2] = {b->ms, b->ms2};
    int cur = 0;
    FieldArgs a = stage_field(b, m, 1);
    a.ms = buf[cur];
    MM_TRY(launch_bx(BX_FWD, lx, gx, a, a, 0.f, s, tx));
    MM_CHECK(run_cols(b, true));
    for (int st = 1; st < S - 1; ++st) {
        FieldArgs ai = stage_field(b, m, st);
        ai.ms = buf[cur];
        FieldArgs af = stage_field(b, m, st + 1);
        af.ms = buf[cur ^ 1];
        // the k_s term (always the last one listed) comes from the fused pass
        float a_last = 0.f;
        if (af.sd.nk > 0 && af.sd.kidx[af.sd.nk - 1] == st) {
            a_last = af.sd.a[af.sd.nk - 1];
            --af.sd.nk;
        }
        MM_TRY(launch_bx(BX_ROW, lx, gx, ai, af, a_last, s, tx));
        cur ^= 1;
        MM_CHECK(run_cols(b, true));
    }
    FieldArgs al = stage_field(b, m, S - 1);
    al.ms = buf[cur];
    MM_TRY(launch_bx(BX_INV, lx, gx, al, al, 0.f, s, tx));
    MM_TRY(launch_bcontroller(b->st, b->n, S - 1, S - 1, 1, b->active, s));
    MM_TRY(launch_bfinalize(list(b, BP_F), grid_of(b, BP_F), buf[cur], m, b->st, s));
    return MM_OK;
}

void drop_graph(mm_batch* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_m = nullptr;
}

// Capture one attempt as a graph (kernel arguments fixed: the state buffer,
// the solver and the grid sizes; everything that changes per attempt lives
// in the members' device-side solver states).
int build_graph(mm_batch* b, float* m) {
    drop_graph(b);
    MM_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int st = enqueue_attempt(b, m);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st != MM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    MM_TRY(e);
    const hipError_t ei = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    MM_TRY(ei);
    b->graph_m = m;
    b->graph_solver = b->solver;
    b->graph_precess = b->precess;
    return MM_OK;
}

int attempt(mm_batch* b, float* m) {
    if (!b->use_graph) return enqueue_attempt(b, m);
    if (!b->graph || b->graph_m != m || b->graph_solver != b->solver || b->graph_precess != b->precess)
        MM_CHECK(build_graph(b, m));
    MM_TRY(hipGraphLaunch(b->graph, b->stream));
    return MM_OK;
}

// First stage derivative of every member at the committed state (logical k_0).
int eval_first(mm_batch* b, const float* m) {
    FieldArgs a = base_field(b, m);
    a.sd.nk = 0;
    a.sd.out_k = 0;
    a.flags = EPI_TORQUE | (b->precess ? EPI_PRECESS : 0);
    return run_field(b, a);
}

int sync_states(mm_batch* b) {
    MM_TRY(hipMemcpyAsync(b->hst, b->st, (size_t)b->n * sizeof(DevState), hipMemcpyDeviceToHost, b->stream));
    MM_TRY(hipStreamSynchronize(b->stream));
    return MM_OK;
}

}  // namespace

extern "C" {

int mm_batch_create(mm_batch** out, int32_t n, const mm_grid* grids, const mm_params* params,
                    const uint8_t* region_dev, void* hip_stream) {
    if (!out || !grids || !params || !region_dev || n < 1) return MM_EINVAL;
    *out = nullptr;
    if (n > 65535) return MM_EUNSUPPORTED;
    for (int i = 0; i < n; ++i) {
        const mm_grid& g = grids[i];
        if (g.nx < 1 || g.ny < 1 || g.nz < 1) return MM_EINVAL;
        if (!finite_pos(g.dx) || !finite_pos(g.dy) || !finite_pos(g.dz)) return MM_EINVAL;
        if (g.pbc[0] || g.pbc[1] || g.pbc[2]) return MM_EUNSUPPORTED;
        if (g.nx > 512 || g.ny > 512 || g.nz > 8) return MM_EUNSUPPORTED;
        if (!batch_supported(pad_len(g.nx), pad_len(g.ny), pad_len(g.nz))) return MM_EUNSUPPORTED;
        MM_CHECK(validate_params(params + i));
    }
    mm_batch* b = new (std::nothrow) mm_batch();
    if (!b) return MM_ENOMEM;
    b->user = (hipStream_t)hip_stream;
    b->n = n;
    (void)hipGetDevice(&b->device);
    int st = MM_OK;
    try {
        b->hmem.resize(n);
        b->hgrid.assign(grids, grids + n);
    } catch (...) {
        delete b;
        return MM_ENOMEM;
    }
    for (int i = 0; i < n; ++i) {
        const mm_grid& g = grids[i];
        BMember& m = b->hmem[i];
        m.nx = g.nx;
        m.ny = g.ny;
        m.nz = g.nz;
        m.nrows = g.ny * g.nz;
        m.px = pad_len(g.nx);
        m.py = pad_len(g.ny);
        m.pz = pad_len(g.nz);
        m.kx = m.px / 2 + 1;
        m.cell_off = b->ncell;
        m.spec_off = b->spec_elems;
        m.khat_off = b->khat_elems;
        m.zker_off = b->zker_elems;
        // rows per spectrum column: py when the y transforms run in place, else ny;
        // kx-major (the planes of one kx adjacent)
        m.zstride = 3LL * (m.pz > 1 && !yz_supported(m.py, m.pz) ? m.py : m.ny);
        m.colstride = m.zstride * m.nz;
        m.idx2 = (float)(1.0 / (g.dx * g.dx));
        m.idy2 = (float)(1.0 / (g.dy * g.dy));
        m.idz2 = (float)(1.0 / (g.dz * g.dz));
        m.cellvol = (float)(g.dx * g.dy * g.dz);
        const long long nc = (long long)g.nx * g.ny * g.nz;
        b->ncell += nc;
        b->spec_elems += m.colstride * m.kx;
        b->khat_elems += (long long)m.kx * (m.py / 2 + 1) * (m.pz / 2 + 1) * (m.pz > 1 ? 6 : 4);
        if (m.pz > 1 && yz_supported(m.py, m.pz)) b->zker_elems += (long long)m.kx * (m.py / 2 + 1) * zkernel_floats(m.pz);
        if (m.pz == 1) b->has2d = true;
        if (m.px > b->pt) b->pt = m.px;
        if (m.py > b->pt) b->pt = m.py;
        if (m.pz > b->pt) b->pt = m.pz;
    }
    // every member's [3][ncell] arrays (and the ensemble's) stay addressable with 32-bit offsets
    if (b->ncell > (1LL << 28)) {
        delete b;
        return MM_EUNSUPPORTED;
    }
    b->twshift = ilog2(b->pt);
    std::vector<std::vector<unsigned int>> items[2] = {std::vector<std::vector<unsigned int>>(BP_N),
                                                       std::vector<std::vector<unsigned int>>(BP_N)};
    for (int p = 0; p < BP_N; ++p) {
        for (int tl : {TILE_WIDE, TILE_NARROW}) {
            bool ok = tl == TILE_WIDE || p == BP_X || p == BP_C3;
            for (int i = 0; i < n && ok; ++i) ok = batch_tile_serves(p, tl, b->hmem[i]);
            b->tile_ok[p][tl] = ok;
            if (!ok) continue;
            for (int i = 0; i < n; ++i) {
                const int t = batch_tiles(p, b->hmem[i], tl);
                if (t > 65536) st = MM_EUNSUPPORTED;
                for (int k = 0; k < t && k < 65536; ++k)
                    items[tl][p].push_back(((unsigned int)i << 16) | (unsigned int)k);
            }
            b->nitems[p][tl] = (int)items[tl][p].size();
        }
    }
    if (st != MM_OK) {
        delete b;
        return st;
    }
    auto A = [&](void** ptr, size_t bytes) {
        if (st != MM_OK || bytes == 0) return;
        const hipError_t e = hipMalloc(ptr, bytes);
        if (e != hipSuccess) st = map_err(e);
    };
    const size_t nc = (size_t)b->ncell;
    A((void**)&b->mem, (size_t)n * sizeof(BMember));
    for (int tl : {TILE_WIDE, TILE_NARROW})
        for (int p = 0; p < BP_N; ++p) A((void**)&b->items[p][tl], items[tl][p].size() * sizeof(unsigned int));
    A((void**)&b->region, nc);
    A((void**)&b->params64, (size_t)n * sizeof(mm_params));
    A((void**)&b->lut, (size_t)n * NREG * sizeof(RegionLut));
    A((void**)&b->ptab, (size_t)n * NREG * NREG * sizeof(float));
    A((void**)&b->tw, (size_t)b->pt * sizeof(cf));
    A((void**)&b->spec, (size_t)b->spec_elems * sizeof(cf));
    A((void**)&b->khat, (size_t)b->khat_elems * sizeof(float));
    A((void**)&b->zker, (size_t)b->zker_elems * sizeof(float));
    A((void**)&b->kbuf, (size_t)MAXK * 3 * nc * sizeof(float));
    A((void**)&b->ms, 3 * nc * sizeof(float));
    A((void**)&b->ms2, 3 * nc * sizeof(float));
    A((void**)&b->st, (size_t)n * sizeof(DevState));
    A((void**)&b->active, sizeof(int));
    if (st == MM_OK && hipHostMalloc((void**)&b->hst, (size_t)n * sizeof(DevState), hipHostMallocDefault) != hipSuccess)
        st = MM_ENOMEM;
    if (st == MM_OK && hipHostMalloc((void**)&b->hactive, sizeof(int), hipHostMallocDefault) != hipSuccess)
        st = MM_ENOMEM;
    if (st == MM_OK) {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device);
        if (e == hipSuccess) e = hipEventRecord(b->ev_in, b->user);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
        // host arrays are copied synchronously (they are the caller's, pageable)
        if (e == hipSuccess) e = hipMemcpy(b->mem, b->hmem.data(), (size_t)n * sizeof(BMember), hipMemcpyHostToDevice);
        for (int tl : {TILE_WIDE, TILE_NARROW})
            for (int p = 0; p < BP_N && e == hipSuccess; ++p)
                if (!items[tl][p].empty())
                    e = hipMemcpy(b->items[p][tl], items[tl][p].data(), items[tl][p].size() * sizeof(unsigned int),
                                  hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->params64, params, (size_t)n * sizeof(mm_params), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpyAsync(b->region, region_dev, nc, hipMemcpyDeviceToDevice, b->stream);
        for (int i = 0; i < n && e == hipSuccess; ++i)
            e = launch_prepare_tables(b->params64 + (size_t)i * (sizeof(mm_params) / sizeof(double)),
                                      b->lut + (size_t)i * NREG, b->ptab + (size_t)i * NREG * NREG, b->stream);
        if (e == hipSuccess) e = launch_twiddles(b->tw, b->pt, b->stream);
        if (e == hipSuccess) e = configure_batch_kernels();
        if (e == hipSuccess)
            e = launch_bset_state(b->st, n, 0.0, 1e-14, INFINITY, 1e-5, 0.8, 0.0, 0.0, 4, 1, 1, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        st = map_err(e);
    }
    if (st != MM_OK) {
        free_batch(b);
        delete b;
        return st;
    }
    *out = b;
    return MM_OK;
}

int mm_batch_demag_kernel_init(mm_batch* b) {
    if (!b) return MM_EINVAL;
    MM_CHECK(enter(b));
    long long maxc = 0, maxp = 0;
    for (const BMember& m : b->hmem) {
        const long long c = (long long)m.nx * m.ny * m.nz, p = (long long)m.px * m.py * m.pz;
        if (c > maxc) maxc = c;
        if (p > maxp) maxp = p;
    }
    double* oct = nullptr;
    double2* work = nullptr;
    hipError_t e = hipMalloc((void**)&oct, (size_t)6 * maxc * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&work, (size_t)maxp * sizeof(double2));
    for (int i = 0; i < b->n && e == hipSuccess; ++i) {
        const BMember& m = b->hmem[i];
        const mm_grid& g = b->hgrid[i];
        e = demag_tensor_octant(m.nx, m.ny, m.nz, g.dx, g.dy, g.dz, oct, b->stream);
        if (e == hipSuccess)
            e = demag_kernel_spectrum(m.nx, m.ny, m.nz, m.px, m.py, m.pz, oct, work, b->khat + m.khat_off,
                                      m.pz > 1 ? 6 : 4, m.kx, b->stream);
        if (e == hipSuccess && m.pz > 1 && yz_supported(m.py, m.pz))
            e = launch_zkernel(b->khat + m.khat_off, b->zker + m.zker_off, (long long)m.kx * (m.py / 2 + 1), m.pz,
                               b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (oct) (void)hipFree(oct);
    if (work) (void)hipFree(work);
    MM_TRY(e);
    b->khat_ready = true;
    b->fsal_valid = false;
    return leave(b);
}

int mm_batch_member(mm_batch* b, int32_t i, int64_t* cell_offset, int64_t* ncell) {
    if (!b || i < 0 || i >= b->n || !cell_offset || !ncell) return MM_EINVAL;
    const BMember& m = b->hmem[i];
    *cell_offset = m.cell_off;
    *ncell = (int64_t)m.nx * m.ny * m.nz;
    return MM_OK;
}

int mm_batch_beff(mm_batch* b, const float* m_dev, float* beff_dev) {
    if (!b || !m_dev || !beff_dev) return MM_EINVAL;
    MM_CHECK(enter(b));
    FieldArgs a = base_field(b, m_dev);
    a.beff = beff_dev;
    a.flags = EPI_BEFF;
    MM_CHECK(run_field(b, a));
    return leave(b);
}

int mm_batch_start(mm_batch* b, int32_t solver, double t0, double dt0, double t_end, const mm_solver_opts* o) {
    if (!b) return MM_EINVAL;
    if (solver != 45 && solver != 23) return MM_EINVAL;
    if (!(isfinite(t0) && finite_pos(dt0)) || isnan(t_end)) return MM_EINVAL;
    double max_err = 1e-5, headroom = 0.8, dt_min = 0.0, dt_max = 0.0;
    int precess = 1;
    if (o) {
        if (o->max_err > 0.0) max_err = o->max_err;
        if (o->headroom > 0.0) headroom = o->headroom;
        if (o->dt_min > 0.0) dt_min = o->dt_min;
        if (o->dt_max > 0.0) dt_max = o->dt_max;
        precess = o->precess ? 1 : 0;
    }
    b->solver = solver;
    b->tb = solver == 45 ? &DP45 : &BS23;
    b->precess = precess;
    double dt = dt0;
    if (isfinite(t_end) && t0 + dt > t_end && t_end > t0) dt = t_end - t0;
    MM_CHECK(enter(b));
    MM_TRY(launch_bset_state(b->st, b->n, t0, dt, t_end, max_err, headroom, dt_min, dt_max, b->tb->order_low, 1, 1,
                             b->stream));
    b->started = true;
    b->fsal_valid = false;
    return leave(b);
}

int mm_batch_run(mm_batch* b, float* m_dev, int64_t max_attempts, int64_t* attempts_out, int32_t* active_out) {
    if (!b || !m_dev || max_attempts < 0) return MM_EINVAL;
    if (!b->started) return MM_ESTATE;
    if (!b->khat_ready) return MM_ESTATE;
    MM_CHECK(enter(b));
    if (!b->fsal_valid || b->fsal_m != m_dev) {
        MM_CHECK(eval_first(b, m_dev));
        b->fsal_valid = true;
        b->fsal_m = m_dev;
    }
    // attempts between two checks of the running count: about 3e7 cells each
    long long per = (long long)(3e7 / (double)b->ncell);
    if (per < 2) per = 2;
    if (per > 32) per = 32;
    long long done = 0;
    int act = b->n;
    while (done < max_attempts) {
        long long nb = max_attempts - done;
        if (nb > per) nb = per;
        for (long long i = 0; i < nb; ++i) MM_CHECK(attempt(b, m_dev));
        done += nb;
        MM_TRY(hipMemcpyAsync(b->hactive, b->active, sizeof(int), hipMemcpyDeviceToHost, b->stream));
        MM_TRY(hipStreamSynchronize(b->stream));
        act = *b->hactive;
        if (act == 0) break;
    }
    if (attempts_out) *attempts_out = done;
    if (active_out) *active_out = act;
    return leave(b);
}

int mm_batch_stats(mm_batch* b, int32_t i, mm_run_stats* out, int32_t* status) {
    if (!b || i < 0 || i >= b->n || !out) return MM_EINVAL;
    MM_CHECK(enter(b));
    MM_CHECK(sync_states(b));
    const DevState& s = b->hst[i];
    out->steps = s.steps;
    out->rejects = s.rejects;
    // the first derivative of a run is one more evaluation per member
    out->evals = s.evals + (s.steps + s.rejects > 0 ? 1 : 0);
    out->t = s.t;
    out->dt = s.dt;
    out->err = s.err;
    if (status) *status = s.status;
    return leave(b);
}

int mm_batch_stats_all(mm_batch* b, mm_run_stats* out, int32_t* status) {
    if (!b || !out) return MM_EINVAL;
    MM_CHECK(enter(b));
    MM_CHECK(sync_states(b));
    for (int i = 0; i < b->n; ++i) {
        const DevState& s = b->hst[i];
        out[i].steps = s.steps;
        out[i].rejects = s.rejects;
        out[i].evals = s.evals + (s.steps + s.rejects > 0 ? 1 : 0);
        out[i].t = s.t;
        out[i].dt = s.dt;
        out[i].err = s.err;
        if (status) status[i] = s.status;
    }
    return leave(b);
}

int mm_batch_set_graph(mm_batch* b, int32_t enable) {
    if (!b) return MM_EINVAL;
    b->use_graph = enable != 0;
    if (!b->use_graph) drop_graph(b);
    return MM_OK;
}

int mm_batch_set_grid(mm_batch* b, int32_t pass, int32_t grid) {
    if (!b || pass < 0 || pass >= BP_N || grid < 0) return MM_EINVAL;
    b->grid[pass] = grid > 0 ? ((grid + 7) / 8) * 8 : 0;
    drop_graph(b);
    return MM_OK;
}

int mm_batch_get_grid(mm_batch* b, int32_t pass, int32_t* grid) {
    if (!b || pass < 0 || pass >= BP_N || !grid) return MM_EINVAL;
    *grid = nitems_of(b, pass) > 0 ? grid_of(b, pass) : 0;
    return MM_OK;
}

int mm_batch_set_tile(mm_batch* b, int32_t pass, int32_t tile) {
    if (!b || pass < 0 || pass >= BP_N || (tile != TILE_WIDE && tile != TILE_NARROW)) return MM_EINVAL;
    if (!b->tile_ok[pass][tile]) return MM_EUNSUPPORTED;
    if (b->tile[pass] != tile) {
        b->tile[pass] = tile;
        b->grid[pass] = 0;  // the persistent grid was chosen for the other list
    }
    drop_graph(b);
    return MM_OK;
}

int mm_batch_get_tile(mm_batch* b, int32_t pass, int32_t* tile) {
    if (!b || pass < 0 || pass >= BP_N || !tile) return MM_EINVAL;
    *tile = b->tile[pass];
    return MM_OK;
}

int mm_batch_autotune(mm_batch* b, const float* m_dev) {
    if (!b || !m_dev) return MM_EINVAL;
    if (!b->khat_ready) return MM_ESTATE;
    MM_CHECK(enter(b));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MM_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MM_EDEVICE;
    }
    int status = MM_OK;
    // stage 2 of the tableau as the representative fused x pass; the column
    // passes run on whatever the spectrum holds (timing only)
    float* m = const_cast<float*>(m_dev);
    FieldArgs ai = stage_field(b, m, 1);
    ai.flags &= ~EPI_CHECK_DONE;
    ai.ms = b->ms;
    FieldArgs af = stage_field(b, m, 2);
    af.flags &= ~EPI_CHECK_DONE;
    af.ms = b->ms2;
    const float a_last = af.sd.nk > 0 ? af.sd.a[af.sd.nk - 1] : 0.f;
    if (af.sd.nk > 0) --af.sd.nk;
    const ColArgs c = base_col(b, false);
    auto launch = [&](int p, int tl, int g) -> hipError_t {
        BatchList l = list(b, p);
        l.items = b->items[p][tl];
        l.nitems = b->nitems[p][tl];
        switch (p) {
            case BP_X:
                return launch_bx(BX_ROW, l, g, ai, af, a_last, b->stream, tl);
            case BP_C3:
                return launch_bcol3(l, g, c, b->stream, tl);
            case BP_Y:
                return launch_bcoly(0, l, g, c, b->stream);
            case BP_Z4:
            case BP_Z8:
            case BP_Z16:
                return launch_bzconv(p, l, g, c, b->stream);
            case BP_YZ4:
            case BP_YZ8:
                return launch_byz(p, l, g, c, b->stream);
            default:
                return hipSuccess;
        }
    };
    // candidates per pass: every tile shape that serves all members, each
    // with one workgroup per tile and 1, 2, 4 x its resident workgroups per
    // CU on every CU
    for (int p = 0; p < BP_N && status == MM_OK; ++p) {
        if (p == BP_F || b->nitems[p][TILE_WIDE] == 0) continue;
        float best = INFINITY;
        int best_g = 0, best_t = TILE_WIDE;
        for (int tl : {TILE_WIDE, TILE_NARROW}) {
            if (!b->tile_ok[p][tl] || status != MM_OK) continue;
            int res = 0;
            if (batch_resident(p, tl, &res) != hipSuccess || res < 1) res = 1;
            const int full = full_grid(b->nitems[p][tl]);
            std::vector<int> cand = {full};
            for (int k : {1, 2, 4}) {
                const int g = ((k * res * b->ncu + 7) / 8) * 8;
                if (g < full) cand.push_back(g);
            }
            for (int g : cand) {
                hipError_t e = launch(p, tl, g);  // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
                for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch(p, tl, g);
                if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    status = map_err(e);
                    break;
                }
                if (ms < best) {
                    best = ms;
                    best_g = g == full ? 0 : g;
                    best_t = tl;
                }
            }
        }
        b->tile[p] = best_t;
        b->grid[p] = best_g;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graph(b);
    b->fsal_valid = false;
    if (status != MM_OK) return status;
    return leave(b);
}

void mm_batch_destroy(mm_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
}

}  // extern "C"
