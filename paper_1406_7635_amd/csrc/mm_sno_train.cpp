// mm_sno_train.cpp -- C ABI of the surrogate's trainer: FP32 master weights,
// Adam moments, the activations of one batch, gradient and update steps.
#include <math.h>
#include <string.h>

#include <new>

#include "../../include/mm.h"
#include "api_common.h"
#include "sno_internal.h"

using namespace mm;

struct mm_sno_trainer {
    hipStream_t stream = nullptr;
    int nx = 0, ny = 0, batch = 0;
    long long step = 0;
    float* w = nullptr;     // weights, gradient, Adam moments: 4 x NW floats
    float* g = nullptr;
    float* m1 = nullptr;
    float* m2 = nullptr;
    float2* tw = nullptr;   // nx then ny twiddles
    float* act = nullptr;   // h[5], z[4], dh[2], dz, y
    float2* modes = nullptr;
    float* part = nullptr;
    double* lpart = nullptr;
    float* scale = nullptr;
    double* loss = nullptr;
    SnoTrainArgs args;
    SnoTrainBufs bufs;
};

namespace {

void free_tr(mm_sno_trainer* t) {
    void* p[] = {t->w, t->tw, t->act, t->modes, t->part, t->lpart, t->scale, t->loss};
    for (void* q : p)
        if (q) (void)hipFree(q);
}

int read_loss(mm_sno_trainer* t, double* out) {
    if (!out) return MM_OK;
    MM_TRY(hipMemcpyAsync(out, t->loss, sizeof(double), hipMemcpyDeviceToHost, t->stream));
    MM_TRY(hipStreamSynchronize(t->stream));
    return MM_OK;
}

}  // namespace

extern "C" {

int mm_sno_train_create(mm_sno_trainer** out, int32_t nx, int32_t ny, int32_t batch, const float* weights,
                        int64_t nweights, void* hip_stream) {
    if (!out || !weights) return MM_EINVAL;
    *out = nullptr;
    if (nweights != SNO_NWEIGHTS || batch < 1) return MM_EINVAL;
    if (nx < 2 * SNO_KX || ny < SNO_KY || nx > 512 || ny > 512 || batch > 256) return MM_EUNSUPPORTED;
    for (int64_t i = 0; i < nweights; ++i)
        if (!isfinite(weights[i])) return MM_EINVAL;
    mm_sno_trainer* t = new (std::nothrow) mm_sno_trainer();
    if (!t) return MM_ENOMEM;
    t->stream = (hipStream_t)hip_stream;
    t->nx = nx;
    t->ny = ny;
    t->batch = batch;
    const long long n = (long long)nx * ny;
    const long long fld = (long long)batch * SNO_C * n;  // one activation array
    const long long kept = (long long)batch * SNO_C * SNO_KY * SNO_KX;
    const long long line = (long long)batch * SNO_C * ny * SNO_KX;
    const int tiles = sno_train_tiles((long long)batch * n);
    const long long nw = SNO_NWEIGHTS;
    hipError_t e = hipMalloc((void**)&t->w, (size_t)(4 * nw) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&t->tw, (size_t)(nx + ny) * sizeof(float2));
    // h[0..4], z[0..3], dh[0..1], dz: 12 activation arrays, then y [B][3][n]
    if (e == hipSuccess) e = hipMalloc((void**)&t->act, (size_t)(12 * fld + 3LL * batch * n) * sizeof(float));
    // H[0..3], modes, modes2: 6 kept-mode arrays, then the line array
    if (e == hipSuccess) e = hipMalloc((void**)&t->modes, (size_t)(6 * kept + line) * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc((void**)&t->part, (size_t)tiles * (SNO_C * SNO_C + SNO_C) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&t->lpart, (size_t)batch * 64 * 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&t->scale, (size_t)batch * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&t->loss, sizeof(double));
    if (e == hipSuccess) e = configure_sno_train(ny);
    if (e == hipSuccess) e = sno_twiddles(t->tw, nx, t->stream);
    if (e == hipSuccess) e = sno_twiddles(t->tw + nx, ny, t->stream);
    if (e == hipSuccess) {
        t->g = t->w + nw;
        t->m1 = t->w + 2 * nw;
        t->m2 = t->w + 3 * nw;
        e = hipMemcpyAsync(t->w, weights, (size_t)nw * sizeof(float), hipMemcpyHostToDevice, t->stream);
    }
    if (e == hipSuccess) e = hipMemsetAsync(t->m1, 0, (size_t)(2 * nw) * sizeof(float), t->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
    const int st = map_err(e);
    if (st != MM_OK) {
        free_tr(t);
        delete t;
        return st;
    }
    SnoTrainArgs& a = t->args;
    a.nx = nx;
    a.ny = ny;
    a.n = (int)n;
    a.batch = batch;
    a.w = t->w;
    a.g = t->g;
    a.twx = t->tw;
    a.twy = t->tw + nx;
    SnoTrainBufs& b = t->bufs;
    float* f = t->act;
    for (int l = 0; l <= SNO_LAYERS; ++l) b.h[l] = f + l * fld;
    for (int l = 0; l < SNO_LAYERS; ++l) b.z[l] = f + (5 + l) * fld;
    b.dh[0] = f + 9 * fld;
    b.dh[1] = f + 10 * fld;
    b.dz = f + 11 * fld;
    b.y = f + 12 * fld;
    for (int l = 0; l < SNO_LAYERS; ++l) b.H[l] = t->modes + l * kept;
    b.modes = t->modes + 4 * kept;
    b.modes2 = t->modes + 5 * kept;
    b.line = t->modes + 6 * kept;
    b.part = t->part;
    b.lpart = t->lpart;
    b.scale = t->scale;
    b.loss = t->loss;
    *out = t;
    return MM_OK;
}

int mm_sno_train_grad(mm_sno_trainer* t, const float* m_dev, const float* target_dev, float* grad_dev,
                      double* loss_out) {
    if (!t || !m_dev || !target_dev) return MM_EINVAL;
    MM_TRY(sno_train_grad(t->args, t->bufs, m_dev, target_dev, t->stream));
    if (grad_dev)
        MM_TRY(hipMemcpyAsync(grad_dev, t->g, (size_t)SNO_NWEIGHTS * sizeof(float), hipMemcpyDeviceToDevice,
                              t->stream));
    return read_loss(t, loss_out);
}

int mm_sno_train_step(mm_sno_trainer* t, const float* m_dev, const float* target_dev, double lr, double* loss_out) {
    if (!t || !m_dev || !target_dev || !(lr >= 0.0) || !isfinite(lr)) return MM_EINVAL;
    MM_TRY(sno_train_grad(t->args, t->bufs, m_dev, target_dev, t->stream));
    t->step += 1;
    MM_TRY(sno_train_adam(t->w, t->g, t->m1, t->m2, SNO_NWEIGHTS, (float)lr, 0.9f, 0.999f, 1e-8f, t->step,
                          t->stream));
    return read_loss(t, loss_out);
}

int mm_sno_train_get_weights(mm_sno_trainer* t, float* weights_host) {
    if (!t || !weights_host) return MM_EINVAL;
    MM_TRY(hipMemcpyAsync(weights_host, t->w, (size_t)SNO_NWEIGHTS * sizeof(float), hipMemcpyDeviceToHost,
                          t->stream));
    MM_TRY(hipStreamSynchronize(t->stream));
    return MM_OK;
}

void mm_sno_train_destroy(mm_sno_trainer* t) {
    if (!t) return;
    (void)hipStreamSynchronize(t->stream);
    free_tr(t);
    delete t;
}

}  // extern "C"
