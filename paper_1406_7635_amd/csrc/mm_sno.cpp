// mm_sno.cpp -- C ABI of the spectral-neural-operator surrogate: weights
// (rounded to BF16 on upload), buffers, forward pass.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/mm.h"
#include "api_common.h"
#include "sno_internal.h"

using namespace mm;

static_assert(SNO_NWEIGHTS == MM_SNO_NWEIGHTS, "weight count of the C ABI");

struct mm_sno {
    hipStream_t stream = nullptr;
    int nx = 0, ny = 0;
    double scale = 1.0;
    uint16_t* w = nullptr;
    float2* tw = nullptr;  // nx x-twiddles then ny y-twiddles
    float* h = nullptr;    // two activation buffers
    float2* modes = nullptr;
    SnoArgs args;
};

namespace {

// FP32 -> BF16, round to nearest even (NaN stays NaN)
uint16_t to_bf16(float f) {
    unsigned int u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

void free_sno(mm_sno* s) {
    void* p[] = {s->w, s->tw, s->h, s->modes};
    for (void* q : p)
        if (q) (void)hipFree(q);
}

int upload(mm_sno* s, const float* weights, int64_t nweights) {
    if (!weights || nweights != SNO_NWEIGHTS) return MM_EINVAL;
    std::vector<uint16_t> hb;
    try {
        hb.resize((size_t)nweights);
    } catch (...) {
        return MM_ENOMEM;
    }
    for (int64_t i = 0; i < nweights; ++i) hb[(size_t)i] = to_bf16(weights[i]);
    MM_TRY(hipStreamSynchronize(s->stream));
    MM_TRY(hipMemcpy(s->w, hb.data(), (size_t)nweights * sizeof(uint16_t), hipMemcpyHostToDevice));
    return MM_OK;
}

}  // namespace

namespace mm {
hipError_t sno_run(const mm_sno* s, const float* m, float* out, hipStream_t stream) {
    return sno_forward(s->args, m, out, stream);
}
void sno_grid(const mm_sno* s, int* nx, int* ny) {
    *nx = s->nx;
    *ny = s->ny;
}
}  // namespace mm

extern "C" {

int mm_sno_create(mm_sno** out, int32_t nx, int32_t ny, const float* weights, int64_t nweights, double out_scale,
                  void* hip_stream) {
    if (!out || !weights) return MM_EINVAL;
    *out = nullptr;
    if (nweights != SNO_NWEIGHTS || !isfinite(out_scale)) return MM_EINVAL;
    if (nx < 2 * SNO_KX || ny < SNO_KY || nx > 512 || ny > 512) return MM_EUNSUPPORTED;
    mm_sno* s = new (std::nothrow) mm_sno();
    if (!s) return MM_ENOMEM;
    s->stream = (hipStream_t)hip_stream;
    s->nx = nx;
    s->ny = ny;
    s->scale = out_scale;
    const size_t n = (size_t)nx * ny;
    hipError_t e = hipMalloc((void**)&s->w, (size_t)SNO_NWEIGHTS * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->tw, (size_t)(nx + ny) * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc((void**)&s->h, 2 * SNO_C * n * sizeof(float));
    const size_t line = (size_t)SNO_C * ny * SNO_KX, kept = (size_t)SNO_C * SNO_KY * SNO_KX;
    if (e == hipSuccess) e = hipMalloc((void**)&s->modes, (2 * line + 2 * kept) * sizeof(float2));
    if (e == hipSuccess) e = configure_sno(ny);
    if (e == hipSuccess) e = sno_twiddles(s->tw, nx, s->stream);
    if (e == hipSuccess) e = sno_twiddles(s->tw + nx, ny, s->stream);
    int st = map_err(e);
    if (st == MM_OK) st = upload(s, weights, nweights);
    if (st != MM_OK) {
        free_sno(s);
        delete s;
        return st;
    }
    SnoArgs& a = s->args;
    memset(&a, 0, sizeof(a));
    a.nx = nx;
    a.ny = ny;
    a.n = nx * ny;
    a.scale = (float)out_scale;
    long long o = 0;
    a.lift = s->w + o;
    o += SNO_C * 3;
    a.lift_b = s->w + o;
    o += SNO_C;
    for (int l = 0; l < SNO_LAYERS; ++l) {
        a.spec[l] = s->w + o;
        o += (long long)SNO_KY * SNO_KX * SNO_C * SNO_C * 2;
        a.pw[l] = s->w + o;
        o += SNO_C * SNO_C;
        a.pw_b[l] = s->w + o;
        o += SNO_C;
    }
    a.proj = s->w + o;
    o += 3 * SNO_C;
    a.proj_b = s->w + o;
    a.twx = s->tw;
    a.twy = s->tw + nx;
    a.h0 = s->h;
    a.h1 = s->h + SNO_C * n;
    a.H1 = s->modes;
    a.G1 = s->modes + line;
    a.Hh = s->modes + 2 * line;
    a.Gh = s->modes + 2 * line + kept;
    *out = s;
    return MM_OK;
}

int mm_sno_set_weights(mm_sno* s, const float* weights, int64_t nweights) {
    if (!s) return MM_EINVAL;
    return upload(s, weights, nweights);
}

int mm_sno_eval(mm_sno* s, const float* m_dev, float* b_dev) {
    if (!s || !m_dev || !b_dev) return MM_EINVAL;
    MM_TRY(sno_forward(s->args, m_dev, b_dev, s->stream));
    return MM_OK;
}

void mm_sno_destroy(mm_sno* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    free_sno(s);
    delete s;
}

}  // extern "C"
