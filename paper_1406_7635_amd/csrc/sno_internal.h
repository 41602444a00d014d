// sno_internal.h -- device arguments and launchers of the spectral neural
// operator (kernels_sno.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mm.h"

namespace mm {

constexpr int SNO_C = 32;       // channels
constexpr int SNO_KX = 16;      // kept kx = 0 .. 15
constexpr int SNO_KY = 16;      // kept ky = -8 .. 7
constexpr int SNO_LAYERS = 4;
// flat weight layout: P[32][3], p[32], per layer R[16][16][32][32][2], W[32][32], b[32], then Q[3][32], q[3]
constexpr long long SNO_LAYER_W = (long long)SNO_KY * SNO_KX * SNO_C * SNO_C * 2 + SNO_C * SNO_C + SNO_C;
constexpr long long SNO_NWEIGHTS = SNO_C * 3 + SNO_C + SNO_LAYERS * SNO_LAYER_W + 3 * SNO_C + 3;

struct SnoArgs {
    int nx, ny, n;                 // grid, n = nx ny
    float scale;                   // output units (B = scale * projection)
    const uint16_t* lift;          // BF16 weights, pointers into one array
    const uint16_t* lift_b;
    const uint16_t* spec[SNO_LAYERS];
    const uint16_t* pw[SNO_LAYERS];
    const uint16_t* pw_b[SNO_LAYERS];
    const uint16_t* proj;
    const uint16_t* proj_b;
    const float2* twx;             // exp(-2 pi i m / nx), m < nx
    const float2* twy;             // exp(-2 pi i m / ny), m < ny
    float* h0;                     // activations [32][ny][nx] (two buffers)
    float* h1;
    float2* H1;                    // [32][ny][16] after the x transform
    float2* Hh;                    // [32][16][16] kept modes
    float2* Gh;                    // [32][16][16] mixed modes
    float2* G1;                    // [32][ny][16] after the inverse y transform
};

// offsets of the parameter groups in the flat weight array
constexpr long long SNO_OFF_P = 0;
constexpr long long SNO_OFF_PB = SNO_C * 3;
constexpr long long SNO_OFF_L0 = SNO_C * 3 + SNO_C;
__host__ __device__ constexpr long long SNO_OFF_R(int l) { return SNO_OFF_L0 + l * SNO_LAYER_W; }
__host__ __device__ constexpr long long SNO_OFF_W(int l) {
    return SNO_OFF_R(l) + (long long)SNO_KY * SNO_KX * SNO_C * SNO_C * 2;
}
__host__ __device__ constexpr long long SNO_OFF_B(int l) { return SNO_OFF_W(l) + SNO_C * SNO_C; }
constexpr long long SNO_OFF_Q = SNO_OFF_L0 + SNO_LAYERS * SNO_LAYER_W;
constexpr long long SNO_OFF_QB = SNO_OFF_Q + 3 * SNO_C;
static_assert(SNO_OFF_QB + 3 == SNO_NWEIGHTS, "flat weight layout");

// Training (kernels_sno_train.hip): FP32 weights, a batch of samples.
struct SnoTrainArgs {
    int nx, ny, n, batch;
    const float* w;                // weights (flat, FP32)
    float* g;                      // gradient of the loss (flat)
    const float2* twx;             // exp(-2 pi i m / nx)
    const float2* twy;             // exp(-2 pi i m / ny)
};
struct SnoTrainBufs {
    float* h[SNO_LAYERS + 1];      // activations [B][32][n]: lift output, then each layer's output
    float* z[SNO_LAYERS];          // pre-GELU values of each layer [B][32][n]
    float2* H[SNO_LAYERS];         // kept modes of each layer's input [B][32][256]
    float2* line;                  // [B][32][ny][16] (x transform / inverse y transform)
    float2* modes;                 // [B][32][256]
    float2* modes2;                // [B][32][256]
    float* y;                      // prediction [B][3][n]
    float* dh[2];                  // gradients with respect to activations [B][32][n]
    float* dz;                     // [B][32][n]
    float* part;                   // per-workgroup partial sums [tiles][1056]
    double* lpart;                 // [B][64][2] loss partial sums
    float* scale;                  // [B] per-sample loss scale
    double* loss;                  // the batch loss
};
hipError_t configure_sno_train(int ny);
int sno_train_tiles(long long pixels);
hipError_t sno_train_grad(const SnoTrainArgs& a, const SnoTrainBufs& s, const float* m, const float* t,
                          hipStream_t st);
hipError_t sno_train_adam(float* w, const float* g, float* m1, float* m2, long long n, float lr, float b1, float b2,
                          float eps, long long step, hipStream_t st);

hipError_t sno_twiddles(float2* tw, int n, hipStream_t s);
// the forward pass of a created surrogate on a given stream, and its grid
hipError_t sno_run(const mm_sno* s, const float* m, float* out, hipStream_t stream);
void sno_grid(const mm_sno* s, int* nx, int* ny);
// the whole forward pass: m [3][n] -> out [3][n]
hipError_t sno_forward(const SnoArgs& a, const float* m, float* out, hipStream_t s);
size_t sno_dftx_lds(int nx);
// raise the LDS limit of the y transform (ny <= 512 rows: 69 KB)
hipError_t configure_sno(int ny);

}  // namespace mm
