// Host-side check of the C ABI's argument validation and error cleanup,
// built with AddressSanitizer / UBSan on the host code and run without a GPU.
//
// Every call below either returns before touching the device (null
// pointers, sizes, non-finite parameters) or, past validation, fails at
// its first HIP call on a machine without a GPU and must then release what
// it had allocated (the context object, its host tables).  Exit status 0 and
// "ALL OK" when every status is the documented one; the sanitizers report
// any out-of-bounds access, leak or undefined behaviour on the way.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mm.h"

static int g_bad = 0;

static void expect(const char* what, int got, int want) {
    if (got != want) {
        std::printf("FAIL %s: got %d (%s), want %d (%s)\n", what, got, mm_strerror(got), want, mm_strerror(want));
        ++g_bad;
    }
}

static void expect_not_ok(const char* what, int got) {
    if (got == MM_OK) {
        std::printf("FAIL %s: got MM_OK without a device\n", what);
        ++g_bad;
    }
}

int main() {
    static mm_params p;  // large (0.3 MB): static storage
    std::memset(&p, 0, sizeof(p));
    for (int r = 0; r < MM_NREGIONS; ++r) {
        p.msat[r] = 8e5;
        p.aex[r] = 1.3e-11;
        p.alpha[r] = 0.01;
        p.anis_u[r][0] = 1.0;
    }
    for (int i = 0; i < MM_NPAIRS; ++i) p.exch_scale[i] = 1.0;
    mm_grid g = {8, 8, 1, 2e-9, 2e-9, 2e-9, {0, 0, 0}};
    std::vector<unsigned char> region(64, 0);
    mm_ctx* c = nullptr;

    // null pointers and invalid sizes: rejected before any device call
    expect("create null out", mm_create(nullptr, &g, &p, region.data(), nullptr), MM_EINVAL);
    expect("create null grid", mm_create(&c, nullptr, &p, region.data(), nullptr), MM_EINVAL);
    expect("create null params", mm_create(&c, &g, nullptr, region.data(), nullptr), MM_EINVAL);
    expect("create null region", mm_create(&c, &g, &p, nullptr, nullptr), MM_EINVAL);
    mm_grid bad = g;
    bad.nx = 0;
    expect("create nx 0", mm_create(&c, &bad, &p, region.data(), nullptr), MM_EINVAL);
    bad = g;
    bad.dy = NAN;
    expect("create dy NaN", mm_create(&c, &bad, &p, region.data(), nullptr), MM_EINVAL);
    bad = g;
    bad.pbc[2] = -1;
    expect("create negative pbc", mm_create(&c, &bad, &p, region.data(), nullptr), MM_EINVAL);
    bad = g;
    bad.nx = 5000;
    expect("create nx 5000", mm_create(&c, &bad, &p, region.data(), nullptr), MM_EUNSUPPORTED);
    bad = g;
    bad.pbc[0] = 1 << 21;
    expect("create huge image count", mm_create(&c, &bad, &p, region.data(), nullptr), MM_EUNSUPPORTED);
    p.msat[3] = -1.0;
    expect("create negative Msat", mm_create(&c, &g, &p, region.data(), nullptr), MM_EINVAL);
    p.msat[3] = 8e5;
    p.exch_scale[77] = INFINITY;
    expect("create infinite exchange scale", mm_create(&c, &g, &p, region.data(), nullptr), MM_EINVAL);
    p.exch_scale[77] = 1.0;
    expect("create left out null", c == nullptr ? 0 : 1, 0);

    // null contexts on every entry point that takes one
    float dummy = 0.f;
    double t = 0.0, dt = 1e-14, e5[5];
    int32_t acc = 0;
    expect("beff null ctx", mm_beff(nullptr, &dummy, &dummy, nullptr), MM_EINVAL);
    expect("beff_noalloc null ctx", mm_beff_noalloc(nullptr, &dummy, &dummy, nullptr), MM_EINVAL);
    expect("torque null ctx", mm_llg_torque(nullptr, &dummy, &dummy, &dummy, 1), MM_EINVAL);
    expect("rk4 null ctx", mm_rk4_step(nullptr, &dummy, 1e-14, 1), MM_EINVAL);
    expect("rk45 null ctx", mm_rk45_step(nullptr, &dummy, &t, &dt, nullptr, &acc, nullptr), MM_EINVAL);
    expect("energy null ctx", mm_energy(nullptr, &dummy, e5), MM_EINVAL);
    expect("demag init null ctx", mm_demag_kernel_init(nullptr), MM_EINVAL);
    expect("set params null ctx", mm_set_params(nullptr, &p), MM_EINVAL);
    mm_destroy(nullptr);

    // past validation: without a device the first HIP call fails, and the
    // partly built context must be released (LeakSanitizer checks it)
    for (int rep = 0; rep < 3; ++rep) {
        c = nullptr;
        expect_not_ok("create without a device", mm_create(&c, &g, &p, region.data(), nullptr));
        expect("create failure leaves out null", c == nullptr ? 0 : 1, 0);
    }

    // ensembles
    mm_batch* b = nullptr;
    mm_grid gs[2] = {g, g};
    static mm_params ps[2];
    std::memcpy(&ps[0], &p, sizeof(p));
    std::memcpy(&ps[1], &p, sizeof(p));
    expect("batch null out", mm_batch_create(nullptr, 2, gs, ps, region.data(), nullptr), MM_EINVAL);
    expect("batch n 0", mm_batch_create(&b, 0, gs, ps, region.data(), nullptr), MM_EINVAL);
    mm_grid gb[1] = {g};
    gb[0].nx = 1024;
    expect("batch member too large", mm_batch_create(&b, 1, gb, ps, region.data(), nullptr), MM_EUNSUPPORTED);
    int32_t gv = 0, tv = 0;
    expect("batch set grid null", mm_batch_set_grid(nullptr, 0, 8), MM_EINVAL);
    expect("batch get grid null", mm_batch_get_grid(nullptr, 0, &gv), MM_EINVAL);
    expect("batch set tile null", mm_batch_set_tile(nullptr, 0, 1), MM_EINVAL);
    expect("batch get tile null", mm_batch_get_tile(nullptr, 0, &tv), MM_EINVAL);
    expect("batch autotune null", mm_batch_autotune(nullptr, &dummy), MM_EINVAL);
    mm_batch_destroy(nullptr);

    // checkpoint calls
    int64_t sz = 0;
    expect("state size null ctx", mm_state_size(nullptr, &sz), MM_EINVAL);
    expect("state save null ctx", mm_state_save(nullptr, &dummy, 4), MM_EINVAL);
    expect("state load null ctx", mm_state_load(nullptr, &dummy, 4, &dummy), MM_EINVAL);

    // surrogate and its trainer
    std::vector<float> w(MM_SNO_NWEIGHTS, 0.f);
    mm_sno* s = nullptr;
    expect("sno null weights", mm_sno_create(&s, 256, 256, nullptr, MM_SNO_NWEIGHTS, 1.0, nullptr), MM_EINVAL);
    expect("sno weight count", mm_sno_create(&s, 256, 256, w.data(), MM_SNO_NWEIGHTS - 1, 1.0, nullptr), MM_EINVAL);
    expect("sno grid too large", mm_sno_create(&s, 1024, 256, w.data(), MM_SNO_NWEIGHTS, 1.0, nullptr),
           MM_EUNSUPPORTED);
    mm_sno_trainer* tr = nullptr;
    w[5] = NAN;
    expect("trainer NaN weight", mm_sno_train_create(&tr, 256, 256, 4, w.data(), MM_SNO_NWEIGHTS, nullptr), MM_EINVAL);
    w[5] = 0.f;
    expect("trainer batch 0", mm_sno_train_create(&tr, 256, 256, 0, w.data(), MM_SNO_NWEIGHTS, nullptr), MM_EINVAL);
    mm_sno_destroy(nullptr);
    mm_sno_train_destroy(nullptr);

    if (g_bad == 0) std::printf("ALL OK\n");
    return g_bad == 0 ? 0 : 1;
}
