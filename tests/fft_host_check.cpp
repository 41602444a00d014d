// Host-side emulation of the register-resident FFT of fft_core.h.
//
// Runs every phase (stage 0, then per exchange: the LDS writes of all threads,
// then their reads and butterflies) for all threads of a group, exactly in the
// order the barrier-separated device code imposes, and compares the result
// with a direct O(P^2) DFT in double precision.  The zero-padded variant
// (inputs n >= P/2 zero) gets NaN in the registers it must ignore.  Exit status 0 when
// every size and direction agrees to FP32 accuracy.  Built and run by the CPU
// test-suite (no GPU needed).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <array>
#include <vector>

#include "fft_core.h"

using mm::cf;

// Emulation of RegFft: every phase for all TPF threads, in barrier order.
template <int P, int TPF, int NF, bool INV, bool HIN>
static void host_regfft(std::vector<cf>& data /* NF * P natural */, const cf* tw, int twshift) {
    using R = mm::RegFft<P, TPF, NF, INV, HIN>;
    constexpr int PPT = R::PPT;
    std::vector<std::array<std::array<cf, PPT>, NF>> regs(TPF);
    for (int t = 0; t < TPF; ++t)
        for (int f = 0; f < NF; ++f)
            for (int m = 0; m < PPT; ++m) {
                const int n = t + TPF * m;
                regs[t][f][m] = (HIN && P >= 2 && 2 * n >= P) ? mm::mkc(NAN, NAN) : data[(size_t)f * P + n];
            }
    auto as_arr = [](std::array<std::array<cf, PPT>, NF>& a) -> cf(&)[NF][PPT] {
        return *reinterpret_cast<cf(*)[NF][PPT]>(&a);
    };
    if (R::NS > 0) {
        for (int t = 0; t < TPF; ++t) R::stage0(as_arr(regs[t]));
        std::vector<cf> buf(mm::seq_len(P), mm::mkc(NAN, NAN));
        for (int s = 1; s < R::NS; ++s) {
            for (int f = 0; f < NF; ++f) {
                for (int t = 0; t < TPF; ++t) R::write(s, as_arr(regs[t]), f, buf.data(), t);
                for (int t = 0; t < TPF; ++t) {
                    cf wt[PPT];
                    R::twiddles(s, t, tw, twshift, wt);
                    R::read_compute(s, as_arr(regs[t]), f, buf.data(), t, wt);
                }
            }
        }
        for (int t = 0; t < TPF; ++t) R::finish(as_arr(regs[t]));
    }
    for (int t = 0; t < TPF; ++t)
        for (int f = 0; f < NF; ++f)
            for (int m = 0; m < PPT; ++m) data[(size_t)f * P + t + TPF * m] = regs[t][f][m];
}

template <int P, int TPF>
static int check_reg(int PT) {
    constexpr int NF = 3;
    std::vector<cf> tw(PT);
    for (int m = 0; m < PT; ++m) {
        double a = -2.0 * M_PI * m / PT;
        tw[m] = mm::mkc((float)cos(a), (float)sin(a));
    }
    int bad = 0;
    for (int mode = 0; mode < 4; ++mode) {
        const int dir = mode & 1, hin = mode >> 1;
        std::vector<cf> data((size_t)NF * P);
        std::vector<double> re(data.size()), im(data.size());
        srand(P * 13 + TPF + mode);
        for (size_t i = 0; i < data.size(); ++i) {
            const bool zero = hin && P >= 2 && 2 * (int)(i % P) >= P;
            re[i] = zero ? 0.0 : (float)(rand() / (double)RAND_MAX - 0.5);
            im[i] = zero ? 0.0 : (float)(rand() / (double)RAND_MAX - 0.5);
            data[i] = mm::mkc((float)re[i], (float)im[i]);
        }
        if (mode == 0) host_regfft<P, TPF, NF, false, false>(data, tw.data(), mm::ilog2(PT));
        else if (mode == 1) host_regfft<P, TPF, NF, true, false>(data, tw.data(), mm::ilog2(PT));
        else if (mode == 2) host_regfft<P, TPF, NF, false, true>(data, tw.data(), mm::ilog2(PT));
        else host_regfft<P, TPF, NF, true, true>(data, tw.data(), mm::ilog2(PT));
        double maxerr = 0, maxref = 0;
        for (int f = 0; f < NF; ++f)
            for (int k = 0; k < P; ++k) {
                double sr = 0, si = 0;
                for (int n = 0; n < P; ++n) {
                    double a = (dir == 0 ? -2.0 : 2.0) * M_PI * (double)((long)n * k % P) / P;
                    sr += re[(size_t)f * P + n] * cos(a) - im[(size_t)f * P + n] * sin(a);
                    si += re[(size_t)f * P + n] * sin(a) + im[(size_t)f * P + n] * cos(a);
                }
                cf g = data[(size_t)f * P + k];
                maxerr = fmax(maxerr, fmax(fabs(g.x - sr), fabs(g.y - si)));
                maxref = fmax(maxref, fmax(fabs(sr), fabs(si)));
            }
        const double tol = 2e-6 * (mm::ilog2(P) + 1) * maxref + 1e-6;
        const bool ok = maxerr <= tol;
        if (!ok) ++bad;
        printf("reg P=%5d TPF=%3d %s%s max_err=%.3e ref=%.3e %s\n", P, TPF, dir ? "inv" : "fwd",
               hin ? " half-input" : "", maxerr, maxref, ok ? "ok" : "FAIL");
    }
    return bad;
}

int main() {
    int bad = 0;
    bad += check_reg<1, 1>(4096);
    bad += check_reg<2, 1>(4096);
    bad += check_reg<4, 1>(4096);
    bad += check_reg<8, 1>(4096);
    bad += check_reg<16, 2>(4096);
    bad += check_reg<32, 4>(4096);
    bad += check_reg<64, 8>(4096);
    bad += check_reg<128, 16>(4096);
    bad += check_reg<256, 32>(4096);
    bad += check_reg<512, 64>(512);
    bad += check_reg<512, 32>(4096);
    bad += check_reg<1024, 64>(4096);
    bad += check_reg<2048, 128>(2048);
    bad += check_reg<2048, 256>(4096);
    bad += check_reg<4096, 256>(4096);
    bad += check_reg<4096, 512>(4096);
    printf("%s\n", bad ? "FAILED" : "ALL OK");
    return bad ? 1 : 0;
}
