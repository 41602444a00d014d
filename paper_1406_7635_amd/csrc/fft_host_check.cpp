// Host-side emulation of the LDS Stockham FFT of fft_core.h.
//
// Runs every stage's read half for all threads of a workgroup, then every
// write half, exactly as the barrier-separated device code does, and compares
// the result with a direct O(P^2) DFT in double precision.  Exit status 0 when
// every size and direction agrees to FP32 accuracy.  Built and run by the CPU
// test-suite (no GPU needed).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fft_core.h"

using mm::cf;

template <int P, int L, int F, int NT, bool INV>
struct HostFft {
    static void run(cf* buf, const cf* tw, int twshift) {
        constexpr int R = mm::stage_radix(P, L);
        using S = mm::Stage<P, R, L, F, NT, INV>;
        std::vector<cf> regs((size_t)NT * S::NB * R);
        for (int tid = 0; tid < NT; ++tid) {
            cf v[S::NB][R];
            S::read(buf, tw, twshift, tid, v);
            for (int q = 0; q < S::NB; ++q)
                for (int r = 0; r < R; ++r) regs[((size_t)tid * S::NB + q) * R + r] = v[q][r];
        }
        for (int tid = 0; tid < NT; ++tid) {
            cf v[S::NB][R];
            for (int q = 0; q < S::NB; ++q)
                for (int r = 0; r < R; ++r) v[q][r] = regs[((size_t)tid * S::NB + q) * R + r];
            S::write(buf, tid, v);
        }
        HostFft<P, L * R, F, NT, INV>::run(buf, tw, twshift);
    }
};

template <int P, int F, int NT, bool INV>
struct HostFft<P, P, F, NT, INV> {
    static void run(cf*, const cf*, int) {}
};

template <int P, int F, int NT>
static int check(int PT) {
    std::vector<cf> tw(PT);
    for (int m = 0; m < PT; ++m) {
        double a = -2.0 * M_PI * m / PT;
        tw[m] = mm::mkc((float)cos(a), (float)sin(a));
    }
    const int twshift = mm::ilog2(PT);
    int bad = 0;
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<cf> buf((size_t)F * mm::seq_len(P), mm::mkc(NAN, NAN));
        std::vector<double> re((size_t)F * P), im((size_t)F * P);
        srand(P * 7 + F + dir);
        for (int f = 0; f < F; ++f)
            for (int i = 0; i < P; ++i) {
                double a = rand() / (double)RAND_MAX - 0.5, b = rand() / (double)RAND_MAX - 0.5;
                re[(size_t)f * P + i] = (float)a;
                im[(size_t)f * P + i] = (float)b;
                buf[(size_t)f * mm::seq_len(P) + mm::lds_pad(i)] = mm::mkc((float)a, (float)b);
            }
        if (dir == 0)
            HostFft<P, 1, F, NT, false>::run(buf.data(), tw.data(), twshift);
        else
            HostFft<P, 1, F, NT, true>::run(buf.data(), tw.data(), twshift);
        double maxerr = 0, maxref = 0;
        for (int f = 0; f < F; ++f)
            for (int k = 0; k < P; ++k) {
                double sr = 0, si = 0;
                for (int n = 0; n < P; ++n) {
                    double a = (dir == 0 ? -2.0 : 2.0) * M_PI * (double)((long)n * k % P) / P;
                    double xr = re[(size_t)f * P + n], xi = im[(size_t)f * P + n];
                    sr += xr * cos(a) - xi * sin(a);
                    si += xr * sin(a) + xi * cos(a);
                }
                cf g = buf[(size_t)f * mm::seq_len(P) + mm::lds_pad(k)];
                maxerr = fmax(maxerr, fmax(fabs(g.x - sr), fabs(g.y - si)));
                maxref = fmax(maxref, fmax(fabs(sr), fabs(si)));
            }
        const double tol = 2e-6 * (mm::ilog2(P) + 1) * maxref + 1e-6;
        const bool ok = maxerr <= tol;
        if (!ok) ++bad;
        printf("P=%5d F=%2d NT=%3d %s max_err=%.3e ref=%.3e %s\n", P, F, NT, dir ? "inv" : "fwd",
               maxerr, maxref, ok ? "ok" : "FAIL");
    }
    return bad;
}

int main() {
    int bad = 0;
    bad += check<1, 3, 256>(4096);
    bad += check<2, 3, 256>(4096);
    bad += check<4, 6, 256>(4096);
    bad += check<8, 3, 256>(4096);
    bad += check<16, 5, 256>(1024);
    bad += check<32, 3, 64>(4096);
    bad += check<64, 48, 256>(4096);
    bad += check<128, 48, 256>(4096);
    bad += check<256, 24, 256>(4096);
    bad += check<512, 12, 256>(512);
    bad += check<1024, 6, 256>(4096);
    bad += check<2048, 3, 256>(2048);
    bad += check<4096, 3, 256>(4096);
    printf("%s\n", bad ? "FAILED" : "ALL OK");
    return bad ? 1 : 0;
}
