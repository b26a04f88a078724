// Exercises the library's host-side ring planning helpers (sht_internal.h)
// under AddressSanitizer and UndefinedBehaviorSanitizer (built and run by
// tests/test_host_sanitizers.py; host code only, no GPU call): for every
// half length up to 8192 the fast-path radix list multiplies back to the
// length, fits the per-thread butterfly limit and unpacks from its 5-bit
// fields, and the LDS layouts cover the buffers the kernels index; the same
// for the Bluestein fast path's convolution lengths up to 4096 (one
// butterfly per thread in every pass).
#include <cstdio>

#include "sht_internal.h"

int main()
{
    int fail = 0, eligible = 0;
    for (int h = 0; h <= 8192; ++h) {
        unsigned long long rads = 0;
        const int np = sht::fast_radices(h, &rads);
        if (np == 0) continue;
        ++eligible;
        long long prod = 1;
        for (int p = 0; p < np; ++p) {
            const int R = (int)((rads >> (5 * p)) & 31);
            if (R != 16 && R != 8 && R != 4 && R != 2 && R != 7 && R != 5 && R != 3) fail = 1;
            if (h / R > sht::fast_maxq(R) * sht::kFastThreads) fail = 1;
            prod *= R;
        }
        if (prod != h || h > sht::kFastMaxH) fail = 1;
        for (int mmax : {0, 100, 4096, sht::kFastMaxModes - 1}) {
            sht::RingLds l = {};
            sht::fast_lds_add(l, 2 * h, mmax);
            const int top = h > mmax ? h : mmax;
            if (l.fft_entries < sht::fast_pad(top) + 1) fail = 1;
            if (l.fft_entries < sht::fast_pad(sht::kFastThreads - 1) + 1) fail = 1;
            if (l.tw_entries < 64 + (2 * h + 63) / 64) fail = 1;
        }
    }
    int blue = 0;
    for (int nb = 0; nb <= 2 * sht::kBlueMaxN; ++nb) {
        unsigned long long rads = 0;
        const int np = sht::blue_radices(nb, &rads);
        if (np == 0) continue;
        ++blue;
        long long prod = 1;
        for (int p = 0; p < np; ++p) {
            const int R = (int)((rads >> (5 * p)) & 31);
            if (R != 8 && R != 4 && R != 2 && R != 7 && R != 5 && R != 3) fail = 1;
            if (nb / R > sht::kBlueThreads) fail = 1;
            prod *= R;
        }
        if (prod != nb || nb > sht::kBlueMaxN) fail = 1;
        for (int h : {nb / 2 + 1, nb + 1}) {   // half lengths whose convolution is nb
            if (h % 2) ++h;
            for (int mmax : {0, 100, 4096, sht::kFastMaxModes - 1}) {
                sht::RingLds l = {};
                sht::blue_lds_add(l, 2 * h, nb, mmax);
                int top = h > mmax ? h : mmax;
                top = top > nb - 1 ? top : nb - 1;
                top = top > sht::kBlueThreads - 1 ? top : sht::kBlueThreads - 1;
                if (l.fft_entries < sht::fast_pad(top) + 1) fail = 1;
                if (l.y_entries < sht::fast_pad(nb - 1) + 1) fail = 1;
                if (l.tw_entries < 64 + (2 * h + 63) / 64) fail = 1;
                if (l.tb_entries < 64 + (nb + 63) / 64) fail = 1;
                if (l.total() != l.fft_entries + l.y_entries + l.tw_entries + l.tb_entries)
                    fail = 1;
            }
        }
    }
    if (blue < 50) fail = 1;
    for (int c = 0; c < sht::kNumRingClasses; ++c) {
        for (int n = 1; n <= 16384; n += 7) {
            sht::RingLds l = {};
            sht::ring_lds_add(l, c, n, (n % 3) ? 0 : 2 * n, n / 2 + 1);
            if (l.fft_entries < 8 * sht::kClassThreads[c]) fail = 1;
            if (l.tw_entries < 64 + (n + 63) / 64) fail = 1;
        }
    }
    if (eligible < 100) fail = 1;
    if (fail) {
        std::fprintf(stderr, "plan driver: invariant violated\n");
        return 1;
    }
    std::printf("plan driver ok (%d fast-path lengths, %d Bluestein fast-path lengths)\n",
                eligible, blue);
    return 0;
}
