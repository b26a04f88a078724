// Device helpers of the Legendre recurrence shared by the FP64 and the
// mixed-precision kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sht_internal.h"

namespace sht {
namespace {

constexpr double kTwoS = 0x1p512;
constexpr double kTwoMinusS = 0x1p-512;

// mu * s^m as (v, k): value v 2^(512 k), k <= 0, v in (2^-513 mu, mu].
// Repeated squaring with the mantissa renormalised after every product.
__device__ inline void seed_mm(double mu, double s, int m, double &v, int &k)
{
    if (m == 0) { v = mu; k = 0; return; }
    if (s == 0.0) { v = 0.0; k = 0; return; }
    int e;
    double b = frexp(s, &e);
    int be = e;
    double r = 1.0;
    int re = 0;
    int p = m;
    while (p) {
        if (p & 1) {
            r *= b; re += be;
            r = frexp(r, &e); re += e;
        }
        p >>= 1;
        if (p) {
            b *= b; be *= 2;
            b = frexp(b, &e); be += e;
        }
    }
    int kk = (re < 0) ? -((-re) / kScaleStep) : 0;
    v = ldexp(mu * r, re - kScaleStep * kk);
    k = kk;
}

__device__ inline double final_scale(int k)
{
    return k == 0 ? 1.0 : (k == -1 ? kTwoMinusS : 0.0);
}

// Block id -> logical id so that consecutive logical ids share an XCD.
__device__ inline long long xcd_logical(long long b, long long total)
{
    const long long nx = 8;
    long long x = b % nx, i = b / nx;
    long long q = total / nx, r = total % nx;
    return x * q + (x < r ? x : r) + i;
}

}  // namespace
}  // namespace sht
