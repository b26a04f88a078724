// Pieces shared by the two mixed-precision Legendre kernels (FP32 and
// 3-way split BF16 matrix-core operands): the lane state rule of the
// recurrence, the exchange of fragment halves, the output tiles and the
// Delta epilogue.
#pragma once

#include "recurrence.h"
#include "sht_internal.h"

namespace sht {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Lane state of the mixed kernels.  u = P_l / c_l is carried as v 2^(512 k),
// k <= 0, as in the FP64 kernel, but a lane moves up to k = 0 as soon as its
// true value passes 2^-400 (|v| > 2^112 at k = -1).  Checked every 16 steps
// (growth below 2^140), every lane with k < 0 then holds a true value below
// 2^-260, which is zero in FP32: the matrix operand is (float)v for k = 0 and
// 0 otherwise.  Values at k = 0 are bounded by sqrt((2l+1)/4pi)/c_l < 2^9
// (addition theorem), so a wave whose lanes all reached k = 0 -- almost every
// wave past its first l-steps -- needs neither the mask nor any rescaling.
constexpr double kEmerge = 0x1p112;
constexpr double kEmergeTrue = 0x1p-400;

__device__ inline void rescale_mixed(double &ua, double &ub, int &k)
{
    if (k < 0) {
        const double lim = (k == -1) ? kEmerge : kTwoS;
        if (fmax(fabs(ua), fabs(ub)) > lim) {
            ua *= kTwoMinusS; ub *= kTwoMinusS;
            k += 1;
        }
    }
}

__device__ inline bool wave_any(bool c) { return __builtin_amdgcn_ballot_w64(c) != 0; }

__device__ inline float opnd(double u, bool live) { return live ? (float)u : 0.0f; }

__device__ inline void swap_halves(float a, float b, float &lo, float &hi)
{
    const v2u r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b),
                                                   false, false);
    lo = __uint_as_float(r[0]);
    hi = __uint_as_float(r[1]);
}

struct MfmaTiles {
    v16f e0, e1, o0, o1;  // even / odd parity, rows 0-31 / 32-63
};

__device__ __forceinline__ void zero_tiles(MfmaTiles &t)
{
    t.e0 = v16f{}; t.e1 = v16f{}; t.o0 = v16f{}; t.o1 = v16f{};
}

__device__ __forceinline__ void add_tiles(MfmaTiles &tot, const MfmaTiles &acc)
{
    tot.e0 += acc.e0; tot.e1 += acc.e1; tot.o0 += acc.o0; tot.o1 += acc.o1;
}

// 16 rows of the recurrence alone, the coefficients read straight from the
// table, used while the whole workgroup is still below 2^-400 (nothing
// staged in LDS; every matrix operand would be 0).  The
// block may run past the m's last row (the table is padded by 16 entries):
// the state is then never used, since the m has no live rows left.
template <bool SEED>
__device__ __forceinline__ void block16_dead_g(double x, double &ua, double &ub,
                                               const double *__restrict__ Am, int r0)
{
    double a[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) a[t] = Am[r0 + t];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        double u0, u1;
        if (SEED && t == 0) {
            u0 = ua;
            u1 = (a[1] * x) * ua;
        } else {
            u0 = fma(a[4 * t] * x, ub, -ua);
            u1 = fma(a[4 * t + 1] * x, u0, -ub);
        }
        const double u2 = fma(a[4 * t + 2] * x, u1, -u0);
        const double u3 = fma(a[4 * t + 3] * x, u2, -u1);
        ua = u2;
        ub = u3;
    }
}

// Delta of one m.  D layout of a 32x32 tile: column = lane % 32 (the ring
// pair), row = 8 (r/4) + 4 (lane/32) + r % 4 = 2 map + Re/Im, so a lane owns
// 8 complex values of one pair.  The mixed forms' Delta is [m][ring][map]
// (maps contiguous): the ring stage reads a ring's modes for all maps at
// once, and the wave writes every map of its rings, so each line is filled
// by one wave.  The parity sums are FP32; north (E + O) and south (E - O)
// are formed exactly in FP64 and rounded once to FP32, the precision the
// contraction carries, so Delta is stored as complex64.
__device__ __forceinline__ void m_store(const MfmaTiles &tot, int i, float2 *__restrict__ delta,
                                        const PairDesc *__restrict__ pairs, int npairs, int pb,
                                        int grp, int nmaps, int nrings, int nm, int lane)
{
    const int hi = lane >> 5;
    const int col = lane & 31;
    float2 *__restrict__ d2 = delta;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const v16f &E = h ? tot.e1 : tot.e0;
        const v16f &O = h ? tot.o1 : tot.o0;
        const int pp = pb * 64 + h * 32 + col;
        if (pp < npairs) {
            const PairDesc d = pairs[pp];
            const long long row = (long long)i * nrings;
            float2 *__restrict__ dn = d2 + (row + d.rn) * nmaps;
            float2 *__restrict__ ds = d2 + (row + (d.rs >= 0 ? d.rs : d.rn)) * nmaps;
#pragma unroll
            for (int r = 0; r < 16; r += 4) {
                // rows r .. r + 3: maps m0 and m0 + 1, adjacent in Delta, so
                // one 16-byte store takes both when the alignment allows
                const int m0 = grp * 16 + 4 * (r >> 2) + 2 * hi;
                float2 n[2], so[2];
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const double er = E[r + 2 * k], ei = E[r + 2 * k + 1];
                    const double orr = O[r + 2 * k], oi = O[r + 2 * k + 1];
                    n[k] = make_float2((float)(er + orr), (float)(ei + oi));
                    so[k] = make_float2((float)(er - orr), (float)(ei - oi));
                }
                if (m0 + 1 < nmaps && (nmaps & 1) == 0) {
                    *reinterpret_cast<float4 *>(dn + m0) =
                        make_float4(n[0].x, n[0].y, n[1].x, n[1].y);
                    if (d.rs >= 0)
                        *reinterpret_cast<float4 *>(ds + m0) =
                            make_float4(so[0].x, so[0].y, so[1].x, so[1].y);
                } else {
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        if (m0 + k < nmaps) {
                            dn[m0 + k] = n[k];
                            if (d.rs >= 0) ds[m0 + k] = so[k];
                        }
                    }
                }
            }
        }
    }
}

}  // namespace
}  // namespace sht
