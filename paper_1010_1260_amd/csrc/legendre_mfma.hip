// Mixed-precision batched Legendre stage on the matrix cores (gfx950).
//
// For a batch of maps sharing one geometry, Delta_m(theta) of Eq. (DeltaDef)
// is, per m, a matrix product: with ring pairs as rows, l as the inner index
// and (map, Re/Im) as columns,
//     C_E[pairs x 32] = Lambda_E[pairs x K] * B_E[K x 32]   (l - m even)
//     C_O[pairs x 32] = Lambda_O[pairs x K] * B_O[K x 32]   (l - m odd)
//     Delta_N = C_E + C_O,  Delta_S = C_E - C_O.
// The recurrence (Eq. assLegRec, seeds Eqs. pmm / pm1m, rescaling of
// Sec. 2.2.2) stays in FP64 on the vector ALUs, exactly as in the FP64
// kernel; only the true values P_lm, rounded to FP32, and the FP32 copy of
// the prescaled coefficients enter v_mfma_f32_32x32x2f32.
//
// Fragment assembly.  Lane r of a wave runs the recurrence of ring pair r
// (rows 0-31: lanes 0-31, rows 32-63: lanes 32-63).  A 32x32x2 A-fragment
// needs, in lanes 32-63, the second K value of rows 0-31; four consecutive
// steps give X0 = P_l, X1 = P_{l+1}, X2 = P_{l+2}, X3 = P_{l+3} per lane, and
// one v_permlane32_swap of (X0, X2) yields the even-parity fragments of both
// row halves ([X0_lo | X2_lo] and [X0_hi | X2_hi]); (X1, X3) gives the odd ones.
//
// Accumulation.  FP32 accumulation over all l-terms loses up to ~1e-6; the
// matrix core accumulates 64 same-parity terms per block, and the block sums
// are added into a second FP32 accumulator (two-level summation).  Emulated
// error of Delta at l_max = 4096: about 1.2e-7 relative.
#include "recurrence.h"
#include "sht_internal.h"

namespace sht {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));


__global__ void k_prescale_f32(const double2 *__restrict__ alm, const double *__restrict__ cn,
                               float *__restrict__ Bf, long long nalm, int nmaps, long long m0len)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nalm * 32) return;
    const long long e = t >> 5;
    const int col = (int)(t & 31);
    const int grp = blockIdx.y;
    const int map = grp * 16 + (col >> 1);
    float v = 0.0f;
    if (map < nmaps) {
        const double2 a = alm[(long long)map * nalm + e];
        const double c = cn[e];
        const double x = (col & 1) ? ((e < m0len) ? 0.0 : a.y * c) : a.x * c;
        v = (float)x;
    }
    Bf[((long long)grp * nalm + e) * 32 + col] = v;
}

// Lane state of the mixed kernels.  u = P_l / c_l is carried as v 2^(512 k),
// k <= 0, as in the FP64 kernel, but a lane moves up to k = 0 as soon as its
// true value passes 2^-400 (|v| > 2^112 at k = -1).  Checked every 16 steps
// (growth below 2^140), every lane with k < 0 then holds a true value below
// 2^-260, which is zero in FP32: the matrix operand is (float)v for k = 0 and
// 0 otherwise.  Values at k = 0 are bounded by sqrt((2l+1)/4pi)/c_l < 2^9
// (addition theorem), so a wave whose lanes all reached k = 0 -- almost every
// wave past its first l-steps -- needs neither the mask nor any rescaling.
constexpr double kEmerge = 0x1p112;

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

// Four MFMAs of one group of 4 l-values: X0..X3 = P_l..P_{l+3} of the lane's
// ring pair; BE / BO = the lane's B elements of the even / odd rows.
__device__ __forceinline__ void mfma4(float X0, float X1, float X2, float X3, float BE, float BO,
                                      MfmaTiles &acc)
{
    float A0E, A1E, A0O, A1O;
    swap_halves(X0, X2, A0E, A1E);
    swap_halves(X1, X3, A0O, A1O);
    acc.e0 = __builtin_amdgcn_mfma_f32_32x32x2f32(A0E, BE, acc.e0, 0, 0, 0);
    acc.e1 = __builtin_amdgcn_mfma_f32_32x32x2f32(A1E, BE, acc.e1, 0, 0, 0);
    acc.o0 = __builtin_amdgcn_mfma_f32_32x32x2f32(A0O, BO, acc.o0, 0, 0, 0);
    acc.o1 = __builtin_amdgcn_mfma_f32_32x32x2f32(A1O, BO, acc.o1, 0, 0, 0);
}

constexpr int kBlk = 16;    // l-steps per block (4 groups of 4)
constexpr int kSuper = 8;   // blocks per flush of the first-level sums (64 terms per parity)

// B elements of a block: row j + 4t (even slot) and j + 4t + 1 (odd slot),
// plus 2 rows in the upper lane half; Bm is the m's uniform row base and lo
// the lane's offset (2 hi 32 + column).
__device__ __forceinline__ void load_b(const float *__restrict__ Bm, int j, unsigned lo,
                                       float (&b)[8])
{
    const float *__restrict__ Bj = Bm + (long long)j * 32;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        b[2 * t] = Bj[lo + 128 * t];
        b[2 * t + 1] = Bj[lo + 128 * t + 32];
    }
}

// One block of 16 l-steps j..j+15, all inside the m's range.
template <bool MASK>
__device__ __forceinline__ void block16(double x, double &ua, double &ub,
                                        const double *__restrict__ Aj, const float (&b)[8],
                                        bool live, MfmaTiles &acc)
{
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double u0 = fma(Aj[4 * t] * x, ub, -ua);
        const double u1 = fma(Aj[4 * t + 1] * x, u0, -ub);
        const double u2 = fma(Aj[4 * t + 2] * x, u1, -u0);
        const double u3 = fma(Aj[4 * t + 3] * x, u2, -u1);
        ua = u2;
        ub = u3;
        if (MASK)
            mfma4(opnd(u0, live), opnd(u1, live), opnd(u2, live), opnd(u3, live), b[2 * t],
                  b[2 * t + 1], acc);
        else
            mfma4((float)u0, (float)u1, (float)u2, (float)u3, b[2 * t], b[2 * t + 1], acc);
    }
}

// kSuper blocks from j with the B rows in registers one block ahead
// (alternating sets); on entry ba holds block 0's rows, on exit the rows of
// block jnext.  MASK: some lane still has k < 0.
template <bool MASK>
__device__ __forceinline__ void super_block(double x, double &ua, double &ub, int &k,
                                            const double *__restrict__ Am,
                                            const float *__restrict__ Bm, unsigned lo, int j,
                                            int jnext, float (&ba)[8], float (&bb)[8],
                                            MfmaTiles &acc)
{
#pragma unroll
    for (int q = 0; q < kSuper; ++q) {
        float(&cur)[8] = (q & 1) ? bb : ba;
        float(&nxt)[8] = (q & 1) ? ba : bb;
        load_b(Bm, (q + 1 < kSuper) ? j + kBlk * (q + 1) : jnext, lo, nxt);
        const bool live = !MASK || k == 0;
        block16<MASK>(x, ua, ub, Am + j + kBlk * q, cur, live, acc);
        if (MASK) rescale_mixed(ua, ub, k);
    }
}

__device__ __forceinline__ void add_tiles(MfmaTiles &tot, const MfmaTiles &acc)
{
    tot.e0 += acc.e0; tot.e1 += acc.e1; tot.o0 += acc.o0; tot.o1 += acc.o1;
}

__device__ void mfma_one_m(double x, double s, int m, int i, long long off, double mum,
                           int lmax, const double *__restrict__ A, const float *__restrict__ Bg,
                           double *__restrict__ delta, const PairDesc *__restrict__ pairs,
                           int npairs, int pb, int grp, int nmaps, int nrings, int nm)
{
    const int len = lmax - m + 1;
    const int lane = threadIdx.x;
    const int hi = lane >> 5;
    const int col = lane & 31;
    const double *__restrict__ Am = A + off;
    // row l of the m's B block: Bm[l * 32 + column]; a lane's K slot adds 2
    // rows in the upper half
    const float *__restrict__ Bm = Bg + off * 32;
    const unsigned lo = (unsigned)(2 * hi * 32 + col);

    double ua, ub;
    int k;
    seed_mm(mum, s, m, ua, k);
    ub = (len >= 2) ? (Am[1] * x) * ua : 0.0;

    MfmaTiles acc, tot;

    // ---- j = 0..3 (seeds), guarded; its sums start the second level
    {
        const bool live = (k == 0);
        const double A2 = (2 < len) ? Am[2] : 0.0;
        const double u2 = fma(A2 * x, ub, -ua);
        const double A3 = (3 < len) ? Am[3] : 0.0;
        const double u3 = fma(A3 * x, u2, -ub);
        const float X0 = opnd(ua, live);
        const float X1 = (len > 1) ? opnd(ub, live) : 0.0f;
        const float X2 = (2 < len) ? opnd(u2, live) : 0.0f;
        const float X3 = (3 < len) ? opnd(u3, live) : 0.0f;
        ua = u2; ub = u3;
        const float BE = (2 * hi < len) ? Bm[lo] : 0.0f;
        const float BO = (1 + 2 * hi < len) ? Bm[lo + 32] : 0.0f;
        tot.e0 = v16f{}; tot.e1 = v16f{}; tot.o0 = v16f{}; tot.o1 = v16f{};
        mfma4(X0, X1, X2, X3, BE, BO, tot);
    }
    acc.e0 = v16f{}; acc.e1 = v16f{}; acc.o0 = v16f{}; acc.o1 = v16f{};

    // ---- super-blocks of kSuper x kBlk steps; the first-level sums start
    // from zero in each and are added into tot at its end
    int j = 4;
    bool mask = wave_any(k < 0);
    float ba[8], bb[8];
    if (j + kSuper * kBlk <= len) {
        load_b(Bm, j, lo, ba);
        while (true) {
            const int jn = j + kSuper * kBlk;
            const bool more = jn + kSuper * kBlk <= len;
            // the prefetch after the last block stays inside the m's range
            const int jnext = more ? jn : j;
            if (mask) {
                super_block<true>(x, ua, ub, k, Am, Bm, lo, j, jnext, ba, bb, acc);
                mask = wave_any(k < 0);
            } else {
                super_block<false>(x, ua, ub, k, Am, Bm, lo, j, jnext, ba, bb, acc);
            }
            add_tiles(tot, acc);
            acc.e0 = v16f{}; acc.e1 = v16f{}; acc.o0 = v16f{}; acc.o1 = v16f{};
            j = jn;
            if (!more) break;
        }
    }

    // ---- remaining whole blocks (fewer than kSuper)
    if (j + kBlk <= len) {
        load_b(Bm, j, lo, ba);
        while (true) {
            const int jn = j + kBlk;
            const bool more = jn + kBlk <= len;
            load_b(Bm, more ? jn : j, lo, bb);
            const bool live = (k == 0);
            block16<true>(x, ua, ub, Am + j, ba, live, acc);
            rescale_mixed(ua, ub, k);
#pragma unroll
            for (int t = 0; t < 8; ++t) ba[t] = bb[t];
            j = jn;
            if (!more) break;
        }
    }

    // ---- tail, guarded
    for (; j < len; j += 4) {
        const bool live = (k == 0);
        const double A0 = Am[j];
        const double A1 = (j + 1 < len) ? Am[j + 1] : 0.0;
        const double A2 = (j + 2 < len) ? Am[j + 2] : 0.0;
        const double A3 = (j + 3 < len) ? Am[j + 3] : 0.0;
        const double u0 = fma(A0 * x, ub, -ua);
        const double u1 = fma(A1 * x, u0, -ub);
        const double u2 = fma(A2 * x, u1, -u0);
        const double u3 = fma(A3 * x, u2, -u1);
        const float X0 = opnd(u0, live);
        const float X1 = (j + 1 < len) ? opnd(u1, live) : 0.0f;
        const float X2 = (j + 2 < len) ? opnd(u2, live) : 0.0f;
        const float X3 = (j + 3 < len) ? opnd(u3, live) : 0.0f;
        ua = u2; ub = u3;
        rescale_mixed(ua, ub, k);
        const float BE = (j + 2 * hi < len) ? Bm[(long long)j * 32 + lo] : 0.0f;
        const float BO = (j + 1 + 2 * hi < len) ? Bm[(long long)j * 32 + lo + 32] : 0.0f;
        mfma4(X0, X1, X2, X3, BE, BO, acc);
    }
    add_tiles(tot, acc);

    // D layout of the 32x32 tile: column = lane % 32, row = 8 (r/4) + 4 (lane/32) + r % 4
    const int map = grp * 16 + (col >> 1);
    if (map >= nmaps) return;
    const int part = col & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const v16f &E = h ? tot.e1 : tot.e0;
        const v16f &O = h ? tot.o1 : tot.o0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * hi + (r & 3);
            const int pp = pb * 64 + h * 32 + row;
            if (pp < npairs) {
                const PairDesc d = pairs[pp];
                const double e = (double)E[r], o = (double)O[r];
                delta[(((long long)map * nrings + d.rn) * nm + i) * 2 + part] = e + o;
                if (d.rs >= 0)
                    delta[(((long long)map * nrings + d.rs) * nm + i) * 2 + part] = e - o;
            }
        }
    }
}

__global__ __launch_bounds__(64) void k_legendre_mfma_f32(
    const PairDesc *__restrict__ pairs, int npairs, int pblocks,
    const int *__restrict__ mval, const long long *__restrict__ moff,
    const double *__restrict__ mu, int nm, int nmpairs, int lmax,
    const double *__restrict__ A, const float *__restrict__ Bf, long long nalm,
    double *__restrict__ delta, int nrings, int nmaps, long long total)
{
    const long long L = xcd_logical(blockIdx.x, total);
    const int pb = (int)(L % pblocks);
    const long long rest = L / pblocks;
    const int q = (int)(rest % nmpairs);
    const int grp = (int)(rest / nmpairs);
    const int p = pb * 64 + threadIdx.x;
    double x = 0.0, s = 0.0;
    if (p < npairs) {
        const PairDesc d = pairs[p];
        x = d.x; s = d.s;
    }
    const float *Bg = Bf + (long long)grp * nalm * 32;
    for (int t = 0; t < 2; ++t) {
        const int i = (t == 0) ? q : nm - 1 - q;
        if (t == 1 && i == q) break;
        mfma_one_m(x, s, mval[i], i, moff[i], mu[i], lmax, A, Bg, delta, pairs, npairs, pb, grp,
                   nmaps, nrings, nm);
    }
}

}  // namespace

size_t mfma_bf_bytes(const sht_plan_s *p)
{
    const size_t groups = (size_t)((p->nmaps + 15) / 16);
    return groups * (size_t)p->nalm * 32 * sizeof(float);
}

hipError_t launch_prescale_f32(const sht_plan_s *p, const double *alm, float *Bf, hipStream_t st)
{
    const long long m0len = (p->mval[0] == 0) ? (p->lmax + 1) : 0;
    const int groups = (p->nmaps + 15) / 16;
    const long long n = p->nalm * 32;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)groups);
    hipLaunchKernelGGL(k_prescale_f32, grid, dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(alm), p->d_cn, Bf, p->nalm, p->nmaps,
                       m0len);
    return hipGetLastError();
}

hipError_t launch_legendre_mfma_f32(const sht_plan_s *p, const float *Bf, double2 *delta,
                                    hipStream_t st)
{
    const int pblocks = (p->npairs + 63) / 64;
    const int nmpairs = (p->nm + 1) / 2;
    const int groups = (p->nmaps + 15) / 16;
    const long long total = (long long)pblocks * nmpairs * groups;
    if (total <= 0 || total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_legendre_mfma_f32, dim3((unsigned)total), dim3(64), 0, st, p->d_pairs,
                       p->npairs, pblocks, p->d_mval, p->d_moff, p->d_mu, p->nm, nmpairs,
                       p->lmax, p->d_A, Bf, p->nalm, reinterpret_cast<double *>(delta),
                       p->nrings, p->nmaps, total);
    return hipGetLastError();
}

}  // namespace sht
