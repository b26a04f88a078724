// Mixed-precision batched Legendre stage with 3-way split BF16 inputs on
// the matrix cores (gfx950, v_mfma_f32_32x32x16_bf16).
//
// Same contraction as the FP32 form (per m, C_E/O[pairs x 32] =
// Lambda_E/O[pairs x K] B_E/O[K x 32], Delta_N = C_E + C_O, Delta_S = C_E - C_O)
// with every FP32 operand x written as x = x_h + x_m + x_l, three BF16 parts
// (8 + 8 + 8 significant bits), and the product taken as the six terms
// A_h B_h + A_h B_m + A_m B_h + A_h B_l + A_m B_m + A_l B_h; the dropped
// terms are below 2^-24 relative.  Accumulation is two-level FP32 as in the
// FP32 form.  The recurrence stays FP64 on the vector units.
//
// Fragments.  A 32x32x16 A-fragment holds, in lanes 0-31, K = 0..7 of rows
// 0-31 and, in lanes 32-63, K = 8..15 of the same rows.  A lane runs 32 steps
// of its own ring pair: the 16 even-parity values give X (K 0-7) and Y
// (K 8-15); v_permlane32_swap of each dword of (X, Y) gives the fragments of
// both row halves, exactly as in the FP32 form.  The B operands are packed by
// the prescale kernel so that each lane reads its 8 K-values as 16 bytes.
#include "recurrence.h"
#include "sht_internal.h"

namespace sht {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

constexpr int kBlkSteps = 32;       // l-steps per block (16 per parity = one K of 16)
constexpr int kFlushBlocks = 4;     // FP32 block sums of 64 same-parity terms

// Packed B layout per m block: [parity 2][level 3][half 2][column 32] x 8 bf16.
constexpr int kBlkElems = 2 * 3 * 2 * 32;  // 16-byte elements per block

__device__ inline void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l)
{
    h = (__bf16)x;
    const float r1 = x - (float)h;
    m = (__bf16)r1;
    const float r2 = r1 - (float)m;
    l = (__bf16)r2;
}

// a'_lm = c_lm a_lm of up to 16 maps, split and packed per 32-step block.
__global__ void k_prescale_bf16x3(const double2 *__restrict__ alm, const double *__restrict__ cn,
                                  const long long *__restrict__ moff,
                                  const int *__restrict__ mval, const long long *__restrict__ boff,
                                  int nm, int lmax, long long nalm, long long nblocks,
                                  int nmaps, long long m0len, v4u *__restrict__ Bb)
{
    // one thread per (block, parity, half, column): writes 3 x 16 bytes
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = blockIdx.y;
    if (t >= nblocks * 128) return;
    const long long blk = t >> 7;
    const int col = (int)(t & 31);
    const int half = (int)((t >> 5) & 1);
    const int par = (int)((t >> 6) & 1);
    // find the m of this block (binary search over boff)
    int lo = 0, hi = nm - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    const int i = lo;
    const int len = lmax - mval[i] + 1;
    const long long b = blk - boff[i];
    const int map = grp * 16 + (col >> 1);
    v8bf H, M, L;
#pragma unroll
    for (int jp = 0; jp < 8; ++jp) {
        const long long j = 32 * b + 2 * (8 * half + jp) + par;
        float x = 0.0f;
        if (j < len && map < nmaps) {
            const long long e = moff[i] + j;
            const double2 a = alm[(long long)map * nalm + e];
            const double c = cn[e];
            x = (float)((col & 1) ? ((e < m0len) ? 0.0 : a.y * c) : a.x * c);
        }
        __bf16 h, m, l;
        split3(x, h, m, l);
        H[jp] = h; M[jp] = m; L[jp] = l;
    }
    v4u *dst = Bb + ((long long)grp * nblocks + blk) * kBlkElems;
    dst[((par * 3 + 0) * 2 + half) * 32 + col] = __builtin_bit_cast(v4u, H);
    dst[((par * 3 + 1) * 2 + half) * 32 + col] = __builtin_bit_cast(v4u, M);
    dst[((par * 3 + 2) * 2 + half) * 32 + col] = __builtin_bit_cast(v4u, L);
}

__device__ inline void swap8(const v8bf &X, const v8bf &Y, v8bf &A0, v8bf &A1)
{
    const v4u x = __builtin_bit_cast(v4u, X);
    const v4u y = __builtin_bit_cast(v4u, Y);
    v4u a0, a1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const v2u r = __builtin_amdgcn_permlane32_swap(x[k], y[k], false, false);
        a0[k] = r[0];
        a1[k] = r[1];
    }
    A0 = __builtin_bit_cast(v8bf, a0);
    A1 = __builtin_bit_cast(v8bf, a1);
}

struct Tiles {
    v16f e0, e1, o0, o1;
};

// 16 same-parity values (FP32) of this lane -> split fragments for both row
// halves, then the six products against the B parts of that parity.
__device__ inline void parity_mfma(const float (&v)[16], const v8bf (&B)[3], v16f &acc0,
                                   v16f &acc1)
{
    v8bf Xh, Xm, Xl, Yh, Ym, Yl;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        __bf16 h, m, l;
        split3(v[t], h, m, l);
        Xh[t] = h; Xm[t] = m; Xl[t] = l;
        split3(v[t + 8], h, m, l);
        Yh[t] = h; Ym[t] = m; Yl[t] = l;
    }
    v8bf A0h, A1h, A0m, A1m, A0l, A1l;
    swap8(Xh, Yh, A0h, A1h);
    swap8(Xm, Ym, A0m, A1m);
    swap8(Xl, Yl, A0l, A1l);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[0], A0h, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[0], A1h, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[1], A0h, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[1], A1h, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[0], A0m, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[0], A1m, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[2], A0h, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[2], A1h, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[1], A0m, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[1], A1m, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[0], A0l, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B[0], A1l, acc1, 0, 0, 0);
}

// tot[0..15] += e0, [16..31] += e1, [32..47] += o0, [48..63] += o1 (per lane)
__device__ inline void flush_tot(const Tiles &acc, float *tot, int lane)
{
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        tot[(r)*64 + lane] += acc.e0[r];
        tot[(16 + r) * 64 + lane] += acc.e1[r];
        tot[(32 + r) * 64 + lane] += acc.o0[r];
        tot[(48 + r) * 64 + lane] += acc.o1[r];
    }
}

__device__ inline void load_b(const v4u *__restrict__ Bblk, int hi, int col, v8bf (&BE)[3],
                              v8bf (&BO)[3])
{
#pragma unroll
    for (int lev = 0; lev < 3; ++lev) {
        BE[lev] = __builtin_bit_cast(v8bf, Bblk[((0 * 3 + lev) * 2 + hi) * 32 + col]);
        BO[lev] = __builtin_bit_cast(v8bf, Bblk[((1 * 3 + lev) * 2 + hi) * 32 + col]);
    }
}

__device__ void bf16_one_m(float *tot, double x, double s, int m, int i, long long off,
                           long long boffi, double mum, int lmax, const double *__restrict__ A,
                           const v4u *__restrict__ Bg, double *__restrict__ delta,
                           const PairDesc *__restrict__ pairs, int npairs, int pb, int grp,
                           int nmaps, int nrings, int nm)
{
    const int len = lmax - m + 1;
    const int lane = threadIdx.x;
    const int hi = lane >> 5;
    const int col = lane & 31;
    const double *__restrict__ Am = A + off;
    const v4u *__restrict__ Bm = Bg + boffi * kBlkElems;
    const int nblk = (len + kBlkSteps - 1) / kBlkSteps;

    double ua, ub;
    int k;
    seed_mm(mum, s, m, ua, k);
    double f = final_scale(k);
    ub = (Am[len > 1 ? 1 : 0] * x) * ua;   // unused when len == 1 (B rows are zero)

    Tiles acc;
    acc.e0 = v16f{}; acc.e1 = v16f{}; acc.o0 = v16f{}; acc.o1 = v16f{};
    // second-level FP32 sums live in LDS (64 values per lane, lane-minor so
    // that a wave's accesses hit consecutive banks)
#pragma unroll
    for (int r = 0; r < 64; ++r) tot[r * 64 + lane] = 0.0f;
    v8bf BE[3], BO[3], NE[3], NO[3];
    load_b(Bm, hi, col, BE, BO);
    for (int b = 0; b < nblk; ++b) {
        const int j0 = b * kBlkSteps;
        const bool more = b + 1 < nblk;
        load_b(Bm + (long long)(more ? b + 1 : b) * kBlkElems, hi, col, NE, NO);
        float e[16], o[16];
#pragma unroll
        for (int t = 0; t < kBlkSteps; ++t) {
            double u;
            if (t < 2 && b == 0) {
                u = (t == 0) ? ua : ub;
            } else {
                // beyond the m's range the coefficient is clamped to a valid
                // entry; the matching B rows are zero
                const int j = min(j0 + t, len - 1);
                const double Aj = Am[j];
                u = fma(Aj * x, ub, -ua);
                ua = ub;
                ub = u;
            }
            const float v = (float)(u * f);
            if (t & 1) o[t >> 1] = v; else e[t >> 1] = v;
            if ((t & 7) == 7 && !(b == 0 && t < 2)) {
                if (fmax(fabs(ua), fabs(ub)) > kTwoS) {
                    ua *= kTwoMinusS; ub *= kTwoMinusS;
                    k += 1;
                    f = final_scale(k);
                }
            }
        }
        parity_mfma(e, BE, acc.e0, acc.e1);
        parity_mfma(o, BO, acc.o0, acc.o1);
        if ((b + 1) % kFlushBlocks == 0) {
            flush_tot(acc, tot, lane);
            acc.e0 = v16f{}; acc.e1 = v16f{}; acc.o0 = v16f{}; acc.o1 = v16f{};
        }
#pragma unroll
        for (int lev = 0; lev < 3; ++lev) { BE[lev] = NE[lev]; BO[lev] = NO[lev]; }
    }
    flush_tot(acc, tot, lane);

    // The tiles hold the transposed product (B operand first): column =
    // lane % 32 is the ring pair, row = 8 (r/4) + 4 (lane/32) + r % 4 is
    // (map, Re/Im), so each lane owns 8 complex values of one pair and a
    // half-wave stores 32 consecutive rings of Delta [map][m][ring].
    double2 *__restrict__ d2 = reinterpret_cast<double2 *>(delta);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int pp = pb * 64 + h * 32 + col;
        if (pp < npairs) {
            const PairDesc d = pairs[pp];
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
                const int map = grp * 16 + 4 * (r >> 2) + 2 * hi + ((r & 3) >> 1);
                if (map < nmaps) {
                    const double er = tot[((h ? 16 : 0) + r) * 64 + lane];
                    const double ei = tot[((h ? 16 : 0) + r + 1) * 64 + lane];
                    const double orr = tot[((h ? 48 : 32) + r) * 64 + lane];
                    const double oi = tot[((h ? 48 : 32) + r + 1) * 64 + lane];
                    d2[((long long)map * nm + i) * nrings + d.rn] = make_double2(er + orr, ei + oi);
                    if (d.rs >= 0)
                        d2[((long long)map * nm + i) * nrings + d.rs] =
                            make_double2(er - orr, ei - oi);
                }
            }
        }
    }
}

__global__ __launch_bounds__(64, 2) void k_legendre_mfma_bf16x3(
    const PairDesc *__restrict__ pairs, int npairs, int pblocks,
    const int *__restrict__ mval, const long long *__restrict__ moff,
    const long long *__restrict__ boff, const double *__restrict__ mu, int nm, int nmpairs,
    int lmax, const double *__restrict__ A, const v4u *__restrict__ Bb, long long nblocks,
    double *__restrict__ delta, int nrings, int nmaps, long long total)
{
    __shared__ float tot[64 * 64];
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
    const v4u *Bg = Bb + (long long)grp * nblocks * kBlkElems;
    for (int t = 0; t < 2; ++t) {
        const int i = (t == 0) ? q : nm - 1 - q;
        if (t == 1 && i == q) break;
        bf16_one_m(tot, x, s, mval[i], i, moff[i], boff[i], mu[i], lmax, A, Bg, delta, pairs,
                   npairs, pb, grp, nmaps, nrings, nm);
    }
}

}  // namespace

long long bf16_blocks(const sht_plan_s *p)
{
    long long nb = 0;
    for (int i = 0; i < p->nm; ++i) nb += (p->lmax - p->mval[i] + 1 + kBlkSteps - 1) / kBlkSteps;
    return nb;
}

size_t bf16_bytes(const sht_plan_s *p)
{
    const size_t groups = (size_t)((p->nmaps + 15) / 16);
    return groups * (size_t)bf16_blocks(p) * kBlkElems * 16;
}

hipError_t launch_prescale_bf16x3(const sht_plan_s *p, const double *alm, void *Bb,
                                  hipStream_t st)
{
    const long long m0len = (p->mval[0] == 0) ? (p->lmax + 1) : 0;
    const int groups = (p->nmaps + 15) / 16;
    const long long nblocks = bf16_blocks(p);
    const long long n = nblocks * 128;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)groups);
    hipLaunchKernelGGL(k_prescale_bf16x3, grid, dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(alm), p->d_cn, p->d_moff, p->d_mval,
                       p->d_boff, p->nm, p->lmax, p->nalm, nblocks, p->nmaps, m0len,
                       reinterpret_cast<v4u *>(Bb));
    return hipGetLastError();
}

hipError_t launch_legendre_mfma_bf16x3(const sht_plan_s *p, const void *Bb, double2 *delta,
                                       hipStream_t st)
{
    const int pblocks = (p->npairs + 63) / 64;
    const int nmpairs = (p->nm + 1) / 2;
    const int groups = (p->nmaps + 15) / 16;
    const long long total = (long long)pblocks * nmpairs * groups;
    if (total <= 0 || total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_legendre_mfma_bf16x3, dim3((unsigned)total), dim3(64), 0, st, p->d_pairs,
                       p->npairs, pblocks, p->d_mval, p->d_moff, p->d_boff, p->d_mu, p->nm,
                       nmpairs, p->lmax, p->d_A, reinterpret_cast<const v4u *>(Bb),
                       bf16_blocks(p), reinterpret_cast<double *>(delta), p->nrings, p->nmaps,
                       total);
    return hipGetLastError();
}

}  // namespace sht
