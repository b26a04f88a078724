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
// The fragment layouts of the two operands are mirror images, so passing the
// B fragment first yields the transposed tile C^T = B^T Lambda^T: each lane
// then owns one ring pair's values for 8 (map, Re/Im) pairs, and the Delta
// stores of a half-wave cover 32 consecutive rings.
//
// Work split.  A workgroup of four waves takes 256 ring pairs and an m-pair
// (m, mmax - m).  Per super-block of 128 l-rows the coefficients A_l (FP64)
// and the B rows (FP32, packed per 16-row block so that each lane reads its 8
// values as two 16-byte words) are copied once into LDS for all four waves
// (double-buffered, one barrier per super-block); while a wave computes block
// q of a super-block, block q of the next one is in flight from global memory
// to LDS, so the recurrence loop never waits on global memory.
//
// Accumulation.  FP32 accumulation over all l-terms loses up to ~1e-6; the
// matrix core accumulates the 64 same-parity terms of a super-block from zero
// and the block sums are added into a second FP32 accumulator (two-level
// summation).  Emulated error of Delta at l_max = 4096: about 1.2e-7 relative.
#include "mixed_common.h"

namespace sht {
namespace {

constexpr int kWaves = 4;                   // waves (64 ring pairs each) sharing an m
constexpr int kThreads = 64 * kWaves;
constexpr int kBlk = 16;                    // l-rows per block
constexpr int kBlkFloats = 64 * 8;          // packed block: [lane 64][slot 8]
constexpr int kSuper = 8;                   // blocks per super-block: 64 terms per parity
constexpr int kSuperRows = kSuper * kBlk;
constexpr int kABytes = kSuperRows * 8;     // A of a super-block in LDS
constexpr int kBufBytes = kABytes + kSuper * kBlkFloats * 4;

// Packed B: slot s = 2t + p of lane (hi, col) in block b of an m holds row
// 16 b + 4 t + 2 hi + p (p = 0: even slot, 1: odd slot) of column col, i.e.
// a'_lm = c_lm a_lm of map col / 2 (Re for even col, Im for odd), zero past
// the m's last row.  One workgroup per kPreBlocks consecutive blocks (bm16:
// the m of each block): the a_lm are read in runs of 16 rows per map (each
// complex value once), and the packed blocks are assembled in LDS and
// written out contiguously.
constexpr int kPreBlocks = 8;

__global__ __launch_bounds__(256) void k_prescale_f32(
    const double2 *__restrict__ alm, const double *__restrict__ cn,
    const long long *__restrict__ moff, const int *__restrict__ mval,
    const long long *__restrict__ boff16, const int *__restrict__ bm16, int lmax,
    long long nalm, long long nblocks, int nmaps, long long m0len, float *__restrict__ Bp)
{
    __shared__ __attribute__((aligned(16))) float stage[kPreBlocks * kBlkFloats];
    const long long blk0 = (long long)blockIdx.x * kPreBlocks;
    const int nb = (int)min((long long)kPreBlocks, nblocks - blk0);
    const int grp = blockIdx.y;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < kPreBlocks * 16 * 16 / 256; ++q) {
        const int idx = tid + 256 * q;
        const int b = idx >> 8, mp = (idx >> 4) & 15, rb = idx & 15;   // block, map, row
        if (b < nb) {
            const int i = bm16[blk0 + b];
            const int len = lmax - mval[i] + 1;
            const long long row = (blk0 + b - boff16[i]) * kBlk + rb;
            const int map = grp * 16 + mp;
            float vr = 0.0f, vi = 0.0f;
            if (row < len && map < nmaps) {
                const long long e = moff[i] + row;
                const double2 a = alm[(long long)map * nalm + e];
                const double c = cn[e];
                vr = (float)(a.x * c);
                vi = (float)((e < m0len) ? 0.0 : a.y * c);
            }
            // row rb = 4 t + 2 hi + p sits in slot 2 t + p of lane 32 hi + col
            const int slot = 2 * (rb >> 2) + (rb & 1);
            const int hi = (rb >> 1) & 1;
            float *s = stage + b * kBlkFloats + (hi * 32 + 2 * mp) * 8 + slot;
            s[0] = vr;
            s[8] = vi;
        }
    }
    __syncthreads();
    const float4 *s4 = reinterpret_cast<const float4 *>(stage);
    float4 *o4 = reinterpret_cast<float4 *>(Bp + ((long long)grp * nblocks + blk0) * kBlkFloats);
#pragma unroll
    for (int q = 0; q < kPreBlocks * kBlkFloats / 4 / 256; ++q) {
        const int w = tid + 256 * q;
        if (w < nb * (kBlkFloats / 4)) o4[w] = s4[w];
    }
}

// Four MFMAs of one group of 4 l-values: X0..X3 = P_l..P_{l+3} of the lane's
// ring pair; BE / BO = the lane's B elements of the even / odd rows.
__device__ __forceinline__ void mfma4(float X0, float X1, float X2, float X3, float BE, float BO,
                                      MfmaTiles &acc)
{
    float A0E, A1E, A0O, A1O;
    swap_halves(X0, X2, A0E, A1E);
    swap_halves(X1, X3, A0O, A1O);
    // B operand first: the tiles hold the transposed product, (map, Re/Im)
    // rows by ring-pair columns (see m_store)
    acc.e0 = __builtin_amdgcn_mfma_f32_32x32x2f32(BE, A0E, acc.e0, 0, 0, 0);
    acc.e1 = __builtin_amdgcn_mfma_f32_32x32x2f32(BE, A1E, acc.e1, 0, 0, 0);
    acc.o0 = __builtin_amdgcn_mfma_f32_32x32x2f32(BO, A0O, acc.o0, 0, 0, 0);
    acc.o1 = __builtin_amdgcn_mfma_f32_32x32x2f32(BO, A1O, acc.o1, 0, 0, 0);
}

// One block of 16 l-rows from LDS: Ab = its 16 coefficients, Bb = the lane's
// 8 packed B values.  SEED: the block holds rows 0..15 of the m, whose first
// group starts the recurrence from P_mm (ua) with P_{m+1,m} = A_1 x P_mm.
// Rows past the m's last one have A = 0 and B = 0 and contribute nothing.
template <bool MASK, bool SEED>
__device__ __forceinline__ void block16(double x, double &ua, double &ub,
                                        const double2 *__restrict__ Ab,
                                        const v4f *__restrict__ Bb, bool live, MfmaTiles &acc)
{
    const v4f b03 = Bb[0], b47 = Bb[1];
    const float b[8] = {b03.x, b03.y, b03.z, b03.w, b47.x, b47.y, b47.z, b47.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double2 a01 = Ab[2 * t], a23 = Ab[2 * t + 1];
        double u0, u1;
        if (SEED && t == 0) {
            u0 = ua;
            u1 = (a01.y * x) * ua;
            ub = u1;
        } else {
            u0 = fma(a01.x * x, ub, -ua);
            u1 = fma(a01.y * x, u0, -ub);
        }
        const double u2 = fma(a23.x * x, u1, -u0);
        const double u3 = fma(a23.y * x, u2, -u1);
        ua = u2;
        ub = u3;
        if (MASK)
            mfma4(opnd(u0, live), opnd(u1, live), opnd(u2, live), opnd(u3, live), b[2 * t],
                  b[2 * t + 1], acc);
        else
            mfma4((float)u0, (float)u1, (float)u2, (float)u3, b[2 * t], b[2 * t + 1], acc);
    }
}

// A block in which no lane of the wave has reached k = 0: every matrix
// operand would be 0, so only the recurrence runs (same arithmetic, so the
// state entering the next block is bitwise that of block16).
template <bool SEED>
__device__ __forceinline__ void block16_dead(double x, double &ua, double &ub,
                                             const double2 *__restrict__ Ab)
{
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double2 a01 = Ab[2 * t], a23 = Ab[2 * t + 1];
        double u0, u1;
        if (SEED && t == 0) {
            u0 = ua;
            u1 = (a01.y * x) * ua;
        } else {
            u0 = fma(a01.x * x, ub, -ua);
            u1 = fma(a01.y * x, u0, -ub);
        }
        const double u2 = fma(a23.x * x, u1, -u0);
        const double u3 = fma(a23.y * x, u2, -u1);
        ua = u2;
        ub = u3;
    }
}

// Copy of super-block sb of an m (its 8 packed B blocks and 128
// coefficients) into LDS buffer `buf`, straight from global memory to LDS
// (no registers); it completes at the workgroup's next barrier.  Every lane
// takes part (the LDS slot of a lane follows its position in the wave): past
// the m's last block or row the copy reads neighbouring data or the padding
// after the tables (128 coefficients, one super-block of B), which only
// lands in rows that are never used or are multiplied by B = 0.
__device__ __forceinline__ void super_dma(char *buf, const float *__restrict__ Bm,
                                          const double *__restrict__ Am, int sb, int tid)
{
    const float *src = Bm + (long long)sb * kSuper * kBlkFloats;
    float *dst = reinterpret_cast<float *>(buf + kABytes);
#pragma unroll
    for (int c = 0; c < kSuper * kBlkFloats / 4 / kThreads; ++c) {
        const int w = tid + kThreads * c;
        __builtin_amdgcn_global_load_lds(src + 4 * w, dst + 4 * w, 16, 0, 0);
    }
    const unsigned *asrc = reinterpret_cast<const unsigned *>(Am + (long long)sb * kSuperRows);
    __builtin_amdgcn_global_load_lds(asrc + tid, reinterpret_cast<unsigned *>(buf) + tid, 4, 0, 0);
}

// The blocks of super-block sb, held in LDS buffer `cur`, while super-block
// sb + 1 is copied into `nxt` (when `more`); the first-level sums start from
// zero and are added into tot at the end.
template <bool MASK>
__device__ __forceinline__ void super_compute(double x, double &ua, double &ub, int &k,
                                              const char *cur, char *nxt, bool more, int sb,
                                              int nb, bool seed, const float *__restrict__ Bm,
                                              const double *__restrict__ Am, int tid,
                                              MfmaTiles &acc, MfmaTiles &tot)
{
    const int lane = tid & 63;
    const double2 *As = reinterpret_cast<const double2 *>(cur);
    const v4f *Bs = reinterpret_cast<const v4f *>(cur + kABytes) + lane * 2;
    zero_tiles(acc);
    if (more) super_dma(nxt, Bm, Am, sb + 1, tid);
    if (seed) {
        if (wave_any(k == 0))
            block16<true, true>(x, ua, ub, As, Bs, k == 0, acc);
        else
            block16_dead<true>(x, ua, ub, As);
    } else if (!MASK || wave_any(k == 0)) {
        block16<MASK, false>(x, ua, ub, As, Bs, !MASK || k == 0, acc);
    } else {
        block16_dead<false>(x, ua, ub, As);
    }
    if (MASK || seed) rescale_mixed(ua, ub, k);
    for (int q = 1; q < nb; ++q) {
        if (!MASK || wave_any(k == 0))
            block16<MASK, false>(x, ua, ub, As + (kBlk / 2) * q, Bs + (kBlkFloats / 4) * q,
                                 !MASK || k == 0, acc);
        else
            block16_dead<false>(x, ua, ub, As + (kBlk / 2) * q);
        if (MASK) rescale_mixed(ua, ub, k);
    }
    add_tiles(tot, acc);
}

// A thread's share of a whole super-block copy (the first live one of an m):
// 64 bytes of packed B and one dword of the coefficients.
struct SuperStage {
    v4f b[kSuper * kBlkFloats / 4 / kThreads];
    unsigned a;
};

__device__ __forceinline__ void super_stage_load(SuperStage &g, const float *__restrict__ Bm,
                                                 int nblk, const double *__restrict__ Am,
                                                 int len, int sb, int tid)
{
    const int b0 = sb * kSuper;
    const int nw = min(kSuper, nblk - b0) * (kBlkFloats / 4);  // 16-byte words present
    const v4f *__restrict__ src = reinterpret_cast<const v4f *>(Bm + (long long)b0 * kBlkFloats);
#pragma unroll
    for (int c = 0; c < kSuper * kBlkFloats / 4 / kThreads; ++c) {
        const int w = tid + kThreads * c;
        g.b[c] = (w < nw) ? src[w] : v4f{};
    }
    const int r = sb * kSuperRows + (tid >> 1);  // dword tid of the 128 coefficients
    g.a = (r < len) ? reinterpret_cast<const unsigned *>(Am + r)[tid & 1] : 0u;
}

__device__ __forceinline__ void super_stage_store(const SuperStage &g, char *buf, int tid)
{
    v4f *B = reinterpret_cast<v4f *>(buf + kABytes);
#pragma unroll
    for (int c = 0; c < kSuper * kBlkFloats / 4 / kThreads; ++c) B[tid + kThreads * c] = g.b[c];
    reinterpret_cast<unsigned *>(buf)[tid] = g.a;
}

// One m of the workgroup's 4 x 64 ring pairs.
struct MState {
    int m, i, len, nblk, nsb, sb0;
    const double *Am;
    const float *Bm;
    double ua, ub;
    int k;
};

// Seed and phase 1: while no lane of the workgroup has reached k = 0, every
// matrix operand is 0 (Q15), so the workgroup runs the recurrence alone, one
// super-block at a time, with no staging.  Then the copy of the first live
// super-block is issued into registers (committed to LDS by m_commit).
__device__ void m_begin(MState &st, SuperStage &g, int i, const int *__restrict__ mval,
                        const long long *__restrict__ soff, const long long *__restrict__ boff16,
                        const double *__restrict__ mu, int lmax, const double *__restrict__ Asb,
                        const float *__restrict__ Bg, double x, double s, int tid)
{
    st.i = i;
    st.m = mval[i];
    st.len = lmax - st.m + 1;
    st.nblk = (st.len + kBlk - 1) / kBlk;
    st.nsb = (st.nblk + kSuper - 1) / kSuper;
    // coefficients from the per-super-block copy, zero past the m's last row:
    // the copies of a super-block run past the m's end, and with A = 0 there
    // the recurrence of the unused rows stays bounded (u_l = -u_{l-2})
    st.Am = Asb + soff[i] * kSuperRows;
    st.Bm = Bg + boff16[i] * kBlkFloats;
    st.ub = 0.0;
    seed_mm(mu[i], s, st.m, st.ua, st.k);
    // k = 0 only above 2^-400, also for the seed (kept exact: a power of two)
    if (st.k == 0 && fabs(st.ua) < kEmergeTrue) {
        st.ua *= kTwoS;
        st.k = -1;
    }
    int sb0 = 0;
    while (sb0 < st.nsb && !__syncthreads_or(st.k == 0)) {
        const int nb = min(kSuper, st.nblk - sb0 * kSuper);
        for (int q = 0; q < nb; ++q) {
            const int r0 = (sb0 * kSuper + q) * kBlk;
            if (r0 == 0)
                block16_dead_g<true>(x, st.ua, st.ub, st.Am, r0);
            else
                block16_dead_g<false>(x, st.ua, st.ub, st.Am, r0);
            rescale_mixed(st.ua, st.ub, st.k);
        }
        ++sb0;
    }
    st.sb0 = sb0;
    if (sb0 < st.nsb) super_stage_load(g, st.Bm, st.nblk, st.Am, st.len, sb0, tid);
}

// The first live super-block goes to buffer A; the following ones alternate.
__device__ __forceinline__ void m_commit(const MState &st, const SuperStage &g, char *ldsA,
                                         int tid)
{
    if (st.sb0 < st.nsb) super_stage_store(g, ldsA, tid);
    __syncthreads();
}

// One super-block of phase 2 (then the barrier that also completes the copy
// of the next one).
__device__ __forceinline__ void m_step(MState &st, int sb, const char *cur, char *nxt, double x,
                                       int tid, bool &mask, MfmaTiles &acc, MfmaTiles &tot)
{
    const bool more = sb + 1 < st.nsb;
    const int nb = min(kSuper, st.nblk - sb * kSuper);
    if (mask) {
        super_compute<true>(x, st.ua, st.ub, st.k, cur, nxt, more, sb, nb, sb == 0, st.Bm,
                            st.Am, tid, acc, tot);
        mask = wave_any(st.k < 0);
    } else {
        super_compute<false>(x, st.ua, st.ub, st.k, cur, nxt, more, sb, nb, false, st.Bm,
                             st.Am, tid, acc, tot);
    }
    __syncthreads();
}

// Phase 2: the live super-blocks on the matrix cores; the second-level sums
// end in tot.  The two LDS buffers are distinct objects and the loop takes
// them in a fixed order, so the compiler sees that the reads of one never
// wait for the copy into the other.
__device__ __forceinline__ void m_compute(MState &st, char *ldsA, char *ldsB, double x, int tid, MfmaTiles &tot)
{
    MfmaTiles acc;
    zero_tiles(tot);
    bool mask = true;  // the first live super-block runs masked
    for (int sb = st.sb0; sb < st.nsb; sb += 2) {
        m_step(st, sb, ldsA, ldsB, x, tid, mask, acc, tot);
        if (sb + 1 < st.nsb) m_step(st, sb + 1, ldsB, ldsA, x, tid, mask, acc, tot);
    }
}

__global__ __launch_bounds__(kThreads, 2) void k_legendre_mfma_f32(
    const PairDesc *__restrict__ pairs, int npairs, int pgroups,
    const int *__restrict__ mval, const long long *__restrict__ soff,
    const long long *__restrict__ boff16, const double *__restrict__ mu, int nm, int nmpairs,
    int lmax, const double *__restrict__ Asb, const float *__restrict__ Bp, long long nblocks,
    float2 *__restrict__ delta, int nrings, int nmaps, long long total)
{
    __shared__ __attribute__((aligned(16))) char ldsA[kBufBytes];
    __shared__ __attribute__((aligned(16))) char ldsB[kBufBytes];
    const long long L = xcd_logical(blockIdx.x, total);
    const int pg = (int)(L % pgroups);
    const long long rest = L / pgroups;
    const int q = (int)(rest % nmpairs);
    const int grp = (int)(rest / nmpairs);
    const int tid = threadIdx.x;
    const int pb = pg * kWaves + (tid >> 6);
    const int p = pb * 64 + (tid & 63);
    double x = 0.0, s = 0.0;
    if (p < npairs) {
        const PairDesc d = pairs[p];
        x = d.x; s = d.s;
    }
    const float *Bg = Bp + (long long)grp * nblocks * kBlkFloats;
    // Both m of the pair are run by every thread of the workgroup, so the
    // barrier count stays uniform.  The second m's recurrence prefix and
    // first copy are issued before the first m's Delta stores, so that its
    // wait for the copy does not also wait for those stores.
    MState st;
    SuperStage g;
    MfmaTiles tot;
    m_begin(st, g, q, mval, soff, boff16, mu, lmax, Asb, Bg, x, s, tid);
    m_commit(st, g, ldsA, tid);
    m_compute(st, ldsA, ldsB, x, tid, tot);
    const int i1 = st.i;
    const int i2 = nm - 1 - q;
    const bool two = i2 != q;
    if (two) m_begin(st, g, i2, mval, soff, boff16, mu, lmax, Asb, Bg, x, s, tid);
    m_store(tot, i1, delta, pairs, npairs, pb, grp, nmaps, nrings, nm, tid & 63);
    if (two) {
        m_commit(st, g, ldsA, tid);
        m_compute(st, ldsA, ldsB, x, tid, tot);
        m_store(tot, st.i, delta, pairs, npairs, pb, grp, nmaps, nrings, nm, tid & 63);
    }
}

}  // namespace

size_t mfma_bf_bytes(const sht_plan_s *p)
{
    const size_t groups = (size_t)((p->nmaps + 15) / 16);
    // plus one super-block: the copies of an m's last super-block may read past it
    return (groups * (size_t)p->nblk16 + kSuper) * kBlkFloats * sizeof(float);
}

hipError_t launch_prescale_f32(const sht_plan_s *p, const double *alm, float *Bp, hipStream_t st)
{
    const long long m0len = (p->mval[0] == 0) ? (p->lmax + 1) : 0;
    const int groups = (p->nmaps + 15) / 16;
    if (p->nblk16 <= 0 || p->nblk16 > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)((p->nblk16 + kPreBlocks - 1) / kPreBlocks), (unsigned)groups);
    hipLaunchKernelGGL(k_prescale_f32, grid, dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(alm), p->d_cn, p->d_moff, p->d_mval,
                       p->d_boff16, p->d_bm16, p->lmax, p->nalm, p->nblk16, p->nmaps, m0len, Bp);
    return hipGetLastError();
}

hipError_t launch_legendre_mfma_f32(const sht_plan_s *p, const float *Bp, float2 *delta,
                                    hipStream_t st)
{
    const int pblocks = (p->npairs + 63) / 64;
    const int pgroups = (pblocks + kWaves - 1) / kWaves;
    const int nmpairs = (p->nm + 1) / 2;
    const int groups = (p->nmaps + 15) / 16;
    const long long total = (long long)pgroups * nmpairs * groups;
    // the plan's zero-padded coefficient copy has the super-block length of this kernel
    if (f16_super_rows() != kSuperRows) return hipErrorInvalidConfiguration;
    if (total <= 0 || total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_legendre_mfma_f32, dim3((unsigned)total), dim3(kThreads), 0, st,
                       p->d_pairs, p->npairs, pgroups, p->d_mval, p->d_soff, p->d_boff16,
                       p->d_mu, p->nm, nmpairs, p->lmax, p->d_Asb, Bp, p->nblk16,
                       delta, p->nrings, p->nmaps, total);
    return hipGetLastError();
}

}  // namespace sht
