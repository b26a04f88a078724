// Mixed-precision batched Legendre stage with 3-way split BF16 inputs on
// the matrix cores (gfx950, v_mfma_f32_32x32x16_bf16).
//
// Same contraction as the FP32 form (per m, C_E/O = B_E/O^T Lambda_E/O^T,
// Delta_N = C_E + C_O, Delta_S = C_E - C_O) with every FP32 operand x written
// as x = x_h + x_m + x_l, three BF16 parts, and the product taken as the six
// terms A_h B_h + A_h B_m + A_m B_h + A_h B_l + A_m B_m + A_l B_h; the dropped
// terms are below 2^-23 relative.  The coefficients are split by rounding
// (prescale); the P_lm by truncation, which is exact in FP32 arithmetic:
// x_h = x with the low 16 bits cleared, r = x - x_h (exact), x_m = r with the
// low 16 bits cleared, x_l = r - x_m (exact, at most 8 significant bits), so
// each part is the high half of an FP32 word and two parts pack into one
// dword with one byte permute.  Accumulation is two-level FP32 as in the FP32
// form (64 same-parity terms per first-level block).  The recurrence stays
// FP64 on the vector units.
//
// Fragments.  A 32x32x16 fragment holds, in lanes 0-31, K = 0..7 of its 32
// columns and, in lanes 32-63, K = 8..15.  A lane runs 32 steps of its own
// ring pair; its 16 values of one parity are exchanged across the wave
// halves as FP32 (one v_permlane32_swap per pair of values) and then split,
// which gives the fragments of both column halves.  The coefficient
// fragment is passed first, so the tiles hold the transposed product as in
// the FP32 form, and the same epilogue stores Delta.
//
// Work split.  As in the FP32 form: a workgroup of four waves takes 256 ring
// pairs and an m-pair; per super-block of 128 l-rows (4 blocks of 32) the
// coefficients A_l and the packed B blocks are copied global-to-LDS while the
// previous super-block is multiplied; a workgroup runs the recurrence alone
// while all its lanes are below 2^-400, then a masked path for its first live
// super-block, then a path with no mask and no rescaling.
#include "mixed_common.h"

namespace sht {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;                   // waves (64 ring pairs each) sharing an m
constexpr int kThreads = 64 * kWaves;
constexpr int kBlkSteps = 32;               // l-rows per block (K = 16 per parity)
// Packed B layout per m block: [parity 2][level 3][half 2][column 32] x 8 bf16.
constexpr int kBlkElems = 2 * 3 * 2 * 32;   // 16-byte elements per block
constexpr int kSuper = 4;                   // blocks per super-block: 64 terms per parity
constexpr int kSuperRows = kSuper * kBlkSteps;
constexpr int kABytes = kSuperRows * 8;     // A of a super-block in LDS
constexpr int kBufBytes = kABytes + kSuper * kBlkElems * 16;

__device__ inline void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l)
{
    h = (__bf16)x;
    const float r1 = x - (float)h;
    m = (__bf16)r1;
    const float r2 = r1 - (float)m;
    l = (__bf16)r2;
}

// a'_lm = c_lm a_lm of up to 16 maps, split and packed per 32-step block.
// One workgroup per kPreBlocks consecutive blocks (bm32: the m of each
// block): the a_lm are read in runs of 32 rows per map (each complex value
// once), split, placed into the packed blocks in LDS, and the blocks are
// written out contiguously.
constexpr int kPreBlocks = 4;

__global__ __launch_bounds__(256) void k_prescale_bf16x3(
    const double2 *__restrict__ alm, const double *__restrict__ cn,
    const long long *__restrict__ moff, const int *__restrict__ mval,
    const long long *__restrict__ boff, const int *__restrict__ bm32, int lmax, long long nalm,
    long long nblocks, int nmaps, long long m0len, v4u *__restrict__ Bb)
{
    __shared__ __attribute__((aligned(16))) __bf16 stage[kPreBlocks * kBlkElems * 8];
    const long long blk0 = (long long)blockIdx.x * kPreBlocks;
    const int nb = (int)min((long long)kPreBlocks, nblocks - blk0);
    const int grp = blockIdx.y;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < kPreBlocks * kBlkSteps * 16 / 256; ++q) {
        const int idx = tid + 256 * q;
        const int b = idx >> 9, mp = (idx >> 5) & 15, rb = idx & 31;   // block, map, row
        if (b < nb) {
            const int i = bm32[blk0 + b];
            const int len = lmax - mval[i] + 1;
            const long long row = (blk0 + b - boff[i]) * kBlkSteps + rb;
            const int map = grp * 16 + mp;
            float xr = 0.0f, xi = 0.0f;
            if (row < len && map < nmaps) {
                const long long e = moff[i] + row;
                const double2 a = alm[(long long)map * nalm + e];
                const double c = cn[e];
                xr = (float)(a.x * c);
                xi = (float)((e < m0len) ? 0.0 : a.y * c);
            }
            // row rb = 2 K + parity; K = 8 half + slot
            const int par = rb & 1, kk = rb >> 1, half = kk >> 3, slot = kk & 7;
            __bf16 h, m, l;
            __bf16 *s = stage + b * kBlkElems * 8;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                split3(c ? xi : xr, h, m, l);
                const int col = 2 * mp + c;
                s[(((par * 3 + 0) * 2 + half) * 32 + col) * 8 + slot] = h;
                s[(((par * 3 + 1) * 2 + half) * 32 + col) * 8 + slot] = m;
                s[(((par * 3 + 2) * 2 + half) * 32 + col) * 8 + slot] = l;
            }
        }
    }
    __syncthreads();
    const v4u *s4 = reinterpret_cast<const v4u *>(stage);
    v4u *o4 = Bb + ((long long)grp * nblocks + blk0) * kBlkElems;
#pragma unroll
    for (int q = 0; q < kPreBlocks * kBlkElems / 256; ++q) {
        const int w = tid + 256 * q;
        if (w < nb * kBlkElems) o4[w] = s4[w];
    }
}

// High halves of two FP32 words: (a >> 16) | (b & 0xffff0000).
__device__ inline unsigned pack_hi(unsigned a, unsigned b)
{
    return __builtin_amdgcn_perm(b, a, 0x07060302u);
}

// Truncation split of 8 FP32 values (K slots 0-7 of a fragment) into the
// packed BF16 fragments of the three parts.
__device__ inline void split_pack(const float (&f)[8], v4u &H, v4u &M, v4u &L)
{
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const float x0 = f[2 * w], x1 = f[2 * w + 1];
        const unsigned u0 = __float_as_uint(x0), u1 = __float_as_uint(x1);
        const float r0 = x0 - __uint_as_float(u0 & 0xffff0000u);
        const float r1 = x1 - __uint_as_float(u1 & 0xffff0000u);
        const unsigned s0 = __float_as_uint(r0), s1 = __float_as_uint(r1);
        const float l0 = r0 - __uint_as_float(s0 & 0xffff0000u);
        const float l1 = r1 - __uint_as_float(s1 & 0xffff0000u);
        H[w] = pack_hi(u0, u1);
        M[w] = pack_hi(s0, s1);
        L[w] = pack_hi(__float_as_uint(l0), __float_as_uint(l1));
    }
}

__device__ __forceinline__ v16f mfma_bf(const v4u &b, const v4u &a, const v16f &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, b),
                                                   __builtin_bit_cast(v8bf, a), c, 0, 0, 0);
}

// The 16 same-parity values of this lane (K = 0..15 of its ring pair) ->
// fragments of both column halves, then the six products against the
// lane's coefficient parts B[level].
__device__ __forceinline__ void parity_mfma(const float (&v)[16], const v4u (&B)[3], v16f &acc0,
                                            v16f &acc1)
{
    float f0[8], f1[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) swap_halves(v[t], v[t + 8], f0[t], f1[t]);
    v4u H0, M0, L0, H1, M1, L1;
    split_pack(f0, H0, M0, L0);
    split_pack(f1, H1, M1, L1);
    acc0 = mfma_bf(B[0], H0, acc0);
    acc1 = mfma_bf(B[0], H1, acc1);
    acc0 = mfma_bf(B[0], M0, acc0);
    acc1 = mfma_bf(B[0], M1, acc1);
    acc0 = mfma_bf(B[1], H0, acc0);
    acc1 = mfma_bf(B[1], H1, acc1);
    acc0 = mfma_bf(B[0], L0, acc0);
    acc1 = mfma_bf(B[0], L1, acc1);
    acc0 = mfma_bf(B[1], M0, acc0);
    acc1 = mfma_bf(B[1], M1, acc1);
    acc0 = mfma_bf(B[2], H0, acc0);
    acc1 = mfma_bf(B[2], H1, acc1);
}

// One block of 32 l-rows from LDS: Ab = its 32 coefficients (as 16 pairs),
// Bs = the block's packed coefficient parts.  SEED: rows 0..31 of the m,
// started from P_mm (ua) with P_{m+1,m} = A_1 x P_mm.  MASK: lanes below
// k = 0 contribute 0, and the scaled exponents are checked every 16 rows.
template <bool MASK, bool SEED>
__device__ __forceinline__ void block32(double x, double &ua, double &ub, int &k,
                                        const double2 *__restrict__ Ab,
                                        const v4u *__restrict__ Bs, int lane, MfmaTiles &acc)
{
    const int hi = lane >> 5, col = lane & 31;
    float ve[16], vo[16];
    bool live = !MASK || k == 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const double2 a = Ab[t];
        double u0, u1;
        if (SEED && t == 0) {
            u0 = ua;
            u1 = (a.y * x) * ua;
        } else {
            u0 = fma(a.x * x, ub, -ua);
            u1 = fma(a.y * x, u0, -ub);
        }
        ua = u0;
        ub = u1;
        ve[t] = MASK ? opnd(u0, live) : (float)u0;
        vo[t] = MASK ? opnd(u1, live) : (float)u1;
        if (MASK && (t == 7 || t == 15)) {
            rescale_mixed(ua, ub, k);
            if (t == 7) live = k == 0;
        }
    }
    v4u BE[3], BO[3];
#pragma unroll
    for (int lev = 0; lev < 3; ++lev) {
        BE[lev] = Bs[((0 * 3 + lev) * 2 + hi) * 32 + col];
        BO[lev] = Bs[((1 * 3 + lev) * 2 + hi) * 32 + col];
    }
    parity_mfma(ve, BE, acc.e0, acc.e1);
    parity_mfma(vo, BO, acc.o0, acc.o1);
}

// A block in which no lane of the wave has reached k = 0: the recurrence
// alone (same arithmetic as block32, so the state is bitwise the same).
template <bool MASK, bool SEED>
__device__ __forceinline__ void block32_dead(double x, double &ua, double &ub, int &k,
                                             const double2 *__restrict__ Ab)
{
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const double2 a = Ab[t];
        double u0, u1;
        if (SEED && t == 0) {
            u0 = ua;
            u1 = (a.y * x) * ua;
        } else {
            u0 = fma(a.x * x, ub, -ua);
            u1 = fma(a.y * x, u0, -ub);
        }
        ua = u0;
        ub = u1;
        if (MASK && (t == 7 || t == 15)) rescale_mixed(ua, ub, k);
    }
}

// Copy of super-block sb of an m (its 4 packed B blocks and 128
// coefficients) global-to-LDS into `buf`; it completes at the workgroup's
// next barrier.  Past the m's last block or row the copy reads
// neighbouring data or the padding after the tables, which lands only in
// rows that are never used or are multiplied by B = 0.
__device__ __forceinline__ void super_dma(char *buf, const v4u *__restrict__ Bm,
                                          const double *__restrict__ Am, int sb, int tid)
{
    // the lane addresses are recomputed at every copy (a few integer
    // operations) rather than kept live, and spilled, across the loop
    asm volatile("" : "+v"(tid));
    const v4u *src = Bm + (long long)sb * kSuper * kBlkElems;
    v4u *dst = reinterpret_cast<v4u *>(buf + kABytes);
#pragma unroll
    for (int c = 0; c < kSuper * kBlkElems / kThreads; ++c) {
        const int w = tid + kThreads * c;
        __builtin_amdgcn_global_load_lds(src + w, dst + w, 16, 0, 0);
    }
    const unsigned *asrc = reinterpret_cast<const unsigned *>(Am + (long long)sb * kSuperRows);
    __builtin_amdgcn_global_load_lds(asrc + tid, reinterpret_cast<unsigned *>(buf) + tid, 4, 0, 0);
}

template <bool MASK>
__device__ __forceinline__ void super_compute(double x, double &ua, double &ub, int &k,
                                              const char *cur, char *nxt, bool more, int sb,
                                              int nb, bool seed, const v4u *__restrict__ Bm,
                                              const double *__restrict__ Am, int tid,
                                              MfmaTiles &acc, MfmaTiles &tot)
{
    const int lane = tid & 63;
    const double2 *As = reinterpret_cast<const double2 *>(cur);
    const v4u *Bs = reinterpret_cast<const v4u *>(cur + kABytes);
    zero_tiles(acc);
    if (more) super_dma(nxt, Bm, Am, sb + 1, tid);
    if (seed) {
        if (wave_any(k == 0))
            block32<true, true>(x, ua, ub, k, As, Bs, lane, acc);
        else
            block32_dead<true, true>(x, ua, ub, k, As);
    } else if (!MASK || wave_any(k == 0)) {
        block32<MASK, false>(x, ua, ub, k, As, Bs, lane, acc);
    } else {
        block32_dead<MASK, false>(x, ua, ub, k, As);
    }
    for (int q = 1; q < nb; ++q) {
        if (!MASK || wave_any(k == 0))
            block32<MASK, false>(x, ua, ub, k, As + (kBlkSteps / 2) * q, Bs + kBlkElems * q,
                                 lane, acc);
        else
            block32_dead<MASK, false>(x, ua, ub, k, As + (kBlkSteps / 2) * q);
    }
    add_tiles(tot, acc);
}

// A thread's share of the first live super-block of an m (register staged).
struct SuperStage {
    v4u b[kSuper * kBlkElems / kThreads];
    unsigned a;
};

__device__ __forceinline__ void super_stage_load(SuperStage &g, const v4u *__restrict__ Bm,
                                                 int nblk, const double *__restrict__ Am,
                                                 int len, int sb, int tid)
{
    const int b0 = sb * kSuper;
    const int nw = min(kSuper, nblk - b0) * kBlkElems;  // 16-byte words present
    const v4u *__restrict__ src = Bm + (long long)b0 * kBlkElems;
#pragma unroll
    for (int c = 0; c < kSuper * kBlkElems / kThreads; ++c) {
        const int w = tid + kThreads * c;
        g.b[c] = (w < nw) ? src[w] : v4u{};
    }
    const int r = sb * kSuperRows + (tid >> 1);  // dword tid of the 128 coefficients
    g.a = (r < len) ? reinterpret_cast<const unsigned *>(Am + r)[tid & 1] : 0u;
}

__device__ __forceinline__ void super_stage_store(const SuperStage &g, char *buf, int tid)
{
    v4u *B = reinterpret_cast<v4u *>(buf + kABytes);
#pragma unroll
    for (int c = 0; c < kSuper * kBlkElems / kThreads; ++c) B[tid + kThreads * c] = g.b[c];
    reinterpret_cast<unsigned *>(buf)[tid] = g.a;
}

struct MState {
    int m, i, len, nblk, nsb, sb0;
    const double *Am;
    const v4u *Bm;
    double ua, ub;
    int k;
};

// Seed and phase 1 (recurrence alone while the whole workgroup is below
// 2^-400), then the register copy of the first live super-block.
__device__ void m_begin(MState &st, SuperStage &g, int i, const int *__restrict__ mval,
                        const long long *__restrict__ soff, const long long *__restrict__ boff,
                        const double *__restrict__ mu, int lmax, const double *__restrict__ Asb,
                        const v4u *__restrict__ Bg, double x, double s, int tid)
{
    st.i = i;
    st.m = mval[i];
    st.len = lmax - st.m + 1;
    st.nblk = (st.len + kBlkSteps - 1) / kBlkSteps;
    st.nsb = (st.nblk + kSuper - 1) / kSuper;
    // coefficients from the per-super-block copy, zero past the m's last row:
    // the copies of a super-block run past the m's end, and with A = 0 there
    // the recurrence of the unused rows stays bounded (u_l = -u_{l-2})
    st.Am = Asb + soff[i] * kSuperRows;
    st.Bm = Bg + boff[i] * kBlkElems;
    st.ub = 0.0;
    seed_mm(mu[i], s, st.m, st.ua, st.k);
    if (st.k == 0 && fabs(st.ua) < kEmergeTrue) {
        st.ua *= kTwoS;
        st.k = -1;
    }
    int sb0 = 0;
    while (sb0 < st.nsb && !__syncthreads_or(st.k == 0)) {
        const int n16 = min(kSuperRows, st.len - sb0 * kSuperRows + 15) / 16;
        for (int q = 0; q < n16; ++q) {
            const int r0 = sb0 * kSuperRows + q * 16;
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

__device__ __forceinline__ void m_commit(const MState &st, const SuperStage &g, char *ldsA,
                                         int tid)
{
    if (st.sb0 < st.nsb) super_stage_store(g, ldsA, tid);
    __syncthreads();
}

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

__device__ __forceinline__ void m_compute(MState &st, char *ldsA, char *ldsB, double x, int tid,
                                          MfmaTiles &tot)
{
    MfmaTiles acc;
    zero_tiles(tot);
    bool mask = true;
    for (int sb = st.sb0; sb < st.nsb; sb += 2) {
        m_step(st, sb, ldsA, ldsB, x, tid, mask, acc, tot);
        if (sb + 1 < st.nsb) m_step(st, sb + 1, ldsB, ldsA, x, tid, mask, acc, tot);
    }
}

__global__ __launch_bounds__(kThreads, 2) void k_legendre_mfma_bf16x3(
    const PairDesc *__restrict__ pairs, int npairs, int pgroups,
    const int *__restrict__ mval, const long long *__restrict__ soff,
    const long long *__restrict__ boff, const double *__restrict__ mu, int nm, int nmpairs,
    int lmax, const double *__restrict__ Asb, const v4u *__restrict__ Bb, long long nblocks,
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
    const v4u *Bg = Bb + (long long)grp * nblocks * kBlkElems;
    MState st;
    SuperStage g;
    MfmaTiles tot;
    m_begin(st, g, q, mval, soff, boff, mu, lmax, Asb, Bg, x, s, tid);
    m_commit(st, g, ldsA, tid);
    m_compute(st, ldsA, ldsB, x, tid, tot);
    const int i1 = st.i;
    const int i2 = nm - 1 - q;
    const bool two = i2 != q;
    if (two) m_begin(st, g, i2, mval, soff, boff, mu, lmax, Asb, Bg, x, s, tid);
    m_store(tot, i1, delta, pairs, npairs, pb, grp, nmaps, nrings, nm, tid & 63);
    if (two) {
        m_commit(st, g, ldsA, tid);
        m_compute(st, ldsA, ldsB, x, tid, tot);
        m_store(tot, st.i, delta, pairs, npairs, pb, grp, nmaps, nrings, nm, tid & 63);
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
    // plus one super-block: the copies of an m's last super-block may read past it
    return (groups * (size_t)bf16_blocks(p) + kSuper) * kBlkElems * 16;
}

hipError_t launch_prescale_bf16x3(const sht_plan_s *p, const double *alm, void *Bb,
                                  hipStream_t st)
{
    const long long m0len = (p->mval[0] == 0) ? (p->lmax + 1) : 0;
    const int groups = (p->nmaps + 15) / 16;
    const long long nblocks = bf16_blocks(p);
    const long long nwg = (nblocks + kPreBlocks - 1) / kPreBlocks;
    if (nwg <= 0 || nwg > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_prescale_bf16x3, dim3((unsigned)nwg, (unsigned)groups), dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(alm), p->d_cn, p->d_moff, p->d_mval,
                       p->d_boff, p->d_bm32, p->lmax, p->nalm, nblocks, p->nmaps, m0len,
                       reinterpret_cast<v4u *>(Bb));
    return hipGetLastError();
}

hipError_t launch_legendre_mfma_bf16x3(const sht_plan_s *p, const void *Bb, float2 *delta,
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
    hipLaunchKernelGGL(k_legendre_mfma_bf16x3, dim3((unsigned)total), dim3(kThreads), 0, st,
                       p->d_pairs, p->npairs, pgroups, p->d_mval, p->d_soff, p->d_boff, p->d_mu, p->nm,
                       nmpairs, p->lmax, p->d_Asb, reinterpret_cast<const v4u *>(Bb),
                       bf16_blocks(p), delta, p->nrings, p->nmaps,
                       total);
    return hipGetLastError();
}

}  // namespace sht
