// Mixed-precision batched Legendre stage with 2-way split FP16 inputs on the
// matrix cores (gfx950, v_mfma_f32_32x32x16_f16).
//
// Same contraction as the FP32 form (per m, C_E/O = B_E/O^T Lambda_E/O^T,
// Delta_N = C_E + C_O, Delta_S = C_E - C_O).  Every FP32 operand x is written
// as x = x_h + x_l with x_h = x rounded to FP16 and x_l = (x - x_h) rounded
// to FP16 (the difference is exact in FP32), about 22 significant bits
// together; the product is taken as the three terms
// A_h B_h + A_h B_l + A_l B_h, the dropped A_l B_l being below 2^-21
// relative.  Products of FP16 numbers are exact in FP32, and accumulation
// is two-level FP32 as in the FP32 form (64 same-parity terms per
// first-level block).  The recurrence stays FP64 on the vector units.
//
// Range.  FP16 carries 5 exponent bits, so both operands are moved into its
// range by powers of two (exact).  The P_lm values: u = P_lm / c_lm is below
// 2^8.75 for l <= 16383 at scaled exponent k = 0 (addition theorem and the
// smallest c_lm), and the seed is multiplied by 2^6, so every matrix operand
// stays below 2^15.  The coefficients: per map and 128-row super-block the
// prescale picks 2^e with the largest magnitude in [2^14, 2^15).  The
// first-level sums of a super-block are multiplied by 2^-(e+6) as they are
// added into the second-level sums (one FMA per entry, as many instructions
// as the plain add).  Past an m's last row the recurrence coefficients are
// zero (a padded copy of the table per super-block), so u stays bounded
// there and its product with the zero coefficients is zero, never 0 * inf.
//
// Fragments and work split are those of the split-BF16 form: a 32x32x16
// fragment holds K = 0..7 of its 32 columns in lanes 0-31 and K = 8..15 in
// lanes 32-63; a lane's 16 same-parity values are exchanged across the wave
// halves as FP32 and then split (one packed conversion per two values, one
// mixed-precision FMA per residual, one packed conversion per two
// residuals).  A workgroup of four waves takes 256 ring pairs and an m-pair;
// per super-block of 128 l-rows the coefficient parts, their scales and A_l
// are copied global-to-LDS while the previous super-block is multiplied; the
// workgroup runs the recurrence alone while all its lanes are below 2^-400,
// then a masked path for its first live super-block, then a path with no
// mask and no rescaling.
#include "mixed_common.h"

namespace sht {
namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));

constexpr int kWaves = 4;                   // waves (64 ring pairs each) sharing an m
constexpr int kThreads = 64 * kWaves;
constexpr int kBlkSteps = 32;               // l-rows per block (K = 16 per parity)
// Packed B layout per block: [parity 2][level 2][half 2][column 32] x 8 fp16.
constexpr int kBlkElems = 2 * 2 * 2 * 32;   // 16-byte elements per block
constexpr int kSuper = 4;                   // blocks per super-block: 64 terms per parity
constexpr int kSuperRows = kSuper * kBlkSteps;
constexpr int kScaleElems = 4;              // 16 FP32 inverse scales (one per map)
constexpr int kSuperElems = kSuper * kBlkElems + kScaleElems;
constexpr int kABytes = kSuperRows * 8;     // A of a super-block in LDS
constexpr int kBufBytes = kABytes + kSuperElems * 16;
constexpr double kPScale = 0x1p6;           // P_lm operands are u * 2^6

// Two FP32 values rounded to FP16 (round to nearest even), packed.  The
// empty asm keeps the compiler from re-deriving either half from x (it would
// convert each value again).
__device__ inline unsigned pk_f16(float a, float b)
{
    const v2h h = {(_Float16)a, (_Float16)b};
    unsigned u = __builtin_bit_cast(unsigned, h);
    asm("" : "+v"(u));
    return u;
}

// x - (float)low / high half of h, exact (one mixed-precision FMA).
__device__ inline float res_lo(unsigned h, float x)
{
    float r;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(x));
    return r;
}
__device__ inline float res_hi(unsigned h, float x)
{
    float r;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r)
        : "v"(h), "v"(x));
    return r;
}

// 8 FP32 values (K slots 0-7 of a fragment) -> packed FP16 high and low parts.
__device__ inline void split_pack(const float (&f)[8], v4u &H, v4u &L)
{
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const unsigned h = pk_f16(f[2 * w], f[2 * w + 1]);
        H[w] = h;
        L[w] = pk_f16(res_lo(h, f[2 * w]), res_hi(h, f[2 * w + 1]));
    }
}

__device__ __forceinline__ v16f mfma_h(const v4u &b, const v4u &a, const v16f &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, b),
                                                  __builtin_bit_cast(v8h, a), c, 0, 0, 0);
}

// a'_lm = c_lm a_lm of up to 16 maps for one 128-row super-block of an m:
// scaled per map by 2^e (largest magnitude into [2^14, 2^15)), split into
// FP16 parts and packed; the inverse scales 2^-(e+6) follow the blocks.
// One workgroup per super-block (sbm: the m of each super-block); thread
// item idx = tid + 256 q is (map idx / 128, row idx % 128), so the a_lm of
// a map are read in runs of 128 rows.
__global__ __launch_bounds__(256) void k_prescale_f16x2(
    const double2 *__restrict__ alm, const double *__restrict__ cn,
    const long long *__restrict__ moff, const int *__restrict__ mval,
    const long long *__restrict__ soff, const int *__restrict__ sbm, int lmax, long long nalm,
    long long nsuper, int nmaps, long long m0len, v4u *__restrict__ Bb)
{
    __shared__ __attribute__((aligned(16))) _Float16 stage[kSuperElems * 8];
    __shared__ float wmax[kWaves][8];
    __shared__ int wexp[16];
    const long long s = blockIdx.x;
    const int grp = blockIdx.y;
    const int tid = threadIdx.x;
    const int i = sbm[s];
    const int len = lmax - mval[i] + 1;
    const long long row0 = (s - soff[i]) * kSuperRows;
    double2 v[8];
    float mx[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int idx = tid + 256 * q;
        const int mp = idx >> 7, rb = idx & 127;
        const long long row = row0 + rb;
        const int map = grp * 16 + mp;
        double2 b = make_double2(0.0, 0.0);
        if (row < len && map < nmaps) {
            const long long e = moff[i] + row;
            const double2 a = alm[(long long)map * nalm + e];
            const double c = cn[e];
            b.x = a.x * c;
            b.y = (e < m0len) ? 0.0 : a.y * c;
        }
        v[q] = b;
        mx[q] = (float)fmax(fabs(b.x), fabs(b.y));   // rounding cannot move a power of two
    }
    // per map (= 2 q + wave / 2): max over its 128 rows, two waves of 64
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        float m = mx[q];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        mx[q] = m;
    }
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) wmax[wave][q] = mx[q];
    }
    __syncthreads();
    if (tid < 16) {
        const int q = tid >> 1, w0 = 2 * (tid & 1);
        const float m = fmaxf(wmax[w0][q], wmax[w0 + 1][q]);
        int e = 0;
        if (m > 0.0f) {
            int E;
            (void)frexpf(m, &E);          // m < 2^E
            e = min(max(15 - E, -120), 120);
        }
        wexp[2 * q + (tid & 1)] = e;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int idx = tid + 256 * q;
        const int mp = idx >> 7, rb = idx & 127;
        const int map = 2 * q + (tid >> 7);   // = mp
        const double sc = ldexp(1.0, wexp[map]);
        const int blk = rb >> 5, r32 = rb & 31;
        const int par = r32 & 1, kk = r32 >> 1, half = kk >> 3, slot = kk & 7;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float x = (float)((c ? v[q].y : v[q].x) * sc);
            const _Float16 h = (_Float16)x;
            const _Float16 l = (_Float16)(x - (float)h);
            const int col = 2 * mp + c;
            _Float16 *st = stage + (size_t)blk * kBlkElems * 8;
            st[(((par * 2 + 0) * 2 + half) * 32 + col) * 8 + slot] = h;
            st[(((par * 2 + 1) * 2 + half) * 32 + col) * 8 + slot] = l;
        }
    }
    if (tid < 16)
        reinterpret_cast<float *>(stage + kSuper * kBlkElems * 8)[tid] =
            (float)ldexp(1.0, -(wexp[tid] + 6));
    __syncthreads();
    const v4u *s4 = reinterpret_cast<const v4u *>(stage);
    v4u *o4 = Bb + ((long long)grp * nsuper + s) * kSuperElems;
#pragma unroll
    for (int q = 0; q < kSuper * kBlkElems / 256; ++q) o4[tid + 256 * q] = s4[tid + 256 * q];
    if (tid < kScaleElems) o4[kSuper * kBlkElems + tid] = s4[kSuper * kBlkElems + tid];
}

// The 16 same-parity values of this lane (K = 0..15 of its ring pair) ->
// fragments of both column halves, then the three products against the
// lane's coefficient parts B[level].
__device__ __forceinline__ void parity_mfma(const float (&v)[16], const v4u (&B)[2], v16f &acc0,
                                            v16f &acc1)
{
    float f0[8], f1[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) swap_halves(v[t], v[t + 8], f0[t], f1[t]);
    v4u H0, L0, H1, L1;
    split_pack(f0, H0, L0);
    split_pack(f1, H1, L1);
    acc0 = mfma_h(B[0], H0, acc0);
    acc1 = mfma_h(B[0], H1, acc1);
    acc0 = mfma_h(B[0], L0, acc0);
    acc1 = mfma_h(B[0], L1, acc1);
    acc0 = mfma_h(B[1], H0, acc0);
    acc1 = mfma_h(B[1], H1, acc1);
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
    v4u BE[2], BO[2];
#pragma unroll
    for (int lev = 0; lev < 2; ++lev) {
        BE[lev] = Bs[((0 * 2 + lev) * 2 + hi) * 32 + col];
        BO[lev] = Bs[((1 * 2 + lev) * 2 + hi) * 32 + col];
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

// tot += acc * (inverse scale of the entry's map).  Entry r of a lane's
// tile row set is row 8 (r/4) + 4 hi + r%4 = 2 map + Re/Im, so the lane's
// maps are 4 j + 2 hi + {0, 1}, j = 0..3.
__device__ __forceinline__ void add_tiles_scaled(MfmaTiles &tot, const MfmaTiles &acc,
                                                 const float *__restrict__ isc, int hi)
{
    float s[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float2 v = reinterpret_cast<const float2 *>(isc)[2 * j + hi];
        s[2 * j] = v.x;
        s[2 * j + 1] = v.y;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float f = s[2 * (r >> 2) + ((r & 3) >> 1)];
        tot.e0[r] = fmaf(acc.e0[r], f, tot.e0[r]);
        tot.e1[r] = fmaf(acc.e1[r], f, tot.e1[r]);
        tot.o0[r] = fmaf(acc.o0[r], f, tot.o0[r]);
        tot.o1[r] = fmaf(acc.o1[r], f, tot.o1[r]);
    }
}

// Copy of super-block sb of an m (its packed B blocks, their inverse scales
// and 128 coefficients) global-to-LDS into `buf`; it completes at the
// workgroup's next barrier.  The padded tables hold whole super-blocks, so
// the copy never reads past the m's own data.
__device__ __forceinline__ void super_dma(char *buf, const v4u *__restrict__ Bm,
                                          const double *__restrict__ Am, int sb, int tid)
{
    // the lane addresses are recomputed at every copy (a few integer
    // operations) rather than kept live, and spilled, across the loop
    asm volatile("" : "+v"(tid));
    const v4u *src = Bm + (long long)sb * kSuperElems;
    v4u *dst = reinterpret_cast<v4u *>(buf + kABytes);
#pragma unroll
    for (int c = 0; c < kSuper * kBlkElems / kThreads; ++c) {
        const int w = tid + kThreads * c;
        __builtin_amdgcn_global_load_lds(src + w, dst + w, 16, 0, 0);
    }
    if (tid < kScaleElems)
        __builtin_amdgcn_global_load_lds(src + kSuper * kBlkElems + tid,
                                         dst + kSuper * kBlkElems + tid, 16, 0, 0);
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
    add_tiles_scaled(tot, acc, reinterpret_cast<const float *>(Bs + kSuper * kBlkElems),
                     lane >> 5);
}

// A thread's share of the first live super-block of an m (register staged).
struct SuperStage {
    v4u b[kSuper * kBlkElems / kThreads];
    v4u sc;
    unsigned a;
};

__device__ __forceinline__ void super_stage_load(SuperStage &g, const v4u *__restrict__ Bm,
                                                 const double *__restrict__ Am, int sb, int tid)
{
    const v4u *__restrict__ src = Bm + (long long)sb * kSuperElems;
#pragma unroll
    for (int c = 0; c < kSuper * kBlkElems / kThreads; ++c) g.b[c] = src[tid + kThreads * c];
    g.sc = (tid < kScaleElems) ? src[kSuper * kBlkElems + tid] : v4u{};
    g.a = reinterpret_cast<const unsigned *>(Am + (long long)sb * kSuperRows)[tid];
}

__device__ __forceinline__ void super_stage_store(const SuperStage &g, char *buf, int tid)
{
    v4u *B = reinterpret_cast<v4u *>(buf + kABytes);
#pragma unroll
    for (int c = 0; c < kSuper * kBlkElems / kThreads; ++c) B[tid + kThreads * c] = g.b[c];
    if (tid < kScaleElems) B[kSuper * kBlkElems + tid] = g.sc;
    reinterpret_cast<unsigned *>(buf)[tid] = g.a;
}

struct MState {
    int m, i, len, nblk, nsb, sb0;
    const double *Am;    // padded coefficients of the m, per super-block
    const v4u *Bm;
    double ua, ub;
    int k;
};

// Seed and phase 1 (recurrence alone while the whole workgroup is below
// 2^-400, coefficients from the plain table), then the register copy of
// the first live super-block.
__device__ void m_begin(MState &st, SuperStage &g, int i, const int *__restrict__ mval,
                        const long long *__restrict__ moff, const long long *__restrict__ soff,
                        const double *__restrict__ mu, int lmax, const double *__restrict__ A,
                        const double *__restrict__ Asb, const v4u *__restrict__ Bg, double x,
                        double s, int tid)
{
    st.i = i;
    st.m = mval[i];
    st.len = lmax - st.m + 1;
    st.nblk = (st.len + kBlkSteps - 1) / kBlkSteps;
    st.nsb = (st.nblk + kSuper - 1) / kSuper;
    const double *Ap = A + moff[i];
    st.Am = Asb + soff[i] * kSuperRows;
    st.Bm = Bg + soff[i] * kSuperElems;
    st.ub = 0.0;
    seed_mm(mu[i], s, st.m, st.ua, st.k);
    if (st.k == 0 && fabs(st.ua) < kEmergeTrue) {
        st.ua *= kTwoS;
        st.k = -1;
    }
    st.ua *= kPScale;
    int sb0 = 0;
    while (sb0 < st.nsb && !__syncthreads_or(st.k == 0)) {
        const int n16 = min(kSuperRows, st.len - sb0 * kSuperRows + 15) / 16;
        for (int q = 0; q < n16; ++q) {
            const int r0 = sb0 * kSuperRows + q * 16;
            if (r0 == 0)
                block16_dead_g<true>(x, st.ua, st.ub, Ap, r0);
            else
                block16_dead_g<false>(x, st.ua, st.ub, Ap, r0);
            rescale_mixed(st.ua, st.ub, st.k);
        }
        ++sb0;
    }
    st.sb0 = sb0;
    if (sb0 < st.nsb) super_stage_load(g, st.Bm, st.Am, sb0, tid);
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

__global__ __launch_bounds__(kThreads, 2) void k_legendre_mfma_f16x2(
    const PairDesc *__restrict__ pairs, int npairs, int pgroups,
    const int *__restrict__ mval, const long long *__restrict__ moff,
    const long long *__restrict__ soff, const double *__restrict__ mu, int nm, int nmpairs,
    int lmax, const double *__restrict__ A, const double *__restrict__ Asb,
    const v4u *__restrict__ Bb, long long nsuper, float2 *__restrict__ delta, int nrings,
    int nmaps, long long total)
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
    const v4u *Bg = Bb + (long long)grp * nsuper * kSuperElems;
    MState st;
    SuperStage g;
    MfmaTiles tot;
    m_begin(st, g, q, mval, moff, soff, mu, lmax, A, Asb, Bg, x, s, tid);
    m_commit(st, g, ldsA, tid);
    m_compute(st, ldsA, ldsB, x, tid, tot);
    const int i1 = st.i;
    const int i2 = nm - 1 - q;
    const bool two = i2 != q;
    if (two) m_begin(st, g, i2, mval, moff, soff, mu, lmax, A, Asb, Bg, x, s, tid);
    m_store(tot, i1, delta, pairs, npairs, pb, grp, nmaps, nrings, nm, tid & 63);
    if (two) {
        m_commit(st, g, ldsA, tid);
        m_compute(st, ldsA, ldsB, x, tid, tot);
        m_store(tot, st.i, delta, pairs, npairs, pb, grp, nmaps, nrings, nm, tid & 63);
    }
}

}  // namespace

int f16_super_rows() { return kSuperRows; }

size_t f16_bytes(const sht_plan_s *p)
{
    const size_t groups = (size_t)((p->nmaps + 15) / 16);
    return groups * (size_t)p->nsuper * kSuperElems * 16;
}

hipError_t launch_prescale_f16x2(const sht_plan_s *p, const double *alm, void *Bb,
                                 hipStream_t st)
{
    const long long m0len = (p->mval[0] == 0) ? (p->lmax + 1) : 0;
    const int groups = (p->nmaps + 15) / 16;
    if (p->nsuper <= 0 || p->nsuper > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_prescale_f16x2, dim3((unsigned)p->nsuper, (unsigned)groups), dim3(256),
                       0, st, reinterpret_cast<const double2 *>(alm), p->d_cn, p->d_moff,
                       p->d_mval, p->d_soff, p->d_sbm, p->lmax, p->nalm, p->nsuper, p->nmaps,
                       m0len, reinterpret_cast<v4u *>(Bb));
    return hipGetLastError();
}

hipError_t launch_legendre_mfma_f16x2(const sht_plan_s *p, const void *Bb, float2 *delta,
                                      hipStream_t st)
{
    const int pblocks = (p->npairs + 63) / 64;
    const int pgroups = (pblocks + kWaves - 1) / kWaves;
    const int nmpairs = (p->nm + 1) / 2;
    const int groups = (p->nmaps + 15) / 16;
    const long long total = (long long)pgroups * nmpairs * groups;
    if (total <= 0 || total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_legendre_mfma_f16x2, dim3((unsigned)total), dim3(kThreads), 0, st,
                       p->d_pairs, p->npairs, pgroups, p->d_mval, p->d_moff, p->d_soff, p->d_mu,
                       p->nm, nmpairs, p->lmax, p->d_A, p->d_Asb,
                       reinterpret_cast<const v4u *>(Bb), p->nsuper,
                       delta, p->nrings, p->nmaps, total);
    return hipGetLastError();
}

}  // namespace sht
