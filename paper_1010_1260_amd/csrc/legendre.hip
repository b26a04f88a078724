// Legendre stage of alm2map and of its adjoint, FP64, for gfx950.
//
// Forward (Eq. DeltaDef, Sec. 2.1; Algorithms 1-2 with the recurrence merged
// into the accumulation, Sec. 2.2.2):
//     Delta_m(theta_r) = sum_{l=m}^{lmax} a_lm P_lm(cos theta_r).
//
// Recurrence.  Eq. (assLegRec) with the sign that yields orthonormal
// functions, P_l = beta_l (x P_{l-1} - P_{l-2} / beta_{l-1}), is rewritten
// for u_l = P_l / c_l with c_m = c_{m+1} = 1 and c_l = (beta_l/beta_{l-1}) c_{l-2}:
//     u_l = (A_l x) u_{l-1} - u_{l-2},      A_l = beta_l c_{l-1} / c_l,
// so one step is a multiply and a fused multiply-add; c_l (between 0.17 and
// 1.13 for l <= 4096) is folded into the coefficients, a'_lm = c_lm a_lm,
// by a prescale kernel.  The seeds are P_mm = mu_m sin^m(theta) (Eq. pmm,
// exponent m/2 on 1-x^2) and P_{m+1,m} = sqrt(2m+3) x P_mm (Eq. pm1m).
//
// Rescaling (Sec. 2.2.2).  A lane carries (v, k) with value v 2^(512 k),
// k <= 0.  Every 8 steps, if |v| > 2^512, both recurrence values and the
// accumulators are multiplied by 2^-512 (exact) and k grows by one.  The
// accumulators therefore always hold sum a' u 2^(512 (k_l - k)), and the
// result is acc * 2^(512 k): 1 for k = 0, 2^-512 for k = -1, 0 below.
//
// Mapping to CDNA4.  One wavefront owns 64*CH ring pairs (CH chains per
// lane); the north/south rings of a pair share the recurrence through the
// parity P_lm(-x) = (-1)^(l+m) P_lm(x): even l-m terms go to E, odd to O,
// Delta_N = E + O, Delta_S = E - O.  (l, m) is uniform across the wave, so
// A_l and a'_lm are read with scalar loads into SGPRs and fed straight into
// the FP64 VALU ops: 4 VALU instructions per (l, m, chain) and no LDS.
// A wave processes the m-pair (m_i, m_{nm-1-i}) whose lengths sum to a
// constant, which balances the triangular work.  Block ids are remapped so
// that the waves sharing an m-pair run on the same XCD (same L2).
#include "recurrence.h"
#include "sht_internal.h"

namespace sht {
namespace {

__global__ void k_prescale(const double2 *__restrict__ alm, const double *__restrict__ cn,
                           double2 *__restrict__ ap, long long nalm, long long m0len)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long b = blockIdx.y;
    if (e >= nalm) return;
    double2 a = alm[b * nalm + e];
    const double c = cn[e];
    a.x *= c;
    a.y = (e < m0len) ? 0.0 : a.y * c;
    ap[b * nalm + e] = a;
}

template <int CH>
struct Chains {
    double x[CH];
    int rn[CH], rs[CH];
};

// One m of an m-pair for CH chains per lane: forward accumulation.
template <int CH, bool CAS>
__device__ inline void fwd_one_m(const Chains<CH> &g, const double (&s)[CH], int m, int i,
                                 long long off, double mum, int lmax,
                                 const double *__restrict__ A, const double2 *__restrict__ ap,
                                 double2 *__restrict__ delta, long long dbase, int nrings)
{
    const int len = lmax - m + 1;
    // The coefficients are only read here and their addresses are uniform
    // across the wave.  CAS: read them through the constant address space,
    // so that they come in by scalar loads also when the kernel stores Delta
    // into the same buffer (the batched kernel's workspace), where the
    // compiler cannot prove that the loads are not clobbered.
    typedef const double __attribute__((address_space(4))) *CDp;
    const double *__restrict__ Ag = A + off;
    const double2 *__restrict__ apg = ap + off;
    const CDp Ac = (CDp)(A + off);
    const CDp amd = (CDp)(ap + off);   // a'_lm as (re, im) pairs
    auto Am = [&](int k) -> double {
        if constexpr (CAS) return Ac[k]; else return Ag[k];
    };
    auto am = [&](int k) -> double2 {
        if constexpr (CAS) return make_double2(amd[2 * k], amd[2 * k + 1]); else return apg[k];
    };
    double u0[CH], u1[CH], Er[CH], Ei[CH], Or[CH], Oi[CH];
    int k[CH];
    {
        const double2 a0 = am(0);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            seed_mm(mum, s[c], m, u0[c], k[c]);
            Er[c] = a0.x * u0[c];
            Ei[c] = a0.y * u0[c];
            Or[c] = 0.0; Oi[c] = 0.0; u1[c] = 0.0;
        }
    }
    if (len >= 2) {
        const double A1 = Am(1);
        const double2 a1 = am(1);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            u1[c] = (A1 * g.x[c]) * u0[c];
            Or[c] = a1.x * u1[c];
            Oi[c] = a1.y * u1[c];
        }
    }
    int j = 2;
    for (; j + 8 <= len; j += 8) {
#pragma unroll
        for (int t = 0; t < 8; t += 2) {
            const double Aa = Am(j + t), Ab = Am(j + t + 1);
            const double2 aa = am(j + t), ab = am(j + t + 1);
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const double u2 = fma(Aa * g.x[c], u1[c], -u0[c]);
                Er[c] = fma(aa.x, u2, Er[c]);
                Ei[c] = fma(aa.y, u2, Ei[c]);
                const double u3 = fma(Ab * g.x[c], u2, -u1[c]);
                Or[c] = fma(ab.x, u3, Or[c]);
                Oi[c] = fma(ab.y, u3, Oi[c]);
                u0[c] = u2; u1[c] = u3;
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (fmax(fabs(u0[c]), fabs(u1[c])) > kTwoS) {
                u0[c] *= kTwoMinusS; u1[c] *= kTwoMinusS;
                Er[c] *= kTwoMinusS; Ei[c] *= kTwoMinusS;
                Or[c] *= kTwoMinusS; Oi[c] *= kTwoMinusS;
                k[c] += 1;
            }
        }
    }
    for (; j < len; ++j) {
        const double Aa = Am(j);
        const double2 aa = am(j);
        if (j & 1) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const double u2 = fma(Aa * g.x[c], u1[c], -u0[c]);
                Or[c] = fma(aa.x, u2, Or[c]);
                Oi[c] = fma(aa.y, u2, Oi[c]);
                u0[c] = u1[c]; u1[c] = u2;
            }
        } else {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const double u2 = fma(Aa * g.x[c], u1[c], -u0[c]);
                Er[c] = fma(aa.x, u2, Er[c]);
                Ei[c] = fma(aa.y, u2, Ei[c]);
                u0[c] = u1[c]; u1[c] = u2;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const double f = final_scale(k[c]);
        // Delta [m][ring]: consecutive lanes write consecutive rings
        if (g.rn[c] >= 0)
            delta[dbase + (long long)i * nrings + g.rn[c]] =
                make_double2((Er[c] + Or[c]) * f, (Ei[c] + Oi[c]) * f);
        if (g.rs[c] >= 0)
            delta[dbase + (long long)i * nrings + g.rs[c]] =
                make_double2((Er[c] - Or[c]) * f, (Ei[c] - Oi[c]) * f);
    }
}

template <int CH>
__global__ __launch_bounds__(64) void k_legendre_fwd(
    const PairDesc *__restrict__ pairs, int npairs, int pblocks,
    const int *__restrict__ mval, const long long *__restrict__ moff,
    const double *__restrict__ mu, int nm, int nmpairs, int lmax,
    const double *__restrict__ A, const double2 *__restrict__ ap, long long nalm,
    double2 *__restrict__ delta, int nrings, long long total)
{
    const long long L = xcd_logical(blockIdx.x, total);
    const int pb = (int)(L % pblocks);
    const long long rest = L / pblocks;
    const int q = (int)(rest % nmpairs);
    const int b = (int)(rest / nmpairs);
    const int lane = threadIdx.x;

    Chains<CH> g;
    double s[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int p = (pb * CH + c) * 64 + lane;
        if (p < npairs) {
            const PairDesc d = pairs[p];
            g.x[c] = d.x; s[c] = d.s; g.rn[c] = d.rn; g.rs[c] = d.rs;
        } else {
            g.x[c] = 0.0; s[c] = 0.0; g.rn[c] = -1; g.rs[c] = -1;
        }
    }
    const double2 *apb = ap + (long long)b * nalm;
    const long long dbase = (long long)b * nrings * nm;
    for (int t = 0; t < 2; ++t) {
        const int i = (t == 0) ? q : nm - 1 - q;
        if (t == 1 && i == q) break;
        fwd_one_m<CH, false>(g, s, mval[i], i, moff[i], mu[i], lmax, A, apb, delta, dbase, nrings);
    }
}

// ------------------------------------------------------------------ adjoint
//
// out_lm = c_lm sum_pairs u_l(x_p) (Dt_N + (-1)^(l-m) Dt_S) 2^(512 k_l)
// A wave owns 64*CH ring pairs and one m-pair; per tile of 16 l-values each
// lane sums its chains, the 64 lane partials go through LDS (16 x 64
// complex, wave-private) and are reduced to one partial per (ring block, l).
// A second kernel adds the ring-block partials in a fixed order and applies
// c_lm, so the result is bitwise reproducible.

constexpr int kAdjTile = 16;
// Row length of the reduction buffer: 64 lane partials plus one pad entry.
// The reduction reads a column (lanes 0..15 take rows 0..15); with rows of
// exactly 64 entries (1 KB) those reads would all fall in one LDS bank.
constexpr int kAdjRow = 65;

template <int CH>
__device__ inline void adj_one_m(const Chains<CH> &g, const double (&s)[CH], int m, int i,
                                 long long off, double mum, int lmax,
                                 const double *__restrict__ A,
                                 const double2 *__restrict__ dt, long long dtbase, int nrings,
                                 double2 *__restrict__ part, double2 (*red)[kAdjRow])
{
    const int len = lmax - m + 1;
    const int lane = threadIdx.x;
    const double *__restrict__ Am = A + off;
    double u0[CH], u1[CH];
    double WEr[CH], WEi[CH], WOr[CH], WOi[CH];  // pair weights times 2^(512 k) factor
    double NEr[CH], NEi[CH], NOr[CH], NOi[CH];  // unscaled pair weights
    int k[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        double2 wn = make_double2(0.0, 0.0), ws = make_double2(0.0, 0.0);
        if (g.rn[c] >= 0) wn = dt[dtbase + (long long)i * nrings + g.rn[c]];
        if (g.rs[c] >= 0) ws = dt[dtbase + (long long)i * nrings + g.rs[c]];
        NEr[c] = wn.x + ws.x; NEi[c] = wn.y + ws.y;
        NOr[c] = wn.x - ws.x; NOi[c] = wn.y - ws.y;
        seed_mm(mum, s[c], m, u0[c], k[c]);
        u1[c] = (len >= 2) ? (Am[1] * g.x[c]) * u0[c] : 0.0;
        const double f = final_scale(k[c]);
        WEr[c] = NEr[c] * f; WEi[c] = NEi[c] * f; WOr[c] = NOr[c] * f; WOi[c] = NOi[c] * f;
    }
    for (int j0 = 0; j0 < len; j0 += kAdjTile) {
        double pr[kAdjTile], pi[kAdjTile];
#pragma unroll
        for (int t = 0; t < kAdjTile; ++t) { pr[t] = 0.0; pi[t] = 0.0; }
#pragma unroll
        for (int t = 0; t < kAdjTile; ++t) {
            const int j = j0 + t;
            if (j < len) {
                const double Aj = (j >= 2) ? Am[j] : 0.0;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    double u;
                    if (j == 0) {
                        u = u0[c];
                    } else if (j == 1) {
                        u = u1[c];
                    } else {
                        u = fma(Aj * g.x[c], u1[c], -u0[c]);
                        u0[c] = u1[c]; u1[c] = u;
                    }
                    if (t & 1) {  // j0 is even, so t carries the parity of l - m
                        pr[t] = fma(u, WOr[c], pr[t]);
                        pi[t] = fma(u, WOi[c], pi[t]);
                    } else {
                        pr[t] = fma(u, WEr[c], pr[t]);
                        pi[t] = fma(u, WEi[c], pi[t]);
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (fmax(fabs(u0[c]), fabs(u1[c])) > kTwoS) {
                u0[c] *= kTwoMinusS; u1[c] *= kTwoMinusS;
                k[c] += 1;
                const double f = final_scale(k[c]);
                WEr[c] = NEr[c] * f; WEi[c] = NEi[c] * f;
                WOr[c] = NOr[c] * f; WOi[c] = NOi[c] * f;
            }
        }
#pragma unroll
        for (int t = 0; t < kAdjTile; ++t) red[t][lane] = make_double2(pr[t], pi[t]);
        __syncthreads();
        {
            const int t = lane & (kAdjTile - 1);
            const int seg = lane / kAdjTile;  // 4 segments of 16 lanes
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const double2 v = red[t][seg * 16 + q];
                sr += v.x; si += v.y;
            }
            sr += __shfl_xor(sr, 16); si += __shfl_xor(si, 16);
            sr += __shfl_xor(sr, 32); si += __shfl_xor(si, 32);
            if (seg == 0 && j0 + t < len) part[off + j0 + t] = make_double2(sr, si);
        }
        __syncthreads();
    }
}

template <int CH>
__global__ __launch_bounds__(64) void k_legendre_adj(
    const PairDesc *__restrict__ pairs, int npairs, int pblocks,
    const int *__restrict__ mval, const long long *__restrict__ moff,
    const double *__restrict__ mu, int nm, int nmpairs, int lmax,
    const double *__restrict__ A, const double2 *__restrict__ dt, int nrings,
    double2 *__restrict__ part, long long nalm, long long total)
{
    __shared__ double2 red[kAdjTile][kAdjRow];
    const long long L = xcd_logical(blockIdx.x, total);
    const int pb = (int)(L % pblocks);
    const long long rest = L / pblocks;
    const int q = (int)(rest % nmpairs);
    const int b = (int)(rest / nmpairs);
    const int lane = threadIdx.x;
    Chains<CH> g;
    double s[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int p = (pb * CH + c) * 64 + lane;
        if (p < npairs) {
            const PairDesc d = pairs[p];
            g.x[c] = d.x; s[c] = d.s; g.rn[c] = d.rn; g.rs[c] = d.rs;
        } else {
            g.x[c] = 0.0; s[c] = 0.0; g.rn[c] = -1; g.rs[c] = -1;
        }
    }
    const long long dtbase = (long long)b * nrings * nm;
    double2 *pp = part + ((long long)b * pblocks + pb) * nalm;
    for (int t = 0; t < 2; ++t) {
        const int i = (t == 0) ? q : nm - 1 - q;
        if (t == 1 && i == q) break;
        adj_one_m<CH>(g, s, mval[i], i, moff[i], mu[i], lmax, A, dt, dtbase, nrings, pp, red);
    }
}

__global__ void k_adj_reduce(const double2 *__restrict__ part, const double *__restrict__ cn,
                             double *__restrict__ alm, long long nalm, int pblocks,
                             long long m0len, int accumulate)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long b = blockIdx.y;
    if (e >= nalm) return;
    double sr = 0.0, si = 0.0;
    const double2 *p = part + b * pblocks * nalm + e;
    for (int k = 0; k < pblocks; ++k) {
        const double2 v = p[(long long)k * nalm];
        sr += v.x; si += v.y;
    }
    const double c = cn[e];
    double2 *o = reinterpret_cast<double2 *>(alm) + b * nalm + e;
    const double2 v = make_double2(sr * c, (e < m0len) ? 0.0 : si * c);
    if (accumulate) {
        const double2 a = *o;
        *o = make_double2(a.x + v.x, a.y + v.y);
    } else {
        *o = v;
    }
}

// ---------------------------------------------------------------- batches
//
// A batch of single-map FP64 plans of different l_max / geometry runs the
// Legendre stage in one persistent launch: a fixed grid of waves takes
// tiles (map, m-pair, ring-pair block) from a work list sorted longest
// first, through an atomic counter.  The counter only hands out work; every
// tile's arithmetic is the same as in the single-plan kernel, so results do
// not depend on the schedule.  The counter is reset by a one-thread kernel
// launched before the persistent kernel (no memset node, so the sequence can
// be captured into a graph).

__global__ void k_batch_reset(int *counter) { *counter = 0; }

__global__ void k_batch_prescale(const BatchMap *__restrict__ maps,
                                 const double *const *__restrict__ alms, char *__restrict__ ws)
{
    const BatchMap &bm = maps[blockIdx.y];
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= bm.nalm) return;
    const double2 *a = reinterpret_cast<const double2 *>(alms[blockIdx.y]);
    double2 v = a[e];
    const double c = bm.cn[e];
    v.x *= c;
    v.y = (e < bm.m0len) ? 0.0 : v.y * c;
    reinterpret_cast<double2 *>(ws + bm.ap_off)[e] = v;
}

template <int CH>
__global__ __launch_bounds__(64) void k_legendre_fwd_batch(const BatchTile *__restrict__ tiles,
                                                           int ntiles,
                                                           const BatchMap *__restrict__ maps,
                                                           char *__restrict__ ws,
                                                           int *__restrict__ counter)
{
    const int lane = threadIdx.x;
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(counter, 1);
        // wave-uniform tile index: the tile, its plan's tables and every
        // coefficient of the recurrence then come through scalar loads, as
        // in the single-plan kernel
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
        if (t >= ntiles) break;
        const BatchTile tile = tiles[t];
        const BatchMap &bm = maps[tile.map];
        Chains<CH> g;
        double s[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int p = (tile.pblock * CH + c) * 64 + lane;
            if (p < bm.npairs) {
                const PairDesc d = bm.pairs[p];
                g.x[c] = d.x; s[c] = d.s; g.rn[c] = d.rn; g.rs[c] = d.rs;
            } else {
                g.x[c] = 0.0; s[c] = 0.0; g.rn[c] = -1; g.rs[c] = -1;
            }
        }
        const double2 *ap = reinterpret_cast<const double2 *>(ws + bm.ap_off);
        double2 *delta = reinterpret_cast<double2 *>(ws + bm.delta_off);
        const int q = tile.mpair;
        // the plan's per-m tables are read through the constant address
        // space (wave-uniform, never written here): scalar loads, so the
        // offsets and with them every coefficient address stay uniform
        typedef const int __attribute__((address_space(4))) *CIp;
        typedef const long long __attribute__((address_space(4))) *CLp;
        typedef const double __attribute__((address_space(4))) *CDp;
        for (int u = 0; u < 2; ++u) {
            const int i = (u == 0) ? q : bm.nm - 1 - q;
            if (u == 1 && i == q) break;
            fwd_one_m<CH, true>(g, s, ((CIp)bm.mval)[i], i, ((CLp)bm.moff)[i], ((CDp)bm.mu)[i],
                          bm.lmax, bm.A, ap, delta, 0, bm.nrings);
        }
    }
}

// The adjoint reduces every 16 l-rows over the wave's lanes through LDS.
// Four ring pairs per lane keep that reduction small next to the recurrence
// and leave registers for two waves per SIMD (224 VGPRs); at l_max 4096 the
// map2alm built on it takes 11.9 ms, against 13.8 ms with eight pairs (one
// wave per SIMD) and 16.7 ms with two.
constexpr int kAdjChains = 4;

}  // namespace

hipError_t launch_prescale(const sht_plan_s *p, const double *alm, double2 *ap, hipStream_t st)
{
    const long long m0len = (p->mval[0] == 0) ? (p->lmax + 1) : 0;
    dim3 grid((unsigned)((p->nalm + 255) / 256), (unsigned)p->nmaps);
    hipLaunchKernelGGL(k_prescale, grid, dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(alm), p->d_cn, ap, p->nalm, m0len);
    return hipGetLastError();
}

int fwd_pblocks(const sht_plan_s *p)
{
    const int per = 64 * p->fwd_chains;
    return (p->npairs + per - 1) / per;
}
int adj_pblocks(const sht_plan_s *p) { return (p->npairs + 64 * kAdjChains - 1) / (64 * kAdjChains); }

hipError_t launch_legendre_fwd(const sht_plan_s *p, const double2 *ap, double2 *delta,
                               hipStream_t st)
{
    const int pblocks = fwd_pblocks(p);
    const int nmpairs = (p->nm + 1) / 2;
    const long long total = (long long)pblocks * nmpairs * p->nmaps;
    if (total <= 0 || total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    auto kern = p->fwd_chains == 1   ? k_legendre_fwd<1>
                : p->fwd_chains == 2 ? k_legendre_fwd<2>
                : p->fwd_chains == 4 ? k_legendre_fwd<4>
                                     : nullptr;
    if (!kern) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(64), 0, st,
                       p->d_pairs, p->npairs, pblocks, p->d_mval, p->d_moff, p->d_mu, p->nm,
                       nmpairs, p->lmax, p->d_A, ap, p->nalm, delta, p->nrings, total);
    return hipGetLastError();
}

size_t adj_part_bytes(const sht_plan_s *p)
{
    return (size_t)p->nmaps * (size_t)adj_pblocks(p) * (size_t)p->nalm * sizeof(double2);
}

hipError_t launch_legendre_adj_ws(const sht_plan_s *p, const double2 *dt, double2 *part,
                                  double *alm, hipStream_t st, bool accumulate)
{
    const int pblocks = adj_pblocks(p);
    const int nmpairs = (p->nm + 1) / 2;
    const long long total = (long long)pblocks * nmpairs * p->nmaps;
    if (total <= 0 || total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_legendre_adj<kAdjChains>, dim3((unsigned)total), dim3(64), 0, st,
                       p->d_pairs, p->npairs, pblocks, p->d_mval, p->d_moff, p->d_mu, p->nm,
                       nmpairs, p->lmax, p->d_A, dt, p->nrings, part, p->nalm, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long m0len = (p->mval[0] == 0) ? (p->lmax + 1) : 0;
    dim3 grid((unsigned)((p->nalm + 255) / 256), (unsigned)p->nmaps);
    hipLaunchKernelGGL(k_adj_reduce, grid, dim3(256), 0, st, part, p->d_cn, alm, p->nalm,
                       pblocks, m0len, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_legendre(const BatchMap *maps, int nmaps, long long max_nalm,
                                 const BatchTile *tiles, int ntiles, int chains, int grid_waves,
                                 const double *const *alms, void *ws, int *counter,
                                 hipStream_t st)
{
    dim3 pg((unsigned)((max_nalm + 255) / 256), (unsigned)nmaps);
    hipLaunchKernelGGL(k_batch_prescale, pg, dim3(256), 0, st, maps, alms, (char *)ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, st, counter);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (chains) {
    case 1:
        hipLaunchKernelGGL(k_legendre_fwd_batch<1>, dim3((unsigned)grid_waves), dim3(64), 0, st,
                           tiles, ntiles, maps, (char *)ws, counter);
        break;
    case 2:
        hipLaunchKernelGGL(k_legendre_fwd_batch<2>, dim3((unsigned)grid_waves), dim3(64), 0, st,
                           tiles, ntiles, maps, (char *)ws, counter);
        break;
    case 4:
        hipLaunchKernelGGL(k_legendre_fwd_batch<4>, dim3((unsigned)grid_waves), dim3(64), 0, st,
                           tiles, ntiles, maps, (char *)ws, counter);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sht
