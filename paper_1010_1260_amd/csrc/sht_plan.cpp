// Host runtime of the C ABI declared in sht.h: descriptor validation, ring
// pairing, recurrence and Fourier tables, workspace layout and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "sht_internal.h"

using sht::PairDesc;
using sht::RingDesc;

namespace {


bool smooth7(long long n)
{
    if (n < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

// smallest 7-smooth integer >= n
int next_smooth7(long long n)
{
    long long v = std::max(1LL, n);
    while (!smooth7(v)) ++v;
    return (int)v;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bluestein convolution length by cost: every 7-smooth length in [L, 1.25 L]
// that stays in the size class of the smallest one, priced by the passes of
// the in-LDS Stockham FFT (radix 8 first, then 4 or 2, then 3, 5, 7): per
// point and pass about 12, 8.5, 5, 8, 13 and 17 flops for radix 8, 4, 2, 3,
// 5, 7, plus 10 for the pass's LDS round trip and barriers.  The smallest
// length often factors into several radix-5 and radix-7 passes (3000 =
// 8 x 3 x 5^3); a slightly longer one with fewer, cheaper passes (3072 =
// 8^3 x 2 x 3) measured faster: ring synthesis at l_max 4096 / nside 2048
// 10.6 -> 10.1 ms for 16 maps, 0.86 -> 0.78 ms for one FP64 map.
int best_smooth7(long long L)
{
    const int first = next_smooth7(L);
    const int cap = first <= 2048 ? 2048 : (first <= 4096 ? 4096 : 8192);
    double best = 1e300;
    int pick = first;
    for (long long c = first; c <= cap && c <= (L * 5) / 4 + 1; ++c) {
        if (!smooth7(c)) continue;
        long long r = c;
        double cost = 0.0;
        while (r > 1) {
            if (r % 8 == 0) { cost += 12 + 10; r /= 8; }
            else if (r % 4 == 0) { cost += 8.5 + 10; r /= 4; }
            else if (r % 2 == 0) { cost += 5 + 10; r /= 2; }
            else if (r % 3 == 0) { cost += 8 + 10; r /= 3; }
            else if (r % 5 == 0) { cost += 13 + 10; r /= 5; }
            else { cost += 17 + 10; r /= 7; }
        }
        cost *= (double)c;
        if (cost < best) { best = cost; pick = (int)c; }
    }
    return pick;
}

// Convolution length of the Bluestein fast path for a convolution of L
// points: the cheapest by the same per-pass costs among the lengths in
// [L, min(1.3 L, kBlueMaxN)] whose radix list holds one butterfly per thread
// in every pass; 0 if there is none.
int best_blue_nb(long long L)
{
    double best = 1e300;
    int pick = 0;
    for (long long c = L; c <= sht::kBlueMaxN && c <= (L * 13) / 10 + 1; ++c) {
        unsigned long long rads = 0;
        const int np = smooth7(c) ? sht::blue_radices((int)c, &rads) : 0;
        if (np == 0) continue;
        double cost = 0.0;
        for (int q = 0; q < np; ++q) {
            switch ((int)((rads >> (5 * q)) & 31)) {
            case 8: cost += 12 + 10; break;
            case 4: cost += 8.5 + 10; break;
            case 2: cost += 5 + 10; break;
            case 3: cost += 8 + 10; break;
            case 5: cost += 13 + 10; break;
            default: cost += 17 + 10; break;
            }
        }
        cost *= (double)c;
        if (cost < best) { best = cost; pick = (int)c; }
    }
    return pick;
}

uint64_t bits(double d)
{
    uint64_t u;
    std::memcpy(&u, &d, sizeof u);
    return u;
}

struct PairKeyHash {
    size_t operator()(const std::pair<uint64_t, uint64_t> &k) const
    {
        return std::hash<uint64_t>()(k.first * 0x9e3779b97f4a7c15ull ^ k.second);
    }
};

// Default launch shape of the FP64 forward Legendre kernel by problem size.
// The best block shape depends on the input size (Sec. 5 proposes tuning
// per size; Sec. 6.1 finds no single segment length / thread count best for
// every size), so the default comes from a table measured over sizes and
// sht_plan_autotune can refine it per plan.  Key: the waves the launch would
// have with one ring pair per lane, per compute unit.  More pairs per lane
// give each wave independent recurrences to interleave but fewer waves to
// hide latency with.  Measured on MI355X (256 compute units) over
// l_max = 64..4096, nside = l_max / 2, 1..16 maps (bench.py --shape-sweep):
// one pair per lane is fastest up to 8 waves per CU (up to 14% ahead), two
// from 32 on (up to 33% ahead at l_max 4096), four never; the switch sits
// between the two measured points.
struct ChainRule {
    double max_waves_per_cu;
    int chains;
};
constexpr ChainRule kFwdChainTable[] = {
    {16.0, 1},
    {1e300, 2},
};

int default_fwd_chains(const sht_plan_s *p)
{
    const double waves1 = (double)((p->npairs + 63) / 64) * (double)((p->nm + 1) / 2) *
                          (double)p->nmaps / (double)std::max(1, p->num_cus);
    for (const ChainRule &r : kFwdChainTable)
        if (waves1 <= r.max_waves_per_cu) return r.chains;
    return 2;
}

template <class T>
sht_status upload(T **dst, const std::vector<T> &src, size_t *acc)
{
    *dst = nullptr;
    if (src.empty()) return SHT_OK;
    const size_t bytes = src.size() * sizeof(T);
    if (hipMalloc((void **)dst, bytes) != hipSuccess) {
        *dst = nullptr;
        return SHT_ERR_OOM;
    }
    if (hipMemcpy(*dst, src.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return SHT_ERR_HIP;
    *acc += bytes;
    return SHT_OK;
}

void free_tables(sht_plan_s *p)
{
    void *ptrs[] = {p->d_pairs, p->d_mval, p->d_moff, p->d_mu, p->d_A, p->d_cn,
                    p->d_minv, p->d_rings, p->d_pool, p->d_boff, p->d_boff16, p->d_bm16,
                    p->d_bm32, p->d_soff, p->d_sbm, p->d_Asb, p->d_pool32};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    for (int c = 0; c < sht::kNumSynthClasses; ++c) {
        if (p->scls[c].d_ids) (void)hipFree(p->scls[c].d_ids);
        p->scls[c].d_ids = nullptr;
    }
    for (int c = 0; c < sht::kNumRingClasses; ++c) {
        if (p->cls[c].d_ids) (void)hipFree(p->cls[c].d_ids);
        p->cls[c].d_ids = nullptr;
        if (p->bcls[c].d_ids) (void)hipFree(p->bcls[c].d_ids);
        p->bcls[c].d_ids = nullptr;
    }
    p->d_pairs = nullptr; p->d_mval = nullptr; p->d_moff = nullptr; p->d_mu = nullptr;
    p->d_A = nullptr; p->d_cn = nullptr; p->d_minv = nullptr; p->d_rings = nullptr;
    p->d_pool = nullptr; p->d_boff = nullptr; p->d_boff16 = nullptr; p->d_bm16 = nullptr;
    p->d_bm32 = nullptr; p->d_soff = nullptr; p->d_sbm = nullptr; p->d_Asb = nullptr;
    p->d_pool32 = nullptr;
}

sht_status check_plan(sht_plan_t p)
{
    if (!p) return SHT_ERR_BAD_HANDLE;
    if (p->magic != sht::kPlanMagic) return SHT_ERR_BAD_HANDLE;
    sht::clear_stale_error();
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SHT_ERR_HIP;
    if (dev != p->device) return SHT_ERR_INVALID_ARG;
    return SHT_OK;
}

sht_status from_hip(hipError_t e) { return e == hipSuccess ? SHT_OK : SHT_ERR_HIP; }

// Recurrence tables in 80-bit extended precision, rounded once to FP64.
// For each m: beta_l = sqrt((4 l^2 - 1) / (l^2 - m^2)) (Eq. betaDef),
// c_m = c_{m+1} = 1, c_l = (beta_l / beta_{l-1}) c_{l-2}, A_l = beta_l c_{l-1} / c_l,
// A at l = m+1 holds beta_{m+1,m} = sqrt(2m+3) (Eq. pm1m).
void recurrence_tables(int lmax, const std::vector<int32_t> &mval,
                       const std::vector<long long> &moff, std::vector<double> &A,
                       std::vector<double> &cn, std::vector<double> &mu)
{
    const size_t nalm = (size_t)moff.back();
    A.assign(nalm, 0.0);
    cn.assign(nalm, 1.0);
    std::vector<long double> beta(lmax + 2), c(lmax + 2);
    for (size_t i = 0; i < mval.size(); ++i) {
        const int m = mval[i];
        const long double M = m;
        const long long off = moff[i];
        const int len = lmax - m + 1;
        for (int j = 1; j < len; ++j) {
            const long double L = m + j;
            beta[j] = std::sqrt((4.0L * L * L - 1.0L) / (L * L - M * M));
        }
        c[0] = 1.0L;
        if (len > 1) {
            c[1] = 1.0L;
            A[off + 1] = (double)beta[1];
        }
        for (int j = 2; j < len; ++j) {
            c[j] = beta[j] / beta[j - 1] * c[j - 2];
            A[off + j] = (double)(beta[j] * c[j - 1] / c[j]);
        }
        for (int j = 0; j < len; ++j) cn[off + j] = (double)c[j];
    }
    // mu_m (Eq. pmm) as the running product mu_m = mu_{m-1} sqrt((2m+1)/(2m))
    const int mmax = mval.back();
    std::vector<long double> mul(mmax + 1);
    mul[0] = 1.0L / std::sqrt(4.0L * 3.141592653589793238462643383279502884L);
    for (int m = 1; m <= mmax; ++m)
        mul[m] = mul[m - 1] * std::sqrt((2.0L * m + 1.0L) / (2.0L * m));
    mu.resize(mval.size());
    for (size_t i = 0; i < mval.size(); ++i) mu[i] = (double)mul[mval[i]];
}

struct PoolBuilder {
    std::vector<double2> pool;
    std::map<long long, long long> unit;  // length -> offset of e^{2 pi i k/len}

    long long roots(long long len)
    {
        auto it = unit.find(len);
        if (it != unit.end()) return it->second;
        const long long off = (long long)pool.size();
        pool.resize(pool.size() + len);
        const long double tp = 2.0L * 3.141592653589793238462643383279502884L;
        for (long long k = 0; k < len; ++k) {
            const long double a = tp * (long double)k / (long double)len;
            pool[off + k] = make_double2((double)std::cos(a), (double)std::sin(a));
        }
        unit[len] = off;
        return off;
    }
    // c_k = e^{i pi k^2 / len}, k < len, with the exact reduction k^2 mod 2 len
    std::map<long long, long long> chirps;
    long long chirp(long long len)
    {
        auto it = chirps.find(len);
        if (it != chirps.end()) return it->second;
        const long long off = (long long)pool.size();
        pool.resize(pool.size() + len);
        const long double pi = 3.141592653589793238462643383279502884L;
        for (long long k = 0; k < len; ++k) {
            const long long q = (k * k) % (2 * len);
            const long double a = pi * (long double)q / (long double)len;
            pool[off + k] = make_double2((double)std::cos(a), (double)std::sin(a));
        }
        chirps[len] = off;
        return off;
    }
    long long reserve(long long len)
    {
        const long long off = (long long)pool.size();
        pool.resize(pool.size() + len, make_double2(0.0, 0.0));
        return off;
    }
};

}  // namespace

// Delta of the forward transform is complex64 in the mixed forms (the
// precision of their FP32 parity sums) and complex128 in FP64.
static bool delta_f32(const sht_plan_s *p) { return p->precision != SHT_FP64; }

// Prescale + Legendre stage of the forward transform into `delta` (complex64
// for the mixed forms, complex128 for FP64).
static sht_status legendre_stage(sht_plan_t p, const double *alm, void *ws, void *delta,
                                 hipStream_t st, hipEvent_t ev_mid)
{
    hipError_t e;
    float2 *d32 = (float2 *)delta;
    if (p->precision == SHT_FP32_MFMA) {
        e = sht::launch_prescale_f32(p, alm, (float *)ws, st);
        if (e == hipSuccess && ev_mid) e = hipEventRecord(ev_mid, st);
        if (e == hipSuccess) e = sht::launch_legendre_mfma_f32(p, (const float *)ws, d32, st);
    } else if (p->precision == SHT_BF16X3_MFMA) {
        e = sht::launch_prescale_bf16x3(p, alm, ws, st);
        if (e == hipSuccess && ev_mid) e = hipEventRecord(ev_mid, st);
        if (e == hipSuccess) e = sht::launch_legendre_mfma_bf16x3(p, ws, d32, st);
    } else if (p->precision == SHT_F16X2_MFMA) {
        e = sht::launch_prescale_f16x2(p, alm, ws, st);
        if (e == hipSuccess && ev_mid) e = hipEventRecord(ev_mid, st);
        if (e == hipSuccess) e = sht::launch_legendre_mfma_f16x2(p, ws, d32, st);
    } else {
        e = sht::launch_prescale(p, alm, (double2 *)ws, st);
        if (e == hipSuccess && ev_mid) e = hipEventRecord(ev_mid, st);
        if (e == hipSuccess)
            e = sht::launch_legendre_fwd(p, (const double2 *)ws, (double2 *)delta, st);
    }
    return e == hipSuccess ? SHT_OK : SHT_ERR_HIP;
}

// Ring synthesis of the forward transform's Delta (in the workspace).
static hipError_t synth_stage(const sht_plan_s *p, const void *delta, double *map, hipStream_t st)
{
    return delta_f32(p) ? sht::launch_ring_synth(p, (const float2 *)delta, map, st)
                        : sht::launch_ring_synth(p, (const double2 *)delta, map, st);
}

extern "C" {

const char *sht_version(void) { return "0.1.0"; }

const char *sht_status_string(sht_status s)
{
    switch (s) {
    case SHT_OK: return "SHT_OK";
    case SHT_ERR_INVALID_ARG: return "SHT_ERR_INVALID_ARG: invalid argument";
    case SHT_ERR_OOM: return "SHT_ERR_OOM: allocation failed";
    case SHT_ERR_HIP: return "SHT_ERR_HIP: HIP runtime error";
    case SHT_ERR_UNSUPPORTED: return "SHT_ERR_UNSUPPORTED: not supported by this build";
    case SHT_ERR_BAD_HANDLE: return "SHT_ERR_BAD_HANDLE: invalid plan handle";
    case SHT_ERR_WORKSPACE: return "SHT_ERR_WORKSPACE: workspace missing or too small";
    }
    return "unknown sht_status";
}

static size_t fwd_workspace_bytes(const sht_plan_s *p);
static size_t workspace_bytes(const sht_plan_s *p);

sht_status sht_plan(sht_plan_t *out, const sht_geometry_desc *d)
{
    if (!out) return SHT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!d) return SHT_ERR_INVALID_ARG;
    // ---- validate
    if (d->lmax < 0 || d->lmax > SHT_MAX_LMAX) return SHT_ERR_INVALID_ARG;
    if (d->nm < 1 || d->nm > d->lmax + 1) return SHT_ERR_INVALID_ARG;
    if (d->nrings < 1 || d->nmaps < 1) return SHT_ERR_INVALID_ARG;
    if (!d->cth || !d->sth || !d->phi0 || !d->nphi) return SHT_ERR_INVALID_ARG;
    if (d->flags & ~SHT_FLAG_NO_PAIRING) return SHT_ERR_INVALID_ARG;
    if (d->precision != SHT_FP64 && d->precision != SHT_FP32_MFMA &&
        d->precision != SHT_BF16X3_MFMA && d->precision != SHT_F16X2_MFMA)
        return SHT_ERR_UNSUPPORTED;
    sht::clear_stale_error();
    std::vector<int32_t> mval(d->nm);
    for (int i = 0; i < d->nm; ++i) {
        mval[i] = d->mval ? d->mval[i] : i;
        if (mval[i] < 0 || mval[i] > d->lmax) return SHT_ERR_INVALID_ARG;
        if (i && mval[i] <= mval[i - 1]) return SHT_ERR_INVALID_ARG;
    }
    const int R = d->nrings;
    std::vector<long long> start(R);
    long long acc = 0;
    for (int r = 0; r < R; ++r) {
        const double x = d->cth[r], s = d->sth[r];
        if (!(x >= -1.0 && x <= 1.0) || !(s >= 0.0 && s <= 1.0)) return SHT_ERR_INVALID_ARG;
        if (std::fabs(x * x + s * s - 1.0) > 1e-12) return SHT_ERR_INVALID_ARG;
        if (!std::isfinite(d->phi0[r])) return SHT_ERR_INVALID_ARG;
        if (d->nphi[r] < 1) return SHT_ERR_INVALID_ARG;
        if (d->nphi[r] > SHT_MAX_NPHI) return SHT_ERR_UNSUPPORTED;
        if (d->ringstart) {
            if (d->ringstart[r] < 0) return SHT_ERR_INVALID_ARG;
            start[r] = d->ringstart[r];
        } else {
            start[r] = acc;
            acc += d->nphi[r];
        }
    }
    long long npix = 0;
    {
        std::vector<int> ord(R);
        for (int r = 0; r < R; ++r) ord[r] = r;
        std::sort(ord.begin(), ord.end(), [&](int a, int b) { return start[a] < start[b]; });
        for (int t = 0; t < R; ++t) {
            const int r = ord[t];
            if (t + 1 < R && start[r] + d->nphi[r] > start[ord[t + 1]]) return SHT_ERR_INVALID_ARG;
            npix = std::max(npix, start[r] + (long long)d->nphi[r]);
        }
    }
    if (d->npix < 0 || (d->npix > 0 && d->npix < npix)) return SHT_ERR_INVALID_ARG;
    if (d->npix > 0) npix = d->npix;
    // ---- Fourier classification per ring
    std::vector<RingDesc> rings(R);
    std::vector<int> ring_class(R), ring_sclass(R);
    sht::RingLds class_lds[sht::kNumRingClasses] = {};
    sht::RingLds sclass_lds[sht::kNumSynthClasses] = {};
    std::vector<int> ring_bclass(R, -1);
    sht::RingLds bclass_lds[sht::kNumRingClasses] = {};
    // the Bluestein fast path takes complex64 Delta (the mixed forms)
    const bool blue_ok = d->precision != SHT_FP64 && mval.back() < sht::kFastMaxModes;
    for (int r = 0; r < R; ++r) {
        const long long n = d->nphi[r];
        RingDesc &g = rings[r];
        std::memset(&g, 0, sizeof g);
        g.start = start[r];
        g.phi0 = d->phi0[r];
        g.n = (int)n;
        g.clen = (int)((n % 2 == 0) ? n / 2 : n);
        g.tw = g.tch = g.twb = g.bq = -1;
        const int spec = (n % 2 == 0) ? g.clen + 1 : g.clen;  // F_k entries
        int fftlen;
        unsigned long long fr = 0;
        if (smooth7(g.clen) && g.clen <= 8192) {
            g.nb = 0;
            fftlen = g.clen;
            // an even ring of 7-smooth half length that the fast path cannot
            // take (a pass would hold too many butterflies per thread) joins
            // the Bluestein fast path
            if (blue_ok && n % 2 == 0 && g.clen % 2 == 0 && sht::fast_radices(g.clen, &fr) == 0) {
                const int nbb = best_blue_nb((long long)g.clen - 1);
                if (nbb > 0) {
                    g.half = 1;
                    g.nb = nbb;
                    fftlen = nbb;
                }
            }
        } else if (n % 2 == 0 && g.clen % 2 == 0) {
            // split into the even- and odd-indexed halves: Bluestein of
            // length clen / 2 needs a convolution of only clen - 1 points
            g.half = 1;
            const int nbb = blue_ok ? best_blue_nb((long long)g.clen - 1) : 0;
            g.nb = nbb > 0 ? nbb : best_smooth7((long long)g.clen - 1);
            if (g.nb > 8192) return SHT_ERR_UNSUPPORTED;
            fftlen = g.nb;
        } else {
            g.nb = best_smooth7(2LL * g.clen - 1);
            if (g.nb > 8192) return SHT_ERR_UNSUPPORTED;
            fftlen = g.nb;
        }
        const int need = std::max(spec, fftlen);
        const int c = fftlen <= 2048 ? 0 : (fftlen <= 4096 ? 1 : 2);
        ring_class[r] = c;
        sht::ring_lds_add(class_lds[c], c, g.n, g.nb, need);
        g.np = (n % 2 == 0 && g.nb == 0 && mval.back() < sht::kFastMaxModes)
                   ? sht::fast_radices(g.clen, &g.rads) : 0;
        if (g.np == 0 && g.half && blue_ok) g.np = sht::blue_radices(g.nb, &g.rads);
        if (g.np > 0 && g.nb == 0) {
            ring_sclass[r] = sht::kFastClass;
            sht::fast_lds_add(sclass_lds[sht::kFastClass], g.n, mval.back());
        } else if (g.np > 0) {
            ring_sclass[r] = sht::kBlueClass;
            sht::blue_lds_add(sclass_lds[sht::kBlueClass], g.n, g.nb, mval.back());
            ring_bclass[r] = c;
            sht::ring_lds_add(bclass_lds[c], c, g.n, g.nb, need);
        } else {
            ring_sclass[r] = c;
            sht::ring_lds_add(sclass_lds[c], c, g.n, g.nb, need);
        }
    }

    sht_plan_s *p = new (std::nothrow) sht_plan_s();
    if (!p) return SHT_ERR_OOM;
    p->magic = 0;
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return SHT_ERR_HIP; }
    p->lmax = d->lmax;
    p->nm = d->nm;
    p->mmax = mval.back();
    p->nrings = R;
    p->nmaps = d->nmaps;
    p->precision = d->precision;
    p->flags = d->flags;
    p->num_cus = 0;
    if (hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
        hipSuccess) {
        delete p;
        return SHT_ERR_HIP;
    }
    p->npix = npix;
    p->mval = mval;
    p->moff.resize(d->nm + 1);
    p->moff[0] = 0;
    for (int i = 0; i < d->nm; ++i) p->moff[i + 1] = p->moff[i] + (d->lmax - mval[i] + 1);
    p->nalm = p->moff.back();
    p->ring_class = ring_class;
    p->ring_sclass = ring_sclass;
    p->ring_need.resize(R);
    p->ring_n.resize(R);
    p->ring_nb.resize(R);
    for (int r = 0; r < R; ++r) {
        const RingDesc &g = rings[r];
        const int spec = (g.n % 2 == 0) ? g.clen + 1 : g.clen;
        p->ring_need[r] = std::max(spec, g.nb ? g.nb : g.clen);
        p->ring_n[r] = g.n;
        p->ring_nb[r] = g.nb;
    }
    p->mcontig = 1;
    for (int i = 0; i < d->nm; ++i)
        if (mval[i] != i) p->mcontig = 0;

    // ---- pairing of mirror rings (cos negated bitwise, sin equal)
    std::vector<PairDesc> pairs;
    {
        std::vector<char> used(R, 0);
        std::unordered_map<std::pair<uint64_t, uint64_t>, std::vector<int>, PairKeyHash> south;
        if (!(d->flags & SHT_FLAG_NO_PAIRING)) {
            for (int r = R - 1; r >= 0; --r)
                if (d->cth[r] < 0.0) south[{bits(d->cth[r]), bits(d->sth[r])}].push_back(r);
            for (int r = 0; r < R; ++r) {
                if (!(d->cth[r] > 0.0)) continue;
                auto it = south.find({bits(-d->cth[r]), bits(d->sth[r])});
                if (it == south.end() || it->second.empty()) continue;
                const int rs = it->second.back();
                it->second.pop_back();
                used[r] = used[rs] = 1;
                pairs.push_back({d->cth[r], d->sth[r], r, rs});
            }
        }
        for (int r = 0; r < R; ++r)
            if (!used[r]) pairs.push_back({d->cth[r], d->sth[r], r, -1});
    }
    p->npairs = (int)pairs.size();

    std::vector<double> A, cn, mu;
    recurrence_tables(d->lmax, mval, p->moff, A, cn, mu);
    std::vector<int32_t> minv(p->mmax + 1, -1);
    for (int i = 0; i < d->nm; ++i) minv[mval[i]] = i;

    // ---- twiddle / chirp / Bluestein tables
    PoolBuilder pb;
    std::vector<int> prep_ids;
    std::map<int, long long> bq_of_len;
    for (int r = 0; r < R; ++r) {
        RingDesc &g = rings[r];
        g.tw = pb.roots(g.n);
        if (g.nb) {
            const int blen = g.half ? g.clen / 2 : g.clen;   // Bluestein length
            g.tch = pb.chirp(blen);
            g.twb = pb.roots(g.nb);
            auto it = bq_of_len.find(blen);
            if (it == bq_of_len.end()) {
                g.bq = pb.reserve(g.nb);
                bq_of_len[blen] = g.bq;
                prep_ids.push_back(r);
            } else {
                g.bq = it->second;
            }
        }
    }
    p->pool_entries = pb.pool.size();

    sht_status st = SHT_OK;
    size_t tb = 0;
    if (st == SHT_OK) st = upload(&p->d_pairs, pairs, &tb);
    if (st == SHT_OK) st = upload(&p->d_mval, mval, &tb);
    if (st == SHT_OK) st = upload(&p->d_moff, p->moff, &tb);
    if (st == SHT_OK) st = upload(&p->d_mu, mu, &tb);
    // 128 zero coefficients past the end: whole 16-row blocks and 128-row
    // super-blocks may be read unguarded (the mixed kernel's recurrence-only
    // phase and its copies to LDS)
    A.resize(A.size() + 128, 0.0);
    if (st == SHT_OK) st = upload(&p->d_A, A, &tb);
    if (st == SHT_OK) st = upload(&p->d_cn, cn, &tb);
    if (st == SHT_OK) st = upload(&p->d_minv, minv, &tb);
    if (st == SHT_OK) {
        std::vector<long long> boff(d->nm);
        long long acc_b = 0;
        for (int i = 0; i < d->nm; ++i) {
            boff[i] = acc_b;
            acc_b += (d->lmax - mval[i] + 1 + 31) / 32;
        }
        st = upload(&p->d_boff, boff, &tb);
        if (st == SHT_OK) {
            std::vector<int32_t> bm32((size_t)acc_b);
            for (int i = 0; i < d->nm; ++i) {
                const long long e = (i + 1 < d->nm) ? boff[i + 1] : acc_b;
                for (long long b = boff[i]; b < e; ++b) bm32[(size_t)b] = i;
            }
            st = upload(&p->d_bm32, bm32, &tb);
        }
    }
    if (st == SHT_OK) {
        std::vector<long long> boff16(d->nm);
        long long acc_b = 0;
        for (int i = 0; i < d->nm; ++i) {
            boff16[i] = acc_b;
            acc_b += (d->lmax - mval[i] + 1 + 15) / 16;
        }
        p->nblk16 = acc_b;
        st = upload(&p->d_boff16, boff16, &tb);
        if (st == SHT_OK) {
            std::vector<int32_t> bm16((size_t)acc_b);
            for (int i = 0; i < d->nm; ++i) {
                const long long e = (i + 1 < d->nm) ? boff16[i + 1] : acc_b;
                for (long long b = boff16[i]; b < e; ++b) bm16[(size_t)b] = i;
            }
            st = upload(&p->d_bm16, bm16, &tb);
        }
    }
    if (st == SHT_OK && p->precision != SHT_FP64) {
        // mixed forms: super-blocks of 128 rows per m, and the recurrence
        // coefficients copied per super-block with zeros past each m's last
        // row (the kernels' super-block copies run past an m's end)
        const int SR = sht::f16_super_rows();
        std::vector<long long> soff(d->nm);
        long long acc_s = 0;
        for (int i = 0; i < d->nm; ++i) {
            soff[i] = acc_s;
            acc_s += (d->lmax - mval[i] + 1 + SR - 1) / SR;
        }
        p->nsuper = acc_s;
        std::vector<int32_t> sbm((size_t)acc_s);
        std::vector<double> Asb((size_t)acc_s * SR, 0.0);
        for (int i = 0; i < d->nm; ++i) {
            const long long e = (i + 1 < d->nm) ? soff[i + 1] : acc_s;
            for (long long b = soff[i]; b < e; ++b) sbm[(size_t)b] = i;
            const int len = d->lmax - mval[i] + 1;
            for (int j = 0; j < len; ++j)
                Asb[(size_t)soff[i] * SR + j] = A[(size_t)p->moff[i] + j];
        }
        st = upload(&p->d_soff, soff, &tb);
        if (st == SHT_OK) st = upload(&p->d_sbm, sbm, &tb);
        if (st == SHT_OK) st = upload(&p->d_Asb, Asb, &tb);
    }
    if (st == SHT_OK) st = upload(&p->d_rings, rings, &tb);
    if (st == SHT_OK) st = upload(&p->d_pool, pb.pool, &tb);
    // longest rings first (tail balance); rings of equal length adjacent so
    // that consecutive workgroups, which the kernels place on one XCD, share
    // twiddle and Bluestein tables in L2
    auto class_ids = [&](const std::vector<int> &cls_of, int c) {
        std::vector<int> ids;
        for (int r = 0; r < R; ++r)
            if (cls_of[r] == c) ids.push_back(r);
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
            return d->nphi[a] > d->nphi[b];
        });
        return ids;
    };
    for (int c = 0; c < sht::kNumRingClasses && st == SHT_OK; ++c) {
        const std::vector<int> ids = class_ids(ring_class, c);
        p->cls[c].count = (int)ids.size();
        p->cls[c].lds = class_lds[c];
        st = upload(&p->cls[c].d_ids, ids, &tb);
    }
    for (int c = 0; c < sht::kNumSynthClasses && st == SHT_OK; ++c) {
        const std::vector<int> ids = class_ids(ring_sclass, c);
        p->scls[c].count = (int)ids.size();
        p->scls[c].lds = sclass_lds[c];
        st = upload(&p->scls[c].d_ids, ids, &tb);
    }
    for (int c = 0; c < sht::kNumRingClasses && st == SHT_OK; ++c) {
        const std::vector<int> ids = class_ids(ring_bclass, c);
        p->bcls[c].count = (int)ids.size();
        p->bcls[c].lds = bclass_lds[c];
        st = upload(&p->bcls[c].d_ids, ids, &tb);
    }
    if (st == SHT_OK && !prep_ids.empty()) {
        int *d_ids = nullptr;
        if (hipMalloc((void **)&d_ids, prep_ids.size() * sizeof(int)) != hipSuccess) {
            st = SHT_ERR_OOM;
        } else {
            if (hipMemcpy(d_ids, prep_ids.data(), prep_ids.size() * sizeof(int),
                          hipMemcpyHostToDevice) != hipSuccess ||
                sht::launch_bluestein_prep(p, d_ids, (int)prep_ids.size(), nullptr) != hipSuccess ||
                hipDeviceSynchronize() != hipSuccess)
                st = SHT_ERR_HIP;
            (void)hipFree(d_ids);
        }
    }
    // the mixed forms' fast paths read their tables (twiddles, kernel
    // spectra) in complex64: 8-byte loads, no conversions in the passes
    if (st == SHT_OK && delta_f32(p) &&
        p->scls[sht::kBlueClass].count + p->scls[sht::kFastClass].count > 0) {
        const size_t bytes = p->pool_entries * sizeof(float2);
        if (hipMalloc((void **)&p->d_pool32, bytes) != hipSuccess) {
            p->d_pool32 = nullptr;
            st = SHT_ERR_OOM;
        } else if (sht::launch_narrow(p->d_pool, p->d_pool32, (long long)p->pool_entries,
                                      nullptr) != hipSuccess ||
                   hipDeviceSynchronize() != hipSuccess) {
            st = SHT_ERR_HIP;
        } else {
            tb += bytes;
        }
    }
    if (st != SHT_OK) {
        free_tables(p);
        delete p;
        return st;
    }
    p->table_bytes = tb;
    p->ws_ap_bytes = align_up(
        p->precision == SHT_FP32_MFMA     ? sht::mfma_bf_bytes(p)
        : p->precision == SHT_BF16X3_MFMA ? sht::bf16_bytes(p)
        : p->precision == SHT_F16X2_MFMA  ? sht::f16_bytes(p)
                                          : (size_t)p->nmaps * (size_t)p->nalm * sizeof(double2),
        256);
    p->ws_dt_bytes = align_up((size_t)p->nmaps * (size_t)R * (size_t)p->nm * sizeof(double2), 256);
    p->ws_delta_bytes = align_up((size_t)p->nmaps * (size_t)R * (size_t)p->nm *
                                     (delta_f32(p) ? sizeof(float2) : sizeof(double2)),
                                 256);
    p->fwd_chains = default_fwd_chains(p);
    p->aux_stream = nullptr;
    p->ev_fork = p->ev_join = nullptr;
    if (hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
        if (p->aux_stream) (void)hipStreamDestroy(p->aux_stream);
        free_tables(p);
        delete p;
        return SHT_ERR_HIP;
    }
    p->magic = sht::kPlanMagic;
    if (sht::log_enabled()) {
        static const char *kPrec[] = {"fp64", "fp32_mfma", "bf16x3_mfma", "f16x2_mfma"};
        int nblue = 0, nfast = 0;
        for (int r = 0; r < R; ++r) {
            nblue += rings[r].nb != 0 && ring_sclass[r] != sht::kBlueClass;
            nfast += ring_sclass[r] == sht::kFastClass;
        }
        sht::log_line("plan l_max=%d nm=%d m_max=%d rings=%d pairs=%d maps=%d precision=%s "
                      "delta=%s", p->lmax, p->nm, p->mmax, R, p->npairs, p->nmaps,
                      kPrec[p->precision], delta_f32(p) ? "complex64" : "complex128");
        sht::log_line("plan synthesis rings: fast path %d (Stockham in registers), Bluestein "
                      "fast path %d, size classes %d / %d / %d (256 / 512 / 1024 threads), of "
                      "which Bluestein %d",
                      nfast, p->scls[sht::kBlueClass].count, p->scls[0].count,
                      p->scls[1].count, p->scls[2].count, nblue);
        // the radix lists of the three longest fast-path ring lengths
        std::map<int, int> longest;   // nphi -> a ring of that length
        for (int r = 0; r < R; ++r)
            if (ring_sclass[r] == sht::kFastClass) longest[-rings[r].n] = r;
        int shown = 0;
        for (const auto &kv : longest) {
            if (shown++ == 3) break;
            const sht::RingDesc &g = rings[kv.second];
            char rl[64];
            int o = 0;
            for (int q = 0; q < g.np; ++q)
                o += std::snprintf(rl + o, sizeof rl - o, q ? "x%d" : "%d",
                                   (int)((g.rads >> (5 * q)) & 31));
            sht::log_line("plan fast ring nphi=%d: half length %d = %s", g.n, g.clen, rl);
        }
        sht::log_line("plan workspace forward=%zu full=%zu bytes, device tables=%zu bytes; "
                      "FP64 forward launch shape %d pair(s) per lane (size table)",
                      fwd_workspace_bytes(p), workspace_bytes(p), p->table_bytes,
                      p->fwd_chains);
    }
    *out = p;
    return SHT_OK;
}

sht_status sht_plan_destroy(sht_plan_t p)
{
    if (!p || p->magic != sht::kPlanMagic) return SHT_ERR_BAD_HANDLE;
    p->magic = sht::kDeadMagic;
    (void)hipEventDestroy(p->ev_join);
    (void)hipEventDestroy(p->ev_fork);
    (void)hipStreamDestroy(p->aux_stream);
    free_tables(p);
    delete p;
    return SHT_OK;
}

// Synthesis needs the prescaled coefficients and Delta; the adjoint needs
// Delta~ and the per-ring-block partial sums, which dominate for many maps.
static size_t fwd_workspace_bytes(const sht_plan_s *p)
{
    return p->ws_ap_bytes + p->ws_delta_bytes;
}

static size_t workspace_bytes(const sht_plan_s *p)
{
    const size_t fwd = fwd_workspace_bytes(p);
    const size_t adj = p->ws_dt_bytes + align_up(sht::adj_part_bytes(p), 256);
    return std::max(fwd, adj);
}

sht_status sht_plan_workspace_size(sht_plan_t p, size_t *bytes)
{
    if (!p || p->magic != sht::kPlanMagic) return SHT_ERR_BAD_HANDLE;
    if (!bytes) return SHT_ERR_INVALID_ARG;
    *bytes = workspace_bytes(p);
    return SHT_OK;
}

sht_status sht_plan_get_info(sht_plan_t p, sht_plan_info *info)
{
    if (!p || p->magic != sht::kPlanMagic) return SHT_ERR_BAD_HANDLE;
    if (!info) return SHT_ERR_INVALID_ARG;
    info->nalm = p->nalm;
    info->npix = p->npix;
    info->nrings = p->nrings;
    info->npairs = p->npairs;
    info->nm = p->nm;
    info->lmax = p->lmax;
    info->mmax = p->mmax;
    info->nmaps = p->nmaps;
    info->workspace_bytes = workspace_bytes(p);
    info->forward_workspace_bytes = fwd_workspace_bytes(p);
    info->delta_bytes = (size_t)p->nmaps * (size_t)p->nrings * (size_t)p->nm * sizeof(double2);
    info->table_bytes = p->table_bytes;
    return SHT_OK;
}

sht_status sht_alm2delta(sht_plan_t p, const double *alm, double *delta, void *ws,
                         size_t ws_bytes, void *stream)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!alm || !delta) return SHT_ERR_INVALID_ARG;
    if (!delta_f32(p)) {
        if (!ws || ws_bytes < p->ws_ap_bytes) return SHT_ERR_WORKSPACE;
        return legendre_stage(p, alm, ws, delta, (hipStream_t)stream, nullptr);
    }
    // mixed forms: complex64 Delta in the workspace, widened into the caller's buffer
    if (!ws || ws_bytes < fwd_workspace_bytes(p)) return SHT_ERR_WORKSPACE;
    float2 *d32 = (float2 *)((char *)ws + p->ws_ap_bytes);
    s = legendre_stage(p, alm, ws, d32, (hipStream_t)stream, nullptr);
    if (s == SHT_OK)
        s = from_hip(sht::launch_widen_delta(p, d32, (double2 *)delta, (hipStream_t)stream));
    return s;
}

sht_status sht_delta2map(sht_plan_t p, const double *delta, double *map, void *stream)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!delta || !map) return SHT_ERR_INVALID_ARG;
    return from_hip(sht::launch_ring_synth(p, (const double2 *)delta, map, (hipStream_t)stream));
}

}  // extern "C"

namespace sht {

bool log_enabled()
{
    static const bool on = [] {
        const char *v = std::getenv("SHT_LOG");
        return v && v[0] && std::strcmp(v, "0") != 0;
    }();
    return on;
}

void log_line(const char *fmt, ...)
{
    if (!log_enabled()) return;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "sht: %s\n", buf);
}

size_t forward_workspace(const sht_plan_s *p) { return fwd_workspace_bytes(p); }

sht_status check_plan_device(sht_plan_t p) { return check_plan(p); }

sht_status forward_transform(sht_plan_t p, const double *alm, double *map, void *ws,
                             hipStream_t st)
{
    void *delta = (char *)ws + p->ws_ap_bytes;
    sht_status s = legendre_stage(p, alm, ws, delta, st, nullptr);
    if (s == SHT_OK) s = from_hip(synth_stage(p, delta, map, st));
    return s;
}

}  // namespace sht

extern "C" {

sht_status sht_alm2map(sht_plan_t p, const double *alm, double *map, void *ws, size_t ws_bytes,
                       void *stream)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!alm || !map) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < fwd_workspace_bytes(p)) return SHT_ERR_WORKSPACE;
    return sht::forward_transform(p, alm, map, ws, (hipStream_t)stream);
}

sht_status sht_plan_get_config(sht_plan_t p, int32_t *chains)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!chains) return SHT_ERR_INVALID_ARG;
    *chains = p->fwd_chains;
    return SHT_OK;
}

sht_status sht_plan_set_config(sht_plan_t p, int32_t chains)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (p->precision != SHT_FP64) return SHT_ERR_UNSUPPORTED;
    if (chains != 1 && chains != 2 && chains != 4) return SHT_ERR_INVALID_ARG;
    const long long pblocks = (p->npairs + 64LL * chains - 1) / (64LL * chains);
    if (pblocks * ((p->nm + 1) / 2) * p->nmaps > 0x7fffffffLL) return SHT_ERR_UNSUPPORTED;
    p->fwd_chains = chains;
    return SHT_OK;
}

sht_status sht_plan_autotune(sht_plan_t p, const double *alm, double *map, void *ws,
                             size_t ws_bytes, const char *cache_path, void *stream)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!alm || !map) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < fwd_workspace_bytes(p)) return SHT_ERR_WORKSPACE;
    if (p->precision != SHT_FP64) return SHT_OK;   // nothing to tune
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) return SHT_ERR_HIP;
    std::ostringstream sig;
    sig << prop.gcnArchName << "|fp64fwd|" << p->lmax << ":" << p->nm << ":" << p->mmax << ":"
        << p->nrings << ":" << p->npairs << ":" << p->npix << ":" << p->nmaps;
    const std::string key = sig.str();
    // cache: one line per tuned plan, "<signature> <chains> <ms per transform>"
    if (cache_path && cache_path[0]) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int ch = 0;
            double ms = 0;
            if ((ls >> k >> ch >> ms) && k == key && sht_plan_set_config(p, ch) == SHT_OK)
                return SHT_OK;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SHT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SHT_ERR_HIP; }
    const int start = p->fwd_chains;
    float best = 1e30f;
    int best_ch = start;
    for (int ch : {1, 2, 4}) {
        if (sht_plan_set_config(p, ch) != SHT_OK) continue;
        s = sht_alm2map(p, alm, map, ws, ws_bytes, stream);   // warm-up
        if (s != SHT_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { s = SHT_ERR_HIP; break; }
        for (int r = 0; r < 3 && s == SHT_OK; ++r) s = sht_alm2map(p, alm, map, ws, ws_bytes, stream);
        if (s != SHT_OK || hipEventRecord(e1, st) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess) {
            s = s == SHT_OK ? SHT_ERR_HIP : s;
            break;
        }
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { s = SHT_ERR_HIP; break; }
        if (ms < best) { best = ms; best_ch = ch; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->fwd_chains = (s == SHT_OK) ? best_ch : start;
    if (s == SHT_OK)
        sht::log_line("autotune plan: %d pair(s) per lane, %.3f ms per call", best_ch, best / 3);
    if (s != SHT_OK) return s;
    if (cache_path && cache_path[0]) {
        std::ofstream outf(cache_path, std::ios::app);
        if (outf) outf << key << " " << best_ch << " " << best / 3 << "\n";
    }
    return SHT_OK;
}

sht_status sht_alm2map_events(sht_plan_t p, const double *alm, double *map, void *ws,
                              size_t ws_bytes, void *stream, void *const *events)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!alm || !map || !events) return SHT_ERR_INVALID_ARG;
    for (int k = 0; k < 4; ++k)
        if (!events[k]) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < fwd_workspace_bytes(p)) return SHT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    void *delta = (char *)ws + p->ws_ap_bytes;
    s = from_hip(hipEventRecord((hipEvent_t)events[0], st));
    if (s == SHT_OK) s = legendre_stage(p, alm, ws, delta, st, (hipEvent_t)events[1]);
    if (s == SHT_OK) s = from_hip(hipEventRecord((hipEvent_t)events[2], st));
    if (s == SHT_OK) s = from_hip(synth_stage(p, delta, map, st));
    if (s == SHT_OK) s = from_hip(hipEventRecord((hipEvent_t)events[3], st));
    return s;
}

sht_status sht_map2delta_adjoint(sht_plan_t p, const double *map, double *delta, void *stream)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!delta || !map) return SHT_ERR_INVALID_ARG;
    return from_hip(sht::launch_ring_anal(p, map, (double2 *)delta, (hipStream_t)stream));
}

sht_status sht_delta2alm_adjoint(sht_plan_t p, const double *delta, double *alm, void *ws,
                                 size_t ws_bytes, void *stream)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!delta || !alm) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < sht::adj_part_bytes(p)) return SHT_ERR_WORKSPACE;
    return from_hip(sht::launch_legendre_adj_ws(p, (const double2 *)delta, (double2 *)ws, alm,
                                                (hipStream_t)stream));
}

sht_status sht_alm2map_adjoint(sht_plan_t p, const double *map, double *alm, void *ws,
                               size_t ws_bytes, void *stream)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!alm || !map) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < workspace_bytes(p)) return SHT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double2 *dt = (double2 *)ws;
    double2 *part = (double2 *)((char *)ws + p->ws_dt_bytes);
    s = from_hip(sht::launch_ring_anal(p, map, dt, st));
    if (s == SHT_OK) s = from_hip(sht::launch_legendre_adj_ws(p, dt, part, alm, st));
    return s;
}

sht_status sht_map2alm(sht_plan_t p, const double *map, const double *ring_weight, double *alm,
                       int32_t niter, double *tmp_map, void *ws, size_t ws_bytes, void *stream)
{
    sht_status s = check_plan(p);
    if (s != SHT_OK) return s;
    if (!map || !alm || !ring_weight || niter < 0 || niter > SHT_MAX_MAP2ALM_ITER)
        return SHT_ERR_INVALID_ARG;
    if (niter > 0 && !tmp_map) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < workspace_bytes(p)) return SHT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double2 *dt = (double2 *)ws;
    double2 *part = (double2 *)((char *)ws + p->ws_dt_bytes);
    void *delta = (char *)ws + p->ws_ap_bytes;
    // a = D adjoint(w s): the analysis with c_m = 1 for every m
    s = from_hip(sht::launch_ring_anal(p, map, dt, st, ring_weight, 1.0));
    if (s == SHT_OK) s = from_hip(sht::launch_legendre_adj_ws(p, dt, part, alm, st, false));
    // a <- a + D adjoint(w (s - alm2map(a)))
    for (int it = 0; it < niter && s == SHT_OK; ++it) {
        s = legendre_stage(p, alm, ws, delta, st, nullptr);
        if (s == SHT_OK) s = from_hip(synth_stage(p, delta, tmp_map, st));
        if (s == SHT_OK)
            s = from_hip(sht::launch_residual(map, tmp_map, (long long)p->nmaps * p->npix, st));
        if (s == SHT_OK) s = from_hip(sht::launch_ring_anal(p, tmp_map, dt, st, ring_weight, 1.0));
        if (s == SHT_OK) s = from_hip(sht::launch_legendre_adj_ws(p, dt, part, alm, st, true));
    }
    return s;
}

}  // extern "C"
