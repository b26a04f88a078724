// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "sht.h"

namespace sht {

constexpr uint64_t kPlanMagic = 0x53485450'4c414e31ull;  // "SHTPLAN1"
constexpr uint64_t kDeadMagic = 0xdeadbeefdeadbeefull;

// Values of the Legendre recurrence are carried as v * 2^(kScaleStep * k),
// k <= 0 (Sec. 2.2.2: real-time rescaling).  A value is rescaled when its
// magnitude exceeds 2^kScaleStep; checks happen every 8 steps, over which
// the normalised recurrence grows by less than 2^140 for l <= 16383, so
// |v| < 2^652 always.  Terms with k <= -2 are below 2^-372 and dropped.
constexpr int kScaleStep = 512;

// Per-ring description for the Fourier kernels (device side).
struct RingDesc {
    long long start;  // first pixel of the ring in the map
    long long tw;     // offset (double2) of e^{+2 pi i k / n}, k < n
    long long tch;    // offset of the Bluestein chirp e^{i pi k^2 / clen}, k < clen
    long long twb;    // offset of e^{+2 pi i k / nb}, k < nb (Bluestein FFT)
    long long bq;     // offset of the Bluestein kernel spectrum (nb entries)
    double phi0;
    int n;            // pixels in the ring
    int clen;         // complex FFT length: n / 2 (n even) or n (n odd)
    int nb;           // Bluestein convolution length (7-smooth), 0 if clen is 7-smooth
    int half;         // 1: the clen-point DFT is two Bluestein DFTs of length clen / 2
                      // (even- and odd-indexed inputs) and one radix-2 step; the
                      // chirp, nb and kernel spectrum are those of length clen / 2
    int np;           // synthesis fast path: number of Stockham passes (0: not on it)
    int pad;
    unsigned long long rads;  // their radices (16, 8, 4, 2, 7, 5, 3; product clen),
                              // 5 bits each, pass p at bits 5p..5p+4
};

// One recurrence unit: a ring, or a ring and its mirror (cos negated,
// same sin), processed together through the parity P_lm(-x) = (-1)^(l+m) P_lm(x).
struct PairDesc {
    double x;     // cos(theta) of the northern member
    double s;     // sin(theta)
    int rn;       // ring index of the northern member
    int rs;       // ring index of the southern member, -1 if unpaired
};

// Rings grouped by FFT length for the Fourier kernels (LDS and register
// budgets differ per class): class 0 up to 2048 points, 1 up to 4096, 2 up to 8192.
// Element strides of a Delta buffer, and the order of the ring stage's
// (map, ring) items.  complex128 Delta (the FP64 Legendre stage's, or a
// caller's) is [map][m][ring]: neighbouring rings of one map share cache
// lines, so the items run map by map.  The mixed forms' complex64 Delta is
// [m][ring][map]: the maps of one ring share lines, so the items run ring by
// ring.
struct DeltaLayout {
    long long map;    // stride between maps
    long long ring;   // between rings
    long long m;      // between the modes of one (map, ring)
};

// LDS of a ring-class workgroup, in complex entries: the spectrum / FFT
// buffer (which also stages partial alias sums during the fold), the second
// convolution buffer of the Bluestein fast path (y, 0 elsewhere), and the
// two-level twiddle tables of the ring length (tw) and of the Bluestein
// length (tb), in that order.
struct RingLds {
    int fft_entries;
    int tw_entries;
    int tb_entries;
    int y_entries;
    int total() const { return fft_entries + y_entries + tw_entries + tb_entries; }
};

struct RingClass {
    int count;        // rings in the class
    RingLds lds;
    int *d_ids;       // device [count] ring indices
};
constexpr int kNumRingClasses = 3;
constexpr int kClassThreads[kNumRingClasses] = {256, 512, 1024};
// Synthesis uses the three classes above for the rings that are not on the
// fast path, plus one class for the fast path: even rings whose half length
// is 7-smooth and at most kFastMaxH, run by kFastThreads-thread workgroups
// with register-held radix-16/8/4/2/7/5/3 butterflies on a padded LDS buffer.
// Mixed-form plans (complex64 Delta) add a Bluestein fast path: even rings
// whose half length h = 2 len has a len that is not 7-smooth, with a
// convolution length nb <= kBlueMaxN, run by kBlueThreads-thread workgroups
// that take the even- and odd-indexed convolutions side by side.
constexpr int kFastClass = 3;
constexpr int kBlueClass = 4;
constexpr int kNumSynthClasses = 5;
constexpr int kFastThreads = 256;
constexpr int kFastMaxH = 4096;
constexpr int kFastMaxModes = 17 * kFastThreads;   // the fold holds m < 4352 in registers
constexpr int kBlueThreads = 512;
constexpr int kBlueMaxN = 4096;
// padded LDS index of the fast path (one spare entry per 16)
inline int fast_pad(int i) { return i + (i >> 4); }
// butterflies per thread a fast pass of radix R holds in registers (at most
// 16 complex values)
__host__ __device__ constexpr int fast_maxq(int R)
{
    return R == 16 ? 1 : R == 8 ? 2 : R == 4 ? 4 : R == 2 ? 8 : R == 7 ? 2 : R == 5 ? 3 : 5;
}

// Radices of the fast path for a complex length h (1 < h <= kFastMaxH,
// 7-smooth): as many 16s as possible, then 8, 4, 2, then 7, 5, 3.  Returns
// the number of passes, 0 if h is not eligible (also when a pass would need
// more butterflies per thread than fast_maxq).
inline int fast_radices(int h, unsigned long long *rads)
{
    int rad[12];
    if (h < 2 || h > kFastMaxH) return 0;
    int np = 0, r = h;
    while (r % 16 == 0 && np < 12) { rad[np++] = 16; r /= 16; }
    if (r % 8 == 0 && np < 12) { rad[np++] = 8; r /= 8; }
    if (r % 4 == 0 && np < 12) { rad[np++] = 4; r /= 4; }
    if (r % 2 == 0 && np < 12) { rad[np++] = 2; r /= 2; }
    for (int f : {7, 5, 3})
        while (r % f == 0 && np < 12) { rad[np++] = f; r /= f; }
    if (r != 1) return 0;
    *rads = 0;
    for (int p = 0; p < np; ++p) {
        if (h / rad[p] > fast_maxq(rad[p]) * kFastThreads) return 0;
        *rads |= (unsigned long long)rad[p] << (5 * p);
    }
    return np;
}

// Radices of the Bluestein fast path for a convolution length nb (7-smooth,
// 1 < nb <= kBlueMaxN): as many 8s as possible, then 4, 2, 7, 5, 3.  Every
// pass holds at most one butterfly per thread (nb / R <= kBlueThreads).
// Returns the number of passes, 0 if nb is not eligible.
inline int blue_radices(int nb, unsigned long long *rads)
{
    int rad[12];
    if (nb < 2 || nb > kBlueMaxN) return 0;
    int np = 0, r = nb;
    while (r % 8 == 0 && np < 12) { rad[np++] = 8; r /= 8; }
    if (r % 4 == 0 && np < 12) { rad[np++] = 4; r /= 4; }
    if (r % 2 == 0 && np < 12) { rad[np++] = 2; r /= 2; }
    for (int f : {7, 5, 3})
        while (r % f == 0 && np < 12) { rad[np++] = f; r /= f; }
    if (r != 1) return 0;
    *rads = 0;
    for (int p = 0; p < np; ++p) {
        if (nb / rad[p] > kBlueThreads) return 0;
        *rads |= (unsigned long long)rad[p] << (5 * p);
    }
    return np;
}

// Grows the Bluestein fast class layout by one ring of n pixels and
// convolution length nb for modes 0..mmax: the first buffer holds the phased
// modes, the spectrum and the alias staging, then the even-indexed
// convolution; the second the odd-indexed one; then the twiddle tables of
// n and nb.
inline void blue_lds_add(RingLds &l, int n, int nb, int mmax)
{
    int top = n / 2 > kBlueThreads - 1 ? n / 2 : kBlueThreads - 1;
    top = top > mmax ? top : mmax;
    top = top > nb - 1 ? top : nb - 1;
    const int need = fast_pad(top) + 1;
    l.fft_entries = l.fft_entries > need ? l.fft_entries : need;
    const int y = fast_pad(nb - 1) + 1;
    l.y_entries = l.y_entries > y ? l.y_entries : y;
    const int tw = 64 + (n + 63) / 64;
    l.tw_entries = l.tw_entries > tw ? l.tw_entries : tw;
    const int tb = 64 + (nb + 63) / 64;
    l.tb_entries = l.tb_entries > tb ? l.tb_entries : tb;
}

// Grows the fast class layout by one ring of n pixels (n even, fast path)
// for modes 0..mmax: the padded buffer holds the phased modes, the spectrum
// (bins 0..n/2), the alias staging of rings with fewer bins than threads and
// the FFT; then the twiddle table.
inline void fast_lds_add(RingLds &l, int n, int mmax)
{
    const int h = n / 2;
    int top = h > kFastThreads - 1 ? h : kFastThreads - 1;
    top = top > mmax ? top : mmax;
    const int need = fast_pad(top) + 1;
    l.fft_entries = l.fft_entries > need ? l.fft_entries : need;
    const int tw = 64 + (n + 63) / 64;
    l.tw_entries = l.tw_entries > tw ? l.tw_entries : tw;
}

// Grows the layout of class c by one ring of n pixels, Bluestein length nb
// (0 if none) and spectrum / FFT need `need`.  A ring with fewer spectrum
// bins than threads stages its partial alias sums in the buffer, which then
// holds at least one entry per thread.
inline void ring_lds_add(RingLds &l, int c, int n, int nb, int need)
{
    const int nt = kClassThreads[c];
    const int bins = (n % 2 == 0) ? n / 2 + 1 : n;
    if (bins < nt && need < nt) need = nt;
    // the synthesis stages the modes in chunks of 8 nt entries
    if (need < 8 * nt) need = 8 * nt;
    l.fft_entries = l.fft_entries > need ? l.fft_entries : need;
    const int tw = 64 + (n + 63) / 64;
    l.tw_entries = l.tw_entries > tw ? l.tw_entries : tw;
    if (nb > 0) {
        const int tb = 64 + (nb + 63) / 64;
        l.tb_entries = l.tb_entries > tb ? l.tb_entries : tb;
    }
}

// One map of a batch of plans (device side): the plan's tables plus the
// offsets of the map's buffers inside the batch workspace.
struct BatchMap {
    const PairDesc *pairs;
    const int32_t *mval;
    const long long *moff;
    const double *mu;
    const double *A;
    const double *cn;
    const int32_t *minv;
    const RingDesc *rings;
    const double2 *pool;
    long long nalm;
    long long ap_off;     // prescaled coefficients (double2 [nalm]) in the workspace
    long long delta_off;  // Delta (double2 [nm][nrings]) in the workspace
    int lmax, mmax, nm, nrings, npairs, mcontig, m0len, pad;
};

// A tile of the persistent Legendre launch: map, m-pair, ring-pair block.
struct BatchTile {
    int map, mpair, pblock, pad;
};

struct BatchClass {
    int count;        // (map, ring) items
    RingLds lds;
    int2 *d_items;    // device [count] (map, ring)
};

}  // namespace sht

struct sht_plan_s {
    uint64_t magic;
    int device;
    int lmax, mmax, nm, nrings, nmaps, npairs, precision;
    uint32_t flags;
    long long nalm, npix;
    std::vector<int32_t> mval;
    std::vector<long long> moff;
    // device tables (owned by the plan)
    sht::PairDesc *d_pairs;
    int32_t *d_mval;
    long long *d_moff;
    double *d_mu;        // mu_m for each m of the set (Eq. pmm)
    double *d_A;         // [nalm] normalised recurrence coefficient, see legendre.hip
    double *d_cn;        // [nalm] normalisation c_lm folded into the coefficients
    int32_t *d_minv;     // [mmax + 1] index of m in the set, -1 if absent
    long long *d_boff;   // [nm] first 32-step block of each m (split-BF16 operand packing)
    int32_t *d_bm32;     // [32-step blocks] index of the m that owns each block
    long long *d_boff16; // [nm] first 16-row block of each m (FP32 matrix-core operand packing)
    int32_t *d_bm16;     // [nblk16] index of the m that owns each 16-row block
    long long nblk16;    // 16-row blocks over all m
    long long *d_soff;   // [nm] first 128-row super-block of each m (split-FP16 operand packing)
    int32_t *d_sbm;      // [nsuper] index of the m that owns each super-block
    double *d_Asb;       // [nsuper][128] d_A per super-block, zero past each m's last row
    long long nsuper;    // 128-row super-blocks over all m
    sht::RingDesc *d_rings;
    double2 *d_pool;     // twiddle and Bluestein tables
    float2 *d_pool32;    // complex64 copy of d_pool (plans with a Bluestein fast path)
    size_t table_bytes;
    size_t pool_entries;
    int mcontig;         // m-set is 0..nm-1
    std::vector<int> ring_class;  // size class of each ring's Fourier step
    std::vector<int> ring_need;   // LDS double2 entries of each ring's spectrum / FFT
    std::vector<int> ring_n;      // pixels of each ring
    std::vector<int> ring_nb;     // Bluestein length of each ring (0: none)
    sht::RingClass cls[sht::kNumRingClasses];     // analysis: every ring
    sht::RingClass scls[sht::kNumSynthClasses];   // synthesis
    // the Bluestein fast path's rings by size class, for synthesis from a
    // caller's complex128 Delta (sht_delta2map), which that path does not take
    sht::RingClass bcls[sht::kNumRingClasses];
    std::vector<int> ring_sclass;  // synthesis class of each ring
    int fwd_chains;      // ring pairs per lane of the FP64 forward Legendre kernel (1, 2, 4)
    int num_cus;         // compute units of the plan's device
    size_t ws_ap_bytes;  // workspace: prescaled coefficients
    // the fast-path synthesis of large plans runs on aux_stream beside the
    // size-class kernels on the caller's stream (fork / join by the events)
    hipStream_t aux_stream;
    hipEvent_t ev_fork, ev_join;
    std::mutex fork_mu;    // one fork / launches / join sequence at a time
    size_t ws_delta_bytes;   // workspace: forward Delta (complex64 for the mixed forms)
    size_t ws_dt_bytes;      // workspace: adjoint Delta~ (complex128)
};

namespace sht {

// hipGetLastError returns the error of any earlier HIP call on the thread,
// the caller's own included (a failed query a framework ignored, say).  Each
// entry point clears it first, so that the launch checks below report only
// the entry point's own launches.
inline void clear_stale_error() { (void)hipGetLastError(); }

// Launchers (legendre.hip / ringfft.hip).  All enqueue on `st` only.
hipError_t launch_prescale(const sht_plan_s *p, const double *alm, double2 *ap, hipStream_t st);
hipError_t launch_legendre_fwd(const sht_plan_s *p, const double2 *ap, double2 *delta,
                               hipStream_t st);
int fwd_pblocks(const sht_plan_s *p);
hipError_t launch_legendre_adj_ws(const sht_plan_s *p, const double2 *dt, double2 *part,
                                  double *alm, hipStream_t st, bool accumulate = false);
size_t adj_part_bytes(const sht_plan_s *p);
size_t mfma_bf_bytes(const sht_plan_s *p);
hipError_t launch_prescale_f32(const sht_plan_s *p, const double *alm, float *Bf, hipStream_t st);
hipError_t launch_legendre_mfma_f32(const sht_plan_s *p, const float *Bf, float2 *delta,
                                    hipStream_t st);
size_t bf16_bytes(const sht_plan_s *p);
hipError_t launch_prescale_bf16x3(const sht_plan_s *p, const double *alm, void *Bb,
                                  hipStream_t st);
hipError_t launch_legendre_mfma_bf16x3(const sht_plan_s *p, const void *Bb, float2 *delta,
                                       hipStream_t st);
size_t f16_bytes(const sht_plan_s *p);
int f16_super_rows();
hipError_t launch_prescale_f16x2(const sht_plan_s *p, const double *alm, void *Bb,
                                 hipStream_t st);
hipError_t launch_legendre_mfma_f16x2(const sht_plan_s *p, const void *Bb, float2 *delta,
                                      hipStream_t st);
hipError_t launch_ring_synth(const sht_plan_s *p, const double2 *delta, double *map,
                             hipStream_t st);
hipError_t launch_ring_synth(const sht_plan_s *p, const float2 *delta, double *map,
                             hipStream_t st);
// the mixed forms' complex64 [m][ring][map] Delta -> complex128 [map][m][ring]
hipError_t launch_widen_delta(const sht_plan_s *p, const float2 *s, double2 *d, hipStream_t st);
hipError_t launch_narrow(const double2 *s, float2 *d, long long n, hipStream_t st);
hipError_t launch_ring_anal(const sht_plan_s *p, const double *map, double2 *dt, hipStream_t st,
                            const double *rw = nullptr, double cfac = 2.0);
hipError_t launch_residual(const double *s, double *r, long long n, hipStream_t st);
hipError_t launch_batch_legendre(const BatchMap *maps, int nmaps, long long max_nalm,
                                 const BatchTile *tiles, int ntiles, int chains, int grid_waves,
                                 const double *const *alms, void *ws, int *counter,
                                 hipStream_t st);
hipError_t launch_ring_synth_batch(const BatchClass *cls, const BatchMap *maps,
                                   double *const *outs, const void *ws, hipStream_t st);
// Decision log: with SHT_LOG set in the environment (to anything but "0"),
// plan and batch creation and the autotuners write one line per decision to
// stderr (ring classes, radix lists, workspace sizes, launch shapes).
bool log_enabled();
void log_line(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

// The forward transform of a plan into a caller workspace of at least
// forward_workspace(p) bytes (no checks: the entry points validate).
size_t forward_workspace(const sht_plan_s *p);
sht_status check_plan_device(sht_plan_t p);
sht_status forward_transform(sht_plan_t p, const double *alm, double *map, void *ws,
                             hipStream_t st);
// Plan time: spectra of the Bluestein chirp kernels.
hipError_t launch_bluestein_prep(const sht_plan_s *p, const int *ring_ids, int nids,
                                 hipStream_t st);

}  // namespace sht
