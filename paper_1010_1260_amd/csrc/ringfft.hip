// Per-ring Fourier step of alm2map and of its adjoint for gfx950: FP64,
// except the synthesis fast paths of the mixed forms (complex64 passes).
//
// Synthesis (Eq. Delta2map, Sec. 2.1, and the wrap rule of Sec. 2.2.2):
//     s_j = sum_{m=-mmax}^{mmax} Delta_m e^{i m (phi0 + 2 pi j / n)},  Delta_{-m} = conj(Delta_m).
// With D_m = Delta_m e^{i m phi0}, every mode is moved to bin m mod n:
//     F_k = sum_{m = k mod n} D_m + sum_{m >= 1, m = -k mod n} conj(D_m),
//     s_j = sum_{k<n} F_k e^{2 pi i j k / n}.
// F is Hermitian, so for even n the real inverse DFT is taken as one complex
// DFT of half length h = n/2:
//     Z_k = (F_k + conj F_{h-k}) + i e^{2 pi i k/n} (F_k - conj F_{h-k}),
//     z_j = sum_{k<h} Z_k e^{2 pi i j k/h},   s_2j = Re z_j,  s_2j+1 = Im z_j;
// odd n use a complex DFT of length n and keep the real part.
//
// Analysis (adjoint): G_k = sum_j g_j e^{-2 pi i j k / n} by the reverse
// construction, then Dt_m = c_m e^{-i m phi0} G_{m mod n} (c_0 = 1, c_m = 2).
//
// One workgroup per ring and map; the whole ring lives in LDS.  The
// synthesis of even rings whose half length is 7-smooth and at most 4096
// (every HEALPix belt ring, and the caps' smooth rings) takes a fast path: a
// persistent 256-thread kernel that loads a ring's modes all at once (the
// next ring's while the current one is transformed), folds them through a
// padded LDS buffer and runs Stockham passes of radix 16, 8, 4, 2, 7, 5, 3
// with the butterflies held in registers, the half-length pre-processing
// fused into the first pass and the pixels stored from the last.  Its passes
// run in complex128 for FP64 plans; for the mixed forms, whose Delta is
// complex64 [m][ring][map], one workgroup takes two maps of a ring (one
// 16-byte load per mode) and runs the passes of both in complex64 (the fold
// adds in FP64 either way).  The mixed forms also take even rings whose half
// length is twice a non-7-smooth number on a Bluestein fast path: a
// persistent 512-thread kernel that loads two maps of a ring per item and,
// map by map, runs the even- and odd-indexed Bluestein convolutions side by
// side in two complex64 buffers.  The other rings are
// grouped by FFT length into three size classes (up to 2048, 4096 and 8192
// points) run by 256-, 512- and 1024-thread workgroups, each with an LDS
// layout computed on the host for the class.  There, DFTs of 7-smooth length run as
// a Stockham auto-sort FFT (radices 8, 4, 2, 3, 5 and 7; every pass loads its
// butterfly inputs into registers, barriers, and stores in place, so one LDS
// buffer suffices).  Other lengths use Bluestein's chirp-z algorithm with a
// 7-smooth convolution length whose kernel spectrum is precomputed at plan
// time; an even length whose half is not 7-smooth is split into the DFTs of
// its even- and odd-indexed inputs (two Bluestein transforms of half length)
// joined by one radix-2 step.  Twiddles come from per-length tables computed
// on the host in extended precision.
#include "sht_internal.h"

// Every fused multiply-add in this file is written out (fma, cmul): no
// contraction, so that all instantiations of the Fourier kernels (single and
// batched, any size class) round identically.
#pragma clang fp contract(off)

namespace sht {
namespace {


// Complex product with its roundings pinned (one product, then one fused
// multiply-add per component), so that every inlined copy of a kernel rounds
// alike whatever the compiler would otherwise contract.
__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
// sign * i * a
__device__ inline double2 muli(double2 a, int sign)
{
    return sign > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// The same operations on complex64, for the FP32 Fourier passes of the mixed
// forms' fast path.
__device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 conjd(float2 a) { return make_float2(a.x, -a.y); }
__device__ inline float2 muli(float2 a, int sign)
{
    return sign > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// Complex element type C from real parts, and conversions between the two
// precisions (rounded once).
template <typename C> __device__ inline C cplx(double x, double y);
template <> __device__ inline double2 cplx<double2>(double x, double y) { return make_double2(x, y); }
template <> __device__ inline float2 cplx<float2>(double x, double y)
{
    return make_float2((float)x, (float)y);
}
template <typename C> __device__ inline C cvt(double2 v) { return cplx<C>(v.x, v.y); }
__device__ inline double2 todbl(double2 v) { return v; }
__device__ inline double2 todbl(float2 v) { return make_double2((double)v.x, (double)v.y); }

// cos / sin of 2 pi q / R (correctly rounded)
template <int R> struct Roots;
template <> struct Roots<3> {
    static constexpr double c[3] = {0x1p+0, -0x1p-1, -0x1p-1};
    static constexpr double s[3] = {0.0, 0x1.bb67ae8584caap-1, -0x1.bb67ae8584caap-1};
};
template <> struct Roots<5> {
    static constexpr double c[5] = {0x1p+0, 0x1.3c6ef372fe950p-2, -0x1.9e3779b97f4a8p-1,
                                    -0x1.9e3779b97f4a8p-1, 0x1.3c6ef372fe950p-2};
    static constexpr double s[5] = {0.0, 0x1.e6f0e134454ffp-1, 0x1.2cf2304755a5ep-1,
                                    -0x1.2cf2304755a5ep-1, -0x1.e6f0e134454ffp-1};
};
template <> struct Roots<7> {
    static constexpr double c[7] = {0x1p+0, 0x1.3f3a0e28bedd1p-1, -0x1.c7b90e3024582p-3,
                                    -0x1.cd4bca9cb5c71p-1, -0x1.cd4bca9cb5c71p-1,
                                    -0x1.c7b90e3024582p-3, 0x1.3f3a0e28bedd1p-1};
    static constexpr double s[7] = {0.0, 0x1.904c37505de4bp-1, 0x1.f329c0558e969p-1,
                                    0x1.bc4c04d71abc1p-2, -0x1.bc4c04d71abc1p-2,
                                    -0x1.f329c0558e969p-1, -0x1.904c37505de4bp-1};
};

// y_k = sum_r v_r e^{sign 2 pi i r k / R}
__device__ inline double fmaS(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float fmaS(float a, float b, float c) { return fmaf(a, b, c); }

template <int R, typename C>
__device__ inline void small_dft(C (&v)[R], int sign)
{
    typedef decltype(C::x) S;
    if constexpr (R == 2) {
        const C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const C s13 = cadd(v[1], v[3]), d13 = muli(csub(v[1], v[3]), sign);
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else if constexpr (R == 16) {
        // 16 = 4 x 4: r = 4a + b, k = c + 4d, w^(rk) = w4^(ac) w16^(bc) w4^(bd)
        C u[4][4];   // u[b][c]
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            C t[4] = {v[b], v[4 + b], v[8 + b], v[12 + b]};
            small_dft<4, C>(t, sign);
#pragma unroll
            for (int c = 0; c < 4; ++c) u[b][c] = t[c];
        }
        constexpr S c1 = (S) 0x1.d906bcf328d46p-1;  // cos(pi/8), correctly rounded
        constexpr S s1 = (S) 0x1.87de2a6aea963p-2;  // sin(pi/8)
        constexpr S hh = (S) 0x1.6a09e667f3bcdp-1;  // 1/sqrt(2)
        // w16^e = (cos, sign sin) of 2 pi e / 16 for e = b c, b, c in 1..3
        const S sg = (S)sign;
        u[1][1] = cmul(u[1][1], cplx<C>(c1, sg * s1));
        u[1][2] = cmul(u[1][2], cplx<C>(hh, sg * hh));
        u[1][3] = cmul(u[1][3], cplx<C>(s1, sg * c1));
        u[2][1] = cmul(u[2][1], cplx<C>(hh, sg * hh));
        u[2][2] = muli(u[2][2], sign);
        u[2][3] = cmul(u[2][3], cplx<C>(-hh, sg * hh));
        u[3][1] = cmul(u[3][1], cplx<C>(s1, sg * c1));
        u[3][2] = cmul(u[3][2], cplx<C>(-hh, sg * hh));
        u[3][3] = cmul(u[3][3], cplx<C>(-c1, -sg * s1));
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            C t[4] = {u[0][c], u[1][c], u[2][c], u[3][c]};
            small_dft<4, C>(t, sign);
#pragma unroll
            for (int d = 0; d < 4; ++d) v[c + 4 * d] = t[d];
        }
    } else if constexpr (R == 8) {
        // two radix-4 DFTs of the even and odd inputs, combined with w8^k
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        small_dft<4, C>(e, sign);
        small_dft<4, C>(o, sign);
        constexpr S h = (S)0x1.6a09e667f3bcdp-1;  // 1/sqrt(2), correctly rounded
        // w8 = e^{sign i pi/4}: w8^1 o1, w8^2 o2 = sign i o2, w8^3 o3
        const C t1 = cplx<C>(h * (o[1].x - sign * o[1].y), h * (o[1].y + sign * o[1].x));
        const C t2 = muli(o[2], sign);
        const C t3 = cplx<C>(-h * (o[3].x + sign * o[3].y), h * (sign * o[3].x - o[3].y));
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], t1);
        v[5] = csub(e[1], t1);
        v[2] = cadd(e[2], t2);
        v[6] = csub(e[2], t2);
        v[3] = cadd(e[3], t3);
        v[7] = csub(e[3], t3);
    } else {
        // odd R: pair r with R - r
        C sp[R / 2], dm[R / 2];
#pragma unroll
        for (int r = 1; r <= R / 2; ++r) {
            sp[r - 1] = cadd(v[r], v[R - r]);
            dm[r - 1] = csub(v[r], v[R - r]);
        }
        C y[R];
        C y0 = v[0];
#pragma unroll
        for (int r = 0; r < R / 2; ++r) y0 = cadd(y0, sp[r]);
        y[0] = y0;
#pragma unroll
        for (int k = 1; k < R; ++k) {
            S ar = v[0].x, ai = v[0].y, br = 0, bi = 0;
#pragma unroll
            for (int r = 1; r <= R / 2; ++r) {
                const S c = (S)Roots<R>::c[(r * k) % R];
                const S s = (S)Roots<R>::s[(r * k) % R];
                ar = fmaS(sp[r - 1].x, c, ar);
                ai = fmaS(sp[r - 1].y, c, ai);
                br = fmaS(dm[r - 1].x, s, br);
                bi = fmaS(dm[r - 1].y, s, bi);
            }
            // + sign * i * (b)
            y[k] = sign > 0 ? cplx<C>(ar - bi, ai + br) : cplx<C>(ar + bi, ai - br);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = y[k];
    }
}

// Twiddles e^{+2 pi i t / L} (t < L <= 16384) from a two-level table in LDS:
// T[b] = w^b for b < 64 and T[64 + a] = w^(64 a), so w^t = T[64 + t/64] T[t % 64]
// (within 2 ulp; T[64] = 1 exactly).  Filled from the plan's full table `tab`
// (entry t at tab[t]) at the start of a workgroup, so that the FFT passes
// never wait on global memory.
constexpr int kTwEntries = 64 + 256;

template <int NT, typename C>
__device__ __attribute__((always_inline)) inline void load_tw(C *T, const double2 *__restrict__ tab,
                                                              int L)
{
    const int n1 = (L + 63) >> 6;
    for (int e = threadIdx.x; e < 64 + n1; e += NT) {
        const int t = (e < 64) ? e : 64 * (e - 64);
        T[e] = (t < L) ? cvt<C>(tab[t]) : cplx<C>(1.0, 0.0);
    }
}

// The same from a complex64 copy of the table.
template <int NT>
__device__ __attribute__((always_inline)) inline void load_tw(float2 *T,
                                                              const float2 *__restrict__ tab,
                                                              int L)
{
    const int n1 = (L + 63) >> 6;
    for (int e = threadIdx.x; e < 64 + n1; e += NT) {
        const int t = (e < 64) ? e : 64 * (e - 64);
        T[e] = (t < L) ? tab[t] : make_float2(1.0f, 0.0f);
    }
}

template <typename C>
__device__ inline C tw_at(const C *T, int t)
{
    return cmul(T[64 + (t >> 6)], T[t & 63]);
}

// One Stockham pass of radix R over n <= MAXN points in LDS.  T is the LDS
// table of e^{+2 pi i t / L} with L = n * tws.  j / Ns is taken as
// umulhi(j, ceil(2^32 / Ns)), which is exact for j, Ns < 2^13.
template <int R, int NT, int MAXN>
__device__ __attribute__((always_inline)) inline void fft_pass(double2 *buf, int n, int Ns, int sign, const double2 *T,
                         int tws)
{
    constexpr int MAXQ = (MAXN / R + NT - 1) / NT;
    const int nb = n / R;
    const int tstep0 = (n / (Ns * R)) * tws;
    const unsigned magic = (unsigned)((0x100000000ull + (unsigned)Ns - 1) / (unsigned)Ns);
    double2 v[MAXQ][R];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = threadIdx.x + q * NT;
        if (j < nb) {
            const int jq = (Ns == 1) ? j : (int)__umulhi((unsigned)j, magic);
            const int k = j - jq * Ns;
            const int ts = tstep0 * k;
            // twiddles w^r, r = 1..R-1, as powers of one table entry w
            double2 w1 = make_double2(1.0, 0.0);
            if (ts != 0) {
                w1 = tw_at(T, ts);
                if (sign < 0) w1.y = -w1.y;
            }
            double2 wr = w1;
            v[q][0] = buf[j];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const double2 x = buf[j + r * nb];
                v[q][r] = (ts != 0) ? cmul(x, wr) : x;
                wr = cmul(wr, w1);
            }
            small_dft<R>(v[q], sign);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = threadIdx.x + q * NT;
        if (j < nb) {
            const int jq = (Ns == 1) ? j : (int)__umulhi((unsigned)j, magic);
            const int k = j - jq * Ns;
            const int base = jq * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

// In-place DFT of 7-smooth length n <= MAXN:
// buf_k <- sum_j buf_j e^{sign 2 pi i j k / n}.
template <int NT, int MAXN>
__device__ __attribute__((always_inline)) inline void fft_lds(double2 *buf, int n, int sign, const double2 *T, int tws)
{
    int Ns = 1, rem = n;
    while (rem > 1) {
        if (rem % 8 == 0) {
            fft_pass<8, NT, MAXN>(buf, n, Ns, sign, T, tws); Ns *= 8; rem /= 8;
        } else if (rem % 4 == 0) {
            fft_pass<4, NT, MAXN>(buf, n, Ns, sign, T, tws); Ns *= 4; rem /= 4;
        } else if (rem % 2 == 0) {
            fft_pass<2, NT, MAXN>(buf, n, Ns, sign, T, tws); Ns *= 2; rem /= 2;
        } else if (rem % 3 == 0) {
            fft_pass<3, NT, MAXN>(buf, n, Ns, sign, T, tws); Ns *= 3; rem /= 3;
        } else if (rem % 5 == 0) {
            fft_pass<5, NT, MAXN>(buf, n, Ns, sign, T, tws); Ns *= 5; rem /= 5;
        } else {
            fft_pass<7, NT, MAXN>(buf, n, Ns, sign, T, tws); Ns *= 7; rem /= 7;
        }
    }
}

// In-place DFT of any length len by Bluestein's algorithm:
// e^{i 2 pi jk/len} = c_j c_k conj(c_{j-k}), c_k = e^{i pi k^2 / len}, as a
// cyclic convolution of 7-smooth length nb >= 2 len - 1.
// ch = this thread's chirps c_k, k = tid + q NT (loaded ahead by the caller),
// TB = LDS table of e^{2 pi i k / nb}, bq = DFT^-(conj c, wrapped) / nb.
// A sign -1 transform is conj(DFT^+(conj x)).
// REG: the chirps are held in registers from the start of the workgroup
// (their load latency overlaps the fold), else read where used.
template <int NT, int MAXN, bool REG>
struct Chirps {
    static constexpr int Q = (MAXN / 2 + NT - 1) / NT;  // len <= (nb + 1) / 2 <= MAXN / 2
    double2 c[REG ? Q : 1];
    const double2 *p;
    __device__ double2 get(int q, int k) const { return REG ? c[REG ? q : 0] : p[k]; }
};

template <int NT, int MAXN, bool REG>
__device__ __attribute__((always_inline)) inline void load_chirps(Chirps<NT, MAXN, REG> &ch,
                                                                  const double2 *__restrict__ chirp,
                                                                  int len)
{
    ch.p = chirp;
    if (REG) {
#pragma unroll
        for (int q = 0; q < Chirps<NT, MAXN, REG>::Q; ++q) {
            const int k = threadIdx.x + q * NT;
            ch.c[REG ? q : 0] = (k < len) ? chirp[k] : make_double2(0.0, 0.0);
        }
    }
}

template <int NT, int MAXN, bool REG>
__device__ __attribute__((always_inline)) inline void bluestein_lds(double2 *buf, int len, int nb, int sign,
                              const Chirps<NT, MAXN, REG> &ch, const double2 *TB,
                              const double2 *__restrict__ bq)
{
    constexpr int QB = MAXN / NT;
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        const int k = threadIdx.x + q * NT;
        if (k < nb) {
            if (q < Chirps<NT, MAXN, REG>::Q && k < len) {
                double2 x = buf[k];
                if (sign < 0) x.y = -x.y;
                buf[k] = cmul(x, ch.get(q < Chirps<NT, MAXN, REG>::Q ? q : 0, k));
            } else {
                buf[k] = make_double2(0.0, 0.0);
            }
        }
    }
    __syncthreads();
    fft_lds<NT, MAXN>(buf, nb, -1, TB, 1);
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        const int k = threadIdx.x + q * NT;
        if (k < nb) buf[k] = cmul(buf[k], bq[k]);
    }
    __syncthreads();
    fft_lds<NT, MAXN>(buf, nb, +1, TB, 1);
#pragma unroll
    for (int q = 0; q < Chirps<NT, MAXN, REG>::Q; ++q) {
        const int j = threadIdx.x + q * NT;
        if (j < len) {
            double2 z = cmul(buf[j], ch.get(q, j));
            if (sign < 0) z.y = -z.y;
            buf[j] = z;
        }
    }
    __syncthreads();
}

// LDS tables of a ring's Fourier step: TW for e^{2 pi i k / n} (n-point
// roots: the half-length FFT and its pre/post twiddles), TB for the
// Bluestein length.
struct RingTables {
    double2 *TW;
    double2 *TB;
};

template <int NT, int MAXN, bool REG>
__device__ __attribute__((always_inline)) inline void ring_tables_load(const RingTables &rt,
                                                                       const RingDesc &d,
                                                                       const double2 *__restrict__ pool,
                                                                       Chirps<NT, MAXN, REG> &ch)
{
    load_tw<NT>(rt.TW, pool + d.tw, d.n);
    if (d.nb != 0) {
        load_tw<NT>(rt.TB, pool + d.twb, d.nb);
        load_chirps<NT, MAXN, REG>(ch, pool + d.tch, d.half ? d.clen / 2 : d.clen);
    }
}

// DFT of even length clen = 2 len whose half length is not 7-smooth:
// with E = DFT_len(x_{2j}) and O = DFT_len(x_{2j+1}) (Bluestein each, one
// after the other in the same LDS buffer), X_j = E_j + w^j O_j and
// X_{j+len} = E_j - w^j O_j, w = e^{sign 2 pi i / clen}.  The ring is even,
// so TW holds the n-th roots with n = 2 clen: w^j = TW(2 j).  PRIV: the
// half kept across each Bluestein transform lives in private memory instead
// of registers (for kernels whose register budget is already spent).
template <int NT, int MAXN, bool REG, bool PRIV>
__device__ __attribute__((always_inline)) inline void split_bluestein(
    double2 *buf, const RingDesc &d, int sign, const double2 *__restrict__ pool,
    const RingTables &rt, const Chirps<NT, MAXN, REG> &ch)
{
    constexpr int QH = (MAXN / 2 + NT - 1) / NT;
    const int len = d.clen / 2;
    const int tid = threadIdx.x;
    double2 keep[QH], odd[QH];
    int zq = 0;   // an opaque zero index keeps the arrays out of registers
    if constexpr (PRIV) asm volatile("" : "+s"(zq));
#pragma unroll
    for (int q = 0; q < QH; ++q) {
        const int j = tid + q * NT;
        if (j < len) {
            keep[q ^ zq] = buf[2 * j];
            odd[q ^ zq] = buf[2 * j + 1];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QH; ++q) {
        const int j = tid + q * NT;
        if (j < len) buf[j] = keep[q ^ zq];
    }
    __syncthreads();
    bluestein_lds<NT, MAXN, REG>(buf, len, d.nb, sign, ch, rt.TB, pool + d.bq);
#pragma unroll
    for (int q = 0; q < QH; ++q) {
        const int j = tid + q * NT;
        if (j < len) keep[q ^ zq] = buf[j];   // E_j
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QH; ++q) {
        const int j = tid + q * NT;
        if (j < len) buf[j] = odd[q ^ zq];
    }
    __syncthreads();
    bluestein_lds<NT, MAXN, REG>(buf, len, d.nb, sign, ch, rt.TB, pool + d.bq);
#pragma unroll
    for (int q = 0; q < QH; ++q) {
        const int j = tid + q * NT;
        if (j < len) {
            double2 w = tw_at(rt.TW, 2 * j);
            if (sign < 0) w.y = -w.y;
            const double2 t = cmul(w, buf[j]);
            const double2 e = keep[q ^ zq];
            buf[j] = cadd(e, t);
            buf[j + len] = csub(e, t);
        }
    }
    __syncthreads();
}

template <int NT, int MAXN, bool REG, bool PRIV = false>
__device__ __attribute__((always_inline)) inline void ring_dft(double2 *buf, const RingDesc &d, int sign,
                                const double2 *__restrict__ pool, const RingTables &rt,
                                const Chirps<NT, MAXN, REG> &ch)
{
    if (d.nb == 0) {
        fft_lds<NT, MAXN>(buf, d.clen, sign, rt.TW, (d.n % 2 == 0) ? 2 : 1);
    } else if (d.half) {
        split_bluestein<NT, MAXN, REG, PRIV>(buf, d, sign, pool, rt, ch);
    } else {
        bluestein_lds<NT, MAXN, REG>(buf, d.clen, d.nb, sign, ch, rt.TB, pool + d.bq);
    }
}

// Block id -> logical id so that consecutive logical ids run on one XCD
// (workgroups are dealt round-robin over the 8 XCDs).
__device__ inline int xcd_logical(int b, int total)
{
    const int x = b % 8, i = b / 8, q = total / 8, r = total % 8;
    return x * q + (x < r ? x : r) + i;
}

// Work item -> (index in the class's ring list, map), so that the
// workgroups running together read Delta entries that share cache lines and
// DRAM pages: for [map][m][ring] Delta map by map, ring by ring
// (neighbouring rings of one map; measured faster than grouping a few rings'
// items of all maps together, which would keep each ring's tables in L2 but
// spreads the Delta reads over all maps); for [m][ring][map] Delta ring by
// ring, map by map (all maps of one ring).
template <bool RM>
__device__ inline void ring_item(long long it, int count, int nmaps, int &i, int &b)
{
    if (RM) {
        i = (int)(it / nmaps);
        b = (int)(it - (long long)i * nmaps);
    } else {
        b = (int)(it / count);
        i = (int)(it - (long long)b * count);
    }
}

// The persistent kernels' share of XCD x (workgroups are dealt to the 8 XCDs
// round-robin): items [lo, hi) of its own numbering, item k -> (i, b).  Map
// by map: a contiguous eighth of all items.  Ring by ring: the rings
// i = x mod 8 (the class's rings are sorted by length, so every XCD gets
// rings of every length), all maps of a ring together.
template <bool RM>
__device__ inline void xcd_share(int count, int nmaps, int x, long long &lo, long long &hi)
{
    if (RM) {
        lo = 0;
        hi = (long long)((count - x + 7) / 8) * nmaps;
    } else {
        const long long total = (long long)count * nmaps;
        lo = total * x / 8;
        hi = total * (x + 1) / 8;
    }
}

template <bool RM>
__device__ inline void xcd_item(long long k, int count, int nmaps, int x, int &i, int &b)
{
    if (RM) {
        const long long q = k / nmaps;
        i = (int)(x + 8 * q);
        b = (int)(k - q * nmaps);
    } else {
        ring_item<false>(k, count, nmaps, i, b);
    }
}

// complex64 Delta (the mixed forms') is [m][ring][map], its items ring by ring
template <typename DT> struct RingMajor {
    static constexpr bool value = false;
};
template <> struct RingMajor<float2> {
    static constexpr bool value = true;
};

// Delta_m for mode m of a ring (zero for m outside the set); Delta is laid
// out [m][ring], so the ring's modes are `dstride` entries apart.  DT is the
// stored element: complex128, or complex64 from the mixed-precision
// Legendre stage (widened exactly).
__device__ inline double2 widen(double2 v) { return v; }
__device__ inline double2 widen(float2 v) { return make_double2((double)v.x, (double)v.y); }

template <typename DT>
__device__ inline double2 load_mode(const DT *__restrict__ drow, long long dstride,
                                    const int *__restrict__ minv, int mcontig, int m)
{
    const int i = mcontig ? m : minv[m];
    return (i >= 0) ? widen(drow[(long long)i * dstride]) : make_double2(0.0, 0.0);
}

// Synthesis: one workgroup per (ring of this size class, map).  LDS: the
// spectrum / FFT buffer, the twiddle tables and the alias staging slots
// (RingLds).
// Synthesis of one ring: drow = its Delta_m row, out = its first pixel.
// Padded LDS indexing of the fast path's spectrum / FFT buffer.
struct PadIdx {   // one spare entry per 16 (bank-conflict-free strided stores)
    __device__ static int at(int i) { return i + (i >> 4); }
};

// Fold a ring's modes into its spectrum F_k, k = 0..kmax (Eq. Delta2map with
// the wrap rule of Sec. 2.2.2; ends with a barrier).  drow = the ring's
// Delta_m row, the i-th m of the set at drow[i dstride].
template <int NT, typename DT>
__device__ __attribute__((always_inline)) inline void fold_ring(double2 *buf, const RingDesc &d,
                                                                const DT *__restrict__ drow,
                                                                long long dstride,
                                                                const int *__restrict__ minv,
                                                                int mcontig, int mmax)
{
    const int n = d.n;
    const bool even = (n % 2) == 0;
    const int h = n / 2;
    const int kmax = even ? h : n - 1;
    const int tid = threadIdx.x;
    // ---- fold the modes into F_k, k = 0..kmax (Sec. 2.2.2 wrap rule).
    // Phases e^{i m phi0}: one sincos per thread for its first mode and one
    // for the stride NT, then a complex multiply per further mode (a few ulp).
    constexpr int kBatch = 8;
    double2 step;   // e^{i NT phi0}
    double2 ph;     // e^{i tid phi0}
    {
        double sn, cs;
        sincos((double)NT * d.phi0, &sn, &cs);
        step = make_double2(cs, sn);
        sincos((double)tid * d.phi0, &sn, &cs);
        ph = make_double2(cs, sn);
    }
    if (n > mmax) {
        // each bin gets at most one direct mode m = k and one mirrored mode
        // m = n - k: F_k = e^{i k phi0} (D_k + e^{-i n phi0} conj(D_{n-k}))
        double2 cn;
        {
            double sn, cs;
            sincos((double)n * d.phi0, &sn, &cs);
            cn = make_double2(cs, -sn);
        }
        const int kdir = min(kmax, mmax);
        for (int k0 = 0; k0 <= kmax; k0 += kBatch * NT) {
            double2 raw[kBatch], rawc[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const int k = k0 + q * NT + tid;
                raw[q] = (k <= kdir) ? load_mode(drow, dstride, minv, mcontig, k) : make_double2(0.0, 0.0);
                rawc[q] = (k >= 1 && k <= kmax && n - k <= mmax)
                              ? load_mode(drow, dstride, minv, mcontig, n - k) : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const int k = k0 + q * NT + tid;
                if (k <= kmax) {
                    double2 D = raw[q];
                    if (k == 0) D.y = 0.0;
                    D = cadd(D, cmul(cn, conjd(rawc[q])));
                    buf[k] = cmul(ph, D);
                }
                ph = cmul(ph, step);
            }
        }
    } else {
        // wrap-around (n <= mmax): bin k gathers its aliases m = k + j n and
        // m = j n - k directly.  With w = e^{i n phi0},
        //   F_k = e^{i k phi0} (sum_j Delta_{k+jn} w^j + sum_{j>=1} conj(Delta_{jn-k}) conj(w^j)).
        // Few bins (small rings): G = NT / B threads share a bin, each taking
        // every G-th alias, and the G partial sums are staged in the spectrum
        // buffer itself (the class layout gives it at least NT entries when
        // some ring has fewer bins than threads) and added in a fixed order.
        // G depends on the ring and NT only, so every launch of the ring
        // rounds alike.  The aliases are fetched two at a time.
        const int B = kmax + 1;
        const int G = (B < NT) ? NT / B : 1;
        double2 step;    // e^{i NT phi0}
        {
            double sn, cs;
            sincos((double)NT * d.phi0, &sn, &cs);
            step = make_double2(cs, sn);
        }
        const int kk = (G > 1) ? tid % B : tid;
        const int g = (G > 1) ? tid / B : 0;
        double2 stepG;   // w^G
        {
            double sn, cs;
            sincos((double)n * (double)G * d.phi0, &sn, &cs);
            stepG = make_double2(cs, sn);
        }
        double2 phb;     // e^{i k phi0} for this thread's first bin
        {
            double sn, cs;
            sincos((double)kk * d.phi0, &sn, &cs);
            phb = make_double2(cs, sn);
        }
        constexpr int U = 2;
        for (int k = kk; k <= kmax && g < G; k += NT) {
            const int jmax = (mmax + k) / n;   // last alias with j n - k <= mmax
            double sr = 0.0, si = 0.0;
            int c = 0;
            double2 wj = make_double2(1.0, 0.0);
            for (int j0 = g; j0 <= jmax; j0 += U * G) {
                double2 Dd[U], Dm[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = j0 + u * G;
                    const int md = k + j * n, mc = j * n - k;
                    Dd[u] = make_double2(0.0, 0.0);
                    Dm[u] = make_double2(0.0, 0.0);
                    if (j <= jmax) {
                        if (md <= mmax) Dd[u] = load_mode(drow, dstride, minv, mcontig, md);
                        if (j >= 1) Dm[u] = load_mode(drow, dstride, minv, mcontig, mc);
                    }
                    if (md == 0) Dd[u].y = 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = j0 + u * G;
                    if (j <= jmax) {
                        if ((c & 31) == 0) {   // re-seed w^j every 32 aliases
                            double sn, cs;
                            sincos((double)j * (double)n * d.phi0, &sn, &cs);
                            wj = make_double2(cs, sn);
                        }
                        const double2 v = cmul(Dd[u], wj);
                        sr += v.x; si += v.y;
                        const double2 vm = cmul(conjd(Dm[u]), conjd(wj));
                        sr += vm.x; si += vm.y;
                        wj = cmul(wj, stepG);
                        ++c;
                    }
                }
            }
            if (G > 1) {
                buf[g * B + k] = make_double2(sr, si);
            } else {
                buf[k] = cmul(phb, make_double2(sr, si));
                phb = cmul(phb, step);
            }
        }
        if (G > 1) {
            __syncthreads();
            // column k of the staged partials is read and then overwritten
            // (entry 0) by thread k alone
            if (tid < B) {
                double sr = 0.0, si = 0.0;
                for (int q = 0; q < G; ++q) {
                    const double2 v = buf[q * B + tid];
                    sr += v.x; si += v.y;
                }
                buf[tid] = cmul(phb, make_double2(sr, si));
            }
        }
    }
    __syncthreads();
}

template <int NT, int MAXN, bool REG, bool PRIV, typename DT>
__device__ __attribute__((always_inline)) inline void synth_ring(double2 *buf, const RingTables &rt, const RingDesc &d,
                           const double2 *__restrict__ pool, const DT *__restrict__ drow,
                           long long dstride, const int *__restrict__ minv, int mcontig, int mmax,
                           double *__restrict__ out)
{
    Chirps<NT, MAXN, REG> ch;
    ring_tables_load<NT, MAXN, REG>(rt, d, pool, ch);
    const int n = d.n;
    const bool even = (n % 2) == 0;
    const int h = n / 2;
    const int tid = threadIdx.x;
    fold_ring<NT>(buf, d, drow, dstride, minv, mcontig, mmax);
    if (even) {
        for (int k = tid; k <= h / 2; k += NT) {
            const int k2 = h - k;
            const double2 Fk = buf[k], Fk2 = buf[k2];
            const double2 e1 = cadd(Fk, conjd(Fk2)), o1 = csub(Fk, conjd(Fk2));
            const double2 Zk = cadd(e1, muli(cmul(tw_at(rt.TW, k), o1), +1));
            const double2 e2 = cadd(Fk2, conjd(Fk)), o2 = csub(Fk2, conjd(Fk));
            const double2 Zk2 = cadd(e2, muli(cmul(tw_at(rt.TW, k2), o2), +1));
            buf[k] = Zk;
            if (k2 != k) buf[k2] = Zk2;
        }
        __syncthreads();
        ring_dft<NT, MAXN, REG, PRIV>(buf, d, +1, pool, rt, ch);
        if ((reinterpret_cast<uintptr_t>(out) & 15) == 0) {
            double2 *o2 = reinterpret_cast<double2 *>(out);
            for (int j = tid; j < h; j += NT) o2[j] = buf[j];
        } else {
            for (int j = tid; j < h; j += NT) {
                const double2 z = buf[j];
                out[2 * j] = z.x;
                out[2 * j + 1] = z.y;
            }
        }
    } else {
        ring_dft<NT, MAXN, REG, PRIV>(buf, d, +1, pool, rt, ch);
        for (int j = tid; j < n; j += NT) out[j] = buf[j].x;
    }
}


// ---------------------------------------------------------------------------
// Fast path of the synthesis: even rings whose half length h is 7-smooth and
// at most kFastMaxH.  The spectrum sits in a padded LDS buffer (PadIdx), each
// Stockham pass holds its butterflies in registers (radix 16, 8, 4, 2, 7, 5,
// 3 from the ring's pass list), the half-length pre-processing Z_k is formed
// while the first pass loads its inputs, and the last pass writes the pixels
// straight from registers: per ring one fold, one barrier pair per inner
// pass and no other LDS round trip.
//
// One pass of radix R over the h-point buffer (input index j + r h/R,
// output index (j / Ns) Ns R + j % Ns + r Ns).  T: the ring's n-th roots.
template <int R, int NT, typename C>
__device__ __attribute__((always_inline)) inline void fast_pass(C *buf, const C *T,
                                                                int h, int Ns, bool first,
                                                                bool last, double *__restrict__ out)
{
    constexpr int MAXQ = fast_maxq(R);   // the plan admits h / R <= MAXQ * kFastThreads
    const int nb = h / R;
    const int tstep0 = (h / (Ns * R)) * 2;   // T holds the roots of n = 2 h
    const unsigned magic = (unsigned)((0x100000000ull + (unsigned)Ns - 1) / (unsigned)Ns);
    // an opaque copy of the thread index: the passes run in a loop over the
    // ring's radix list, and address arithmetic hoisted out of every radix's
    // case would stay live across all of them
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    C v[MAXQ][R];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = tid + q * NT;
        if (j < nb) {
            if (first) {
                // Z_k = (F_k + conj F_{h-k}) + i e^{2 pi i k/n} (F_k - conj F_{h-k})
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int k = j + r * nb;
                    const C Fk = buf[PadIdx::at(k)], Fk2 = buf[PadIdx::at(h - k)];
                    const C e1 = cadd(Fk, conjd(Fk2)), o1 = csub(Fk, conjd(Fk2));
                    v[q][r] = cadd(e1, muli(cmul(tw_at(T, k), o1), +1));
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = buf[PadIdx::at(j + r * nb)];
            }
            if (Ns > 1) {
                const int jq = (int)__umulhi((unsigned)j, magic);
                const int ts = tstep0 * (j - jq * Ns);
                if (ts != 0) {
                    const C w1 = tw_at(T, ts);
                    C wr = w1;
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        v[q][r] = cmul(v[q][r], wr);
                        wr = cmul(wr, w1);
                    }
                }
            }
            small_dft<R, C>(v[q], +1);
        }
    }
    if (last) {
        // Ns R = h: j < Ns, output z_{j + r nb} = pixels 2 (j + r nb), 2 (j + r nb) + 1
        const bool al = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
        double2 *o2 = reinterpret_cast<double2 *>(out);
        // pixels are float64 whatever the precision of the passes
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int j = tid + q * NT;
            if (j < nb) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = j + r * nb;
                    if (al) {
                        o2[i] = todbl(v[q][r]);
                    } else {
                        out[2 * i] = (double)v[q][r].x;
                        out[2 * i + 1] = (double)v[q][r].y;
                    }
                }
            }
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int j = tid + q * NT;
            if (j < nb) {
                const int jq = (Ns == 1) ? j : (int)__umulhi((unsigned)j, magic);
                const int base = jq * Ns * R + (j - jq * Ns);
#pragma unroll
                for (int r = 0; r < R; ++r) buf[PadIdx::at(base + r * Ns)] = v[q][r];
            }
        }
        __syncthreads();
    }
}

// Fold of a fast-path ring (modes m = 0..mmax <= kFastMaxModes - 1, n even).
// Every thread loads its modes m = tid + q NT at once, multiplies them by
// e^{i m phi0} and stores them at buf[PadIdx(m)]; then bin k sums its
// aliases m = k + j n and conj of m = j n - k in a fixed order (j ascending,
// direct before mirrored), in place: below index n/2 + 1 the buffer entry m
// is read only by bin m, whose own thread then overwrites it with F_m.  Rings
// with fewer bins than threads split each bin's aliases over G = NT / bins
// threads and add the G partial sums in a fixed order.  Ends with a barrier.
template <int NT, typename DT>
struct FastModes {
    static constexpr int Q = (kFastMaxModes + NT - 1) / NT;
    DT v[Q];   // as stored (complex64 or complex128), widened at use
};

// Loads of the fold: modes m = tid + q NT of one ring.  Each load waits for
// the one before it: the loads of all workgroups then move through the m
// rows of Delta together, so the DRAM rows they open serve the neighbouring
// rings too.  Issued all at once they reach DRAM as a burst over thousands
// of rows, which measured 17% slower (split-FP16 belt rings, 16 maps at
// l_max 4096 / nside 2048: 3.43 ms paced, 4.00 ms as a burst).
template <int NT, typename DT>
__device__ __attribute__((always_inline)) inline void load_fast(FastModes<NT, DT> &raw,
                                                                const DT *__restrict__ drow,
                                                                long long dstride,
                                                                const int *__restrict__ minv,
                                                                int mcontig, int mmax)
{
    constexpr int QM = FastModes<NT, DT>::Q;
    // an opaque thread index keeps the per-q addresses from being hoisted
    // out of the persistent kernels' ring loop (where they would stay live)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (mcontig) {
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int m = tid + q * NT;
            raw.v[q] = (m <= mmax) ? drow[(long long)m * dstride] : DT{};
            // s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15)
            if (q + 1 < QM) __builtin_amdgcn_s_waitcnt(0x0F70);
        }
    } else {
        // every position lookup first, then the loads
        int pos[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int m = tid + q * NT;
            pos[q] = (m <= mmax) ? minv[m] : -1;
        }
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            raw.v[q] = (pos[q] >= 0) ? drow[(long long)pos[q] * dstride] : DT{};
            if (q + 1 < QM) __builtin_amdgcn_s_waitcnt(0x0F70);
        }
    }
}

template <int NT, typename C, typename DT>
__device__ __attribute__((always_inline)) inline void fold_fast(C *buf, const RingDesc &d,
                                                                const FastModes<NT, DT> &raw,
                                                                int mmax)
{
    constexpr int QM = FastModes<NT, DT>::Q;
    const int tid = threadIdx.x;
    double2 ph, step;   // e^{i tid phi0}, e^{i NT phi0}
    {
        double sn, cs;
        sincos((double)tid * d.phi0, &sn, &cs);
        ph = make_double2(cs, sn);
        sincos((double)NT * d.phi0, &sn, &cs);
        step = make_double2(cs, sn);
    }
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int m = tid + q * NT;
        if (m <= mmax) {
            double2 v = widen(raw.v[q]);
            if (m == 0) v.y = 0.0;
            buf[PadIdx::at(m)] = cvt<C>(cmul(ph, v));
        }
        ph = cmul(ph, step);
    }
    __syncthreads();
    const int n = d.n;
    const int h = n / 2;
    const int B = h + 1;
    if (n > mmax) {
        // at most one direct mode (m = k) and one mirrored mode (m = n - k)
        for (int k = tid; k <= h; k += NT) {
            double2 F = (k <= mmax) ? todbl(buf[PadIdx::at(k)]) : make_double2(0.0, 0.0);
            if (k >= 1 && n - k <= mmax) F = cadd(F, conjd(todbl(buf[PadIdx::at(n - k)])));
            buf[PadIdx::at(k)] = cvt<C>(F);
        }
    } else if (B >= NT) {
        for (int k = tid; k <= h; k += NT) {
            const int jmax = (mmax + k) / n;
            double sr = 0.0, si = 0.0;
            for (int j = 0; j <= jmax; ++j) {
                if (k + j * n <= mmax) {
                    const double2 v = todbl(buf[PadIdx::at(k + j * n)]);
                    sr += v.x; si += v.y;
                }
                if (j >= 1) {
                    const double2 v = todbl(buf[PadIdx::at(j * n - k)]);
                    sr += v.x; si -= v.y;
                }
            }
            buf[PadIdx::at(k)] = cplx<C>(sr, si);
        }
    } else {
        const int G = NT / B;
        const int kk = tid % B, g = tid / B;
        double sr = 0.0, si = 0.0;
        if (g < G) {
            const int jmax = (mmax + kk) / n;
            for (int j = g; j <= jmax; j += G) {
                if (kk + j * n <= mmax) {
                    const double2 v = todbl(buf[PadIdx::at(kk + j * n)]);
                    sr += v.x; si += v.y;
                }
                if (j >= 1) {
                    const double2 v = todbl(buf[PadIdx::at(j * n - kk)]);
                    sr += v.x; si -= v.y;
                }
            }
        }
        __syncthreads();
        if (g < G) buf[PadIdx::at(g * B + kk)] = cplx<C>(sr, si);
        __syncthreads();
        if (tid < B) {
            // column tid of the partials; entry 0 of it is this thread's own
            double tr = 0.0, ti = 0.0;
            for (int q = 0; q < G; ++q) {
                const double2 v = todbl(buf[PadIdx::at(q * B + tid)]);
                tr += v.x; ti += v.y;
            }
            buf[PadIdx::at(tid)] = cplx<C>(tr, ti);
        }
    }
    __syncthreads();
}

template <int NT, typename C>
__device__ __attribute__((always_inline)) inline void fft_fast(C *buf, const C *T,
                                                               const RingDesc &d,
                                                               double *__restrict__ out);

// Synthesis of one fast-path ring: buf = padded spectrum buffer, T = LDS
// twiddle table, out = the ring's first pixel.
template <int NT, typename C, typename DT>
__device__ __attribute__((always_inline)) inline void synth_fast(C *buf, C *T,
                                                                 const RingDesc &d,
                                                                 const double2 *__restrict__ pool,
                                                                 const DT *__restrict__ drow,
                                                                 long long dstride,
                                                                 const int *__restrict__ minv,
                                                                 int mcontig, int mmax,
                                                                 double *__restrict__ out)
{
    load_tw<NT>(T, pool + d.tw, d.n);
    FastModes<NT, DT> raw;
    load_fast<NT>(raw, drow, dstride, minv, mcontig, mmax);
    fold_fast<NT>(buf, d, raw, mmax);
    fft_fast<NT, C>(buf, T, d, out);
}

// The Stockham passes of a fast-path ring (after the fold) and the pixel
// stores of the last one.
template <int NT, typename C>
__device__ __attribute__((always_inline)) inline void fft_fast(C *buf, const C *T,
                                                               const RingDesc &d,
                                                               double *__restrict__ out)
{
    const int h = d.n / 2;
    int Ns = 1;
    for (int p = 0; p < d.np; ++p) {
        const int R = (int)((d.rads >> (5 * p)) & 31);
        const bool first = p == 0, last = p == d.np - 1;
        switch (R) {
        case 16: fast_pass<16, NT, C>(buf, T, h, Ns, first, last, out); break;
        case 8: fast_pass<8, NT, C>(buf, T, h, Ns, first, last, out); break;
        case 4: fast_pass<4, NT, C>(buf, T, h, Ns, first, last, out); break;
        case 2: fast_pass<2, NT, C>(buf, T, h, Ns, first, last, out); break;
        case 7: fast_pass<7, NT, C>(buf, T, h, Ns, first, last, out); break;
        case 5: fast_pass<5, NT, C>(buf, T, h, Ns, first, last, out); break;
        default: fast_pass<3, NT, C>(buf, T, h, Ns, first, last, out); break;
        }
        Ns *= R;
    }
}

// ---------------------------------------------------------------------------
// Fast path, two maps per workgroup (mixed forms, complex64 Delta
// [m][ring][map]): maps 2p and 2p + 1 of a ring are adjacent in Delta, so one
// 16-byte load per mode brings both; the two spectra sit in two padded LDS
// buffers, and every Stockham pass takes its butterflies in both with the
// same twiddles and one barrier pair.  `two` is false for the last map of an
// odd map count (its partner's loads read zeros and its stores are skipped).
template <int NT>
struct FastModes2 {
    static constexpr int Q = FastModes<NT, float2>::Q;
    float4 v[Q];   // (map 2p, map 2p + 1) of mode tid + q NT
};

template <int NT>
__device__ __attribute__((always_inline)) inline void load_fast2(
    FastModes2<NT> &raw, const float2 *__restrict__ drow, long long dstride,
    const int *__restrict__ minv, int mcontig, int mmax, bool aligned, bool two)
{
    constexpr int QM = FastModes2<NT>::Q;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    // paced like load_fast: each load waits for the one before it
    if (mcontig && aligned) {
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int m = tid + q * NT;
            raw.v[q] = (m <= mmax) ? *reinterpret_cast<const float4 *>(drow + (long long)m * dstride)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
            if (q + 1 < QM) __builtin_amdgcn_s_waitcnt(0x0F70);
        }
        return;
    }
    int pos[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int m = tid + q * NT;
        pos[q] = (m > mmax) ? -1 : (mcontig ? m : minv[m]);
    }
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        float2 e0 = make_float2(0.f, 0.f), e1 = e0;
        if (pos[q] >= 0) {
            const float2 *e = drow + (long long)pos[q] * dstride;
            e0 = e[0];
            if (two) e1 = e[1];
        }
        raw.v[q] = make_float4(e0.x, e0.y, e1.x, e1.y);
        if (q + 1 < QM) __builtin_amdgcn_s_waitcnt(0x0F70);
    }
}

// fold_fast for both maps (same order of additions per map).
template <int NT>
__device__ __attribute__((always_inline)) inline void fold_fast2(float2 *X0, float2 *X1,
                                                                 const RingDesc &d,
                                                                 const FastModes2<NT> &raw,
                                                                 int mmax)
{
    constexpr int QM = FastModes2<NT>::Q;
    const int tid = threadIdx.x;
    double2 ph, step;
    {
        double sn, cs;
        sincos((double)tid * d.phi0, &sn, &cs);
        ph = make_double2(cs, sn);
        sincos((double)NT * d.phi0, &sn, &cs);
        step = make_double2(cs, sn);
    }
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int m = tid + q * NT;
        if (m <= mmax) {
            const float4 r = raw.v[q];
            double2 v0 = make_double2((double)r.x, (double)r.y);
            double2 v1 = make_double2((double)r.z, (double)r.w);
            if (m == 0) { v0.y = 0.0; v1.y = 0.0; }
            X0[PadIdx::at(m)] = cvt<float2>(cmul(ph, v0));
            X1[PadIdx::at(m)] = cvt<float2>(cmul(ph, v1));
        }
        ph = cmul(ph, step);
    }
    __syncthreads();
    const int n = d.n;
    const int h = n / 2;
    const int B = h + 1;
    if (n > mmax) {
        for (int k = tid; k <= h; k += NT) {
            double2 F0 = (k <= mmax) ? todbl(X0[PadIdx::at(k)]) : make_double2(0.0, 0.0);
            double2 F1 = (k <= mmax) ? todbl(X1[PadIdx::at(k)]) : make_double2(0.0, 0.0);
            if (k >= 1 && n - k <= mmax) {
                F0 = cadd(F0, conjd(todbl(X0[PadIdx::at(n - k)])));
                F1 = cadd(F1, conjd(todbl(X1[PadIdx::at(n - k)])));
            }
            X0[PadIdx::at(k)] = cvt<float2>(F0);
            X1[PadIdx::at(k)] = cvt<float2>(F1);
        }
    } else if (B >= NT) {
        for (int k = tid; k <= h; k += NT) {
            const int jmax = (mmax + k) / n;
            double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;
            for (int j = 0; j <= jmax; ++j) {
                if (k + j * n <= mmax) {
                    const double2 a = todbl(X0[PadIdx::at(k + j * n)]);
                    const double2 c = todbl(X1[PadIdx::at(k + j * n)]);
                    s0r += a.x; s0i += a.y; s1r += c.x; s1i += c.y;
                }
                if (j >= 1) {
                    const double2 a = todbl(X0[PadIdx::at(j * n - k)]);
                    const double2 c = todbl(X1[PadIdx::at(j * n - k)]);
                    s0r += a.x; s0i -= a.y; s1r += c.x; s1i -= c.y;
                }
            }
            X0[PadIdx::at(k)] = cplx<float2>(s0r, s0i);
            X1[PadIdx::at(k)] = cplx<float2>(s1r, s1i);
        }
    } else {
        const int G = NT / B;
        const int kk = tid % B, g = tid / B;
        double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;
        if (g < G) {
            const int jmax = (mmax + kk) / n;
            for (int j = g; j <= jmax; j += G) {
                if (kk + j * n <= mmax) {
                    const double2 a = todbl(X0[PadIdx::at(kk + j * n)]);
                    const double2 c = todbl(X1[PadIdx::at(kk + j * n)]);
                    s0r += a.x; s0i += a.y; s1r += c.x; s1i += c.y;
                }
                if (j >= 1) {
                    const double2 a = todbl(X0[PadIdx::at(j * n - kk)]);
                    const double2 c = todbl(X1[PadIdx::at(j * n - kk)]);
                    s0r += a.x; s0i -= a.y; s1r += c.x; s1i -= c.y;
                }
            }
        }
        __syncthreads();
        if (g < G) {
            X0[PadIdx::at(g * B + kk)] = cplx<float2>(s0r, s0i);
            X1[PadIdx::at(g * B + kk)] = cplx<float2>(s1r, s1i);
        }
        __syncthreads();
        if (tid < B) {
            double t0r = 0.0, t0i = 0.0, t1r = 0.0, t1i = 0.0;
            for (int q = 0; q < G; ++q) {
                const double2 a = todbl(X0[PadIdx::at(q * B + tid)]);
                const double2 c = todbl(X1[PadIdx::at(q * B + tid)]);
                t0r += a.x; t0i += a.y; t1r += c.x; t1i += c.y;
            }
            X0[PadIdx::at(tid)] = cplx<float2>(t0r, t0i);
            X1[PadIdx::at(tid)] = cplx<float2>(t1r, t1i);
        }
    }
    __syncthreads();
}

// fast_pass over both buffers.
template <int R>
__device__ __attribute__((always_inline)) inline void fast_pass2(float2 *X0, float2 *X1,
                                                                 const float2 *T, int h, int Ns,
                                                                 bool first, bool last,
                                                                 double *__restrict__ out0,
                                                                 double *__restrict__ out1,
                                                                 bool two)
{
    typedef float2 C;
    constexpr int NT = kFastThreads;
    constexpr int MAXQ = fast_maxq(R);
    const int nb = h / R;
    const int tstep0 = (h / (Ns * R)) * 2;
    const unsigned magic = (unsigned)((0x100000000ull + (unsigned)Ns - 1) / (unsigned)Ns);
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    C a[MAXQ][R], b[MAXQ][R];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = tid + q * NT;
        if (j < nb) {
            if (first) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int k = j + r * nb;
                    const C w = tw_at(T, k);
                    const C F0 = X0[PadIdx::at(k)], G0 = X0[PadIdx::at(h - k)];
                    const C F1 = X1[PadIdx::at(k)], G1 = X1[PadIdx::at(h - k)];
                    a[q][r] = cadd(cadd(F0, conjd(G0)), muli(cmul(w, csub(F0, conjd(G0))), +1));
                    b[q][r] = cadd(cadd(F1, conjd(G1)), muli(cmul(w, csub(F1, conjd(G1))), +1));
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int k = PadIdx::at(j + r * nb);
                    a[q][r] = X0[k];
                    b[q][r] = X1[k];
                }
            }
            if (Ns > 1) {
                const int jq = (int)__umulhi((unsigned)j, magic);
                const int ts = tstep0 * (j - jq * Ns);
                if (ts != 0) {
                    const C w1 = tw_at(T, ts);
                    C wr = w1;
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        a[q][r] = cmul(a[q][r], wr);
                        b[q][r] = cmul(b[q][r], wr);
                        wr = cmul(wr, w1);
                    }
                }
            }
            small_dft<R, C>(a[q], +1);
            small_dft<R, C>(b[q], +1);
        }
    }
    if (last) {
        const bool al = ((reinterpret_cast<uintptr_t>(out0) | reinterpret_cast<uintptr_t>(out1)) &
                         15) == 0;
        double2 *o0 = reinterpret_cast<double2 *>(out0);
        double2 *o1 = reinterpret_cast<double2 *>(out1);
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int j = tid + q * NT;
            if (j < nb) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = j + r * nb;
                    if (al) {
                        o0[i] = todbl(a[q][r]);
                        if (two) o1[i] = todbl(b[q][r]);
                    } else {
                        out0[2 * i] = (double)a[q][r].x;
                        out0[2 * i + 1] = (double)a[q][r].y;
                        if (two) {
                            out1[2 * i] = (double)b[q][r].x;
                            out1[2 * i + 1] = (double)b[q][r].y;
                        }
                    }
                }
            }
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int j = tid + q * NT;
            if (j < nb) {
                const int jq = (Ns == 1) ? j : (int)__umulhi((unsigned)j, magic);
                const int base = jq * Ns * R + (j - jq * Ns);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int k = PadIdx::at(base + r * Ns);
                    X0[k] = a[q][r];
                    X1[k] = b[q][r];
                }
            }
        }
        __syncthreads();
    }
}

__device__ __attribute__((always_inline)) inline void fft_fast2(float2 *X0, float2 *X1,
                                                                const float2 *T,
                                                                const RingDesc &d,
                                                                double *__restrict__ out0,
                                                                double *__restrict__ out1,
                                                                bool two)
{
    const int h = d.n / 2;
    int Ns = 1;
    for (int p = 0; p < d.np; ++p) {
        const int R = (int)((d.rads >> (5 * p)) & 31);
        const bool first = p == 0, last = p == d.np - 1;
        switch (R) {
        case 16: fast_pass2<16>(X0, X1, T, h, Ns, first, last, out0, out1, two); break;
        case 8: fast_pass2<8>(X0, X1, T, h, Ns, first, last, out0, out1, two); break;
        case 4: fast_pass2<4>(X0, X1, T, h, Ns, first, last, out0, out1, two); break;
        case 2: fast_pass2<2>(X0, X1, T, h, Ns, first, last, out0, out1, two); break;
        case 7: fast_pass2<7>(X0, X1, T, h, Ns, first, last, out0, out1, two); break;
        case 5: fast_pass2<5>(X0, X1, T, h, Ns, first, last, out0, out1, two); break;
        default: fast_pass2<3>(X0, X1, T, h, Ns, first, last, out0, out1, two); break;
        }
        Ns *= R;
    }
}

// Persistent over (ring, map pair) items, ring by ring (XCD x takes the
// rings i = x mod 8).  LDS: two spectra of lds.fft_entries each, then the
// twiddle table.
__global__ __launch_bounds__(kFastThreads, 2) void k_ring_synth_fast2(
    const int *__restrict__ ids, int count, int nmaps, const RingDesc *__restrict__ rings,
    const float2 *__restrict__ pool32, const float2 *__restrict__ delta,
    const int *__restrict__ minv, int mcontig, int mmax, DeltaLayout dl,
    double *__restrict__ map, long long npix, RingLds lds)
{
    extern __shared__ double2 lds_raw[];
    float2 *X0 = reinterpret_cast<float2 *>(lds_raw);
    float2 *X1 = X0 + lds.fft_entries;
    float2 *T = X1 + lds.fft_entries;
    const int npairs = (nmaps + 1) / 2;
    const bool aligned = (nmaps % 2) == 0;
    const int per = (int)(gridDim.x / 8);
    const int x = (int)(blockIdx.x % 8), w = (int)(blockIdx.x / 8);
    long long lo, hi;
    xcd_share<true>(count, npairs, x, lo, hi);
    long long it = lo + w;
    if (it >= hi) return;
    int i, pi;
    xcd_item<true>(it, count, npairs, x, i, pi);
    int r = ids[i];
    long long b = 2LL * pi;
    bool two = b + 1 < nmaps;
    FastModes2<kFastThreads> raw;
    load_fast2<kFastThreads>(raw, delta + b * dl.map + r * dl.ring, dl.m, minv, mcontig, mmax,
                             aligned, two);
    for (bool first = true;; first = false) {
        const RingDesc d = rings[r];
        double *out0 = map + b * npix + d.start;
        double *out1 = two ? out0 + npix : out0;
        const bool two_now = two;
        if (!first) __syncthreads();   // the previous ring's last pass has read X0, X1, T
        load_tw<kFastThreads>(T, pool32 + d.tw, d.n);
        fold_fast2<kFastThreads>(X0, X1, d, raw, mmax);
        const long long nx = it + per;
        if (nx < hi) {
            xcd_item<true>(nx, count, npairs, x, i, pi);
            r = ids[i];
            b = 2LL * pi;
            two = b + 1 < nmaps;
            load_fast2<kFastThreads>(raw, delta + b * dl.map + r * dl.ring, dl.m, minv, mcontig,
                                     mmax, aligned, two);
        }
        fft_fast2(X0, X1, T, d, out0, out1, two_now);
        if (nx >= hi) break;
        it = nx;
    }
}

//
// Persistent: the grid is a multiple of 8 workgroups; the (map, ring) items,
// in the order of ring_item, are split into 8 contiguous ranges, one per XCD
// (workgroups are dealt to the XCDs round-robin), and the workgroups of an
// XCD take its items in turn.  The loads of a workgroup's
// next ring are issued before the Fourier passes of the current one, so that
// their latency is hidden behind the passes.
// This kernel takes complex128 Delta (FP64 plans, or a caller's Delta): its
// passes run in complex128, two workgroups per CU.  The mixed forms'
// complex64 Delta goes to k_ring_synth_fast2 (two maps per workgroup, the
// passes in complex64; measured on the belt rings of 16 maps: complex128 one
// map per workgroup 3.88 ms, complex64 one map per workgroup at three per CU
// 3.10 ms, two maps per workgroup 2.47 ms).
template <typename DT> struct FastPrec;
template <> struct FastPrec<double2> {
    typedef double2 C;
    static constexpr int kBlocks = 2;
};

template <typename DT>
__global__ __launch_bounds__(kFastThreads, FastPrec<DT>::kBlocks) void k_ring_synth_fast(
    const int *__restrict__ ids, int count, int nmaps, const RingDesc *__restrict__ rings,
    const double2 *__restrict__ pool, const DT *__restrict__ delta,
    const int *__restrict__ minv, int mcontig, int mmax, DeltaLayout dl,
    double *__restrict__ map, long long npix, RingLds lds)
{
    typedef typename FastPrec<DT>::C C;
    extern __shared__ double2 lds_raw[];
    C *buf = reinterpret_cast<C *>(lds_raw);
    C *T = buf + lds.fft_entries;
    const int per = (int)(gridDim.x / 8);
    const int x = (int)(blockIdx.x % 8), w = (int)(blockIdx.x / 8);
    long long lo, hi;
    xcd_share<RingMajor<DT>::value>(count, nmaps, x, lo, hi);
    long long it = lo + w;
    if (it >= hi) return;
    int i, bi;
    xcd_item<RingMajor<DT>::value>(it, count, nmaps, x, i, bi);
    long long b = bi;
    int r = ids[i];
    FastModes<kFastThreads, DT> raw;
    load_fast<kFastThreads>(raw, delta + b * dl.map + r * dl.ring, dl.m, minv, mcontig, mmax);
    for (bool first = true;; first = false) {
        const RingDesc d = rings[r];
        double *out = map + b * npix + d.start;
        if (!first) __syncthreads();   // the previous ring's last pass has read buf and T
        load_tw<kFastThreads>(T, pool + d.tw, d.n);
        fold_fast<kFastThreads>(buf, d, raw, mmax);
        const long long nx = it + per;
        if (nx < hi) {
            xcd_item<RingMajor<DT>::value>(nx, count, nmaps, x, i, bi);
            b = bi;
            r = ids[i];
            load_fast<kFastThreads>(raw, delta + b * dl.map + r * dl.ring, dl.m, minv, mcontig, mmax);
        }
        fft_fast<kFastThreads, C>(buf, T, d, out);
        if (nx >= hi) break;
        it = nx;
    }
}

__global__ __launch_bounds__(kFastThreads, 2) void k_ring_synth_batch_fast(
    const int2 *__restrict__ items, const BatchMap *__restrict__ maps,
    double *const *__restrict__ outs, const char *__restrict__ ws, RingLds lds)
{
    extern __shared__ double2 buf[];
    const int2 it = items[xcd_logical(blockIdx.x, gridDim.x)];
    const BatchMap &bm = maps[it.x];
    const RingDesc d = bm.rings[it.y];
    const double2 *delta = reinterpret_cast<const double2 *>(ws + bm.delta_off);
    synth_fast<kFastThreads, double2>(buf, buf + lds.fft_entries, d, bm.pool, delta + it.y,
                                      bm.nrings, bm.minv, bm.mcontig, bm.mmax,
                                      outs[it.x] + d.start);
}

// ---------------------------------------------------------------------------
// Bluestein fast path of the mixed forms: even rings whose half length
// h = 2 len has a len that is not 7-smooth.  As in split_bluestein, the
// h-point DFT of Z is z_j = E_j + w^j O_j, z_{j+len} = E_j - w^j O_j
// (w = e^{2 pi i / h}), with E, O the len-point DFTs of Z's even- and
// odd-indexed entries, each a Bluestein transform: a cyclic convolution of
// 7-smooth length nb >= 2 len - 1 with the conjugate chirp.  The two
// convolutions run side by side in two padded complex64 LDS buffers X and Y:
// each Stockham pass takes its butterflies in both, so one barrier pair
// serves the two.  The first forward pass forms Z from the folded spectrum
// and multiplies by the chirp, the first inverse pass multiplies by the
// kernel's spectrum bq, and the last inverse pass multiplies by the chirp,
// combines E and O and writes the pixels.  The chirp
// c_k = e^{i pi k^2 / len} = e^{2 pi i (k^2 mod h) / h} is read from the
// ring's n-th roots (n = 2 h) in LDS.
enum BlueIn { kBlueInZ, kBlueInBuf, kBlueInBq };

struct BlueRing {
    int h, len;
    float inv_h;         // 1 / h, rounded
    const float2 *bq;    // kernel spectrum DFT^-(conj chirp, wrapped) / nb
};

// k^2 mod h for k < 2^11 and h < 2^13, exactly: k^2 < 2^22 is exact in
// FP32, and the rounded quotient k^2 * (1/h) is within 0.05 of k^2 / h, so
// one correction either way restores the remainder.
__device__ inline int sq_mod(int k, int h, float inv_h)
{
    const int k2 = k * k;
    const int q = (int)((float)k2 * inv_h);
    int r = k2 - q * h;
    r = (r < 0) ? r + h : r;
    return (r >= h) ? r - h : r;
}

// One pass of radix R over both nb-point buffers of each of NM maps (input
// index j + r nb/R, output index (j / Ns) Ns R + j % Ns + r Ns); TB holds the
// nb-th roots, TW the n-th roots; the maps share every twiddle.  last:
// Ns R = nb, the pass ends in the pixel stores (of the first nout maps).
// The kernel runs one map per workgroup: two maps (four buffers) fit one
// workgroup per CU and measured slower (caps of 16 maps at nside 2048:
// 4.01 against 3.75 ms), unlike the fast path's two-map kernel.
template <int R, int sign, int NM>
__device__ __attribute__((always_inline)) inline void blue_pass(
    float2 *const (&X)[NM], float2 *const (&Y)[NM], const float2 *TW, const float2 *TB, int L,
    int Ns, int in, bool last, const BlueRing &br, double *const (&out)[NM], int nout)
{
    typedef float2 C;
    constexpr int NT = kBlueThreads;
    const int nbf = L / R;   // the plan admits nb / R <= NT: one butterfly per thread
    const int tstep0 = L / (Ns * R);
    const unsigned magic = (unsigned)((0x100000000ull + (unsigned)Ns - 1) / (unsigned)Ns);
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int j = tid;
    C a[NM][R], b[NM][R];
    if (j < nbf) {
        if (in == kBlueInZ) {
            const int h = br.h;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = j + r * nbf;
                if (k < br.len) {
                    // Z_t = (F_t + conj F_{h-t}) + i e^{2 pi i t/n} (F_t - conj F_{h-t}),
                    // t = 2k and 2k + 1
                    const int t0 = 2 * k, t1 = t0 + 1;
                    const C w0 = tw_at(TW, t0), w1 = tw_at(TW, t1);
                    const C c = tw_at(TW, 2 * sq_mod(k, h, br.inv_h));
#pragma unroll
                    for (int mm = 0; mm < NM; ++mm) {
                        const C F0 = X[mm][PadIdx::at(t0)], G0 = X[mm][PadIdx::at(h - t0)];
                        const C F1 = X[mm][PadIdx::at(t1)], G1 = X[mm][PadIdx::at(h - t1)];
                        const C z0 = cadd(cadd(F0, conjd(G0)), muli(cmul(w0, csub(F0, conjd(G0))), +1));
                        const C z1 = cadd(cadd(F1, conjd(G1)), muli(cmul(w1, csub(F1, conjd(G1))), +1));
                        a[mm][r] = cmul(z0, c);
                        b[mm][r] = cmul(z1, c);
                    }
                } else {
#pragma unroll
                    for (int mm = 0; mm < NM; ++mm) {
                        a[mm][r] = make_float2(0.f, 0.f);
                        b[mm][r] = make_float2(0.f, 0.f);
                    }
                }
            }
        } else if (in == kBlueInBq) {
            // the kernel spectrum's global loads go out before the LDS reads
            C wq[R];
#pragma unroll
            for (int r = 0; r < R; ++r) wq[r] = br.bq[j + r * nbf];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = PadIdx::at(j + r * nbf);
#pragma unroll
                for (int mm = 0; mm < NM; ++mm) {
                    a[mm][r] = cmul(X[mm][k], wq[r]);
                    b[mm][r] = cmul(Y[mm][k], wq[r]);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = PadIdx::at(j + r * nbf);
#pragma unroll
                for (int mm = 0; mm < NM; ++mm) {
                    a[mm][r] = X[mm][k];
                    b[mm][r] = Y[mm][k];
                }
            }
        }
        if (Ns > 1) {
            const int jq = (int)__umulhi((unsigned)j, magic);
            const int ts = tstep0 * (j - jq * Ns);
            if (ts != 0) {
                C w1 = tw_at(TB, ts);
                if (sign < 0) w1.y = -w1.y;
                C wr = w1;
#pragma unroll
                for (int r = 1; r < R; ++r) {
#pragma unroll
                    for (int mm = 0; mm < NM; ++mm) {
                        a[mm][r] = cmul(a[mm][r], wr);
                        b[mm][r] = cmul(b[mm][r], wr);
                    }
                    wr = cmul(wr, w1);
                }
            }
        }
#pragma unroll
        for (int mm = 0; mm < NM; ++mm) {
            small_dft<R, C>(a[mm], sign);
            small_dft<R, C>(b[mm], sign);
        }
    }
    if (last) {
        // j < Ns: outputs o = j + r nbf; for o < len, E_o = c_o a, O_o = c_o b
        const int h = br.h, len = br.len;
        if (j < nbf) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int o = j + r * nbf;
                if (o < len) {
                    const C c = tw_at(TW, 2 * sq_mod(o, h, br.inv_h));
                    const C w = tw_at(TW, 2 * o);
#pragma unroll
                    for (int mm = 0; mm < NM; ++mm) {
                        if (mm < nout) {
                            const C E = cmul(a[mm][r], c);
                            const C t = cmul(w, cmul(b[mm][r], c));
                            const double2 z0 = todbl(cadd(E, t)), z1 = todbl(csub(E, t));
                            double *op = out[mm];
                            if ((reinterpret_cast<uintptr_t>(op) & 15) == 0) {
                                double2 *o2 = reinterpret_cast<double2 *>(op);
                                o2[o] = z0;
                                o2[o + len] = z1;
                            } else {
                                op[2 * o] = z0.x;
                                op[2 * o + 1] = z0.y;
                                op[2 * (o + len)] = z1.x;
                                op[2 * (o + len) + 1] = z1.y;
                            }
                        }
                    }
                }
            }
        }
    } else {
        __syncthreads();
        if (j < nbf) {
            const int jq = (Ns == 1) ? j : (int)__umulhi((unsigned)j, magic);
            const int base = jq * Ns * R + (j - jq * Ns);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = PadIdx::at(base + r * Ns);
#pragma unroll
                for (int mm = 0; mm < NM; ++mm) {
                    X[mm][k] = a[mm][r];
                    Y[mm][k] = b[mm][r];
                }
            }
        }
        __syncthreads();
    }
}

// The passes of one direction of a Bluestein fast-path ring's convolutions:
// sign -1 (forward, from the folded spectra) or +1 (inverse, ending in the
// pixel stores).
template <int sign, int NM>
__device__ __attribute__((always_inline)) inline void blue_dir(
    float2 *const (&X)[NM], float2 *const (&Y)[NM], const float2 *TW, const float2 *TB,
    const RingDesc &d, const BlueRing &br, double *const (&out)[NM], int nout)
{
    const int L = d.nb;
    int Ns = 1;
    for (int p = 0; p < d.np; ++p) {
        const int R = (int)((d.rads >> (5 * p)) & 31);
        const int in = (p > 0) ? kBlueInBuf : (sign < 0 ? kBlueInZ : kBlueInBq);
        const bool last = sign > 0 && p == d.np - 1;
        switch (R) {
        case 8: blue_pass<8, sign, NM>(X, Y, TW, TB, L, Ns, in, last, br, out, nout); break;
        case 4: blue_pass<4, sign, NM>(X, Y, TW, TB, L, Ns, in, last, br, out, nout); break;
        case 2: blue_pass<2, sign, NM>(X, Y, TW, TB, L, Ns, in, last, br, out, nout); break;
        case 7: blue_pass<7, sign, NM>(X, Y, TW, TB, L, Ns, in, last, br, out, nout); break;
        case 5: blue_pass<5, sign, NM>(X, Y, TW, TB, L, Ns, in, last, br, out, nout); break;
        default: blue_pass<3, sign, NM>(X, Y, TW, TB, L, Ns, in, last, br, out, nout); break;
        }
        Ns *= R;
    }
}

// Persistent like k_ring_synth_fast; complex64 Delta [m][ring][map] only.
// Items are (ring, map pair), ring by ring: one 16-byte load per mode brings
// the modes of maps 2p and 2p + 1 (paced like load_fast), and the two maps
// are then folded and transformed one after the other in the same buffers
// (half the load rounds per map: caps of 16 maps at nside 2048 3.73 ->
// 3.33 ms).  The next pair's loads go out after the second map's fold.
__global__ __launch_bounds__(kBlueThreads, 4) void k_ring_synth_blue(
    const int *__restrict__ ids, int count, int nmaps, const RingDesc *__restrict__ rings,
    const float2 *__restrict__ pool32, const float2 *__restrict__ delta,
    const int *__restrict__ minv, int mcontig, int mmax, DeltaLayout dl,
    double *__restrict__ map, long long npix, RingLds lds)
{
    typedef float2 C;
    constexpr int QM = FastModes2<kBlueThreads>::Q;
    extern __shared__ double2 lds_raw[];
    C *X = reinterpret_cast<C *>(lds_raw);
    C *Y = X + lds.fft_entries;
    C *TW = Y + lds.y_entries;
    C *TB = TW + lds.tw_entries;
    float2 *const Xs[1] = {X}, *const Ys[1] = {Y};
    const int npairs = (nmaps + 1) / 2;
    const bool aligned = (nmaps % 2) == 0;
    const int per = (int)(gridDim.x / 8);
    const int x = (int)(blockIdx.x % 8), w = (int)(blockIdx.x / 8);
    long long lo, hi;
    xcd_share<true>(count, npairs, x, lo, hi);
    long long it = lo + w;
    if (it >= hi) return;
    int i, pi;
    xcd_item<true>(it, count, npairs, x, i, pi);
    int r = ids[i];
    long long b = 2LL * pi;
    bool two = b + 1 < nmaps;
    FastModes2<kBlueThreads> raw;
    load_fast2<kBlueThreads>(raw, delta + b * dl.map + r * dl.ring, dl.m, minv, mcontig, mmax,
                             aligned, two);
    for (bool first = true;; first = false) {
        const RingDesc d = rings[r];
        BlueRing br;
        br.h = d.n / 2;
        br.len = br.h / 2;
        br.inv_h = 1.0f / (float)br.h;
        br.bq = pool32 + d.bq;
        double *const outA[1] = {map + b * npix + d.start};
        double *const outB[1] = {map + (b + 1) * npix + d.start};
        const bool twoB = two;
        if (!first) __syncthreads();   // the previous ring's last pass has read TW
        load_tw<kBlueThreads>(TW, pool32 + d.tw, d.n);
        load_tw<kBlueThreads>(TB, pool32 + d.twb, d.nb);
        FastModes<kBlueThreads, float2> one;
#pragma unroll
        for (int q = 0; q < QM; ++q) one.v[q] = make_float2(raw.v[q].x, raw.v[q].y);
        fold_fast<kBlueThreads>(X, d, one, mmax);
        blue_dir<-1, 1>(Xs, Ys, TW, TB, d, br, outA, 1);
        blue_dir<+1, 1>(Xs, Ys, TW, TB, d, br, outA, 1);
        if (twoB) {
#pragma unroll
            for (int q = 0; q < QM; ++q) one.v[q] = make_float2(raw.v[q].z, raw.v[q].w);
            __syncthreads();   // the first map's last pass has read X and Y
            fold_fast<kBlueThreads>(X, d, one, mmax);
        }
        const long long nx = it + per;
        if (nx < hi) {
            xcd_item<true>(nx, count, npairs, x, i, pi);
            r = ids[i];
            b = 2LL * pi;
            two = b + 1 < nmaps;
            load_fast2<kBlueThreads>(raw, delta + b * dl.map + r * dl.ring, dl.m, minv, mcontig,
                                     mmax, aligned, two);
        }
        if (twoB) {
            blue_dir<-1, 1>(Xs, Ys, TW, TB, d, br, outB, 1);
            blue_dir<+1, 1>(Xs, Ys, TW, TB, d, br, outB, 1);
        }
        if (nx >= hi) break;
        it = nx;
    }
}

template <int NT, int MAXN, typename DT>
__global__ __launch_bounds__(NT, 4) void k_ring_synth(
    const int *__restrict__ ids, int count, int nmaps, const RingDesc *__restrict__ rings,
    const double2 *__restrict__ pool, const DT *__restrict__ delta,
    const int *__restrict__ minv, int mcontig, int mmax, DeltaLayout dl,
    double *__restrict__ map, long long npix, RingLds lds)
{
    extern __shared__ double2 buf[];
    int i, bi;
    ring_item<RingMajor<DT>::value>(xcd_logical(blockIdx.x, gridDim.x), count, nmaps, i, bi);
    const int r = ids[i];
    const long long b = bi;
    const RingDesc d = rings[r];
    double2 *tw = buf + lds.fft_entries;
    const RingTables rt = {tw, tw + lds.tw_entries};
    synth_ring<NT, MAXN, false, false>(buf, rt, d,
                               pool, delta + b * dl.map + r * dl.ring, dl.m, minv,
                               mcontig, mmax, map + b * npix + d.start);
}

// Batched synthesis: work item (map, ring) of a batch of plans.
template <int NT, int MAXN>
__global__ __launch_bounds__(NT, 4) void k_ring_synth_batch(
    const int2 *__restrict__ items, const BatchMap *__restrict__ maps,
    double *const *__restrict__ outs, const char *__restrict__ ws, RingLds lds)
{
    extern __shared__ double2 buf[];
    const int2 it = items[xcd_logical(blockIdx.x, gridDim.x)];
    const BatchMap &bm = maps[it.x];
    const RingDesc d = bm.rings[it.y];
    const double2 *delta = reinterpret_cast<const double2 *>(ws + bm.delta_off);
    double2 *tw = buf + lds.fft_entries;
    const RingTables rt = {tw, tw + lds.tw_entries};
    synth_ring<NT, MAXN, false, true>(buf, rt, d,
                                bm.pool, delta + it.y, bm.nrings, bm.minv, bm.mcontig,
                                bm.mmax, outs[it.x] + d.start);
}

// Analysis (adjoint of the synthesis): G_k by a real DFT, then
// Dt_m = c_m e^{-i m phi0} G_{m mod n} with c_0 = 1 and c_m = cfac for m > 0
// (cfac = 2: the adjoint; cfac = 1: the quadrature analysis), times the
// ring's pixel weight rw[r] when rw is given.
template <int NT, int MAXN>
__global__ __launch_bounds__(NT, 4) void k_ring_anal(
    const int *__restrict__ ids, const RingDesc *__restrict__ rings,
    const double2 *__restrict__ pool, const double *__restrict__ map, long long npix,
    const int *__restrict__ mval, int mcontig, int nm, int nrings, double2 *__restrict__ dt,
    RingLds lds, const double *__restrict__ rw, double cfac)
{
    extern __shared__ double2 buf[];
    const int r = ids[xcd_logical(blockIdx.x, gridDim.x)];
    const int b = blockIdx.y;
    const RingDesc d = rings[r];
    const RingTables rt = {buf + lds.fft_entries, buf + lds.fft_entries + lds.tw_entries};
    Chirps<NT, MAXN, false> ch;
    ring_tables_load<NT, MAXN, false>(rt, d, pool, ch);
    const double *in = map + (long long)b * npix + d.start;
    const int n = d.n;
    const bool even = (n % 2) == 0;
    const int h = n / 2;
    const int tid = threadIdx.x;
    if (even) {
        if ((reinterpret_cast<uintptr_t>(in) & 15) == 0) {
            const double2 *i2 = reinterpret_cast<const double2 *>(in);
            for (int j = tid; j < h; j += NT) buf[j] = i2[j];
        } else {
            for (int j = tid; j < h; j += NT) buf[j] = make_double2(in[2 * j], in[2 * j + 1]);
        }
        __syncthreads();
        ring_dft<NT, MAXN, false>(buf, d, -1, pool, rt, ch);
        for (int k = tid; k <= h / 2; k += NT) {
            const int k2 = h - k;
            const double2 Zk = buf[k];
            const double2 Zk2 = buf[k2 == h ? 0 : k2];
            // G_k = (Z_k + conj Z_{h-k})/2 - (i/2) e^{-2 pi i k/n} (Z_k - conj Z_{h-k})
            const double2 a1 = cadd(Zk, conjd(Zk2)), b1 = csub(Zk, conjd(Zk2));
            const double2 G1 = csub(a1, muli(cmul(conjd(tw_at(rt.TW, k)), b1), +1));
            const double2 a2 = cadd(Zk2, conjd(Zk)), b2 = csub(Zk2, conjd(Zk));
            const double2 G2 = csub(a2, muli(cmul(conjd(tw_at(rt.TW, k2)), b2), +1));
            buf[k] = make_double2(0.5 * G1.x, 0.5 * G1.y);
            if (k2 != k) buf[k2] = make_double2(0.5 * G2.x, 0.5 * G2.y);
        }
        __syncthreads();
    } else {
        for (int j = tid; j < n; j += NT) buf[j] = make_double2(in[j], 0.0);
        __syncthreads();
        ring_dft<NT, MAXN, false>(buf, d, -1, pool, rt, ch);
    }
    const int kmax = even ? h : n - 1;
    double2 *orow = dt + (long long)b * nm * nrings + r;   // [m][ring]
    double2 step, ph;   // e^{-i NT phi0}, e^{-i m phi0} for this thread's mode
    {
        double sn, cs;
        sincos((double)NT * d.phi0, &sn, &cs);
        step = make_double2(cs, -sn);
    }
    bool first = true;
    const double w = rw ? rw[r] : 1.0;
    for (int i = tid; i < nm; i += NT) {
        const int m = mval[i];
        const int kk = m % n;
        const double2 G = (kk <= kmax) ? buf[kk] : conjd(buf[n - kk]);
        if (first || !mcontig) {
            double sn, cs;
            sincos((double)m * d.phi0, &sn, &cs);
            ph = make_double2(cs, -sn);
            first = false;
        } else {
            ph = cmul(ph, step);
        }
        double2 v;
        if (m == 0) {
            v = make_double2(G.x, 0.0);
        } else {
            v = cmul(G, ph);
            v.x *= cfac; v.y *= cfac;
        }
        if (rw) { v.x *= w; v.y *= w; }
        orow[(long long)i * nrings] = v;
    }
}

// Spectrum of the Bluestein kernel b_k = conj(c_k) (wrapped to negative k),
// scaled by 1 / nb, one workgroup per listed ring.
__global__ __launch_bounds__(512) void k_bluestein_prep(
    const RingDesc *__restrict__ rings, const int *__restrict__ ids, double2 *pool)
{
    extern __shared__ double2 buf[];
    const RingDesc d = rings[ids[blockIdx.x]];
    const int len = d.half ? d.clen / 2 : d.clen, nb = d.nb;
    const double2 *chirp = pool + d.tch;
    for (int k = threadIdx.x; k < nb; k += 512) {
        int m = -1;
        if (k < len) m = k;
        else if (k > nb - len) m = nb - k;
        buf[k] = (m >= 0) ? conjd(chirp[m]) : make_double2(0.0, 0.0);
    }
    load_tw<512>(buf + 8192, pool + d.twb, nb);
    __syncthreads();
    fft_lds<512, 8192>(buf, nb, -1, buf + 8192, 1);
    const double inv = 1.0 / (double)nb;
    for (int k = threadIdx.x; k < nb; k += 512)
        pool[d.bq + k] = make_double2(buf[k].x * inv, buf[k].y * inv);
}

// The layout of the ring stage's Delta by its element type: complex64 is the
// mixed Legendre stage's [m][ring][map], complex128 the FP64 stage's (or a
// caller's) [map][m][ring].
DeltaLayout delta_layout(const sht_plan_s *p, const float2 *)
{
    return DeltaLayout{1, p->nmaps, (long long)p->nrings * p->nmaps};
}
DeltaLayout delta_layout(const sht_plan_s *p, const double2 *)
{
    return DeltaLayout{(long long)p->nm * p->nrings, 1, p->nrings};
}

hipError_t set_lds(const void *fn, size_t bytes)
{
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int NT, int MAXN, typename DT>
hipError_t synth_class(const sht_plan_s *p, const RingClass &rc, const DT *delta, double *map,
                       hipStream_t st)
{
    if (rc.count == 0) return hipSuccess;
    const size_t lds = (size_t)rc.lds.total() * sizeof(double2);
    hipError_t e = set_lds((const void *)k_ring_synth<NT, MAXN, DT>, lds);
    if (e != hipSuccess) return e;
    const long long items = (long long)rc.count * p->nmaps;
    if (items > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_ring_synth<NT, MAXN, DT>), dim3((unsigned)items), dim3(NT), lds, st,
                       rc.d_ids, rc.count, p->nmaps, p->d_rings, p->d_pool, delta, p->d_minv,
                       p->mcontig, p->mmax, delta_layout(p, delta), map, p->npix, rc.lds);
    return hipGetLastError();
}

template <int NT, int MAXN>
hipError_t anal_class(const sht_plan_s *p, int c, const double *map, double2 *dt, hipStream_t st,
                      const double *rw, double cfac)
{
    const RingClass &rc = p->cls[c];
    if (rc.count == 0) return hipSuccess;
    const size_t lds =
        (size_t)(rc.lds.fft_entries + rc.lds.tw_entries + rc.lds.tb_entries) * sizeof(double2);
    hipError_t e = set_lds((const void *)k_ring_anal<NT, MAXN>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ring_anal<NT, MAXN>), dim3((unsigned)rc.count, (unsigned)p->nmaps),
                       dim3(NT), lds, st, rc.d_ids, p->d_rings, p->d_pool, map, p->npix,
                       p->d_mval, p->mcontig, p->nm, p->nrings, dt, rc.lds, rw, cfac);
    return hipGetLastError();
}

}  // namespace

// Size classes (FFT length limit): 0 -> 2048, 1 -> 4096, 2 -> 8192.
static_assert(kClassThreads[0] == 256 && kClassThreads[1] == 512 && kClassThreads[2] == 1024,
              "class thread counts must match the kernel instantiations");
template <typename DT>
hipError_t synth_fast_class(const sht_plan_s *p, const DT *delta, double *map, hipStream_t st)
{
    const RingClass &rc = p->scls[kFastClass];
    if (rc.count == 0) return hipSuccess;
    const size_t lds = (size_t)rc.lds.total() * sizeof(typename FastPrec<DT>::C);
    hipError_t e = set_lds((const void *)k_ring_synth_fast<DT>, lds);
    if (e != hipSuccess) return e;
    // as many workgroups per CU as the LDS of a ring allows (two), a multiple of 8
    const long long items = (long long)rc.count * p->nmaps;
    long long grid = (long long)FastPrec<DT>::kBlocks * (p->num_cus > 0 ? p->num_cus : 256);
    if (grid > items) grid = items;
    grid = ((grid + 7) / 8) * 8;
    hipLaunchKernelGGL((k_ring_synth_fast<DT>), dim3((unsigned)grid), dim3(kFastThreads), lds,
                       st, rc.d_ids, rc.count, p->nmaps, p->d_rings, p->d_pool, delta,
                       p->d_minv, p->mcontig, p->mmax, delta_layout(p, delta), map, p->npix,
                       rc.lds);
    return hipGetLastError();
}

// complex64 Delta: two maps per workgroup, two workgroups per CU.
template <>
hipError_t synth_fast_class<float2>(const sht_plan_s *p, const float2 *delta, double *map,
                                    hipStream_t st)
{
    const RingClass &rc = p->scls[kFastClass];
    if (rc.count == 0) return hipSuccess;
    if (!p->d_pool32) return hipErrorInvalidConfiguration;
    const size_t lds =
        (size_t)(2 * rc.lds.fft_entries + rc.lds.tw_entries) * sizeof(float2);
    hipError_t e = set_lds((const void *)k_ring_synth_fast2, lds);
    if (e != hipSuccess) return e;
    const long long items = (long long)rc.count * ((p->nmaps + 1) / 2);
    long long grid = 2LL * (p->num_cus > 0 ? p->num_cus : 256);
    if (grid > items) grid = items;
    grid = ((grid + 7) / 8) * 8;
    hipLaunchKernelGGL(k_ring_synth_fast2, dim3((unsigned)grid), dim3(kFastThreads), lds, st,
                       rc.d_ids, rc.count, p->nmaps, p->d_rings, p->d_pool32, delta, p->d_minv,
                       p->mcontig, p->mmax, delta_layout(p, delta), map, p->npix, rc.lds);
    return hipGetLastError();
}

// The Bluestein fast path (complex64 Delta only): two 512-thread
// workgroups per CU, persistent.
hipError_t synth_blue_class(const sht_plan_s *p, const float2 *delta, double *map,
                            hipStream_t st)
{
    const RingClass &rc = p->scls[kBlueClass];
    if (rc.count == 0) return hipSuccess;
    if (!p->d_pool32) return hipErrorInvalidConfiguration;
    const size_t lds = (size_t)rc.lds.total() * sizeof(float2);
    hipError_t e = set_lds((const void *)k_ring_synth_blue, lds);
    if (e != hipSuccess) return e;
    const long long items = (long long)rc.count * ((p->nmaps + 1) / 2);
    long long grid = 2LL * (p->num_cus > 0 ? p->num_cus : 256);
    if (grid > items) grid = items;
    grid = ((grid + 7) / 8) * 8;
    hipLaunchKernelGGL(k_ring_synth_blue, dim3((unsigned)grid), dim3(kBlueThreads), lds, st,
                       rc.d_ids, rc.count, p->nmaps, p->d_rings, p->d_pool32, delta, p->d_minv,
                       p->mcontig, p->mmax, delta_layout(p, delta), map, p->npix, rc.lds);
    return hipGetLastError();
}

// complex128 Delta (FP64 plans have no ring in the class; a mixed-form plan
// given a caller's complex128 Delta): the class's rings by size class.
hipError_t synth_blue_class(const sht_plan_s *p, const double2 *delta, double *map,
                            hipStream_t st)
{
    hipError_t e = synth_class<1024, 8192, double2>(p, p->bcls[2], delta, map, st);
    if (e == hipSuccess) e = synth_class<512, 4096, double2>(p, p->bcls[1], delta, map, st);
    if (e == hipSuccess) e = synth_class<256, 2048, double2>(p, p->bcls[0], delta, map, st);
    return e;
}

// The fast-path kernel (LDS-bound at two or three workgroups per CU), the
// Bluestein fast path and the size-class kernels write disjoint rings.  For
// large plans the fast path runs on the plan's auxiliary stream beside the
// others (forked from and joined back into the caller's stream by events, so
// the call stays ordered on `st` and capturable): their workgroups then
// share the CUs and fill each other's tails (FP64 size classes: 10.6 -> 10.2
// ms for 16 maps at l_max 4096 / nside 2048; with the mixed forms' two fast
// paths: 5.93 -> 5.84 ms).
// Small plans launch everything on `st` (a fork costs microseconds).
constexpr long long kForkItems = 4096;

template <typename DT>
static hipError_t ring_synth_dt(const sht_plan_s *p, const DT *delta, double *map, hipStream_t st)
{
    const long long fast = (long long)p->scls[kFastClass].count * p->nmaps;
    const long long rest = (long long)(p->scls[0].count + p->scls[1].count + p->scls[2].count +
                                       p->scls[kBlueClass].count) *
                           p->nmaps;
    const bool fork = p->aux_stream && fast > 0 && rest > 0 && fast + rest >= kForkItems;
    // the fork and join events belong to the plan: calls from several host
    // threads take turns through the whole sequence
    std::unique_lock<std::mutex> lock(const_cast<sht_plan_s *>(p)->fork_mu, std::defer_lock);
    if (fork) lock.lock();
    hipError_t e = hipSuccess;
    if (fork) {
        e = hipEventRecord(p->ev_fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->aux_stream, p->ev_fork, 0);
    }
    if (e == hipSuccess) e = synth_fast_class<DT>(p, delta, map, fork ? p->aux_stream : st);
    if (e == hipSuccess) e = synth_blue_class(p, delta, map, st);
    if (e == hipSuccess) e = synth_class<1024, 8192, DT>(p, p->scls[2], delta, map, st);
    if (e == hipSuccess) e = synth_class<512, 4096, DT>(p, p->scls[1], delta, map, st);
    if (e == hipSuccess) e = synth_class<256, 2048, DT>(p, p->scls[0], delta, map, st);
    if (fork) {
        // join even after a failed launch, so that `st` never runs ahead of
        // work already queued on the auxiliary stream
        const hipError_t j = hipEventRecord(p->ev_join, p->aux_stream);
        const hipError_t w = (j == hipSuccess) ? hipStreamWaitEvent(st, p->ev_join, 0) : j;
        if (e == hipSuccess) e = w;
    }
    return e;
}

hipError_t launch_ring_synth(const sht_plan_s *p, const double2 *delta, double *map,
                             hipStream_t st)
{
    return ring_synth_dt(p, delta, map, st);
}

hipError_t launch_ring_synth(const sht_plan_s *p, const float2 *delta, double *map,
                             hipStream_t st)
{
    return ring_synth_dt(p, delta, map, st);
}

// Complex64 Delta widened to complex128 (the stage entry point's layout).
__global__ __launch_bounds__(256) void k_narrow(const double2 *__restrict__ s,
                                                float2 *__restrict__ d, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) d[i] = make_float2((float)s[i].x, (float)s[i].y);
}

hipError_t launch_narrow(const double2 *s, float2 *d, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256;
    if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)nb), dim3(256), 0, st, s, d, n);
    return hipGetLastError();
}

// complex64 [m][ring][map] Delta of the mixed forms -> complex128
// [map][m][ring] (exact), one thread per output entry.
__global__ __launch_bounds__(256) void k_widen_delta(const float2 *__restrict__ s,
                                                     double2 *__restrict__ d, int nmaps, int nm,
                                                     int nrings)
{
    const long long n = (long long)nmaps * nm * nrings;
    const long long o = (long long)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    const long long per_map = (long long)nm * nrings;
    const int b = (int)(o / per_map);
    const long long rem = o - b * per_map;   // i * nrings + r
    const float2 v = s[rem * nmaps + b];
    d[o] = make_double2((double)v.x, (double)v.y);
}

hipError_t launch_widen_delta(const sht_plan_s *p, const float2 *s, double2 *d, hipStream_t st)
{
    const long long n = (long long)p->nmaps * p->nm * p->nrings;
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256;
    if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_widen_delta, dim3((unsigned)nb), dim3(256), 0, st, s, d, p->nmaps, p->nm,
                       p->nrings);
    return hipGetLastError();
}

hipError_t launch_ring_anal(const sht_plan_s *p, const double *map, double2 *dt, hipStream_t st,
                            const double *rw, double cfac)
{
    hipError_t e = anal_class<1024, 8192>(p, 2, map, dt, st, rw, cfac);
    if (e == hipSuccess) e = anal_class<512, 4096>(p, 1, map, dt, st, rw, cfac);
    if (e == hipSuccess) e = anal_class<256, 2048>(p, 0, map, dt, st, rw, cfac);
    return e;
}

// r = s - r over n doubles (residual of the refined analysis)
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ s,
                                                  double *__restrict__ r, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) r[i] = s[i] - r[i];
}

hipError_t launch_residual(const double *s, double *r, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256;
    if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_residual, dim3((unsigned)nb), dim3(256), 0, st, s, r, n);
    return hipGetLastError();
}

template <int NT, int MAXN>
hipError_t synth_batch_class(const BatchClass &bc, const BatchMap *maps, double *const *outs,
                             const void *ws, hipStream_t st)
{
    if (bc.count == 0) return hipSuccess;
    const size_t lds = (size_t)bc.lds.total() * sizeof(double2);
    hipError_t e = set_lds((const void *)k_ring_synth_batch<NT, MAXN>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ring_synth_batch<NT, MAXN>), dim3((unsigned)bc.count), dim3(NT), lds, st,
                       bc.d_items, maps, outs, (const char *)ws, bc.lds);
    return hipGetLastError();
}

hipError_t launch_ring_synth_batch(const BatchClass *cls, const BatchMap *maps,
                                   double *const *outs, const void *ws, hipStream_t st)
{
    hipError_t e = hipSuccess;
    const BatchClass &fc = cls[kFastClass];
    if (fc.count > 0) {
        const size_t lds = (size_t)fc.lds.total() * sizeof(double2);
        e = set_lds((const void *)k_ring_synth_batch_fast, lds);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_ring_synth_batch_fast, dim3((unsigned)fc.count),
                               dim3(kFastThreads), lds, st, fc.d_items, maps, outs,
                               (const char *)ws, fc.lds);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = synth_batch_class<1024, 8192>(cls[2], maps, outs, ws, st);
    if (e == hipSuccess) e = synth_batch_class<512, 4096>(cls[1], maps, outs, ws, st);
    if (e == hipSuccess) e = synth_batch_class<256, 2048>(cls[0], maps, outs, ws, st);
    return e;
}

hipError_t launch_bluestein_prep(const sht_plan_s *p, const int *ring_ids, int nids,
                                 hipStream_t st)
{
    if (nids <= 0) return hipSuccess;
    const size_t lds = (size_t)(8192 + kTwEntries) * sizeof(double2);
    hipError_t e = set_lds((const void *)k_bluestein_prep, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bluestein_prep, dim3((unsigned)nids), dim3(512), lds, st,
                       p->d_rings, ring_ids, p->d_pool);
    return hipGetLastError();
}

}  // namespace sht
