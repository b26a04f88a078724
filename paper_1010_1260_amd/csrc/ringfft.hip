// Per-ring Fourier step of alm2map and of its adjoint, FP64, for gfx950.
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
// One workgroup (512 threads) per ring and map; the whole ring lives in LDS.
// DFTs of 7-smooth length run as a Stockham auto-sort FFT (radices 4, 2, 3,
// 5, 7; every pass loads its butterfly inputs into registers, barriers, and
// stores in place, so one LDS buffer suffices).  Other lengths use
// Bluestein's chirp-z algorithm with a power-of-two convolution whose
// kernel spectrum is precomputed at plan time.  Twiddles come from
// per-length tables computed on the host in extended precision.
#include "sht_internal.h"

namespace sht {
namespace {

constexpr int kRingThreads = 512;
constexpr int kMaxFft = 8192;

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
// sign * i * a
__device__ inline double2 muli(double2 a, int sign)
{
    return sign > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

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
template <int R>
__device__ inline void small_dft(double2 (&v)[R], int sign)
{
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const double2 s13 = cadd(v[1], v[3]), d13 = muli(csub(v[1], v[3]), sign);
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else {
        // odd R: pair r with R - r
        double2 sp[R / 2], dm[R / 2];
#pragma unroll
        for (int r = 1; r <= R / 2; ++r) {
            sp[r - 1] = cadd(v[r], v[R - r]);
            dm[r - 1] = csub(v[r], v[R - r]);
        }
        double2 y[R];
        double2 y0 = v[0];
#pragma unroll
        for (int r = 0; r < R / 2; ++r) y0 = cadd(y0, sp[r]);
        y[0] = y0;
#pragma unroll
        for (int k = 1; k < R; ++k) {
            double ar = v[0].x, ai = v[0].y, br = 0.0, bi = 0.0;
#pragma unroll
            for (int r = 1; r <= R / 2; ++r) {
                const double c = Roots<R>::c[(r * k) % R];
                const double s = Roots<R>::s[(r * k) % R];
                ar = fma(sp[r - 1].x, c, ar);
                ai = fma(sp[r - 1].y, c, ai);
                br = fma(dm[r - 1].x, s, br);
                bi = fma(dm[r - 1].y, s, bi);
            }
            // + sign * i * (b)
            y[k] = sign > 0 ? make_double2(ar - bi, ai + br) : make_double2(ar + bi, ai - br);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = y[k];
    }
}

// One Stockham pass of radix R over n points in LDS.  tw[idx * tws] is
// e^{+2 pi i idx / n}.
template <int R, int NT>
__device__ void fft_pass(double2 *buf, int n, int Ns, int sign, const double2 *__restrict__ tw,
                         int tws)
{
    constexpr int MAXQ = (kMaxFft / R + NT - 1) / NT;
    const int nb = n / R;
    const int tstep0 = n / (Ns * R);
    double2 v[MAXQ][R];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = threadIdx.x + q * NT;
        if (j < nb) {
            const int k = j % Ns;
            const int ts = tstep0 * k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = buf[j + r * nb];
                if (r > 0 && ts != 0) {
                    double2 w = tw[(long long)(r * ts) * tws];
                    if (sign < 0) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[q][r] = x;
            }
            small_dft<R>(v[q], sign);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = threadIdx.x + q * NT;
        if (j < nb) {
            const int k = j % Ns;
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

// In-place DFT of 7-smooth length n <= kMaxFft:
// buf_k <- sum_j buf_j e^{sign 2 pi i j k / n}.
template <int NT>
__device__ void fft_lds(double2 *buf, int n, int sign, const double2 *__restrict__ tw, int tws)
{
    int Ns = 1, rem = n;
    while (rem > 1) {
        if (rem % 4 == 0) {
            fft_pass<4, NT>(buf, n, Ns, sign, tw, tws); Ns *= 4; rem /= 4;
        } else if (rem % 2 == 0) {
            fft_pass<2, NT>(buf, n, Ns, sign, tw, tws); Ns *= 2; rem /= 2;
        } else if (rem % 3 == 0) {
            fft_pass<3, NT>(buf, n, Ns, sign, tw, tws); Ns *= 3; rem /= 3;
        } else if (rem % 5 == 0) {
            fft_pass<5, NT>(buf, n, Ns, sign, tw, tws); Ns *= 5; rem /= 5;
        } else {
            fft_pass<7, NT>(buf, n, Ns, sign, tw, tws); Ns *= 7; rem /= 7;
        }
    }
}

// In-place DFT of any length len (<= kMaxFft / 2) by Bluestein's algorithm:
// e^{i 2 pi jk/len} = c_j c_k conj(c_{j-k}), c_k = e^{i pi k^2 / len}.
// tch[q] = e^{2 pi i q / (2 len)}, twb = e^{2 pi i k / nb}, bq = DFT^-(conj c, wrapped) / nb.
// A sign -1 transform is conj(DFT^+(conj x)).
template <int NT>
__device__ void bluestein_lds(double2 *buf, int len, int nb, int sign,
                              const double2 *__restrict__ tch, const double2 *__restrict__ twb,
                              const double2 *__restrict__ bq)
{
    const int two_len = 2 * len;
    for (int k = threadIdx.x; k < nb; k += NT) {
        if (k < len) {
            double2 x = buf[k];
            if (sign < 0) x.y = -x.y;
            const int q = (int)(((long long)k * k) % two_len);
            buf[k] = cmul(x, tch[q]);
        } else {
            buf[k] = make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    fft_lds<NT>(buf, nb, -1, twb, 1);
    for (int k = threadIdx.x; k < nb; k += NT) buf[k] = cmul(buf[k], bq[k]);
    __syncthreads();
    fft_lds<NT>(buf, nb, +1, twb, 1);
    for (int j = threadIdx.x; j < len; j += NT) {
        const int q = (int)(((long long)j * j) % two_len);
        double2 z = cmul(buf[j], tch[q]);
        if (sign < 0) z.y = -z.y;
        buf[j] = z;
    }
    __syncthreads();
}

template <int NT>
__device__ inline void ring_dft(double2 *buf, const RingDesc &d, int sign,
                                const double2 *__restrict__ pool)
{
    if (d.nb == 0) {
        fft_lds<NT>(buf, d.clen, sign, pool + d.tw, (d.n % 2 == 0) ? 2 : 1);
    } else {
        bluestein_lds<NT>(buf, d.clen, d.nb, sign, pool + d.tch, pool + d.twb, pool + d.bq);
    }
}

__device__ inline double2 phase_mode(double2 dl, int m, double phi0, int sign)
{
    if (m == 0) return make_double2(dl.x, 0.0);
    double sn, cs;
    sincos((double)m * phi0, &sn, &cs);
    return cmul(dl, make_double2(cs, sign > 0 ? sn : -sn));
}

__global__ __launch_bounds__(kRingThreads) void k_ring_synth(
    const RingDesc *__restrict__ rings, const double2 *__restrict__ pool,
    const double2 *__restrict__ delta, const int *__restrict__ minv, int mmax, int nm,
    int nrings, double *__restrict__ map, long long npix)
{
    extern __shared__ double2 buf[];
    const int r = blockIdx.x;
    const int b = blockIdx.y;
    const RingDesc d = rings[r];
    const double2 *drow = delta + ((long long)b * nrings + r) * nm;
    const long long pix0 = (long long)b * npix + d.start;
    double *out = map + pix0;
    const int n = d.n;
    const bool even = (n % 2) == 0;
    const int h = n / 2;
    const int kmax = even ? h : n - 1;
    // fold: F_k, k = 0..kmax
    for (int k = threadIdx.x; k <= kmax; k += kRingThreads) {
        double fr = 0.0, fi = 0.0;
        for (int m = k; m <= mmax; m += n) {
            const int i = minv[m];
            if (i >= 0) {
                const double2 D = phase_mode(drow[i], m, d.phi0, +1);
                fr += D.x; fi += D.y;
            }
        }
        for (int m = n - k; m <= mmax; m += n) {
            const int i = minv[m];
            if (i >= 0) {
                const double2 D = phase_mode(drow[i], m, d.phi0, +1);
                fr += D.x; fi -= D.y;
            }
        }
        buf[k] = make_double2(fr, fi);
    }
    __syncthreads();
    if (even) {
        const double2 *tw = pool + d.tw;
        for (int k = threadIdx.x; k <= h / 2; k += kRingThreads) {
            const int k2 = h - k;
            const double2 Fk = buf[k], Fk2 = buf[k2];
            const double2 e1 = cadd(Fk, conjd(Fk2)), o1 = csub(Fk, conjd(Fk2));
            const double2 Zk = cadd(e1, muli(cmul(tw[k], o1), +1));
            const double2 e2 = cadd(Fk2, conjd(Fk)), o2 = csub(Fk2, conjd(Fk));
            const double2 Zk2 = cadd(e2, muli(cmul(tw[k2], o2), +1));
            buf[k] = Zk;
            if (k2 != k) buf[k2] = Zk2;
        }
        __syncthreads();
        ring_dft<kRingThreads>(buf, d, +1, pool);
        if ((pix0 & 1) == 0) {
            double2 *o2 = reinterpret_cast<double2 *>(out);
            for (int j = threadIdx.x; j < h; j += kRingThreads) o2[j] = buf[j];
        } else {
            for (int j = threadIdx.x; j < h; j += kRingThreads) {
                const double2 z = buf[j];
                out[2 * j] = z.x;
                out[2 * j + 1] = z.y;
            }
        }
    } else {
        ring_dft<kRingThreads>(buf, d, +1, pool);
        for (int j = threadIdx.x; j < n; j += kRingThreads) out[j] = buf[j].x;
    }
}

__global__ __launch_bounds__(kRingThreads) void k_ring_anal(
    const RingDesc *__restrict__ rings, const double2 *__restrict__ pool,
    const double *__restrict__ map, long long npix, const int *__restrict__ mval, int nm,
    int nrings, double2 *__restrict__ dt)
{
    extern __shared__ double2 buf[];
    const int r = blockIdx.x;
    const int b = blockIdx.y;
    const RingDesc d = rings[r];
    const long long pix0 = (long long)b * npix + d.start;
    const double *in = map + pix0;
    const int n = d.n;
    const bool even = (n % 2) == 0;
    const int h = n / 2;
    if (even) {
        if ((pix0 & 1) == 0) {
            const double2 *i2 = reinterpret_cast<const double2 *>(in);
            for (int j = threadIdx.x; j < h; j += kRingThreads) buf[j] = i2[j];
        } else {
            for (int j = threadIdx.x; j < h; j += kRingThreads)
                buf[j] = make_double2(in[2 * j], in[2 * j + 1]);
        }
        __syncthreads();
        ring_dft<kRingThreads>(buf, d, -1, pool);
        const double2 *tw = pool + d.tw;
        for (int k = threadIdx.x; k <= h / 2; k += kRingThreads) {
            const int k2 = h - k;
            const double2 Zk = buf[k];
            const double2 Zk2 = buf[k2 == h ? 0 : k2];
            // G_k = (Z_k + conj Z_{h-k})/2 - (i/2) e^{-2 pi i k/n} (Z_k - conj Z_{h-k})
            const double2 a1 = cadd(Zk, conjd(Zk2)), b1 = csub(Zk, conjd(Zk2));
            const double2 G1 = csub(a1, muli(cmul(conjd(tw[k]), b1), +1));
            const double2 a2 = cadd(Zk2, conjd(Zk)), b2 = csub(Zk2, conjd(Zk));
            const double2 G2 = csub(a2, muli(cmul(conjd(tw[k2]), b2), +1));
            buf[k] = make_double2(0.5 * G1.x, 0.5 * G1.y);
            if (k2 != k) buf[k2] = make_double2(0.5 * G2.x, 0.5 * G2.y);
        }
        __syncthreads();
    } else {
        for (int j = threadIdx.x; j < n; j += kRingThreads) buf[j] = make_double2(in[j], 0.0);
        __syncthreads();
        ring_dft<kRingThreads>(buf, d, -1, pool);
    }
    const int kmax = even ? h : n - 1;
    double2 *orow = dt + ((long long)b * nrings + r) * nm;
    for (int i = threadIdx.x; i < nm; i += kRingThreads) {
        const int m = mval[i];
        const int kk = m % n;
        const double2 G = (kk <= kmax) ? buf[kk] : conjd(buf[n - kk]);
        double2 v;
        if (m == 0) {
            v = make_double2(G.x, 0.0);
        } else {
            double sn, cs;
            sincos((double)m * d.phi0, &sn, &cs);
            v = cmul(G, make_double2(cs, -sn));
            v.x *= 2.0; v.y *= 2.0;
        }
        orow[i] = v;
    }
}

// Spectrum of the Bluestein kernel b_k = conj(c_k) (wrapped to negative k),
// scaled by 1 / nb, one workgroup per listed ring.
__global__ __launch_bounds__(kRingThreads) void k_bluestein_prep(
    const RingDesc *__restrict__ rings, const int *__restrict__ ids, double2 *pool)
{
    extern __shared__ double2 buf[];
    const RingDesc d = rings[ids[blockIdx.x]];
    const int len = d.clen, nb = d.nb, two_len = 2 * len;
    const double2 *tch = pool + d.tch;
    for (int k = threadIdx.x; k < nb; k += kRingThreads) {
        int m = -1;
        if (k < len) m = k;
        else if (k > nb - len) m = nb - k;
        double2 v = make_double2(0.0, 0.0);
        if (m >= 0) v = conjd(tch[(int)(((long long)m * m) % two_len)]);
        buf[k] = v;
    }
    __syncthreads();
    fft_lds<kRingThreads>(buf, nb, -1, pool + d.twb, 1);
    const double inv = 1.0 / (double)nb;
    for (int k = threadIdx.x; k < nb; k += kRingThreads)
        pool[d.bq + k] = make_double2(buf[k].x * inv, buf[k].y * inv);
}

hipError_t set_lds(const void *fn, size_t bytes)
{
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

hipError_t launch_ring_synth(const sht_plan_s *p, const double2 *delta, double *map,
                             hipStream_t st)
{
    const size_t lds = (size_t)p->lds_complex * sizeof(double2);
    hipError_t e = set_lds((const void *)k_ring_synth, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ring_synth, dim3((unsigned)p->nrings, (unsigned)p->nmaps),
                       dim3(kRingThreads), lds, st, p->d_rings, p->d_pool, delta, p->d_minv,
                       p->mmax, p->nm, p->nrings, map, p->npix);
    return hipGetLastError();
}

hipError_t launch_ring_anal(const sht_plan_s *p, const double *map, double2 *dt, hipStream_t st)
{
    const size_t lds = (size_t)p->lds_complex * sizeof(double2);
    hipError_t e = set_lds((const void *)k_ring_anal, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ring_anal, dim3((unsigned)p->nrings, (unsigned)p->nmaps),
                       dim3(kRingThreads), lds, st, p->d_rings, p->d_pool, map, p->npix,
                       p->d_mval, p->nm, p->nrings, dt);
    return hipGetLastError();
}

hipError_t launch_bluestein_prep(const sht_plan_s *p, const int *ring_ids, int nids,
                                 hipStream_t st)
{
    if (nids <= 0) return hipSuccess;
    const size_t lds = (size_t)p->lds_complex * sizeof(double2);
    hipError_t e = set_lds((const void *)k_bluestein_prep, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bluestein_prep, dim3((unsigned)nids), dim3(kRingThreads), lds, st,
                       p->d_rings, ring_ids, p->d_pool);
    return hipGetLastError();
}

}  // namespace sht
