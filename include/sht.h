/*
 * sht.h -- C ABI of the MI355X (gfx950) inverse spherical harmonic transform.
 *
 * The transform synthesises real maps on iso-latitude rings from harmonic
 * coefficients (Hupca, Falcou, Grigori, Stompor, "Spherical harmonic
 * transform with GPUs", INRIA RR-7409):
 *
 *   s(theta, phi) = sum_{l=0}^{lmax} sum_{m=-l}^{l} a_lm Y_lm(theta, phi)     Eq. (alm2mapDef)
 *
 * computed in two stages: the Legendre stage
 *
 *   Delta_m(theta_r) = sum_{l=m}^{lmax} a_lm P_lm(cos theta_r)                Eq. (DeltaDef)
 *
 * (the two-point recurrence of Eq. (assLegRec) run on the fly with
 * real-time rescaling, Sec. 2.2.2, Algorithm 2) and, per ring, the Fourier
 * sum s(theta_r, phi) = sum_m e^{i m phi} Delta_m(theta_r) (Eq. Delta2map)
 * with modes wrapped modulo the ring's pixel count (Sec. 2.2.2).
 *
 * Conventions
 *  - Orthonormal P_lm without Condon-Shortley phase (mu_m > 0, Eq. pmm).
 *  - Only m >= 0 is stored; a_{l,-m} = (-1)^m conj(a_lm) (Sec. 2.1).  The
 *    imaginary part of a_l0 is ignored on input and written as 0 on output.
 *  - Coefficients: complex128 interleaved (re, im), m-major packed: for the
 *    i-th m of the m-set, l = m..lmax are contiguous, starting at
 *    off_i = sum_{j<i} (lmax - m_j + 1).  nalm = off_nm.
 *  - Maps: float64, RING order; pixel j of ring r sits at ringstart[r] + j and
 *    at azimuth phi0[r] + 2 pi j / nphi[r].
 *  - Batches: nmaps maps share one geometry; map b's coefficients start at
 *    alm + 2 * b * nalm (doubles), its pixels at map + b * npix.
 *
 * Ownership and streams
 *  - The plan owns its own device tables, allocated on the device that is
 *    current when sht_plan is called, and one auxiliary stream with two
 *    events: for large plans the synthesis forks part of its Fourier work
 *    onto that stream and joins it back into `stream` before returning, so
 *    every call stays ordered on `stream`.  Every device pointer passed to the
 *    other calls (coefficients, maps, workspace) is owned by the caller and
 *    must be on that device, 16-byte aligned.
 *  - sht_alm2map* and sht_alm2map_adjoint* only enqueue kernels on `stream`
 *    (a hipStream_t; NULL is the null stream).  They never allocate memory
 *    and never synchronise, so they can be captured into a HIP graph.
 *  - A plan is immutable after creation, apart from its launch shape
 *    (sht_plan_set_config, sht_plan_autotune), which changes no result.
 *    Calls on different streams are safe if they use distinct workspaces
 *    (host threads take turns through the fork and join).  While a call is
 *    being captured into a HIP graph, the plan's auxiliary stream is part of
 *    the capture: do not use the same plan from another thread meanwhile.
 *
 * Errors: every call returns an sht_status; nothing throws across the ABI.
 * Argument errors are detected on the host before anything is enqueued.
 * A device-side failure shows up as SHT_ERR_HIP on the call that observes it.
 */
#ifndef SHT_H
#define SHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sht_plan_s *sht_plan_t;

typedef enum {
    SHT_OK = 0,
    SHT_ERR_INVALID_ARG = -1, /* a descriptor field or pointer is invalid       */
    SHT_ERR_OOM = -2,         /* host or device allocation failed (plan only)   */
    SHT_ERR_HIP = -3,         /* a HIP runtime call failed                      */
    SHT_ERR_UNSUPPORTED = -4, /* valid request this build does not implement    */
    SHT_ERR_BAD_HANDLE = -5,  /* NULL, destroyed or foreign plan handle         */
    SHT_ERR_WORKSPACE = -6    /* workspace NULL or smaller than required        */
} sht_status;

typedef enum {
    SHT_FP64 = 0,      /* FP64 recurrence and FP64 accumulation                          */
    SHT_FP32_MFMA = 1, /* FP64 recurrence; the l-sum of each batch of up to 16 maps runs on
                          the matrix cores with FP32 inputs (P_lm and prescaled a_lm
                          rounded to FP32) and two-level FP32 accumulation.  The ring
                          Fourier step and the adjoint stay FP64.  Relative L2 error of
                          a map against FP64 about 1e-7.                                  */
    SHT_BF16X3_MFMA = 2, /* as SHT_FP32_MFMA, with every FP32 operand split into three BF16
                           parts (8+8+8 bits) and six BF16 matrix-core products per
                           tile; same accuracy class, higher matrix-core rate.          */
    SHT_F16X2_MFMA = 3  /* as SHT_FP32_MFMA, with every FP32 operand split into two FP16
                           parts (11+11 bits) and three FP16 matrix-core products per
                           tile (the dropped low x low term is below 2^-21 relative);
                           both operands are scaled by powers of two into FP16's range
                           (the coefficients per map and 128-row block of l), so the
                           accuracy class is that of the FP32 form.  Fewest matrix-core
                           and vector instructions of the mixed forms.
                           All mixed forms hold a_lm P_lm sums in FP32: coefficients
                           must stay within FP32 range (|a_lm| below about 1e30).    */
} sht_precision;

#define SHT_MAX_LMAX 16383
/* largest ring the per-ring Fourier kernels hold in LDS.  With h = nphi/2:
 * even nphi: h <= 8192, and h even, or h a product of 3, 5, 7, or h <= 4096;
 * odd nphi: nphi <= 8192, and nphi a product of 3, 5, 7, or nphi <= 4096.
 * sht_plan returns SHT_ERR_UNSUPPORTED for any other ring (16382 and 8191,
 * say).  Every HEALPix ring up to nside 4096 is supported. */
#define SHT_MAX_NPHI 16384

/* Geometry and problem description for sht_plan.  All pointers are host
 * pointers; sht_plan copies what it needs, so they may be freed afterwards. */
typedef struct {
    int32_t lmax;             /* band limit, 0 <= lmax <= SHT_MAX_LMAX               */
    int32_t nm;               /* number of m in the m-set, 1 <= nm <= lmax + 1      */
    const int32_t *mval;      /* [nm] strictly increasing, 0 <= m <= lmax;
                                 NULL means m = 0, 1, ..., nm - 1                   */
    int32_t nrings;           /* >= 1                                               */
    const double *cth;        /* [nrings] cos(theta_r), in [-1, 1]                  */
    const double *sth;        /* [nrings] sin(theta_r) >= 0, cth^2 + sth^2 = 1 (1e-12) */
    const double *phi0;       /* [nrings] azimuth of the first pixel of ring r      */
    const int64_t *nphi;      /* [nrings] pixels in ring r, 1..SHT_MAX_NPHI          */
    const int64_t *ringstart; /* [nrings] first pixel of ring r; NULL = packed in
                                 ring order.  Rings may not overlap.                */
    int32_t nmaps;            /* maps per call, >= 1                                */
    int32_t precision;        /* sht_precision                                      */
    uint32_t flags;           /* SHT_FLAG_*                                         */
    int64_t npix;             /* pixels per map in the caller's map buffers (the
                                 stride between maps); 0 = max(ringstart + nphi).
                                 Larger values let a plan over part of the rings
                                 (a latitude band, one shard of ring pairs) write
                                 into a full-sky map.  Smaller: SHT_ERR_INVALID_ARG */
} sht_geometry_desc;

/* Treat every ring on its own even when its mirror ring (cth negated
 * bitwise, sth equal) is present.  Results are the same up to rounding. */
#define SHT_FLAG_NO_PAIRING 1u

typedef struct {
    int64_t nalm;             /* complex coefficients per map                       */
    int64_t npix;             /* pixels per map (desc.npix, else max of ringstart + nphi) */
    int32_t nrings;
    int32_t npairs;           /* recurrence units: mirror pairs + unpaired rings    */
    int32_t nm;
    int32_t lmax;
    int32_t mmax;
    int32_t nmaps;
    size_t workspace_bytes;   /* for sht_alm2map / sht_alm2map_adjoint              */
    size_t delta_bytes;       /* nmaps * nrings * nm * 16                          */
    size_t table_bytes;       /* device memory held by the plan                     */
    size_t forward_workspace_bytes; /* enough for sht_alm2map, sht_alm2map_events and
                                       sht_plan_autotune (no adjoint partial sums)  */
} sht_plan_info;

/* Build a plan: validate the descriptor, pair mirror rings, precompute the
 * recurrence tables (mu_m of Eq. pmm, beta_lm of Eq. betaDef folded into the
 * normalised form described in the library source) and the per-ring Fourier
 * tables, and upload them to the current device.
 * Returns SHT_ERR_INVALID_ARG for a bad descriptor, SHT_ERR_UNSUPPORTED for a
 * ring longer than the kernels support, SHT_ERR_OOM / SHT_ERR_HIP on
 * allocation failure.  *out is NULL on failure. */
sht_status sht_plan(sht_plan_t *out, const sht_geometry_desc *desc);

/* Release the plan's device tables.  The handle is invalid afterwards;
 * passing it again returns SHT_ERR_BAD_HANDLE (best effort).  Work still
 * queued that uses the plan must have completed. */
sht_status sht_plan_destroy(sht_plan_t plan);

sht_status sht_plan_get_info(sht_plan_t plan, sht_plan_info *info);

/* Bytes of device workspace every call of the plan can use (the largest
 * need: sht_alm2map_adjoint and sht_map2alm).  Synthesis alone needs only
 * sht_plan_info.forward_workspace_bytes. */
sht_status sht_plan_workspace_size(sht_plan_t plan, size_t *bytes);

/* Launch shape of an FP64 plan's forward Legendre kernel: chains = ring
 * pairs per lane (1, 2 or 4).  The best shape depends on the input size
 * (Sec. 5, which proposes tuning per size): sht_plan picks a default from a
 * table measured over sizes on MI355X.  Results do not depend on it (every
 * ring pair runs the same arithmetic); only the time does.
 * sht_plan_set_config: SHT_ERR_INVALID_ARG for other values,
 * SHT_ERR_UNSUPPORTED on mixed-precision plans (their kernels have no such
 * choice) or when the launch would exceed the grid limit.  Do not change the
 * shape while another host thread enqueues work on the same plan. */
sht_status sht_plan_get_config(sht_plan_t plan, int32_t *chains);
sht_status sht_plan_set_config(sht_plan_t plan, int32_t chains);

/* Autotuner of the launch shape above: times sht_alm2map at every chain
 * count on the given buffers (alm read, map overwritten, ws as for
 * sht_alm2map; synchronises `stream`) and keeps the fastest.  If cache_path
 * is not NULL, a line "<plan signature> <chains> <ms>" is looked up first
 * (no timing if found) and appended after tuning.  On mixed-precision plans
 * it does nothing and returns SHT_OK. */
sht_status sht_plan_autotune(sht_plan_t plan, const double *alm, double *map, void *ws,
                             size_t ws_bytes, const char *cache_path, void *stream);

/* alm2map (Eq. alm2mapDef): alm device complex128 [nmaps][nalm] (read),
 * map device float64 [nmaps][npix] (written at every ring pixel; pixels not
 * covered by any ring are left untouched), ws device scratch of at least
 * sht_plan_info.forward_workspace_bytes (contents on entry ignored). */
sht_status sht_alm2map(sht_plan_t plan, const double *alm, double *map,
                       void *ws, size_t ws_bytes, void *stream);

/* map2alm (Eq. map2almDef, Sec. 2.1): the quadrature-weighted analysis
 *     a_lm = sum_r w_r sum_j s_rj conj(Y_lm(theta_r, phi0_r + 2 pi j / nphi_r)),
 * i.e. D * adjoint(w s) with D = 1 for m = 0 and 1/2 for m > 0 (the adjoint
 * counts m and -m together).  On Gauss-Legendre rings with w_r the node
 * weight times 2 pi / nphi_r, nrings > lmax and nphi_r > 2 lmax it inverts
 * sht_alm2map exactly; on other grids it is the usual approximate analysis,
 * refined by niter Jacobi steps a <- a + map2alm(s - alm2map(a)).
 *   map          device float64 [nmaps][npix] (read; only ring pixels are used)
 *   ring_weight  device float64 [nrings]: weight of one pixel of ring r
 *   alm          device complex128 [nmaps][nalm] (written; Im of m = 0 is 0)
 *   niter        0 .. SHT_MAX_MAP2ALM_ITER refinement steps
 *   tmp_map      device float64 [nmaps][npix] scratch, required when niter > 0
 *                (may be NULL otherwise); its contents are overwritten
 *   ws           workspace of at least sht_plan_workspace_size bytes
 * The refinement's alm2map runs in the plan's precision; the analysis is
 * FP64.  Errors: SHT_ERR_INVALID_ARG for NULL pointers, niter out of range
 * or a missing tmp_map; SHT_ERR_WORKSPACE for a short workspace. */
#define SHT_MAX_MAP2ALM_ITER 100
sht_status sht_map2alm(sht_plan_t plan, const double *map, const double *ring_weight,
                       double *alm, int32_t niter, double *tmp_map, void *ws, size_t ws_bytes,
                       void *stream);

/* sht_alm2map that also records caller-created HIP events (hipEvent_t) on
 * `stream` at its stage boundaries, for stage timing:
 * events[0] before the coefficient prescale, events[1] before the Legendre
 * kernel, events[2] before the ring synthesis, events[3] after it.
 * events must hold 4 valid events; otherwise as sht_alm2map. */
sht_status sht_alm2map_events(sht_plan_t plan, const double *alm, double *map,
                              void *ws, size_t ws_bytes, void *stream,
                              void *const *events);

/* Adjoint of sht_alm2map with respect to the real inner products
 * <map, map'> = sum_p map_p map'_p and <a, a'> = sum Re(conj(a) a') over the
 * stored coefficients: alm_lm = c_m sum_p map_p P_lm(cos theta_p) e^{-i m phi_p},
 * c_0 = 1, c_{m>0} = 2 -- the gradient of a real loss of the map with respect
 * to (Re a_lm, Im a_lm), packed as complex.  map device float64 [nmaps][npix]
 * (read), alm device complex128 [nmaps][nalm] (written; Im of m = 0 is 0). */
sht_status sht_alm2map_adjoint(sht_plan_t plan, const double *map, double *alm,
                               void *ws, size_t ws_bytes, void *stream);

/* alm2map for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same transform and kernels as sht_alm2map, with the workspace taken from a
 * device array of SHT_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device until the process ends (its address is looked up on the first call
 * on a device).  Calls nothing that allocates.  Returns SHT_ERR_WORKSPACE when
 * sht_plan_info.forward_workspace_bytes exceeds SHT_NOALLOC_SCRATCH_BYTES.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (different streams, or host threads) race and must be
 * serialised by the caller.  The array's contents on entry are ignored (no
 * part of it needs to start at zero). */
#define SHT_NOALLOC_SCRATCH_BYTES (64u << 20)
sht_status sht_alm2map_noalloc(sht_plan_t plan, const double *alm, double *map, void *stream);

/* The two stages on their own (same kernels as sht_alm2map).
 * delta: device complex128 [nmaps][nm][nrings], Delta_m(theta_r) of
 * Eq. (DeltaDef) for the i-th m of the set at [b][i][r] (rings contiguous:
 * the Legendre stage writes whole runs of rings per m).
 * The mixed forms keep Delta as complex64 inside sht_alm2map (the precision
 * of their FP32 sums), laid out [m][ring][map] (maps contiguous, read by the
 * ring stage for all maps of a ring together), and their ring FFTs on the
 * fast paths run in complex64 (the alias fold adds in FP64); sht_alm2delta
 * of a mixed plan writes that complex64 Delta into the workspace and widens
 * it exactly into `delta` in the layout above, so it needs sht_plan_info.forward_workspace_bytes (FP64 plans: the
 * coefficient part only).  sht_delta2map always reads complex128 and runs
 * the Fourier stage in FP64, on any plan. */
sht_status sht_alm2delta(sht_plan_t plan, const double *alm, double *delta,
                         void *ws, size_t ws_bytes, void *stream);
sht_status sht_delta2map(sht_plan_t plan, const double *delta, double *map, void *stream);

/* Adjoint stages: map -> Delta~ (ring analysis) and Delta~ -> alm; Delta~ has
 * the layout of delta above. */
sht_status sht_map2delta_adjoint(sht_plan_t plan, const double *map, double *delta,
                                 void *stream);
sht_status sht_delta2alm_adjoint(sht_plan_t plan, const double *delta, double *alm,
                                 void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Batches of maps with different l_max and geometry (not in the paper; for
 * callers that transform many small and large maps together).  The batch
 * refers to the device tables of single-map FP64 plans, which must outlive it.
 * The Legendre stage of all maps runs as one persistent launch that takes
 * (map, m-pair, ring-pair block) tiles, longest first, from an atomic
 * counter; the counter only distributes work, so results are identical to
 * the single-plan transforms and independent of the launch shape.  The
 * per-ring Fourier step runs as one launch per ring size class.
 *
 * Streams: the work counter lives in the caller's workspace (its first 256
 * bytes), so transforms of one batch on different streams are safe when
 * they use distinct workspaces, as for plans.  A captured graph keeps the
 * workspace it was captured with: replays of one graph must not overlap.
 * ------------------------------------------------------------------------- */
typedef struct sht_batch_s *sht_batch_t;

/* plans: host array of n plan handles, each with nmaps = 1 and SHT_FP64, all
 * on the current device.  Uploads the work lists (device memory owned by
 * the batch).  SHT_ERR_UNSUPPORTED for a batched or mixed-precision plan. */
sht_status sht_plan_batch(sht_batch_t *out, const sht_plan_t *plans, int32_t n);
sht_status sht_batch_destroy(sht_batch_t batch);
sht_status sht_batch_workspace_size(sht_batch_t batch, size_t *bytes);

/* alms: DEVICE array of n device pointers, alms[i] = complex128 [nalm_i] of
 * map i; maps: DEVICE array of n device pointers, maps[i] = float64 [npix_i].
 * ws: device workspace of sht_batch_workspace_size bytes.  Enqueues on
 * `stream` only; no allocation, no synchronisation. */
sht_status sht_alm2map_batch(sht_batch_t batch, const double *const *alms,
                             double *const *maps, void *ws, size_t ws_bytes, void *stream);

/* Launch shape of the batch: chains (ring pairs per lane: 1, 2 or 4) and
 * persistent waves per compute unit (1..32).  The default comes from a table
 * measured over sizes (Sec. 6.1: the best shape depends on the size), keyed
 * by work tiles of 128 ring pairs per compute unit; every shape gives the
 * same results. */
sht_status sht_batch_get_config(sht_batch_t batch, int32_t *chains, int32_t *waves_per_cu);
sht_status sht_batch_set_config(sht_batch_t batch, int32_t chains, int32_t waves_per_cu);

/* Autotuner: times every (chains in {1, 2, 4}, waves per CU in {4, 8, 16, 32})
 * candidate on the given
 * buffers (synchronising `stream`) and keeps the fastest.  If cache_path is
 * not NULL, a line "<batch signature> <chains> <waves_per_cu> <ms>" is looked
 * up first (no timing if found) and appended after tuning.  The outputs are
 * overwritten. */
sht_status sht_batch_autotune(sht_batch_t batch, const double *const *alms,
                              double *const *maps, void *ws, size_t ws_bytes,
                              const char *cache_path, void *stream);

/* Capture one sht_alm2map_batch on `stream` (not the null stream) into a HIP
 * graph held by the batch; sht_batch_graph_launch replays it on any stream
 * with the captured buffers.  Re-capturing replaces the graph. */
sht_status sht_batch_graph_capture(sht_batch_t batch, const double *const *alms,
                                   double *const *maps, void *ws, size_t ws_bytes,
                                   void *stream);
sht_status sht_batch_graph_launch(sht_batch_t batch, void *stream);

/* Static description of a status code. */
const char *sht_status_string(sht_status status);

/* Library version, "major.minor.patch". */
const char *sht_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SHT_H */
