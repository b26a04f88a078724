// Batches of plans with different l_max / geometry: one persistent Legendre
// launch and one Fourier launch per ring size class for all maps, an
// autotuner for the launch shape with an on-disk cache, and HIP graph
// capture of the whole sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "sht_internal.h"

using sht::BatchClass;
using sht::BatchMap;
using sht::BatchTile;

namespace {

constexpr uint64_t kBatchMagic = 0x53485442'41544348ull;  // "SHTBATCH"
const int kChainChoices[] = {1, 2, 4};
const int kWaveChoices[] = {4, 8, 16, 32};  // persistent waves per CU

// Default launch shape of the batch by size (the best shape depends on the
// input size, Sec. 6.1; Sec. 5 proposes tuning per size).  Key: work tiles of
// 128 ring pairs (two chains per lane) per compute unit.  Measured on MI355X
// (256 compute units) over batches of uniform l_max 128..2048 (4 to 64 maps)
// and the uneven 16- and 64-map draws, every shape of {1, 2, 4} chains x
// {4, 8, 16, 32} waves per CU: up to 4 tiles per CU two chains and 4 waves
// are fastest, up to 16 four chains and 8 waves, above that four chains and
// 16 waves (the residency limit of the four-chain kernel's 128 VGPRs; two
// chains at 32 waves come within 1% at the largest sizes).  The former fixed
// choice (2, 8) was up to 2.4x slower above 100 tiles per CU.
struct BatchShapeRule {
    double max_tiles_per_cu;
    int chains, waves_per_cu;
};
constexpr BatchShapeRule kBatchShapeTable[] = {
    {4.0, 2, 4},
    {16.0, 4, 8},
    {1e300, 4, 16},
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// The workspace starts with the persistent launch's work counter (reset by
// a kernel at the start of every transform), so that transforms of one
// batch with distinct workspaces share no device state.
constexpr size_t kCounterBytes = 256;

}  // namespace

struct sht_batch_s {
    uint64_t magic;
    int device;
    int n;
    int num_cus;
    std::vector<sht_plan_t> plans;  // not owned; must outlive the batch
    BatchMap *d_maps;
    BatchTile *d_tiles[3];           // work lists for 1, 2, 4 chains per lane
    int ntiles[3];
    BatchClass cls[sht::kNumSynthClasses];
    long long max_nalm;
    size_t ws_bytes;
    int chains;                      // launch shape in use
    int waves_per_cu;
    std::string signature;
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
};

namespace {

int chain_index(int c) { return c == 1 ? 0 : (c == 2 ? 1 : 2); }

sht_status check_batch(sht_batch_t b)
{
    if (!b || b->magic != kBatchMagic) return SHT_ERR_BAD_HANDLE;
    sht::clear_stale_error();
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SHT_ERR_HIP;
    if (dev != b->device) return SHT_ERR_INVALID_ARG;
    return SHT_OK;
}

void free_batch(sht_batch_s *b)
{
    if (b->d_maps) (void)hipFree(b->d_maps);
    for (int i = 0; i < 3; ++i)
        if (b->d_tiles[i]) (void)hipFree(b->d_tiles[i]);
    for (int c = 0; c < sht::kNumSynthClasses; ++c)
        if (b->cls[c].d_items) (void)hipFree(b->cls[c].d_items);
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
}

sht_status enqueue(sht_batch_t b, const double *const *alms, double *const *maps, void *ws,
                   hipStream_t st)
{
    const int ci = chain_index(b->chains);
    hipError_t e = sht::launch_batch_legendre(
        b->d_maps, b->n, b->max_nalm, b->d_tiles[ci], b->ntiles[ci], b->chains,
        b->waves_per_cu * b->num_cus, alms, ws, static_cast<int *>(ws), st);
    if (e == hipSuccess) e = sht::launch_ring_synth_batch(b->cls, b->d_maps, maps, ws, st);
    return e == hipSuccess ? SHT_OK : SHT_ERR_HIP;
}

}  // namespace

extern "C" {

sht_status sht_plan_batch(sht_batch_t *out, const sht_plan_t *plans, int32_t n)
{
    if (!out) return SHT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!plans || n < 1) return SHT_ERR_INVALID_ARG;
    sht::clear_stale_error();
    int dev = -1;
    for (int i = 0; i < n; ++i) {
        const sht_plan_s *p = plans[i];
        if (!p || p->magic != sht::kPlanMagic) return SHT_ERR_BAD_HANDLE;
        if (p->nmaps != 1 || p->precision != SHT_FP64) return SHT_ERR_UNSUPPORTED;
        if (i == 0) dev = p->device;
        if (p->device != dev) return SHT_ERR_INVALID_ARG;
    }
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return SHT_ERR_HIP;
    if (cur != dev) return SHT_ERR_INVALID_ARG;

    sht_batch_s *b = new (std::nothrow) sht_batch_s();
    if (!b) return SHT_ERR_OOM;
    b->magic = 0;
    b->device = dev;
    b->n = n;
    b->plans.assign(plans, plans + n);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) { delete b; return SHT_ERR_HIP; }
    b->num_cus = prop.multiProcessorCount;

    // per-map descriptors and workspace layout (after the work counter)
    std::vector<BatchMap> maps(n);
    size_t off = kCounterBytes;
    std::ostringstream sig;
    sig << prop.gcnArchName << "|n=" << n;
    b->max_nalm = 0;
    for (int i = 0; i < n; ++i) {
        const sht_plan_s *p = plans[i];
        BatchMap &m = maps[i];
        std::memset(&m, 0, sizeof m);
        m.pairs = p->d_pairs; m.mval = p->d_mval; m.moff = p->d_moff; m.mu = p->d_mu;
        m.A = p->d_A; m.cn = p->d_cn; m.minv = p->d_minv; m.rings = p->d_rings;
        m.pool = p->d_pool;
        m.nalm = p->nalm;
        m.ap_off = (long long)off;
        off = align_up(off + (size_t)p->nalm * sizeof(double2), 256);
        m.delta_off = (long long)off;
        off = align_up(off + (size_t)p->nrings * (size_t)p->nm * sizeof(double2), 256);
        m.lmax = p->lmax; m.mmax = p->mmax; m.nm = p->nm; m.nrings = p->nrings;
        m.npairs = p->npairs; m.mcontig = p->mcontig;
        m.m0len = (p->mval[0] == 0) ? p->lmax + 1 : 0;
        b->max_nalm = std::max(b->max_nalm, p->nalm);
        sig << "|" << p->lmax << ":" << p->nrings << ":" << p->nm << ":" << p->npix;
    }
    b->ws_bytes = std::max<size_t>(off, 256);
    b->signature = sig.str();

    // work lists: tiles longest first (a tile of map i costs ~ (lmax_i + 2) steps)
    sht_status st = SHT_OK;
    for (int ci = 0; ci < 3 && st == SHT_OK; ++ci) {
        const int ch = kChainChoices[ci];
        std::vector<BatchTile> tiles;
        for (int i = 0; i < n; ++i) {
            const sht_plan_s *p = plans[i];
            const int pblocks = (p->npairs + 64 * ch - 1) / (64 * ch);
            const int nmpairs = (p->nm + 1) / 2;
            for (int q = 0; q < nmpairs; ++q)
                for (int pb = 0; pb < pblocks; ++pb) tiles.push_back({i, q, pb, 0});
        }
        std::stable_sort(tiles.begin(), tiles.end(), [&](const BatchTile &a, const BatchTile &c) {
            return plans[a.map]->lmax > plans[c.map]->lmax;
        });
        b->ntiles[ci] = (int)tiles.size();
        if (hipMalloc((void **)&b->d_tiles[ci], tiles.size() * sizeof(BatchTile)) != hipSuccess ||
            hipMemcpy(b->d_tiles[ci], tiles.data(), tiles.size() * sizeof(BatchTile),
                      hipMemcpyHostToDevice) != hipSuccess)
            st = SHT_ERR_OOM;
    }
    // Fourier work items per ring size class, map by map and ring by ring:
    // the workgroups that run together then read neighbouring rings of one
    // map, whose Delta entries share cache lines
    for (int c = 0; c < sht::kNumSynthClasses && st == SHT_OK; ++c) {
        std::vector<int2> items;
        sht::RingLds lds = {};
        for (int i = 0; i < n; ++i) {
            const sht_plan_s *p = plans[i];
            for (int r = 0; r < p->nrings; ++r)
                if (p->ring_sclass[r] == c) {
                    if (c == sht::kBlueClass) {   // the batch takes FP64 plans only
                        st = SHT_ERR_UNSUPPORTED;
                        break;
                    }
                    items.push_back(make_int2(i, r));
                    if (c == sht::kFastClass)
                        sht::fast_lds_add(lds, p->ring_n[r], p->mmax);
                    else
                        sht::ring_lds_add(lds, c, p->ring_n[r], p->ring_nb[r], p->ring_need[r]);
                }
        }
        b->cls[c].count = (int)items.size();
        b->cls[c].lds = lds;
        if (!items.empty() &&
            (hipMalloc((void **)&b->cls[c].d_items, items.size() * sizeof(int2)) != hipSuccess ||
             hipMemcpy(b->cls[c].d_items, items.data(), items.size() * sizeof(int2),
                       hipMemcpyHostToDevice) != hipSuccess))
            st = SHT_ERR_OOM;
    }
    if (st == SHT_OK &&
        (hipMalloc((void **)&b->d_maps, maps.size() * sizeof(BatchMap)) != hipSuccess ||
         hipMemcpy(b->d_maps, maps.data(), maps.size() * sizeof(BatchMap),
                   hipMemcpyHostToDevice) != hipSuccess))
        st = SHT_ERR_OOM;
    if (st != SHT_OK) {
        free_batch(b);
        delete b;
        return st;
    }
    {
        const double tiles = (double)b->ntiles[chain_index(2)] / (double)std::max(1, b->num_cus);
        for (const BatchShapeRule &r : kBatchShapeTable)
            if (tiles <= r.max_tiles_per_cu) {
                b->chains = r.chains;
                b->waves_per_cu = r.waves_per_cu;
                break;
            }
        sht::log_line("batch maps=%d tiles of 128 pairs per CU=%.1f: launch shape %d chain(s) "
                      "x %d waves per CU (size table); workspace %zu bytes",
                      n, tiles, b->chains, b->waves_per_cu, b->ws_bytes);
    }
    b->magic = kBatchMagic;
    *out = b;
    return SHT_OK;
}

sht_status sht_batch_destroy(sht_batch_t b)
{
    if (!b || b->magic != kBatchMagic) return SHT_ERR_BAD_HANDLE;
    b->magic = sht::kDeadMagic;
    free_batch(b);
    delete b;
    return SHT_OK;
}

sht_status sht_batch_workspace_size(sht_batch_t b, size_t *bytes)
{
    if (!b || b->magic != kBatchMagic) return SHT_ERR_BAD_HANDLE;
    if (!bytes) return SHT_ERR_INVALID_ARG;
    *bytes = b->ws_bytes;
    return SHT_OK;
}

sht_status sht_batch_get_config(sht_batch_t b, int32_t *chains, int32_t *waves_per_cu)
{
    if (!b || b->magic != kBatchMagic) return SHT_ERR_BAD_HANDLE;
    if (chains) *chains = b->chains;
    if (waves_per_cu) *waves_per_cu = b->waves_per_cu;
    return SHT_OK;
}

sht_status sht_batch_set_config(sht_batch_t b, int32_t chains, int32_t waves_per_cu)
{
    if (!b || b->magic != kBatchMagic) return SHT_ERR_BAD_HANDLE;
    if (chains != 1 && chains != 2 && chains != 4) return SHT_ERR_INVALID_ARG;
    if (waves_per_cu < 1 || waves_per_cu > 32) return SHT_ERR_INVALID_ARG;
    b->chains = chains;
    b->waves_per_cu = waves_per_cu;
    return SHT_OK;
}

sht_status sht_alm2map_batch(sht_batch_t b, const double *const *alms, double *const *maps,
                             void *ws, size_t ws_bytes, void *stream)
{
    sht_status s = check_batch(b);
    if (s != SHT_OK) return s;
    if (!alms || !maps) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < b->ws_bytes) return SHT_ERR_WORKSPACE;
    return enqueue(b, alms, maps, ws, (hipStream_t)stream);
}

sht_status sht_batch_autotune(sht_batch_t b, const double *const *alms, double *const *maps,
                              void *ws, size_t ws_bytes, const char *cache_path, void *stream)
{
    sht_status s = check_batch(b);
    if (s != SHT_OK) return s;
    if (!alms || !maps) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < b->ws_bytes) return SHT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    // cache lookup: one line per tuned batch, "<signature> <chains> <waves_per_cu> <ms>"
    if (cache_path && cache_path[0]) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string key;
            int ch = 0, wpc = 0;
            double ms = 0;
            if ((ls >> key >> ch >> wpc >> ms) && key == b->signature &&
                sht_batch_set_config(b, ch, wpc) == SHT_OK)
                return SHT_OK;
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SHT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SHT_ERR_HIP; }
    float best = 1e30f;
    int best_ch = b->chains, best_w = b->waves_per_cu;
    for (int ch : kChainChoices) {
        for (int w : kWaveChoices) {
            b->chains = ch;
            b->waves_per_cu = w;
            s = enqueue(b, alms, maps, ws, st);  // warm-up
            if (s != SHT_OK) break;
            if (hipEventRecord(e0, st) != hipSuccess) { s = SHT_ERR_HIP; break; }
            for (int r = 0; r < 3 && s == SHT_OK; ++r) s = enqueue(b, alms, maps, ws, st);
            if (s != SHT_OK || hipEventRecord(e1, st) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess) {
                s = s == SHT_OK ? SHT_ERR_HIP : s;
                break;
            }
            float ms = 0;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { s = SHT_ERR_HIP; break; }
            if (ms < best) { best = ms; best_ch = ch; best_w = w; }
        }
        if (s != SHT_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->chains = best_ch;
    b->waves_per_cu = best_w;
    if (s == SHT_OK)
        sht::log_line("autotune batch: %d chain(s) x %d waves per CU, %.3f ms per call",
                      best_ch, best_w, best / 3);
    if (s != SHT_OK) return s;
    if (cache_path && cache_path[0]) {
        std::ofstream outf(cache_path, std::ios::app);
        if (outf) outf << b->signature << " " << best_ch << " " << best_w << " " << best / 3 << "\n";
    }
    return SHT_OK;
}

sht_status sht_batch_graph_capture(sht_batch_t b, const double *const *alms, double *const *maps,
                                   void *ws, size_t ws_bytes, void *stream)
{
    sht_status s = check_batch(b);
    if (s != SHT_OK) return s;
    if (!alms || !maps || !stream) return SHT_ERR_INVALID_ARG;
    if (!ws || ws_bytes < b->ws_bytes) return SHT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    if (b->graph_exec) { (void)hipGraphExecDestroy(b->graph_exec); b->graph_exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return SHT_ERR_HIP;
    s = enqueue(b, alms, maps, ws, st);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (s != SHT_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return s != SHT_OK ? s : SHT_ERR_HIP;
    }
    hipGraphExec_t ge = nullptr;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return SHT_ERR_HIP;
    }
    b->graph = g;
    b->graph_exec = ge;
    return SHT_OK;
}

sht_status sht_batch_graph_launch(sht_batch_t b, void *stream)
{
    sht_status s = check_batch(b);
    if (s != SHT_OK) return s;
    if (!b->graph_exec) return SHT_ERR_INVALID_ARG;
    return hipGraphLaunch(b->graph_exec, (hipStream_t)stream) == hipSuccess ? SHT_OK : SHT_ERR_HIP;
}

}  // extern "C"
