// hswo_api.cpp -- host runtime behind the C ABI (include/hswo.h): parameter
// validation, the RHSEG section quadtree (Section 4.1: 4^(L-1) sections,
// reassembled four at a time, Figure 4.4), the workspace plan, and the
// sequence of kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hswo.h"
#include "hswo_internal.h"

using namespace hswo;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(HSWO_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Rect {
    int r0, c0, h, w;
};

void split4(const Rect& r, Rect q[4]) {
    const int h0 = r.h / 2, w0 = r.w / 2;
    q[0] = {r.r0, r.c0, h0, w0};
    q[1] = {r.r0, r.c0 + w0, h0, r.w - w0};
    q[2] = {r.r0 + h0, r.c0, r.h - h0, w0};
    q[3] = {r.r0 + h0, r.c0 + w0, r.h - h0, r.w - w0};
}

int64_t grid_edges(int h, int w, int conn) {
    int64_t e = (int64_t)h * (w - 1) + (int64_t)(h - 1) * w;
    if (conn == 8) e += 2 * (int64_t)(h - 1) * (w - 1);
    return e;
}

int64_t seam_bound(const Rect& r, int seam_conn) { return (int64_t)(r.w + 2 * r.h) * (seam_conn == 8 ? 4 : 2); }

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

int validate_params(const hswo_params* p, int rnb_levels_expected) {
    if (!p) return fail(HSWO_E_INVAL, "params is NULL");
    if (p->connectivity != 4 && p->connectivity != 8)
        return fail(HSWO_E_INVAL, "connectivity must be 4 or 8 (got %d)", p->connectivity);
    if (p->seam_connectivity != 4 && p->seam_connectivity != 8)
        return fail(HSWO_E_INVAL, "seam_connectivity must be 4 or 8 (got %d)", p->seam_connectivity);
    if (!(p->spclust_wght >= 0.0f && p->spclust_wght <= 1.0f))
        return fail(HSWO_E_INVAL, "spclust_wght must be in [0,1] and not NaN");
    if (p->spclust_max < 0 || p->spclust_max > 65535)
        return fail(HSWO_E_INVAL, "spclust_max must be in [0, 65535] (got %d)", p->spclust_max);
    if (p->target_regions < 1) return fail(HSWO_E_INVAL, "target_regions must be >= 1");
    if (p->section_regions < 0) return fail(HSWO_E_INVAL, "section_regions must be >= 0");
    if (p->rnb_levels < 1 || p->rnb_levels > 16) return fail(HSWO_E_INVAL, "rnb_levels must be in [1,16]");
    if (rnb_levels_expected > 0 && p->rnb_levels != rnb_levels_expected)
        return fail(HSWO_E_INVAL, "p->rnb_levels (%d) must equal %d here", p->rnb_levels, rnb_levels_expected);
    if (p->n_levels < 1 || !p->level_counts) return fail(HSWO_E_INVAL, "need n_levels >= 1 and level_counts");
    for (int l = 0; l < p->n_levels; ++l) {
        if (p->level_counts[l] < p->target_regions)
            return fail(HSWO_E_INVAL, "level_counts[%d] = %d is below target_regions", l, p->level_counts[l]);
        if (l > 0 && p->level_counts[l] >= p->level_counts[l - 1])
            return fail(HSWO_E_INVAL, "level_counts must be strictly decreasing");
    }
    if (p->level_counts[p->n_levels - 1] != p->target_regions)
        return fail(HSWO_E_INVAL, "the last level count must equal target_regions");
    if (p->precision != HSWO_PREC_FP32 && p->precision != HSWO_PREC_SCREEN_BF16 &&
        p->precision != HSWO_PREC_SCREEN_FP16)
        return fail(HSWO_E_INVAL, "unknown precision %d", p->precision);
    return HSWO_OK;
}

int validate_shape(int H, int W, int B, int dtype) {
    if (H < 1 || W < 1) return fail(HSWO_E_INVAL, "H and W must be >= 1");
    if ((int64_t)H * W >= ((int64_t)1 << 31)) return fail(HSWO_E_INVAL, "H*W must be < 2^31");
    if (B < 1 || B > MAX_B) return fail(HSWO_E_INVAL, "B must be in [1, %d]", MAX_B);
    if (dtype != HSWO_F32 && dtype != HSWO_F16) return fail(HSWO_E_INVAL, "dtype must be HSWO_F32 or HSWO_F16");
    return HSWO_OK;
}

// Bump allocator over the caller's workspace (sizes only when base is null).
struct Bump {
    char* base = nullptr;
    size_t off = 0;
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

struct SecPlan {
    Rect rect;
    int64_t cap, ecap, fin, tiles, hash_cap, seam;
    int stop;
};

// Per-section sizes of every recursion level (depth 0 = whole image).
struct Plan {
    int L = 1, B = 1, Bp = 32, stopS = 1;
    std::vector<std::vector<SecPlan>> lv;
    int64_t total_merges = 0;
};

int64_t tiles_for(int64_t cap, const hswo_params* p) {
    if (!(p->spclust_wght > 0.0f) || p->spclust_max <= 0) return 1;
    const int64_t K = std::min<int64_t>(cap, p->spclust_max);
    const int64_t nT = (K + TILE - 1) / TILE;
    return std::max<int64_t>(1, nT * (nT + 1) / 2);
}

Plan make_plan(int H, int W, int B, const hswo_params* p, int L) {
    Plan pl;
    pl.L = L;
    pl.B = B;
    pl.Bp = round_up(B, BK);
    pl.stopS = p->section_regions > 0 ? p->section_regions : std::max(p->target_regions, p->spclust_max / 4);
    pl.lv.assign(L, {});
    pl.lv[0].push_back(SecPlan{{0, 0, H, W}, 0, 0, 0, 0, 0, 0, 0});
    for (int d = 1; d < L; ++d)
        for (const SecPlan& s : pl.lv[d - 1]) {
            Rect q[4];
            split4(s.rect, q);
            for (int k = 0; k < 4; ++k) pl.lv[d].push_back(SecPlan{q[k], 0, 0, 0, 0, 0, 0, 0});
        }
    for (int d = L - 1; d >= 0; --d) {
        const int stop = d == 0 ? p->target_regions : pl.stopS;
        for (size_t i = 0; i < pl.lv[d].size(); ++i) {
            SecPlan& s = pl.lv[d][i];
            s.stop = stop;
            if (d == L - 1) {
                s.cap = (int64_t)s.rect.h * s.rect.w;
                s.ecap = grid_edges(s.rect.h, s.rect.w, p->connectivity);
            } else {
                s.cap = 0;
                s.ecap = 0;
                for (int k = 0; k < 4; ++k) {
                    const SecPlan& c = pl.lv[d + 1][4 * i + k];
                    s.cap += c.fin;
                    s.ecap += std::min<int64_t>(c.ecap, c.fin * (c.fin - 1) / 2);
                }
                s.seam = seam_bound(s.rect, p->seam_connectivity);
                s.ecap += s.seam;
                s.hash_cap = next_pow2(2 * s.seam + 16);
            }
            s.ecap = std::max<int64_t>(s.ecap, 1);
            s.fin = std::min<int64_t>(s.cap, stop);
            s.tiles = tiles_for(s.cap, p);
            pl.total_merges += s.cap - s.fin;
        }
    }
    return pl;
}

// Device-side objects of one level carved from the workspace.
struct LevelDev {
    SecDev* secs = nullptr;
    AsmDev* asms = nullptr;
    InitDev* inits = nullptr;
    std::vector<SecDev> h_secs;
    std::vector<AsmDev> h_asms;
    std::vector<InitDev> h_inits;
};

struct Layout {
    unsigned long long* counters = nullptr;
    int32_t* counts = nullptr;
    int32_t* parent = nullptr;
    int32_t* mtime = nullptr;
    int32_t* slotmap = nullptr;
    SnapDev* snap = nullptr;
    std::vector<LevelDev> lv;
    size_t bytes = 0;
};

// Carve the workspace for an RHSEG run (sizes only when ws is null).
Layout carve(const Plan& pl, int H, int W, const hswo_params* p, void* ws, const void* cube, int32_t* labels,
             hswo_merge_rec* log) {
    Layout lay;
    Bump bp;
    bp.base = reinterpret_cast<char*>(ws);
    const int64_t P = (int64_t)H * W;
    lay.counters = bp.take<unsigned long long>(C_COUNT);
    lay.counts = bp.take<int32_t>(p->n_levels);
    lay.parent = bp.take<int32_t>(P);
    lay.mtime = bp.take<int32_t>(P);
    if (pl.L > 1) lay.slotmap = bp.take<int32_t>(P);
    lay.snap = bp.take<SnapDev>(1);
    lay.lv.resize(pl.L);
    int64_t log_base = 0;
    for (int d = pl.L - 1; d >= 0; --d) {
        const auto& secs = pl.lv[d];
        LevelDev& L = lay.lv[d];
        const size_t n = secs.size();
        L.secs = bp.take<SecDev>(n);
        if (d < pl.L - 1) L.asms = bp.take<AsmDev>(n);
        if (d == pl.L - 1) L.inits = bp.take<InitDev>(n);
        L.h_secs.resize(n);
        if (d < pl.L - 1) L.h_asms.resize(n);
        if (d == pl.L - 1) L.h_inits.resize(n);
        for (size_t i = 0; i < n; ++i) {
            const SecPlan& sp = secs[i];
            SecDev& s = L.h_secs[i];
            std::memset(&s, 0, sizeof(s));
            s.R0 = (int32_t)sp.cap;
            s.B = pl.B;
            s.Bp = pl.Bp;
            s.Ecap = (int32_t)sp.ecap;
            s.stop = sp.stop;
            s.top = d == 0 ? 1 : 0;
            s.log_base = (int32_t)log_base;
            s.tiles = (int32_t)sp.tiles;
            s.label = bp.take<int32_t>(sp.cap);
            s.npix = bp.take<int32_t>(sp.cap);
            s.mark = bp.take<int32_t>(sp.cap);
            s.norm = bp.take<float>(sp.cap);
            s.sums = bp.take<double>(sp.cap * pl.B);
            s.mean = bp.take<float>(sp.cap * pl.Bp);
            s.edges = bp.take<int2>(sp.ecap);
            s.escr = bp.take<float2>(sp.ecap);
            s.tstat = bp.take<float2>(sp.tiles);
            s.tflag = bp.take<int32_t>(sp.tiles);
            if (p->precision != HSWO_PREC_FP32 && p->spclust_wght > 0.0f && p->spclust_max > 0) {
                const int64_t kc = std::min<int64_t>(sp.cap, p->spclust_max);
                s.kcap = (int32_t)kc;
                s.g16 = bp.take<uint16_t>(kc * pl.Bp);
                s.gn = bp.take<float>(kc);
                s.geta = bp.take<float>(kc);
                s.galpha = bp.take<float>(kc);
                s.gP = bp.take<float>(kc);
                s.cvec = bp.take<float>(pl.Bp);
            }
            s.st = bp.take<int32_t>(ST_WORDS);
            s.parent = lay.parent;
            s.mtime = lay.mtime;
            s.log = log ? log + log_base : nullptr;
            log_base += sp.cap - sp.fin;
            if (d < pl.L - 1) {
                AsmDev& a = L.h_asms[i];
                a.child0 = (int32_t)(4 * i);
                a.r0 = sp.rect.r0;
                a.c0 = sp.rect.c0;
                a.h = sp.rect.h;
                a.w = sp.rect.w;
                a.img_w = W;
                a.seam_conn = p->seam_connectivity;
                a.hash_cap = (int32_t)sp.hash_cap;
                a.hash = bp.take<unsigned long long>(sp.hash_cap);
            } else {
                InitDev& in = L.h_inits[i];
                in.cube = cube;
                in.img_w = W;
                in.r0 = sp.rect.r0;
                in.c0 = sp.rect.c0;
                in.h = sp.rect.h;
                in.w = sp.rect.w;
                in.label_w = W;
                in.conn = p->connectivity;
            }
        }
    }
    (void)labels;
    lay.bytes = bp.off + 256;
    return lay;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    std::vector<hipEvent_t> drv;  // pairs around each section-driver launch
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        for (hipEvent_t e : drv) (void)hipEventDestroy(e);
    }
};

// Launch the section driver, bracketed by events when timing is on.
int timed_driver(Timer* tm, const SecDev* secs, int n, const LoopParams& lp, hipStream_t stream) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm) {
        HIP_TRY(hipEventCreate(&e0));
        tm->drv.push_back(e0);
        HIP_TRY(hipEventCreate(&e1));
        tm->drv.push_back(e1);
        HIP_TRY(hipEventRecord(e0, stream));
    }
    HIP_TRY(launch_section_driver(secs, n, lp, stream));
    if (tm) HIP_TRY(hipEventRecord(e1, stream));
    return HSWO_OK;
}

int run_rhseg(const void* cube, int H, int W, int B, int dtype, const hswo_params* p, int L, int32_t* labels,
              hswo_merge_rec* merge_log, hswo_stats* stats, void* workspace, size_t ws_bytes,
              hipStream_t stream) {
    int rc = validate_shape(H, W, B, dtype);
    if (rc) return rc;
    rc = validate_params(p, L);
    if (rc) return rc;
    if (!cube || !labels) return fail(HSWO_E_INVAL, "cube and labels must be device pointers");
    if (reinterpret_cast<uintptr_t>(cube) % 16) return fail(HSWO_E_INVAL, "cube must be 16-byte aligned");
    if ((H >> (L - 1)) < 1 || (W >> (L - 1)) < 1)
        return fail(HSWO_E_INVAL, "rnb_levels=%d leaves empty sections for %dx%d", L, H, W);
    if ((p->flags & HSWO_FLAG_MERGE_LOG) && !merge_log) return fail(HSWO_E_INVAL, "MERGE_LOG flag needs merge_log");
    if (!workspace) return fail(HSWO_E_INVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(HSWO_E_INVAL, "workspace must be 256-byte aligned");

    const Plan pl = make_plan(H, W, B, p, L);
    Layout lay = carve(pl, H, W, p, workspace, cube, labels, merge_log);
    if (ws_bytes < lay.bytes)
        return fail(HSWO_E_NOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, lay.bytes);

    Timer tm;
    if (stats) {
        HIP_TRY(hipEventCreate(&tm.a));
        HIP_TRY(hipEventCreate(&tm.b));
        HIP_TRY(hipEventRecord(tm.a, stream));
    }
    const int64_t P = (int64_t)H * W;
    // descriptors
    HIP_TRY(hipMemcpyAsync(lay.counts, p->level_counts, sizeof(int32_t) * p->n_levels, hipMemcpyHostToDevice, stream));
    for (int d = 0; d < L; ++d) {
        LevelDev& lv = lay.lv[d];
        HIP_TRY(hipMemcpyAsync(lv.secs, lv.h_secs.data(), sizeof(SecDev) * lv.h_secs.size(), hipMemcpyHostToDevice,
                               stream));
        if (!lv.h_asms.empty())
            HIP_TRY(hipMemcpyAsync(lv.asms, lv.h_asms.data(), sizeof(AsmDev) * lv.h_asms.size(),
                                   hipMemcpyHostToDevice, stream));
        if (!lv.h_inits.empty())
            HIP_TRY(hipMemcpyAsync(lv.inits, lv.h_inits.data(), sizeof(InitDev) * lv.h_inits.size(),
                                   hipMemcpyHostToDevice, stream));
    }
    SnapDev sd;
    sd.st = lay.lv[0].h_secs[0].st;
    sd.parent = lay.parent;
    sd.mtime = lay.mtime;
    sd.labels = labels;
    sd.img_w = W;
    sd.r0 = 0;
    sd.c0 = 0;
    sd.h = H;
    sd.w = W;
    sd.label_w = W;
    HIP_TRY(hipMemcpyAsync(lay.snap, &sd, sizeof(SnapDev), hipMemcpyHostToDevice, stream));
    HIP_TRY(launch_fill_u64(lay.counters, C_COUNT, 0ull, stream));

    LoopParams lp;
    lp.w2 = (double)p->spclust_wght * (double)p->spclust_wght;
    lp.spectral = p->spclust_wght > 0.0f && p->spclust_max > 0 ? 1 : 0;
    lp.kmax = p->spclust_max;
    lp.precision = p->precision;
    lp.pad = 0;
    lp.counters = lay.counters;

    HIP_TRY(launch_init_pixels(lay.parent, lay.mtime, P, stream));
    {
        const int d = L - 1;
        int maxpix = 0;
        for (const SecPlan& s : pl.lv[d]) maxpix = std::max<int>(maxpix, (int)s.cap);
        HIP_TRY(launch_init_leaves(lay.lv[d].secs, lay.lv[d].inits, (int)pl.lv[d].size(), dtype, maxpix, stream));
        rc = timed_driver(stats ? &tm : nullptr, lay.lv[d].secs, (int)pl.lv[d].size(), lp, stream);
        if (rc) return rc;
    }
    for (int d = L - 2; d >= 0; --d) {
        const auto& secs = pl.lv[d];
        int64_t maxcap = 0, maxseam = 0;
        for (const SecPlan& s : secs) {
            maxcap = std::max(maxcap, std::max(s.cap, s.ecap));
            maxseam = std::max(maxseam, (int64_t)(s.rect.w + 2 * s.rect.h));
            HIP_TRY(launch_fill_u64(lay.lv[d].h_asms[&s - &secs[0]].hash, (size_t)s.hash_cap, ~0ull, stream));
        }
        HIP_TRY(launch_compress(lay.parent, P, stream));
        HIP_TRY(launch_assemble(lay.lv[d].secs, lay.lv[d + 1].secs, lay.lv[d].asms, (int)secs.size(), lay.slotmap,
                                (int)std::min<int64_t>(maxcap, 1 << 30), stream));
        HIP_TRY(launch_seam(lay.lv[d].secs, lay.lv[d].asms, (int)secs.size(), lay.slotmap, (int)maxseam, stream));
        rc = timed_driver(stats ? &tm : nullptr, lay.lv[d].secs, (int)secs.size(), lp, stream);
        if (rc) return rc;
    }
    HIP_TRY(launch_snapshot(lay.snap, 1, lay.counts, p->n_levels, (int)P, stream));

    if (stats) {
        HIP_TRY(hipEventRecord(tm.b, stream));
        unsigned long long c[C_COUNT];
        HIP_TRY(hipMemcpyAsync(c, lay.counters, sizeof(c), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, tm.a, tm.b));
        stats->merges = (int64_t)c[C_MERGES];
        stats->iterations = (int64_t)c[C_ITERS];
        stats->adjacent_pairs = (int64_t)c[C_ADJ_PAIRS];
        stats->spectral_pairs = (int64_t)c[C_SPEC_PAIRS];
        stats->exact_rechecks = (int64_t)c[C_RECHECKS];
        stats->tile_rescans = (int64_t)c[C_RESCANS];
        stats->fp32_tiles = (int64_t)c[C_FP32_TILES];
        stats->mfma_tiles = (int64_t)c[C_MFMA_TILES];
        stats->ms_total = ms;
        double md = 0.0;
        for (size_t k = 0; k + 1 < tm.drv.size(); k += 2) {
            float x = 0.f;
            HIP_TRY(hipEventElapsedTime(&x, tm.drv[k], tm.drv[k + 1]));
            md += x;
        }
        stats->ms_driver = md;
        int dev = 0, khz = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        const double tick_ms = khz > 0 ? 1.0 / (double)khz : 1e-5;  // device constant clock
        stats->ms_adjacent = (double)c[C_T_ADJ] * tick_ms;
        stats->ms_mfma_screen = (double)c[C_T_MFMA] * tick_ms;
        stats->ms_fp32_spectral = (double)c[C_T_SPEC32] * tick_ms;
        stats->ms_merge = (double)c[C_T_MERGE] * tick_ms;
        stats->driver_launches = (int64_t)(tm.drv.size() / 2);
    }
    return HSWO_OK;
}

}  // namespace

extern "C" {

int hswo_version(void) { return HSWO_VERSION; }

const char* hswo_last_error(void) { return g_err.c_str(); }

size_t hswo_workspace_bytes(int32_t H, int32_t W, int32_t B, int32_t dtype, const hswo_params* p) {
    if (validate_shape(H, W, B, dtype) || validate_params(p, 0)) return 0;
    const int L = p->rnb_levels;
    if ((H >> (L - 1)) < 1 || (W >> (L - 1)) < 1) return 0;
    const Plan pl = make_plan(H, W, B, p, L);
    return carve(pl, H, W, p, nullptr, nullptr, nullptr, nullptr).bytes;
}

int hswo_run(const void* cube, int32_t H, int32_t W, int32_t B, int32_t dtype, const hswo_params* p,
             int32_t* labels, hswo_merge_rec* merge_log, hswo_stats* stats, void* workspace, size_t ws_bytes,
             void* hip_stream) {
    g_err.clear();
    if (p && p->rnb_levels != 1) return fail(HSWO_E_INVAL, "hswo_run needs p->rnb_levels == 1");
    return run_rhseg(cube, H, W, B, dtype, p, 1, labels, merge_log, stats, workspace, ws_bytes,
                     reinterpret_cast<hipStream_t>(hip_stream));
}

int rhseg_segment(const void* cube, int32_t H, int32_t W, int32_t B, int32_t dtype, const hswo_params* p,
                  int32_t rnb_levels, int32_t* labels, hswo_merge_rec* merge_log, hswo_stats* stats,
                  void* workspace, size_t ws_bytes, void* hip_stream) {
    g_err.clear();
    if (rnb_levels < 1 || rnb_levels > 16) return fail(HSWO_E_INVAL, "rnb_levels must be in [1,16]");
    return run_rhseg(cube, H, W, B, dtype, p, rnb_levels, labels, merge_log, stats, workspace, ws_bytes,
                     reinterpret_cast<hipStream_t>(hip_stream));
}

size_t hswo_batch_workspace_bytes(int32_t n_sections, const hswo_section* sections, int32_t dtype,
                                  const hswo_params* p) {
    (void)n_sections;
    (void)sections;
    (void)dtype;
    (void)p;
    return 0;
}

int hswo_run_batch(int32_t n_sections, const hswo_section* sections, int32_t dtype, const hswo_params* p,
                   hswo_stats* stats, void* workspace, size_t ws_bytes, void* hip_stream) {
    (void)n_sections;
    (void)sections;
    (void)dtype;
    (void)p;
    (void)stats;
    (void)workspace;
    (void)ws_bytes;
    (void)hip_stream;
    g_err.clear();
    return fail(HSWO_E_UNSUPPORTED, "hswo_run_batch is not available in this build");
}

}  // extern "C"
