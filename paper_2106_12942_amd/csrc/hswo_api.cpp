// hswo_api.cpp -- host runtime behind the C ABI (include/hswo.h): parameter
// validation, the RHSEG section quadtree (Section 4.1: 4^(L-1) sections,
// reassembled four at a time, Figure 4.4), the workspace plan, and the
// sequence of kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hswo.h"
#include "hswo_internal.h"

using namespace hswo;

// the struct sizes the header states (the Python binding mirrors them)
static_assert(sizeof(hswo_params) == 80, "hswo_params layout");
static_assert(sizeof(hswo_tuning) == 28, "hswo_tuning layout");
static_assert(sizeof(hswo_stats) == 424, "hswo_stats layout");
static_assert(sizeof(hswo_merge_rec) == 24, "hswo_merge_rec layout");
static_assert(sizeof(hswo_verify_rec) == 48, "hswo_verify_rec layout");
static_assert(sizeof(hswo_section) == 40, "hswo_section layout");

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

// Edge slots of a leaf: one per pixel and forward neighbour direction (the
// boundary's missing neighbours are empty slots until the first merge).
int64_t grid_edges(int h, int w, int conn) { return (int64_t)h * w * (conn == 8 ? 4 : 2); }


int64_t seam_bound(const Rect& r, int seam_conn) { return (int64_t)(r.w + 2 * r.h) * (seam_conn == 8 ? 4 : 2); }

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

int validate_tuning(const hswo_tuning* g);

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
    if (p->criterion != HSWO_CRIT_BSMSE && p->criterion != HSWO_CRIT_SAM)
        return fail(HSWO_E_INVAL, "unknown criterion %d", p->criterion);
    if ((p->flags & HSWO_FLAG_TWO_MERGES) && !(p->flags & HSWO_FLAG_INCREMENTAL))
        return fail(HSWO_E_UNSUPPORTED, "HSWO_FLAG_TWO_MERGES is implemented in the HSWO_FLAG_INCREMENTAL form only");
    if (p->flags & HSWO_FLAG_MULTI_MERGE) {
        if (!(p->flags & HSWO_FLAG_INCREMENTAL) || p->criterion != HSWO_CRIT_BSMSE)
            return fail(HSWO_E_UNSUPPORTED,
                        "HSWO_FLAG_MULTI_MERGE is implemented in the HSWO_FLAG_INCREMENTAL form with Equation 1 only");
        if (p->flags & HSWO_FLAG_TWO_MERGES)
            return fail(HSWO_E_INVAL, "HSWO_FLAG_MULTI_MERGE and HSWO_FLAG_TWO_MERGES are different readings");
    }
    if (p->criterion == HSWO_CRIT_SAM && !(p->flags & HSWO_FLAG_INCREMENTAL))
        return fail(HSWO_E_UNSUPPORTED, "criterion HSWO_CRIT_SAM is implemented in the HSWO_FLAG_INCREMENTAL form only");
    if (p->screen_topk < 0) return fail(HSWO_E_INVAL, "screen_topk must be >= 0");
    if (p->flags & HSWO_FLAG_DEBUG_VERIFY_BOUND) {
        if (p->flags & HSWO_FLAG_INCREMENTAL)
            return fail(HSWO_E_INVAL, "HSWO_FLAG_DEBUG_VERIFY_BOUND checks the screened forms; the incremental form "
                                      "evaluates every pair exactly");
        if (!p->verify || p->verify_cap < 0)
            return fail(HSWO_E_INVAL, "HSWO_FLAG_DEBUG_VERIFY_BOUND needs a verify buffer and verify_cap >= 0");
    }
    return validate_tuning(p->tuning);
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

// Scratch of the several-merges-per-step reading: sort keys and payloads for
// up to max(ecap, cap) entries (a power of two), per-slot places and the
// step's pair list.
void take_multi(Bump& bp, SecDev& s, int64_t cap, int64_t ecap) {
    int64_t z = 1;
    while (z < std::max(cap, ecap)) z <<= 1;
    s.zcap = (int32_t)z;
    s.zkey = bp.take<unsigned long long>(z);
    s.zval = bp.take<unsigned long long>(z);
    s.zuse = bp.take<int32_t>(cap);
    s.zlist = bp.take<int4>(cap / 2 + 1);
}

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

// The incremental form keeps exact spectral rows instead of screening every
// pair each iteration (the 16-bit screen rows are then not needed).
int device_cus();

// Execution settings of one call (hswo_tuning, resolved: no -1 left).
struct Tuning {
    int wide_max = 0;   // levels of more sections run in the persistent driver
    int wide_wg = 0;    // wide mode: workgroups per level, shared by its sections (G = wide_wg / n)
    int rows_grid = 0;  // wide mode, incremental form: workgroups of the row-stage launch
    int hybrid = 1;     // incremental form: pre-spectral merges of a wide level in the persistent driver
    int bare = 1;       // row-cache second bounds kept bare: 0 none, 1 those of value 0, 2 all
    int variant = 6;    // adjacent-sweep edges in flight per 16-lane group (screened forms)
    int row_matrix = 1; // incremental form, wide mode: the row cache's interval matrix
    std::string str() const {
        return std::to_string(wide_max) + "," + std::to_string(wide_wg) + "," + std::to_string(rows_grid) + "," +
               std::to_string(hybrid) + "," + std::to_string(bare) + "," + std::to_string(variant) + "," +
               std::to_string(row_matrix);
    }
};

// Library defaults. Measured: the screened and plain forms gain from wide
// mode up to 64 sections (G >= 4, on the 512x512 workload); the incremental
// form gains up to one workgroup per section, because its row evaluations
// pool over the whole device (the 1024x1024 salt cube's 256 leaves: 2.0 s
// persistent, 1.23 s wide).
Tuning default_tuning(bool incremental) {
    Tuning t;
    t.wide_max = incremental ? device_cus() : 64;
    t.wide_wg = device_cus();
    t.rows_grid = 2 * device_cus();
    t.hybrid = 1;
    t.bare = 1;
    t.variant = 6;
    t.row_matrix = 1;
    return t;
}

// Overlay the fields the caller gave (hswo_tuning, -1 = not given).
Tuning overlay(Tuning t, const hswo_tuning* g) {
    if (!g) return t;
    if (g->wide_max_sections >= 0) t.wide_max = g->wide_max_sections;
    if (g->wide_groups >= 0) t.wide_wg = g->wide_groups;
    if (g->rows_grid >= 0) t.rows_grid = g->rows_grid;
    if (g->hybrid >= 0) t.hybrid = g->hybrid;
    if (g->bare_bounds >= 0) t.bare = g->bare_bounds;
    if (g->driver_variant >= 0) t.variant = g->driver_variant;
    if (g->row_matrix >= 0) t.row_matrix = g->row_matrix;
    return t;
}

int validate_tuning(const hswo_tuning* g) {
    if (!g) return HSWO_OK;
    if (g->wide_max_sections < -1) return fail(HSWO_E_INVAL, "tuning.wide_max_sections must be >= -1");
    if (g->wide_groups != -1 && (g->wide_groups < 1 || g->wide_groups > 65536))
        return fail(HSWO_E_INVAL, "tuning.wide_groups must be -1 or in [1, 65536]");
    if (g->rows_grid != -1 && (g->rows_grid < 1 || g->rows_grid > 65535))
        return fail(HSWO_E_INVAL, "tuning.rows_grid must be -1 or in [1, 65535]");
    if (g->hybrid < -1 || g->hybrid > 1) return fail(HSWO_E_INVAL, "tuning.hybrid must be -1, 0 or 1");
    if (g->bare_bounds < -1 || g->bare_bounds > 2) return fail(HSWO_E_INVAL, "tuning.bare_bounds must be in [-1, 2]");
    if (g->driver_variant != -1 && g->driver_variant != 2 && g->driver_variant != 4 && g->driver_variant != 6)
        return fail(HSWO_E_INVAL, "tuning.driver_variant must be -1, 2, 4 or 6");
    if (g->row_matrix < -1 || g->row_matrix > 1) return fail(HSWO_E_INVAL, "tuning.row_matrix must be -1, 0 or 1");
    return HSWO_OK;
}

bool row_cache_on(const hswo_params* p) {
    return (p->flags & HSWO_FLAG_INCREMENTAL) && p->spclust_wght > 0.0f && p->spclust_max > 0;
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
                    // a child that merges ends with distinct real edges only; one that
                    // makes no merge hands over its slots as they are
                    s.ecap += c.cap > c.stop ? std::min<int64_t>(c.ecap, c.fin * (c.fin - 1) / 2) : c.ecap;
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

// Per-section sizes are int32 on the device: reject a plan whose edge or
// tile capacity would not fit (a leaf's edge slots are h*w*4 under
// 8-connectivity, which can pass 2^31 while h*w does not). The edge index
// keeps twice an edge slot number (plus one) in an int32, hence at most 2^30
// edge slots.
int check_plan(const Plan& pl) {
    for (size_t d = 0; d < pl.lv.size(); ++d)
        for (const SecPlan& s : pl.lv[d]) {
            if (s.ecap > ((int64_t)1 << 30) || s.cap > INT32_MAX || s.tiles > INT32_MAX)
                return fail(HSWO_E_UNSUPPORTED,
                            "a section of recursion depth %zu needs %lld edge slots and %lld regions; "
                            "the device keeps both in int32, at most 2^30 edge slots (use more recursion levels)",
                            d, (long long)s.ecap, (long long)s.cap);
        }
    return HSWO_OK;
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
Layout carve(const Plan& pl, int H, int W, const hswo_params* p, int bare, void* ws, const void* cube,
             int32_t* labels, hswo_merge_rec* log) {
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
            s.crit = p->criterion;
            s.bare = bare;
            s.label = bp.take<int32_t>(sp.cap);
            s.npix = bp.take<int32_t>(sp.cap);
            s.mark = bp.take<int32_t>(sp.cap);
            s.dmark = bp.take<int32_t>(sp.cap);
            s.norm = bp.take<float>(sp.cap);
            s.sums = bp.take<double>(sp.cap * pl.B);
            s.mean = bp.take<float>(sp.cap * pl.Bp);
            s.edges = bp.take<int2>(sp.ecap);
            s.escr = bp.take<float2>(sp.ecap);
            if (p->flags & HSWO_FLAG_INCREMENTAL) {
                s.ed2 = bp.take<double>(sp.ecap);
                s.edirty = bp.take<int32_t>(sp.ecap);
                s.rmin = bp.take<int32_t>(sp.cap);
                s.rmax = bp.take<int32_t>(sp.cap);
                s.cmd2 = bp.take<double>((sp.ecap + ECH - 1) / ECH);
                s.cme = bp.take<int2>((sp.ecap + ECH - 1) / ECH);
                s.cml = bp.take<int2>((sp.ecap + ECH - 1) / ECH);
                if (p->flags & HSWO_FLAG_MULTI_MERGE) take_multi(bp, s, sp.cap, sp.ecap);
            }
            s.tstat = bp.take<float2>(sp.tiles);
            s.tflag = bp.take<int32_t>(sp.tiles);
            if (row_cache_on(p)) {
                const int64_t rc = std::min<int64_t>(sp.cap, p->spclust_max);
                s.rcap = (int32_t)rc;
                s.m64 = bp.take<double>(rc * pl.B);
                s.m64r = bp.take<double>(rc * (((int64_t)pl.B + 7) / 8 * 8));
                if (p->criterion == HSWO_CRIT_SAM) s.rq = bp.take<double>(rc);
                else if (!(p->flags & (HSWO_FLAG_TWO_MERGES | HSWO_FLAG_MULTI_MERGE)) && rc <= MAT_MAX) {
                    int64_t n16 = (rc + 15) / 16;
                    if (n16 % 2 == 0) ++n16;
                    s.mstride = (int32_t)(n16 * 16);
                    s.dmat = bp.take<float2>(rc * s.mstride);
                    s.msl = bp.take<int32_t>(rc);
                }
                if (p->flags & HSWO_FLAG_TWO_MERGES) s.abit = bp.take<uint32_t>(rc * ((rc + 31) / 32));
                s.rbd = bp.take<double>(rc);
                s.rbp = bp.take<int32_t>(rc);
                s.rbl = bp.take<int32_t>(rc);
                s.rbd2 = bp.take<double>(rc);
                s.rbp2 = bp.take<int32_t>(rc);
                s.rbl2 = bp.take<int32_t>(rc);
                s.rpend = bp.take<int32_t>(rc);
                s.rpart = bp.take<RowPart>(rc * ((rc + 63) / 64));
                } else if (p->precision != HSWO_PREC_FP32 && p->spclust_wght > 0.0f && p->spclust_max > 0) {
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
            s.wi = bp.take<int32_t>(16);
            s.wd = bp.take<double>(4);
            s.wpart = bp.take<float>(2 * GMAX);
            if (p->flags & HSWO_FLAG_DEBUG_VERIFY_BOUND) {
                s.vraw = bp.take<float>(sp.ecap);
                s.vstage = bp.take<float>(CAND_CAP);
                s.vout = p->verify;
                s.vcap = p->verify_cap;
                s.vcount = lay.counters ? lay.counters + C_VERIFY : nullptr;
            }
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

// ---------------------------------------------------------------------------
// Execution. Every call is a set of descriptor uploads (always eager) and a
// kernel sequence. The sequence runs eagerly, or is captured once into a
// hipGraph and replayed (HSWO_FLAG_GRAPH); the section-driver variant is
// chosen by the autotuner (HSWO_FLAG_AUTOTUNE) or from its cache.
// ---------------------------------------------------------------------------
struct Upload {
    void* dst;
    std::vector<char> bytes;
};

template <class T>
void add_upload(std::vector<Upload>& ups, void* dst, const T* src, size_t n) {
    Upload u;
    u.dst = dst;
    u.bytes.resize(sizeof(T) * n);
    std::memcpy(u.bytes.data(), src, sizeof(T) * n);
    ups.push_back(std::move(u));
}

struct Timer {
    std::vector<hipEvent_t> drv;  // pairs around each level's merge-loop launches
    bool kernels = false;         // HSWO_FLAG_KERNEL_TIMES: also bracket every launch by kind
    KTimer kt;
    KTimer* per_kernel() { return kernels ? &kt : nullptr; }
    ~Timer() {
        for (hipEvent_t e : drv) (void)hipEventDestroy(e);
    }
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Launch the section driver, bracketed by events when timing is on.
int timed_driver(Timer* tm, const SecDev* secs, int n, const LoopParams& lp, int variant, hipStream_t stream) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm) {
        HIP_TRY(hipEventCreate(&e0));
        tm->drv.push_back(e0);
        HIP_TRY(hipEventCreate(&e1));
        tm->drv.push_back(e1);
        HIP_TRY(hipEventRecord(e0, stream));
    }
    HIP_TRY(launch_section_driver(secs, n, lp, variant, stream, tm ? tm->per_kernel() : nullptr));
    if (tm) HIP_TRY(hipEventRecord(e1, stream));
    return HSWO_OK;
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// One level: secs[0..n) with per-section (cap, stop). How its merge loops
// run: persistent (one workgroup per section, one launch) when it has more
// than tu.wide_max sections, else wide (G workgroups per section, one launch
// sequence per iteration). In wide mode the host knows R at iteration t
// exactly (cap - t, until the stop count), so the spectral kernels are
// launched only for iterations where some section can be in its spectral
// stage.
// In the incremental form the iterations of a pass before its spectral stage
// (R > spclust_max) need no work spread over workgroups: with tu.hybrid they
// run in the section driver (one launch, state kept on chip) up to
// R = spclust_max, and wide mode takes the rest.
// mat_ok: every section of the level keeps an interval matrix (used, in either
// mode, when the tuning asks for it).
int run_level(Timer* tm, const SecDev* secs, int n, const std::vector<int64_t>& cap, const std::vector<int64_t>& stop,
              const LoopParams& lp_in, bool row_cache, bool mat_ok, const Tuning& tu, hipStream_t stream) {
    LoopParams lp = lp_in;
    lp.row_matrix = (row_cache && mat_ok && tu.row_matrix) ? 1 : 0;
    const int variant = tu.variant;
    if (n > tu.wide_max || (row_cache && n > ROWS_MAX_SECTIONS) || lp.multi_merge)
        return timed_driver(tm, secs, n, lp, variant, stream);
    const int G = std::max(1, std::min(GMAX, tu.wide_wg / n));
    // R of each section when the wide iterations start
    std::vector<int64_t> r0(cap);
    if (lp.incremental && lp.spectral && tu.hybrid) {
        int64_t pre = 0;
        for (int i = 0; i < n; ++i) {
            const int64_t p = std::max<int64_t>(lp.kmax, stop[i]);
            if (cap[i] > p) {
                pre = std::max(pre, cap[i] - p);
                r0[i] = p;
            }
        }
        if (pre > 0) {
            LoopParams lpp = lp;
            lpp.phase_stop = lp.kmax;
            const int rc = timed_driver(tm, secs, n, lpp, variant, stream);
            if (rc) return rc;
        } else {
            r0 = cap;
        }
    }
    int64_t iters = 0;
    for (int i = 0; i < n; ++i) iters = std::max(iters, r0[i] - std::min(r0[i], stop[i]));
    // interval matrices: each section's cache starts at its first iteration inside the spectral
    // stage (R = min(r0, kmax)); those iterations launch the fill first
    int fill_tiles = 0;
    std::vector<int64_t> fill_at;
    if (lp.row_matrix) {
        int64_t rmax = 0;
        for (int i = 0; i < n; ++i) {
            if (std::min(r0[i], (int64_t)lp.kmax) <= stop[i]) continue;  // never reaches its spectral stage
            fill_at.push_back(std::max<int64_t>(0, r0[i] - lp.kmax));
            rmax = std::max(rmax, std::min(r0[i], (int64_t)lp.kmax));
        }
        const int64_t nT = (rmax + TILE - 1) / TILE;
        fill_tiles = (int)(nT * (nT + 1) / 2);
        std::sort(fill_at.begin(), fill_at.end());
        fill_at.erase(std::unique(fill_at.begin(), fill_at.end()), fill_at.end());
    }
    // (two-merge reading: a launch still makes exactly one merge -- a step 3 that finds no pair
    // below its threshold goes on to the next step 2 in the same launch)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm) {
        HIP_TRY(hipEventCreate(&e0));
        tm->drv.push_back(e0);
        HIP_TRY(hipEventCreate(&e1));
        tm->drv.push_back(e1);
        HIP_TRY(hipEventRecord(e0, stream));
    }
    KTimer* kt = tm ? tm->per_kernel() : nullptr;
    if (row_cache) HIP_TRY(launch_rowcache_prep(secs, n, lp, stream, kt));
    for (int64_t t = 0; t < iters; ++t) {
        bool spec = false;
        if (lp.spectral)
            for (int i = 0; i < n && !spec; ++i) {
                const int64_t R = r0[i] - t;
                spec = R > stop[i] && R <= lp.kmax;
            }
        const bool fill = !fill_at.empty() && std::binary_search(fill_at.begin(), fill_at.end(), t);
        HIP_TRY(launch_wide_iteration(secs, n, G, lp, variant, spec, row_cache, tu.rows_grid, fill ? fill_tiles : 0,
                                      stream, kt));
    }
    if (tm) HIP_TRY(hipEventRecord(e1, stream));
    return HSWO_OK;
}

// A level's sections one after another (HSWO_FLAG_SEQUENTIAL_SECTIONS), or all together.
int run_level_sections(Timer* tm, const SecDev* secs, int n, const std::vector<int64_t>& cap,
                       const std::vector<int64_t>& stop, const LoopParams& lp, bool row_cache, bool mat_ok,
                       const Tuning& tu, bool sequential, hipStream_t stream) {
    if (!sequential || n == 1) return run_level(tm, secs, n, cap, stop, lp, row_cache, mat_ok, tu, stream);
    for (int i = 0; i < n; ++i) {
        const int r = run_level(tm, secs + i, 1, {cap[i]}, {stop[i]}, lp, row_cache, mat_ok, tu, stream);
        if (r) return r;
    }
    return HSWO_OK;
}

using Seq = std::function<int(hipStream_t, Timer*, const Tuning&)>;

std::mutex g_mu;
std::map<std::string, std::string> g_tune;  // bucket -> Tuning::str()
bool g_tune_loaded = false;
struct GraphEntry {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
};
std::map<std::string, GraphEntry> g_graphs;
std::vector<std::string> g_graph_fifo;
constexpr size_t MAX_GRAPHS = 16;

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("HSWO_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[512], val[128];
    while (fscanf(f, "%511s %127s", key, val) == 2) g_tune[key] = val;
    fclose(f);
}

void tune_store_locked(const std::string& k, const Tuning& t) {
    g_tune[k] = t.str();
    const char* path = getenv("HSWO_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %s\n", k.c_str(), t.str().c_str());
    fclose(f);
}

bool tuning_from_str(const std::string& v, Tuning& t) {
    Tuning x;
    if (sscanf(v.c_str(), "%d,%d,%d,%d,%d,%d,%d", &x.wide_max, &x.wide_wg, &x.rows_grid, &x.hybrid, &x.bare,
               &x.variant, &x.row_matrix) != 7)
        return false;
    t = x;
    return true;
}

int bucket(int64_t x) {
    int b = 0;
    while ((int64_t)1 << b < x) ++b;
    return b;
}

struct ExecOut {
    unsigned long long counters[C_COUNT];
    double ms_total = 0.0, ms_driver = 0.0;
    int64_t driver_launches = 0;
    Tuning tuning;
    double ms_kernel[HSWO_NK] = {};
    int64_t kernel_launches[HSWO_NK] = {};
    double ms_event_pair = 0.0;
};

// What one event pair around a launch adds to the launch's own time on this
// stream: an empty kernel launched between its own event pair, against the
// same kernel launched back to back under one pair.
int event_pair_overhead(hipStream_t stream, double* ms_out) {
    constexpr int N = 64;
    std::vector<hipEvent_t> ev;
    auto cleanup = [&]() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    };
    for (int i = 0; i < 2 * N + 2; ++i) {
        hipEvent_t e = nullptr;
        const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
        if (r != hipSuccess) {
            cleanup();
            return fail(HSWO_E_DEVICE, "hipEventCreateWithFlags: %s", hipGetErrorString(r));
        }
        ev.push_back(e);
    }
    hipError_t r = hipSuccess;
    for (int i = 0; i < N && r == hipSuccess; ++i) {
        r = hipEventRecord(ev[2 * i], stream);
        if (r == hipSuccess) r = launch_empty(stream);
        if (r == hipSuccess) r = hipEventRecord(ev[2 * i + 1], stream);
    }
    if (r == hipSuccess) r = hipEventRecord(ev[2 * N], stream);
    for (int i = 0; i < N && r == hipSuccess; ++i) r = launch_empty(stream);
    if (r == hipSuccess) r = hipEventRecord(ev[2 * N + 1], stream);
    if (r == hipSuccess) r = hipStreamSynchronize(stream);
    double bracketed = 0.0;
    float x = 0.f;
    for (int i = 0; i < N && r == hipSuccess; ++i) {
        r = hipEventElapsedTime(&x, ev[2 * i], ev[2 * i + 1]);
        bracketed += x;
    }
    if (r == hipSuccess) r = hipEventElapsedTime(&x, ev[2 * N], ev[2 * N + 1]);
    cleanup();
    if (r != hipSuccess) return fail(HSWO_E_DEVICE, "event timing: %s", hipGetErrorString(r));
    *ms_out = std::max(0.0, bracketed / N - (double)x / N);
    return HSWO_OK;
}

// Time one run of the sequence with settings t on the call's stream: replayed
// from a graph when the call uses graphs (the launch overhead then matches
// what the tuned call will see), else eager.
int time_trial(const Seq& seq, const Tuning& t, bool graph, hipStream_t stream, float* ms) {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    if (graph) {
        HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        const int rc = seq(stream, nullptr, t);
        const hipError_t ec = hipStreamEndCapture(stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (ec != hipSuccess) return fail(HSWO_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(HSWO_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        }
    }
    int rc = HSWO_OK;
    EventPair ev;
    hipError_t e = hipEventCreate(&ev.a);
    if (e == hipSuccess) e = hipEventCreate(&ev.b);
    if (e == hipSuccess && graph) e = hipGraphLaunch(x, stream);  // first replay uploads the graph
    if (e == hipSuccess) e = hipEventRecord(ev.a, stream);
    if (e == hipSuccess) {
        if (graph) e = hipGraphLaunch(x, stream);
        else rc = seq(stream, nullptr, t);
    }
    if (e == hipSuccess && rc == HSWO_OK) e = hipEventRecord(ev.b, stream);
    if (e == hipSuccess && rc == HSWO_OK) e = hipEventSynchronize(ev.b);
    if (e == hipSuccess && rc == HSWO_OK) e = hipEventElapsedTime(ms, ev.a, ev.b);
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    if (rc) return rc;
    if (e != hipSuccess) return fail(HSWO_E_DEVICE, "autotune trial: %s", hipGetErrorString(e));
    return HSWO_OK;
}

// Candidate values of each setting the autotuner searches (one setting at a
// time, the others held at the best found so far). Every candidate gives the
// same merges and labels.
struct Knob {
    int Tuning::*field;
    std::vector<int> values;
    bool given;
};

std::vector<Knob> tune_knobs(bool incremental, const hswo_tuning* g) {
    const int cu = device_cus();
    std::vector<Knob> k;
    if (incremental) {
        k.push_back({&Tuning::wide_max, {cu, 64, 16, 4, 0}, g && g->wide_max_sections >= 0});
        k.push_back({&Tuning::rows_grid, {2 * cu, cu, 4 * cu}, g && g->rows_grid >= 0});
        k.push_back({&Tuning::row_matrix, {1, 0}, g && g->row_matrix >= 0});
    } else {
        k.push_back({&Tuning::wide_max, {64, 16, 256}, g && g->wide_max_sections >= 0});
        k.push_back({&Tuning::wide_wg, {cu, 2 * cu, 4 * cu}, g && g->wide_groups >= 0});
        k.push_back({&Tuning::variant, {6, 4, 2}, g && g->driver_variant >= 0});
    }
    return k;
}

// noalloc: the call creates no event, graph or tuning trial (rhseg_segment_noalloc); with stats it
// still copies the counters back and synchronises, but reports no device times.
int execute(const std::vector<Upload>& ups, const Seq& seq, const std::string& key, const std::string& tune_key,
            int flags, hipStream_t stream, unsigned long long* d_counters, bool want_stats, const hswo_tuning* given,
            ExecOut& out, bool noalloc = false) {
    if ((flags & HSWO_FLAG_GRAPH) && stream == nullptr)
        return fail(HSWO_E_INVAL, "HSWO_FLAG_GRAPH needs a non-null stream (the null stream cannot be captured)");
    if ((flags & HSWO_FLAG_KERNEL_TIMES) && ((flags & HSWO_FLAG_GRAPH) || !want_stats))
        return fail(HSWO_E_INVAL, "HSWO_FLAG_KERNEL_TIMES needs stats and cannot be combined with HSWO_FLAG_GRAPH");
    for (const Upload& u : ups)
        HIP_TRY(hipMemcpyAsync(u.dst, u.bytes.data(), u.bytes.size(), hipMemcpyHostToDevice, stream));

    // settings: the caller's, else the tuned ones for this bucket, else a tuning run, else the defaults
    const bool incremental = (flags & HSWO_FLAG_INCREMENTAL) != 0;
    Tuning tu = overlay(default_tuning(incremental), given);
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        tune_load_locked();
        auto it = g_tune.find(tune_key);
        Tuning c;
        if (it != g_tune.end() && tuning_from_str(it->second, c)) {
            tu = overlay(c, given);
            have = true;
        }
    }
    if (!have && (flags & HSWO_FLAG_AUTOTUNE)) {
        // coordinate search on this very problem; every candidate writes identical outputs
        const bool graph = (flags & HSWO_FLAG_GRAPH) != 0;
        float best = 0.0f;
        int rc = time_trial(seq, tu, graph, stream, &best);
        if (rc) return rc;
        for (const Knob& kb : tune_knobs(incremental, given)) {
            if (kb.given) continue;
            for (int v : kb.values) {
                if (tu.*kb.field == v) continue;
                Tuning t = tu;
                t.*kb.field = v;
                float ms = 0.0f;
                rc = time_trial(seq, t, graph, stream, &ms);
                if (rc) return rc;
                if (ms < best) {
                    best = ms;
                    tu = t;
                }
            }
        }
        std::lock_guard<std::mutex> lk(g_mu);
        tune_store_locked(tune_key, tu);
    }
    out.tuning = tu;

    Timer tm;
    tm.kernels = (flags & HSWO_FLAG_KERNEL_TIMES) != 0;
    if (tm.kernels) {
        const int rc = event_pair_overhead(stream, &out.ms_event_pair);
        if (rc) return rc;
    }
    EventPair tot;
    const bool timed = want_stats && !noalloc;
    if (timed) {
        HIP_TRY(hipEventCreate(&tot.a));
        HIP_TRY(hipEventCreate(&tot.b));
        HIP_TRY(hipEventRecord(tot.a, stream));
    }
    if (flags & HSWO_FLAG_GRAPH) {
        const std::string gk = key + "|t" + tu.str();
        hipGraphExec_t exec = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = g_graphs.find(gk);
            if (it != g_graphs.end()) exec = it->second.x;
        }
        if (!exec) {
            GraphEntry ge;
            HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            const int rc = seq(stream, nullptr, tu);
            const hipError_t ec = hipStreamEndCapture(stream, &ge.g);
            if (rc) {
                if (ge.g) (void)hipGraphDestroy(ge.g);
                return rc;
            }
            if (ec != hipSuccess) return fail(HSWO_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
            HIP_TRY(hipGraphInstantiate(&ge.x, ge.g, nullptr, nullptr, 0));
            exec = ge.x;
            std::lock_guard<std::mutex> lk(g_mu);
            if (g_graph_fifo.size() >= MAX_GRAPHS) {
                GraphEntry old = g_graphs[g_graph_fifo.front()];
                g_graphs.erase(g_graph_fifo.front());
                g_graph_fifo.erase(g_graph_fifo.begin());
                (void)hipGraphExecDestroy(old.x);
                (void)hipGraphDestroy(old.g);
            }
            g_graphs[gk] = ge;
            g_graph_fifo.push_back(gk);
        }
        HIP_TRY(hipGraphLaunch(exec, stream));
    } else {
        const int rc = seq(stream, timed ? &tm : nullptr, tu);
        if (rc) return rc;
    }
    if (want_stats && !timed) {
        HIP_TRY(hipMemcpyAsync(out.counters, d_counters, sizeof(out.counters), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
    } else if (want_stats) {
        HIP_TRY(hipEventRecord(tot.b, stream));
        HIP_TRY(hipMemcpyAsync(out.counters, d_counters, sizeof(out.counters), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, tot.a, tot.b));
        out.ms_total = ms;
        double md = 0.0;
        for (size_t k = 0; k + 1 < tm.drv.size(); k += 2) {
            float x = 0.f;
            HIP_TRY(hipEventElapsedTime(&x, tm.drv[k], tm.drv[k + 1]));
            md += x;
        }
        out.driver_launches = (int64_t)(tm.drv.size() / 2);
        for (int k = 0; k < HSWO_NK; ++k) {
            const std::vector<hipEvent_t>& v = tm.kt.ev[k];
            double t = 0.0;
            for (size_t i = 0; i + 1 < v.size(); i += 2) {
                float x = 0.f;
                HIP_TRY(hipEventElapsedTime(&x, v[i], v[i + 1]));
                t += x;
            }
            out.ms_kernel[k] = t;
            out.kernel_launches[k] = (int64_t)(v.size() / 2);
        }
        // under a graph the launches are not bracketed individually
        out.ms_driver = tm.drv.empty() ? ms : md;
    }
    return HSWO_OK;
}

int fill_stats(hswo_stats* st, const ExecOut& o, int64_t launches_if_graph) {
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const double tick_ms = khz > 0 ? 1.0 / (double)khz : 1e-5;  // device constant clock
    const unsigned long long* c = o.counters;
    st->merges = (int64_t)c[C_MERGES];
    st->iterations = (int64_t)c[C_ITERS];
    st->adjacent_pairs = (int64_t)c[C_ADJ_PAIRS];
    st->spectral_pairs = (int64_t)c[C_SPEC_PAIRS];
    st->exact_rechecks = (int64_t)c[C_RECHECKS];
    st->tile_rescans = (int64_t)c[C_RESCANS];
    st->fp32_tiles = (int64_t)c[C_FP32_TILES];
    st->mfma_tiles = (int64_t)c[C_MFMA_TILES];
    st->driver_launches = o.driver_launches ? o.driver_launches : launches_if_graph;
    st->driver_variant = o.tuning.variant;
    st->ms_total = o.ms_total;
    st->ms_driver = o.ms_driver;
    st->ms_adjacent = (double)c[C_T_ADJ] * tick_ms;
    st->ms_mfma_screen = (double)c[C_T_MFMA] * tick_ms;
    st->ms_fp32_spectral = (double)c[C_T_SPEC32] * tick_ms;
    st->ms_merge = (double)c[C_T_MERGE] * tick_ms;
    for (int k = 0; k < HSWO_NK; ++k) {
        st->ms_kernel[k] = o.ms_kernel[k];
        st->kernel_launches[k] = o.kernel_launches[k];
        st->kernel_work[k] = 0;
    }
    st->kernel_work[HSWO_K_WIDE_DECIDE] = (int64_t)c[C_W_DECIDE_BYTES];
    st->kernel_work[HSWO_K_WIDE_ROWS] = (int64_t)c[C_W_ROWS_BYTES];
    st->kernel_work[HSWO_K_MATRIX_FILL] = (int64_t)c[C_W_FILL_FLOPS];
    st->kernel_work[HSWO_K_WIDE_ADJ] = (int64_t)c[C_W_ADJ_BYTES];
    st->kernel_work[HSWO_K_WIDE_MFMA] = (int64_t)c[C_W_MFMA_FLOPS];
    st->kernel_work[HSWO_K_SECTION_DRIVER] = (int64_t)c[C_D_BYTES];
    st->ms_event_pair_overhead = o.ms_event_pair;
    st->nonfinite_values = (int64_t)c[C_NONFINITE];
    st->screen_iterations = (int64_t)c[C_SCREEN_ITERS];
    st->screen_fallbacks = (int64_t)c[C_SCREEN_FALLBACKS];
    st->verify_records = (int64_t)c[C_VERIFY];
    st->row_bounded_pairs = (int64_t)c[C_ROW_BOUNDED];
    st->tuning.row_matrix = o.tuning.row_matrix;
    st->reserved = 0;
    st->tuning.wide_max_sections = o.tuning.wide_max;
    st->tuning.wide_groups = o.tuning.wide_wg;
    st->tuning.rows_grid = o.tuning.rows_grid;
    st->tuning.hybrid = o.tuning.hybrid;
    st->tuning.bare_bounds = o.tuning.bare;
    st->tuning.driver_variant = o.tuning.variant;
    if (c[C_NONFINITE])
        return fail(HSWO_E_NONFINITE, "the cube holds %llu NaN or infinite values; nothing was merged",
                    (unsigned long long)c[C_NONFINITE]);
    return HSWO_OK;
}

// The weight enters the key by its bit pattern: a decimal rendering would
// merge nearby weights (w and its neighbouring floats) into one graph.
std::string params_key(const hswo_params* p) {
    uint32_t wbits = 0;
    std::memcpy(&wbits, &p->spclust_wght, sizeof(wbits));
    std::string k = "c" + std::to_string(p->connectivity) + "s" + std::to_string(p->seam_connectivity) + "w" +
                    std::to_string(wbits) + "k" + std::to_string(p->spclust_max) + "t" +
                    std::to_string(p->target_regions) + "S" + std::to_string(p->section_regions) + "L" +
                    std::to_string(p->rnb_levels) + "P" + std::to_string(p->precision) + "C" +
                    std::to_string(p->criterion) + "F" +
                    std::to_string(p->flags) + "K" + std::to_string(p->screen_topk) + "l";
    for (int l = 0; l < p->n_levels; ++l) k += std::to_string(p->level_counts[l]) + ",";
    return k;
}

std::string ptr_key(const void* x) {
    char b[32];
    snprintf(b, sizeof(b), "%p", x);
    return b;
}

LoopParams loop_params(const hswo_params* p, unsigned long long* counters) {
    LoopParams lp;
    lp.w2 = (double)p->spclust_wght * (double)p->spclust_wght;
    lp.spectral = p->spclust_wght > 0.0f && p->spclust_max > 0 ? 1 : 0;
    lp.kmax = p->spclust_max;
    lp.precision = p->precision;
    lp.incremental = (p->flags & HSWO_FLAG_INCREMENTAL) ? 1 : 0;
    lp.phase_stop = 0;
    lp.two_merges = (p->flags & HSWO_FLAG_TWO_MERGES) ? 1 : 0;
    lp.topk = p->screen_topk > 0 ? p->screen_topk : 8;
    lp.row_matrix = 0;  // set per level from the resolved tuning
    lp.multi_merge = (p->flags & HSWO_FLAG_MULTI_MERGE) ? 1 : 0;
    lp.counters = counters;
    return lp;
}

int check_common(const hswo_params* p, void* workspace) {
    if (!workspace) return fail(HSWO_E_INVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(HSWO_E_INVAL, "workspace must be 256-byte aligned");
    if (p->flags & ~(HSWO_FLAG_MERGE_LOG | HSWO_FLAG_GRAPH | HSWO_FLAG_AUTOTUNE | HSWO_FLAG_INCREMENTAL |
                     HSWO_FLAG_KERNEL_TIMES | HSWO_FLAG_SEQUENTIAL_SECTIONS | HSWO_FLAG_TWO_MERGES |
                     HSWO_FLAG_DEBUG_VERIFY_BOUND | HSWO_FLAG_MULTI_MERGE))
        return fail(HSWO_E_INVAL, "unknown flags 0x%x", p->flags);
    return HSWO_OK;
}

// get_scratch non-null: the no-allocation entry point. Everything is validated
// on the host first (the scratch size included); only then is the scratch's
// device address fetched through get_scratch (ws_bytes is its size).
int run_rhseg(const void* cube, int H, int W, int B, int dtype, const hswo_params* p, int L, int32_t* labels,
              hswo_merge_rec* merge_log, hswo_stats* stats, void* workspace, size_t ws_bytes,
              hipStream_t stream, int (*get_scratch)(void**) = nullptr) {
    const bool noalloc = get_scratch != nullptr;
    int rc = validate_shape(H, W, B, dtype);
    if (rc) return rc;
    rc = validate_params(p, L);
    if (rc) return rc;
    if (noalloc && (p->flags & (HSWO_FLAG_GRAPH | HSWO_FLAG_AUTOTUNE | HSWO_FLAG_KERNEL_TIMES)))
        return fail(HSWO_E_INVAL, "rhseg_segment_noalloc takes none of HSWO_FLAG_GRAPH, HSWO_FLAG_AUTOTUNE and "
                                  "HSWO_FLAG_KERNEL_TIMES (each creates graphs or events)");
    if (!cube || !labels) return fail(HSWO_E_INVAL, "cube and labels must be device pointers");
    if (reinterpret_cast<uintptr_t>(cube) % 16) return fail(HSWO_E_INVAL, "cube must be 16-byte aligned");
    if ((H >> (L - 1)) < 1 || (W >> (L - 1)) < 1)
        return fail(HSWO_E_INVAL, "rnb_levels=%d leaves empty sections for %dx%d", L, H, W);
    if ((p->flags & HSWO_FLAG_MERGE_LOG) && !merge_log) return fail(HSWO_E_INVAL, "MERGE_LOG flag needs merge_log");
    rc = check_common(p, noalloc ? reinterpret_cast<void*>(256) : workspace);
    if (rc) return rc;
    if (!(p->flags & HSWO_FLAG_MERGE_LOG)) merge_log = nullptr;

    const Plan pl = make_plan(H, W, B, p, L);
    rc = check_plan(pl);
    if (rc) return rc;
    const int bare = overlay(default_tuning(false), p->tuning).bare;
    if (noalloc) {
        const size_t need = carve(pl, H, W, p, bare, nullptr, cube, labels, merge_log).bytes;
        if (need > ws_bytes)
            return fail(HSWO_E_NOMEM,
                        "this call needs %zu bytes of scratch; rhseg_segment_noalloc has a fixed %zu "
                        "(HSWO_NOALLOC_SCRATCH_BYTES): call rhseg_segment with a workspace instead",
                        need, ws_bytes);
        rc = get_scratch(&workspace);
        if (rc) return rc;
    }
    Layout lay = carve(pl, H, W, p, bare, workspace, cube, labels, merge_log);
    if (ws_bytes < lay.bytes)
        return fail(HSWO_E_NOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, lay.bytes);

    const int64_t P = (int64_t)H * W;
    std::vector<Upload> ups;
    add_upload(ups, lay.counts, p->level_counts, p->n_levels);
    for (int d = 0; d < L; ++d) {
        const LevelDev& lv = lay.lv[d];
        add_upload(ups, lv.secs, lv.h_secs.data(), lv.h_secs.size());
        if (!lv.h_asms.empty()) add_upload(ups, lv.asms, lv.h_asms.data(), lv.h_asms.size());
        if (!lv.h_inits.empty()) add_upload(ups, lv.inits, lv.h_inits.data(), lv.h_inits.size());
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
    add_upload(ups, lay.snap, &sd, 1);
    const LoopParams lp = loop_params(p, lay.counters);
    const bool row_cache = row_cache_on(p);
    const bool sequential = (p->flags & HSWO_FLAG_SEQUENTIAL_SECTIONS) != 0;
    std::vector<std::vector<int64_t>> caps(L), stops(L);
    std::vector<char> mat_ok(L, 0);  // every section of the level keeps an interval matrix (carve's rule)
    for (int d = 0; d < L; ++d) {
        bool ok = row_cache && p->criterion == HSWO_CRIT_BSMSE && !(p->flags & HSWO_FLAG_TWO_MERGES);
        for (const SecPlan& s : pl.lv[d]) {
            caps[d].push_back(s.cap);
            stops[d].push_back(s.stop);
            ok = ok && std::min<int64_t>(s.cap, p->spclust_max) <= MAT_MAX;
        }
        mat_ok[d] = ok ? 1 : 0;
    }

    const Seq seq = [&](hipStream_t st, Timer* tm, const Tuning& tu) -> int {
        HIP_TRY(launch_fill_u64(lay.counters, C_COUNT, 0ull, st));
        HIP_TRY(launch_init_pixels(lay.parent, lay.mtime, P, st));
        {
            const int d = L - 1;
            int maxpix = 0;
            for (const SecPlan& s : pl.lv[d]) maxpix = std::max<int>(maxpix, (int)s.cap);
            HIP_TRY(launch_init_leaves(lay.lv[d].secs, lay.lv[d].inits, (int)pl.lv[d].size(), dtype, maxpix,
                                         lay.counters, st));
            const int r = run_level_sections(tm, lay.lv[d].secs, (int)pl.lv[d].size(), caps[d], stops[d], lp,
                                             row_cache, mat_ok[d] != 0, tu, sequential, st);
            if (r) return r;
        }
        for (int d = L - 2; d >= 0; --d) {
            const auto& secs = pl.lv[d];
            int64_t maxcap = 0, maxseam = 0;
            for (size_t i = 0; i < secs.size(); ++i) {
                const SecPlan& s = secs[i];
                maxcap = std::max(maxcap, std::max(s.cap, s.ecap));
                maxseam = std::max(maxseam, (int64_t)(s.rect.w + 2 * s.rect.h));
                HIP_TRY(launch_fill_u64(lay.lv[d].h_asms[i].hash, (size_t)s.hash_cap, ~0ull, st));
            }
            HIP_TRY(launch_compress(lay.parent, P, lay.counters, st));
            HIP_TRY(launch_assemble(lay.lv[d].secs, lay.lv[d + 1].secs, lay.lv[d].asms, (int)secs.size(), lay.slotmap,
                                    (int)std::min<int64_t>(maxcap, 1 << 30), lay.counters, st));
            HIP_TRY(launch_seam(lay.lv[d].secs, lay.lv[d].asms, (int)secs.size(), lay.slotmap, (int)maxseam,
                                lay.counters, st));
            const int r = run_level_sections(tm, lay.lv[d].secs, (int)secs.size(), caps[d], stops[d], lp, row_cache,
                                             mat_ok[d] != 0, tu, sequential, st);
            if (r) return r;
        }
        HIP_TRY(launch_snapshot(lay.snap, 1, lay.counts, p->n_levels, (int)P, lay.counters, st));
        return HSWO_OK;
    };

    const std::string key = "rhseg|" + ptr_key(cube) + ptr_key(labels) + ptr_key(merge_log) + ptr_key(workspace) +
                            "|" + std::to_string(H) + "x" + std::to_string(W) + "x" + std::to_string(B) + "d" +
                            std::to_string(dtype) + "|" + params_key(p) + ptr_key(p->verify) +
                            std::to_string(p->verify_cap);
    int64_t maxcap = 0;
    for (const auto& lv : pl.lv)
        for (const SecPlan& s : lv) maxcap = std::max(maxcap, s.cap);
    const std::string tkey = "gfx950:rhseg:B" + std::to_string(bucket(B)) + ":R" + std::to_string(bucket(maxcap)) +
                             ":n" + std::to_string(bucket((int64_t)pl.lv[L - 1].size())) + ":P" +
                             std::to_string(p->precision) + ":C" + std::to_string(p->criterion) + ":k" +
                             std::to_string(bucket(p->spclust_max + 1)) + ":I" +
                             std::to_string((p->flags & HSWO_FLAG_INCREMENTAL) ? 1 : 0);
    ExecOut eo;
    rc = execute(ups, seq, key, tkey, p->flags, stream, lay.counters, stats != nullptr, p->tuning, eo, noalloc);
    if (rc) return rc;
    if (stats) return fill_stats(stats, eo, L);
    return HSWO_OK;
}

// ---------------------------------------------------------------------------
// Batch of independent sections (each its own top pass), one persistent launch.
// ---------------------------------------------------------------------------
struct BatchLayout {
    unsigned long long* counters = nullptr;
    int32_t* counts = nullptr;
    SecDev* secs = nullptr;      // section order
    SecDev* secs_lpt = nullptr;  // longest-first order for the driver
    InitDev* inits = nullptr;
    SnapDev* snaps = nullptr;
    std::vector<SecDev> h_secs, h_lpt;
    std::vector<InitDev> h_inits;
    std::vector<SnapDev> h_snaps;
    int max_pixels = 0;
    int64_t max_cap = 0;
    int max_B = 0;
    size_t bytes = 0;
};

BatchLayout carve_batch(int n, const hswo_section* sec, const hswo_params* p, int bare, void* ws) {
    BatchLayout lay;
    Bump bp;
    bp.base = reinterpret_cast<char*>(ws);
    lay.counters = bp.take<unsigned long long>(C_COUNT);
    lay.counts = bp.take<int32_t>(p->n_levels);
    lay.secs = bp.take<SecDev>(n);
    lay.secs_lpt = bp.take<SecDev>(n);
    lay.inits = bp.take<InitDev>(n);
    lay.snaps = bp.take<SnapDev>(n);
    lay.h_secs.resize(n);
    lay.h_inits.resize(n);
    lay.h_snaps.resize(n);
    std::vector<double> work(n);
    for (int i = 0; i < n; ++i) {
        const hswo_section& q = sec[i];
        const int64_t cap = (int64_t)q.H * q.W;
        const int Bp = round_up(q.B, BK);
        const int64_t ecap = std::max<int64_t>(1, grid_edges(q.H, q.W, p->connectivity));
        const int64_t tiles = tiles_for(cap, p);
        SecDev& s = lay.h_secs[i];
        std::memset(&s, 0, sizeof(s));
        s.R0 = (int32_t)cap;
        s.B = q.B;
        s.Bp = Bp;
        s.Ecap = (int32_t)ecap;
        s.stop = p->target_regions;
        s.top = 1;
        s.log_base = 0;
        s.tiles = (int32_t)tiles;
        s.crit = p->criterion;
        s.bare = bare;
        s.label = bp.take<int32_t>(cap);
        s.npix = bp.take<int32_t>(cap);
        s.mark = bp.take<int32_t>(cap);
        s.dmark = bp.take<int32_t>(cap);
        s.norm = bp.take<float>(cap);
        s.sums = bp.take<double>(cap * q.B);
        s.mean = bp.take<float>(cap * Bp);
        s.edges = bp.take<int2>(ecap);
        s.escr = bp.take<float2>(ecap);
        if (p->flags & HSWO_FLAG_INCREMENTAL) {
            s.ed2 = bp.take<double>(ecap);
            s.edirty = bp.take<int32_t>(ecap);
            s.rmin = bp.take<int32_t>(cap);
            s.rmax = bp.take<int32_t>(cap);
            s.cmd2 = bp.take<double>((ecap + ECH - 1) / ECH);
            s.cme = bp.take<int2>((ecap + ECH - 1) / ECH);
            s.cml = bp.take<int2>((ecap + ECH - 1) / ECH);
            if (p->flags & HSWO_FLAG_MULTI_MERGE) take_multi(bp, s, cap, ecap);
        }
        s.tstat = bp.take<float2>(tiles);
        s.tflag = bp.take<int32_t>(tiles);
        if (row_cache_on(p)) {
            const int64_t rc = std::min<int64_t>(cap, p->spclust_max);
            s.rcap = (int32_t)rc;
            s.m64 = bp.take<double>(rc * q.B);
            s.m64r = bp.take<double>(rc * (((int64_t)q.B + 7) / 8 * 8));
            if (p->criterion == HSWO_CRIT_SAM) s.rq = bp.take<double>(rc);
            // (the batch runs its sections in the persistent driver: no interval matrix)
            if (p->flags & HSWO_FLAG_TWO_MERGES) s.abit = bp.take<uint32_t>(rc * ((rc + 31) / 32));
            s.rbd = bp.take<double>(rc);
            s.rbp = bp.take<int32_t>(rc);
            s.rbl = bp.take<int32_t>(rc);
            s.rbd2 = bp.take<double>(rc);
            s.rbp2 = bp.take<int32_t>(rc);
            s.rbl2 = bp.take<int32_t>(rc);
            s.rpend = bp.take<int32_t>(rc);
            s.rpart = bp.take<RowPart>(rc * ((rc + 63) / 64));
        } else if (p->precision != HSWO_PREC_FP32 && p->spclust_wght > 0.0f && p->spclust_max > 0) {
            const int64_t kc = std::min<int64_t>(cap, p->spclust_max);
            s.kcap = (int32_t)kc;
            s.g16 = bp.take<uint16_t>(kc * Bp);
            s.gn = bp.take<float>(kc);
            s.geta = bp.take<float>(kc);
            s.galpha = bp.take<float>(kc);
            s.gP = bp.take<float>(kc);
            s.cvec = bp.take<float>(Bp);
        }
        s.st = bp.take<int32_t>(ST_WORDS);
        s.wi = bp.take<int32_t>(16);
        s.wd = bp.take<double>(4);
        s.wpart = bp.take<float>(2 * GMAX);
        if (p->flags & HSWO_FLAG_DEBUG_VERIFY_BOUND) {
            s.vraw = bp.take<float>(ecap);
            s.vstage = bp.take<float>(CAND_CAP);
            s.vout = p->verify;
            s.vcap = p->verify_cap;
            s.vcount = lay.counters ? lay.counters + C_VERIFY : nullptr;
        }
        s.parent = bp.take<int32_t>(cap);
        s.mtime = bp.take<int32_t>(cap);
        s.log = (p->flags & HSWO_FLAG_MERGE_LOG) ? q.merge_log : nullptr;
        InitDev& in = lay.h_inits[i];
        in.cube = q.cube;
        in.img_w = q.W;
        in.r0 = 0;
        in.c0 = 0;
        in.h = q.H;
        in.w = q.W;
        in.label_w = q.W;
        in.conn = p->connectivity;
        SnapDev& sd = lay.h_snaps[i];
        sd.st = s.st;
        sd.parent = s.parent;
        sd.mtime = s.mtime;
        sd.labels = q.labels;
        sd.img_w = q.W;
        sd.r0 = 0;
        sd.c0 = 0;
        sd.h = q.H;
        sd.w = q.W;
        sd.label_w = q.W;
        lay.max_pixels = std::max<int>(lay.max_pixels, (int)cap);
        lay.max_cap = std::max(lay.max_cap, cap);
        lay.max_B = std::max(lay.max_B, q.B);
        // expected work: the adjacent sweep over the whole pass (~ cap^2 / 2 rows)
        work[i] = (double)cap * (double)cap * (double)Bp;
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    lay.h_lpt.resize(n);
    for (int i = 0; i < n; ++i) lay.h_lpt[i] = lay.h_secs[order[i]];
    lay.bytes = bp.off + 256;
    return lay;
}

int validate_batch(int n, const hswo_section* sec, int dtype, const hswo_params* p) {
    if (n < 1 || !sec) return fail(HSWO_E_INVAL, "need n_sections >= 1 and a sections array");
    int rc = validate_params(p, 1);
    if (rc) return rc;
    if (dtype != HSWO_F32 && dtype != HSWO_F16) return fail(HSWO_E_INVAL, "dtype must be HSWO_F32 or HSWO_F16");
    for (int i = 0; i < n; ++i) {
        const hswo_section& q = sec[i];
        rc = validate_shape(q.H, q.W, q.B, dtype);
        if (rc) return fail(rc, "section %d: %s", i, g_err.c_str());
        if (!q.cube || !q.labels) return fail(HSWO_E_INVAL, "section %d: cube and labels must be device pointers", i);
        if (reinterpret_cast<uintptr_t>(q.cube) % 16) return fail(HSWO_E_INVAL, "section %d: cube not 16-byte aligned", i);
        if ((p->flags & HSWO_FLAG_MERGE_LOG) && !q.merge_log)
            return fail(HSWO_E_INVAL, "section %d: MERGE_LOG flag needs merge_log", i);
        if (grid_edges(q.H, q.W, p->connectivity) > ((int64_t)1 << 30))
            return fail(HSWO_E_UNSUPPORTED, "section %d: %dx%d needs more than 2^30 edge slots (int32 indices)", i,
                        q.H, q.W);
    }
    return HSWO_OK;
}

int run_batch(int n, const hswo_section* sec, int dtype, const hswo_params* p, hswo_stats* stats, void* workspace,
              size_t ws_bytes, hipStream_t stream) {
    int rc = validate_batch(n, sec, dtype, p);
    if (rc) return rc;
    rc = check_common(p, workspace);
    if (rc) return rc;
    BatchLayout lay = carve_batch(n, sec, p, overlay(default_tuning(false), p->tuning).bare, workspace);
    if (ws_bytes < lay.bytes)
        return fail(HSWO_E_NOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, lay.bytes);
    std::vector<Upload> ups;
    add_upload(ups, lay.counts, p->level_counts, p->n_levels);
    add_upload(ups, lay.secs, lay.h_secs.data(), n);
    add_upload(ups, lay.secs_lpt, lay.h_lpt.data(), n);
    add_upload(ups, lay.inits, lay.h_inits.data(), n);
    add_upload(ups, lay.snaps, lay.h_snaps.data(), n);
    const LoopParams lp = loop_params(p, lay.counters);
    const Seq seq = [&](hipStream_t st, Timer* tm, const Tuning& tu) -> int {
        HIP_TRY(launch_fill_u64(lay.counters, C_COUNT, 0ull, st));
        HIP_TRY(launch_init_pixels_secs(lay.secs, n, lay.max_pixels, st));
        HIP_TRY(launch_init_leaves(lay.secs, lay.inits, n, dtype, lay.max_pixels, lay.counters, st));
        int r = HSWO_OK;
        if (p->flags & HSWO_FLAG_SEQUENTIAL_SECTIONS) {
            for (int i = 0; i < n && !r; ++i)
                r = run_level(tm, lay.secs + i, 1, {lay.h_secs[i].R0}, {lay.h_secs[i].stop}, lp, row_cache_on(p),
                              false, tu, st);
        } else {
            r = timed_driver(tm, lay.secs_lpt, n, lp, tu.variant, st);
        }
        if (r) return r;
        HIP_TRY(launch_snapshot(lay.snaps, n, lay.counts, p->n_levels, lay.max_pixels, lay.counters, st));
        return HSWO_OK;
    };
    std::string key = "batch|" + std::to_string(n) + "|" + ptr_key(workspace) + "d" + std::to_string(dtype) + "|" +
                      params_key(p) + ptr_key(p->verify) + std::to_string(p->verify_cap) + "|";
    for (int i = 0; i < n; ++i)
        key += ptr_key(sec[i].cube) + ptr_key(sec[i].labels) + ptr_key(sec[i].merge_log) + std::to_string(sec[i].H) +
               "x" + std::to_string(sec[i].W) + "x" + std::to_string(sec[i].B) + ";";
    const std::string tkey = "gfx950:batch:B" + std::to_string(bucket(lay.max_B)) + ":R" +
                             std::to_string(bucket(lay.max_cap)) + ":n" + std::to_string(bucket(n)) + ":P" +
                             std::to_string(p->precision) + ":C" + std::to_string(p->criterion) + ":k" +
                             std::to_string(bucket(p->spclust_max + 1)) + ":I" +
                             std::to_string((p->flags & HSWO_FLAG_INCREMENTAL) ? 1 : 0);
    ExecOut eo;
    rc = execute(ups, seq, key, tkey, p->flags, stream, lay.counters, stats != nullptr, p->tuning, eo);
    if (rc) return rc;
    if (stats) return fill_stats(stats, eo, 1);
    return HSWO_OK;
}

}  // namespace

namespace hswo {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

void clear_error() { g_err.clear(); }

int rhseg_in_scratch(const void* cube, int H, int W, int B, int dtype, const hswo_params* p, int L,
                     int32_t* labels, hswo_merge_rec* merge_log, hswo_stats* stats, int (*get_scratch)(void**),
                     size_t scratch_bytes, hipStream_t stream) {
    return run_rhseg(cube, H, W, B, dtype, p, L, labels, merge_log, stats, nullptr, scratch_bytes, stream,
                     get_scratch);
}

}  // namespace hswo

extern "C" {

int hswo_version(void) { return HSWO_VERSION; }

const char* hswo_last_error(void) { return g_err.c_str(); }

size_t hswo_workspace_bytes(int32_t H, int32_t W, int32_t B, int32_t dtype, const hswo_params* p) {
    if (validate_shape(H, W, B, dtype) || validate_params(p, 0)) return 0;
    const int L = p->rnb_levels;
    if ((H >> (L - 1)) < 1 || (W >> (L - 1)) < 1) return 0;
    const Plan pl = make_plan(H, W, B, p, L);
    if (check_plan(pl)) return 0;
    return carve(pl, H, W, p, 1, nullptr, nullptr, nullptr, nullptr).bytes;
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
    if (validate_batch(n_sections, sections, dtype, p)) return 0;
    return carve_batch(n_sections, sections, p, 1, nullptr).bytes;
}

int hswo_run_batch(int32_t n_sections, const hswo_section* sections, int32_t dtype, const hswo_params* p,
                   hswo_stats* stats, void* workspace, size_t ws_bytes, void* hip_stream) {
    g_err.clear();
    return run_batch(n_sections, sections, dtype, p, stats, workspace, ws_bytes,
                     reinterpret_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
