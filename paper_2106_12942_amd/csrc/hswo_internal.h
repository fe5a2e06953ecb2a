// hswo_internal.h -- device-side descriptors shared by the host runtime
// (hswo_api.cpp) and the kernels (hswo_driver.hip, hswo_wide.hip,
// hswo_levels.hip and the dev_*.h device headers). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include <cstddef>
#include <cstdint>

#include "hswo.h"

namespace hswo {

constexpr int NT = 512;          // threads per section-driver workgroup (8 wave64)
constexpr int NWAVE = NT / 64;
constexpr int TILE = 64;         // spectral tile edge (pairs TILE x TILE)
constexpr int BK = 32;           // band chunk staged in LDS; mean rows padded to a multiple
constexpr int CAND_CAP = 10240;  // candidate list capacity (LDS)
constexpr int MAX_B = 4096;

// counters accumulated per call (device, u64)
enum Counter {
    C_MERGES = 0,
    C_ITERS,
    C_ADJ_PAIRS,
    C_SPEC_PAIRS,
    C_RECHECKS,
    C_RESCANS,
    C_FP32_TILES,   // spectral tiles screened in FP32 (all of them on the plain path)
    C_MFMA_TILES,   // 128 x 128 super tiles screened on matrix cores
    C_T_ADJ,        // 100 MHz ticks in the adjacent stage (screen + exact), summed over sections
    C_T_MFMA,       // ... matrix-core screen (row build, row terms, tiles)
    C_T_SPEC32,     // ... FP32 spectral tiles + exact re-check
    C_T_MERGE,      // ... merge
    C_W_DECIDE_BYTES, // k_wide_decide, incremental form: algorithmic bytes (see hswo_stats.kernel_work)
    C_W_ROWS_BYTES,   // k_wide_rows: algorithmic bytes (see hswo_stats.kernel_work)
    C_W_ADJ_BYTES,    // k_wide_adj: FP32 mean rows read once + edge endpoints + counts and norms
    C_W_MFMA_FLOPS,   // k_wide_mfma: 2 flops per band per unique pair of the screened sections
    C_D_BYTES,        // k_section_driver, incremental form: algorithmic bytes (see hswo_stats.kernel_work)
    C_NONFINITE,      // non-finite cube values found at initialisation; every later kernel of the call
                      // does nothing when this is non-zero, so no output is written
    C_SCREEN_ITERS,   // screened decisions (adjacent and spectral stages counted separately)
    C_SCREEN_FALLBACKS, // ... whose re-check set held more than screen_topk pairs
    C_VERIFY,         // HSWO_FLAG_DEBUG_VERIFY_BOUND records produced
    C_ROW_BOUNDED,    // row-cache pairs rescanned from the interval matrix
    C_W_FILL_FLOPS,   // k_mat_fill: 3 FP32 flops per band per pair bounded
    C_COUNT
};

constexpr int ST_WORDS = 16;  // per-section state words
constexpr int MAT_MAX = 4096; // largest row cache that keeps the interval matrix (128 MiB per section)
constexpr int ECH = 256;      // edge slots per chunk of the incremental form's per-chunk minima
constexpr int EIDX_MIN = 8192; // wide mode: edge lists at least this long go through the edge index in a merge
constexpr int GMAX = 256;     // wide mode: most workgroups per section
constexpr int STILE = 128;    // matrix-core super tile edge (4 spectral tiles)

// Partial result of a row-cache task: the least and second least candidates
// of one row over a range of columns (64, then the whole row).
struct RowPart {
    double d2;
    int32_t lab;   // partner label (orders equal D2 for a fixed row)
    int32_t slot;  // partner slot (-1: none)
    double d2b;    // the second least candidate
    int32_t labb;
    int32_t slotb;
};

// One section of one recursion level (or one independent batch section).
struct SecDev {
    int32_t R0;      // slot capacity (regions at the start of the pass, upper bound)
    int32_t B;       // bands
    int32_t Bp;      // float row stride: B rounded up to a multiple of BK
    int32_t Ecap;    // edge capacity
    int32_t stop;    // stop count of this pass
    int32_t top;     // 1: top pass (merge times recorded for the level snapshots)
    int32_t log_base;// index of this section's first merge record
    int32_t tiles;   // capacity of tstat (spectral tiles)
    int32_t* label;  // [R0] region label (smallest pixel index of the region)
    int32_t* npix;   // [R0] pixel count
    double* sums;    // [R0][B] FP64 band sums
    float* mean;     // [R0][Bp] FP32 mean spectrum (screen copy), zero padded
    float* norm;     // [R0] upper bound of the L2 norm of the FP32 mean row
    int32_t* mark;   // [R0] per-iteration marks for edge de-duplication
    int32_t* dmark;  // [R0] incremental merge: least edge slot per neighbour of the merged pair
    int2* edges;     // [Ecap] adjacent slot pairs
    float2* escr;    // [Ecap] per-edge screen bounds (lower, upper)
    float2* tstat;   // [tiles] per-tile bounds (min lower, min upper)
    int32_t* tflag;  // [tiles] matrix-core screen: tile may hold a pair below the threshold
    // 16-bit screen rows (precision forms only), slots [0, kcap):
    uint16_t* g16;   // [kcap][Bp] round16(mean - c), zero padded
    float* gn;       // [kcap] sum of squares of the 16-bit row (FP32, from an FP64 sum)
    float* geta;     // [kcap] bound on || g16 row - (true mean - c) ||_2
    float* galpha;   // [kcap] per-iteration sqrt(T / n) + eta
    float* gP;       // [kcap] per-iteration (1 - kappa) * gn - alpha^2
    float* cvec;     // [Bp] centring spectrum, fixed when the spectral stage starts
    int32_t kcap;    // rows available for the 16-bit screen (0 on the plain path)
    int32_t rcap;    // rows of the spectral row cache (0 when it is off)
    int32_t crit;    // HSWO_CRIT_* dissimilarity criterion
    int32_t bare;    // row cache: second bounds kept bare when their partner merges -- 0 none, 1 those of
                     // value 0, 2 all (result-neutral; more light steps, more of them fall back)
    // incremental adjacent stage: exact D2 per edge slot and the edges to refresh
    double* ed2;     // [Ecap]
    int32_t* edirty; // [Ecap]
    // its edge index: per live slot the range of edge slots that can touch it, per chunk of ECH
    // edge slots the least cached key (value, edge slot or -1); valid while st[12] = 1
    int32_t* rmin;   // [R0]
    int32_t* rmax;   // [R0]
    double* cmd2;    // [ceil(Ecap / ECH)]
    int2* cme;       // [ceil(Ecap / ECH)] the slots of that key's pair, the lower label's first; x = -1: none
    int2* cml;       // [ceil(Ecap / ECH)] the labels (lo, hi) of that key
    // spectral row cache (incremental form), slots [0, rcap):
    double* m64;     // [B][rcap] FP64 mean spectra S/n (spectral angle: the sums S), band-major
                     //           (column j = slot j); not kept with the interval matrix, which has no
                     //           exact row tasks
    double* m64r;    // [rcap][B8] the same rows slot-major, B8 = B rounded up to 8
    float2* dmat;    // [rcap][rcap] Equation 1, one-merge reading, rcap <= MAT_MAX: FP32 bounds on every
                     //   pair's value, kept by Ward's update at each merge (used in wide mode); its rows
                     //   and columns are indexed by msl, not by slot
    int32_t* msl;    // [rcap] matrix row of each live slot (the identity when the cache starts)
    int32_t mstride; // entries between matrix rows: rcap rounded up to an odd multiple of 16 (128 bytes),
                     // so the entries of a column fall on different memory channels
    double* rq;      // [rcap] spectral angle only: |S|^2 of each slot (pairwise tree over the bands)
    uint32_t* abit;  // [rcap][ceil(rcap / 32)] two-merge reading only: adjacency bitmap of the live slots
    double* rbd;     // [rcap] exact D2 of the row's cached pair
    int32_t* rbp;    // [rcap] partner slot of that pair (-1: none or pending, -2: light step pending)
    int32_t* rbl;    // [rcap] partner label of that pair
    double* rbd2;    // [rcap] second bound: the least D2 over the row's other partners at its last full
                     //        evaluation (valid while rbp2 >= 0, i.e. while that partner is alive)
    int32_t* rbp2;   // [rcap] partner slot of the second bound (-1: none, -3: a bound of value 0 whose
                     //        partner has merged since; it still bounds the row's other pairs)
    int32_t* rbl2;   // [rcap] its partner label
    int32_t* rpend;  // [rcap] rows to re-evaluate: [0] the last merge's survivor, then stale rows
    RowPart* rpart;  // [rcap][ceil(rcap / 64)] per-row, per-64-column least two candidates
    // several merges per step (HSWO_FLAG_MULTI_MERGE, persistent driver): a step's zero-valued pairs
    unsigned long long* zkey;  // [zcap] sort keys (labels, or a mean-row hash and a label)
    unsigned long long* zval;  // [zcap] what goes with each key (slots)
    int32_t* zuse;   // [R0] per slot: taken by the step, then its place in the step's list (-1: none)
    int4* zlist;     // [R0 / 2 + 1] the step's pairs in merge order: slot of lo, slot of hi, kind
    int32_t zcap;    // a power of two >= max(Ecap, R0)
    // wide mode iteration scratch
    int32_t* wi;     // [16]
    double* wd;      // [4]
    float* wpart;    // [2 * GMAX]
    int32_t* st;     // state: [0] R, [1] E, [2] R at pass start, [3] merges done, [4] 16-bit rows ready,
                     //        [5] per-edge exact D2 cache valid,
                     //        [6] row cache: 0 off, 1 means ready (every row pending), 2 valid,
                     //        [7] pending rows of the row cache,
                     //        [8] incremental form: next adjacent minimum cached (wd[2], wi[8..11]),
                     //        [9] empty edge slots left by incremental merges,
                     //        [10] two-merge reading: step 3 due (threshold in wd[3]),
                     //        [11] rows appended to the pending list by failed light steps,
                     //        [12] incremental form: edge index (slot ranges, chunk minima) valid
    int32_t* parent; // label-indexed union-find parent (image or batch section)
    int32_t* mtime;  // label-indexed merge time: -1 non-top merge, k top merge, INT_MAX alive
    hswo_merge_rec* log;  // section merge log base (may be null)
    // HSWO_FLAG_DEBUG_VERIFY_BOUND only (null otherwise): the FP32 sum of squares of each edge's
    // adjacent screen, the FP32 sum of each spectral candidate in the LDS list, and the output
    float* vraw;     // [Ecap]
    float* vstage;   // [CAND_CAP]
    hswo_verify_rec* vout;
    int64_t vcap;
    unsigned long long* vcount;  // records produced (counters[C_VERIFY])
};

// Leaf initialisation: where a section's pixels come from.
struct InitDev {
    const void* cube;  // image (rhseg) or section cube (batch)
    int32_t img_w;     // row length of the cube in pixels
    int32_t r0, c0, h, w;  // section rectangle inside the cube
    int32_t label_w;   // labels are (r0+r)*label_w + (c0+c)
    int32_t conn;      // 4 or 8
};

// Reassembly of four children into a parent section.
struct AsmDev {
    int32_t child0;    // index of the first of the four children in the child level's SecDev array
    int32_t r0, c0, h, w;  // parent rectangle (image coordinates)
    int32_t img_w;
    int32_t seam_conn;
    int32_t hash_cap;  // power of two
    unsigned long long* hash;
};

// Label snapshot of one top pass.
struct SnapDev {
    const int32_t* st;     // top section state (R at pass start in st[2])
    const int32_t* parent;
    const int32_t* mtime;
    int32_t* labels;       // [n_levels][H][W]
    int32_t img_w;         // width of the parent/mtime index space
    int32_t r0, c0, h, w;  // pixels covered
    int32_t label_w;       // labels are (r0+r)*label_w + (c0+c) in parent/mtime
};

struct LoopParams {
    double w2;        // spclust_wght^2 in FP64
    int32_t spectral; // w > 0
    int32_t kmax;     // spectral stage iff R <= kmax
    int32_t precision;
    int32_t incremental;  // adjacent minimum from cached exact per-edge D2 (only changed edges re-scored)
    int32_t phase_stop;   // section driver: also stop at this region count (0: the pass's stop only)
    int32_t two_merges;   // two-merge reading of the step list (adjacent merge, then non-adjacent merge)
    int32_t topk;         // screened forms: re-check sets larger than this count as fallbacks
    int32_t row_matrix;   // wide mode: keep and rescan the interval matrix (hswo_tuning.row_matrix)
    int32_t multi_merge;  // several merges per step for identical regions (HSWO_FLAG_MULTI_MERGE)
    unsigned long long* counters;  // [C_COUNT]
};

// Per-kernel-kind event pairs (HSWO_FLAG_KERNEL_TIMES), host side.
struct KTimer {
    std::vector<hipEvent_t> ev[HSWO_NK];  // (start, end) of each launch of a kind
    hipError_t pair(int kind, hipEvent_t* a, hipEvent_t* b) {
        // no system-scope fence: the stamps then hold only the launch itself
        hipError_t r = hipEventCreateWithFlags(a, hipEventDisableSystemFence);
        if (r != hipSuccess) return r;
        ev[kind].push_back(*a);
        r = hipEventCreateWithFlags(b, hipEventDisableSystemFence);
        if (r != hipSuccess) return r;
        ev[kind].push_back(*b);
        return hipSuccess;
    }
    ~KTimer() {
        for (auto& v : ev)
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
    }
};

// Launch, bracketed by a pair of events of the given kind (recorded on the
// same stream right before and after it) when per-kernel timing is on.
#define KLAUNCH(kind, kern, grid, block, ...)                                 \
    do {                                                                   \
        hipEvent_t a_ = nullptr, b_ = nullptr;                             \
        if (kt) {                                                          \
            const hipError_t r_ = kt->pair((kind), &a_, &b_);              \
            if (r_ != hipSuccess) return r_;                               \
            const hipError_t q_ = hipEventRecord(a_, s);                   \
            if (q_ != hipSuccess) return q_;                               \
        }                                                                  \
        hipLaunchKernelGGL(kern, grid, block, 0, s, __VA_ARGS__);          \
        if (kt) {                                                          \
            const hipError_t q_ = hipEventRecord(b_, s);                   \
            if (q_ != hipSuccess) return q_;                               \
        }                                                                  \
    } while (0)

// kernel launchers (hswo_driver.hip, hswo_wide.hip, hswo_levels.hip)
hipError_t launch_init_pixels(int32_t* parent, int32_t* mtime, int64_t n, hipStream_t s);
hipError_t launch_init_pixels_secs(const SecDev* secs, int n, int max_pixels, hipStream_t s);
hipError_t launch_init_leaves(const SecDev* secs, const InitDev* init, int n, int dtype, int max_pixels,
                              unsigned long long* counters, hipStream_t s);
hipError_t launch_section_driver(const SecDev* secs, int n, const LoopParams& lp, int variant, hipStream_t s,
                                 KTimer* kt);
constexpr int DRIVER_VARIANTS[3] = {2, 4, 6};  // adjacent-stage edges in flight per lane group
// fill_tiles > 0: the row caches that start in this iteration first get their interval matrix
// (k_mat_fill, fill_tiles 64 x 64 tiles per section)
hipError_t launch_wide_iteration(const SecDev* secs, int n, int G, const LoopParams& lp, int variant,
                                 bool spectral_possible, bool row_cache, int rows_grid, int fill_tiles, hipStream_t s,
                                 KTimer* kt);
int default_rows_grid();
constexpr int ROWS_MAX_SECTIONS = 1024;  // sections a row-cache task pool launch can cover
hipError_t launch_rowcache_prep(const SecDev* secs, int n, const LoopParams& lp, hipStream_t s, KTimer* kt);
hipError_t launch_compress(int32_t* parent, int64_t n, const unsigned long long* gate, hipStream_t s);
hipError_t launch_empty(hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s);
hipError_t launch_assemble(const SecDev* parents, const SecDev* children, const AsmDev* asm_, int n,
                           int32_t* slotmap, int max_cap, const unsigned long long* gate, hipStream_t s);
hipError_t launch_seam(const SecDev* parents, const AsmDev* asm_, int n, const int32_t* slotmap,
                       int max_seam, const unsigned long long* gate, hipStream_t s);
hipError_t launch_snapshot(const SnapDev* snaps, int n, const int32_t* counts, int n_levels, int max_pixels,
                           const unsigned long long* gate, hipStream_t s);

// host runtime (hswo_api.cpp), for the no-allocation entry point (hswo_noalloc.hip)
int set_error(int code, const char* msg);  // sets hswo_last_error(); returns code
void clear_error();
// RHSEG as rhseg_segment, with a fixed device scratch of scratch_bytes as the workspace and no event,
// graph or tuning trial created; refuses HSWO_FLAG_GRAPH, HSWO_FLAG_AUTOTUNE and
// HSWO_FLAG_KERNEL_TIMES. Every argument is validated on the host (the scratch size included) before
// get_scratch is called for the scratch's device address on the current device.
int rhseg_in_scratch(const void* cube, int H, int W, int B, int dtype, const hswo_params* p, int L,
                     int32_t* labels, hswo_merge_rec* merge_log, hswo_stats* stats, int (*get_scratch)(void**),
                     size_t scratch_bytes, hipStream_t stream);

}  // namespace hswo
