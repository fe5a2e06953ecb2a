/*
 * hswo.h -- C ABI of libhswo: hierarchical step-wise optimisation (HSWO /
 * HSEG) region merging and its recursive approximation RHSEG on MI355X
 * (gfx950), for hyperspectral cubes.
 *
 * Method (Section 4.1 of the paper):
 *   Every pixel starts as a region. Each iteration evaluates the
 *   dissimilarity of every spatially adjacent region pair, and -- when
 *   spectral clustering is on -- of every non-adjacent pair; the most similar
 *   pair is merged (the four HSEG steps of Section 4.1). RHSEG splits the
 *   image into 4^(L-1) sections, runs HSEG on the deepest sections,
 *   reassembles each group of four with links across the split lines
 *   (Figure 4.4) and runs HSEG again on the reassembled section, up to the
 *   whole image.
 *   Dissimilarity: square root of the band-sum MSE, Equation 1,
 *     sqrt( n_i n_j / (n_i + n_j) * sum_b (mu_ib - mu_jb)^2 ).
 *
 * Readings where the paper is silent (the same in the CPU oracle):
 *   - One merge per iteration. The best non-adjacent pair N is merged instead
 *     of the best adjacent pair A iff D2(N) < w^2 * D2(A) (D2 = the squared
 *     criterion, w = spclust_wght), strict, so A wins exact ties.
 *   - The spectral (non-adjacent) stage of a section is active iff w > 0 and
 *     the section's live region count R <= spclust_max.
 *   - Ties are broken on the lexicographic key (D2, lo, hi) with lo < hi the
 *     two region labels. The merged region keeps label lo.
 *   - A region's label is its smallest row-major pixel index (0-based); the
 *     output label maps hold these values.
 *   - D2 is decided in IEEE FP64 with one fixed operation order:
 *       fac = (n_i * n_j) / (n_i + n_j)
 *       d_b = S_ib / n_i - S_jb / n_j;  q_b = d_b * d_b
 *       acc = pairwise tree sum of q_0..q_{B-1} zero-padded to a power of two
 *       D2  = fac * acc
 *     with S the FP64 band sums, no fused multiply-add. Lower precisions are
 *     used only as screens with certified error bounds; every decision is
 *     re-checked with the formula above, so the merge sequence and the label
 *     maps do not depend on the screen's precision.
 *   - RHSEG splits a section at floor(h/2), floor(w/2) into TL, TR, BL, BR.
 *     Inside a leaf, pixels are linked under `connectivity`; at every
 *     reassembly, pixel pairs across the split lines are linked under
 *     `seam_connectivity` (8 follows the paper's 8-neighbourhood).
 *   - A non-top pass stops at section_regions regions; the top pass stops at
 *     target_regions and writes the label maps of the requested levels.
 *
 * Conventions for every entry point:
 *   - Device pointers are HIP device memory of the current device. The cube
 *     and every output are owned by the caller. The library allocates no
 *     device memory: the scratch it needs is the caller's `workspace`, at
 *     least hswo_workspace_bytes() bytes, 256-byte aligned. Between calls it
 *     keeps only the autotuner's choices and, with HSWO_FLAG_GRAPH, captured
 *     graphs.
 *   - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the null
 *     stream). Outputs are valid once that stream has completed. When `stats`
 *     is non-NULL the call synchronises the stream before returning to fill
 *     it in.
 *   - Parameters are validated on the host before anything is enqueued; on
 *     error nothing is written and the error code is returned, with a message
 *     available from hswo_last_error(). No C++ exception crosses the ABI.
 *   - Non-finite input: the first kernel counts NaN and infinite cube
 *     values; when there is one, every later kernel of the call returns at
 *     once, so nothing is merged and the label maps and the merge log are
 *     left as they were. A call with stats (which synchronises) then returns
 *     HSWO_E_NONFINITE and stats->nonfinite_values; an asynchronous call
 *     (stats NULL) cannot return it -- pass stats to learn it.
 */
#ifndef HSWO_H
#define HSWO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSWO_VERSION 10100 /* 1.1.0 */

/* return codes */
#define HSWO_OK 0
#define HSWO_E_INVAL (-1)       /* invalid argument */
#define HSWO_E_NOMEM (-2)       /* workspace too small (see hswo_workspace_bytes) */
#define HSWO_E_DEVICE (-3)      /* a HIP call failed */
#define HSWO_E_NONFINITE (-4)   /* the cube holds a NaN or an infinity (reported when the call synchronises:
                                   stats non-NULL; see "Non-finite input" below) */
#define HSWO_E_UNSUPPORTED (-5) /* valid request this library version does not implement */

/* cube element types */
#define HSWO_F32 0
#define HSWO_F16 1

/* screening precision for the non-adjacent (spectral) stage */
#define HSWO_PREC_FP32 0      /* plain: FP32 vector ALU screen */
#define HSWO_PREC_SCREEN_BF16 1 /* Gram cross-term on BF16 matrix cores, FP32 accumulate */
#define HSWO_PREC_SCREEN_FP16 2 /* Gram cross-term on FP16 matrix cores, FP32 accumulate */

/* dissimilarity criterion (Section 4.1 names several usable ones; the paper
   evaluates Equation 1) */
#define HSWO_CRIT_BSMSE 0 /* Equation 1, ranked on its square D2 (above) */
#define HSWO_CRIT_SAM 1   /* spectral angle between the mean spectra, ranked on
                             D = 1 - sign(c) c^2 with c the cosine (sin^2 of the angle up to
                             90 degrees, rising to 2 at 180), in one fixed FP64 order:
                               dot = pairwise tree over b of S_ib * S_jb,
                               q_i = pairwise tree over b of S_ib * S_ib (likewise q_j),
                               t = (dot * dot) / (q_i * q_j),
                               D = 1 - t if dot >= 0 else 1 + t, raised to 0 if negative;
                               D = 1 when q_i * q_j == 0 (a zero spectrum).
                             The counts cancel, so the band sums serve. Decision rule and
                             tie-break are those of Equation 1 with D in place of D2 (the
                             weight enters squared: D is the square of sin(angle)), so the
                             merge log's d2 field holds D. HSWO_FLAG_INCREMENTAL form only
                             (other forms return HSWO_E_UNSUPPORTED). */

/* flags */
#define HSWO_FLAG_MERGE_LOG 1 /* fill merge_log (must be non-NULL) */
#define HSWO_FLAG_DEBUG_VERIFY_BOUND 128 /* screened forms (not HSWO_FLAG_INCREMENTAL): for every pair a
                                            screen passes on to the FP64 re-check, write the screen's
                                            estimate, its certified bounds and the canonical D2 to
                                            p->verify (hswo_verify_rec; up to p->verify_cap records,
                                            hswo_stats.verify_records counts them all). Costs time;
                                            for checking the screens' error bounds. */
#define HSWO_FLAG_GRAPH 2     /* capture the call's kernel sequence into a hipGraph on first use and
                                 replay it on later calls with the same pointers, shapes and
                                 parameters (needs a non-null stream); graphs are cached per
                                 process (up to 16, oldest evicted) */
#define HSWO_FLAG_INCREMENTAL 8 /* keep each adjacent pair's exact D2 and re-score only the pairs a merge
                                   changed (the adjacent minimum is then a reduction over the cached
                                   values); same merges and labels as the full per-iteration sweep */
#define HSWO_FLAG_KERNEL_TIMES 16 /* bracket every merge-loop kernel launch with hipEvents on the call's
                                     stream and report per-kernel device time in hswo_stats
                                     (ms_kernel, kernel_launches); needs stats, not with
                                     HSWO_FLAG_GRAPH */
#define HSWO_FLAG_SEQUENTIAL_SECTIONS 32 /* run the sections of a level one after another, each
                                             with the whole device (the unbatched path, for
                                             comparison); same merges and labels */
#define HSWO_FLAG_TWO_MERGES 64 /* the other reading of the HSEG step list (Section 4.1): each iteration
                                    merges the least adjacent pair (step 2), then -- when the spectral
                                    stage is on at the count that merge left and the stop count is not
                                    reached -- the least NON-adjacent pair of the resulting partition
                                    if its D2 < w^2 * D2 of step 2's pair (step 3). Changes the result.
                                    HSWO_FLAG_INCREMENTAL form only (else HSWO_E_UNSUPPORTED). */
#define HSWO_FLAG_MULTI_MERGE 256 /* several merges per step for identical regions (Section 6.2): a
                                     step whose winner has the value 0 merges a greedy disjoint set
                                     of zero-valued pairs -- adjacent pairs by (lo, hi), then, with the
                                     spectral stage on at the step's start, non-adjacent pairs by
                                     (lo, hi), skipping a pair one of whose regions is taken -- one
                                     after another until the stop count; other steps merge one pair.
                                     Later merges of a step carry kind + 2 in the merge log. Changes
                                     the result. HSWO_FLAG_INCREMENTAL form and Equation 1 only (else
                                     HSWO_E_UNSUPPORTED), not with HSWO_FLAG_TWO_MERGES (HSWO_E_INVAL);
                                     every level runs in the persistent section driver. */
#define HSWO_FLAG_AUTOTUNE 4  /* on the first call for a shape bucket, time candidate execution
                                 settings (hswo_tuning: workgroups per section, which levels run
                                 persistent, the row-stage grid and interval matrix, the
                                 section-driver variant) on the
                                 call itself -- all give identical results -- and keep the fastest;
                                 the choice is cached per process and appended to the file named by
                                 the environment variable HSWO_TUNE_CACHE if set. Settings given
                                 explicitly in p->tuning are not tuned. */

/* Execution settings. None of them changes a merge or a label; they only
   decide how the work is spread over the device. -1 in a field = the
   library's default (or, with HSWO_FLAG_AUTOTUNE, the tuned value). */
typedef struct hswo_tuning {
    int32_t wide_max_sections;  /* recursion levels of more sections than this run in the persistent
                                   section driver (one workgroup per section, one launch), the others
                                   in wide mode (several workgroups per section, a launch sequence per
                                   merge); 0 = every level persistent. Default: the device's CU count
                                   in the incremental form, 64 in the others */
    int32_t wide_groups;        /* wide mode: workgroups per section of the screened sweeps, 1..256;
                                   default CUs / sections */
    int32_t rows_grid;          /* wide mode, incremental form: workgroups of the row-stage launch,
                                   >= 1; default 2 x CUs */
    int32_t hybrid;             /* incremental form: 1 = the merges of a wide level before its spectral
                                   stage run in the persistent driver first, 0 = all in wide mode;
                                   default 1 */
    int32_t bare_bounds;        /* incremental form: row-cache second bounds kept after their partner
                                   merges: 0 none, 1 those of value 0, 2 all; default 1 */
    int32_t driver_variant;     /* adjacent-sweep edges in flight per 16-lane group of the screened
                                   forms: 2, 4 or 6; default 6 */
    int32_t row_matrix;         /* incremental form, Equation 1, one-merge reading: 1 = the
                                   row cache keeps certified FP32 bounds on every pair's value, brought
                                   up to date at each merge by Ward's update (O(R) per merge); a row
                                   whose cached pair went stale is rescanned from its bounds and only
                                   the pairs that can be among its least two are evaluated in FP64;
                                   0 = stale rows re-evaluated in FP64 against every column. Up to
                                   4096 row-cache slots (spclust_max); default 1 */
} hswo_tuning;                  /* 28 bytes */

/* One pair checked under HSWO_FLAG_DEBUG_VERIFY_BOUND. */
typedef struct hswo_verify_rec {
    int32_t lo, hi;   /* labels of the pair, lo < hi */
    int32_t stage;    /* HSWO_SCREEN_* that passed the pair on */
    int32_t r;        /* live regions in the section at that iteration */
    double screen;    /* the screen's estimate of D2 */
    double lower;     /* the certified bounds the screen relies on: lower <= D2 <= upper must hold */
    double upper;
    double d2;        /* the canonical FP64 D2 of the pair */
} hswo_verify_rec;    /* 48 bytes */

#define HSWO_SCREEN_ADJ_FP32 0   /* adjacent pairs, FP32 sum of squares of the mean rows */
#define HSWO_SCREEN_SPEC_FP32 1  /* non-adjacent stage, FP32 tiles */
#define HSWO_SCREEN_SPEC_16 2    /* non-adjacent stage, 16-bit Gram cross-term on the matrix cores
                                    (estimate from N_i + N_j - 2 G_ij of the centred 16-bit rows) */

typedef struct hswo_params {
    int32_t connectivity;       /* 4 or 8: pixel links inside a leaf section */
    int32_t seam_connectivity;  /* 4 or 8: pixel links across RHSEG split lines */
    float spclust_wght;         /* spectral clustering weight w, 0 <= w <= 1 (not NaN) */
    int32_t spclust_max;        /* spectral stage iff R <= spclust_max; 0 = never; <= 65535 */
    int32_t target_regions;     /* >= 1: stop count of the top pass */
    int32_t section_regions;    /* stop count of non-top passes; 0 = max(target, spclust_max/4) */
    int32_t rnb_levels;         /* L >= 1 recursion levels (4^(L-1) leaf sections) */
    int32_t n_levels;           /* number of label maps to output, >= 1 */
    const int32_t* level_counts;/* HOST pointer, n_levels entries, strictly decreasing,
                                   all >= target_regions, last == target_regions */
    int32_t precision;          /* HSWO_PREC_* */
    int32_t flags;              /* HSWO_FLAG_* */
    int32_t criterion;          /* HSWO_CRIT_* dissimilarity criterion (0 = Equation 1) */
    int32_t screen_topk;        /* screened forms: the re-check set of an iteration is every pair whose
                                   certified lower bound reaches the least upper bound (so it always
                                   holds the exact minimum); an iteration whose set holds more than
                                   screen_topk pairs counts as a fallback in hswo_stats
                                   (screen_fallbacks). 0 = 8; >= 0 */
    hswo_verify_rec* verify;    /* device, HSWO_FLAG_DEBUG_VERIFY_BOUND only: verify_cap records */
    int64_t verify_cap;
    const hswo_tuning* tuning;  /* HOST pointer, optional (NULL = defaults / autotuned) */
} hswo_params;                  /* 80 bytes */

typedef struct hswo_merge_rec {
    int32_t lo, hi;   /* labels of the merged regions, lo < hi; lo survives */
    int32_t kind;     /* 0 adjacent (spatial stage), 1 non-adjacent (spectral stage); + 2 for the
                         second and later merges of one step (HSWO_FLAG_MULTI_MERGE) */
    int32_t r_after;  /* live regions in the section after the merge */
    double d2;        /* the canonical FP64 squared criterion of the merge */
} hswo_merge_rec;     /* 24 bytes */

/* kernel kinds of hswo_stats.ms_kernel / kernel_launches */
#define HSWO_K_SECTION_DRIVER 0 /* one workgroup per section runs a whole pass */
#define HSWO_K_WIDE_ADJ 1       /* wide mode: adjacent screen, edges split over G workgroups */
#define HSWO_K_WIDE_DECIDE 2    /* wide mode: decision and merge, one workgroup per section */
#define HSWO_K_WIDE_MFMA 3      /* wide mode: matrix-core tile screen of the spectral stage */
#define HSWO_K_WIDE_FP32 4      /* wide mode: FP32 tile screen of the spectral stage */
#define HSWO_K_WIDE_FINISH 5    /* wide mode: spectral decision and merge */
#define HSWO_K_WIDE_ROWS 6      /* wide mode, incremental form: row-cache re-evaluation */
#define HSWO_K_ROWCACHE_PREP 7  /* incremental form: row cache start at a pass start */
#define HSWO_K_MATRIX_FILL 8    /* wide mode, incremental form: the interval matrix of row caches that
                                   start, 64 x 64 pair tiles of FP32 mean differences */
#define HSWO_NK 9

typedef struct hswo_stats {
    int64_t merges;              /* merges performed */
    int64_t iterations;          /* merge-loop iterations over all sections */
    int64_t adjacent_pairs;      /* adjacent pairs of the method, summed over iterations (live edges
                                    per iteration, whether screened or read from the cache) */
    int64_t spectral_pairs;      /* unordered pairs of the method's spectral stage, summed over the
                                    iterations where it is active (R (R - 1) / 2 each) */
    int64_t exact_rechecks;      /* pairs evaluated in canonical FP64 (screen re-checks, cache
                                    re-scoring, row-cache rows, and the pairs a rescan from the
                                    interval matrix could not rule out) */
    int64_t tile_rescans;        /* spectral tiles re-screened to collect candidates */
    int64_t fp32_tiles;          /* 64 x 64 spectral tiles screened in FP32 */
    int64_t mfma_tiles;          /* 128 x 128 super tiles screened on matrix cores (16-bit forms) */
    int64_t driver_launches;     /* launches of the section-driver kernel */
    int64_t driver_variant;      /* section-driver variant used (adjacent-stage edges in flight) */
    double ms_total;             /* device time of the call (hipEvents), ms */
    double ms_driver;            /* device time inside section-driver launches (hipEvents), ms */
    /* per-stage time inside the merge loop, summed over sections (device
       constant clock), ms: adjacent stage, matrix-core screen, FP32
       spectral tiles with the exact re-check, merge */
    double ms_adjacent, ms_mfma_screen, ms_fp32_spectral, ms_merge;
    /* with HSWO_FLAG_KERNEL_TIMES: device time (hipEvents around each launch)
       and launches per kernel kind HSWO_K_*; zero otherwise */
    double ms_kernel[HSWO_NK];
    int64_t kernel_launches[HSWO_NK];
    /* algorithmic work of the kind's launches, counted on the device (0 where
       not defined): HSWO_K_WIDE_DECIDE (incremental form) bytes =
       16 per edge slot (endpoints and cached D2 read for the minimum)
       + 24 per band per merge (two FP64 sum rows read, one written)
       + in the spectral stage 12 per live row (cached pair) and 32 per
       pending row per 64 live rows (least two candidates of each 64 columns),
       + 8 per band per live region when rows whose second bound no longer
       holds are evaluated in full before the minimum;
       HSWO_K_WIDE_ROWS bytes = exact row tasks (up to 4 rows by 64 columns):
       the columns' FP64 mean rows read once (8 per band and column) + 8 per
       band per row; matrix rescans: 8 per pair of a rescanned row (its
       bounds) + 16 per band (two FP64 mean rows) and 16 per pair evaluated
       exactly;
       HSWO_K_MATRIX_FILL flops = 3 FP32 flops per band per pair bounded;
       HSWO_K_SECTION_DRIVER (incremental form) bytes = the HSWO_K_WIDE_DECIDE
       count for the iterations it runs + 8 per band per live region for each
       iteration whose row-cache stage evaluates rows (every FP64 row read
       once);
       HSWO_K_WIDE_ADJ bytes = per section and iteration, the FP32 mean rows
       read once (4 per band per live region) + 8 per edge slot + 8 per region;
       HSWO_K_WIDE_MFMA flops = 2 per band per unique pair of every section
       screened on matrix cores */
    int64_t kernel_work[HSWO_NK];
    /* with HSWO_FLAG_KERNEL_TIMES: what one event pair around a launch adds to
       the launch's own time, measured in the same call on an empty kernel
       (bracketed launches minus back-to-back launches), ms; ms_kernel[k] minus
       kernel_launches[k] times this is the kind's launch time */
    double ms_event_pair_overhead;
    int64_t nonfinite_values;    /* NaN or infinite cube values found (then nothing was merged) */
    int64_t screen_iterations;   /* iterations whose decision went through a certified screen (screened
                                    forms; adjacent and spectral stages counted separately) */
    int64_t screen_fallbacks;    /* ... of which the re-check set held more than screen_topk pairs */
    int64_t verify_records;      /* HSWO_FLAG_DEBUG_VERIFY_BOUND: records produced (written up to
                                    verify_cap) */
    int64_t row_bounded_pairs;   /* incremental form: row-cache pairs rescanned from the interval
                                    matrix (hswo_tuning.row_matrix); those it could not rule out are
                                    counted in exact_rechecks */
    hswo_tuning tuning;          /* the execution settings the call used */
    int32_t reserved;
} hswo_stats;   /* 424 bytes */

/* One independent section for hswo_run_batch. */
typedef struct hswo_section {
    const void* cube;   /* device, H x W x B, band-interleaved by pixel, dtype of the call */
    int32_t H, W, B;
    int32_t* labels;    /* device, [n_levels][H][W] int32; labels are local pixel indices */
    hswo_merge_rec* merge_log; /* device, H*W - target records, or NULL */
} hswo_section;

/* Library version (HSWO_VERSION). */
int hswo_version(void);

/* Message of the last error returned on the calling thread ("" if none). */
const char* hswo_last_error(void);

/* Workspace needed by hswo_run / rhseg_segment for this shape and parameters
   (rnb_levels taken from p). Returns 0 if the parameters are invalid. */
size_t hswo_workspace_bytes(int32_t H, int32_t W, int32_t B, int32_t dtype, const hswo_params* p);

/*
 * HSEG on the whole image as one section (RHSEG with L = 1; Section 4.1,
 * the four HSEG steps). p->rnb_levels must be 1.
 *   cube       device, H x W x B (band-interleaved by pixel), dtype HSWO_F32 or
 *              HSWO_F16, finite values, 16-byte aligned
 *   labels     device, [p->n_levels][H][W] int32 output
 *   merge_log  device, (H*W - target) records in merge order, or NULL
 *   stats      host, optional (synchronises the stream)
 *   workspace  device scratch, ws_bytes >= hswo_workspace_bytes(...)
 */
int hswo_run(const void* cube, int32_t H, int32_t W, int32_t B, int32_t dtype, const hswo_params* p,
             int32_t* labels, hswo_merge_rec* merge_log, hswo_stats* stats, void* workspace,
             size_t ws_bytes, void* hip_stream);

/*
 * RHSEG (Section 4.1, recursive approximation of HSEG, Figures 4.3 and 4.4)
 * with rnb_levels = L. Arguments as hswo_run. The merge log lists the merges
 * of the deepest level first, the sections of a level in quadtree order (TL,
 * TR, BL, BR, recursively), merges of a section in order.
 */
int rhseg_segment(const void* cube, int32_t H, int32_t W, int32_t B, int32_t dtype,
                  const hswo_params* p, int32_t rnb_levels, int32_t* labels,
                  hswo_merge_rec* merge_log, hswo_stats* stats, void* workspace, size_t ws_bytes,
                  void* hip_stream);

/*
 * Many independent sections, each segmented as its own top pass (HSEG on a
 * section, Section 4.1; sections are independent, as RHSEG's sections of one
 * level are), all in one persistent launch. Every section uses the same
 * parameters (p->rnb_levels must be 1) and the same dtype; H, W, B may
 * differ. Labels are local pixel indices of each section.
 */
size_t hswo_batch_workspace_bytes(int32_t n_sections, const hswo_section* sections, int32_t dtype,
                                  const hswo_params* p);
int hswo_run_batch(int32_t n_sections, const hswo_section* sections, int32_t dtype,
                   const hswo_params* p, hswo_stats* stats, void* workspace, size_t ws_bytes,
                   void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops and harnesses that forbid hipMalloc): rhseg_segment without a
 * workspace argument. The scratch is the library's own static device array of
 * HSWO_NOALLOC_SCRATCH_BYTES (one copy per GPU, held from the library's first
 * use of that GPU until the process ends); the call allocates nothing, creates
 * no event or graph, and otherwise behaves as rhseg_segment (same merges,
 * labels, merge log and errors).
 *   - A shape and parameters whose scratch exceeds HSWO_NOALLOC_SCRATCH_BYTES
 *     (see hswo_workspace_bytes) return HSWO_E_NOMEM before anything is
 *     enqueued; p->flags may not hold HSWO_FLAG_GRAPH, HSWO_FLAG_AUTOTUNE or
 *     HSWO_FLAG_KERNEL_TIMES (HSWO_E_INVAL). With stats the call synchronises
 *     the stream and fills the counters; its device times are 0.
 *   - Every call on one GPU shares that GPU's array: calls that overlap on
 *     one GPU (from two threads, or on two streams) race and must not be
 *     made. The array keeps the last call's contents; no call depends on them.
 */
#define HSWO_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20) /* 256 MiB */
int rhseg_segment_noalloc(const void* cube, int32_t H, int32_t W, int32_t B, int32_t dtype,
                          const hswo_params* p, int32_t rnb_levels, int32_t* labels,
                          hswo_merge_rec* merge_log, hswo_stats* stats, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HSWO_H */
