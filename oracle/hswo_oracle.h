/*
 * hswo_oracle.h -- plain FP64 CPU oracle for HSWO / HSEG / RHSEG.
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU library
 * (libhswo). Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it; no product code path calls into it.
 *
 * Method (Section 4.1 of the paper):
 *   HSEG loop (the four numbered steps of Section 4.1): every pixel starts
 *   as a region; each iteration finds the spatially adjacent pair with the
 *   smallest dissimilarity, and (spectral clustering) the smallest
 *   non-adjacent pair; the non-adjacent pair is merged instead when it is
 *   smaller than the adjacent minimum, weighted by the spectral clustering
 *   weight; stop at the requested region count.
 *   RHSEG: the image is split into 4^(L-1) sections, HSEG runs on the
 *   deepest sections, the four sections of a parent are reassembled with
 *   8-neighbourhood links across the split lines (Figure 4.4), and HSEG
 *   runs again on the parent, up to level 1.
 *   Criterion (Equation 1): sqrt( n_i n_j / (n_i + n_j) * sum_b (mu_ib - mu_jb)^2 ).
 *   The oracle ranks on the squared value D2 (sqrt is monotone).
 *   Alternative criterion (Section 4.1 lists the spectral angle among the
 *   usable ones): the spectral angle, ranked on 1 - sign(c) c^2 with c its
 *   cosine, i.e. sin^2 of the angle up to 90 degrees; the decision rule and
 *   the squared weight are the same as for Equation 1.
 *
 * Readings taken where the paper is silent:
 *   one merge per iteration (two_merges selects the other reading of the
 *   step list: step 2's adjacent merge, then step 3's non-adjacent merge on
 *   the partition it left); the non-adjacent pair wins iff
 *   D2_na < w^2 * D2_adj (strict); spectral stage active iff w > 0 and
 *   R <= spclust_max; ties broken lexicographically on (D2, lo, hi) where
 *   lo < hi are region labels; a region's label is its smallest row-major
 *   pixel index; canonical FP64 criterion with fixed operation order (band
 *   terms summed as a zero-padded pairwise tree) and no fused multiply-add.
 */
#ifndef HSWO_ORACLE_H
#define HSWO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_params {
    int32_t connectivity;       /* 4 or 8, inside a section */
    int32_t seam_connectivity;  /* 4 or 8, across RHSEG split lines */
    float spclust_wght;         /* spectral clustering weight w in [0,1] */
    int32_t spclust_max;        /* spectral stage active iff R <= this (0: never) */
    int32_t target_regions;     /* stop count of the top pass */
    int32_t section_regions;    /* stop count of non-top passes (0: max(target, spclust_max/4)) */
    int32_t rnb_levels;         /* L >= 1 */
    int32_t n_levels;           /* number of label snapshots */
    const int32_t* level_counts;/* strictly decreasing, last == target */
    int32_t brute;              /* 1: recompute every pair every iteration */
    int32_t n_threads;          /* worker threads over independent sections */
    int32_t criterion;          /* ORACLE_CRIT_BSMSE (Equation 1) or ORACLE_CRIT_SAM */
    int32_t two_merges;         /* 1: each iteration merges the best adjacent pair (step 2), then the
                                   best non-adjacent pair of the result if it is below w^2 times the
                                   first merge's value (step 3); 0: one merge per iteration */
    int32_t multi_merge;        /* 1: several merges per step for identical regions: a step whose
                                   one-merge winner has the value 0 merges every pair of a greedy
                                   disjoint set of zero-valued pairs, taken in the one-merge rule's
                                   order (adjacent pairs by (lo, hi), then, with the spectral stage
                                   on at the step's start, non-adjacent pairs by (lo, hi)), until the
                                   pass's stop count; later merges of a step carry kind + 2 in the
                                   log. Equation 1 only, not with two_merges */
    /* optional: called after each section of a recursion level has finished
       (depth 0 = the whole image), with how many of that level's sections are
       done; calls are serialised. Reports progress only. */
    void (*progress)(int32_t depth, int32_t done, int32_t total);
} oracle_params;

#define ORACLE_CRIT_BSMSE 0 /* Equation 1, ranked on its square D2 */
#define ORACLE_CRIT_SAM 1   /* spectral angle, ranked on 1 - sign(c) c^2 (c its cosine) */

typedef struct oracle_merge {
    int32_t lo, hi;     /* region labels, lo < hi; lo survives */
    int32_t kind;       /* 0 adjacent, 1 non-adjacent (spectral); + 2 for the second and later
                           merges of one step (multi_merge) */
    int32_t r_after;    /* live regions in the section after this merge */
    double d2;          /* canonical FP64 squared criterion */
} oracle_merge;

/* Canonical squared criterion of Equation 1 from band sums and counts. */
double oracle_d2(const double* Si, const double* Sj, int64_t ni, int64_t nj, int32_t B);

/* Spectral angle criterion from band sums: 1 - sign(c) c^2, c = cos(angle). */
double oracle_sam(const double* Si, const double* Sj, int32_t B);

/*
 * Run RHSEG (HSWO/HSEG when rnb_levels == 1) on a float32 H x W x B cube
 * (band-interleaved by pixel, host memory).
 *   labels   : [n_levels][H][W] int32 output (required)
 *   log      : optional, capacity H*W records; merges in level order,
 *              sections of a level in quadtree order (TL, TR, BL, BR, recursively)
 *   n_log    : optional, number of records written
 *   out_*    : optional final regions of the top pass: up to H*W entries
 * Returns 0 on success, -1 on invalid parameters.
 */
int oracle_rhseg(const float* cube, int32_t H, int32_t W, int32_t B, const oracle_params* p,
                 int32_t* labels, oracle_merge* log, int64_t* n_log,
                 int32_t* out_R, int32_t* out_label, int64_t* out_n, double* out_S);

#ifdef __cplusplus
}
#endif

#endif
