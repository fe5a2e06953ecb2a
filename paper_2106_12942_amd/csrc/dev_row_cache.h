// dev_row_cache.h -- part of the device code of the HSWO / HSEG / RHSEG merge loop.
//
// The incremental form's spectral row cache: adjacency bits, the
// segmented-lane exact evaluation and the per-row least pairs.
#pragma once

#include "dev_screen.h"

namespace hswo {

namespace {

// ---------------------------------------------------------------------------
// Spectral row cache (incremental form). Every live slot i keeps a pair
// (i, p_i) with its exact D2. Invariant: every pair (a, b) of live slots has
// key(a, b) >= the key cached in row a or in row b, and every cached key is
// the key of a live pair. The least cached key is then the exact spectral
// minimum. A merge changes only the survivor's statistics and removes a slot,
// so re-evaluating the survivor's row in full, and every row whose cached
// partner was one of the merged pair, restores the invariant; all other rows
// keep their (still valid) pairs.
// ---------------------------------------------------------------------------


// Binary counter of finished subtrees for the band sum of one pair: group
// sum v (a subtree of GB bands, group index g) joins the counter; level l
// holds a finished subtree of GB * 2^l bands.
template <int LV>
__device__ __forceinline__ void counter_push(double (&part)[LV], double v, int g) {
    bool carry = true;
#pragma unroll
    for (int l = 0; l < LV; ++l) {
        if (carry) {
            if ((g >> l) & 1) {
                v = part[l] + v;
            } else {
                part[l] = v;
                carry = false;
            }
        }
    }
}

// Sum of the unfinished subtrees after ng groups: they sit at the set bits of
// ng, and the lower ones are the right-hand operands (the zero padding in
// between adds nothing).
template <int LV>
__device__ __forceinline__ double counter_total(const double (&part)[LV], int ng) {
    double acc = 0.0;
    bool have = false;
#pragma unroll
    for (int l = 0; l < LV; ++l)
        if ((ng >> l) & 1) {
            acc = have ? part[l] + acc : part[l];
            have = true;
        }
    return acc;
}

// Adjacency bitmap of the live slots (two-merge reading: its spectral step
// takes the least NON-adjacent pair, so the row evaluations are masked):
// row i holds bit j iff slots i and j share an edge. Rebuilt from the edge
// list (empty slots skipped) by the whole block.
__device__ void abit_build(const SecDev& s, int R, int E) {
    const int AW = (s.rcap + 31) >> 5;
    const int nw = R * AW;
    for (int x = threadIdx.x; x < nw; x += NT) s.abit[x] = 0u;
    __syncthreads();
    for (int e = threadIdx.x; e < E; e += NT) {
        const int2 ed = s.edges[e];
        if (ed.x >= 0) {
            atomicOr(&s.abit[(size_t)ed.x * AW + (ed.y >> 5)], 1u << (ed.y & 31));
            atomicOr(&s.abit[(size_t)ed.y * AW + (ed.x >> 5)], 1u << (ed.x & 31));
        }
    }
    __syncthreads();
}

// The bitmap after a merge of slots lo_s and hi_s (R live slots before it),
// without a rebuild: the survivor (slot surv: lo_s, or hi_s when lo_s is the
// last slot) takes the union of the pair's rows; every other live row ORs
// the pair's two bits into the survivor's; the region in the last slot moves
// to hi_s (its row is copied, and its bit in every row follows). The first
// two touch disjoint rows; a barrier orders the survivor row's own bits and
// the copy after them. Called by the whole block.
__device__ void abit_merge(const SecDev& s, int lo_s, int hi_s, int R) {
    const int AW = (s.rcap + 31) >> 5;
    const int last = R - 1;
    const int surv = (lo_s == last) ? hi_s : lo_s;
    const bool moves = hi_s != last && surv != hi_s;
    uint32_t* rl = s.abit + (size_t)lo_s * AW;
    uint32_t* rh = s.abit + (size_t)hi_s * AW;
    uint32_t* rs = s.abit + (size_t)surv * AW;
    for (int w = threadIdx.x; w < AW; w += NT) rs[w] = rl[w] | rh[w];
    for (int y = threadIdx.x; y < R; y += NT) {
        if (y == lo_s || y == hi_s) continue;
        uint32_t* row = s.abit + (size_t)y * AW;
        const uint32_t v = ((row[lo_s >> 5] >> (lo_s & 31)) | (row[hi_s >> 5] >> (hi_s & 31))) & 1u;
        const uint32_t vl = (row[last >> 5] >> (last & 31)) & 1u;
        if (surv == lo_s) {
            row[lo_s >> 5] = (row[lo_s >> 5] & ~(1u << (lo_s & 31))) | (v << (lo_s & 31));
            const uint32_t vh = moves ? vl : 0u;
            row[hi_s >> 5] = (row[hi_s >> 5] & ~(1u << (hi_s & 31))) | (vh << (hi_s & 31));
        } else {
            row[hi_s >> 5] = (row[hi_s >> 5] & ~(1u << (hi_s & 31))) | (v << (hi_s & 31));
        }
        row[last >> 5] &= ~(1u << (last & 31));  // the last slot is empty now (the survivor is never there)
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t bl = (rs[last >> 5] >> (last & 31)) & 1u;
        rs[lo_s >> 5] &= ~(1u << (lo_s & 31));
        rs[hi_s >> 5] &= ~(1u << (hi_s & 31));
        if (moves) {
            rs[last >> 5] &= ~(1u << (last & 31));
            rs[hi_s >> 5] |= bl << (hi_s & 31);
        }
    }
    if (moves) {
        const uint32_t* rx = s.abit + (size_t)last * AW;
        for (int w = threadIdx.x; w < AW; w += NT) rh[w] = rx[w];
    }
    __syncthreads();
}

__device__ __forceinline__ bool abit_test(const SecDev& s, int i, int j) {
    const int AW = (s.rcap + 31) >> 5;
    return (s.abit[(size_t)i * AW + (j >> 5)] >> (j & 31)) & 1u;
}

// The canonical criterion of pair (si, sj) by one lane (any lanes may hold
// different pairs; si < 0: no pair, result meaningless). The bands go in
// fixed groups of 8 (pairwise inside a group) whose sums join a binary
// counter of finished subtrees: the same perfect tree over the zero-padded
// bands as exact_d2_wave, as in the row tasks. Worth it when a block has many
// pairs to score at once (a survivor of high degree): 512 at a time instead
// of 64 / L per wavefront. Out of line to keep its counters out of its
// callers' registers.
__device__ __noinline__ double exact_lane(const SecDev& s, int si, int sj) {
    constexpr int GB = 8, LV = 10;  // up to 1023 groups: B <= 4096
    if (si < 0) return 0.0;
    const int B = s.B;
    const bool sam = s.crit == HSWO_CRIT_SAM;
    const double* Si = s.sums + (size_t)si * B;
    const double* Sj = s.sums + (size_t)sj * B;
    const int n_i = s.npix[si], n_j = s.npix[sj];
    const double dni = (double)n_i, dnj = (double)n_j;
    const int ng = (B + GB - 1) / GB;
    if (sam) {
        double pd[LV], pi[LV], pj[LV];
        for (int g = 0; g < ng; ++g) {
            const int b0 = g * GB;
            double td[GB], ti[GB], tj[GB];
#pragma unroll
            for (int k = 0; k < GB; ++k) {
                const bool in = b0 + k < B;
                const double x = in ? Si[b0 + k] : 0.0, y = in ? Sj[b0 + k] : 0.0;
                td[k] = x * y;
                ti[k] = x * x;
                tj[k] = y * y;
            }
#pragma unroll
            for (int h = 1; h < GB; h <<= 1)
#pragma unroll
                for (int k = 0; k < GB; k += 2 * h) {
                    td[k] = td[k] + td[k + h];
                    ti[k] = ti[k] + ti[k + h];
                    tj[k] = tj[k] + tj[k + h];
                }
            counter_push<LV>(pd, td[0], g);
            counter_push<LV>(pi, ti[0], g);
            counter_push<LV>(pj, tj[0], g);
        }
        return sam_value(counter_total<LV>(pd, ng), counter_total<LV>(pi, ng), counter_total<LV>(pj, ng));
    }
    double p[LV];
    for (int g = 0; g < ng; ++g) {
        const int b0 = g * GB;
        double t[GB];
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            const bool in = b0 + k < B;
            const double d = in ? Si[b0 + k] / dni - Sj[b0 + k] / dnj : 0.0;
            t[k] = d * d;
        }
#pragma unroll
        for (int h = 1; h < GB; h <<= 1)
#pragma unroll
            for (int k = 0; k < GB; k += 2 * h) t[k] = t[k] + t[k + h];
        counter_push<LV>(p, t[0], g);
    }
    return ((dni * dnj) / (double)(n_i + n_j)) * counter_total<LV>(p, ng);
}

// Start the row cache of a section at R live slots: FP64 means of every slot
// (spectral angle: the sums and their squared norms); every row is then
// pending (state 1).
// mat: the section keeps the interval matrix; the FP32 mean rows (zero
// padded to Bp) and their norm bounds, which the matrix fill reads, are then
// rebuilt from the FP64 means as well.
__device__ void rowcache_begin(Smem& sh, const SecDev& s, int R, int E, bool mat) {
    const int B = s.B;
    const size_t kc = (size_t)s.rcap;
    const int tot = R * B;
    const int B8 = (B + 7) & ~7;
    const bool sam = s.crit == HSWO_CRIT_SAM;
    for (int x = threadIdx.x; x < tot; x += NT) {
        const int b = x / R, i = x - b * R;
        const double v = s.sums[(size_t)i * B + b];
        const double m = sam ? v : v / (double)s.npix[i];
        if (!mat) s.m64[(size_t)b * kc + i] = m;  // the exact row tasks' columns (the matrix has its own)
        s.m64r[(size_t)i * B8 + b] = m;
        if (mat) s.mean[(size_t)i * s.Bp + b] = (float)m;
    }
    if (mat) {
        for (int i = threadIdx.x; i < R; i += NT) s.msl[i] = i;  // matrix row of each slot
        for (int x = threadIdx.x; x < R * (s.Bp - B); x += NT) {
            const int i = x / (s.Bp - B), b = B + x % (s.Bp - B);
            s.mean[(size_t)i * s.Bp + b] = 0.0f;
        }
        __syncthreads();
        for (int i = wave_id(); i < R; i += NWAVE) {  // the norm bound the FP32 screen uses
            double q = 0.0;
            for (int b = lane_id(); b < B; b += 64) {
                const double m = (double)s.mean[(size_t)i * s.Bp + b];
                q += m * m;
            }
            for (int o = 32; o >= 1; o >>= 1) q += __shfl_xor(q, o);
            if (lane_id() == 0) s.norm[i] = (float)(sqrt(q) * (1.0 + 0x1p-20));
        }
    }
    if (sam) {
        for (int i = wave_id(); i < R; i += NWAVE) {
            const double* Si = s.sums + (size_t)i * B;
            const double q = wave_dot_tree(Si, Si, B);
            if (lane_id() == 0) s.rq[i] = q;
        }
    }
    for (int i = threadIdx.x; i < R; i += NT) {
        s.rbp[i] = -1;
        s.rbd[i] = __builtin_huge_val();
        s.rbp2[i] = -1;
    }
    __syncthreads();
    if (s.abit) abit_build(s, R, E);
    if (threadIdx.x == 0) {
        s.st[6] = 1;
        s.st[7] = 0;
        s.st[11] = 0;
    }
    __syncthreads();
}

__device__ __forceinline__ bool cand_less(double d1, int l1, double d2, int l2) {
    return d1 < d2 || (d1 == d2 && l1 < l2);
}

// r := the least two candidates of r and o (each holds its least two, from
// disjoint columns), in (D2, partner label) order; symmetric in r and o.
__device__ __forceinline__ void top2_merge(RowPart& r, const RowPart& o) {
    if (cand_less(o.d2, o.lab, r.d2, r.lab)) {
        if (cand_less(o.d2b, o.labb, r.d2, r.lab)) {
            r.d2b = o.d2b;
            r.labb = o.labb;
            r.slotb = o.slotb;
        } else {
            r.d2b = r.d2;
            r.labb = r.lab;
            r.slotb = r.slot;
        }
        r.d2 = o.d2;
        r.lab = o.lab;
        r.slot = o.slot;
    } else if (cand_less(o.d2, o.lab, r.d2b, r.labb)) {
        r.d2b = o.d2;
        r.labb = o.lab;
        r.slotb = o.slot;
    }
}

__device__ __forceinline__ RowPart shfl_xor_part(const RowPart& r, int o) {
    RowPart t;
    t.d2 = __shfl_xor(r.d2, o);
    t.lab = __shfl_xor(r.lab, o);
    t.slot = __shfl_xor(r.slot, o);
    t.d2b = __shfl_xor(r.d2b, o);
    t.labb = __shfl_xor(r.labb, o);
    t.slotb = __shfl_xor(r.slotb, o);
    return t;
}

// Light step of row j (marked rbp = -2 by the merge: its cached partner was
// merged, its second bound's partner is alive), taken by the lane that holds
// column j of the survivor's row: the row's new pair is the lesser of its
// pair with the survivor (c, exact, masked) and its second bound, which is
// then spent. Exact: the second bound is at or below every pair the row had
// at its last full evaluation except its old partner, and each pair created
// since is bounded by its other row, evaluated in full when it was created.
// A bare bound (rbp2 = -3: its partner has merged since) still bounds the
// row's old pairs, so the step stands when c is at or below it; otherwise the
// row is appended to the pending list (rpend[np + k], k counted in st[11])
// for a full evaluation before the decision.
__device__ __forceinline__ void light_step(const SecDev& s, int j, int surv, int lsurv, double c, double d2b, int lb,
                                           int pb, int np) {
    if (cand_less(c, lsurv, d2b, lb) || (c == d2b && lsurv == lb)) {
        s.rbd[j] = c;
        s.rbp[j] = surv;
        s.rbl[j] = lsurv;
    } else if (pb >= 0) {
        s.rbd[j] = d2b;
        s.rbp[j] = pb;
        s.rbl[j] = lb;
        s.rbp2[j] = -1;
    } else {
        s.rbp[j] = -1;
        s.rpend[np + atomicAdd(&s.st[11], 1)] = j;
    }
}

// One column's candidate of a row as a partial (second: none).
__device__ __forceinline__ RowPart part_of(double d2, int lab, int slot) {
    RowPart r;
    r.d2 = d2;
    r.lab = lab;
    r.slot = slot;
    r.d2b = __builtin_huge_val();
    r.labb = INT_MAX;
    r.slotb = -1;
    return r;
}

}  // namespace

}  // namespace hswo
