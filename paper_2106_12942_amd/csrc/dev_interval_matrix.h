// dev_interval_matrix.h -- part of the device code of the HSWO / HSEG / RHSEG merge loop.
//
// The interval matrix of the row cache (FP32 bounds of every pair kept by
// Ward's update), the row rescans and the least cached spectral pair.
#pragma once

#include "dev_row_cache.h"

namespace hswo {

namespace {

// ---------------------------------------------------------------------------
// Interval matrix of the row cache (Equation 1, wide mode). Entry (i, j)
// holds FP32 bounds [lo, hi] on the exact real value D(i, j) of Equation 1's
// square for the FP64 mean rows of slots i and j (the canonical FP64 value
// lies within a relative (B + 8) 2^-53 < 2^-40 of it for B <= 4096).
//  - A pair evaluated exactly stores its canonical value widened by 2^-40
//    and rounded outward (mat_entry); an exact 0 stays [0, 0].
//  - A merge of (a, b) gives the survivor's row by Ward's update, exact in
//    real arithmetic for this criterion:
//      D(k, a u b) = ((n_a + n_k) D(k, a) + (n_b + n_k) D(k, b) - n_k D(a, b))
//                    / (n_a + n_b + n_k),
//    evaluated on the bounds (lower bounds with the upper bound of D(a, b)
//    and the other way round), widened by the FP64 rounding of the formula
//    and rounded outward (mat_update).
//  - A row whose cached pair is stale is rescanned from its bounds: pairs
//    whose lower bound exceeds the row's second least upper bound cannot be
//    among its least two, and the others are evaluated exactly.
// ---------------------------------------------------------------------------
constexpr double MAT_REL = 0x1p-40;

__device__ __forceinline__ float2 mat_entry(double c) {
    if (!(c < __builtin_huge_val())) return make_float2(__builtin_huge_valf(), __builtin_huge_valf());
    return make_float2(__double2float_rd(c * (1.0 - MAT_REL)), __double2float_ru(c * (1.0 + MAT_REL)));
}

// Ward's update on bounds: e_a, e_b the bounds of D(k, a), D(k, b); [d_lo, d_hi]
// those of D(a, b); na, nb, nk the pixel counts before the merge. Each FP64
// operation errs by at most 2^-53 of its result; scaled by the reciprocal of
// the denominator every intermediate is at most t (the sum of the absolute
// terms over the denominator) in magnitude, so widening by 2^-48 t covers
// the few roundings of each bound.
__device__ __forceinline__ float2 mat_update(float2 e_a, float2 e_b, double d_lo, double d_hi, double na, double nb,
                                             double nk) {
    const double ca = na + nk, cb = nb + nk, inv = 1.0 / (na + nb + nk);
    const double lo = (ca * (double)e_a.x + cb * (double)e_b.x - nk * d_hi) * inv;
    const double hi = (ca * (double)e_a.y + cb * (double)e_b.y - nk * d_lo) * inv;
    const double t = (ca * (double)e_a.y + cb * (double)e_b.y + nk * d_hi) * inv;
    const double slack = t * 0x1p-48;
    return make_float2(__double2float_rd(fmax(lo - slack, 0.0)), __double2float_ru(hi + slack));
}

// Exact D2 of KR pending rows against 64 columns (one block task; a pair per
// lane and wave). The bands are added in the perfect binary tree over the
// zero-padded bands (P = next power of two >= B) that exact_d2_wave uses:
// wave w < nbc takes the aligned subtree of bands [w cs, (w + 1) cs), in
// groups of 8 bands (fixed subtrees) combined through a binary counter; the
// nbc chunk sums are then added in tree order from LDS. Column means come from
// the band-major copy (coalesced over the lanes), row means from the
// slot-major copy (the same for the whole wavefront). Each row's least two
// candidates among the 64 columns go to rpart; the lanes of the survivor's
// row (row 0 when not `all`) also take the light steps. Pending rows: the
// first np slots (all) or rpend[0, np). Called by the whole block.
// SAM: the spectral angle criterion (rows hold band sums; the tree adds the
// products of the two rows and the result is finished with the rows' squared
// norms).
template <int KR, bool SAM>
__device__ void row_block_task(double (*rsum)[4][64], const SecDev& s, int R, int np, bool all, int bq, int c) {
    constexpr int GB = 8;
    constexpr int LV = 7;  // up to 64 groups of 8 bands per wave (4096 bands over 8 waves)
    const int lane = lane_id(), w = wave_id();
    const int B = s.B, B8 = (B + 7) & ~7;
    const size_t kc = (size_t)s.rcap;
    int P = 1;
    while (P < B) P <<= 1;
    const int nbc = min(NWAVE, max(1, P / GB));
    const int cs = P / nbc;
    const int j = (c << 6) + lane;
    const bool jv = j < R;
    int ir[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int q = bq * KR + r;
        int v = -1;
        if (q < np) v = all ? q : s.rpend[q];
        ir[r] = __builtin_amdgcn_readfirstlane(v);
    }
    // light steps ride on the survivor's row (row 0 of the pending list, finished by wave 0)
    const bool light = !all && bq == 0 && w == 0 && jv;
    const int lmark = light ? s.rbp[j] : 0;
    if (w < nbc) {  // wavefront-uniform
        const int b_lo = w * cs;
        const int ngw = (cs + GB - 1) / GB;
        double part[KR][LV];
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int l = 0; l < LV; ++l) part[r][l] = 0.0;
        const double* mj = s.m64 + (jv ? j : 0);
        int gd = 0;
        for (int g = 0; g < ngw; ++g) {
            const int b0 = b_lo + g * GB;
            if (b0 >= B) break;  // the rest of the chunk is zero padding
            double cv[GB];
#pragma unroll
            for (int k = 0; k < GB; ++k) cv[k] = (b0 + k < B) ? mj[(size_t)(b0 + k) * kc] : 0.0;
#pragma unroll
            for (int r = 0; r < KR; ++r) {
                if (ir[r] < 0) continue;  // wavefront-uniform
                const double* mi = s.m64r + (size_t)ir[r] * B8 + b0;
                double qv[GB];
#pragma unroll
                for (int k = 0; k < GB; ++k) {
                    if (SAM) {
                        qv[k] = (b0 + k < B) ? mi[k] * cv[k] : 0.0;
                    } else {
                        const double d = (b0 + k < B) ? mi[k] - cv[k] : 0.0;
                        qv[k] = d * d;
                    }
                }
#pragma unroll
                for (int h = 1; h < GB; h <<= 1)
#pragma unroll
                    for (int k = 0; k < GB; k += 2 * h) qv[k] = qv[k] + qv[k + h];
                counter_push<LV>(part[r], qv[0], g);
            }
            gd = g + 1;
        }
#pragma unroll
        for (int r = 0; r < KR; ++r) rsum[w][r][lane] = counter_total<LV>(part[r], gd);
    }
    __syncthreads();
    if (w < KR) {  // wavefront r finishes row r of the batch
        const int q = bq * KR + w;
        if (q < np) {  // wavefront-uniform
            const int i = all ? q : s.rpend[q];
            double v[NWAVE];
#pragma unroll
            for (int k = 0; k < NWAVE; ++k) v[k] = (k < nbc) ? rsum[k][w][lane] : 0.0;
#pragma unroll
            for (int h = 1; h < NWAVE; h <<= 1)
#pragma unroll
                for (int k = 0; k < NWAVE; k += 2 * h) v[k] = v[k] + v[k + h];
            double d2;
            if (SAM) {
                d2 = sam_value(v[0], s.rq[i], jv ? s.rq[j] : 1.0);
            } else {
                const int n_i = s.npix[i];
                const int n_j = jv ? s.npix[j] : 1;
                const double dni = (double)n_i, dnj = (double)n_j;
                const double fac = (dni * dnj) / (double)(n_i + n_j);
                d2 = fac * v[0];
            }
            int lab = jv ? s.label[j] : INT_MAX, slot = j;
            if (!jv || j == i || (s.abit && abit_test(s, i, j))) {
                d2 = __builtin_huge_val();
                lab = INT_MAX;
                slot = -1;
            }
            if (light && lmark == -2) light_step(s, j, i, s.label[i], d2, s.rbd2[j], s.rbl2[j], s.rbp2[j], np);
            // for a fixed row the pair order (D2, lo, hi) is the order of (D2, partner label)
            RowPart rp = part_of(d2, lab, slot);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) top2_merge(rp, shfl_xor_part(rp, o));
            if (lane == 0) s.rpart[(size_t)q * ((R + 63) >> 6) + c] = rp;
        }
    }
    __syncthreads();  // rsum is reused by the next task
}

// The canonical Equation 1 value of pair (si, sj) by a whole wavefront (every
// lane gets it), from the FP64 means of the row cache (m64r): lane l holds
// bands 4l..4l+3 of each 256-band chunk, butterflies build the chunk's
// subtree, and a binary counter joins the chunk sums -- the perfect tree over
// the zero-padded bands of exact_d2_wave, which divides the sums on the fly
// (the stored means are those quotients), so the value is bit-identical.
__device__ double exact_wave_means(const SecDev& s, int si, int sj) {
    constexpr int LV = 5;  // up to 16 chunks of 256 bands: B <= 4096
    const int lane = lane_id();
    const int B = s.B, B8 = (B + 7) & ~7;
    const double* Mi = s.m64r + (size_t)si * B8;
    const double* Mj = s.m64r + (size_t)sj * B8;
    const int nchk = (B + 255) >> 8;
    double part[LV];
    for (int c = 0; c < nchk; ++c) {
        const int b = (c << 8) + (lane << 2);
        double q[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double d = (b + k < B) ? Mi[b + k] - Mj[b + k] : 0.0;
            q[k] = d * d;
        }
        double t = (q[0] + q[1]) + (q[2] + q[3]);
        t = t + __shfl_xor(t, 1);
        t = t + __shfl_xor(t, 2);
        t = t + __shfl_xor(t, 4);
        t = t + __shfl_xor(t, 8);
        t = t + __shfl_xor(t, 16);
        t = t + __shfl_xor(t, 32);
        counter_push<LV>(part, t, c);
    }
    const int n_i = s.npix[si], n_j = s.npix[sj];
    const double dni = (double)n_i, dnj = (double)n_j;
    return ((dni * dnj) / (double)(n_i + n_j)) * counter_total<LV>(part, nchk);
}

// Exact values of a wavefront's row-rescan candidates (pairs (i, cand[k]),
// k < n) into val[k], and the matrix entries of those pairs tightened to
// them, over groups of P consecutive candidates starting at first and
// advancing by stride (both multiples of P): P = 64 / L pairs at once in
// L-lane segments (exact_seg_means, one memory round trip per group) for
// B <= 1024, else P = 1 pair at a time over the whole wavefront
// (exact_wave_means). Either way the canonical value.
__device__ __forceinline__ int rescan_group(const SecDev& s) { return s.B <= 1024 ? 64 / mean_lanes(s.B) : 1; }

__device__ void rescan_eval(const SecDev& s, int i, const int* cand, double* val, int n, int first, int stride) {
    const int lane = lane_id();
    const size_t rc = (size_t)s.mstride;
    const int mi = s.msl[i];
    if (s.B <= 1024) {
        const int L = mean_lanes(s.B), seg = lane / L;
        for (int k0 = first; k0 < n; k0 += stride) {  // wavefront-uniform
            const int k = k0 + seg;
            const int j = k < n ? cand[k] : -1;
            const double v = exact_seg_means(s, j >= 0 ? i : -1, j, L);
            if (j >= 0 && (lane & (L - 1)) == 0) {
                val[k] = v;
                const float2 me = mat_entry(v);
                const int mj = s.msl[j];
                s.dmat[(size_t)mi * rc + mj] = me;
                s.dmat[(size_t)mj * rc + mi] = me;
            }
        }
    } else {
        for (int k = first; k < n; k += stride) {
            const int j = cand[k];
            const double v = exact_wave_means(s, i, j);
            if (lane == 0) {
                val[k] = v;
                const float2 me = mat_entry(v);
                const int mj = s.msl[j];
                s.dmat[(size_t)mi * rc + mj] = me;
                s.dmat[(size_t)mj * rc + mi] = me;
            }
        }
    }
}

// The two least of (a1 <= a2) and (b1 <= b2), into (a1, a2).
__device__ __forceinline__ void least_two(double& a1, double& a2, double b1, double b2) {
    const double big = fmax(a1, b1);
    a1 = fmin(a1, b1);
    a2 = fmin(big, fmin(a2, b2));
}


// LDS of row_matrix_task.
constexpr int MAT_CAND = 1024;  // candidates per round
struct RowMatLds {
    double m1[NWAVE], m2[NWAVE];
    int cand[MAT_CAND];
    double val[MAT_CAND];
    int ncand;
};

// One pending row q of a section, rescanned from the interval matrix by a
// whole workgroup: the row's threshold T is its second least upper bound
// (widened to the canonical value); a pair whose lower bound (likewise
// widened) exceeds T has two pairs strictly below it, so the row's least two
// by (D2, label) are among the others. Those are evaluated exactly
// (exact_wave_means, one wavefront per pair; a call of exact_seg_means here
// costs the kernel a call frame and twice the registers, and measured twice
// as slow) -- except pairs bounded by
// [0, 0], whose canonical value is 0 -- and their bounds tightened to the
// exact value. The row's least two go to its first chunk entry of rpart and
// +inf to the others, which is what the exact row tasks leave for the
// decision to reduce. Returns the number of exact evaluations (thread 0).
[[maybe_unused]] __device__ int row_matrix_task(RowMatLds& L, const SecDev& s, int R, int q, bool all) {
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    const size_t rc = (size_t)s.mstride;
    const int i = all ? q : s.rpend[q];
    const int mi = s.msl[i];
    const float2* Di = s.dmat + (size_t)mi * rc;
    const int nx = (R + NT - 1) / NT;  // bounds per thread
    double m1 = __builtin_huge_val(), m2 = __builtin_huge_val();
    for (int x = 0; x < nx; ++x) {
        const int j = x * NT + tid;
        if (j < R && j != i) least_two(m1, m2, (double)Di[s.msl[j]].y * (1.0 + MAT_REL), __builtin_huge_val());
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) least_two(m1, m2, __shfl_xor(m1, o), __shfl_xor(m2, o));
    if (lane == 0) {
        L.m1[w] = m1;
        L.m2[w] = m2;
    }
    if (tid == 0) L.ncand = 0;
    __syncthreads();
    m1 = L.m1[0];
    m2 = L.m2[0];
#pragma unroll
    for (int k = 1; k < NWAVE; ++k) least_two(m1, m2, L.m1[k], L.m2[k]);
    const double T = m2;
    RowPart best = part_of(__builtin_huge_val(), INT_MAX, -1);
    int nexact = 0;
    // candidates in rounds of at most MAT_CAND (block-uniform loop over the register slots)
    int x0 = 0;
    while (x0 < nx) {
        int x = x0;
        for (; x < nx; ++x) {
            // the round takes slots until it could overflow (NT per slot)
            if (L.ncand + NT > MAT_CAND) break;  // block-uniform: read after a barrier
            const int j = x * NT + tid;
            const float2 e = (j < R && j != i) ? Di[s.msl[j]] : make_float2(__builtin_huge_valf(), __builtin_huge_valf());
            const bool cand = j < R && j != i && (double)e.x * (1.0 - MAT_REL) <= T;
            if (cand) {
                if (e.y == 0.0f) {
                    top2_merge(best, part_of(0.0, s.label[j], j));  // bounded by [0, 0]: exactly 0
                } else {
                    L.cand[atomicAdd(&L.ncand, 1)] = j;
                }
            }
            __syncthreads();
        }
        const int n = L.ncand;
        for (int k = w; k < n; k += NWAVE) {
            const int j = L.cand[k];
            const double v = exact_wave_means(s, i, j);
            if (lane == 0) {
                L.val[k] = v;
                const float2 me = mat_entry(v);
                const int mj = s.msl[j];
                s.dmat[(size_t)mi * rc + mj] = me;
                s.dmat[(size_t)mj * rc + mi] = me;
            }
        }
        __syncthreads();
        for (int k = tid; k < n; k += NT) top2_merge(best, part_of(L.val[k], s.label[L.cand[k]], L.cand[k]));
        nexact += n;
        __syncthreads();
        if (tid == 0) L.ncand = 0;
        __syncthreads();
        x0 = x;
    }
    // the row's least two over the block
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) top2_merge(best, shfl_xor_part(best, o));
    RowPart* wb = reinterpret_cast<RowPart*>(L.val);  // the values are consumed
    if (lane == 0) wb[w] = best;
    __syncthreads();
    const int nch = (R + 63) >> 6;
    if (tid == 0) {
        RowPart b = wb[0];
        for (int k = 1; k < NWAVE; ++k) top2_merge(b, wb[k]);
        s.rpart[(size_t)q * nch] = b;
    }
    for (int c = 1 + tid; c < nch; c += NT) s.rpart[(size_t)q * nch + c] = part_of(__builtin_huge_val(), INT_MAX, -1);
    __syncthreads();  // LDS is reused by the next task
    return nexact;
}

// One wavefront evaluates KR pending rows against 64 columns over all bands
// (lane = column), for a workgroup that has the whole section to itself:
// its waves take different column chunks. Bands are added in groups of 8
// (fixed subtrees) through a binary counter of LV levels, which is the same
// perfect binary tree as exact_d2_wave's; the next group's column values are
// loaded before the current group is added.
template <int KR, int LV, bool SAM>
__device__ void row_wave_task(const SecDev& s, int R, int np, bool all, int bq, int c) {
    constexpr int GB = 8;
    const int lane = lane_id();
    const int B = s.B, B8 = (B + 7) & ~7;
    const size_t kc = (size_t)s.rcap;
    const int j = (c << 6) + lane;
    const bool jv = j < R;
    int ir[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int q = bq * KR + r;
        int v = -1;
        if (q < np) v = all ? q : s.rpend[q];
        ir[r] = __builtin_amdgcn_readfirstlane(v);
    }
    const int n_j = jv ? s.npix[j] : 1;
    const double q_j = (SAM && jv) ? s.rq[j] : 1.0;
    const int l_j = jv ? s.label[j] : INT_MAX;
    // light steps ride on the survivor's row (row 0 of the pending list)
    const bool light = !all && bq == 0 && jv;
    const int lmark = light ? s.rbp[j] : 0;
    const double* mj = s.m64 + (jv ? j : 0);
    double part[KR][LV];
#pragma unroll
    for (int r = 0; r < KR; ++r)
#pragma unroll
        for (int l = 0; l < LV; ++l) part[r][l] = 0.0;
    const int ng = (B + GB - 1) / GB;
    double cv[GB], nx[GB];
#pragma unroll
    for (int k = 0; k < GB; ++k) cv[k] = (k < B) ? mj[(size_t)k * kc] : 0.0;
    for (int g = 0; g < ng; ++g) {
        const int b0 = g * GB;
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            const int b = b0 + GB + k;
            nx[k] = (b < B) ? mj[(size_t)b * kc] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            if (ir[r] < 0) continue;  // wavefront-uniform
            const double* mi = s.m64r + (size_t)ir[r] * B8 + b0;
            double qv[GB];
#pragma unroll
            for (int k = 0; k < GB; ++k) {
                if (SAM) {
                    qv[k] = (b0 + k < B) ? mi[k] * cv[k] : 0.0;
                } else {
                    const double d = (b0 + k < B) ? mi[k] - cv[k] : 0.0;
                    qv[k] = d * d;
                }
            }
#pragma unroll
            for (int h = 1; h < GB; h <<= 1)
#pragma unroll
                for (int k = 0; k < GB; k += 2 * h) qv[k] = qv[k] + qv[k + h];
            counter_push<LV>(part[r], qv[0], g);
        }
#pragma unroll
        for (int k = 0; k < GB; ++k) cv[k] = nx[k];
    }
    const int nch = (R + 63) >> 6;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        if (ir[r] < 0) continue;  // wavefront-uniform
        const int i = ir[r];
        double d2;
        if (SAM) {
            d2 = sam_value(counter_total<LV>(part[r], ng), s.rq[i], q_j);
        } else {
            const int n_i = s.npix[i];
            const double dni = (double)n_i, dnj = (double)n_j;
            const double fac = (dni * dnj) / (double)(n_i + n_j);
            d2 = fac * counter_total<LV>(part[r], ng);
        }
        int lab = l_j, slot = j;
        if (!jv || j == i || (s.abit && abit_test(s, i, j))) {
            d2 = __builtin_huge_val();
            lab = INT_MAX;
            slot = -1;
        }
        if (light && r == 0 && lmark == -2) light_step(s, j, i, s.label[i], d2, s.rbd2[j], s.rbl2[j], s.rbp2[j], np);
        RowPart rp = part_of(d2, lab, slot);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) top2_merge(rp, shfl_xor_part(rp, o));
        if (lane == 0) {
            s.rpart[(size_t)(bq * KR + r) * nch + c] = rp;
        }
    }
}

// The rows that failed their light step (rpend[np, np + nf)) evaluated in
// full by this block, before the decision: a wavefront task per row and
// 64-column chunk, with the partials where the row stage puts them.
__device__ __forceinline__ void rows_fallback_body(const SecDev& s, int R, int np, int nf) {
    const int nch = (R + 63) >> 6;
    const int ntask = nf * nch;
    for (int t = wave_id(); t < ntask; t += NWAVE) {
        const int q = np + t / nch, c = t % nch;
        if (s.crit == HSWO_CRIT_SAM) {
            if (s.B <= 512)
                row_wave_task<1, 7, true>(s, R, np + nf, false, q, c);
            else
                row_wave_task<1, 10, true>(s, R, np + nf, false, q, c);
        } else if (s.B <= 512) {
            row_wave_task<1, 7, false>(s, R, np + nf, false, q, c);
        } else {
            row_wave_task<1, 10, false>(s, R, np + nf, false, q, c);
        }
    }
}

// The same with one pair per lane through exact_lane (same values), for a
// kernel whose registers are taken: a call of the full row evaluation would
// give it a stack.
__device__ __forceinline__ void rows_fallback_lanes(const SecDev& s, int R, int np, int nf) {
    const int nch = (R + 63) >> 6;
    const int ntask = nf * nch;
    for (int t = wave_id(); t < ntask; t += NWAVE) {
        const int q = np + t / nch, c = t % nch;
        const int i = s.rpend[q];
        const int j = (c << 6) + lane_id();
        const bool ok = j < R && j != i && !(s.abit && abit_test(s, i, j));
        const double d2 = exact_lane(s, ok ? i : -1, j);
        RowPart rp = ok ? part_of(d2, s.label[j], j) : part_of(__builtin_huge_val(), INT_MAX, -1);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) top2_merge(rp, shfl_xor_part(rp, o));
        if (lane_id() == 0) s.rpart[(size_t)q * nch + c] = rp;
    }
}

// Number of tasks of a section's row cache stage this iteration (4 rows by 64 columns each).
__device__ __forceinline__ int row_task_count(int R, int np) { return ((np + 3) / 4) * ((R + 63) >> 6); }

__device__ __forceinline__ KeyD pair_key(const SecDev& s, double d2, int a, int b) {
    const int la = s.label[a], lb = s.label[b];
    KeyD k;
    k.d2 = d2;
    if (la < lb) {
        k.lo = la;
        k.hi = lb;
        k.si = a;
        k.sj = b;
    } else {
        k.lo = lb;
        k.hi = la;
        k.si = b;
        k.sj = a;
    }
    return k;
}

// Least pair over all live slots, from the cached rows.
// Best pair of pending row q from its column-chunk partials.
__device__ __forceinline__ RowPart row_from_parts(const SecDev& s, int q, int nch) {
    RowPart b = part_of(__builtin_huge_val(), INT_MAX, -1);
    for (int c = 0; c < nch; ++c) top2_merge(b, s.rpart[(size_t)q * nch + c]);
    return b;
}



__device__ __forceinline__ KeyD row_key(double d2, int i, int li, int p, int lp) {
    KeyD k;
    k.d2 = d2;
    if (li < lp) {
        k.lo = li;
        k.hi = lp;
        k.si = i;
        k.sj = p;
    } else {
        k.lo = lp;
        k.hi = li;
        k.si = p;
        k.sj = i;
    }
    return k;
}

// The spectral minimum from the row cache: the pending rows (the first np
// slots when `all`, else rpend[0, np)) are finished from their partials, the
// other rows are read as cached (a pending row has rbp = -1), and the least
// key of both is returned to every thread. Every read happens before the
// block reduction and every write after it, so the cached rows are read
// unchanged; the finished rows are held in LDS when they fit.
__device__ KeyD spectral_min_rows(Smem& sh, const SecDev& s, int R, int np, bool all) {
    constexpr int HOLD = (int)(sizeof(sh.u.rsum) / sizeof(RowPart));
    RowPart* held = reinterpret_cast<RowPart*>(&sh.u.rsum[0][0][0]);
    const int nch = (R + 63) >> 6;
    KeyD best = key_none();
    int c2 = 1;
    while (c2 < nch) c2 <<= 1;
    if (c2 <= 64) {
        // a segment of c2 lanes per pending row, a lane per partial, reduced by butterflies
        const int rpw = 64 / c2;
        const int lane = lane_id(), sub = lane / c2, c = lane % c2;
        for (int q0 = wave_id() * rpw; q0 < np; q0 += NWAVE * rpw) {
            const int q = q0 + sub;
            RowPart r = part_of(__builtin_huge_val(), INT_MAX, -1);
            if (q < np && c < nch) r = s.rpart[(size_t)q * nch + c];
            for (int o = c2 >> 1; o >= 1; o >>= 1) top2_merge(r, shfl_xor_part(r, o));
            if (c == 0 && q < np) {
                const int i = all ? q : s.rpend[q];
                if (np <= HOLD) held[q] = r;
                if (r.slot >= 0) {
                    const KeyD k = row_key(r.d2, i, s.label[i], r.slot, r.lab);
                    if (key_less(k, best)) best = k;
                }
            }
        }
    } else {
        for (int q = threadIdx.x; q < np; q += NT) {
            const int i = all ? q : s.rpend[q];
            const RowPart r = row_from_parts(s, q, nch);
            if (np <= HOLD) held[q] = r;
            if (r.slot >= 0) {
                const KeyD k = row_key(r.d2, i, s.label[i], r.slot, r.lab);
                if (key_less(k, best)) best = k;
            }
        }
    }
    if (!all)
        for (int i = threadIdx.x; i < R; i += NT) {
            const int p = s.rbp[i];
            const double d2 = s.rbd[i];
            const int li = s.label[i], lp = s.rbl[i];
            if (p < 0) continue;
            const KeyD k = row_key(d2, i, li, p, lp);
            if (key_less(k, best)) best = k;
        }
    const KeyD M = block_min_key(sh, best);  // barriers: every read above is done
    for (int q = threadIdx.x; q < np; q += NT) {
        const int i = all ? q : s.rpend[q];
        const RowPart r = np <= HOLD ? held[q] : row_from_parts(s, q, nch);
        s.rbd[i] = r.d2;
        s.rbp[i] = r.slot;
        s.rbl[i] = r.lab;
        s.rbd2[i] = r.d2b;
        s.rbp2[i] = r.slotb;
        s.rbl2[i] = r.labb;
    }
    __syncthreads();
    return M;
}

}  // namespace

}  // namespace hswo
