// dev_exact.h -- part of the device code of the HSWO / HSEG / RHSEG merge loop.
//
// Canonical FP64 evaluation of Equation 1 (and of the spectral angle): one
// wavefront per pair with a fixed pairwise band tree, the segmented-lane
// forms for many pairs at once, and the batched re-scoring of edge lists.
#pragma once

#include "dev_common.h"

namespace hswo {

namespace {

__device__ double wave_dot_tree(const double* x, const double* y, int B) {
    const int lane = lane_id();
    const int nch = (B + 255) >> 8;
    double u = 0.0;
    for (int c = 0; c < nch; ++c) {
        double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
        const int b = (c << 8) + (lane << 2);
        if (b + 3 < B) {
            q0 = x[b] * y[b];
            q1 = x[b + 1] * y[b + 1];
            q2 = x[b + 2] * y[b + 2];
            q3 = x[b + 3] * y[b + 3];
        } else {
            if (b < B) q0 = x[b] * y[b];
            if (b + 1 < B) q1 = x[b + 1] * y[b + 1];
            if (b + 2 < B) q2 = x[b + 2] * y[b + 2];
        }
        double t = (q0 + q1) + (q2 + q3);
        t = t + __shfl_xor(t, 1);
        t = t + __shfl_xor(t, 2);
        t = t + __shfl_xor(t, 4);
        t = t + __shfl_xor(t, 8);
        t = t + __shfl_xor(t, 16);
        t = t + __shfl_xor(t, 32);
        if (lane == c) u = t;
    }
    u = u + __shfl_xor(u, 1);
    u = u + __shfl_xor(u, 2);
    u = u + __shfl_xor(u, 4);
    u = u + __shfl_xor(u, 8);
    return __shfl(u, 0);
}

// Spectral angle criterion from the dot product of two band-sum rows and
// their squared norms: 1 - sign(c) c^2 with c the cosine (sin^2 of the angle
// up to 90 degrees, rising to 2 at 180); 1 for a zero row; rounding below 0
// is raised to 0.
__device__ __forceinline__ double sam_value(double dot, double qi, double qj) {
    const double den = qi * qj;
    if (den == 0.0) return 1.0;
    const double t = (dot * dot) / den;
    const double d = dot >= 0.0 ? 1.0 - t : 1.0 + t;
    return d > 0.0 ? d : 0.0;
}

__device__ double exact_d2_wave(Smem& sh, const SecDev& s, int si, int sj) {
    const int lane = lane_id();
    const int B = s.B;
    if (s.crit == HSWO_CRIT_SAM) {
        const double* Xi = s.sums + (size_t)si * B;
        const double* Xj = s.sums + (size_t)sj * B;
        const double dot = wave_dot_tree(Xi, Xj, B);
        const double qi = wave_dot_tree(Xi, Xi, B);
        const double qj = wave_dot_tree(Xj, Xj, B);
        return sam_value(dot, qi, qj);
    }
    const int n_i = s.npix[si], n_j = s.npix[sj];
    const double dni = (double)n_i, dnj = (double)n_j;
    const double* Si = s.sums + (size_t)si * B;
    const double* Sj = s.sums + (size_t)sj * B;
    const int nch = (B + 255) >> 8;
    double* cs = sh.csum[wave_id()];
    for (int c = 0; c < nch; ++c) {
        double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
        const int b = (c << 8) + (lane << 2);
        if (b + 3 < B) {
            double d;
            d = Si[b] / dni - Sj[b] / dnj; q0 = d * d;
            d = Si[b + 1] / dni - Sj[b + 1] / dnj; q1 = d * d;
            d = Si[b + 2] / dni - Sj[b + 2] / dnj; q2 = d * d;
            d = Si[b + 3] / dni - Sj[b + 3] / dnj; q3 = d * d;
        } else {
            double d;
            if (b < B) { d = Si[b] / dni - Sj[b] / dnj; q0 = d * d; }
            if (b + 1 < B) { d = Si[b + 1] / dni - Sj[b + 1] / dnj; q1 = d * d; }
            if (b + 2 < B) { d = Si[b + 2] / dni - Sj[b + 2] / dnj; q2 = d * d; }
        }
        double t = (q0 + q1) + (q2 + q3);
        t = t + __shfl_xor(t, 1);
        t = t + __shfl_xor(t, 2);
        t = t + __shfl_xor(t, 4);
        t = t + __shfl_xor(t, 8);
        t = t + __shfl_xor(t, 16);
        t = t + __shfl_xor(t, 32);
        if (lane == 0) cs[c] = t;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    double u = (lane < nch) ? cs[lane] : 0.0;
    u = u + __shfl_xor(u, 1);
    u = u + __shfl_xor(u, 2);
    u = u + __shfl_xor(u, 4);
    u = u + __shfl_xor(u, 8);
    const double acc = __shfl(u, 0);
    const double fac = (dni * dnj) / (double)(n_i + n_j);
    return fac * acc;
}

// Exact score of edge e into the per-edge cache (one wavefront; +inf for an
// empty slot).
__device__ __forceinline__ void score_edge_exact(Smem& sh, const SecDev& s, int e) {
    const int2 ed = s.edges[e];
    double v = __builtin_huge_val();
    if (ed.x >= 0) {
        int a = ed.x, b = ed.y;
        if (s.label[a] > s.label[b]) {
            const int t = a; a = b; b = t;
        }
        v = exact_d2_wave(sh, s, a, b);
    }
    if (lane_id() == 0) s.ed2[e] = v;
}

// Lanes per pair of the segmented exact evaluation: the least power of two L
// with 4L >= B when B <= 256 (a segment then holds every band in one pass);
// 0 for wider cubes (one pair per wavefront, exact_d2_wave).
__device__ __forceinline__ int seg_lanes(int B) {
    if (B > 256) return 0;
    int L = 1;
    while (4 * L < B) L <<= 1;
    return L;
}

// The canonical criterion of pair (si, sj) by an L-lane segment of a
// wavefront (4L >= B): lane m of the segment holds bands 4m..4m+3 and
// butterflies stay inside the segment. That is the perfect tree over the
// zero-padded bands that exact_d2_wave builds (its extra zero leaves add
// nothing), so the value is bit-identical. Every lane of the wavefront calls
// it with the same L, each segment with its own pair; a segment without a
// pair passes si < 0 (its result is meaningless). Kept out of line: inlined
// at its three call sites it pushes the decision kernel into scratch.
__device__ __noinline__ double exact_seg(const SecDev& s, int si, int sj, int L) {
    const int B = s.B;
    const int b = (lane_id() & (L - 1)) << 2;
    const bool sam = s.crit == HSWO_CRIT_SAM;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;  // Equation 1: t0; spectral angle: dot, q_i, q_j
    double fac = 0.0;
    if (si >= 0) {
        const double* Si = s.sums + (size_t)si * B;
        const double* Sj = s.sums + (size_t)sj * B;
        double x[4], y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = (b + k < B) ? Si[b + k] : 0.0;
            y[k] = (b + k < B) ? Sj[b + k] : 0.0;
        }
        if (sam) {
            t0 = (x[0] * y[0] + x[1] * y[1]) + (x[2] * y[2] + x[3] * y[3]);
            t1 = (x[0] * x[0] + x[1] * x[1]) + (x[2] * x[2] + x[3] * x[3]);
            t2 = (y[0] * y[0] + y[1] * y[1]) + (y[2] * y[2] + y[3] * y[3]);
        } else {
            const int n_i = s.npix[si], n_j = s.npix[sj];
            const double dni = (double)n_i, dnj = (double)n_j;
            double q[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double d = x[k] / dni - y[k] / dnj;
                q[k] = (b + k < B) ? d * d : 0.0;
            }
            t0 = (q[0] + q[1]) + (q[2] + q[3]);
            fac = (dni * dnj) / (double)(n_i + n_j);
        }
    }
    for (int o = 1; o < L; o <<= 1) {
        t0 = t0 + __shfl_xor(t0, o);
        if (sam) {
            t1 = t1 + __shfl_xor(t1, o);
            t2 = t2 + __shfl_xor(t2, o);
        }
    }
    return sam ? sam_value(t0, t1, t2) : fac * t0;
}

// Segment width of exact_seg_means: lanes of 16 bands each over the bands
// zero-padded to a power of two P (one lane for P <= 16); B <= 1024.
__device__ __forceinline__ int mean_lanes(int B) {
    int P = 16;
    while (P < B) P <<= 1;
    return P / 16;
}

// The canonical criterion of Equation 1 for pair (si, sj) by an L-lane
// segment (L = mean_lanes(B)) from the row cache's FP64 means (m64r, the
// stored quotients S / n, so no division per band): lane m of the segment
// adds its aligned run of 16 bands 16m..16m+15 as a perfect binary tree in
// registers, and the segment's butterflies join the runs in tree order -- the
// same zero-padded pairwise tree, so the same value, as the other exact
// evaluations. All 32 loads of a lane are independent, so a segment costs one
// memory round trip; 64 / L pairs per wavefront. For slots whose means are
// current (row cache running). si < 0: no pair (result meaningless).
__device__ __noinline__ double exact_seg_means(const SecDev& s, int si, int sj, int L) {
    const int B = s.B, B8 = (B + 7) & ~7;
    const int b0 = (lane_id() & (L - 1)) << 4;
    double t0 = 0.0, fac = 0.0;
    if (si >= 0) {
        const double* Mi = s.m64r + (size_t)si * B8;
        const double* Mj = s.m64r + (size_t)sj * B8;
        double x[16], y[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const bool in = b0 + k < B;
            x[k] = in ? Mi[b0 + k] : 0.0;
            y[k] = in ? Mj[b0 + k] : 0.0;
        }
        double q[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double d = x[k] - y[k];
            q[k] = d * d;
        }
#pragma unroll
        for (int w = 1; w < 16; w <<= 1)
#pragma unroll
            for (int k = 0; k < 16; k += 2 * w) q[k] = q[k] + q[k + w];
        t0 = q[0];
        const int n_i = s.npix[si], n_j = s.npix[sj];
        const double dni = (double)n_i, dnj = (double)n_j;
        fac = (dni * dnj) / (double)(n_i + n_j);
    }
    for (int o = 1; o < L; o <<= 1) t0 = t0 + __shfl_xor(t0, o);
    return fac * t0;
}

// exact_seg_means for the two pairs (si, sj) and (si, sk) at once: the
// segment loads si's run once and both partners' runs together (one memory
// round trip for two pairs). The value of (si, sk) goes to v2. The canonical
// value does not depend on the pair's order (a difference and its negation
// square alike, the count factor is symmetric), so si may be either end.
// si < 0: no pair; sk < 0: no second pair (those results are meaningless).
__device__ __noinline__ double exact_seg_means2(const SecDev& s, int si, int sj, int sk, int L, double& v2) {
    const int B = s.B, B8 = (B + 7) & ~7;
    const int b0 = (lane_id() & (L - 1)) << 4;
    double t0 = 0.0, t1 = 0.0, fac0 = 0.0, fac1 = 0.0;
    if (si >= 0) {
        const int sk2 = sk >= 0 ? sk : sj;
        const double* Mi = s.m64r + (size_t)si * B8;
        const double* Mj = s.m64r + (size_t)sj * B8;
        const double* Mk = s.m64r + (size_t)sk2 * B8;
        double x[16], y[16], z[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const bool in = b0 + k < B;
            x[k] = in ? Mi[b0 + k] : 0.0;
            y[k] = in ? Mj[b0 + k] : 0.0;
            z[k] = in ? Mk[b0 + k] : 0.0;
        }
        double q[16], r[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double d = x[k] - y[k];
            const double e = x[k] - z[k];
            q[k] = d * d;
            r[k] = e * e;
        }
#pragma unroll
        for (int w = 1; w < 16; w <<= 1)
#pragma unroll
            for (int k = 0; k < 16; k += 2 * w) {
                q[k] = q[k] + q[k + w];
                r[k] = r[k] + r[k + w];
            }
        t0 = q[0];
        t1 = r[0];
        const int n_i = s.npix[si], n_j = s.npix[sj], n_k = s.npix[sk2];
        const double dni = (double)n_i, dnj = (double)n_j, dnk = (double)n_k;
        fac0 = (dni * dnj) / (double)(n_i + n_j);
        fac1 = (dni * dnk) / (double)(n_i + n_k);
    }
    for (int o = 1; o < L; o <<= 1) {
        t0 = t0 + __shfl_xor(t0, o);
        t1 = t1 + __shfl_xor(t1, o);
    }
    v2 = fac1 * t1;
    return fac0 * t0;
}

// One pair per lane, for many pairs at once (defined with the row tasks' counter).
__device__ __noinline__ double exact_lane(const SecDev& s, int si, int sj);

// A merge that re-scores more edges than this takes them one per lane
// (exact_lane): the survivor of a region that keeps absorbing its neighbours.
// The pass-start scoring of every edge stays in segments, which measured
// faster there.
constexpr int LANE_PAIRS_MIN = 256;

// Exact scores of the edges list[0, n) (list == nullptr: edges [0, n)) into
// the per-edge cache, +inf for an empty slot; 64 / L edges per wavefront
// when the bands fit an L-lane segment. Called by the whole block.
__device__ void score_edges(Smem& sh, const SecDev& s, const int* list, int n) {
    const int L = seg_lanes(s.B);
    if (L == 0) {
        for (int i = wave_id(); i < n; i += NWAVE) score_edge_exact(sh, s, list ? list[i] : i);
        return;
    }
    const int ppw = 64 / L, sub = lane_id() / L;
    for (int i0 = wave_id() * ppw; i0 < n; i0 += NWAVE * ppw) {  // wavefront-uniform trip count
        const int i = i0 + sub;
        int e = -1, a = -1, b = -1;
        if (i < n) {
            e = list ? list[i] : i;
            const int2 ed = s.edges[e];
            a = ed.x;
            b = ed.y;
        }
        const double v = exact_seg(s, a, b, L);
        if (e >= 0 && (lane_id() & (L - 1)) == 0) s.ed2[e] = a >= 0 ? v : __builtin_huge_val();
    }
}

}  // namespace

}  // namespace hswo
