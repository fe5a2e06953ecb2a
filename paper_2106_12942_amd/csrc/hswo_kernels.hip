// hswo_kernels.hip -- CDNA4 (gfx950) kernels of the HSWO / HSEG / RHSEG hot path.
//
// The method is the HSEG loop of Section 4.1 of the paper: every iteration
// scores all spatially adjacent region pairs and, when spectral clustering is
// on, all non-adjacent pairs with Equation 1, takes the minimum, merges that
// pair and updates the region statistics and adjacency. Here one workgroup
// owns one section and runs the whole loop on the device (no host round trip
// per merge, unlike the paper's CPU-side merge of Section 4.2):
//
//   adjacent stage   16 lanes per edge stream the two FP32 mean rows (float4,
//                    coalesced), an FP32 sum of squares with a certified
//                    error bound; per-edge (lower, upper) bounds go to scratch.
//   spectral stage   all pairs i < j in 64 x 64 tiles staged through LDS,
//                    FP32, with per-tile (min lower, min upper).
//   decision         every pair whose lower bound can reach the minimum is
//                    re-scored with the canonical FP64 formula (one wavefront
//                    per pair, fixed pairwise band tree), and the exact
//                    lexicographic minimum (D2, lo, hi) decides.
//   merge            FP64 band sums, counts, FP32 mean row and norm of the
//                    survivor; swap-remove of the dead slot; one block pass
//                    relabels, de-duplicates and compacts the edge list.
//
// The spectral stage scores all pairs without masking adjacent ones: if the
// overall minimum M is below w^2 * D2(A) (A the best adjacent pair) it cannot
// be adjacent, because every adjacent pair has D2 >= D2(A) >= w^2 D2(A); and
// if it is not below, no non-adjacent pair is. So the merge chosen is the one
// the paper's step 3 chooses, with no adjacency test inside the tiles.
//
// Compiled with -ffp-contract=off: every FP64 operation of the re-check is a
// single IEEE round-to-nearest operation in the order written; FMAs in the
// screens are written explicitly (fmaf).

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "hswo_internal.h"

namespace hswo {

namespace {

constexpr float U32 = 5.9604645e-08f;  // 2^-24, unit roundoff of FP32

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// 16-bit screen formats: PREC 1 = bfloat16, PREC 2 = float16 (round to nearest even)
template <int PREC>
struct Fmt16;
template <>
struct Fmt16<1> {
    typedef bf16x8 V;
    static constexpr double U = 0x1p-8;     // unit roundoff
    static constexpr double SUB = 0x1p-133; // largest rounding error below the normal range
    static __device__ __forceinline__ uint16_t enc(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
    static __device__ __forceinline__ float dec(uint16_t h) { return (float)__builtin_bit_cast(__bf16, h); }
    static __device__ __forceinline__ f32x16 mfma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Fmt16<2> {
    typedef f16x8 V;
    static constexpr double U = 0x1p-11;
    static constexpr double SUB = 0x1p-25;
    static __device__ __forceinline__ uint16_t enc(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
    static __device__ __forceinline__ float dec(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
    static __device__ __forceinline__ f32x16 mfma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

constexpr int TLIST = 1024;          // tile list chunk (LDS)
constexpr int KSLAB = 256;           // bands of the 16-bit operands staged in LDS at a time
constexpr int G16_LD = KSLAB + 8;    // LDS row stride (elements) of the 16-bit operand tiles

struct KeyD {
    double d2;
    int lo, hi;  // labels, lo < hi
    int si, sj;  // slots of lo and hi
};

__device__ __forceinline__ KeyD key_none() {
    KeyD k;
    k.d2 = __builtin_huge_val();
    k.lo = INT_MAX;
    k.hi = INT_MAX;
    k.si = -1;
    k.sj = -1;
    return k;
}

__device__ __forceinline__ bool key_less(const KeyD& a, const KeyD& b) {
    if (a.d2 != b.d2) return a.d2 < b.d2;
    if (a.lo != b.lo) return a.lo < b.lo;
    return a.hi < b.hi;
}

__device__ __forceinline__ bool key_exists(const KeyD& k) { return k.lo != INT_MAX; }

// Whether a section's row cache keeps the interval matrix (set per level by
// the host: wide mode, and every section of the level has one).
__device__ __forceinline__ bool row_matrix_on(const SecDev& s, const LoopParams& lp) {
    return lp.row_matrix && s.dmat != nullptr;
}

// Non-finite input found at initialisation: every later kernel of the call
// returns at once, so nothing is merged and no output is written.
__device__ __forceinline__ bool gated(const unsigned long long* counters) {
    return counters != nullptr && counters[C_NONFINITE] != 0ull;
}

struct Smem {
    union {
        struct {
            float As[BK][TILE + 4];
            float Cs[BK][TILE + 4];
            int cand[CAND_CAP];
        } f;
        struct {
            uint16_t A[STILE][G16_LD];
            uint16_t C[STILE][G16_LD];
            float Prow[STILE], Arow[STILE], Pcol[STILE], Acol[STILE];
        } g;
        double rsum[NWAVE][4][64];  // row cache: per-wave band-chunk sums of a task
    } u;
    float redf[2][NWAVE];
    int redi[NWAVE];
    double redd[NWAVE];
    KeyD redk[NWAVE];
    double csum[NWAVE][16];
    int ncand;
    int ntl;                 // entries of tlist
    int npend;               // rows appended to the row cache's pending list
    int tlist[TLIST];        // tiles gathered for a pass (one barrier instead of one per tile)
    int bcast_i[4];
    int idx[8];              // incremental merge: slot ranges and the chunk range scanned
    int zc[2];               // several merges per step: list counters
    int eread;               // incremental merge: edge slots (and chunk records) it read
    unsigned long long cnt[C_COUNT];  // per-block counters and stage clocks (thread 0 only)
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}

// minimum of two floats over the block; every thread gets both results
__device__ __forceinline__ float2 block_min_f2(Smem& sh, float a, float b) {
    a = wave_min_f(a);
    b = wave_min_f(b);
    if (lane_id() == 0) {
        sh.redf[0][wave_id()] = a;
        sh.redf[1][wave_id()] = b;
    }
    __syncthreads();
    float ra = sh.redf[0][0], rb = sh.redf[1][0];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) {
        ra = fminf(ra, sh.redf[0][w]);
        rb = fminf(rb, sh.redf[1][w]);
    }
    __syncthreads();
    return make_float2(ra, rb);
}

// minimum of a double over the block; every thread gets the result
__device__ double block_min_d(Smem& sh, double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    if (lane_id() == 0) sh.redd[wave_id()] = v;
    __syncthreads();
    double r = sh.redd[0];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) r = fmin(r, sh.redd[w]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum_d(Smem& sh, double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0) sh.redd[wave_id()] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) r += sh.redd[w];
    __syncthreads();
    return r;
}

__device__ __forceinline__ KeyD shfl_key(const KeyD& k, int o) {
    KeyD r;
    r.d2 = __shfl_xor(k.d2, o);
    r.lo = __shfl_xor(k.lo, o);
    r.hi = __shfl_xor(k.hi, o);
    r.si = __shfl_xor(k.si, o);
    r.sj = __shfl_xor(k.sj, o);
    return r;
}

__device__ KeyD block_min_key(Smem& sh, KeyD k) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        KeyD x = shfl_key(k, o);
        if (key_less(x, k)) k = x;
    }
    if (lane_id() == 0) sh.redk[wave_id()] = k;
    __syncthreads();
    KeyD r = sh.redk[0];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w)
        if (key_less(sh.redk[w], r)) r = sh.redk[w];
    __syncthreads();
    return r;
}

// exclusive prefix of a 0/1 flag over the block; returns the prefix, *total set
__device__ __forceinline__ int block_scan_flag(Smem& sh, bool f, int* total) {
    const unsigned long long m = __ballot(f);
    const int lane = lane_id();
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) sh.redi[wave_id()] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) {
        const int c = sh.redi[w];
        if (w < wave_id()) before += c;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return before + below;
}

// Certified bounds on the canonical D2 of a pair from its FP32 screen.
//   s      FP32 sum over bands of (m_a - m_b)^2, FMA accumulated
//   na,nb  pixel counts; Na,Nb upper bounds of the FP32 mean-row norms
//   gam    accumulation bound ~ (2B + 32) u
// m_a = fl32(fl64(S_a / n_a)) is within ~u|mu_a| of the true mean per band and
// the per-band difference rounds once, so ||d~ - d|| <= ~2u(Na + Nb); the
// computed s is within gam of ||d~||^2. The FP64 canonical value differs from
// the real value by far less than the 32u margin.
__device__ __forceinline__ float2 screen_bounds(float s, int na, int nb, float Na, float Nb, float gam) {
    const float fa = (float)na, fb = (float)nb;
    const float w = (fa * fb) / (fa + fb);
    const float r = sqrtf(s);
    const float eta = 3.0f * U32 * (Na + Nb);
    const float rl = fmaxf(r * (1.0f - gam) - eta, 0.0f);
    const float rh = r * (1.0f + gam) + eta;
    return make_float2(w * rl * rl * (1.0f - 32.0f * U32), w * rh * rh * (1.0f + 32.0f * U32));
}

// Canonical FP64 squared criterion, evaluated by one whole wavefront (all 64
// lanes must call it with the same arguments; every lane gets the result).
// With the spectral angle criterion, that criterion's value instead.
//   fac = (n_i n_j)/(n_i + n_j); d_b = S_ib/n_i - S_jb/n_j; q_b = d_b*d_b;
//   acc = pairwise tree over b of q_b, zero-padded to a power of two.
// Lane l holds bands 4l..4l+3 of each 256-band chunk: two in-register levels,
// six butterfly levels across lanes (a+b == b+a bitwise, so both lanes of a
// pair hold the same sum). Chunk sums are parked in LDS and combined by a
// 16-leaf tree (again butterflies, over lanes 0..15). Zero padding beyond
// the next power of two only adds +0.0, which is exact.
// Pairwise tree over the zero-padded band index of x_b * y_b, by one whole
// wavefront (every lane gets the result): the lane layout of exact_d2_wave,
// with lane c keeping chunk c's sum for the final 16-leaf tree.
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

// ---------------------------------------------------------------------------
// HSWO_FLAG_DEBUG_VERIFY_BOUND: for every pair a screen passes on to the FP64
// re-check, the screen's estimate of D2, the certified bounds it relies on and
// the canonical D2 go to the caller's buffer.
// ---------------------------------------------------------------------------
__device__ void verify_put(const SecDev& s, int lo, int hi, int stage, int R, double screen, double lower,
                           double upper, double d2) {
    const unsigned long long k = atomicAdd(s.vcount, 1ull);
    if ((long long)k < s.vcap) {
        hswo_verify_rec r;
        r.lo = lo;
        r.hi = hi;
        r.stage = stage;
        r.r = R;
        r.screen = screen;
        r.lower = lower;
        r.upper = upper;
        r.d2 = d2;
        s.vout[k] = r;
    }
}

// The matrix-core Gram value g_i . g_j of two 16-bit screen rows, accumulated
// as the tile screen does (16 bands per instruction, in band order). Every
// row of the A operand is g_i and every column of B is g_j, so each output
// element is that dot product. Called by a whole wavefront.
template <int PREC>
__device__ float gram16_wave(const SecDev& s, int i, int j) {
    typedef Fmt16<PREC> F;
    typedef typename F::V V;
    const int lane = lane_id();
    const uint16_t* gi = s.g16 + (size_t)i * s.Bp;
    const uint16_t* gj = s.g16 + (size_t)j * s.Bp;
    f32x16 acc = {};
    for (int kk = 0; kk < s.Bp; kk += 16) {
        const int kc = kk + 8 * (lane >> 5);
        const V a = *reinterpret_cast<const V*>(gi + kc);
        const V b = *reinterpret_cast<const V*>(gj + kc);
        acc = F::mfma(a, b, acc);
    }
    return __shfl(acc[0], 0);
}

// Bounds on D2 implied by a 16-bit Gram value: ||g_i - g_j||^2 lies within
// kappa (N_i + N_j) of N_i + N_j - 2 G (FP32 accumulation), and the true mean
// difference lies within eta_i + eta_j of g_i - g_j.
__device__ void verify_gram16(const SecDev& s, int a, int b, float G, double fac, double& est, double& lower,
                              double& upper) {
    const double kappa = (2.0 * s.Bp + 64.0) * 0x1p-24;
    const double Ni = (double)s.gn[a], Nj = (double)s.gn[b];
    const double sh = Ni + Nj - 2.0 * (double)G;
    const double err = kappa * (Ni + Nj);
    const double eta = (double)s.geta[a] + (double)s.geta[b];
    const double rl = fmax(sqrt(fmax(sh - err, 0.0)) - eta, 0.0);
    const double rh = sqrt(fmax(sh + err, 0.0)) + eta;
    est = fac * fmax(sh, 0.0);
    lower = fac * rl * rl * (1.0 - 0x1p-40);
    upper = fac * rh * rh * (1.0 + 0x1p-40);
}

// Exact lexicographic minimum over the first n entries of the LDS candidate
// list. Adjacent mode: entries are edge indices; spectral mode: (i<<16)|j.
// dbg (HSWO_FLAG_DEBUG_VERIFY_BOUND): 0 off; 1 adjacent FP32 screen; 2
// spectral FP32 tiles; 3 / 4 the same plus the BF16 / FP16 matrix-core
// screen; R is the section's live region count.
__device__ KeyD exact_best_of_list(Smem& sh, const SecDev& s, int n, bool edge_mode, int dbg, int R) {
    KeyD best = key_none();
    for (int c = wave_id(); c < n; c += NWAVE) {
        const int ent = sh.u.f.cand[c];
        int a, b;
        if (edge_mode) {
            const int2 e = s.edges[ent];
            a = e.x;
            b = e.y;
        } else {
            a = (int)((unsigned)ent >> 16);
            b = (int)((unsigned)ent & 0xffffu);
        }
        int la = s.label[a], lb = s.label[b];
        if (la > lb) {
            const int t = a; a = b; b = t;
            const int u = la; la = lb; lb = u;
        }
        KeyD k;
        k.d2 = exact_d2_wave(sh, s, a, b);
        k.lo = la;
        k.hi = lb;
        k.si = a;
        k.sj = b;
        if (key_less(k, best)) best = k;
        if (dbg) {  // wavefront-uniform
            const float raw = dbg == 1 ? s.vraw[ent] : s.vstage[c];
            const float gam = (float)(2 * s.B + 32) * U32;
            const float2 lu = screen_bounds(raw, s.npix[a], s.npix[b], s.norm[a], s.norm[b], gam);
            const double na = (double)s.npix[a], nb = (double)s.npix[b];
            const double fac = (na * nb) / (na + nb);
            if (lane_id() == 0)
                verify_put(s, la, lb, dbg == 1 ? HSWO_SCREEN_ADJ_FP32 : HSWO_SCREEN_SPEC_FP32, R, fac * (double)raw,
                           (double)lu.x, (double)lu.y, k.d2);
            if (dbg >= 3) {
                const float G = dbg == 3 ? gram16_wave<1>(s, a, b) : gram16_wave<2>(s, a, b);
                double est, lower, upper;
                verify_gram16(s, a, b, G, fac, est, lower, upper);
                if (lane_id() == 0) verify_put(s, la, lb, HSWO_SCREEN_SPEC_16, R, est, lower, upper, k.d2);
            }
        }
    }
    return block_min_key(sh, best);
}

// Flush the candidate list into `best` when it is fuller than `keep_room`
// allows. Must be called by the whole block at a point where all appends of
// the current round are done.
__device__ void flush_candidates(Smem& sh, const SecDev& s, KeyD& best, int& nchk, bool edge_mode,
                                 int keep_room, int dbg, int R) {
    __syncthreads();
    const int n = sh.ncand;
    __syncthreads();  // every thread has read n before anyone appends again
    if (n > CAND_CAP - keep_room) {
        const int m = n < CAND_CAP ? n : CAND_CAP;
        const KeyD k = exact_best_of_list(sh, s, m, edge_mode, dbg, R);
        if (key_less(k, best)) best = k;
        nchk += m;
        if (threadIdx.x == 0) sh.ncand = 0;
        __syncthreads();
    }
}

// 64 x 64 FP32 spectral tile: thread (ty, tx) of 16 x 32 accumulates the
// 4 x 2 pairs rows ib*64+4ty+{0..3}, cols jb*64+2tx+{0,1}.
__device__ void tile_sums_fp32(Smem& sh, const SecDev& s, int ib, int jb, int R, float acc[4][2]) {
    const int tid = threadIdx.x;
    const int ty = tid >> 5, tx = tid & 31;
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a][0] = acc[a][1] = 0.0f;
    const int lrow = tid >> 3, lb = (tid & 7) << 2;
    const int ia = ib * TILE + lrow, ic = jb * TILE + lrow;
    for (int k0 = 0; k0 < s.Bp; k0 += BK) {
        float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vc = va;
        if (ia < R) va = *reinterpret_cast<const float4*>(s.mean + (size_t)ia * s.Bp + k0 + lb);
        if (ic < R) vc = *reinterpret_cast<const float4*>(s.mean + (size_t)ic * s.Bp + k0 + lb);
        sh.u.f.As[lb + 0][lrow] = va.x;
        sh.u.f.As[lb + 1][lrow] = va.y;
        sh.u.f.As[lb + 2][lrow] = va.z;
        sh.u.f.As[lb + 3][lrow] = va.w;
        sh.u.f.Cs[lb + 0][lrow] = vc.x;
        sh.u.f.Cs[lb + 1][lrow] = vc.y;
        sh.u.f.Cs[lb + 2][lrow] = vc.z;
        sh.u.f.Cs[lb + 3][lrow] = vc.w;
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < BK; ++kk) {
            const float4 a = *reinterpret_cast<const float4*>(&sh.u.f.As[kk][ty * 4]);
            const float2 c = *reinterpret_cast<const float2*>(&sh.u.f.Cs[kk][tx * 2]);
            float d;
            d = a.x - c.x; acc[0][0] = fmaf(d, d, acc[0][0]);
            d = a.x - c.y; acc[0][1] = fmaf(d, d, acc[0][1]);
            d = a.y - c.x; acc[1][0] = fmaf(d, d, acc[1][0]);
            d = a.y - c.y; acc[1][1] = fmaf(d, d, acc[1][1]);
            d = a.z - c.x; acc[2][0] = fmaf(d, d, acc[2][0]);
            d = a.z - c.y; acc[2][1] = fmaf(d, d, acc[2][1]);
            d = a.w - c.x; acc[3][0] = fmaf(d, d, acc[3][0]);
            d = a.w - c.y; acc[3][1] = fmaf(d, d, acc[3][1]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 16-bit matrix-core screen of the spectral stage (precision forms).
//
// Rows are centred by a section-wide spectrum c and rounded to 16 bits:
// g_i = round16(fl32(m_i - c)). With N_i = ||g_i||^2 and G_ij = g_i . g_j,
// ||g_i - g_j||^2 = N_i + N_j - 2 G_ij, and the true mean difference d_ij
// satisfies | ||d_ij|| - ||g_i - g_j|| | <= eta_i + eta_j, where eta_i bounds
// ||g_i - (mu_i - c)||: 16-bit rounding u16 ||m_i - c||, the FP32 centring
// rounding, the FP32 mean rounding ~u32 ||m_i||, and sub-normal spacing.
//
// D2 = n_i n_j/(n_i+n_j) ||d||^2 < T implies ||d|| < sqrt(T/n_i + T/n_j)
// <= sqrt(T/n_i) + sqrt(T/n_j), hence ||g_i - g_j|| < alpha_i + alpha_j with
// alpha_i = sqrt(T/n_i) + eta_i. With the FP32 accumulation error of the
// matrix core and of the combination bounded by kappa (N_i + N_j), every pair
// with D2 < T satisfies
//     (1-kappa)(N_i + N_j) - (alpha_i + alpha_j)^2 < 2 G_ij,
// i.e. P_i + P_j - 2 alpha_i alpha_j < 2 G_ij with P_i = (1-kappa) N_i - alpha_i^2
// (rounded down) and alpha rounded up. A 64 x 64 tile in which no pair passes
// this test holds no pair that can beat T, so only the tiles that pass go on
// to the FP32 screen and the FP64 re-check: the merge chosen is unchanged.
// ---------------------------------------------------------------------------

// One wavefront rebuilds the 16-bit row of slot i and its N and eta.
template <int PREC>
__device__ void row16(const SecDev& s, int i) {
    typedef Fmt16<PREC> F;
    const int lane = lane_id();
    const float* m = s.mean + (size_t)i * s.Bp;
    uint16_t* g = s.g16 + (size_t)i * s.Bp;
    double sq = 0.0, an = 0.0, mn = 0.0;
    for (int b = lane; b < s.Bp; b += 64) {
        const float mv = m[b];
        const float ac = mv - s.cvec[b];
        const uint16_t hv = F::enc(ac);
        const double gv = (double)F::dec(hv);
        g[b] = hv;
        sq += gv * gv;
        an += (double)ac * (double)ac;
        mn += (double)mv * (double)mv;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        sq += __shfl_xor(sq, o);
        an += __shfl_xor(an, o);
        mn += __shfl_xor(mn, o);
    }
    if (lane == 0) {
        s.gn[i] = (float)sq;
        const double eta = (F::U + 0x1p-23) * sqrt(an) + 0x1.02p-24 * sqrt(mn) + F::SUB * sqrt((double)s.Bp);
        s.geta[i] = (float)(eta * (1.0 + 0x1p-20));
    }
}

// When the spectral stage starts: fix the centring spectrum (band means of
// the live rows) and build every live row.
template <int PREC>
__device__ void build16_all(const SecDev& s, int R) {
    const int tid = threadIdx.x;
    for (int b = tid; b < s.Bp; b += NT) {
        double acc = 0.0;
        for (int i = 0; i < R; ++i) acc += (double)s.mean[(size_t)i * s.Bp + b];
        s.cvec[b] = b < s.B ? (float)(acc / (double)R) : 0.0f;
    }
    __syncthreads();
    for (int i = wave_id(); i < R; i += NWAVE) row16<PREC>(s, i);
    __syncthreads();
}

// Per-iteration row terms of the tile test for threshold T.
__device__ void prep_alpha_p(const SecDev& s, int R, double T) {
    const double kappa = (2.0 * s.Bp + 64.0) * 0x1p-24;
    for (int i = threadIdx.x; i < R; i += NT) {
        const double a = (sqrt(T / (double)s.npix[i]) + (double)s.geta[i]) * (1.0 + 0x1p-20);
        const float af = (float)(a * (1.0 + 0x1p-22));
        const double P = (1.0 - kappa) * (double)s.gn[i] - (double)af * (double)af * (1.0 + 0x1p-20);
        s.galpha[i] = af;
        s.gP[i] = (float)(P - fabs(P) * 0x1p-21);
    }
    __syncthreads();
}

__device__ __forceinline__ int tile_index(int ib, int jb, int nT) { return ib * nT - ib * (ib - 1) / 2 + (jb - ib); }

__device__ __forceinline__ void tile_coords(int t, int nT, int& ib, int& jb) {
    ib = 0;
    int len = nT;
    while (t >= len) {
        t -= len;
        ++ib;
        --len;
    }
    jb = ib + t;
}

// Matrix-core pass over the 128 x 128 super tiles q = g0, g0 + gstride, ...
// of pairs i < j < R: sets tflag of every 64 x 64 tile holding a pair that
// passes the test above (flags are cleared beforehand).
// Wave w computes rows 32*(w>>1) .. +31 and columns 64*(w&1) .. +63 of the
// super tile, which lie in exactly one 64 x 64 tile.
template <int PREC>
__device__ int mfma_screen(Smem& sh, const SecDev& s, int R, int g0, int gstride) {
    typedef Fmt16<PREC> F;
    typedef typename F::V V;
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    const int wi = w >> 1, wj = w & 1;
    const int nT = (R + TILE - 1) / TILE, nS = (R + STILE - 1) / STILE;
    const int Bp = s.Bp;
    const int nslab = (Bp + KSLAB - 1) / KSLAB;
    int nsup = 0, q = 0;
    for (int IB = 0; IB < nS; ++IB) {
        bool a_ready = false;  // the row block stays in LDS across this row of super tiles
        for (int JB = IB; JB < nS; ++JB, ++q) {
            if (q < g0 || (q - g0) % gstride != 0) continue;  // block-uniform
            ++nsup;
            f32x16 acc0 = {}, acc1 = {};
            for (int sl = 0; sl < nslab; ++sl) {
                const int k0 = sl * KSLAB;
                const int kw = min(KSLAB, Bp - k0);  // a multiple of 32
                const int segs = kw >> 3;           // 16-byte segments per row
                __syncthreads();  // previous reads of the LDS tiles are done
                if (!a_ready) {
                    for (int idx = tid; idx < STILE * segs; idx += NT) {
                        const int r = idx / segs, sg = idx % segs;
                        const int gr = IB * STILE + r;
                        uint4 v = make_uint4(0u, 0u, 0u, 0u);
                        if (gr < R) v = *reinterpret_cast<const uint4*>(s.g16 + (size_t)gr * Bp + k0 + sg * 8);
                        *reinterpret_cast<uint4*>(&sh.u.g.A[r][sg * 8]) = v;
                    }
                    if (tid < STILE) {
                        const int r = IB * STILE + tid;
                        sh.u.g.Prow[tid] = r < R ? s.gP[r] : 0.0f;
                        sh.u.g.Arow[tid] = r < R ? s.galpha[r] : 0.0f;
                    }
                }
                for (int idx = tid; idx < STILE * segs; idx += NT) {
                    const int r = idx / segs, sg = idx % segs;
                    const int gc = JB * STILE + r;
                    uint4 v = make_uint4(0u, 0u, 0u, 0u);
                    if (gc < R) v = *reinterpret_cast<const uint4*>(s.g16 + (size_t)gc * Bp + k0 + sg * 8);
                    *reinterpret_cast<uint4*>(&sh.u.g.C[r][sg * 8]) = v;
                }
                if (sl == 0 && tid >= STILE && tid < 2 * STILE) {
                    const int c = JB * STILE + tid - STILE;
                    sh.u.g.Pcol[tid - STILE] = c < R ? s.gP[c] : 0.0f;
                    sh.u.g.Acol[tid - STILE] = c < R ? s.galpha[c] : 0.0f;
                }
                __syncthreads();
                for (int kk = 0; kk < kw; kk += 16) {
                    const int kc = kk + 8 * (lane >> 5);
                    const V a = *reinterpret_cast<const V*>(&sh.u.g.A[32 * wi + (lane & 31)][kc]);
                    const V b0 = *reinterpret_cast<const V*>(&sh.u.g.C[64 * wj + (lane & 31)][kc]);
                    const V b1 = *reinterpret_cast<const V*>(&sh.u.g.C[64 * wj + 32 + (lane & 31)][kc]);
                    acc0 = F::mfma(a, b0, acc0);
                    acc1 = F::mfma(a, b1, acc1);
                }
                a_ready = (nslab == 1);
            }
            bool any = false;
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
                const int jl = 64 * wj + 32 * sb + (lane & 31);
                const int gj = JB * STILE + jl;
                const float Pj = sh.u.g.Pcol[jl], Aj = sh.u.g.Acol[jl];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int il = 32 * wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int gi = IB * STILE + il;
                    const float g2 = 2.0f * (sb ? acc1[r] : acc0[r]);
                    const float t = fmaf(-2.0f * sh.u.g.Arow[il], Aj, sh.u.g.Prow[il] + Pj);
                    any = any || (gi < gj && gj < R && t < g2);
                }
            }
            const unsigned long long ball = __ballot(any);
            if (lane == 0 && ball) {
                const int ti = 2 * IB + (wi >> 1), tj = 2 * JB + wj;
                if (ti <= tj && tj < nT) s.tflag[tile_index(ti, tj, nT)] = 1;
            }
        }
    }
    __syncthreads();
    return nsup;
}

// One merge (Section 4.1: the merged region replaces both). lo_s keeps the
// region; the slot hi_s is freed and the last live slot R-1 moves into it.
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
// (exact_wave_means, one wavefront per pair) -- except pairs bounded by
// [0, 0], whose canonical value is 0 -- and their bounds tightened to the
// exact value. The row's least two go to its first chunk entry of rpart and
// +inf to the others, which is what the exact row tasks leave for the
// decision to reduce. Returns the number of exact evaluations (thread 0).
__device__ int row_matrix_task(RowMatLds& L, const SecDev& s, int R, int q, bool all) {
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

// Statistics part of a merge (HSEG step 4): the survivor lo takes hi's band
// sums and pixel count; its FP32 screen row (and 16-bit row, FP64 mean
// copies) are refreshed; union-find parent, merge time and log record.
// rc: row cache state of the section (0 off, 1 or 2 means maintained).
// screens: keep the FP32 mean row and its norm bound current (the screened
// and plain forms read them; the incremental form does not).
__device__ void merge_stats(Smem& sh, const SecDev& s, int lo_s, int hi_s, int R, int kind, double d2, int g_ready,
                            int prec, int rc, bool screens, bool mat, int stamp) {
    const int tid = threadIdx.x;
    const int B = s.B, Bp = s.Bp;
    const int lo_l = s.label[lo_s], hi_l = s.label[hi_s];
    const int n_new = s.npix[lo_s] + s.npix[hi_s];
    const double dn = (double)n_new;
    double* Slo = s.sums + (size_t)lo_s * B;
    const double* Shi = s.sums + (size_t)hi_s * B;
    float* Mlo = s.mean + (size_t)lo_s * Bp;
    double nrm = 0.0;
    for (int b = tid; b < B; b += NT) {
        const double v = Slo[b] + Shi[b];
        Slo[b] = v;
        if (rc) {
            const double m = s.crit == HSWO_CRIT_SAM ? v : v / dn;
            if (!mat) s.m64[(size_t)b * s.rcap + lo_s] = m;
            s.m64r[(size_t)lo_s * ((B + 7) & ~7) + b] = m;
        }
        if (screens) {
            const float m = (float)(v / dn);
            Mlo[b] = m;
            nrm += (double)m * (double)m;
        }
    }
    if (screens)
        nrm = block_sum_d(sh, nrm);  // contains barriers: all reads of s.npix done
    else
        __syncthreads();  // all reads of s.npix done
    if (rc && s.crit == HSWO_CRIT_SAM && wave_id() == 1) {  // the survivor's squared norm (sums written above)
        const double q = wave_dot_tree(Slo, Slo, B);
        if (lane_id() == 0) s.rq[lo_s] = q;
    }
    if (g_ready && wave_id() == 0) {  // keep the survivor's 16-bit screen row current
        if (prec == 1)
            row16<1>(s, lo_s);
        else
            row16<2>(s, lo_s);
    }
    if (tid == 0) {
        s.npix[lo_s] = n_new;
        if (screens) s.norm[lo_s] = (float)(sqrt(nrm) * (1.0 + 0x1p-20));
        s.parent[hi_l] = lo_l;
        const int k = stamp;  // the section's merge count (st[3])
        s.mtime[hi_l] = s.top ? k : -1;
        if (s.log) {
            hswo_merge_rec rec;
            rec.lo = lo_l;
            rec.hi = hi_l;
            rec.kind = kind;
            rec.r_after = R - 1;
            rec.d2 = d2;
            s.log[k] = rec;
        }
        s.st[3] = k + 1;
    }
}

// Edge list part of a merge, by a full pass: relabel hi -> lo, drop the
// merged pair and duplicate (lo, x) edges, rename the moved slot, compact in
// place (writes never pass reads). With inc the cached D2 moves along, and
// the edges that touch the survivor are listed in edirty (count in
// sh.bcast_i[2]) for re-scoring.
__device__ void merge_edges_full(Smem& sh, const SecDev& s, int lo_s, int hi_s, int R, int& E, int stamp, bool inc) {
    const int tid = threadIdx.x;
    // mark the neighbours of the survivor
    for (int e = tid; e < E; e += NT) {
        const int2 ed = s.edges[e];
        if (ed.x == lo_s) s.mark[ed.y] = stamp;
        if (ed.y == lo_s) s.mark[ed.x] = stamp;
    }
    __syncthreads();
    const int last = R - 1;
    const int surv = (lo_s == last) ? hi_s : lo_s;  // the survivor's slot after the swap-remove
    if (tid == 0) sh.bcast_i[2] = 0;
    int newE = 0;
    for (int e0 = 0; e0 < E; e0 += NT) {
        const int e = e0 + tid;
        bool keep = false;
        int a = 0, b = 0;
        double v = 0.0;
        if (e < E) {
            if (inc) v = s.ed2[e];
            const int2 ed = s.edges[e];
            a = ed.x;
            b = ed.y;
            const bool hi_edge = (a == hi_s) || (b == hi_s);
            if (a == hi_s) a = lo_s;
            if (b == hi_s) b = lo_s;
            keep = (a != b);
            if (keep && hi_edge) {
                const int other = (a == lo_s) ? b : a;
                if (s.mark[other] == stamp) keep = false;
            }
            if (a == last) a = hi_s;
            if (b == last) b = hi_s;
        }
        int tot;
        const int pos = block_scan_flag(sh, keep, &tot);  // barrier: chunk fully read
        if (keep) {
            s.edges[newE + pos] = make_int2(a, b);
            if (inc) {
                s.ed2[newE + pos] = v;
                if (a == surv || b == surv) s.edirty[atomicAdd(&sh.bcast_i[2], 1)] = newE + pos;
            }
        }
        newE += tot;
    }
    E = newE;
    __syncthreads();
}

// Slot part of a merge: swap-remove (the last live slot moves into the freed
// one) and, with the row cache (rc == 2), the row entries: the moved row's
// entries follow it, partners that moved are renamed, and the survivor and
// every row whose cached partner was one of the merged pair are listed for a
// full evaluation (rpend, count in st[7] and sh.npend) -- or, a row whose
// second bound's partner is alive, marked for a light step (rbp = -2), which
// the survivor's row evaluation takes. Kept out of line: inlined, it pushes
// the decision kernel into scratch.
// mat: the row cache keeps the interval matrix (rc == 2); d2 is the merged
// pair's canonical value. The survivor's bounds row comes from Ward's update
// of its and the merged region's matrix rows; matrix rows are indexed
// through msl, so moving a slot moves no matrix entry.
__device__ __noinline__ void merge_slots(Smem& sh, const SecDev& s, int lo_s, int hi_s, int R, int g_ready, int rc,
                                         bool screens, bool mat, double d2) {
    const int tid = threadIdx.x;
    const int B = s.B, Bp = s.Bp;
    const int last = R - 1;
    const int surv = (lo_s == last) ? hi_s : lo_s;
    if (mat && rc == 2) {
        // the survivor keeps matrix row ml (its row and column rewritten in place: every thread
        // reads and writes its own entries of row ml, and no column it writes is read); row mh
        // is dropped, and the slot that moves takes its matrix row along (below)
        const size_t rcp = (size_t)s.mstride;
        const float2 de = mat_entry(d2);
        const double n_hi = (double)s.npix[hi_s];
        const double n_lo = (double)s.npix[lo_s] - n_hi;  // merge_stats has added n_hi to the survivor
        const int ml = s.msl[lo_s], mh = s.msl[hi_s];
        float2* Dl = s.dmat + (size_t)ml * rcp;
        const float2* Dh = s.dmat + (size_t)mh * rcp;
        for (int k = tid; k < R; k += NT) {
            if (k == lo_s || k == hi_s) continue;
            const int mk = s.msl[k];
            const float2 v = mat_update(Dl[mk], Dh[mk], (double)de.x, (double)de.y, n_lo, n_hi, (double)s.npix[k]);
            Dl[mk] = v;
            s.dmat[(size_t)mk * rcp + ml] = v;
        }
        __syncthreads();  // every read of npix and msl above is done before the slot moves below
        if (tid == 0) {
            if (lo_s == last) s.msl[hi_s] = ml;          // the survivor moves into hi_s
            else if (hi_s != last) s.msl[hi_s] = s.msl[last];
        }
    }
    if (hi_s != last) {
        const double* Ssrc = s.sums + (size_t)last * B;
        double* Sdst = s.sums + (size_t)hi_s * B;
        for (int b = tid; b < B; b += NT) Sdst[b] = Ssrc[b];
        if (screens) {
            const float* Msrc = s.mean + (size_t)last * Bp;
            float* Mdst = s.mean + (size_t)hi_s * Bp;
            for (int b = tid; b < Bp; b += NT) Mdst[b] = Msrc[b];
        }
        if (tid == 0) {
            s.label[hi_s] = s.label[last];
            s.npix[hi_s] = s.npix[last];
            if (screens) s.norm[hi_s] = s.norm[last];
            s.mark[hi_s] = s.mark[last];
        }
        if (rc) {
            const size_t kc = (size_t)s.rcap, B8 = (size_t)((B + 7) & ~7);
            for (int b = tid; b < B; b += NT) {
                if (!mat) s.m64[(size_t)b * kc + hi_s] = s.m64[(size_t)b * kc + last];
                s.m64r[(size_t)hi_s * B8 + b] = s.m64r[(size_t)last * B8 + b];
            }
            if (s.crit == HSWO_CRIT_SAM && tid == 0) s.rq[hi_s] = s.rq[last];
        }
        if (g_ready) {
            const uint16_t* Gsrc = s.g16 + (size_t)last * Bp;
            uint16_t* Gdst = s.g16 + (size_t)hi_s * Bp;
            for (int b = tid; b < Bp; b += NT) Gdst[b] = Gsrc[b];
            if (tid == 0) {
                s.gn[hi_s] = s.gn[last];
                s.geta[hi_s] = s.geta[last];
            }
        }
    }
    if (rc == 2) {
        if (tid == 0) sh.npend = 1;
        __syncthreads();
        for (int i = tid; i < R; i += NT) {
            if (i == lo_s || i == hi_s) continue;
            const int ni = (i == last) ? hi_s : i;
            const int p = s.rbp[i];
            // the second bound follows a moved partner; when its partner is merged it stays as a
            // bare bound (-3) by default only if its value is 0 (identical spectra, where the
            // merged region usually ties again), else it is dropped (the interval matrix keeps
            // no second bounds)
            int np2 = -1;
            if (!mat) {
                const int p2 = s.rbp2[i];
                np2 = p2 == last ? hi_s : p2;
                if (p2 == lo_s || p2 == hi_s)  // the value is read only here
                    np2 = (s.bare == 2 || (s.bare == 1 && s.rbd2[i] == 0.0)) ? -3 : -1;
                if (ni != i) {
                    s.rbd2[ni] = s.rbd2[i];
                    s.rbl2[ni] = s.rbl2[i];
                }
                if (ni != i || np2 != p2) s.rbp2[ni] = np2;
            }
            if (p == lo_s || p == hi_s) {
                // stale: a light step (marked -2) when it has a second bound, else a full evaluation
                // (with the interval matrix always the rescan of its bounds row)
                if (np2 != -1 && !mat) {
                    s.rbp[ni] = -2;
                } else {
                    s.rbp[ni] = -1;
                    s.rpend[atomicAdd(&sh.npend, 1)] = ni;
                }
            } else {
                // only a moved row or a moved partner changes the entry
                const int np = (p == last) ? hi_s : p;
                if (ni != i) {
                    s.rbd[ni] = s.rbd[i];
                    s.rbl[ni] = s.rbl[i];
                }
                if (ni != i || np != p) s.rbp[ni] = np;
            }
        }
        if (tid == 0) {
            s.rpend[0] = surv;
            s.rbp[surv] = -1;
        }
        __syncthreads();
        if (tid == 0) {
            s.st[7] = sh.npend;
            s.st[11] = 0;  // rows the light steps will append
        }
    }
    __syncthreads();
}

// Merge of (lo_s, hi_s) (HSEG step 4). rc: row cache state (0 off, 1 means
// maintained, 2 rows maintained).
__device__ __forceinline__ void merge_pair(Smem& sh, const SecDev& s, int lo_s, int hi_s, int R, int& E, int stamp,
                           int kind, double d2, int g_ready, int prec, int rc) {
    merge_stats(sh, s, lo_s, hi_s, R, kind, d2, g_ready, prec, rc, true, false, stamp);
    const bool inc = s.ed2 != nullptr && s.st[5] != 0;
    merge_edges_full(sh, s, lo_s, hi_s, R, E, stamp, inc);
    merge_slots(sh, s, lo_s, hi_s, R, g_ready, rc, true, false, 0.0);
    if (inc) {  // re-score the survivor's edges; every other edge keeps its cached value
        const int nd = sh.bcast_i[2];
        score_edges(sh, s, s.edirty, nd);
        __syncthreads();
    }
}

// Remove the empty slots (-1, -1) of the edge list, keeping order, with the
// cached D2 moving along.
__device__ void compact_edges(Smem& sh, const SecDev& s, int& E) {
    int newE = 0;
    for (int e0 = 0; e0 < E; e0 += NT) {
        const int e = e0 + threadIdx.x;
        bool keep = false;
        int2 ed = make_int2(-1, -1);
        double v = 0.0;
        if (e < E) {
            ed = s.edges[e];
            v = s.ed2[e];
            keep = ed.x >= 0;
        }
        int tot;
        const int pos = block_scan_flag(sh, keep, &tot);  // barrier: chunk fully read
        if (keep) {
            s.edges[newE + pos] = ed;
            s.ed2[newE + pos] = v;
        }
        newE += tot;
    }
    E = newE;
    __syncthreads();
}

// Edge index of the incremental form: for every live slot the range
// [rmin, rmax] of edge slots that can touch it (conservative: a merge gives
// the survivor the union of both ranges, a moving slot keeps its range), and
// for every chunk of ECH edge slots the least key (D2, lo, hi) of its cached
// values (cmd2, cme: value and edge slot, -1 for none). Rebuilt from scratch
// when st[12] is 0 (pass start, compaction).

// Least key of chunk c into cmd2[c] / cme[c]; one wavefront.
__device__ void chunk_min_wave(const SecDev& s, int c, int E) {
    // the chunk's values at once, their least over the wavefront, then the labels of only the
    // slots that hold it (one round of loads each, whatever the chunk holds)
    const int lane = lane_id();
    constexpr int PER = ECH / 64;
    double v[PER];
    double m = __builtin_huge_val();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = c * ECH + k * 64 + lane;
        v[k] = e < E ? s.ed2[e] : __builtin_huge_val();
        m = fmin(m, v[k]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmin(m, __shfl_xor(m, o));
    KeyD best = key_none();
    if (m < __builtin_huge_val()) {  // wavefront-uniform
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (v[k] != m) continue;
            const int e = c * ECH + k * 64 + lane;
            const int2 ed = s.edges[e];
            const int la = s.label[ed.x], lb = s.label[ed.y];
            KeyD kk;
            kk.d2 = m;
            kk.lo = min(la, lb);
            kk.hi = max(la, lb);
            kk.si = 2 * e + (la > lb ? 1 : 0);  // the edge slot rides in si, with which end is lo
            kk.sj = 0;
            if (key_less(kk, best)) best = kk;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const KeyD x = shfl_key(best, o);
        if (key_less(x, best)) best = x;
    }
    if (lane == 0) {
        s.cmd2[c] = best.d2;
        s.cme[c] = key_exists(best) ? best.si : -1;
        s.cml[c] = make_int2(best.lo, best.hi);
    }
}

// Ranges and chunk minima from scratch (st[12] = 1 after); whole block.
__device__ __noinline__ void edge_index_build(const SecDev& s, int R, int E) {
    for (int i = threadIdx.x; i < R; i += NT) {
        s.rmin[i] = INT_MAX;
        s.rmax[i] = -1;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < E; e += NT) {
        const int2 ed = s.edges[e];
        if (ed.x >= 0) {
            atomicMin(&s.rmin[ed.x], e);
            atomicMax(&s.rmax[ed.x], e);
            atomicMin(&s.rmin[ed.y], e);
            atomicMax(&s.rmax[ed.y], e);
        }
    }
    for (int c = wave_id(); c < (E + ECH - 1) / ECH; c += NWAVE) chunk_min_wave(s, c, E);
    __syncthreads();
    if (threadIdx.x == 0) s.st[12] = 1;
    __syncthreads();
}

// The least adjacent key over every chunk's minimum, with its slots; whole block.
__device__ KeyD chunks_min_key(Smem& sh, const SecDev& s, int E) {
    // each chunk's record holds its least key's labels: one round of loads, then the winner's
    // slots from its edge
    KeyD best = key_none();
    for (int c = threadIdx.x; c < (E + ECH - 1) / ECH; c += NT) {
        const int e2 = s.cme[c];
        const double d2 = s.cmd2[c];
        const int2 lab = s.cml[c];
        if (e2 < 0) continue;
        KeyD k;
        k.d2 = d2;
        k.lo = lab.x;
        k.hi = lab.y;
        k.si = e2;
        k.sj = 0;
        if (key_less(k, best)) best = k;
    }
    best = block_min_key(sh, best);
    if (key_exists(best)) {
        const int2 ed = s.edges[best.si >> 1];
        const bool flip = (best.si & 1) != 0;  // the edge's second end is lo
        best.si = flip ? ed.y : ed.x;
        best.sj = flip ? ed.x : ed.y;
    }
    return best;
}

constexpr int LCAP = CAND_CAP / 3;  // edges listed per merge by the incremental form (L, L2, neighbours)

// The index path of merge_pair_inc's edge listing: the edges touching the
// merged pair go to L (their other endpoint to XL), those touching the slot
// that moves to L2, scanning only the chunks of the slot ranges; the ranges
// and the first chunk range go to sh.idx (ua, ub, ma, mb, a0, a1). Whole
// block, ends with a barrier.
__device__ __noinline__ void merge_index_scan(Smem& sh, const SecDev& s, int lo_s, int hi_s, int R, int E, int* L,
                                              int* XL, int* L2) {
    const int last = R - 1;
    const bool moved = last != lo_s && last != hi_s;
    // the index's state and the three slots' ranges in one round of loads (the ranges are read
    // again after a rebuild)
    const int valid = s.st[12];
    int ua = min(s.rmin[lo_s], s.rmin[hi_s]);
    int ub = max(s.rmax[lo_s], s.rmax[hi_s]);
    int ma = moved ? s.rmin[last] : INT_MAX;
    int mb = moved ? s.rmax[last] : -1;
    if (valid == 0) {  // block-uniform
        edge_index_build(s, R, E);
        ua = min(s.rmin[lo_s], s.rmin[hi_s]);
        ub = max(s.rmax[lo_s], s.rmax[hi_s]);
        ma = moved ? s.rmin[last] : INT_MAX;
        mb = moved ? s.rmax[last] : -1;
    }
    const int tid = threadIdx.x;
    int a0 = 0, a1 = 0, b0 = 0, b1 = 0;  // chunk-aligned [a0, a1) and [b0, b1)
    if (ua <= ub) {
        a0 = (ua / ECH) * ECH;
        a1 = min(E, (ub / ECH + 1) * ECH);
    }
    if (ma <= mb) {
        b0 = (ma / ECH) * ECH;
        b1 = min(E, (mb / ECH + 1) * ECH);
    }
    for (int pass = 0; pass < 2; ++pass) {  // block-uniform
        const int r0 = pass ? b0 : a0, r1 = pass ? b1 : a1;
        for (int e = r0 + tid; e < r1; e += NT) {
            if (pass && e >= a0 && e < a1) continue;  // scanned in the first pass
            const int2 ed = s.edges[e];
            const int a = ed.x, b = ed.y;
            if (a < 0) continue;
            const bool ta = a == lo_s || a == hi_s, tb = b == lo_s || b == hi_s;
            if (ta || tb) {
                const int k = atomicAdd(&sh.bcast_i[0], 1);
                if (k < LCAP) {
                    L[k] = e;
                    XL[k] = (ta && tb) ? -1 : (ta ? b : a);
                }
            } else if (a == last || b == last) {
                const int k = atomicAdd(&sh.bcast_i[1], 1);
                if (k < LCAP) L2[k] = e;
            }
        }
    }
    if (tid == 0) {
        sh.idx[0] = ua;
        sh.idx[1] = ub;
        sh.idx[2] = ma;
        sh.idx[3] = mb;
        sh.idx[4] = a0;
        sh.idx[5] = a1;
        sh.idx[6] = (a1 - a0) + (b1 - b0) - max(0, min(a1, b1) - max(a0, b0));  // slots scanned
        sh.idx[7] = 0;                                                          // chunks re-minimised
    }
    __syncthreads();
}

// The index path's end of a merge: the chunk minima taken anew of the chunks
// that hold an edge the merge changed -- the edges it listed in L (nL of
// them, all inside [a0, a1)), whose chunks are flagged in LDS; the renamed
// edges of the moved slot keep their keys -- then the survivor's and the
// moved slot's ranges, and the least key over all chunks. A chunk range too
// long for the flags takes every chunk of [a0, a1) anew.
__device__ __noinline__ KeyD merge_index_finish(Smem& sh, const SecDev& s, int a0, int a1, int surv, int hi_s,
                                                bool moved, int ua, int ub, int ma, int mb, int E, const int* L,
                                                int nL) {
    constexpr int FLAG_WORDS = (int)(sizeof(sh.u.f.As) / sizeof(unsigned));
    const int c0 = a0 / ECH, c1 = (a1 + ECH - 1) / ECH;
    const int nw = (c1 - c0 + 31) >> 5;
    const bool flagged = nw <= FLAG_WORDS;  // block-uniform
    unsigned* fl = reinterpret_cast<unsigned*>(&sh.u.f.As[0][0]);  // free during a merge
    if (flagged)
        for (int w = threadIdx.x; w < nw; w += NT) fl[w] = 0u;
    __syncthreads();  // the re-scored values are written, the flags cleared
    if (flagged) {
        for (int k = threadIdx.x; k < nL; k += NT) {
            const int c = L[k] / ECH - c0;
            atomicOr(&fl[c >> 5], 1u << (c & 31));
        }
        __syncthreads();
    }
    for (int c = c0 + wave_id(); c < c1; c += NWAVE)  // wavefront-uniform
        if (!flagged || ((fl[(c - c0) >> 5] >> ((c - c0) & 31)) & 1u)) {
            chunk_min_wave(s, c, E);
            if (lane_id() == 0) atomicAdd(&sh.idx[7], 1);
        }
    __syncthreads();  // the chunk count is complete
    if (threadIdx.x == 0) {
        s.rmin[surv] = ua;
        s.rmax[surv] = ub;
        if (moved) {
            s.rmin[hi_s] = ma;
            s.rmax[hi_s] = mb;
        }
        // read: the scanned slots, the re-minimised chunks' slots and every chunk record
        sh.eread = sh.idx[6] + sh.idx[7] * ECH + (E + ECH - 1) / ECH;
    }
    __syncthreads();
    return chunks_min_key(sh, s, E);
}



// Merge in the incremental form (every edge slot holds its exact D2). One
// pass over the edge slots lists the edges that touch the merged pair (L)
// and those that touch the slot that will move (L2), and takes the least key
// over every edge not in L, whose D2 cannot change. Only the listed edges are
// then rewritten: one edge per neighbour x of the merged pair becomes
// (survivor, x) and is re-scored, the others become empty slots; the edge
// list is compacted when a quarter of it is empty, and at the last merge of a
// pass. Returns true with the least adjacent key after the merge in anext;
// false (full pass taken) when a list would overflow.
template <int U>
// eidx_min: edge lists at least this long go through the edge index (the
// persistent driver, whose merges follow one another in one launch, gains
// from it at any length; a wide-mode decision launch only on long lists).
__device__ __forceinline__ bool merge_pair_inc(Smem& sh, const SecDev& s, int lo_s, int hi_s, int R, int& E, int stamp, int kind,
                               double d2, int rc, KeyD& anext, int& nchk, bool mat, int eidx_min, int& empty_slots) {
    const int tid = threadIdx.x;
    const int l_surv = s.label[lo_s];  // the survivor's label, whichever slot it ends in
    merge_stats(sh, s, lo_s, hi_s, R, kind, d2, 0, 0, rc, false, mat, stamp);
    const int last = R - 1;
    const int surv = (lo_s == last) ? hi_s : lo_s;
    int* L = sh.u.f.cand;
    int* L2 = sh.u.f.cand + LCAP;
    int* XL = sh.u.f.cand + 2 * LCAP;  // per edge of L: its other endpoint (-1: the merged pair itself)
    if (tid == 0) {
        sh.bcast_i[0] = 0;  // |L|
        sh.bcast_i[1] = 0;  // |L2|
        sh.bcast_i[2] = 0;  // kept edges
        sh.bcast_i[3] = 0;  // emptied slots
        sh.eread = E;       // a pass over every slot (the index path counts its own)
    }
    __syncthreads();
    // A long edge list goes through its index: every edge that touches the
    // merged pair lies in the union of their slot ranges, every edge of the
    // slot that moves in its range, so only the chunks of those ranges are
    // scanned; the next adjacent minimum is then the least of the chunk
    // minima, those of the changed chunks taken anew. A short list takes one
    // pass over every slot, which also yields the least key of the edges the
    // merge cannot change (the index is then rebuilt when it is next used).
    const bool use_index = E >= eidx_min;  // block-uniform
    const bool moved = last != lo_s && last != hi_s;
    int ua = 0, ub = -1, ma = INT_MAX, mb = -1;
    int a0 = 0, a1 = 0;  // the first chunk range the index path scanned
    double vmin = __builtin_huge_val();
    double bv = __builtin_huge_val();
    int be = -1;
    if (use_index) {
        merge_index_scan(sh, s, lo_s, hi_s, R, E, L, XL, L2);
        ua = sh.idx[0];
        ub = sh.idx[1];
        ma = sh.idx[2];
        mb = sh.idx[3];
        a0 = sh.idx[4];
        a1 = sh.idx[5];
    } else {
        // least cached D2 of this thread's edges that do not touch the merged pair
        // (labels are read only to order exact ties inside the thread)
        int bla = 0, blb = 0;
        // U: pairs of edge slots per thread with loads in flight together
        for (int e0 = 2 * tid; e0 < E; e0 += 2 * NT * U) {
            int4 ed[U];
            double2 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * 2 * NT;
                ed[u] = make_int4(-1, -1, -1, -1);
                v[u] = make_double2(__builtin_huge_val(), __builtin_huge_val());
                if (e + 1 < E) {
                    ed[u] = *reinterpret_cast<const int4*>(s.edges + e);
                    v[u] = *reinterpret_cast<const double2*>(s.ed2 + e);
                } else if (e < E) {
                    const int2 x = s.edges[e];
                    ed[u] = make_int4(x.x, x.y, -1, -1);
                    v[u].x = s.ed2[e];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = e0 + u * 2 * NT + h;
                    const int a = h ? ed[u].z : ed[u].x, b = h ? ed[u].w : ed[u].y;
                    const double vv = h ? v[u].y : v[u].x;
                    const bool ta = a == lo_s || a == hi_s, tb = b == lo_s || b == hi_s;
                    const bool touch = ta || tb;
                    if (a >= 0 && touch) {
                        const int k = atomicAdd(&sh.bcast_i[0], 1);
                        if (k < LCAP) {
                            L[k] = e;
                            XL[k] = (ta && tb) ? -1 : (ta ? b : a);
                        }
                    }
                    if (a >= 0 && !touch && (a == last || b == last)) {
                        const int k = atomicAdd(&sh.bcast_i[1], 1);
                        if (k < LCAP) L2[k] = e;
                    }
                    if (a >= 0 && !touch) {
                        if (vv < bv) {
                            bv = vv;
                            be = e;
                            bla = -1;  // labels not loaded
                        } else if (vv == bv && vv < __builtin_huge_val()) {
                            // exact tie: order by (lo, hi) labels
                            if (bla < 0) {
                                const int2 x = s.edges[be];
                                const int p = s.label[x.x], q = s.label[x.y];
                                bla = min(p, q);
                                blb = max(p, q);
                            }
                            const int p = s.label[a], q = s.label[b];
                            const int lo = min(p, q), hi = max(p, q);
                            if (lo < bla || (lo == bla && hi < blb)) {
                                be = e;
                                bla = lo;
                                blb = hi;
                            }
                        }
                    }
                }
        }
        __syncthreads();
        vmin = block_min_d(sh, bv);
    }
    KeyD best = key_none();
    if (!use_index && be >= 0 && bv == vmin) {
        const int2 x = s.edges[be];
        const int a = x.x, b = x.y;
        const int na = (a == last) ? hi_s : a, nb = (b == last) ? hi_s : b;
        const int la = s.label[a], lb = s.label[b];
        best.d2 = bv;
        if (la < lb) {
            best.lo = la;
            best.hi = lb;
            best.si = na;
            best.sj = nb;
        } else {
            best.lo = lb;
            best.hi = la;
            best.si = nb;
            best.sj = na;
        }
    }
    const int n1 = sh.bcast_i[0], n2 = sh.bcast_i[1];
    if (n1 > LCAP || n2 > LCAP) {
        // a very high degree at the merged pair: the full pass
        merge_edges_full(sh, s, lo_s, hi_s, R, E, stamp, true);
        merge_slots(sh, s, lo_s, hi_s, R, 0, rc, false, mat, d2);
        const int nd = sh.bcast_i[2];
        score_edges(sh, s, s.edirty, nd);
        nchk += nd;
        __syncthreads();
        if (tid == 0) {
            s.st[9] = 0;
            s.st[12] = 0;  // the edge list was compacted: ranges and chunk minima are rebuilt
        }
        empty_slots = 0;
        return false;
    }
    // rename the moved slot in L2 (the edges of L carry their neighbour in XL)
    for (int k = tid; k < n2; k += NT) {
        const int e = L2[k];
        int2 ed = s.edges[e];
        if (ed.x == last) ed.x = hi_s;
        if (ed.y == last) ed.y = hi_s;
        s.edges[e] = ed;
    }
    __syncthreads();  // L2 is read through before its space is reused as K below
    // one edge per neighbour survives: the least edge slot (compared in LDS
    // for a short list, by an atomic minimum per neighbour otherwise)
    const bool short_list = n1 <= 64;
    if (!short_list) {
        for (int k = tid; k < n1; k += NT)
            if (XL[k] >= 0) s.dmark[XL[k]] = INT_MAX;
        __syncthreads();
        for (int k = tid; k < n1; k += NT)
            if (XL[k] >= 0) atomicMin(&s.dmark[XL[k]], L[k]);
        __syncthreads();
    }
    int* K = L2;  // L2 is consumed: indices into L of the kept edges
    // and the label of each kept edge's other end, read now (a slot that moves keeps its label):
    // the staging tiles are free during a merge and hold LCAP entries
    static_assert(sizeof(sh.u.f.As) + sizeof(sh.u.f.Cs) >= LCAP * sizeof(int), "kept-edge labels fit");
    int* KL = reinterpret_cast<int*>(&sh.u.f.As[0][0]);
    for (int k = tid; k < n1; k += NT) {
        const int e = L[k], x = XL[k];
        bool keep = x >= 0;
        if (keep) {
            if (short_list) {
                for (int q = 0; q < n1; ++q)
                    if (XL[q] == x && L[q] < e) {
                        keep = false;
                        break;
                    }
            } else {
                keep = s.dmark[x] == e;
            }
        }
        if (keep) {
            s.edges[e] = make_int2(surv, x == last ? hi_s : x);
            const int pos = atomicAdd(&sh.bcast_i[2], 1);
            K[pos] = k;
            KL[pos] = s.label[x];
        } else {
            s.edges[e] = make_int2(-1, -1);
            s.ed2[e] = __builtin_huge_val();
            atomicAdd(&sh.bcast_i[3], 1);
        }
    }
    __syncthreads();
    merge_slots(sh, s, lo_s, hi_s, R, 0, rc, false, mat, d2);  // ends with a barrier
    const int nk = sh.bcast_i[2];
    const int emptied = sh.bcast_i[3];
    // with the row cache running the FP64 means of every live slot are current (the survivor's
    // written above): Equation 1 from them, without a division per band, in 16-band lane runs
    const bool means = rc != 0 && s.crit == HSWO_CRIT_BSMSE && s.B <= 1024;
    const int Ls = nk > LANE_PAIRS_MIN ? -1 : (means ? mean_lanes(s.B) : seg_lanes(s.B));
    if (Ls < 0) {
        // a survivor of high degree: one re-scored edge per lane
        for (int q0 = 0; q0 < nk; q0 += NT) {  // block-uniform trip count
            const int q = q0 + tid;
            int a = -1, b = -1, la = 0, lb = 0, e = -1;
            if (q < nk) {
                const int k = K[q];
                e = L[k];
                const int x = XL[k] == last ? hi_s : XL[k];
                const int lx = KL[q];
                a = surv;
                b = x;
                la = l_surv;
                lb = lx;
                if (la > lb) {
                    a = x;
                    b = surv;
                    la = lx;
                    lb = l_surv;
                }
            }
            const double v = exact_lane(s, a, b);
            if (q < nk) {
                KeyD kk;
                kk.d2 = v;
                kk.lo = la;
                kk.hi = lb;
                kk.si = a;
                kk.sj = b;
                s.ed2[e] = v;
                if (key_less(kk, best)) best = kk;
            }
        }
    } else if (Ls == 0) {
        for (int q = wave_id(); q < nk; q += NWAVE) {
            const int k = K[q];
            const int e = L[k];
            const int x = XL[k] == last ? hi_s : XL[k];
            const int lx = KL[q];
            int a = surv, b = x, la = l_surv, lb = lx;
            if (la > lb) {
                a = x;
                b = surv;
                la = lx;
                lb = l_surv;
            }
            KeyD kk;
            kk.d2 = exact_d2_wave(sh, s, a, b);
            kk.lo = la;
            kk.hi = lb;
            kk.si = a;
            kk.sj = b;
            if (lane_id() == 0) s.ed2[e] = kk.d2;
            if (key_less(kk, best)) best = kk;
        }
    } else {
        // 64 / Ls re-scored edges per wavefront at once
        const int ppw = 64 / Ls, sub = lane_id() / Ls;
        for (int q0 = wave_id() * ppw; q0 < nk; q0 += NWAVE * ppw) {  // wavefront-uniform trip count
            const int q = q0 + sub;
            int a = -1, b = -1, la = 0, lb = 0, e = -1;
            if (q < nk) {
                const int k = K[q];
                e = L[k];
                const int x = XL[k] == last ? hi_s : XL[k];
                const int lx = KL[q];
                a = surv;
                b = x;
                la = l_surv;
                lb = lx;
                if (la > lb) {
                    a = x;
                    b = surv;
                    la = lx;
                    lb = l_surv;
                }
            }
            const double v = means ? exact_seg_means(s, a, b, Ls) : exact_seg(s, a, b, Ls);
            if (q < nk) {
                KeyD kk;
                kk.d2 = v;
                kk.lo = la;
                kk.hi = lb;
                kk.si = a;
                kk.sj = b;
                if ((lane_id() & (Ls - 1)) == 0) s.ed2[e] = v;
                if (key_less(kk, best)) best = kk;
            }
        }
    }
    nchk += nk;
    if (use_index) {
        anext = merge_index_finish(sh, s, a0, a1, surv, hi_s, moved, ua, ub, ma, mb, E, L, n1);
    } else {
        anext = block_min_key(sh, best);  // the re-scored edges and the least of the others
        if (tid == 0) s.st[12] = 0;        // the index was not kept up to date
    }
    const int empty = empty_slots + emptied;  // st[9], kept by the caller
    if (4 * empty > E || R - 1 <= s.stop) {
        compact_edges(sh, s, E);
        if (tid == 0) {
            s.st[9] = 0;
            s.st[12] = 0;  // slot numbers changed: ranges and chunk minima are rebuilt
        }
        empty_slots = 0;
    } else {
        if (tid == 0) s.st[9] = empty;
        empty_slots = empty;
    }
    return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// Stages of one merge-loop iteration, as block-level functions over a range
// of the work, shared by the persistent driver (one workgroup does all of a
// section's work) and the wide kernels (G workgroups share the sweeps).
// ---------------------------------------------------------------------------

// Adjacent screen of edges [e_begin, e_end): 16 lanes per edge, EPG edges per
// lane group in flight; each lane streams 4 consecutive bands of both rows of
// EPG edges per 64-band chunk (2*EPG float4 loads outstanding per lane).
// Writes each edge's bounds to escr; returns this thread's least upper bound.
template <int EPG>
__device__ float adj_screen_range(const SecDev& s, int e_begin, int e_end, float gam) {
    const int tid = threadIdx.x;
    const int g = tid >> 4, gl = tid & 15;
    float myU = __builtin_huge_valf();
    for (int e0 = e_begin; e0 < e_end; e0 += (NT / 16) * EPG) {
        int ea[EPG], eb[EPG];
        float acc[EPG];
#pragma unroll
        for (int k = 0; k < EPG; ++k) {
            const int e = e0 + g * EPG + k;
            ea[k] = -1;
            eb[k] = -1;
            if (e < e_end) {
                const int2 ed = s.edges[e];
                ea[k] = ed.x;
                eb[k] = ed.y;
            }
            acc[k] = 0.0f;
        }
        for (int c = 0; c < s.Bp; c += 64) {
            const int b = c + gl * 4;
            if (b < s.Bp) {
                float4 x[EPG], y[EPG];
#pragma unroll
                for (int k = 0; k < EPG; ++k) {
                    x[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                    y[k] = x[k];
                    if (ea[k] >= 0) {
                        x[k] = *reinterpret_cast<const float4*>(s.mean + (size_t)ea[k] * s.Bp + b);
                        y[k] = *reinterpret_cast<const float4*>(s.mean + (size_t)eb[k] * s.Bp + b);
                    }
                }
#pragma unroll
                for (int k = 0; k < EPG; ++k) {
                    float d;
                    d = x[k].x - y[k].x; acc[k] = fmaf(d, d, acc[k]);
                    d = x[k].y - y[k].y; acc[k] = fmaf(d, d, acc[k]);
                    d = x[k].z - y[k].z; acc[k] = fmaf(d, d, acc[k]);
                    d = x[k].w - y[k].w; acc[k] = fmaf(d, d, acc[k]);
                }
            }
        }
        float mine = 0.0f;
        int ma = -1, mb = -1;
#pragma unroll
        for (int k = 0; k < EPG; ++k) {
            float v = acc[k];
            v += __shfl_xor(v, 8);
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 1);
            if (gl == k) {
                mine = v;
                ma = ea[k];
                mb = eb[k];
            }
        }
        if (gl < EPG) {
            const int e = e0 + g * EPG + gl;
            if (ma >= 0) {
                const float2 lu = screen_bounds(mine, s.npix[ma], s.npix[mb], s.norm[ma], s.norm[mb], gam);
                s.escr[e] = lu;
                if (s.vraw) s.vraw[e] = mine;
                myU = fminf(myU, lu.y);
            } else if (e < e_end) {
                s.escr[e] = make_float2(__builtin_huge_valf(), __builtin_huge_valf());  // empty slot
            }
        }
    }
    return myU;
}

// Exact best adjacent pair: every edge whose lower bound reaches Ua is
// re-scored in FP64.
__device__ KeyD adj_collect(Smem& sh, const SecDev& s, int R, int E, float Ua, int& nchk) {
    const int dbg = s.vout ? 1 : 0;
    constexpr int SPAN = NT * 16;  // edges appended between two fullness checks (<= CAND_CAP)
    const int tid = threadIdx.x;
    KeyD A = key_none();
    for (int e0 = 0; e0 < E; e0 += SPAN) {
        const int e1 = min(E, e0 + SPAN);
        for (int e = e0 + tid; e < e1; e += NT) {
            const float lo = s.escr[e].x;
            if (lo <= Ua && lo < __builtin_huge_valf()) {  // empty slots have +inf bounds
                const int k = atomicAdd(&sh.ncand, 1);
                if (k < CAND_CAP) sh.u.f.cand[k] = e;
            }
        }
        flush_candidates(sh, s, A, nchk, true, SPAN, dbg, R);
    }
    flush_candidates(sh, s, A, nchk, true, CAND_CAP, dbg, R);
    return A;
}

// Incremental adjacent stage: the exact lexicographic minimum over the cached
// per-edge D2 (scoring every edge first when the cache is not yet valid).
// Labels are read only for values that can still win.
__device__ KeyD adj_incremental(Smem& sh, const SecDev& s, int E, bool init, int& nchk) {
    if (init) {
        score_edges(sh, s, nullptr, E);
        nchk += E;
        __syncthreads();
    }
    KeyD best = key_none();
    constexpr int U = 4;  // cached values per thread with loads in flight together
    for (int e0 = threadIdx.x; e0 < E; e0 += NT * U) {
        double vv[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int e = e0 + q * NT;
            vv[q] = e < E ? s.ed2[e] : __builtin_huge_val();
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const double v = vv[q];
            if (v <= best.d2 && v < __builtin_huge_val()) {
                const int2 ed = s.edges[e0 + q * NT];
                int a = ed.x, b = ed.y;
                int la = s.label[a], lb = s.label[b];
                if (la > lb) {
                    const int t = a; a = b; b = t;
                    const int w = la; la = lb; lb = w;
                }
                KeyD k;
                k.d2 = v;
                k.lo = la;
                k.hi = lb;
                k.si = a;
                k.sj = b;
                if (key_less(k, best)) best = k;
            }
        }
    }
    return block_min_key(sh, best);
}

// FP32 spectral tiles t = t0, t0 + stride, ...: per-tile (min lower, min
// upper) to tstat. With use16 only the tiles the matrix-core screen flagged
// are screened (the others get +inf). Returns the least upper bound seen
// (block-uniform) and counts the tiles screened.
__device__ float fp32_tiles(Smem& sh, const SecDev& s, int R, bool use16, float gam, int t0, int stride,
                            int& nproc) {
    const int tid = threadIdx.x;
    const int ty = tid >> 5, tx = tid & 31;
    const int nT = (R + TILE - 1) / TILE;
    const int ntiles = nT * (nT + 1) / 2;
    float Us = __builtin_huge_valf();
    for (int c0 = t0; c0 < ntiles; c0 += stride * TLIST) {
        // gather this workgroup's tiles t = c0, c0 + stride, ... (flagged ones with use16)
        if (tid == 0) sh.ntl = 0;
        __syncthreads();
        for (int k = tid; k < TLIST; k += NT) {
            const int t = c0 + k * stride;
            if (t >= ntiles) break;
            if (!use16 || s.tflag[t]) {
                sh.tlist[atomicAdd(&sh.ntl, 1)] = t;
            } else {
                s.tstat[t] = make_float2(__builtin_huge_valf(), __builtin_huge_valf());
            }
        }
        __syncthreads();
        const int nt = sh.ntl;
        for (int q = 0; q < nt; ++q) {
            const int t = sh.tlist[q];
            int ib, jb;
            tile_coords(t, nT, ib, jb);
            ++nproc;
            float acc[4][2];
            tile_sums_fp32(sh, s, ib, jb, R, acc);
            float mL = __builtin_huge_valf(), mU = __builtin_huge_valf();
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int i = ib * TILE + ty * 4 + a, j = jb * TILE + tx * 2 + c;
                    if (i < j && j < R) {
                        const float2 lu = screen_bounds(acc[a][c], s.npix[i], s.npix[j], s.norm[i], s.norm[j], gam);
                        mL = fminf(mL, lu.x);
                        mU = fminf(mU, lu.y);
                    }
                }
            const float2 lu = block_min_f2(sh, mL, mU);
            if (tid == 0) s.tstat[t] = lu;
            Us = fminf(Us, lu.y);
        }
        __syncthreads();  // tlist is rewritten by the next chunk
    }
    return Us;
}

// Exact best non-adjacent candidate: re-screen every tile whose least lower
// bound reaches theta (and is below T), collect its pairs with lower <= theta
// and < T, re-score them in FP64.
// prec16: the 16-bit screen that flagged the tiles (0 none, 1 BF16, 2 FP16),
// for HSWO_FLAG_DEBUG_VERIFY_BOUND.
__device__ KeyD spectral_collect(Smem& sh, const SecDev& s, int R, double T, double theta, float gam, int& nchk,
                                 int& nresc, int prec16) {
    const int tid = threadIdx.x;
    const int dbg = s.vout ? 2 + prec16 : 0;
    const int ty = tid >> 5, tx = tid & 31;
    const int nT = (R + TILE - 1) / TILE;
    const int ntiles = nT * (nT + 1) / 2;
    KeyD M = key_none();
    for (int c0 = 0; c0 < ntiles; c0 += TLIST) {
        if (tid == 0) sh.ntl = 0;
        __syncthreads();
        for (int t = c0 + tid; t < min(ntiles, c0 + TLIST); t += NT) {
            const float tl = s.tstat[t].x;
            if ((double)tl <= theta && (double)tl < T) sh.tlist[atomicAdd(&sh.ntl, 1)] = t;
        }
        __syncthreads();
        const int nt = sh.ntl;
        for (int q = 0; q < nt; ++q) {
            const int t = sh.tlist[q];
            int ib, jb;
            tile_coords(t, nT, ib, jb);
            ++nresc;
            float acc[4][2];
            tile_sums_fp32(sh, s, ib, jb, R, acc);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int i = ib * TILE + ty * 4 + a, j = jb * TILE + tx * 2 + c;
                    if (i < j && j < R) {
                        const float lo = screen_bounds(acc[a][c], s.npix[i], s.npix[j], s.norm[i], s.norm[j], gam).x;
                        if ((double)lo <= theta && (double)lo < T) {
                            const int k = atomicAdd(&sh.ncand, 1);
                            if (k < CAND_CAP) {
                                sh.u.f.cand[k] = (int)(((unsigned)i << 16) | (unsigned)j);
                                if (dbg) s.vstage[k] = acc[a][c];
                            }
                        }
                    }
                }
            flush_candidates(sh, s, M, nchk, false, TILE * TILE, dbg, R);
        }
        __syncthreads();  // tlist is rewritten by the next chunk
    }
    flush_candidates(sh, s, M, nchk, false, CAND_CAP, dbg, R);
    return M;
}

__device__ void clear_tile_flags(const SecDev& s, int R) {
    const int nT = (R + TILE - 1) / TILE;
    const int ntiles = nT * (nT + 1) / 2;
    for (int t = threadIdx.x; t < ntiles; t += NT) s.tflag[t] = 0;
}

// The merge decision (one merge per iteration; the non-adjacent minimum wins
// only below w^2 times the adjacent minimum).
__device__ __forceinline__ bool decide(bool spectral, const KeyD& A, const KeyD& M, double T, KeyD& win, int& kind) {
    if (spectral && key_exists(M) && M.d2 < T) {
        win = M;
        kind = 1;
        return true;
    }
    if (key_exists(A)) {
        win = A;
        kind = 0;
        return true;
    }
    return false;
}

// One 64 x 64 tile t (upper triangle, numbered as the spectral tiles) of a
// section's interval matrix, by the whole block. Each pair's squared distance
// of the FP32 mean rows (rebuilt from the FP64 means by rowcache_begin) is
// summed in FP32 by a 4 x 2 register tile per thread from LDS-staged 32-band
// slices (As, Cs: BK bands of the two row blocks, row pitch P);
// screen_bounds turns it into certified bounds on the canonical value, which
// are widened to the real value and rounded outward into both (i, j) and
// (j, i). Returns the tile's pairs.
template <int P>
__device__ unsigned long long mat_fill_tile(float (*As)[P], float (*Cs)[P], const SecDev& s, int R, int t) {
    const int nT = (R + TILE - 1) / TILE;
    int ib, jb;
    tile_coords(t, nT, ib, jb);
    const int tid = threadIdx.x;
    const int ty = tid >> 5, tx = tid & 31;
    float acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a][0] = acc[a][1] = 0.0f;
    const int lrow = tid >> 3, lb = (tid & 7) << 2;
    const int ia = ib * TILE + lrow, ic = jb * TILE + lrow;
    for (int k0 = 0; k0 < s.Bp; k0 += BK) {
        float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vc = va;
        if (ia < R) va = *reinterpret_cast<const float4*>(s.mean + (size_t)ia * s.Bp + k0 + lb);
        if (ic < R) vc = *reinterpret_cast<const float4*>(s.mean + (size_t)ic * s.Bp + k0 + lb);
        As[lb + 0][lrow] = va.x;
        As[lb + 1][lrow] = va.y;
        As[lb + 2][lrow] = va.z;
        As[lb + 3][lrow] = va.w;
        Cs[lb + 0][lrow] = vc.x;
        Cs[lb + 1][lrow] = vc.y;
        Cs[lb + 2][lrow] = vc.z;
        Cs[lb + 3][lrow] = vc.w;
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < BK; ++kk) {
            const float4 a = *reinterpret_cast<const float4*>(&As[kk][ty * 4]);
            const float2 c = *reinterpret_cast<const float2*>(&Cs[kk][tx * 2]);
            float d;
            d = a.x - c.x; acc[0][0] = fmaf(d, d, acc[0][0]);
            d = a.x - c.y; acc[0][1] = fmaf(d, d, acc[0][1]);
            d = a.y - c.x; acc[1][0] = fmaf(d, d, acc[1][0]);
            d = a.y - c.y; acc[1][1] = fmaf(d, d, acc[1][1]);
            d = a.z - c.x; acc[2][0] = fmaf(d, d, acc[2][0]);
            d = a.z - c.y; acc[2][1] = fmaf(d, d, acc[2][1]);
            d = a.w - c.x; acc[3][0] = fmaf(d, d, acc[3][0]);
            d = a.w - c.y; acc[3][1] = fmaf(d, d, acc[3][1]);
        }
        __syncthreads();
    }
    const float gam = (float)(2 * s.B + 32) * U32;
    const size_t rc = (size_t)s.mstride;  // matrix row stride
    const float2 inf2 = make_float2(__builtin_huge_valf(), __builtin_huge_valf());
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = ib * TILE + ty * 4 + a, j = jb * TILE + tx * 2 + c;
            if (i >= R || j >= R || (ib == jb && j < i)) continue;
            float2 e = inf2;
            if (i != j) {
                const float2 lu = screen_bounds(acc[a][c], s.npix[i], s.npix[j], s.norm[i], s.norm[j], gam);
                e = make_float2(__double2float_rd((double)lu.x * (1.0 - MAT_REL)),
                                __double2float_ru((double)lu.y * (1.0 + MAT_REL)));
            }
            s.dmat[(size_t)i * rc + j] = e;
            s.dmat[(size_t)j * rc + i] = e;
        }
    return (unsigned long long)min(TILE, R - ib * TILE) * (unsigned long long)min(TILE, R - jb * TILE);
}

// LDS of row_matrix_wave: per wavefront, a candidate list and its values.
constexpr int WAVE_CAND = 128;
struct RowWaveLds {
    int cand[NWAVE][WAVE_CAND];
    double val[NWAVE][WAVE_CAND];
};

// row_matrix_task by one wavefront (the section's workgroup rescans several
// pending rows at once, one per wavefront, with no block barrier): the same
// threshold, candidates, exact evaluations, tightened bounds and least two,
// so the same entry of rpart. Candidates go to the wavefront's LDS list in
// rounds of at most WAVE_CAND (ballot-compacted); LDS operations of one
// wavefront complete in order, so its lanes read what its lanes wrote.
// Returns the number of exact evaluations (every lane).
__device__ int row_matrix_wave(RowWaveLds& L, const SecDev& s, int R, int q, bool all) {
    const int lane = lane_id(), w = wave_id();
    const size_t rc = (size_t)s.mstride;
    const int i = all ? q : s.rpend[q];
    const int mi = s.msl[i];
    const float2* Di = s.dmat + (size_t)mi * rc;
    double m1 = __builtin_huge_val(), m2 = __builtin_huge_val();
    for (int j = lane; j < R; j += 64)
        if (j != i) least_two(m1, m2, (double)Di[s.msl[j]].y * (1.0 + MAT_REL), __builtin_huge_val());
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) least_two(m1, m2, __shfl_xor(m1, o), __shfl_xor(m2, o));
    const double T = m2;
    RowPart best = part_of(__builtin_huge_val(), INT_MAX, -1);
    int nexact = 0, n = 0;
    int* cl = L.cand[w];
    double* vl = L.val[w];
    for (int j0 = 0; j0 < R; j0 += 64) {  // wavefront-uniform
        const int j = j0 + lane;
        const float2 e = (j < R && j != i) ? Di[s.msl[j]] : make_float2(__builtin_huge_valf(), __builtin_huge_valf());
        const bool cand = j < R && j != i && (double)e.x * (1.0 - MAT_REL) <= T;
        if (cand && e.y == 0.0f) top2_merge(best, part_of(0.0, s.label[j], j));  // bounded by [0, 0]: exactly 0
        const bool put = cand && e.y != 0.0f;
        const unsigned long long mask = __ballot(put);
        const int cnt = __popcll(mask);
        if (n + cnt > WAVE_CAND) {  // wavefront-uniform: evaluate what the list holds first
            for (int k = 0; k < n; ++k) {
                const int jj = cl[k];
                const double v = exact_wave_means(s, i, jj);
                if (lane == 0) {
                    vl[k] = v;
                    const float2 me = mat_entry(v);
                    const int mj = s.msl[jj];
                    s.dmat[(size_t)mi * rc + mj] = me;
                    s.dmat[(size_t)mj * rc + mi] = me;
                }
            }
            for (int k = lane; k < n; k += 64) top2_merge(best, part_of(vl[k], s.label[cl[k]], cl[k]));
            nexact += n;
            n = 0;
        }
        if (put) cl[n + __popcll(mask & ((1ull << lane) - 1ull))] = j;
        n += cnt;
    }
    for (int k = 0; k < n; ++k) {
        const int jj = cl[k];
        const double v = exact_wave_means(s, i, jj);
        if (lane == 0) {
            vl[k] = v;
            const float2 me = mat_entry(v);
            const int mj = s.msl[jj];
            s.dmat[(size_t)mi * rc + mj] = me;
            s.dmat[(size_t)mj * rc + mi] = me;
        }
    }
    for (int k = lane; k < n; k += 64) top2_merge(best, part_of(vl[k], s.label[cl[k]], cl[k]));
    nexact += n;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) top2_merge(best, shfl_xor_part(best, o));
    const int nch = (R + 63) >> 6;
    if (lane == 0) s.rpart[(size_t)q * nch] = best;
    for (int c = 1 + lane; c < nch; c += 64) s.rpart[(size_t)q * nch + c] = part_of(__builtin_huge_val(), INT_MAX, -1);
    return nexact;
}

// ---------------------------------------------------------------------------
// Several merges per step (HSWO_FLAG_MULTI_MERGE): the future-work item of
// Section 6.2, read for identical regions. A step whose winner has the value
// 0 merges a greedy disjoint set of zero-valued pairs: adjacent pairs ranked
// by (lo, hi) first, then -- with the spectral stage on at the step's start --
// non-adjacent ones by (lo, hi), a pair being skipped when one of its regions
// is already taken, until the pass's stop count. The pairs are disjoint, so
// merging them one after another in that order is the step.
//
// Adjacent zero pairs are the edges whose cached exact value is 0. For the
// non-adjacent ones: Equation 1 is 0 exactly when the two FP64 mean rows S/n
// are equal band by band (two different means of float32 or float16 data are
// at least 2^-232 apart, so a difference never squares to 0, and a sum of
// non-negative terms is 0 only when every term is). The regions left unused
// by the adjacent pass therefore fall into classes of equal mean rows, found
// by sorting them on a hash of the row and comparing the members of each run
// of equal hashes exactly. No two of those members are adjacent (the greedy
// matching over the adjacent zero pairs is maximal), so within a class the
// greedy pairs the members in label order, two by two.
// ---------------------------------------------------------------------------

// Bitonic sort of key[0, n) ascending, val alongside; n a power of two. The
// whole block calls it (global memory, a barrier after every pass).
__device__ void block_sort_kv(unsigned long long* key, unsigned long long* val, int n) {
    for (int k = 2; k <= n; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += NT) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const unsigned long long a = key[i], b = key[ixj];
                    if ((a > b) == ((i & k) == 0)) {
                        key[i] = b;
                        key[ixj] = a;
                        const unsigned long long t = val[i];
                        val[i] = val[ixj];
                        val[ixj] = t;
                    }
                }
            }
            __syncthreads();
        }
}

__device__ __forceinline__ unsigned long long zmix(unsigned long long x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// One wavefront: a 32-bit hash of slot i's FP64 mean row from the row cache
// (0 and -0 hash alike, as they compare equal); the same on every lane.
__device__ unsigned int mean_row_hash(const SecDev& s, int i) {
    const double* M = s.m64r + (size_t)i * ((s.B + 7) & ~7);
    unsigned int h0 = 0, h1 = 0;
    for (int b = lane_id(); b < s.B; b += 64) {
        const double m = M[b] == 0.0 ? 0.0 : M[b];
        const unsigned long long x = zmix((unsigned long long)__double_as_longlong(m) ^ zmix((unsigned long long)b + 1));
        h0 ^= (unsigned int)x;
        h1 ^= (unsigned int)(x >> 32);
    }
    for (int o = 32; o >= 1; o >>= 1) {
        h0 ^= __shfl_xor(h0, o);
        h1 ^= __shfl_xor(h1, o);
    }
    return h0 ^ (h1 * 0x9e3779b9u);
}

// One wavefront: are the FP64 mean rows of slots i and j equal in every band?
__device__ bool mean_rows_equal(const SecDev& s, int i, int j) {
    const int B8 = (s.B + 7) & ~7;
    const double* Mi = s.m64r + (size_t)i * B8;
    const double* Mj = s.m64r + (size_t)j * B8;
    int eq = 1;
    for (int b = lane_id(); b < s.B; b += 64) eq &= Mi[b] == Mj[b] ? 1 : 0;
    return __all(eq) != 0;
}

// Pads key[n, n2) with the largest key and sorts key[0, n2), n2 the least
// power of two >= n. Whole block.
__device__ void zsort(const SecDev& s, int n) {
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    for (int q = n + threadIdx.x; q < n2; q += NT) s.zkey[q] = ~0ull;
    __syncthreads();
    if (n > 1) block_sort_kv(s.zkey, s.zval, n2);
}

// The step's pairs into s.zlist in merge order (x slot of lo, y slot of hi,
// z kind), at most cap of them; returns how many (block-uniform, >= 1 when
// the step's winner has the value 0). spectral: the spectral stage is on at
// the step's start (the row cache then holds every live slot's mean row).
// Leaves s.zuse[slot] = 2 * place + (0 lo, 1 hi) for the listed slots, -1
// for the others.
__device__ __noinline__ int zero_step_list(Smem& sh, const SecDev& s, int R, int E, bool spectral, int cap) {
    const int tid = threadIdx.x;
    for (int i = tid; i < R; i += NT) s.zuse[i] = 0;
    if (tid == 0) sh.zc[0] = 0;
    __syncthreads();
    // adjacent pairs of value 0 (empty edge slots hold +inf), ranked by (lo, hi)
    for (int e = tid; e < E; e += NT) {
        if (s.ed2[e] == 0.0) {
            const int2 ed = s.edges[e];
            int a = ed.x, b = ed.y;
            int la = s.label[a], lb = s.label[b];
            if (la > lb) {
                const int t = a; a = b; b = t;
                const int u = la; la = lb; lb = u;
            }
            const int q = atomicAdd(&sh.zc[0], 1);
            s.zkey[q] = ((unsigned long long)(unsigned)la << 32) | (unsigned)lb;
            s.zval[q] = ((unsigned long long)(unsigned)a << 32) | (unsigned)b;
        }
    }
    __syncthreads();
    const int na = sh.zc[0];
    zsort(s, na);
    // the greedy pass over them, in rank order (one thread)
    if (tid == 0) {
        int k = 0;
        for (int q = 0; q < na && k < cap; ++q) {
            const unsigned long long v = s.zval[q];
            const int a = (int)(v >> 32), b = (int)(unsigned)v;
            if (s.zuse[a] || s.zuse[b]) continue;
            s.zuse[a] = 1;
            s.zuse[b] = 1;
            s.zlist[k] = make_int4(a, b, 0, 0);
            ++k;
        }
        sh.zc[1] = k;
    }
    __syncthreads();
    int k = sh.zc[1];
    if (spectral && k < cap) {
        // the unused regions ranked by (hash of the mean row, label)
        if (tid == 0) sh.zc[0] = 0;
        __syncthreads();
        for (int i = wave_id(); i < R; i += NWAVE) {
            if (s.zuse[i]) continue;  // wavefront-uniform
            const unsigned int h = mean_row_hash(s, i);
            if (lane_id() == 0) {
                const int q = atomicAdd(&sh.zc[0], 1);
                s.zkey[q] = ((unsigned long long)h << 32) | (unsigned)s.label[i];
                s.zval[q] = (unsigned long long)(unsigned)i;
            }
        }
        __syncthreads();
        const int nb = sh.zc[0];
        zsort(s, nb);
        // each member's class head: the first member of its hash run with an equal row
        for (int y = wave_id(); y < nb; y += NWAVE) {
            const unsigned int hy = (unsigned int)(s.zkey[y] >> 32);
            const int sy = (int)(unsigned)s.zval[y];
            int p = y;
            while (p > 0 && (unsigned int)(s.zkey[p - 1] >> 32) == hy) --p;
            int head = y;
            for (int x = p; x < y; ++x)  // wavefront-uniform
                if (mean_rows_equal(s, (int)(unsigned)s.zval[x], sy)) {
                    head = x;
                    break;
                }
            if (lane_id() == 0) s.zval[y] = ((unsigned long long)(unsigned)head << 32) | (unsigned)sy;
        }
        __syncthreads();
        // a member of odd rank in its class pairs with the class member before it
        if (tid == 0) sh.zc[0] = 0;
        __syncthreads();
        int4* tmp = s.zlist + k;  // past the adjacent pairs
        for (int y = tid; y < nb; y += NT) {
            const int h = (int)(s.zval[y] >> 32);
            int rank = 0, prev = -1;
            for (int z = h; z < y; ++z)
                if ((int)(s.zval[z] >> 32) == h) {
                    ++rank;
                    prev = z;
                }
            if (rank & 1) {
                const int q = atomicAdd(&sh.zc[0], 1);
                tmp[q] = make_int4((int)(unsigned)s.zval[prev], (int)(unsigned)s.zval[y], (int)(unsigned)s.zkey[prev],
                                   (int)(unsigned)s.zkey[y]);
            }
        }
        __syncthreads();
        // ranked by (lo, hi) and appended after the adjacent pairs
        const int nz = sh.zc[0];
        for (int q = tid; q < nz; q += NT) {
            const int4 t = tmp[q];
            s.zkey[q] = ((unsigned long long)(unsigned)t.z << 32) | (unsigned)t.w;
            s.zval[q] = ((unsigned long long)(unsigned)t.x << 32) | (unsigned)t.y;
        }
        __syncthreads();
        zsort(s, nz);
        const int take = min(nz, cap - k);
        for (int q = tid; q < take; q += NT) {
            const unsigned long long v = s.zval[q];
            s.zlist[k + q] = make_int4((int)(v >> 32), (int)(unsigned)v, 1, 0);
        }
        k += take;
        __syncthreads();
    }
    // place of every listed slot, for the renames of the moves
    for (int i = tid; i < R; i += NT) s.zuse[i] = -1;
    __syncthreads();
    for (int q = tid; q < k; q += NT) {
        const int4 z = s.zlist[q];
        s.zuse[z.x] = 2 * q;
        s.zuse[z.y] = 2 * q + 1;
    }
    __syncthreads();
    return k;
}

// ---------------------------------------------------------------------------
// The persistent section driver: one workgroup runs the whole HSEG loop of
// one section; one launch covers every section of a recursion level.
// ---------------------------------------------------------------------------
template <int EPG>
__global__ void __launch_bounds__(NT) k_section_driver(const SecDev* __restrict__ secs, int n_sec,
                                                       LoopParams lp) {
    __shared__ Smem sh;
    if ((int)blockIdx.x >= n_sec || gated(lp.counters)) return;
    const SecDev& s = secs[blockIdx.x];
    const int tid = threadIdx.x;
    int R = s.st[0];
    int E = s.st[1];
    int g_ready = s.st[4];
    const int prec = s.kcap > 0 ? lp.precision : 0;
    const float gam = (float)(2 * s.B + 32) * U32;
    const bool row_cache = lp.incremental && s.rcap > 0;
    int rcs = row_cache ? s.st[6] : 0;   // row cache state, block-uniform
    int npend = row_cache ? s.st[7] : 0; // pending rows (state 2)
    int merges = s.st[3];
    int empty_slots = s.st[9];  // empty edge slots left by incremental merges (kept in st[9] too)
    bool avalid = false;  // incremental form: the least adjacent key after the last merge is known
    KeyD anext = key_none();
    // the row cache keeps the interval matrix (Equation 1, one-merge reading, rcap <= MAT_MAX)
    const bool mat = row_cache && row_matrix_on(s, lp);
    // two-merge reading: step 3 (the non-adjacent merge) is due, below thr3
    int st3 = lp.two_merges ? s.st[10] : 0;
    double thr3 = st3 ? s.wd[3] : 0.0;
    if (tid == 0) {
        sh.ncand = 0;
        for (int c = 0; c < C_COUNT; ++c) sh.cnt[c] = 0ull;
    }
    __syncthreads();
// thread 0 adds a plain value (never pass a call: the argument is evaluated by thread 0 only)
#define CNT_ADD(k, v)                             \
    do {                                          \
        if (tid == 0) sh.cnt[k] += (unsigned long long)(v); \
    } while (0)

    const int stop_here = max(s.stop, lp.phase_stop);
    while (R > stop_here) {
        unsigned long long tk0 = wall_clock64();
        // adjacent stage: full screen of every edge, or the cached exact values
        int nchk = 0;
        KeyD A;
        if (lp.incremental) {
            if (avalid) {
                A = anext;
            } else {
                A = adj_incremental(sh, s, E, s.st[5] == 0, nchk);
                if (tid == 0) s.st[5] = 1;
            }
        } else {
            const float myU = adj_screen_range<EPG>(s, 0, E, gam);
            const float Ua = block_min_f2(sh, myU, myU).x;
            const int c0 = nchk;
            A = adj_collect(sh, s, R, E, Ua, nchk);
            CNT_ADD(C_SCREEN_ITERS, 1);
            CNT_ADD(C_SCREEN_FALLBACKS, nchk - c0 > lp.topk ? 1 : 0);
        }
        CNT_ADD(C_ADJ_PAIRS, E - empty_slots);
        unsigned long long tk1 = wall_clock64();
        CNT_ADD(C_T_ADJ, tk1 - tk0);
        tk0 = tk1;

        // spectral stage
        KeyD M = key_none();
        const bool spectral = lp.spectral && R <= lp.kmax;
        const double T = key_exists(A) ? lp.w2 * A.d2 : __builtin_huge_val();
        if (spectral && row_cache && mat) {
            // interval matrix: filled when the cache starts (tile after tile), then the rows --
            // all of them at the start, else the pending ones -- rescanned from their bounds
            if (rcs == 0) {
                rowcache_begin(sh, s, R, E, true);
                rcs = 1;
            }
            const bool all = rcs == 1;
            const int rows = all ? R : npend;
            if (all) {
                const int nT = (R + TILE - 1) / TILE;
                unsigned long long pairs = 0;
                for (int t = 0; t < nT * (nT + 1) / 2; ++t) pairs += mat_fill_tile<TILE + 4>(sh.u.f.As, sh.u.f.Cs, s, R, t);
                CNT_ADD(C_W_FILL_FLOPS, 3ull * (unsigned long long)s.B * pairs);
                __syncthreads();
            }
            // one pending row per wavefront at a time
            static_assert(sizeof(RowWaveLds) <= sizeof(Smem::u), "the wavefronts' candidate lists live in the union");
            RowWaveLds& wl = *reinterpret_cast<RowWaveLds*>(&sh.u);
            int ex = 0;
            for (int q = wave_id(); q < rows; q += NWAVE) ex += row_matrix_wave(wl, s, R, q, all);
            if (lane_id() == 0) sh.redi[wave_id()] = ex;
            __syncthreads();  // every row's entry is written
            if (tid == 0)
                for (int k = 1; k < NWAVE; ++k) ex += sh.redi[k];
            __syncthreads();  // the counts are read before the reductions below reuse redi
            M = spectral_min_rows(sh, s, R, rows, all);
            rcs = 2;
            npend = 0;
            CNT_ADD(C_RECHECKS, ex);
            CNT_ADD(C_ROW_BOUNDED, (unsigned long long)rows * (unsigned long long)(R - 1));
            CNT_ADD(C_D_BYTES, 12ull * (unsigned long long)R + 8ull * (unsigned long long)rows * (unsigned long long)R +
                                   (unsigned long long)ex * (16ull * (unsigned long long)s.B + 16ull));
            CNT_ADD(C_SPEC_PAIRS, (unsigned long long)R * (unsigned long long)(R - 1) / 2ull);
            tk1 = wall_clock64();
            CNT_ADD(C_T_SPEC32, tk1 - tk0);
            tk0 = tk1;
        } else if (spectral && row_cache) {
            // exact rows: all of them when the cache starts, else the pending ones
            if (rcs == 0) {
                rowcache_begin(sh, s, R, E, false);
                rcs = 1;
            }
            const bool all = rcs == 1;
            const int rows = all ? R : npend;
            // the section has the workgroup to itself: each wavefront takes its own tasks
            const int nch = (R + 63) >> 6;
            const int ntask = row_task_count(R, rows);
            if (s.crit == HSWO_CRIT_SAM) {
                if (s.B <= 512) {
                    for (int t = wave_id(); t < ntask; t += NWAVE)
                        row_wave_task<4, 7, true>(s, R, rows, all, t / nch, t % nch);
                } else {
                    for (int t = wave_id(); t < ntask; t += NWAVE)
                        row_wave_task<4, 10, true>(s, R, rows, all, t / nch, t % nch);
                }
            } else if (s.B <= 512) {
                for (int t = wave_id(); t < ntask; t += NWAVE)
                    row_wave_task<4, 7, false>(s, R, rows, all, t / nch, t % nch);
            } else {
                for (int t = wave_id(); t < ntask; t += NWAVE)
                    row_wave_task<4, 10, false>(s, R, rows, all, t / nch, t % nch);
            }
            __syncthreads();
            // rows whose light step fell back on a full evaluation (appended by other wavefronts)
            const int nf = all ? 0 : __hip_atomic_load(&s.st[11], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (nf > 0) {
                rows_fallback_body(s, R, rows, nf);
                __syncthreads();
            }
            M = spectral_min_rows(sh, s, R, rows + nf, all);
            rcs = 2;
            npend = 0;
            // bytes: cached pairs, row partials, and every live FP64 row read once by the row stage
            // (once more by the fallback)
            CNT_ADD(C_D_BYTES, 12ull * (unsigned long long)R +
                                   32ull * (unsigned long long)(rows + nf) * (unsigned long long)nch +
                                   (rows ? 8ull * (unsigned long long)s.B * (unsigned long long)R : 0ull) +
                                   (nf ? 8ull * (unsigned long long)s.B * (unsigned long long)R : 0ull));
            CNT_ADD(C_RECHECKS, (unsigned long long)nf * (unsigned long long)(R - 1));
            CNT_ADD(C_SPEC_PAIRS, (unsigned long long)R * (unsigned long long)(R - 1) / 2ull);
            CNT_ADD(C_RECHECKS, (unsigned long long)rows * (unsigned long long)(R - 1));
            tk1 = wall_clock64();
            CNT_ADD(C_T_SPEC32, tk1 - tk0);
            tk0 = tk1;
        } else if (spectral) {
            if (prec && !g_ready) {
                if (prec == 1)
                    build16_all<1>(s, R);
                else
                    build16_all<2>(s, R);
                g_ready = 1;
            }
            // matrix-core pass: flags the tiles that may hold a pair below T
            const bool use16 = prec && T < __builtin_huge_val();
            if (use16) {
                prep_alpha_p(s, R, T);
                clear_tile_flags(s, R);
                // the screen is a block-level function: the whole block calls it, then thread 0 counts
                const int nsup = prec == 1 ? mfma_screen<1>(sh, s, R, 0, 1) : mfma_screen<2>(sh, s, R, 0, 1);
                CNT_ADD(C_MFMA_TILES, nsup);
            }
            tk1 = wall_clock64();
            CNT_ADD(C_T_MFMA, tk1 - tk0);
            tk0 = tk1;
            int nf = 0, nresc = 0;
            const float Us = fp32_tiles(sh, s, R, use16, gam, 0, 1, nf);
            const double theta = fmin((double)Us, T);
            const int c1 = nchk;
            M = spectral_collect(sh, s, R, T, theta, gam, nchk, nresc, use16 ? prec : 0);
            CNT_ADD(C_SCREEN_ITERS, 1);
            CNT_ADD(C_SCREEN_FALLBACKS, nchk - c1 > lp.topk ? 1 : 0);
            CNT_ADD(C_FP32_TILES, nf);
            CNT_ADD(C_SPEC_PAIRS, (unsigned long long)R * (unsigned long long)(R - 1) / 2ull);
            CNT_ADD(C_RESCANS, nresc);
            tk1 = wall_clock64();
            CNT_ADD(C_T_SPEC32, tk1 - tk0);
            tk0 = tk1;
        }

        KeyD win;
        int kind;
        bool step2 = false;
        if (st3 && key_exists(M) && M.d2 < thr3) {
            // two-merge reading, step 3: the least non-adjacent pair is below w^2 times step 2's value
            win = M;
            kind = 1;
        } else if (lp.two_merges && key_exists(A)) {
            // step 2: the least adjacent pair, whatever the spectral minimum -- also at once when
            // step 3 found no pair (nothing changed since, so the next iteration starts here)
            win = A;
            kind = 0;
            step2 = true;
        } else if (!decide(spectral, A, M, T, win, kind)) {
            break;  // no pair left (not in a connected section)
        }
        st3 = 0;
        CNT_ADD(C_RECHECKS, nchk);
        CNT_ADD(C_ITERS, 1);
        // a step of several merges (incremental form): its pairs, then one merge each; a slot that a
        // merge moves keeps its place in the list. With more than one merge the row cache drops to
        // state 1: every row is evaluated anew at the next spectral iteration. (The list holds the
        // winner whenever its value is 0; were it empty, the winner merges alone below.)
        const int np = (lp.multi_merge && win.d2 == 0.0) ? zero_step_list(sh, s, R, E, spectral, R - stop_here) : 0;
        if (np > 0) {
            if (np > 1 && rcs == 2) rcs = 1;
            for (int t = 0; t < np; ++t) {  // block-uniform
                const int4 z = s.zlist[t];
                int nre = 0;
                CNT_ADD(C_MERGES, 1);
                avalid = merge_pair_inc<8>(sh, s, z.x, z.y, R, E, merges, z.z + (t ? 2 : 0), 0.0, rcs, anext, nre,
                                           false, 0, empty_slots);
                CNT_ADD(C_RECHECKS, nre);
                CNT_ADD(C_D_BYTES, 16ull * (unsigned long long)sh.eread + 24ull * (unsigned long long)s.B);
                ++merges;
                --R;
                if (tid == 0 && z.y != R) {  // slot R (the old last) moved into z.y
                    const int pl = s.zuse[R];
                    if (pl >= 0 && (pl >> 1) > t) {
                        int4* ze = s.zlist + (pl >> 1);
                        if (pl & 1)
                            ze->y = z.y;
                        else
                            ze->x = z.y;
                        s.zuse[z.y] = pl;
                    }
                }
                __syncthreads();
            }
            if (rcs == 2) npend = sh.npend;
            if (row_cache && rcs == 0 && lp.spectral && R <= lp.kmax && R > s.stop) {
                rowcache_begin(sh, s, R, E, row_matrix_on(s, lp));
                rcs = 1;
            }
            CNT_ADD(C_T_MERGE, wall_clock64() - tk0);
            continue;
        }
        CNT_ADD(C_MERGES, 1);
        if (lp.incremental) {
            int nre = 0;
            avalid = merge_pair_inc<8>(sh, s, win.si, win.sj, R, E, merges, kind, win.d2, rcs, anext, nre, mat, 0,
                                       empty_slots);
            CNT_ADD(C_RECHECKS, nre);
            CNT_ADD(C_D_BYTES, 16ull * (unsigned long long)sh.eread + 24ull * (unsigned long long)s.B);
        } else {
            merge_pair(sh, s, win.si, win.sj, R, E, merges, kind, win.d2, g_ready, prec, rcs);
        }
        ++merges;
        --R;
        if (rcs == 2) npend = sh.npend;
        if (s.abit && rcs) abit_merge(s, win.si, win.sj, R + 1);
        if (row_cache && rcs == 0 && lp.spectral && R <= lp.kmax && R > s.stop) {
            rowcache_begin(sh, s, R, E, mat);  // the spectral stage starts with the next iteration
            rcs = 1;
        }
        if (step2 && lp.spectral && R <= lp.kmax && R > s.stop) {
            st3 = 1;
            thr3 = lp.w2 * win.d2;
        }
        CNT_ADD(C_T_MERGE, wall_clock64() - tk0);
    }
#undef CNT_ADD
    if (tid == 0) {
        s.st[0] = R;
        s.st[1] = E;
        s.st[4] = g_ready;
        if (row_cache) {
            s.st[6] = rcs;
            s.st[7] = npend;
            s.st[11] = 0;  // appended rows are folded in within their iteration
        }
        s.st[8] = 0;  // the driver keeps its adjacent minimum in registers
        if (lp.two_merges) {
            s.st[10] = st3;
            s.wd[3] = thr3;
        }
        if (lp.counters)
            for (int c = 0; c < C_COUNT; ++c)
                if (sh.cnt[c]) atomicAdd(&lp.counters[c], sh.cnt[c]);
    }
}

// ---------------------------------------------------------------------------
// Wide mode: one merge-loop iteration of every section of a level as five
// launches, G workgroups per section sharing the sweeps. Launch boundaries
// order the phases; a section that has reached its stop count does nothing.
//   1 k_wide_adj       adjacent screen, edges split over G workgroups
//   2 k_wide_decide    adjacent decision; merge now if the spectral stage is off
//   3 k_wide_mfma      matrix-core tile screen, super tiles split over G
//   4 k_wide_fp32      FP32 tile screen, tiles split over G
//   5 k_wide_finish    spectral decision and merge
// Per-section iteration scratch: wi[0] phase (0 idle, 1 adjacent merged,
// 2 spectral pending), wi[1..4] A's lo, hi, si, sj, wi[5] use16, wi[6] checks;
// wd[0] A's D2, wd[1] T; wpart[g] adjacent and wpart[GMAX + g] spectral
// partial least upper bounds.
// ---------------------------------------------------------------------------
template <int EPG>
__global__ void __launch_bounds__(NT) k_wide_adj(const SecDev* __restrict__ secs, int G,
                                                 unsigned long long* counters) {
    __shared__ float red[NWAVE];  // only a block minimum: keep LDS small so several blocks fit a CU
    if (gated(counters)) return;
    const SecDev& s = secs[blockIdx.y];
    const int R = s.st[0], E = s.st[1];
    if (R <= s.stop) return;
    const float gam = (float)(2 * s.B + 32) * U32;
    const int per = (E + G - 1) / G;
    const int e0 = blockIdx.x * per, e1 = min(E, e0 + per);
    float U = wave_min_f(adj_screen_range<EPG>(s, e0, e1, gam));
    if (lane_id() == 0) red[wave_id()] = U;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w) U = fminf(U, red[w]);
        s.wpart[blockIdx.x] = U;
        if (blockIdx.x == 0 && counters)
            atomicAdd(&counters[C_W_ADJ_BYTES],
                      4ull * (unsigned long long)R * (unsigned long long)s.B + 8ull * (unsigned long long)E + 8ull * R);
    }
}

// Row cache stage of one iteration (incremental form): G workgroups per
// section share the rows to re-evaluate (every row when the cache starts).
// Prefix sum of per-section task counts in pre[1..n] (pre[0] = 0), by wave 0.
__device__ __forceinline__ void task_prefix(int* pre, int n) {
    __syncthreads();
    if (wave_id() == 0) {  // inclusive scan of the task counts, 64 sections per step
        const int lane = lane_id();
        int carry = 0;
        for (int k0 = 0; k0 < n; k0 += 64) {  // wavefront-uniform
            const int k = k0 + lane;
            int v = k < n ? pre[k + 1] : 0;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(v, o);
                if (lane >= o) v += u;
            }
            if (k < n) pre[k + 1] = v + carry;
            carry += __shfl(v, 63);
        }
        if (lane == 0) pre[0] = 0;
    }
    __syncthreads();
}

// Section of task t: k with pre[k] <= t < pre[k + 1].
__device__ __forceinline__ int task_section(const int* pre, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(NT) k_wide_rows(const SecDev* __restrict__ secs, int n, LoopParams lp) {
    __shared__ double rsum[NWAVE][4][64];
    __shared__ int pre[ROWS_MAX_SECTIONS + 1];
    if (gated(lp.counters)) return;
    // tasks of every section of the level in one pool: section k owns tasks
    // [pre[k], pre[k + 1])
    for (int k = threadIdx.x; k < n; k += NT) {
        const SecDev& s = secs[k];
        const int R = s.st[0], mode = s.st[6];
        int cnt = 0;
        if (s.rcap > 0 && R > s.stop && R <= lp.kmax && (mode == 1 || mode == 2)) {
            const int np = mode == 1 ? R : s.st[7];
            cnt = row_task_count(R, np);
            if (blockIdx.x == 0 && lp.counters) {
                const unsigned long long pairs = (unsigned long long)np * (unsigned long long)(R - 1);
                atomicAdd(&lp.counters[C_RECHECKS], pairs);
                // columns read once per group of 4 rows, each task's rows once
                const unsigned long long B = (unsigned long long)s.B;
                const unsigned long long nch = (unsigned long long)((R + 63) >> 6);
                atomicAdd(&lp.counters[C_W_ROWS_BYTES], (unsigned long long)((np + 3) / 4) * (unsigned long long)R * B * 8ull +
                                                            (unsigned long long)np * nch * B * 8ull);
            }
        }
        pre[k + 1] = cnt;
    }
    task_prefix(pre, n);
    const int total = pre[n];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int k = task_section(pre, n, t);
        const SecDev s = secs[k];
        const int R = s.st[0];
        const bool all = s.st[6] == 1;
        const int np = all ? R : s.st[7];
        const int nch = (R + 63) >> 6;
        const int lt = t - pre[k];
        if (s.crit == HSWO_CRIT_SAM)
            row_block_task<4, true>(rsum, s, R, np, all, lt / nch, lt % nch);
        else
            row_block_task<4, false>(rsum, s, R, np, all, lt / nch, lt % nch);
    }
}

// Row stage of a level whose row caches keep the interval matrix: every row
// rescanned from its bounds when the cache starts (after k_mat_fill), else
// each pending row (one workgroup per row, row_matrix_task), in one pool over
// the level's sections.
__global__ void __launch_bounds__(NT) k_mat_rows(const SecDev* __restrict__ secs, int n, LoopParams lp) {
    __shared__ RowMatLds lds;
    __shared__ int pre[ROWS_MAX_SECTIONS + 1];
    if (gated(lp.counters)) return;
    for (int k = threadIdx.x; k < n; k += NT) {
        const SecDev& s = secs[k];
        const int R = s.st[0], mode = s.st[6];
        int cnt = 0;
        if (s.rcap > 0 && R > s.stop && R <= lp.kmax && (mode == 1 || mode == 2)) {
            cnt = mode == 1 ? R : s.st[7];
            if (blockIdx.x == 0 && lp.counters) {
                const unsigned long long np = (unsigned long long)cnt;
                atomicAdd(&lp.counters[C_ROW_BOUNDED], np * (unsigned long long)(R - 1));
                atomicAdd(&lp.counters[C_W_ROWS_BYTES], 8ull * np * (unsigned long long)R);  // the bounds rows
            }
        }
        pre[k + 1] = cnt;
    }
    task_prefix(pre, n);
    const int total = pre[n];
    unsigned long long ex = 0, exb = 0;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int k = task_section(pre, n, t);
        const SecDev s = secs[k];
        const int ne = row_matrix_task(lds, s, s.st[0], t - pre[k], s.st[6] == 1);
        ex += (unsigned long long)ne;
        exb += (unsigned long long)ne * (16ull * (unsigned long long)s.B + 16ull);  // two FP64 rows, two entries
    }
    if (threadIdx.x == 0 && ex && lp.counters) {
        atomicAdd(&lp.counters[C_RECHECKS], ex);
        atomicAdd(&lp.counters[C_W_ROWS_BYTES], exb);
    }
}

// Interval matrix of every section whose row cache starts in this iteration
// (state 1 with the matrix kept): one tile per workgroup (blockIdx.x; blockIdx.y
// the section).
__global__ void __launch_bounds__(NT) k_mat_fill(const SecDev* __restrict__ secs, LoopParams lp) {
    __shared__ float As[BK][TILE], Cs[BK][TILE];
    if (gated(lp.counters)) return;
    const SecDev& s = secs[blockIdx.y];
    const int R = s.st[0];
    if (!row_matrix_on(s, lp) || s.st[6] != 1 || R <= s.stop || R > lp.kmax) return;
    const int nT = (R + TILE - 1) / TILE;
    if ((int)blockIdx.x >= nT * (nT + 1) / 2) return;
    const unsigned long long pairs = mat_fill_tile<TILE>(As, Cs, s, R, (int)blockIdx.x);
    if (threadIdx.x == 0 && lp.counters) atomicAdd(&lp.counters[C_W_FILL_FLOPS], 3ull * (unsigned long long)s.B * pairs);
}

// Start the row caches of the sections whose pass begins inside the spectral
// stage (one workgroup per section).
__global__ void __launch_bounds__(NT) k_rowcache_prep(const SecDev* __restrict__ secs, LoopParams lp) {
    __shared__ Smem sh;
    if (gated(lp.counters)) return;
    const SecDev& s = secs[blockIdx.x];
    const int R = s.st[0];
    if (s.rcap == 0 || R <= s.stop || R > lp.kmax || s.st[6] != 0) return;
    rowcache_begin(sh, s, R, s.st[1], row_matrix_on(s, lp));
}

__global__ void __launch_bounds__(NT) k_wide_decide(const SecDev* __restrict__ secs, int G, LoopParams lp) {
    __shared__ Smem sh;
    if (gated(lp.counters)) return;
    const SecDev& s = secs[blockIdx.x];
    const int tid = threadIdx.x;
    const int R = s.st[0];
    int E = s.st[1];
    // rows whose light step in k_wide_rows fell back on a full evaluation
    const int nfall = s.st[11];
    if (R <= s.stop) {
        if (tid == 0) s.wi[0] = 0;
        return;
    }
    const int prec = s.kcap > 0 ? lp.precision : 0;
    if (tid == 0) sh.ncand = 0;
    __syncthreads();
    int nchk = 0;
    KeyD A;
    if (lp.incremental) {
        if (s.st[8]) {  // cached by the last merge
            A.d2 = s.wd[2];
            A.lo = s.wi[8];
            A.hi = s.wi[9];
            A.si = s.wi[10];
            A.sj = s.wi[11];
        } else {
            A = adj_incremental(sh, s, E, s.st[5] == 0, nchk);
            if (tid == 0) s.st[5] = 1;
        }
        __syncthreads();
    } else {
        float Ua = __builtin_huge_valf();
        for (int g = 0; g < G; ++g) Ua = fminf(Ua, s.wpart[g]);
        A = adj_collect(sh, s, R, E, Ua, nchk);
        if (tid == 0 && lp.counters) {
            atomicAdd(&lp.counters[C_SCREEN_ITERS], 1ull);
            if (nchk > lp.topk) atomicAdd(&lp.counters[C_SCREEN_FALLBACKS], 1ull);
        }
    }
    int empty_slots = s.st[9];
    const int Elive = E - empty_slots;
    const bool spectral = lp.spectral && R <= lp.kmax;
    const double T = key_exists(A) ? lp.w2 * A.d2 : __builtin_huge_val();
    const bool row_cache = lp.incremental && s.rcap > 0;
    if (!spectral || row_cache) {
        // the adjacent stage alone, or the spectral minimum from the row cache
        // (its pending rows were re-evaluated by k_wide_rows)
        int rcs = row_cache ? s.st[6] : 0;
        KeyD M = key_none();
        unsigned long long decide_bytes = 0;  // algorithmic bytes of this iteration (incremental form)
        if (spectral) {
            const bool all = rcs == 1;
            const int np = all ? R : s.st[7];
            const int nf = all ? 0 : nfall;
            if (nf > 0) {
                rows_fallback_lanes(s, R, np, nf);
                __syncthreads();
                nchk += nf * (R - 1);
                decide_bytes += 8ull * (unsigned long long)s.B * (unsigned long long)R;
            }
            M = spectral_min_rows(sh, s, R, np + nf, all);
            rcs = 2;
            decide_bytes += 12ull * (unsigned long long)R +
                            32ull * (unsigned long long)(np + nf) * (unsigned long long)((R + 63) >> 6);
        }
        KeyD win;
        int kind;
        bool merge_now, step2 = false;
        const bool st3 = lp.two_merges && s.st[10];
        if (st3 && key_exists(M) && M.d2 < s.wd[3]) {
            // two-merge reading, step 3: the least non-adjacent pair is below w^2 times step 2's value
            merge_now = true;
            win = M;
            kind = 1;
        } else if (lp.two_merges && key_exists(A)) {
            // step 2: the least adjacent pair, whatever the spectral minimum -- also at once when
            // step 3 found no pair (nothing changed since, so the next iteration starts here)
            merge_now = true;
            win = A;
            kind = 0;
            step2 = true;
        } else {
            merge_now = decide(spectral, A, M, T, win, kind);
        }
        if (lp.two_merges) __syncthreads();  // every thread has read st[10] and wd[3] (kernel-uniform)
        if (lp.two_merges && tid == 0) {
            s.st[10] = (step2 && lp.spectral && R - 1 <= lp.kmax && R - 1 > s.stop) ? 1 : 0;
            s.wd[3] = step2 ? lp.w2 * win.d2 : 0.0;
        }
        if (!merge_now && row_cache && tid == 0) {
            s.st[6] = rcs;  // the pending rows were folded in above
            s.st[7] = 0;
            s.st[11] = 0;
        }
        if (merge_now) {
            const int stamp = s.st[3];
            if (!lp.incremental) decide_bytes += 16ull * (unsigned long long)E + 24ull * (unsigned long long)s.B;
            if (lp.incremental) {
                KeyD an;
                const bool av = merge_pair_inc<4>(sh, s, win.si, win.sj, R, E, stamp, kind, win.d2, rcs, an, nchk,
                                                  row_matrix_on(s, lp), EIDX_MIN, empty_slots);
                decide_bytes += 16ull * (unsigned long long)sh.eread + 24ull * (unsigned long long)s.B;
                if (tid == 0) {
                    s.st[8] = av ? 1 : 0;
                    s.wd[2] = an.d2;
                    s.wi[8] = an.lo;
                    s.wi[9] = an.hi;
                    s.wi[10] = an.si;
                    s.wi[11] = an.sj;
                }
            } else {
                merge_pair(sh, s, win.si, win.sj, R, E, stamp, kind, win.d2, s.st[4], prec, rcs);
            }
            if (tid == 0) {
                s.st[0] = R - 1;
                s.st[1] = E;
                if (row_cache) s.st[6] = rcs;
            }
            if (s.abit && rcs) abit_merge(s, win.si, win.sj, R);
            if (row_cache && rcs == 0 && lp.spectral && R - 1 <= lp.kmax && R - 1 > s.stop)
                rowcache_begin(sh, s, R - 1, E, row_matrix_on(s, lp));
        }
        if (tid == 0) {
            s.wi[0] = 1;
            if (lp.counters) {
                atomicAdd(&lp.counters[C_ITERS], 1ull);
                if (merge_now) atomicAdd(&lp.counters[C_MERGES], 1ull);
                atomicAdd(&lp.counters[C_ADJ_PAIRS], (unsigned long long)Elive);
                atomicAdd(&lp.counters[C_RECHECKS], (unsigned long long)nchk);
                if (spectral)
                    atomicAdd(&lp.counters[C_SPEC_PAIRS], (unsigned long long)R * (unsigned long long)(R - 1) / 2ull);
                if (lp.incremental)
                    atomicAdd(&lp.counters[C_W_DECIDE_BYTES], decide_bytes);
            }
        }
        return;
    }
    int g_ready = s.st[4];
    if (prec && !g_ready) {
        if (prec == 1)
            build16_all<1>(s, R);
        else
            build16_all<2>(s, R);
        g_ready = 1;
    }
    const bool use16 = prec && T < __builtin_huge_val();
    if (use16) {
        prep_alpha_p(s, R, T);
        clear_tile_flags(s, R);
    }
    if (tid == 0) {
        s.st[4] = g_ready;
        s.wi[0] = 2;
        s.wi[1] = A.lo;
        s.wi[2] = A.hi;
        s.wi[3] = A.si;
        s.wi[4] = A.sj;
        s.wi[5] = use16 ? 1 : 0;
        s.wi[6] = nchk;
        s.wd[0] = A.d2;
        s.wd[1] = T;
        if (lp.counters) atomicAdd(&lp.counters[C_ADJ_PAIRS], (unsigned long long)E);
    }
}

template <int PREC>
__global__ void __launch_bounds__(NT) k_wide_mfma(const SecDev* __restrict__ secs, int G, LoopParams lp) {
    __shared__ Smem sh;
    if (gated(lp.counters)) return;
    const SecDev s = secs[blockIdx.y];
    if (s.wi[0] != 2 || !s.wi[5]) return;
    const int R = s.st[0];
    const int n = mfma_screen<PREC>(sh, s, R, blockIdx.x, G);
    if (threadIdx.x == 0 && lp.counters) {
        atomicAdd(&lp.counters[C_MFMA_TILES], (unsigned long long)n);
        if (blockIdx.x == 0)
            atomicAdd(&lp.counters[C_W_MFMA_FLOPS],
                      (unsigned long long)s.B * (unsigned long long)R * (unsigned long long)(R - 1));
    }
}

__global__ void __launch_bounds__(NT) k_wide_fp32(const SecDev* __restrict__ secs, int G, LoopParams lp) {
    __shared__ Smem sh;
    if (gated(lp.counters)) return;
    const SecDev& s = secs[blockIdx.y];
    if (s.wi[0] != 2) return;
    const float gam = (float)(2 * s.B + 32) * U32;
    int nf = 0;
    const float Us = fp32_tiles(sh, s, s.st[0], s.wi[5] != 0, gam, blockIdx.x, G, nf);
    if (threadIdx.x == 0) {
        s.wpart[GMAX + blockIdx.x] = Us;
        if (lp.counters) atomicAdd(&lp.counters[C_FP32_TILES], (unsigned long long)nf);
    }
}

__global__ void __launch_bounds__(NT) k_wide_finish(const SecDev* __restrict__ secs, int G, LoopParams lp) {
    __shared__ Smem sh;
    if (gated(lp.counters)) return;
    const SecDev& s = secs[blockIdx.x];
    const int tid = threadIdx.x;
    if (s.wi[0] != 2) return;
    const int R = s.st[0];
    int E = s.st[1];
    const int prec = s.kcap > 0 ? lp.precision : 0;
    if (tid == 0) sh.ncand = 0;
    __syncthreads();
    KeyD A;
    A.d2 = s.wd[0];
    A.lo = s.wi[1];
    A.hi = s.wi[2];
    A.si = s.wi[3];
    A.sj = s.wi[4];
    const double T = s.wd[1];
    int nchk = s.wi[6], nresc = 0;
    float Us = __builtin_huge_valf();
    for (int g = 0; g < G; ++g) Us = fminf(Us, s.wpart[GMAX + g]);
    const double theta = fmin((double)Us, T);
    const float gam = (float)(2 * s.B + 32) * U32;
    const int c1 = nchk;
    const KeyD M = spectral_collect(sh, s, R, T, theta, gam, nchk, nresc, s.wi[5] ? prec : 0);
    if (tid == 0 && lp.counters) {
        atomicAdd(&lp.counters[C_SCREEN_ITERS], 1ull);
        if (nchk - c1 > lp.topk) atomicAdd(&lp.counters[C_SCREEN_FALLBACKS], 1ull);
    }
    KeyD win;
    int kind;
    if (decide(true, A, M, T, win, kind)) {
        merge_pair(sh, s, win.si, win.sj, R, E, s.st[3], kind, win.d2, s.st[4], prec, 0);
        if (tid == 0) {
            s.st[0] = R - 1;
            s.st[1] = E;
        }
    }
    if (tid == 0 && lp.counters) {
        atomicAdd(&lp.counters[C_ITERS], 1ull);
        atomicAdd(&lp.counters[C_MERGES], 1ull);
        atomicAdd(&lp.counters[C_SPEC_PAIRS], (unsigned long long)R * (unsigned long long)(R - 1) / 2ull);
        atomicAdd(&lp.counters[C_RECHECKS], (unsigned long long)nchk);
        atomicAdd(&lp.counters[C_RESCANS], (unsigned long long)nresc);
    }
}

// ---------------------------------------------------------------------------
// Initialisation, reassembly, compression and snapshots.
// ---------------------------------------------------------------------------
__global__ void k_init_pixels(int32_t* parent, int32_t* mtime, int64_t n) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        parent[p] = (int32_t)p;
        mtime[p] = INT_MAX;
    }
}

// Batch sections: labels are local pixel indices of each section.
__global__ void k_init_pixels_secs(const SecDev* __restrict__ secs) {
    const SecDev& s = secs[blockIdx.y];
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < s.R0; p += gridDim.x * blockDim.x) {
        s.parent[p] = p;
        s.mtime[p] = INT_MAX;
    }
}

template <typename T>
__device__ __forceinline__ float load_px(const void* cube, size_t idx) {
    return (float)reinterpret_cast<const T*>(cube)[idx];
}

template <>
__device__ __forceinline__ float load_px<__half>(const void* cube, size_t idx) {
    return __half2float(reinterpret_cast<const __half*>(cube)[idx]);
}

// Every pixel of a leaf section becomes a region (HSEG step 1): label = its
// pixel index, one pixel, band sums = its spectrum; plus the section's grid
// edges under 4- or 8-connectivity.
template <typename T>
__global__ void k_init_leaves(const SecDev* __restrict__ secs, const InitDev* __restrict__ init,
                              unsigned long long* counters) {
    const SecDev& s = secs[blockIdx.y];
    const InitDev in = init[blockIdx.y];
    const int h = in.h, w = in.w, B = s.B, Bp = s.Bp;
    const int P = h * w;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // band sums and mean rows; non-finite values are counted (the call then stops)
    unsigned nonfinite = 0;
    for (int64_t idx = t0; idx < (int64_t)P * Bp; idx += stride) {
        const int k = (int)(idx / Bp), b = (int)(idx % Bp);
        const int r = k / w, c = k % w;
        float v = 0.0f;
        if (b < B) {
            v = load_px<T>(in.cube, ((size_t)(in.r0 + r) * in.img_w + (in.c0 + c)) * B + b);
            nonfinite += isfinite(v) ? 0u : 1u;
            s.sums[(size_t)k * B + b] = (double)v;
        }
        s.mean[(size_t)k * Bp + b] = v;
    }
    if (nonfinite) atomicAdd(&counters[C_NONFINITE], (unsigned long long)nonfinite);
    // per-pixel region data
    for (int64_t k = t0; k < P; k += stride) {
        const int r = (int)k / w, c = (int)k % w;
        s.label[k] = (in.r0 + r) * in.label_w + (in.c0 + c);
        s.npix[k] = 1;
        s.mark[k] = -1;
        const size_t base = ((size_t)(in.r0 + r) * in.img_w + (in.c0 + c)) * B;
        double nrm = 0.0;
        for (int b = 0; b < B; ++b) {
            const double v = (double)load_px<T>(in.cube, base + b);
            nrm += v * v;
        }
        s.norm[k] = (float)(sqrt(nrm) * (1.0 + 0x1p-20));
    }
    // grid edges in pixel order: pixel k owns slots k*nf .. k*nf+nf-1 for its
    // right, down (and, under 8-connectivity, down-right, down-left)
    // neighbours, so the two rows of consecutive edges stay close. Slots
    // without a neighbour hold (-1,-1): the screen gives them +inf bounds and
    // the first merge's order-preserving compaction removes them.
    const int nf = in.conn == 8 ? 4 : 2;
    const int64_t E0 = (int64_t)P * nf;
    for (int64_t e = t0; e < E0; e += stride) {
        const int k = (int)(e / nf), f = (int)(e % nf);
        const int r = k / w, c = k % w;
        int a = -1, b = -1;
        if (f == 0 && c + 1 < w) {
            a = k;
            b = k + 1;
        } else if (f == 1 && r + 1 < h) {
            a = k;
            b = k + w;
        } else if (f == 2 && r + 1 < h && c + 1 < w) {
            a = k;
            b = k + w + 1;
        } else if (f == 3 && r + 1 < h && c >= 1) {
            a = k;
            b = k + w - 1;
        }
        s.edges[e] = make_int2(a, b);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.st[0] = P;
        s.st[1] = (int)E0;
        s.st[2] = P;
        s.st[3] = 0;
        s.st[4] = 0;
        s.st[5] = 0;
        s.st[6] = 0;
        s.st[7] = 0;
        s.st[8] = 0;
        s.st[9] = 0;
        s.st[10] = 0;
        s.st[11] = 0;
        s.st[12] = 0;
    }
}

// Path compression of the label union-find: parent[p] becomes p's root.
// Concurrent updates only ever store an ancestor, so every walk still ends
// at the root.
__global__ void k_compress(int32_t* parent, int64_t n, const unsigned long long* gate) {
    if (gated(gate)) return;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        int x = parent[p];
        for (int64_t step = 0; step < n; ++step) {  // a chain is never longer than n
            const int y = parent[x];
            if (y == x) break;
            x = y;
        }
        parent[p] = x;
    }
}

__global__ void k_empty() {}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Reassembly (Figure 4.4), part 1: the parent's regions are the live regions
// of its four children in order TL, TR, BL, BR; children's edges are kept.
__global__ void k_assemble(const SecDev* __restrict__ parents, const SecDev* __restrict__ children,
                           const AsmDev* __restrict__ asm_, int32_t* slotmap, const unsigned long long* gate) {
    if (gated(gate)) return;
    const SecDev p = parents[blockIdx.y];
    const AsmDev a = asm_[blockIdx.y];
    int off[5], eoff[5];
    off[0] = 0;
    eoff[0] = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        off[c + 1] = off[c] + children[a.child0 + c].st[0];
        eoff[c + 1] = eoff[c] + children[a.child0 + c].st[1];
    }
    if (off[4] > p.R0 || eoff[4] > p.Ecap) {
        // cannot happen when every child pass ran to its stop count (sections
        // are connected); never write past the parent's capacity
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            p.st[0] = 0;
            p.st[1] = 0;
            p.st[2] = 0;
            p.st[3] = 0;
            p.st[4] = 0;
            p.st[5] = 0;
            p.st[6] = 0;
            p.st[7] = 0;
            p.st[8] = 0;
            p.st[9] = 0;
            p.st[10] = 0;
            p.st[11] = 0;
            p.st[12] = 0;
        }
        return;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int B = p.B, Bp = p.Bp;
    for (int c = 0; c < 4; ++c) {
        const SecDev ch = children[a.child0 + c];
        const int Rc = off[c + 1] - off[c], Ec = eoff[c + 1] - eoff[c];
        for (int64_t k = t0; k < Rc; k += stride) {
            const int ps = off[c] + (int)k;
            const int lab = ch.label[k];
            p.label[ps] = lab;
            p.npix[ps] = ch.npix[k];
            p.norm[ps] = ch.norm[k];
            p.mark[ps] = -1;
            slotmap[lab] = ps;
        }
        for (int64_t idx = t0; idx < (int64_t)Rc * B; idx += stride)
            p.sums[(size_t)off[c] * B + idx] = ch.sums[idx];
        for (int64_t idx = t0; idx < (int64_t)Rc * Bp; idx += stride)
            p.mean[(size_t)off[c] * Bp + idx] = ch.mean[idx];
        for (int64_t e = t0; e < Ec; e += stride) {
            const int2 ed = ch.edges[e];
            // empty slots (a child that made no merge still has them) stay empty
            p.edges[eoff[c] + e] = ed.x < 0 ? make_int2(-1, -1) : make_int2(ed.x + off[c], ed.y + off[c]);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.st[0] = off[4];
        p.st[1] = eoff[4];
        p.st[2] = off[4];
        p.st[3] = 0;
        p.st[4] = 0;
        p.st[5] = 0;
        p.st[6] = 0;
        p.st[7] = 0;
        p.st[8] = 0;
        p.st[9] = 0;
        p.st[10] = 0;
        p.st[11] = 0;
        p.st[12] = 0;
    }
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// Reassembly, part 2: link the regions on either side of the two split lines
// (pixel pairs in different quadrants that are neighbours under the seam
// connectivity), one edge per distinct region pair.
__global__ void k_seam(const SecDev* __restrict__ parents, const AsmDev* __restrict__ asm_,
                       const int32_t* __restrict__ slotmap, const unsigned long long* gate) {
    if (gated(gate)) return;
    const SecDev p = parents[blockIdx.y];
    const AsmDev a = asm_[blockIdx.y];
    const int h0 = a.h / 2, w0 = a.w / 2;
    const int rs = a.r0 + h0 - 1;      // row above the horizontal split
    const int cs0 = a.c0 + w0 - 1;     // columns either side of the vertical split
    const int ncand = a.w + 2 * a.h;   // candidate pixels: that row, those two columns
    const int noff = a.seam_conn == 8 ? 4 : 2;
    const int dr[4] = {0, 1, 1, 1};
    const int dc[4] = {1, 0, 1, -1};
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)ncand * noff;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(idx / noff), o = (int)(idx % noff);
        int r, c;
        if (ci < a.w) {
            r = rs;
            c = a.c0 + ci;
        } else {
            const int k = ci - a.w;
            r = a.r0 + (k >> 1);
            c = cs0 + (k & 1);
        }
        if (r < a.r0 || c < a.c0 || c >= a.c0 + a.w) continue;
        const int r2 = r + dr[o], c2 = c + dc[o];
        if (r2 >= a.r0 + a.h || c2 < a.c0 || c2 >= a.c0 + a.w) continue;
        const int q1 = (r - a.r0 >= h0 ? 2 : 0) + (c - a.c0 >= w0 ? 1 : 0);
        const int q2 = (r2 - a.r0 >= h0 ? 2 : 0) + (c2 - a.c0 >= w0 ? 1 : 0);
        if (q1 == q2) continue;
        const int la = p.parent[(size_t)r * a.img_w + c];
        const int lb = p.parent[(size_t)r2 * a.img_w + c2];
        if (la == lb) continue;
        int sa = slotmap[la], sb = slotmap[lb];
        if (sa > sb) {
            const int t = sa; sa = sb; sb = t;
        }
        const unsigned long long key = ((unsigned long long)(unsigned)sa << 32) | (unsigned)sb;
        unsigned long long hsh = mix64(key) & (unsigned long long)(a.hash_cap - 1);
        for (int probe = 0; probe < a.hash_cap; ++probe) {
            const unsigned long long old = atomicCAS(&a.hash[hsh], ~0ull, key);
            if (old == ~0ull) {
                const int e = atomicAdd(&p.st[1], 1);
                p.edges[e] = make_int2(sa, sb);
                break;
            }
            if (old == key) break;
            hsh = (hsh + 1) & (unsigned long long)(a.hash_cap - 1);
        }
    }
}

// Label maps of the requested hierarchy levels of a top pass. A level with
// count c is the state after k = max(0, R_start - c) top-pass merges: walk
// from the pixel's region at the start of the pass along merges made before k.
__global__ void k_snapshot(const SnapDev* __restrict__ snaps, const int32_t* __restrict__ counts, int n_levels,
                           const unsigned long long* gate) {
    if (gated(gate)) return;
    const SnapDev sd = snaps[blockIdx.y];
    const int P = sd.h * sd.w;
    const int Rs = sd.st[2];
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)P * n_levels;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int lvl = (int)(idx / P), k = (int)(idx % P);
        const int r = k / sd.w, c = k % sd.w;
        const int kcut = Rs - counts[lvl] > 0 ? Rs - counts[lvl] : 0;
        int x = (sd.r0 + r) * sd.label_w + (sd.c0 + c);
        int steps = 0;
        while (sd.mtime[x] < kcut && steps <= P) {  // bounded: a valid chain is shorter than P
            x = sd.parent[x];
            ++steps;
        }
        sd.labels[idx] = steps > P ? -1 : x;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t n, int bs, int cap) {
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_init_pixels(int32_t* parent, int32_t* mtime, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_init_pixels, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, parent, mtime, n);
    return hipGetLastError();
}

hipError_t launch_init_pixels_secs(const SecDev* secs, int n, int max_pixels, hipStream_t s) {
    hipLaunchKernelGGL(k_init_pixels_secs, dim3(grid_for(max_pixels, 256, 256), n), dim3(256), 0, s, secs);
    return hipGetLastError();
}

hipError_t launch_init_leaves(const SecDev* secs, const InitDev* init, int n, int dtype, int max_pixels,
                              unsigned long long* counters, hipStream_t s) {
    const dim3 grid(grid_for((int64_t)max_pixels * 8, 256, 1024), n);
    if (dtype == HSWO_F16)
        hipLaunchKernelGGL(k_init_leaves<__half>, grid, dim3(256), 0, s, secs, init, counters);
    else
        hipLaunchKernelGGL(k_init_leaves<float>, grid, dim3(256), 0, s, secs, init, counters);
    return hipGetLastError();
}

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

hipError_t launch_section_driver(const SecDev* secs, int n, const LoopParams& lp, int variant, hipStream_t s,
                                 KTimer* kt) {
    // variant = edges in flight per 16-lane group in the adjacent stage (tunable, result-neutral)
    if (variant == 2)
        KLAUNCH(HSWO_K_SECTION_DRIVER, k_section_driver<2>, dim3(n), dim3(NT), secs, n, lp);
    else if (variant == 4)
        KLAUNCH(HSWO_K_SECTION_DRIVER, k_section_driver<4>, dim3(n), dim3(NT), secs, n, lp);
    else
        KLAUNCH(HSWO_K_SECTION_DRIVER, k_section_driver<6>, dim3(n), dim3(NT), secs, n, lp);
    return hipGetLastError();
}

int default_rows_grid() {
    static int g = 0;
    if (!g) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        g = 2 * cus;
    }
    return g;
}

hipError_t launch_rowcache_prep(const SecDev* secs, int n, const LoopParams& lp, hipStream_t s, KTimer* kt) {
    KLAUNCH(HSWO_K_ROWCACHE_PREP, k_rowcache_prep, dim3(n), dim3(NT), secs, lp);
    return hipGetLastError();
}

hipError_t launch_wide_iteration(const SecDev* secs, int n, int G, const LoopParams& lp, int variant,
                                 bool spectral_possible, bool row_cache, int rows_grid, int fill_tiles, hipStream_t s,
                                 KTimer* kt) {
    const dim3 grid(G, n);
    if (row_cache) {  // incremental form: cached adjacent values and spectral rows
        if (spectral_possible) {
            if (lp.row_matrix) {
                if (fill_tiles > 0)
                    KLAUNCH(HSWO_K_MATRIX_FILL, k_mat_fill, dim3(fill_tiles, n), dim3(NT), secs, lp);
                KLAUNCH(HSWO_K_WIDE_ROWS, k_mat_rows, dim3(rows_grid), dim3(NT), secs, n, lp);
            } else {
                KLAUNCH(HSWO_K_WIDE_ROWS, k_wide_rows, dim3(rows_grid), dim3(NT), secs, n, lp);
            }
        }
        KLAUNCH(HSWO_K_WIDE_DECIDE, k_wide_decide, dim3(n), dim3(NT), secs, G, lp);
        return hipGetLastError();
    }
    if (!lp.incremental) {
        if (variant == 2)
            KLAUNCH(HSWO_K_WIDE_ADJ, k_wide_adj<2>, grid, dim3(NT), secs, G, lp.counters);
        else if (variant == 4)
            KLAUNCH(HSWO_K_WIDE_ADJ, k_wide_adj<4>, grid, dim3(NT), secs, G, lp.counters);
        else
            KLAUNCH(HSWO_K_WIDE_ADJ, k_wide_adj<6>, grid, dim3(NT), secs, G, lp.counters);
    }
    KLAUNCH(HSWO_K_WIDE_DECIDE, k_wide_decide, dim3(n), dim3(NT), secs, G, lp);
    if (spectral_possible) {
        if (lp.precision == 1)
            KLAUNCH(HSWO_K_WIDE_MFMA, k_wide_mfma<1>, grid, dim3(NT), secs, G, lp);
        else if (lp.precision == 2)
            KLAUNCH(HSWO_K_WIDE_MFMA, k_wide_mfma<2>, grid, dim3(NT), secs, G, lp);
        KLAUNCH(HSWO_K_WIDE_FP32, k_wide_fp32, grid, dim3(NT), secs, G, lp);
        KLAUNCH(HSWO_K_WIDE_FINISH, k_wide_finish, dim3(n), dim3(NT), secs, G, lp);
    }
    return hipGetLastError();
}

hipError_t launch_compress(int32_t* parent, int64_t n, const unsigned long long* gate, hipStream_t s) {
    hipLaunchKernelGGL(k_compress, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, parent, n, gate);
    return hipGetLastError();
}

hipError_t launch_empty(hipStream_t s) {
    hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for((int64_t)n, 256, 4096)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_assemble(const SecDev* parents, const SecDev* children, const AsmDev* asm_, int n,
                           int32_t* slotmap, int max_cap, const unsigned long long* gate, hipStream_t s) {
    const dim3 grid(grid_for((int64_t)max_cap * 64, 256, 512), n);
    hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, s, parents, children, asm_, slotmap, gate);
    return hipGetLastError();
}

hipError_t launch_seam(const SecDev* parents, const AsmDev* asm_, int n, const int32_t* slotmap, int max_seam,
                       const unsigned long long* gate, hipStream_t s) {
    const dim3 grid(grid_for((int64_t)max_seam * 4, 256, 256), n);
    hipLaunchKernelGGL(k_seam, grid, dim3(256), 0, s, parents, asm_, slotmap, gate);
    return hipGetLastError();
}

hipError_t launch_snapshot(const SnapDev* snaps, int n, const int32_t* counts, int n_levels, int max_pixels,
                           const unsigned long long* gate, hipStream_t s) {
    const dim3 grid(grid_for((int64_t)max_pixels * n_levels, 256, 4096), n);
    hipLaunchKernelGGL(k_snapshot, grid, dim3(256), 0, s, snaps, counts, n_levels, gate);
    return hipGetLastError();
}

}  // namespace hswo
