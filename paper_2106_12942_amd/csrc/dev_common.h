// dev_common.h -- part of the device code of the HSWO / HSEG / RHSEG merge loop.
//
// Device building blocks shared by every kernel of the merge loop: the
// 16-bit operand formats, the exact lexicographic key (D2, lo, hi), the
// block's shared-memory union and the wave and block reductions.
#pragma once

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
[[maybe_unused]] __device__ double block_min_d(Smem& sh, double v) {
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

[[maybe_unused]] __device__ KeyD block_min_key(Smem& sh, KeyD k) {
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

}  // namespace

}  // namespace hswo
