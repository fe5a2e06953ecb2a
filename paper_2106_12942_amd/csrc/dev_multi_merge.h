// dev_multi_merge.h -- part of the device code of the HSWO / HSEG / RHSEG merge loop.
//
// Several merges per step for identical regions (the zero-valued pairs of
// a step, adjacent and non-adjacent).
#pragma once

#include "dev_stages.h"

namespace hswo {

namespace {

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
[[maybe_unused]] __device__ __noinline__ int zero_step_list(Smem& sh, const SecDev& s, int R, int E, bool spectral, int cap) {
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

}  // namespace

}  // namespace hswo
