// dev_stages.h -- part of the device code of the HSWO / HSEG / RHSEG merge loop.
//
// Block-level stages of one merge-loop iteration (adjacent screen and
// collection, spectral tiles, the decision of step 3, interval-matrix tile
// fills and wave rescans), shared by the persistent driver and wide mode.
#pragma once

#include "dev_merge.h"

namespace hswo {

namespace {

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
[[maybe_unused]] __device__ int row_matrix_wave(RowWaveLds& L, const SecDev& s, int R, int q, bool all) {
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
    const int P = rescan_group(s);
    for (int j0 = 0; j0 < R; j0 += 64) {  // wavefront-uniform
        const int j = j0 + lane;
        const float2 e = (j < R && j != i) ? Di[s.msl[j]] : make_float2(__builtin_huge_valf(), __builtin_huge_valf());
        const bool cand = j < R && j != i && (double)e.x * (1.0 - MAT_REL) <= T;
        if (cand && e.y == 0.0f) top2_merge(best, part_of(0.0, s.label[j], j));  // bounded by [0, 0]: exactly 0
        const bool put = cand && e.y != 0.0f;
        const unsigned long long mask = __ballot(put);
        const int cnt = __popcll(mask);
        if (n + cnt > WAVE_CAND) {  // wavefront-uniform: evaluate what the list holds first
            rescan_eval(s, i, cl, vl, n, 0, P);
            for (int k = lane; k < n; k += 64) top2_merge(best, part_of(vl[k], s.label[cl[k]], cl[k]));
            nexact += n;
            n = 0;
        }
        if (put) cl[n + __popcll(mask & ((1ull << lane) - 1ull))] = j;
        n += cnt;
    }
    rescan_eval(s, i, cl, vl, n, 0, P);
    for (int k = lane; k < n; k += 64) top2_merge(best, part_of(vl[k], s.label[cl[k]], cl[k]));
    nexact += n;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) top2_merge(best, shfl_xor_part(best, o));
    const int nch = (R + 63) >> 6;
    if (lane == 0) s.rpart[(size_t)q * nch] = best;
    for (int c = 1 + lane; c < nch; c += 64) s.rpart[(size_t)q * nch + c] = part_of(__builtin_huge_val(), INT_MAX, -1);
    return nexact;
}

}  // namespace

}  // namespace hswo
