// dev_screen.h -- part of the device code of the HSWO / HSEG / RHSEG merge loop.
//
// Screens of the spectral stage: the debug record of every screened pair,
// the FP64 re-check of candidate lists, the FP32 tile sums and the 16-bit
// matrix-core tile screen of the precision forms.
#pragma once

#include "dev_exact.h"

namespace hswo {

namespace {

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

}  // namespace

}  // namespace hswo
