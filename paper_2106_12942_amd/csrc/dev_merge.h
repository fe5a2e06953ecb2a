// dev_merge.h -- part of the device code of the HSWO / HSEG / RHSEG merge loop.
//
// The merge (HSEG step 4) and the incremental form's edge state: region
// statistics of the survivor, relabelling and de-duplication of the edge
// list (full pass or per-slot ranges), compaction, and the edge index of
// per-chunk least keys that the decision reads.
#pragma once

#include "dev_interval_matrix.h"

namespace hswo {

namespace {

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
constexpr int MERGE_XB = 4;  // entries per thread and round in merge_slots' loops over the live slots

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
        // MERGE_XB entries per thread with their loads in flight together: the slot map and
        // counts, then the two rows' bounds, then the stores (a loop over single entries waits
        // for each entry's two dependent loads in turn, its stores ordering the next loads)
        for (int k0 = 0; k0 < R; k0 += MERGE_XB * NT) {  // block-uniform
            int mk[MERGE_XB];
            double nk[MERGE_XB];
#pragma unroll
            for (int x = 0; x < MERGE_XB; ++x) {
                const int k = k0 + x * NT + tid;
                const bool on = k < R && k != lo_s && k != hi_s;
                mk[x] = on ? s.msl[k] : -1;
                nk[x] = on ? (double)s.npix[k] : 0.0;
            }
            float2 el[MERGE_XB], eh[MERGE_XB];
#pragma unroll
            for (int x = 0; x < MERGE_XB; ++x) {
                el[x] = mk[x] >= 0 ? Dl[mk[x]] : make_float2(0.0f, 0.0f);
                eh[x] = mk[x] >= 0 ? Dh[mk[x]] : make_float2(0.0f, 0.0f);
            }
#pragma unroll
            for (int x = 0; x < MERGE_XB; ++x)
                if (mk[x] >= 0) {
                    const float2 v = mat_update(el[x], eh[x], (double)de.x, (double)de.y, n_lo, n_hi, nk[x]);
                    Dl[mk[x]] = v;
                    s.dmat[(size_t)mk[x] * rcp + ml] = v;
                }
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
        for (int i0 = 0; i0 < R; i0 += MERGE_XB * NT) {  // block-uniform
            // the rows' cached partners loaded together first (the loop body stores row state)
            int pv[MERGE_XB], p2v[MERGE_XB];
#pragma unroll
            for (int x = 0; x < MERGE_XB; ++x) {
                const int i = i0 + x * NT + tid;
                const bool on = i < R && i != lo_s && i != hi_s;
                pv[x] = on ? s.rbp[i] : -1;
                p2v[x] = (on && !mat) ? s.rbp2[i] : -1;
            }
#pragma unroll
            for (int x = 0; x < MERGE_XB; ++x) {
                const int i = i0 + x * NT + tid;
                if (i >= R || i == lo_s || i == hi_s) continue;
                const int ni = (i == last) ? hi_s : i;
                const int p = pv[x];
                // the second bound follows a moved partner; when its partner is merged it stays as a
                // bare bound (-3) by default only if its value is 0 (identical spectra, where the
                // merged region usually ties again), else it is dropped (the interval matrix keeps
                // no second bounds)
                int np2 = -1;
                if (!mat) {
                    const int p2 = p2v[x];
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
// values (cmd2 the value, cml the labels, cme the pair's slots in label
// order, x = -1 for none). A merge renames the slot that moves in the records
// that name it, so the least record yields the next pair's slots without a
// load of its edge. Rebuilt from scratch when st[12] is 0 (pass start,
// compaction).

// Least key of chunk c into cmd2[c] / cme[c] / cml[c]; one wavefront.
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
            kk.si = la < lb ? ed.x : ed.y;
            kk.sj = la < lb ? ed.y : ed.x;
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
        s.cme[c] = key_exists(best) ? make_int2(best.si, best.sj) : make_int2(-1, -1);
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
    // each chunk's record holds its least key's labels and slots: one round of loads
    KeyD best = key_none();
    for (int c = threadIdx.x; c < (E + ECH - 1) / ECH; c += NT) {
        const int2 sl = s.cme[c];
        const double d2 = s.cmd2[c];
        const int2 lab = s.cml[c];
        if (sl.x < 0) continue;
        KeyD k;
        k.d2 = d2;
        k.lo = lab.x;
        k.hi = lab.y;
        k.si = sl.x;
        k.sj = sl.y;
        if (key_less(k, best)) best = k;
    }
    return block_min_key(sh, best);
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
    // rename the moved slot in L2 (the edges of L carry their neighbour in XL), and in the
    // chunk records of those edges (every edge of the moved slot is in L or L2, and the chunks
    // of L are taken anew; threads that share a chunk write the same record)
    for (int k = tid; k < n2; k += NT) {
        const int e = L2[k];
        int2 ed = s.edges[e];
        if (ed.x == last) ed.x = hi_s;
        if (ed.y == last) ed.y = hi_s;
        s.edges[e] = ed;
        if (use_index) {
            const int2 r = s.cme[e / ECH];
            if (r.x == last || r.y == last)
                s.cme[e / ECH] = make_int2(r.x == last ? hi_s : r.x, r.y == last ? hi_s : r.y);
        }
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
    } else if (means) {
        // 2 x 64 / Ls re-scored edges per wavefront at once: two per segment, which shares the
        // survivor's run between them (exact_seg_means2)
        const int ppw = 64 / Ls, sub = lane_id() / Ls;
        for (int q0 = wave_id() * 2 * ppw; q0 < nk; q0 += NWAVE * 2 * ppw) {  // wavefront-uniform trip count
            const int qa = q0 + sub, qb = q0 + ppw + sub;  // qb < nk implies qa < nk
            int xa = -1, xb = -1, ea = -1, eb = -1, la = 0, lb = 0;
            if (qa < nk) {
                const int k = K[qa];
                ea = L[k];
                xa = XL[k] == last ? hi_s : XL[k];
                la = KL[qa];
            }
            if (qb < nk) {
                const int k = K[qb];
                eb = L[k];
                xb = XL[k] == last ? hi_s : XL[k];
                lb = KL[qb];
            }
            double vb;
            const double va = exact_seg_means2(s, qa < nk ? surv : -1, xa, xb, Ls, vb);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = h ? qb : qa;
                if (q < nk) {
                    const int x = h ? xb : xa, lx = h ? lb : la;
                    KeyD kk;
                    kk.d2 = h ? vb : va;
                    kk.lo = min(l_surv, lx);
                    kk.hi = max(l_surv, lx);
                    kk.si = l_surv < lx ? surv : x;
                    kk.sj = l_surv < lx ? x : surv;
                    if ((lane_id() & (Ls - 1)) == 0) s.ed2[h ? eb : ea] = kk.d2;
                    if (key_less(kk, best)) best = kk;
                }
            }
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
            const double v = exact_seg(s, a, b, Ls);
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

}  // namespace hswo
