// hswo_wide.hip -- CDNA4 (gfx950) kernels of the HSWO / HSEG / RHSEG hot path:
// wide mode (one merge-loop iteration of every section of a level per
// launch sequence, several workgroups per section) and the row-cache and
// interval-matrix task pools.

#include "dev_multi_merge.h"

namespace hswo {

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
// launchers
// ---------------------------------------------------------------------------

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

}  // namespace hswo
