// hswo_driver.hip -- CDNA4 (gfx950) kernels of the HSWO / HSEG / RHSEG hot path:
// the persistent section driver.
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
// That is the screened and plain forms. The incremental form (the fastest)
// keeps instead the exact FP64 value of every edge slot and an index of
// per-chunk least keys over the edge list, so a merge touches only the edges
// of the merged pair and of the slot that moves; and, once the spectral
// stage is on, per-row least pairs backed by an interval matrix of certified
// FP32 bounds that Ward's recurrence keeps valid across merges, so only the
// rows whose cached partner was merged are rescanned, and only the pairs
// whose lower bound can beat a row's second least upper bound are evaluated
// exactly.
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

#include "dev_multi_merge.h"

namespace hswo {

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
// launcher
// ---------------------------------------------------------------------------

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

}  // namespace hswo
