/*
 * hswo_oracle.cpp -- plain FP64 CPU oracle for HSWO / HSEG / RHSEG.
 *
 * TEST INFRASTRUCTURE ONLY (see hswo_oracle.h). Built with g++ -O2
 * -ffp-contract=off and no fast-math, so every floating-point operation below
 * is one IEEE-754 round-to-nearest operation in the order written.
 *
 * Two modes compute the same thing:
 *   brute  : every iteration recomputes the criterion for every adjacent
 *            pair and (when the spectral stage is on) every non-adjacent
 *            pair, straight from the region sums and counts.
 *   cached : keeps each region's best adjacent and best non-adjacent key and
 *            refreshes only what a merge changes. The criterion is a pure
 *            function of (sums, counts), so both modes must produce the same
 *            merge sequence; the tests check that.
 */
#include "hswo_oracle.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

namespace {

/* ---- Equation 1, squared, canonical operation order --------------------- *
 * fac = (n_i * n_j) / (n_i + n_j); per band d = S_i/n_i - S_j/n_j and d*d;
 * the band terms are added as a pairwise tree over the band index, padded
 * with zeros to the next power of two (adding +0.0 is exact, so the padding
 * changes nothing); D2 = fac * sum. */
double pairwise_sum(const double* v, int n /* a power of two */) {
    if (n == 1) return v[0];
    return pairwise_sum(v, n / 2) + pairwise_sum(v + n / 2, n / 2);
}

double criterion(const double* Si, const double* Sj, int64_t ni, int64_t nj, int B) {
    const double dni = (double)ni, dnj = (double)nj;
    const double fac = (dni * dnj) / (double)(ni + nj);
    int P = 1;
    while (P < B) P *= 2;
    double sq[4096];  /* B <= 4096 is validated on entry */
    for (int b = 0; b < P; ++b) sq[b] = 0.0;
    for (int b = 0; b < B; ++b) {
        const double d = Si[b] / dni - Sj[b] / dnj;
        sq[b] = d * d;
    }
    return fac * pairwise_sum(sq, P);
}

/* ---- spectral angle criterion (listed among the usable dissimilarities in
 * Section 4.1), ranked without acos or sqrt ------------------------------- *
 * c = <S_i, S_j> / (|S_i| |S_j|) is the cosine of the angle between the two
 * mean spectra (the counts cancel, so band sums serve). The ranked value is
 * D = 1 - sign(c) c^2, which equals sin^2(theta) for theta <= 90 degrees and
 * rises monotonically to 2 at 180 degrees, so it orders pairs exactly as the
 * angle does; like Equation 1 it is the square of the angle-like quantity
 * sin(theta), which is why the spectral weight enters squared for both.
 * Canonical order: dot, q_i = |S_i|^2 and q_j = |S_j|^2 are each a pairwise
 * tree over the zero-padded band index; t = (dot * dot) / (q_i * q_j);
 * D = 1 - t if dot >= 0 else 1 + t; D < 0 (rounding) is raised to 0; a zero
 * spectrum (q_i * q_j == 0) gives D = 1, as for orthogonal spectra. */
double sam(const double* Si, const double* Sj, int B) {
    int P = 1;
    while (P < B) P *= 2;
    double dt[4096], qi[4096], qj[4096];
    for (int b = 0; b < P; ++b) dt[b] = qi[b] = qj[b] = 0.0;
    for (int b = 0; b < B; ++b) {
        dt[b] = Si[b] * Sj[b];
        qi[b] = Si[b] * Si[b];
        qj[b] = Sj[b] * Sj[b];
    }
    const double dot = pairwise_sum(dt, P);
    const double den = pairwise_sum(qi, P) * pairwise_sum(qj, P);
    if (den == 0.0) return 1.0;
    const double t = (dot * dot) / den;
    const double d = dot >= 0.0 ? 1.0 - t : 1.0 + t;
    return d > 0.0 ? d : 0.0;
}

double pair_value(int crit, const double* Si, const double* Sj, int64_t ni, int64_t nj, int B) {
    return crit == ORACLE_CRIT_SAM ? sam(Si, Sj, B) : criterion(Si, Sj, ni, nj, B);
}

/* ---- merge key: (D2, lo, hi), compared lexicographically (tie-break) ----- */
struct Key {
    double d2 = std::numeric_limits<double>::infinity();
    int lo = std::numeric_limits<int>::max();
    int hi = std::numeric_limits<int>::max();
};
const Key KEY_NONE = Key();
bool key_less(const Key& a, const Key& b) {
    if (a.d2 != b.d2) return a.d2 < b.d2;
    if (a.lo != b.lo) return a.lo < b.lo;
    return a.hi < b.hi;
}
bool key_exists(const Key& k) { return k.lo != std::numeric_limits<int>::max(); }

struct Rect {
    int r0, c0, h, w;
};

/* Quadrants of a rectangle: split at floor(h/2), floor(w/2); order TL, TR, BL, BR. */
void split4(const Rect& r, Rect q[4]) {
    const int h0 = r.h / 2, w0 = r.w / 2;
    q[0] = {r.r0, r.c0, h0, w0};
    q[1] = {r.r0, r.c0 + w0, h0, r.w - w0};
    q[2] = {r.r0 + h0, r.c0, r.h - h0, w0};
    q[3] = {r.r0 + h0, r.c0 + w0, r.h - h0, r.w - w0};
}

/* Global region state, indexed by region label (a pixel index). Sections of
   one recursion level own disjoint label sets, so threads never share one. */
struct State {
    int H, W, B;
    std::vector<int64_t> n;
    std::vector<double> S;                 /* label * B + b */
    std::vector<int> parent;               /* union-find over labels */
    /* spatial adjacency between live labels; the mapped value is the cached
       D2 of the edge (cached mode only) */
    std::vector<std::map<int, double>> adj;
    std::vector<Key> best_adj;             /* cached mode: best key over neighbours */
    double* Sp(int l) { return &S[(size_t)l * B]; }
    int find(int p) const {
        while (parent[p] != p) p = parent[p];
        return p;
    }
};

struct Snapshot {
    int32_t* labels;       /* [n_levels][H][W] */
    const int32_t* counts;
    int n_levels;
};

/* One HSEG pass over the live regions of one section. */
class Pass {
  public:
    Pass(State& st, const oracle_params& p, std::vector<int> live, int stop, bool top, const Rect& rect,
         const Snapshot* snap)
        : st_(st), p_(p), live_(std::move(live)), stop_(stop), top_(top), rect_(rect), snap_(snap) {
        w2_ = (double)p.spclust_wght * (double)p.spclust_wght;
    }

    void run(std::vector<oracle_merge>& log) {
        std::sort(live_.begin(), live_.end());
        int R = (int)live_.size();
        if (top_) snapshot_levels_at_start(R);
        if (!p_.brute) init_cache();
        if (p_.two_merges) {
            run_two_merges(log, R);
            return;
        }
        if (p_.multi_merge) {
            run_multi_merge(log, R);
            return;
        }
        while (R > stop_) {
            const bool spectral = spectral_at(R);
            Key A, N = KEY_NONE;
            if (p_.brute) {
                A = brute_adjacent();
                if (spectral) N = brute_nonadjacent();
            } else {
                if (spectral && !dense_on_) init_dense();
                A = cached_adjacent();
                if (spectral) N = cached_nonadjacent();
            }
            Key win;
            int kind;
            if (!winner(spectral, A, N, win, kind)) break;
            merge(win.lo, win.hi);
            --R;
            log.push_back({win.lo, win.hi, kind, R, win.d2});
            if (top_) snapshot_if_level(R);
        }
    }

  private:
    /* Step 3 of the HSEG loop: the non-adjacent pair is merged when it is
       smaller than the (weighted) adjacent minimum, else the adjacent pair;
       false when there is no pair at all. */
    bool winner(bool spectral, const Key& A, const Key& N, Key& win, int& kind) const {
        if (spectral && key_exists(N) && (!key_exists(A) || N.d2 < w2_ * A.d2)) {
            win = N;
            kind = 1;
        } else if (key_exists(A)) {
            win = A;
            kind = 0;
        } else {
            return false;
        }
        return true;
    }
    bool spectral_at(int R) const { return p_.spclust_wght > 0.0f && R <= p_.spclust_max; }
    Key adjacent_min() { return p_.brute ? brute_adjacent() : cached_adjacent(); }
    Key nonadjacent_min() {
        if (p_.brute) return brute_nonadjacent();
        if (!dense_on_) init_dense();
        return cached_nonadjacent();
    }
    void record(const Key& k, int kind, int& R, std::vector<oracle_merge>& log) {
        merge(k.lo, k.hi);
        --R;
        log.push_back({k.lo, k.hi, kind, R, k.d2});
        if (top_) snapshot_if_level(R);
    }

    /* The step list of Section 4.1 read with two merges per iteration: step 2
       merges the best adjacent pair A; step 3 then takes the best
       non-adjacent pair N of the partition that step 2 left (when the
       spectral stage is on at its region count) and merges it too iff it is
       below w^2 times A's value. Step 3 is skipped once step 2 has reached
       the stop count. Without any adjacent pair, the iteration falls back to
       the one-merge rule (N merged if it exists). */
    void run_two_merges(std::vector<oracle_merge>& log, int R) {
        while (R > stop_) {
            const Key A = adjacent_min();
            if (!key_exists(A)) {
                if (!spectral_at(R)) break;
                const Key N = nonadjacent_min();
                if (!key_exists(N)) break;
                record(N, 1, R, log);
                continue;
            }
            record(A, 0, R, log);
            if (R <= stop_ || !spectral_at(R)) continue;
            const Key N = nonadjacent_min();
            if (key_exists(N) && A.d2 * w2_ > N.d2) record(N, 1, R, log);  // strict, as in one-merge mode
        }
    }

    /* Several merges per step, the future-work item of Section 6.2 read for
       identical regions. A step starts like a one-merge iteration: the
       adjacent minimum A, the non-adjacent minimum N when the spectral stage
       is on, and the one-merge rule's winner. A winner above 0 is the step's
       only merge. A winner of value 0 opens a step of several merges: the
       zero-valued pairs are ranked the way the one-merge rule ranks them at
       that moment -- adjacent pairs first, by (lo, hi), then (spectral stage
       on) non-adjacent pairs, by (lo, hi) -- and taken greedily, a pair being
       skipped when one of its regions is already taken. The taken pairs are
       disjoint, so merging them one after another in that order changes
       neither the value nor the adjacency of a pair still to come; the step
       stops early at the pass's stop count. Its first merge is the winner. */
    void run_multi_merge(std::vector<oracle_merge>& log, int R) {
        while (R > stop_) {
            const bool spectral = spectral_at(R);
            if (!p_.brute && spectral && !dense_on_) init_dense();
            const Key A = adjacent_min();
            const Key N = spectral ? nonadjacent_min() : KEY_NONE;
            Key win;
            int kind;
            if (!winner(spectral, A, N, win, kind)) break;
            if (win.d2 != 0.0) {
                record(win, kind, R, log);
                continue;
            }
            std::vector<Key> za, zn;
            for (int i : live_)
                for (auto& kv : st_.adj[i])
                    if (i < kv.first && value_of(i, kv.first, kv.second) == 0.0) za.push_back(key(i, kv.first, 0.0));
            if (spectral)
                for (size_t a = 0; a < live_.size(); ++a)
                    for (size_t b = a + 1; b < live_.size(); ++b) {
                        const int i = live_[a], j = live_[b];
                        if (st_.adj[i].count(j)) continue;
                        if (nonadjacent_value(i, j) == 0.0) zn.push_back(key(i, j, 0.0));
                    }
            std::sort(za.begin(), za.end(), key_less);
            std::sort(zn.begin(), zn.end(), key_less);
            std::vector<std::pair<Key, int>> take;
            std::set<int> used;  /* labels taken in this step */
            for (int pass = 0; pass < 2; ++pass)
                for (const Key& k : pass == 0 ? za : zn)
                    if (!used.count(k.lo) && !used.count(k.hi)) {
                        used.insert(k.lo);
                        used.insert(k.hi);
                        take.push_back({k, pass});
                    }
            for (size_t t = 0; t < take.size() && R > stop_; ++t) {
                const Key& k = take[t].first;
                merge(k.lo, k.hi);
                --R;
                log.push_back({k.lo, k.hi, take[t].second + (t ? 2 : 0), R, k.d2});
                if (top_) snapshot_if_level(R);
            }
        }
    }
    /* the value of an adjacent pair: recomputed (brute) or the cached one */
    double value_of(int i, int j, double cached) { return p_.brute ? d2(i, j) : cached; }
    double nonadjacent_value(int i, int j) { return p_.brute ? d2(i, j) : Dat(didx_[i], didx_[j]); }

    double d2(int a, int b) {
        const int lo = std::min(a, b), hi = std::max(a, b);
        return pair_value(p_.criterion, st_.Sp(lo), st_.Sp(hi), st_.n[lo], st_.n[hi], st_.B);
    }
    Key key(int a, int b, double v) { return {v, std::min(a, b), std::max(a, b)}; }

    /* ---------------- brute mode -------------------------------------- */
    Key brute_adjacent() {
        Key best = KEY_NONE;
        for (int i : live_)
            for (auto& kv : st_.adj[i])
                if (i < kv.first) {
                    Key k = key(i, kv.first, d2(i, kv.first));
                    if (key_less(k, best)) best = k;
                }
        return best;
    }
    Key brute_nonadjacent() {
        Key best = KEY_NONE;
        for (size_t a = 0; a < live_.size(); ++a)
            for (size_t b = a + 1; b < live_.size(); ++b) {
                const int i = live_[a], j = live_[b];
                if (st_.adj[i].count(j)) continue;
                Key k = key(i, j, d2(i, j));
                if (key_less(k, best)) best = k;
            }
        return best;
    }

    /* ---------------- cached mode ------------------------------------- */
    /* State::best_adj[l]: lexicographic minimum over l's neighbours.
       dense: D2 of every live pair once the spectral stage is on, and each
       row's minimum over non-adjacent partners. */
    bool dense_on_ = false;
    std::map<int, int> didx_;               /* label -> dense index */
    std::vector<int> dlabel_;               /* dense index -> label */
    std::vector<double> D_;                 /* dense D2 matrix */
    std::vector<Key> best_na_;              /* per dense row */
    std::vector<char> dalive_;

    void refresh_best_adj(int i) {
        Key best = KEY_NONE;
        for (auto& kv : st_.adj[i]) {
            Key k = key(i, kv.first, kv.second);
            if (key_less(k, best)) best = k;
        }
        st_.best_adj[i] = best;
    }
    void init_cache() {
        for (int i : live_)
            for (auto& kv : st_.adj[i])
                if (i < kv.first) {
                    const double v = d2(i, kv.first);
                    kv.second = v;
                    st_.adj[kv.first][i] = v;
                }
        for (int i : live_) refresh_best_adj(i);
    }
    Key cached_adjacent() {
        Key best = KEY_NONE;
        for (int i : live_)
            if (key_less(st_.best_adj[i], best)) best = st_.best_adj[i];
        return best;
    }
    double& Dat(int a, int b) { return D_[(size_t)a * dlabel_.size() + b]; }
    void refresh_best_na(int a) {
        Key best = KEY_NONE;
        const int la = dlabel_[a];
        for (size_t b = 0; b < dlabel_.size(); ++b) {
            if (!dalive_[b] || (int)b == a) continue;
            const int lb = dlabel_[b];
            if (st_.adj[la].count(lb)) continue;
            Key k = key(la, lb, Dat(a, (int)b));
            if (key_less(k, best)) best = k;
        }
        best_na_[a] = best;
    }
    void init_dense() {
        dense_on_ = true;
        dlabel_ = live_;
        const size_t R = dlabel_.size();
        for (size_t a = 0; a < R; ++a) didx_[dlabel_[a]] = (int)a;
        D_.assign(R * R, 0.0);
        dalive_.assign(R, 1);
        for (size_t a = 0; a < R; ++a)
            for (size_t b = a + 1; b < R; ++b) {
                const double v = d2(dlabel_[a], dlabel_[b]);
                Dat((int)a, (int)b) = v;
                Dat((int)b, (int)a) = v;
            }
        best_na_.assign(R, KEY_NONE);
        for (size_t a = 0; a < R; ++a) refresh_best_na((int)a);
    }
    Key cached_nonadjacent() {
        Key best = KEY_NONE;
        for (size_t a = 0; a < dlabel_.size(); ++a)
            if (dalive_[a] && key_less(best_na_[a], best)) best = best_na_[a];
        return best;
    }

    /* ---------------- merge (Section 4.1: the merged region replaces both) */
    void merge(int lo, int hi) {
        double* Slo = st_.Sp(lo);
        const double* Shi = st_.Sp(hi);
        for (int b = 0; b < st_.B; ++b) Slo[b] = Slo[b] + Shi[b];
        st_.n[lo] += st_.n[hi];
        st_.parent[hi] = lo;
        /* adjacency of the merged region: union of both, minus the pair */
        std::vector<int> hin;
        for (auto& kv : st_.adj[hi]) hin.push_back(kv.first);
        for (int x : hin) {
            st_.adj[x].erase(hi);
            if (x != lo) {
                st_.adj[x][lo] = 0.0;
                st_.adj[lo][x] = 0.0;
            }
        }
        st_.adj[lo].erase(hi);
        st_.adj[hi].clear();
        live_.erase(std::lower_bound(live_.begin(), live_.end(), hi));
        if (p_.brute) return;

        /* cached mode: refresh what the merge changed */
        st_.best_adj[hi] = KEY_NONE;
        for (auto& kv : st_.adj[lo]) {
            const double v = d2(lo, kv.first);
            kv.second = v;
            st_.adj[kv.first][lo] = v;
        }
        refresh_best_adj(lo);
        for (auto& kv : st_.adj[lo]) {
            const int x = kv.first;
            const Key& bx = st_.best_adj[x];
            if (bx.lo == lo || bx.hi == lo || bx.lo == hi || bx.hi == hi)
                refresh_best_adj(x);
            else {
                Key k = key(x, lo, kv.second);
                if (key_less(k, bx)) st_.best_adj[x] = k;
            }
        }
        if (dense_on_) {
            const int a = didx_[lo], h = didx_[hi];
            dalive_[h] = 0;
            for (size_t b = 0; b < dlabel_.size(); ++b) {
                if (!dalive_[b] || (int)b == a) continue;
                const double v = d2(lo, dlabel_[b]);
                Dat(a, (int)b) = v;
                Dat((int)b, a) = v;
            }
            refresh_best_na(a);
            for (size_t b = 0; b < dlabel_.size(); ++b) {
                if (!dalive_[b] || (int)b == a) continue;
                const Key& bb = best_na_[b];
                if (bb.lo == lo || bb.hi == lo || bb.lo == hi || bb.hi == hi) {
                    refresh_best_na((int)b);
                } else if (!st_.adj[dlabel_[b]].count(lo)) {
                    Key k = key(dlabel_[b], lo, Dat((int)b, a));
                    if (key_less(k, bb)) best_na_[b] = k;
                }
            }
        }
    }

    /* ---------------- hierarchy snapshots (top pass only) -------------- */
    void write_level(int l) {
        int32_t* out = snap_->labels + (size_t)l * st_.H * st_.W;
        for (int r = rect_.r0; r < rect_.r0 + rect_.h; ++r)
            for (int c = rect_.c0; c < rect_.c0 + rect_.w; ++c) out[(size_t)r * st_.W + c] = st_.find(r * st_.W + c);
    }
    void snapshot_levels_at_start(int R) {
        for (int l = 0; l < snap_->n_levels; ++l)
            if (snap_->counts[l] >= R) write_level(l);
    }
    void snapshot_if_level(int R) {
        for (int l = 0; l < snap_->n_levels; ++l)
            if (snap_->counts[l] == R) write_level(l);
    }

    State& st_;
    const oracle_params& p_;
    std::vector<int> live_;
    int stop_;
    bool top_;
    Rect rect_;
    const Snapshot* snap_;
    double w2_;
};

/* Neighbour offsets (forward half) for 4- or 8-connectivity. */
int forward_offsets(int conn, int dr[4], int dc[4]) {
    dr[0] = 0; dc[0] = 1;
    dr[1] = 1; dc[1] = 0;
    if (conn == 4) return 2;
    dr[2] = 1; dc[2] = 1;
    dr[3] = 1; dc[3] = -1;
    return 4;
}

int quadrant_of(const Rect& r, int row, int col) {
    const int h0 = r.h / 2, w0 = r.w / 2;
    return (row - r.r0 >= h0 ? 2 : 0) + (col - r.c0 >= w0 ? 1 : 0);
}

void build_level_rects(const Rect& root, int L, std::vector<std::vector<Rect>>& levels) {
    levels.assign(L, {});
    levels[0].push_back(root);
    for (int d = 1; d < L; ++d)
        for (const Rect& r : levels[d - 1]) {
            Rect q[4];
            split4(r, q);
            for (int k = 0; k < 4; ++k) levels[d].push_back(q[k]);
        }
}

template <class F>
void parallel_for(int n, int n_threads, F f) {
    if (n_threads <= 1 || n <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    const int T = std::min(n, n_threads);
    for (int t = 0; t < T; ++t)
        th.emplace_back([&]() {
            for (int i = next++; i < n; i = next++) f(i);
        });
    for (auto& x : th) x.join();
}

}  // namespace

extern "C" double oracle_d2(const double* Si, const double* Sj, int64_t ni, int64_t nj, int32_t B) {
    if (B < 1 || B > 4096) return std::numeric_limits<double>::quiet_NaN();
    return criterion(Si, Sj, ni, nj, B);
}

extern "C" double oracle_sam(const double* Si, const double* Sj, int32_t B) {
    if (B < 1 || B > 4096) return std::numeric_limits<double>::quiet_NaN();
    return sam(Si, Sj, B);
}

extern "C" int oracle_rhseg(const float* cube, int32_t H, int32_t W, int32_t B, const oracle_params* p,
                            int32_t* labels, oracle_merge* log, int64_t* n_log, int32_t* out_R,
                            int32_t* out_label, int64_t* out_n, double* out_S) {
    if (!cube || !p || !labels || H < 1 || W < 1 || B < 1 || B > 4096) return -1;
    if ((int64_t)H * W >= (int64_t)1 << 31) return -1;
    if (p->connectivity != 4 && p->connectivity != 8) return -1;
    if (p->seam_connectivity != 4 && p->seam_connectivity != 8) return -1;
    if (!(p->spclust_wght >= 0.0f && p->spclust_wght <= 1.0f)) return -1;
    if (p->criterion != ORACLE_CRIT_BSMSE && p->criterion != ORACLE_CRIT_SAM) return -1;
    if (p->multi_merge && (p->two_merges || p->criterion != ORACLE_CRIT_BSMSE)) return -1;
    if (p->target_regions < 1 || p->rnb_levels < 1 || p->rnb_levels > 16) return -1;
    if ((H >> (p->rnb_levels - 1)) < 1 || (W >> (p->rnb_levels - 1)) < 1) return -1;
    if (p->n_levels < 1 || !p->level_counts) return -1;
    for (int l = 0; l < p->n_levels; ++l) {
        if (p->level_counts[l] < p->target_regions) return -1;
        if (l > 0 && p->level_counts[l] >= p->level_counts[l - 1]) return -1;
    }
    if (p->level_counts[p->n_levels - 1] != p->target_regions) return -1;

    const int L = p->rnb_levels;
    int stopS = p->section_regions;
    if (stopS <= 0) stopS = std::max(p->target_regions, p->spclust_max / 4);

    State st;
    st.H = H;
    st.W = W;
    st.B = B;
    const size_t P = (size_t)H * W;
    st.n.assign(P, 1);
    st.S.resize(P * B);
    for (size_t i = 0; i < P * B; ++i) st.S[i] = (double)cube[i];
    st.parent.resize(P);
    for (size_t i = 0; i < P; ++i) st.parent[i] = (int)i;
    st.adj.assign(P, {});
    if (!p->brute) st.best_adj.assign(P, KEY_NONE);

    Snapshot snap{labels, p->level_counts, p->n_levels};
    std::vector<std::vector<Rect>> levels;
    build_level_rects({0, 0, H, W}, L, levels);
    std::vector<oracle_merge> all_log;
    std::vector<int> top_live;
    int dr[4], dc[4];

    for (int d = L - 1; d >= 0; --d) {
        const std::vector<Rect>& secs = levels[d];
        const bool top = (d == 0);
        const int stop = top ? p->target_regions : stopS;
        std::vector<std::vector<oracle_merge>> logs(secs.size());
        std::vector<std::vector<int>> finals(secs.size());
        std::mutex progress_mu;
        int done = 0;
        parallel_for((int)secs.size(), p->n_threads, [&](int s) {
            const Rect& r = secs[s];
            std::vector<int> live;
            if (d == L - 1) {
                /* leaf: every pixel is a region (HSEG step 1) */
                const int nf = forward_offsets(p->connectivity, dr, dc);
                for (int row = r.r0; row < r.r0 + r.h; ++row)
                    for (int col = r.c0; col < r.c0 + r.w; ++col) {
                        const int a = row * W + col;
                        live.push_back(a);
                        for (int k = 0; k < nf; ++k) {
                            const int r2 = row + dr[k], c2 = col + dc[k];
                            if (r2 < r.r0 || r2 >= r.r0 + r.h || c2 < r.c0 || c2 >= r.c0 + r.w) continue;
                            const int b = r2 * W + c2;
                            st.adj[a][b] = 0.0;
                            st.adj[b][a] = 0.0;
                        }
                    }
            } else {
                /* reassembly (Figure 4.4): live regions of the four children,
                   plus links between neighbouring pixels across the split lines */
                for (int row = r.r0; row < r.r0 + r.h; ++row)
                    for (int col = r.c0; col < r.c0 + r.w; ++col) {
                        const int a = row * W + col;
                        if (st.parent[a] == a) live.push_back(a);
                    }
                const int nf = forward_offsets(p->seam_connectivity, dr, dc);
                for (int row = r.r0; row < r.r0 + r.h; ++row)
                    for (int col = r.c0; col < r.c0 + r.w; ++col) {
                        for (int k = 0; k < nf; ++k) {
                            const int r2 = row + dr[k], c2 = col + dc[k];
                            if (r2 < r.r0 || r2 >= r.r0 + r.h || c2 < r.c0 || c2 >= r.c0 + r.w) continue;
                            if (quadrant_of(r, row, col) == quadrant_of(r, r2, c2)) continue;
                            const int a = st.find(row * W + col), b = st.find(r2 * W + c2);
                            if (a == b) continue;
                            st.adj[a][b] = 0.0;
                            st.adj[b][a] = 0.0;
                        }
                    }
            }
            Pass pass(st, *p, std::move(live), stop, top, r, &snap);
            pass.run(logs[s]);
            if (p->progress) {
                std::lock_guard<std::mutex> lk(progress_mu);
                p->progress(d, ++done, (int32_t)secs.size());
            }
        });
        for (auto& lg : logs) all_log.insert(all_log.end(), lg.begin(), lg.end());
    }

    if (log)
        for (size_t i = 0; i < all_log.size(); ++i) log[i] = all_log[i];
    if (n_log) *n_log = (int64_t)all_log.size();
    if (out_R) {
        int R = 0;
        for (size_t a = 0; a < P; ++a)
            if (st.parent[a] == (int)a) {
                if (out_label) out_label[R] = (int32_t)a;
                if (out_n) out_n[R] = st.n[a];
                if (out_S) std::memcpy(out_S + (size_t)R * B, st.Sp((int)a), sizeof(double) * B);
                ++R;
            }
        *out_R = R;
    }
    return 0;
}
