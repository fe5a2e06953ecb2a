"""CPU model of the spectral row cache with a second bound per row (no GPU).

Each live region i keeps its cached pair (K1: value and partner) and, from
its last full evaluation, K2: the least key over its other partners then.
After a merge (lo, hi -> lo), a row whose cached partner was lo or hi is
"light" if its K2 partner is still alive: its new cached pair is the lesser
of the pair with the survivor and K2 (then K2 is spent), with no full
evaluation. Other stale rows, and the survivor, are evaluated in full.

Why that is exact: K2 bounds every pair the row had at its evaluation except
its K1 partner. A pair created later, (i, s) with s a survivor, is bounded
by row s: s was evaluated in full when it was created, and a light step only
lowers a row's key to something at or below its own K2. So every live pair is
still bounded by the key cached in one of its rows, and the least cached key
is the least pair.

The model runs real merge sequences from the oracle (Equation 1, the
spectral angle, salt ties, and the two-merge reading's masked minimum) and
checks that invariant and the cached minimum against brute force after every
merge, and that the light path does the bulk of the work where it should."""
import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import synth

INF = float("inf")


def _bsmse(Si, Sj, ni, nj):
    d = Si / ni - Sj / nj
    return (ni * nj / (ni + nj)) * float(np.sum(d * d))


def _sam(Si, Sj, ni, nj):
    dot = float(Si @ Sj)
    den = float(Si @ Si) * float(Sj @ Sj)
    if den == 0.0:
        return 1.0
    t = dot * dot / den
    return max(0.0, 1.0 - t if dot >= 0 else 1.0 + t)


def _gkey(v, i, j):
    return (v, min(i, j), max(i, j))


class Model:
    """Row cache over region labels, with optional adjacency masking.

    keep_dead: a second bound of value 0 whose partner merged stays as a
    bare lower bound (its value and label); a stale row with such a bound
    takes the light step when its pair with the survivor is at or below the
    bound, and is evaluated in full otherwise (`fallback` counts those).
    Bounds above 0 are dropped: there the merged region's pair usually lies
    above the bound, and the light step would mostly fall back."""

    def __init__(self, S, n, labels, crit, adj=None, keep_dead=False):
        self.keep_dead = keep_dead
        self.dead = set()  # rows whose second bound's partner has merged
        self.fallback = 0
        self.S = {int(l): S[k].copy() for k, l in enumerate(labels)}
        self.n = {int(l): float(n[k]) for k, l in enumerate(labels)}
        self.crit = _sam if crit == "sam" else _bsmse
        self.adj = adj  # label -> set of labels, or None (no mask)
        self.K1 = {}
        self.K2 = {}
        self.full = set(self.S)
        self.light = set()
        self.surv = None
        self.n_full = 0
        self.n_light = 0

    def value(self, i, j):
        if self.adj is not None and j in self.adj[i]:
            return INF
        return self.crit(self.S[i], self.S[j], self.n[i], self.n[j])

    def evaluate(self):
        for i in self.full:
            row = sorted((self.value(i, j), j) for j in self.S if j != i)
            row = [r for r in row if r[0] < INF]
            self.K1[i] = row[0] if row else None
            self.K2[i] = row[1] if len(row) > 1 else None
            self.n_full += 1
        for i in sorted(self.light):
            c = (self.value(i, self.surv), self.surv)
            if c <= self.K2[i]:  # also for a bare bound: it stays a lower bound of the row's old pairs
                self.K1[i] = c if c[0] < INF else None
                self.n_light += 1
            elif i not in self.dead:
                self.K1[i], self.K2[i] = self.K2[i], None
                self.n_light += 1
            else:  # a bare bound below the new pair: look at the row in full
                row = sorted((self.value(i, j), j) for j in self.S if j != i)
                row = [r for r in row if r[0] < INF]
                self.K1[i] = row[0] if row else None
                self.K2[i] = row[1] if len(row) > 1 else None
                self.dead.discard(i)
                self.fallback += 1
        for i in self.full:
            self.dead.discard(i)
        self.full, self.light = set(), set()

    def minimum(self):
        ks = [_gkey(k[0], i, k[1]) for i, k in self.K1.items() if k is not None]
        return min(ks) if ks else None

    def check(self):
        """Every cached key is a live pair's exact key; every live pair is
        bounded below by the cached key of one of its rows. Returns the
        brute-force least pair."""
        best = None
        labs = sorted(self.S)
        for i in labs:
            k = self.K1.get(i)
            if k is not None:
                assert k[1] in self.S and k[0] == self.value(i, k[1]), f"row {i} holds a stale pair"
        for a, i in enumerate(labs):
            for j in labs[a + 1:]:
                v = self.value(i, j)
                if v == INF:
                    continue
                g = _gkey(v, i, j)
                bounds = [_gkey(self.K1[r][0], r, self.K1[r][1]) for r in (i, j) if self.K1.get(r) is not None]
                assert bounds and min(bounds) <= g, f"pair ({i},{j}) unwitnessed"
                best = g if best is None or g < best else best
        return best

    def merge(self, lo, hi):
        self.S[lo] = self.S[lo] + self.S.pop(hi)
        self.n[lo] += self.n.pop(hi)
        self.K1.pop(hi, None)
        self.K2.pop(hi, None)
        if self.adj is not None:
            nb = (self.adj[lo] | self.adj.pop(hi)) - {lo, hi}
            for x in self.adj:
                if hi in self.adj[x]:
                    self.adj[x].discard(hi)
                    if x != lo:
                        self.adj[x].add(lo)
            self.adj[lo] = nb
            for x in nb:
                self.adj[x].add(lo)
        self.full = {lo}
        self.light = set()
        self.K1[lo] = self.K2[lo] = None
        for i in self.S:
            if i == lo:
                continue
            if self.K2.get(i) is not None and self.K2[i][1] in (lo, hi) and i not in self.dead:
                if self.keep_dead and self.K2[i][0] == 0.0:
                    self.dead.add(i)  # a bare lower bound from now on (value and partner label kept)
                else:
                    self.K2[i] = None  # its partner changed: no longer a live pair's key
            k = self.K1.get(i)
            if k is not None and k[1] in (lo, hi):
                (self.light if self.K2.get(i) is not None else self.full).add(i)
                self.K1[i] = None
            # a row without any candidate (every other region adjacent) stays so: adjacency
            # only grows, and its new pair with the survivor is bounded by the survivor's row
        self.surv = lo


def _pixel_adjacency(H, W, conn):
    adj = {p: set() for p in range(H * W)}
    offs = [(0, 1), (1, 0)] + ([(1, 1), (1, -1)] if conn == 8 else [])
    for r in range(H):
        for c in range(W):
            for dr, dc in offs:
                r2, c2 = r + dr, c + dc
                if 0 <= r2 < H and 0 <= c2 < W:
                    a, b = r * W + c, r2 * W + c2
                    adj[a].add(b)
                    adj[b].add(a)
    return adj


def _replay(cube, crit, kmax, two_merges=False, w=0.5, conn=4, keep_dead=False):
    """Oracle merge sequence of one section; the model takes over at R = kmax."""
    H, W, B = cube.shape
    ref = oracle.rhseg(cube, connectivity=conn, spclust_wght=w, spclust_max=kmax, target_regions=2,
                       level_counts=[2], criterion=crit, two_merges=two_merges)
    S = cube.reshape(-1, B).astype(np.float64)
    n = np.ones(H * W)
    adj = _pixel_adjacency(H, W, conn) if two_merges else None
    # the region state at R = kmax, by replaying the merges before it
    regS = {p: S[p].copy() for p in range(H * W)}
    regn = {p: 1.0 for p in range(H * W)}
    k = 0
    while len(regS) > kmax:
        lo, hi = int(ref.log["lo"][k]), int(ref.log["hi"][k])
        regS[lo] = regS[lo] + regS.pop(hi)
        regn[lo] += regn.pop(hi)
        if adj is not None:
            nb = (adj[lo] | adj.pop(hi)) - {lo, hi}
            for x in adj:
                if hi in adj[x]:
                    adj[x].discard(hi)
                    if x != lo:
                        adj[x].add(lo)
            adj[lo] = nb
            for x in nb:
                adj[x].add(lo)
        k += 1
    labels = sorted(regS)
    m = Model(np.array([regS[l] for l in labels]), np.array([regn[l] for l in labels]), labels, crit, adj,
              keep_dead=keep_dead)
    return m, ref.log[k:]


CASES = [
    ("bsmse voronoi", lambda: synth.voronoi_scene(12, 12, 10, 8, 30.0, 19).cube, "bsmse", False),
    ("bsmse salt ties", lambda: synth.mixer_scene(12, 12, 8, 6, 25.0, 17, salt=0.3).cube, "bsmse", False),
    ("sam voronoi (one region grows)", lambda: synth.voronoi_scene(12, 12, 10, 8, 30.0, 23).cube, "sam", False),
    ("sam signed", lambda: synth.random_cube(11, 12, 4, seed=3), "sam", False),
    ("two-merge masked", lambda: synth.voronoi_scene(12, 12, 10, 8, 30.0, 29).cube, "bsmse", True),
    ("two-merge masked sam", lambda: synth.voronoi_scene(12, 12, 6, 8, 30.0, 31).cube, "sam", True),
]


@pytest.mark.parametrize("keep_dead", [False, True], ids=["bound_dropped", "bare_bound_kept"])
@pytest.mark.parametrize("name,make,crit,two", CASES, ids=[c[0] for c in CASES])
def test_second_bound_keeps_the_minimum(name, make, crit, two, keep_dead):
    cube = make()
    H, W, _ = cube.shape
    m, log = _replay(cube, crit, kmax=H * W // 2, two_merges=two, w=1.0 if two else 0.5, keep_dead=keep_dead)
    spectral = 0
    for rec in log:
        m.evaluate()
        got, want = m.minimum(), m.check()
        assert got == want, (name, got, want)
        if rec["kind"] == 1:  # a non-adjacent merge takes the least (masked) pair
            spectral += 1
            assert (got[1], got[2]) == (int(rec["lo"]), int(rec["hi"]))
        m.merge(int(rec["lo"]), int(rec["hi"]))
    assert m.n_light > 0
    if two:
        assert spectral > 0


def test_light_rows_carry_the_spectral_angle_pattern():
    """Under the spectral angle one region absorbs its neighbours one by one
    and is nearly every row's cached partner: the second bound turns those
    rows' re-evaluations into light steps."""
    cube = synth.voronoi_scene(16, 16, 12, 6, 30.0, 41).cube
    m, log = _replay(cube, "sam", kmax=128)
    m.evaluate()
    start = m.n_full  # the cache start evaluates every row
    for rec in log:
        m.merge(int(rec["lo"]), int(rec["hi"]))
        m.evaluate()
    full = m.n_full - start
    assert m.n_light > 1.2 * full, (m.n_light, full)


def test_bare_bounds_spare_full_evaluations_on_salt_ties():
    """Identical salt spectra tie at D2 = 0: a stale row's second bound often
    names a salt region that has merged too. Kept as a bare lower bound it
    still allows the light step whenever the pair with the survivor is at or
    below it."""
    cube = synth.mixer_scene(16, 16, 8, 6, 25.0, 17, salt=0.2).cube
    runs, fallback = {}, 0
    for keep in (False, True):
        m, log = _replay(cube, "bsmse", kmax=160, w=1.0, keep_dead=keep)
        m.evaluate()
        start = m.n_full
        for rec in log:
            m.merge(int(rec["lo"]), int(rec["hi"]))
            m.evaluate()
            assert m.minimum() == m.check()
        runs[keep] = (m.n_full - start + m.fallback, m.n_light)
        fallback = m.fallback
    assert runs[True][0] < 0.7 * runs[False][0], runs
    assert fallback < 0.1 * runs[True][1], (fallback, runs)  # zero bounds rarely fall back
