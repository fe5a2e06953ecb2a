"""CPU emulation of the incremental form's edge index (no GPU).

The incremental form caches the exact D2 of every edge slot and keeps an
index over the edge list: per live slot a conservative range [rmin, rmax] of
the edge slots that can touch it, and per chunk of edge slots the least key
(D2, lo label, hi label) of its values together with that pair's slots. A
merge scans only the chunks of the merged pair's ranges and of the moving
slot's range, rewrites one edge per neighbour (the least edge slot) and
empties the others, moves the last slot into the freed one (renaming it in
its edges and in the chunk records that name it), re-scores the kept edges,
takes the minima of the chunks holding a rewritten edge anew, and reads the
next adjacent pair, slots included, off the least chunk record. A quarter of
the slots empty, the list is compacted in order and the index rebuilt.

The model below does those steps with the kernels' conventions and checks,
after every merge of a real sequence, that the scanned lists hold every edge
of the slots concerned, that every chunk record equals the least key of its
chunk with the right slots, and that the least record is the least live edge.
Driven by its own least record on an adjacent-only run, it must reproduce the
oracle's merge log (labels and FP64 values bit for bit); driven by the
oracle's log with spectral merges, the records must keep track through merges
of non-adjacent pairs.
"""
import numpy as np
import pytest

import oracle
from paper_2106_12942_amd import synth

class EdgeIndex:
    def __init__(self, cube, conn, ech):
        H, W, B = cube.shape
        self.S = cube.reshape(-1, B).astype(np.float64).copy()
        self.n = np.ones(H * W, dtype=np.int64)
        self.lab = np.arange(H * W)
        self.R = H * W
        self.ech = ech
        offs = [(0, 1), (1, 0)] + ([(1, 1), (1, -1)] if conn == 8 else [])
        self.edges = []  # pixel k owns slots k*nf .. k*nf+nf-1; a boundary slot is (-1, -1)
        for k in range(H * W):
            y, x = divmod(k, W)
            for dy, dx in offs:
                yy, xx = y + dy, x + dx
                self.edges.append((k, yy * W + xx) if 0 <= yy < H and 0 <= xx < W else (-1, -1))
        self.ed2 = [self.value(a, b) if a >= 0 else np.inf for a, b in self.edges]
        self.empty = 0
        self.valid = False

    def value(self, a, b):
        return oracle.criterion_d2(self.S[a], self.S[b], int(self.n[a]), int(self.n[b]))

    def key(self, e):
        a, b = self.edges[e]
        la, lb = self.lab[a], self.lab[b]
        return (self.ed2[e], la, lb, a, b) if la < lb else (self.ed2[e], lb, la, b, a)

    def chunk_min(self, c):
        best = None
        for e in range(c * self.ech, min(len(self.edges), (c + 1) * self.ech)):
            if self.edges[e][0] >= 0 and self.ed2[e] < np.inf:
                k = self.key(e)
                if best is None or k[:3] < best[:3]:
                    best = k
        return best

    def build(self):
        self.rmin = np.full(self.R, np.iinfo(np.int64).max)
        self.rmax = np.full(self.R, -1)
        for e, (a, b) in enumerate(self.edges):
            if a >= 0:
                for v in (a, b):
                    self.rmin[v] = min(self.rmin[v], e)
                    self.rmax[v] = max(self.rmax[v], e)
        self.rec = [self.chunk_min(c) for c in range(self.nchunks())]
        self.valid = True

    def nchunks(self):
        return (len(self.edges) + self.ech - 1) // self.ech

    def least(self):
        ks = [r for r in self.rec if r is not None]
        return min(ks, key=lambda r: r[:3]) if ks else None

    def merge(self, lo_s, hi_s):
        """Merge of slots lo_s (the lower label, the survivor's label) and hi_s."""
        if not self.valid:
            self.build()
        E, last, ech = len(self.edges), self.R - 1, self.ech
        moved = last not in (lo_s, hi_s)
        surv = hi_s if lo_s == last else lo_s
        # statistics: the survivor's sums and count in lo_s's slot
        self.S[lo_s] += self.S[hi_s]
        self.n[lo_s] += self.n[hi_s]
        # the scan: the chunks of the merged pair's ranges, then those of the moving slot's
        ua, ub = min(self.rmin[lo_s], self.rmin[hi_s]), max(self.rmax[lo_s], self.rmax[hi_s])
        ma, mb = (self.rmin[last], self.rmax[last]) if moved else (np.iinfo(np.int64).max, -1)
        a0, a1 = ((ua // ech) * ech, min(E, (ub // ech + 1) * ech)) if ua <= ub else (0, 0)
        b0, b1 = ((ma // ech) * ech, min(E, (mb // ech + 1) * ech)) if ma <= mb else (0, 0)
        L, XL, L2 = [], [], []
        for e in sorted(set(range(a0, a1)) | set(range(b0, b1))):
            a, b = self.edges[e]
            if a < 0:
                continue
            ta, tb = a in (lo_s, hi_s), b in (lo_s, hi_s)
            if ta or tb:
                L.append(e)
                XL.append(-1 if ta and tb else (b if ta else a))
            elif last in (a, b):
                L2.append(e)
        touch = [e for e, (a, b) in enumerate(self.edges) if a >= 0 and ({a, b} & {lo_s, hi_s})]
        assert sorted(L) == touch, "the range scan missed an edge of the merged pair"
        if moved:
            assert sorted(L2) == [e for e, (a, b) in enumerate(self.edges)
                                  if a >= 0 and last in (a, b) and not ({a, b} & {lo_s, hi_s})]
        # rename the moving slot in its edges and in the chunk records that name it
        for e in L2:
            a, b = self.edges[e]
            self.edges[e] = (hi_s if a == last else a, hi_s if b == last else b)
            r = self.rec[e // ech]
            if r is not None and last in (r[3], r[4]):
                self.rec[e // ech] = r[:3] + tuple(hi_s if v == last else v for v in r[3:])
        # one edge per neighbour survives: the least edge slot
        kept, emptied = [], 0
        for e, x in zip(L, XL):
            if x >= 0 and e == min(f for f, y in zip(L, XL) if y == x):
                self.edges[e] = (surv, hi_s if x == last else x)
                kept.append(e)
            else:
                self.edges[e] = (-1, -1)
                self.ed2[e] = np.inf
                emptied += 1
        # the last slot moves into the freed one (the survivor itself when it is the last)
        if hi_s != last:
            self.S[hi_s], self.n[hi_s], self.lab[hi_s] = self.S[last], self.n[last], self.lab[last]
        self.R -= 1
        self.S, self.n, self.lab = self.S[: self.R], self.n[: self.R], self.lab[: self.R]
        for e in kept:
            self.ed2[e] = self.value(*self.edges[e])
        # the chunks of rewritten edges taken anew, then the ranges
        for c in sorted({e // ech for e in L}):
            self.rec[c] = self.chunk_min(c)
        self.rmin[surv], self.rmax[surv] = ua, ub
        if moved:
            self.rmin[hi_s], self.rmax[hi_s] = ma, mb
        self.rmin, self.rmax = self.rmin[: self.R], self.rmax[: self.R]
        self.empty += emptied
        if 4 * self.empty > E:  # in-order compaction; the index is rebuilt when next used
            keep = [e for e in range(E) if self.edges[e][0] >= 0]
            self.edges = [self.edges[e] for e in keep]
            self.ed2 = [self.ed2[e] for e in keep]
            self.empty = 0
            self.valid = False
            self.build()
        return kept


def _check(ix):
    """Every record is its chunk's least key with the right slots; the least record is the least live edge."""
    for c in range(ix.nchunks()):
        assert ix.rec[c] == ix.chunk_min(c), f"chunk {c} record is stale"
    live = [ix.key(e) for e, (a, b) in enumerate(ix.edges) if a >= 0]
    want = min(live, key=lambda k: k[:3]) if live else None
    got = ix.least()
    assert got == want
    if got is not None:
        a, b = got[3], got[4]
        assert ix.lab[a] == got[1] and ix.lab[b] == got[2], "record slots do not hold its labels"
    return got


@pytest.mark.parametrize("ech", [4, 16])
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("salt", [0.0, 0.3])
def test_index_drives_the_adjacent_only_merge_sequence(ech, conn, salt):
    if salt:
        cube = synth.mixer_scene(9, 11, 6, 5, 25.0, 23, salt=salt).cube
    else:
        cube = synth.voronoi_scene(9, 11, 6, 7, 30.0, 29).cube
    ref = oracle.rhseg(cube, connectivity=conn, seam_connectivity=8, spclust_wght=0.0, spclust_max=0,
                       target_regions=1, section_regions=0, rnb_levels=1, level_counts=[1])
    ix = EdgeIndex(cube, conn, ech)
    ix.build()
    moves = 0
    for rec in ref.log:
        k = _check(ix)
        assert (k[1], k[2]) == (rec["lo"], rec["hi"])
        assert np.float64(k[0]).tobytes() == np.float64(rec["d2"]).tobytes()
        moves += int(ix.R - 1 not in (k[3], k[4]))
        ix.merge(k[3], k[4])
    assert ix.R == 1 and moves > 0


@pytest.mark.parametrize("ech", [4, 16])
def test_index_tracks_merges_of_non_adjacent_pairs(ech):
    cube = synth.voronoi_scene(10, 10, 8, 9, 30.0, 31).cube
    ref = oracle.rhseg(cube, connectivity=4, seam_connectivity=8, spclust_wght=0.8, spclust_max=100,
                       target_regions=2, section_regions=0, rnb_levels=1, level_counts=[2])
    assert (np.asarray(ref.log["kind"]) == 1).sum() > 20
    ix = EdgeIndex(cube, 4, ech)
    ix.build()
    for rec in ref.log:
        k = _check(ix)
        if rec["kind"] == 0:  # an adjacent merge is the least edge
            assert (k[1], k[2]) == (rec["lo"], rec["hi"])
        lo_s = int(np.nonzero(ix.lab == rec["lo"])[0][0])
        hi_s = int(np.nonzero(ix.lab == rec["hi"])[0][0])
        ix.merge(lo_s, hi_s)
    _check(ix)
