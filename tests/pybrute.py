"""Independent pure-Python HSEG/RHSEG for tiny images (a third opinion).

Written separately from the C++ oracle and sharing nothing with it: each
iteration re-derives the regions, their band sums, their pixel counts and
their spatial adjacency from the current label map, instead of maintaining
them through merges. It follows the HSEG steps of Section 4.1 and
Equation 1 under the same readings as the oracle (one merge per iteration,
non-adjacent pair wins iff D2_na < w^2 D2_adj, lexicographic (D2, lo, hi)
tie-break, smaller label survives, RHSEG quadrant split at floor(h/2),
floor(w/2), reassembly links under the seam connectivity).

``exact=True`` evaluates Equation 1 in rational arithmetic (fractions), so
its decisions are the mathematically exact ones; otherwise the squared
criterion is evaluated in IEEE double in the canonical order (band sums,
then per-band means and squared differences, summed as a pairwise tree over
the band index zero-padded to a power of two, then the size factor).
``criterion="sam"`` ranks on the spectral angle instead, as 1 - sign(c) c^2
with c the cosine between the regions' band-sum vectors (rational when
exact; otherwise dot product and squared norms as pairwise trees).
``two_merges=True`` reads the step list with two merges per iteration: the
best adjacent pair, then the best non-adjacent pair of the resulting
partition if it is below w^2 times the first merge's value.
``multi_merge=True`` merges identical regions several at a time (the
future-work item of Section 6.2): when a step's one-merge winner has the
value 0, the step merges a greedy disjoint set of the zero-valued pairs, in
the order adjacent pairs by (lo, hi) then (spectral stage on at the step's
start) non-adjacent pairs by (lo, hi), one after another until the stop
count; its later merges are logged with kind + 2. Here the zero pairs are
found by re-deriving regions and adjacency before every merge of the step
and taking the least eligible zero pair whose regions the step has not
touched yet, rather than from one ranked list.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Sequence, Tuple


def _quadrants(r0, c0, h, w):
    h0, w0 = h // 2, w // 2
    return [(r0, c0, h0, w0), (r0, c0 + w0, h0, w - w0), (r0 + h0, c0, h - h0, w0),
            (r0 + h0, c0 + w0, h - h0, w - w0)]


def _leaf_map(H, W, L):
    """Leaf-section id of every pixel."""
    leaf = [[-1] * W for _ in range(H)]
    rects = [(0, 0, H, W)]
    for _ in range(L - 1):
        rects = [q for r in rects for q in _quadrants(*r)]
    for k, (r0, c0, h, w) in enumerate(rects):
        for r in range(r0, r0 + h):
            for c in range(c0, c0 + w):
                leaf[r][c] = k
    return leaf


def _tree(terms):
    """Pairwise tree over the band index, zero-padded to a power of two."""
    terms = list(terms)
    while len(terms) & (len(terms) - 1):
        terms.append(0.0)
    while len(terms) > 1:
        terms = [terms[2 * k] + terms[2 * k + 1] for k in range(len(terms) // 2)]
    return terms[0]


def _sam(xs_i, xs_j, exact):
    """Spectral angle ranked as 1 - sign(c) c^2, c the cosine of the angle
    between the regions' mean spectra (equal to that of their band sums)."""
    B = len(xs_i[0])
    Si = [sum(Fraction(x[b]) for x in xs_i) for b in range(B)]
    Sj = [sum(Fraction(x[b]) for x in xs_j) for b in range(B)]
    if exact:
        dot = sum(Si[b] * Sj[b] for b in range(B))
        den = sum(v * v for v in Si) * sum(v * v for v in Sj)
        if den == 0:
            return Fraction(1)
        t = dot * dot / den
        return max(Fraction(0), 1 - t if dot >= 0 else 1 + t)
    Si = [float(v) for v in Si]
    Sj = [float(v) for v in Sj]
    dot = _tree(Si[b] * Sj[b] for b in range(B))
    den = _tree(v * v for v in Si) * _tree(v * v for v in Sj)
    if den == 0.0:
        return 1.0
    t = (dot * dot) / den
    return max(0.0, 1.0 - t if dot >= 0.0 else 1.0 + t)


def _criterion(xs_i, xs_j, exact, crit="bsmse"):
    if crit == "sam":
        return _sam(xs_i, xs_j, exact)
    # Equation 1 squared, from the two regions' pixel vectors
    ni, nj = len(xs_i), len(xs_j)
    B = len(xs_i[0])
    if exact:
        Si = [sum(Fraction(x[b]) for x in xs_i) for b in range(B)]
        Sj = [sum(Fraction(x[b]) for x in xs_j) for b in range(B)]
        acc = sum((Si[b] / ni - Sj[b] / nj) ** 2 for b in range(B))
        return Fraction(ni * nj, ni + nj) * acc
    # band sums of quantised inputs are exact in double whatever the order
    Si = [float(sum(Fraction(x[b]) for x in xs_i)) for b in range(B)]
    Sj = [float(sum(Fraction(x[b]) for x in xs_j)) for b in range(B)]
    fac = (float(ni) * float(nj)) / float(ni + nj)
    terms = []
    for b in range(B):
        d = Si[b] / float(ni) - Sj[b] / float(nj)
        terms.append(d * d)
    # pairwise tree over the band index, zero-padded to a power of two
    while len(terms) & (len(terms) - 1):
        terms.append(0.0)
    while len(terms) > 1:
        terms = [terms[2 * k] + terms[2 * k + 1] for k in range(len(terms) // 2)]
    acc = terms[0]
    return fac * acc


def _hseg_pass(cube, lab, rect, leaf, conn, seam, w, kmax, stop, log, snaps, counts, top, crit, two=False,
               multi=False):
    r0, c0, h, wd = rect
    H = len(cube)
    W = len(cube[0])
    pix = [(r, c) for r in range(r0, r0 + h) for c in range(c0, c0 + wd)]
    w2 = float(w) * float(w)

    def regions():
        reg: Dict[int, List] = {}
        for (r, c) in pix:
            reg.setdefault(lab[r][c], []).append(cube[r][c])
        return reg

    def adjacency():
        adj = set()
        for (r, c) in pix:
            for dr, dc in ((0, 1), (1, 0), (1, 1), (1, -1)):
                r2, c2 = r + dr, c + dc
                if not (r0 <= r2 < r0 + h and c0 <= c2 < c0 + wd):
                    continue
                if dr != 0 and dc != 0:
                    need8 = conn if leaf[r][c] == leaf[r2][c2] else seam
                    if need8 != 8:
                        continue
                a, b = lab[r][c], lab[r2][c2]
                if a != b:
                    adj.add((min(a, b), max(a, b)))
        return adj

    def snap(R):
        for li, cnt in enumerate(counts):
            if cnt == R:
                snaps[li] = [row[:] for row in lab]

    reg = regions()
    R = len(reg)
    if top:
        for li, cnt in enumerate(counts):
            if cnt >= R:
                snaps[li] = [row[:] for row in lab]
    def best_pairs(spectral):
        reg = regions()
        adj = adjacency()
        labels = sorted(reg)
        A = None
        N = None
        for i_idx, i in enumerate(labels):
            for j in labels[i_idx + 1:]:
                isadj = (i, j) in adj
                if not isadj and not spectral:
                    continue
                key = (_criterion(reg[i], reg[j], log.exact, crit), i, j)
                if isadj:
                    A = key if A is None or key < A else A
                else:
                    N = key if N is None or key < N else N
        return A, N

    def apply(win, kind):
        _, lo, hi = win
        for (r, c) in pix:
            if lab[r][c] == hi:
                lab[r][c] = lo
        log.append((lo, hi, kind, len(regions()), win[0]))
        if top:
            snap(len(regions()))

    def below(N, A):
        return N[0] < (w2 * A[0] if not log.exact else Fraction(w) ** 2 * A[0])

    while two and R > stop:
        # step 2: the best adjacent pair; step 3 on the partition it leaves
        A, N = best_pairs(w > 0 and R <= kmax)
        if A is None:
            if N is None or not (w > 0 and R <= kmax):
                break
            apply(N, 1)
            R -= 1
            continue
        apply(A, 0)
        R -= 1
        if R <= stop or not (w > 0 and R <= kmax):
            continue
        _, N = best_pairs(True)
        if N is not None and below(N, A):
            apply(N, 1)
            R -= 1
    while multi and R > stop:
        spectral = w > 0 and R <= kmax
        A, N = best_pairs(spectral)
        if spectral and N is not None and (A is None or below(N, A)):
            win, kind = N, 1
        elif A is not None:
            win, kind = A, 0
        else:
            break
        if win[0] != 0:
            apply(win, kind)
            R -= 1
            continue
        # a step of several merges: each time the least zero-valued pair (adjacent ones first,
        # non-adjacent ones only with the spectral stage on at the step's start) whose two regions
        # no merge of this step has touched
        touched = set()
        first = True
        while R > stop:
            reg = regions()
            adj = adjacency()
            labels = sorted(l for l in reg if l not in touched)
            pick = None
            for want_adj in (True, False):
                if not want_adj and not spectral:
                    break
                for i_idx, i in enumerate(labels):
                    for j in labels[i_idx + 1:]:
                        if ((i, j) in adj) != want_adj:
                            continue
                        if _criterion(reg[i], reg[j], log.exact, crit) == 0:
                            pick = (0.0 if not log.exact else Fraction(0), i, j)
                            break
                    if pick is not None:
                        break
                if pick is not None:
                    k = 0 if want_adj else 1
                    break
            if pick is None:
                break
            apply(pick, k + (0 if first else 2))
            R -= 1
            first = False
            touched.update(pick[1:])
    while not two and not multi and R > stop:
        reg = regions()
        adj = adjacency()
        labels = sorted(reg)
        spectral = w > 0 and R <= kmax
        A = None
        N = None
        for i_idx, i in enumerate(labels):
            for j in labels[i_idx + 1:]:
                isadj = (i, j) in adj
                if not isadj and not spectral:
                    continue
                v = _criterion(reg[i], reg[j], log.exact, crit)
                key = (v, i, j)
                if isadj:
                    if A is None or key < A:
                        A = key
                else:
                    if N is None or key < N:
                        N = key
        if spectral and N is not None and (A is None or N[0] < (w2 * A[0] if not log.exact else Fraction(w) ** 2 * A[0])):
            win, kind = N, 1
        elif A is not None:
            win, kind = A, 0
        else:
            break
        _, lo, hi = win
        for (r, c) in pix:
            if lab[r][c] == hi:
                lab[r][c] = lo
        R -= 1
        log.append((lo, hi, kind, R, win[0]))
        if top:
            snap(R)


class _Log(list):
    exact = False


def rhseg(cube, *, connectivity=4, seam_connectivity=8, spclust_wght=0.0, spclust_max=0,
          target_regions=1, section_regions=0, rnb_levels=1, level_counts=None, exact=False, criterion="bsmse",
          two_merges=False, multi_merge=False, **_):
    """cube: nested lists or an array H x W x B. Returns (labels per level, log)."""
    cube = [[[float(v) for v in px] for px in row] for row in (cube.tolist() if hasattr(cube, "tolist") else cube)]
    H, W = len(cube), len(cube[0])
    counts = list(level_counts) if level_counts is not None else [target_regions]
    S = section_regions if section_regions > 0 else max(target_regions, spclust_max // 4)
    L = rnb_levels
    lab = [[r * W + c for c in range(W)] for r in range(H)]
    leaf = _leaf_map(H, W, L)
    levels = [[(0, 0, H, W)]]
    for _ in range(L - 1):
        levels.append([q for r in levels[-1] for q in _quadrants(*r)])
    log = _Log()
    log.exact = exact
    snaps = [None] * len(counts)
    for d in range(L - 1, -1, -1):
        top = d == 0
        for rect in levels[d]:
            _hseg_pass(cube, lab, rect, leaf, connectivity, seam_connectivity, spclust_wght,
                       spclust_max, target_regions if top else S, log, snaps, counts, top, criterion, two_merges,
                       multi_merge)
    return snaps, list(log)
