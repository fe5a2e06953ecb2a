"""CPU model of the adjacency bitmap's update at a merge (two-merge
reading), against a rebuild from the edge set (no GPU).

Slots 0..R-1 hold the live regions. A merge of slots lo_s and hi_s keeps the
survivor in slot surv (lo_s, or hi_s when lo_s is the last slot) and moves
the last slot into hi_s (swap-remove). The update the kernels make, instead
of a rebuild:
  1. the survivor's row := row(lo_s) | row(hi_s), without the pair's own
     bits, and with the moved slot's bit renamed (last -> hi_s);
  2. every other live row y: bit(y, surv) := bit(y, lo_s) | bit(y, hi_s),
     the other of the pair's bits cleared, then bit(y, hi_s) := bit(y, last)
     when the last slot moves, and bit(y, last) cleared;
  3. the moved slot's row is copied into hi_s.
Steps 1 and 2 touch disjoint rows; step 3 follows them."""
import numpy as np
import pytest


def update(bits, R, lo_s, hi_s):
    """bits: R x R bool matrix (rows are slots); returns the (R-1) x (R-1) result."""
    last = R - 1
    surv = hi_s if lo_s == last else lo_s
    moves = hi_s != last and surv != hi_s  # region at `last` moves into hi_s
    b = bits.copy()
    # step 1: survivor row in place
    row = b[lo_s] | b[hi_s]
    row[lo_s] = row[hi_s] = False
    if moves:
        row[hi_s] = row[last]
        row[last] = False
    b[surv] = row
    # step 2: columns of every other live row
    for y in range(R):
        if y in (lo_s, hi_s):
            continue
        v = b[y, lo_s] | b[y, hi_s]
        if surv == lo_s:
            b[y, lo_s] = v
            b[y, hi_s] = b[y, last] if moves else False
        else:  # lo_s == last: the survivor sits in hi_s
            b[y, hi_s] = v
        b[y, last] = False  # the survivor is never in the last slot
    # step 3: the moved row
    if moves:
        b[hi_s] = b[last]
    return b[: R - 1, : R - 1]


def rebuild(adj, slot_of):
    R = len(slot_of)
    b = np.zeros((R, R), bool)
    for r1, nb in adj.items():
        for r2 in nb:
            b[slot_of[r1], slot_of[r2]] = True
    return b


@pytest.mark.parametrize("seed", range(20))
def test_update_equals_rebuild(seed):
    rng = np.random.default_rng(seed)
    R = int(rng.integers(2, 40))
    # random symmetric adjacency over region ids 0..R-1 (region i starts in slot i)
    adj = {i: set() for i in range(R)}
    for _ in range(int(rng.integers(R, 4 * R))):
        i, j = rng.integers(0, R, 2)
        if i != j:
            adj[int(i)].add(int(j))
            adj[int(j)].add(int(i))
    slots = list(range(R))  # slots[s] = region in slot s
    bits = rebuild(adj, {r: s for s, r in enumerate(slots)})
    while len(slots) > 1:
        Rn = len(slots)
        lo_s, hi_s = sorted(int(x) for x in rng.choice(Rn, 2, replace=False))
        if rng.random() < 0.5:
            lo_s, hi_s = hi_s, lo_s  # the surviving slot need not be the smaller one
        L, H = slots[lo_s], slots[hi_s]
        # region graph contraction: H merges into L
        nb = (adj[L] | adj.pop(H)) - {L, H}
        for x in adj:
            adj[x].discard(H)
            if x != L and x in nb:
                adj[x].add(L)
        adj[L] = nb
        # slots: swap-remove, the survivor keeps L's id
        last = Rn - 1
        surv = hi_s if lo_s == last else lo_s
        new = slots[:]
        new[surv] = L
        if hi_s != last and surv != hi_s:
            new[hi_s] = slots[last]
        slots = new[:last]
        bits = update(bits, Rn, lo_s, hi_s)
        want = rebuild(adj, {r: s for s, r in enumerate(slots)})
        assert np.array_equal(bits, want), (seed, Rn, lo_s, hi_s)
