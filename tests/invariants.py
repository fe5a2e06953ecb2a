"""Properties of a segmentation hierarchy that hold at any size.

Shared by the oracle pins and the GPU parity tests; they read only label
maps, cubes and merge logs, never either implementation's internals.
"""
import numpy as np


def canonical_labels(lab):
    """Relabel so that every region carries its smallest row-major pixel index."""
    flat = lab.ravel()
    idx = np.arange(flat.size)
    uniq, inv = np.unique(flat, return_inverse=True)
    mins = np.full(uniq.size, flat.size, dtype=np.int64)
    np.minimum.at(mins, inv, idx)
    return mins[inv].reshape(lab.shape).astype(np.int32)


transform_labels = canonical_labels


def check_partition_levels(labels, counts):
    """Every level is a partition with canonical labels, the requested number of
    regions (or the top pass's starting count, for counts at or above it), and
    each level is a union of regions of the previous, finer, level."""
    labels = np.asarray(labels)
    start = len(np.unique(labels[0]))
    for li, c in enumerate(counts):
        lab = labels[li]
        assert lab.min() >= 0
        assert np.array_equal(canonical_labels(lab), lab), f"level {li}: labels not canonical"
        nd = len(np.unique(lab))
        assert nd == c or (nd < c and nd == start), f"level {li}: {nd} regions, want {c}"
        if li > 0:
            fine, coarse = labels[li - 1].ravel(), lab.ravel()
            u, inv = np.unique(fine, return_inverse=True)
            first = np.full(u.size, -1, dtype=np.int64)
            first[inv[::-1]] = coarse[::-1]
            assert np.array_equal(first[inv], coarse), f"level {li} does not nest level {li - 1}"


def sse_of_partition(cube, lab):
    """Sum over pixels of the squared distance to their region's mean spectrum."""
    X = cube.reshape(-1, cube.shape[-1]).astype(np.float64)
    u, inv = np.unique(lab.ravel(), return_inverse=True)
    n = np.bincount(inv).astype(np.float64)
    S = np.zeros((u.size, X.shape[1]))
    np.add.at(S, inv, X)
    mu = S / n[:, None]
    return float(((X - mu[inv]) ** 2).sum())


def leaf_map(H, W, L):
    leaf = np.zeros((H, W), dtype=np.int64)
    rects = [(0, 0, H, W)]
    for _ in range(L - 1):
        nxt = []
        for (r0, c0, h, w) in rects:
            h0, w0 = h // 2, w // 2
            nxt += [(r0, c0, h0, w0), (r0, c0 + w0, h0, w - w0), (r0 + h0, c0, h - h0, w0),
                    (r0 + h0, c0 + w0, h - h0, w - w0)]
        rects = nxt
    for k, (r0, c0, h, w) in enumerate(rects):
        leaf[r0:r0 + h, c0:c0 + w] = k
    return leaf


def adjacency_linked(lab, a, b, L, conn, seam):
    """True iff some neighbouring pixel pair joins region a and region b.
    Orthogonal neighbours are always linked; diagonal neighbours are linked
    under 8-connectivity: `conn` inside a leaf section, `seam` across a split."""
    H, W = lab.shape
    leaf = leaf_map(H, W, L)
    for dr, dc in ((0, 1), (1, 0), (1, 1), (1, -1)):
        r1 = slice(0, H - dr)
        r2 = slice(dr, H)
        c1 = slice(max(0, -dc), W - max(0, dc))
        c2 = slice(max(0, dc), W - max(0, -dc) if dc < 0 else W)
        if dc < 0:
            c1, c2 = slice(1, W), slice(0, W - 1)
        A, Bm = lab[r1, c1], lab[r2, c2]
        hit = ((A == a) & (Bm == b)) | ((A == b) & (Bm == a))
        if not hit.any():
            continue
        if dr == 0 or dc == 0:
            return True
        same = leaf[r1, c1] == leaf[r2, c2]
        ok = np.where(same, conn == 8, seam == 8)
        if (hit & ok).any():
            return True
    return False
