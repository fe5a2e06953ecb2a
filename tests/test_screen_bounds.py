"""Soundness of the screens' certified bounds, emulated on the CPU.

The GPU screens never decide a merge; they only prune pairs that provably
cannot be the minimum. These tests redo the screens' arithmetic in numpy
(IEEE float32 per operation, float16 / bfloat16 rounding to nearest even) on
adversarial pairs and check, against the canonical FP64 value of Equation 1
from the oracle:
  * the FP32 screen's [lower, upper] always contains the exact value;
  * the 16-bit matrix-core tile test never discards a pair whose exact value
    is below the threshold T, whatever order the matrix core accumulates in;
  * the interval matrix's bounds, kept by Ward's update over merge chains,
    contain the canonical values, and a row rescan thresholded at the row's
    second least upper bound finds the row's least two pairs.
"""
import numpy as np
import pytest

import oracle

U = np.float32(2.0 ** -24)
f32 = np.float32


def fma32(a, b, c):
    # a*b is exact in double for float32 inputs; one more rounding to float32
    return f32(np.float64(a) * np.float64(b) + np.float64(c))


def row_mean32(S, n):
    return (S / np.float64(n)).astype(np.float32)


def norm_up(m):
    return f32(np.sqrt(np.sum(m.astype(np.float64) ** 2)) * (1.0 + 2.0 ** -20))


def fp32_screen(Sa, na, Sb, nb, order):
    """FP32 screen of one pair: FMA accumulation over bands in `order`."""
    ma, mb = row_mean32(Sa, na), row_mean32(Sb, nb)
    acc = f32(0.0)
    for b in order:
        d = f32(ma[b] - mb[b])
        acc = fma32(d, d, acc)
    B = len(Sa)
    gam = f32(2 * B + 32) * U
    fa, fb = f32(na), f32(nb)
    w = f32(f32(fa * fb) / f32(fa + fb))
    r = f32(np.sqrt(acc))
    eta = f32(f32(3.0) * U) * f32(norm_up(ma) + norm_up(mb))
    rl = max(f32(f32(r * f32(1 - gam)) - eta), f32(0))
    rh = f32(f32(r * f32(1 + gam)) + eta)
    lower = f32(f32(f32(w * rl) * rl) * f32(1 - 32 * U))
    upper = f32(f32(f32(w * rh) * rh) * f32(1 + 32 * U))
    return lower, upper


def pair_cases(rng, n_cases):
    for k in range(n_cases):
        B = int(rng.choice([1, 3, 32, 128, 224, 1000, 4096]))
        kind = k % 5
        base = rng.uniform(0, 2000, size=B)
        if kind == 0:  # unrelated regions
            mu_a, mu_b = base, rng.uniform(0, 2000, size=B)
        elif kind == 1:  # nearly identical large means
            mu_a = base
            mu_b = base + rng.normal(0, 1e-3, size=B)
        elif kind == 2:  # identical
            mu_a = mu_b = base
        elif kind == 3:  # moderate differences
            mu_a = base
            mu_b = base + rng.normal(0, 5.0, size=B)
        else:  # one band differs
            mu_a = base
            mu_b = base.copy()
            mu_b[rng.integers(B)] += rng.uniform(1e-4, 10.0)
        na = int(rng.choice([1, 2, 7, 1000, 10 ** 6]))
        nb = int(rng.choice([1, 3, 64, 5000, 2 * 10 ** 6]))
        # band sums on the 2^-6 grid, as the quantised inputs produce
        Sa = np.round(mu_a * na * 64) / 64
        Sb = np.round(mu_b * nb * 64) / 64
        yield Sa, na, Sb, nb


def test_fp32_screen_brackets_the_canonical_value():
    rng = np.random.default_rng(2024)
    for Sa, na, Sb, nb in pair_cases(rng, 300):
        exact = oracle.criterion_d2(Sa, Sb, na, nb)
        B = len(Sa)
        for order in (np.arange(B), np.arange(B)[::-1], rng.permutation(B)):
            lo, up = fp32_screen(Sa, na, Sb, nb, order)
            assert lo <= exact <= up, (na, nb, B, lo, exact, up)


def bf16_round(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def f16_round(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


FMT = {"bf16": (bf16_round, 2.0 ** -8, 2.0 ** -133), "fp16": (f16_round, 2.0 ** -11, 2.0 ** -25)}


def row16(m, c, fmt):
    rnd, u16, sub = FMT[fmt]
    ac = (m - c).astype(np.float32)
    g = rnd(ac)
    sq = np.sum(g.astype(np.float64) ** 2)
    an = np.sum(ac.astype(np.float64) ** 2)
    mn = np.sum(m.astype(np.float64) ** 2)
    eta = ((u16 + 2.0 ** -23) * np.sqrt(an) + 1.0078125 * 2.0 ** -24 * np.sqrt(mn) + sub * np.sqrt(len(m)))
    return g, f32(sq), f32(eta * (1.0 + 2.0 ** -20))


def alpha_p(T, n, gn, geta, Bp):
    kappa = (2.0 * Bp + 64.0) * 2.0 ** -24
    a = (np.sqrt(T / n) + np.float64(geta)) * (1.0 + 2.0 ** -20)
    af = f32(a * (1.0 + 2.0 ** -22))
    P = (1.0 - kappa) * np.float64(gn) - np.float64(af) * np.float64(af) * (1.0 + 2.0 ** -20)
    return af, f32(P - abs(P) * 2.0 ** -21)


def dot32(ga, gb, order):
    acc = f32(0.0)
    for b in order:
        acc = f32(acc + f32(ga[b] * gb[b]))  # products of 16-bit values are exact in float32
    return acc


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_16bit_tile_test_never_drops_a_pair_below_threshold(fmt):
    rng = np.random.default_rng(7 if fmt == "bf16" else 8)
    checked = 0
    for Sa, na, Sb, nb in pair_cases(rng, 200):
        exact = oracle.criterion_d2(Sa, Sb, na, nb)
        B = len(Sa)
        Bp = (B + 31) // 32 * 32
        ma = np.zeros(Bp, np.float32)
        mb = np.zeros(Bp, np.float32)
        ma[:B], mb[:B] = row_mean32(Sa, na), row_mean32(Sb, nb)
        c = np.zeros(Bp, np.float32)
        c[:B] = ((ma[:B].astype(np.float64) + mb[:B].astype(np.float64)) / 2 +
                 rng.normal(0, 50, size=B)).astype(np.float32)
        ga, gna, ea = row16(ma, c, fmt)
        gb, gnb, eb = row16(mb, c, fmt)
        # thresholds just above the exact value: the pair must pass
        for T in (exact * (1 + 1e-12) + 1e-300, exact * 1.01 + 1e-6, exact * 4 + 1.0):
            aa, pa = alpha_p(T, na, gna, ea, Bp)
            ab, pb = alpha_p(T, nb, gnb, eb, Bp)
            for order in (np.arange(Bp), np.arange(Bp)[::-1], rng.permutation(Bp)):
                G = dot32(ga, gb, order)
                t = fma32(f32(-2.0) * aa, ab, f32(pa + pb))
                assert t < f32(2.0) * G or exact >= T, (fmt, na, nb, B, exact, T)
                checked += 1
    assert checked > 0


# ---------------------------------------------------------------------------
# Interval matrix of the row cache: exact entries widened and rounded outward,
# Ward's update on bounds at every merge
# ---------------------------------------------------------------------------
MAT_REL = 2.0 ** -40


def f32_down(x):
    f = np.float32(x)
    return np.nextafter(f, np.float32(-np.inf)) if np.float64(f) > x else f


def f32_up(x):
    f = np.float32(x)
    return np.nextafter(f, np.float32(np.inf)) if np.float64(f) < x else f


def mat_entry(c):
    """Model of the kernels' entry from a canonical value."""
    if not np.isfinite(c):
        return np.float32(np.inf), np.float32(np.inf)
    return f32_down(c * (1.0 - MAT_REL)), f32_up(c * (1.0 + MAT_REL))


def mat_update(ea, eb, d, na, nb, nk):
    """Model of the kernels' Ward update on bounds."""
    d_lo, d_hi = (float(v) for v in d)
    ca, cb, den = na + nk, nb + nk, na + nb + nk
    lo = (ca * float(ea[0]) + cb * float(eb[0]) - nk * d_hi) / den
    hi = (ca * float(ea[1]) + cb * float(eb[1]) - nk * d_lo) / den
    t = (ca * float(ea[1]) + cb * float(eb[1]) + nk * d_hi) / den
    return f32_down(max(lo - t * 2.0 ** -48, 0.0)), f32_up(hi + t * 2.0 ** -48)


@pytest.mark.parametrize("kind", ["voronoi", "salt", "tiny"])
def test_ward_update_bounds_hold_over_merge_chains(kind):
    """Merge random pairs of regions until few are left, updating every
    entry of the survivor's row by Ward's update on bounds (entries never
    refreshed from exact values, so the widening accumulates): the canonical
    value of every pair stays inside its widened bounds."""
    rng = np.random.default_rng({"voronoi": 1, "salt": 2, "tiny": 3}[kind])
    B = {"voronoi": 32, "salt": 224, "tiny": 3}[kind]
    R = 40
    base = rng.uniform(0, 2000, size=(4, B))
    cls = rng.integers(0, 4, size=R)
    mu = base[cls] + rng.normal(0, {"voronoi": 30.0, "salt": 5.0, "tiny": 1e-3}[kind], size=(R, B))
    if kind == "salt":
        mu[rng.random(R) < 0.3] = 2000.0  # identical spectra: exact zeros
    n = rng.integers(1, 20, size=R).astype(np.int64)
    S = np.round(mu * n[:, None] * 64) / 64
    live = list(range(R))
    E = {}
    for i in live:
        for j in live:
            if i < j:
                E[(i, j)] = mat_entry(oracle.criterion_d2(S[i], S[j], int(n[i]), int(n[j])))
    key = lambda a, b: (min(a, b), max(a, b))
    checked = 0
    while len(live) > 3:
        a, b = rng.choice(live, size=2, replace=False)
        a, b = int(min(a, b)), int(max(a, b))
        d = E[(a, b)]
        for k in live:
            if k in (a, b):
                continue
            E[key(k, a)] = mat_update(E[key(k, a)], E[key(k, b)], d, float(n[a]), float(n[b]), float(n[k]))
        S[a] = S[a] + S[b]
        n[a] += n[b]
        live.remove(b)
        for k in live:
            if k == a:
                continue
            c = oracle.criterion_d2(S[min(a, k)], S[max(a, k)], int(n[min(a, k)]), int(n[max(a, k)]))
            lo, hi = E[key(k, a)]
            assert float(lo) * (1 - MAT_REL) <= c <= float(hi) * (1 + MAT_REL), (kind, a, k, lo, c, hi)
            if c == 0.0:
                assert float(hi) == 0.0 or float(lo) == 0.0
            checked += 1
    assert checked > 100


def test_exact_zero_entries_stay_exact():
    """Identical spectra give [0, 0], and Ward's update of two [0, 0] rows
    with a zero-valued merge keeps [0, 0] (the rescan trusts it without
    evaluating)."""
    z = mat_entry(0.0)
    assert float(z[0]) == 0.0 and float(z[1]) == 0.0
    u = mat_update(z, z, z, 3.0, 5.0, 7.0)
    assert float(u[0]) == 0.0 and float(u[1]) == 0.0


def _rescan(E, S, n, live, i, lab):
    """Model of a row rescan: T is the row's second least upper bound (widened to
    the canonical value); only the pairs whose widened lower bound reaches T are
    evaluated (a pair bounded by [0, 0] is exactly 0); the row's least two by
    (D2, label) among them."""
    key = lambda a, b: (min(a, b), max(a, b))
    ups = sorted(float(E[key(i, j)][1]) * (1 + MAT_REL) for j in live if j != i)
    T = ups[1] if len(ups) > 1 else np.inf
    cands = []
    for j in live:
        if j == i:
            continue
        lo, hi = E[key(i, j)]
        if float(lo) * (1 - MAT_REL) <= T:
            if float(hi) == 0.0:
                v = 0.0
            else:
                a, b = key(i, j)
                v = oracle.criterion_d2(S[a], S[b], int(n[a]), int(n[b]))
            cands.append((v, lab[j]))
    return sorted(cands)[:2], len(cands)


@pytest.mark.parametrize("kind", ["voronoi", "salt"])
def test_rescan_keeps_each_rows_least_two(kind):
    """Over a merge chain whose matrix is kept by Ward's update on bounds only,
    every row's rescan (threshold at its second least upper bound) finds the
    row's least two pairs by (D2, label), ties and exact zeros included, and
    evaluates fewer pairs than the row holds."""
    rng = np.random.default_rng({"voronoi": 11, "salt": 12}[kind])
    B, R = 24, 36
    base = rng.uniform(0, 2000, size=(5, B))
    cls = rng.integers(0, 5, size=R)
    mu = base[cls] + rng.normal(0, 30.0, size=(R, B))
    if kind == "salt":
        mu[rng.random(R) < 0.3] = 2000.0
    n = rng.integers(1, 20, size=R).astype(np.int64)
    S = np.round(mu * n[:, None] * 64) / 64
    lab = rng.permutation(R)  # labels need not follow the slots
    live = list(range(R))
    key = lambda a, b: (min(a, b), max(a, b))
    E = {(i, j): mat_entry(oracle.criterion_d2(S[i], S[j], int(n[i]), int(n[j]))) for i in live for j in live
         if i < j}
    evaluated = held = 0
    while len(live) > 3:
        a, b = (int(v) for v in sorted(rng.choice(live, size=2, replace=False)))
        d = E[(a, b)]
        for k in live:
            if k not in (a, b):
                E[key(k, a)] = mat_update(E[key(k, a)], E[key(k, b)], d, float(n[a]), float(n[b]), float(n[k]))
        S[a] = S[a] + S[b]
        n[a] += n[b]
        live.remove(b)
        for i in live:
            got, nc = _rescan(E, S, n, live, i, lab)
            brute = sorted((oracle.criterion_d2(S[min(i, j)], S[max(i, j)], int(n[min(i, j)]), int(n[max(i, j)])),
                            lab[j]) for j in live if j != i)[:2]
            assert got == brute, (kind, len(live), i)
            evaluated += nc
            held += len(live) - 1
    assert evaluated < held
