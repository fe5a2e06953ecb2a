"""Soundness of the screens' certified bounds, emulated on the CPU.

The GPU screens never decide a merge; they only prune pairs that provably
cannot be the minimum. These tests redo the screens' arithmetic in numpy
(IEEE float32 per operation, float16 / bfloat16 rounding to nearest even) on
adversarial pairs and check, against the canonical FP64 value of Equation 1
from the oracle:
  * the FP32 screen's [lower, upper] always contains the exact value;
  * the 16-bit matrix-core tile test never discards a pair whose exact value
    is below the threshold T, whatever order the matrix core accumulates in.
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
