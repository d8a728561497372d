"""The split searches' window, modelled on the CPU: for two adjacent sorted
runs X, Y whose positions divisible by S are sampled, the co-ranks of the
samples' merge at the two integers D0 = ceil((d - rX - rY) / S) and D0 + 1
confine the merge-path co-rank c of diagonal d (X elements among the first
d outputs of the stable merge, X first on equal keys) from X's side, and the
count of Y's samples before the split, D - (X's), confines it from Y's side.
Checked here against brute-force merges of small runs with repeated keys,
for several spacings and offsets; the window must hold c, be narrower than
2S, and be narrower than S whenever the next merged sample is X's and Y has
samples on both sides of the split.  (The kernels compute the same bounds;
the GPU parity tests check their co-ranks through the sorted outputs.)"""
import random


def corank(X, Y, d):
    i = j = 0
    for _ in range(d):
        if j >= len(Y) or (i < len(X) and X[i] <= Y[j]):
            i += 1
        else:
            j += 1
    return i


def first_true(l, h, pred):
    while l < h and not pred(l):
        l += 1
    return l


def window(S, xs, X, Y, d):
    """(l, h, tight) for diagonal d: the window [l, h] and whether the
    X-side bracket had k1 > k0 with both Y bounds available."""
    nx, ny = len(X), len(Y)
    ys, ye = xs + nx, xs + nx + ny
    at = {xs + t: X[t] for t in range(nx)}
    at.update({ys + t: Y[t] for t in range(ny)})
    ja, jc, je = -(-xs // S), -(-ys // S), -(-ye // S)
    KA, KC = jc - ja, je - jc
    rA, rC = ja * S - xs, jc * S - ys
    smp = lambda j: at[j * S]
    D0 = -((rA + rC - d) // S)  # ceil((d - rA - rC) / S)
    Dc = min(max(D0, 0), KA + KC)
    k0 = first_true(max(Dc - KC, 0), min(Dc, KA), lambda i: smp(ja + i) > smp(jc + Dc - 1 - i))
    if D0 < 0:
        k1 = 0
    elif D0 >= KA + KC:
        k1 = KA
    else:
        m0 = Dc - k0
        k1 = k0 + (1 if k0 < KA and (m0 >= KC or smp(ja + k0) <= smp(jc + m0)) else 0)
    l = 0 if k0 == 0 else rA + (k0 - 1) * S + 1
    h = nx if k1 >= KA else rA + k1 * S
    l, h = max(l, d - ny if d > ny else 0), min(h, d, nx)
    tight = False
    if 0 <= D0 < KA + KC:
        kyl = D0 - k0
        kyh = kyl if k1 > k0 else kyl + 1
        if kyh < KC:
            l = max(l, d - rC - kyh * S)
        if kyl >= 1:
            hi_c = d - rC - (kyl - 1) * S - 1
            if hi_c < h:
                h = max(hi_c, l)
        tight = k1 > k0 and kyl >= 1 and kyh < KC
    return l, h, tight


def test_window_holds_the_corank():
    rng = random.Random(7)
    cases = tight_cases = 0
    for _ in range(1500):
        S = rng.choice([2, 3, 4, 8, 16])
        xs = rng.randint(0, 3 * S)
        top = rng.choice([2, 9, 1000])
        X = sorted(rng.randint(0, top) for _ in range(rng.randint(1, 70)))
        Y = sorted(rng.randint(0, top) for _ in range(rng.randint(1, 70)))
        for d in range(len(X) + len(Y)):
            c = corank(X, Y, d)
            l, h, tight = window(S, xs, X, Y, d)
            assert l <= c <= h, (S, xs, d, l, h, c)
            assert h - l < 2 * S, (S, xs, d, l, h)
            if tight:
                assert h - l < S, (S, xs, d, l, h)
                tight_cases += 1
            assert first_true(l, h, lambda i: X[i] > Y[d - 1 - i]) == c
            cases += 1
    assert tight_cases > cases // 10  # the one-spacing case is common
