"""Host check of the bound the residue planes rely on: for an exact integer
|acc| < 2^51 and a modulus after the first two (odd, p <= 253), the remainder acc - q p with
q = round-to-nearest(fl(acc * fl(1/p))) lies in [-(p+1)/2, (p+1)/2], so it
is already a signed byte without centring.  IEEE binary64 steps in numpy
(the product and the reciprocal each rounded once, as on the GPU); the
moduli come from the oracle."""
import numpy as np

from oracle import crt


def test_uncentred_remainder_fits_a_signed_byte():
    g = np.random.default_rng(11)
    mods = crt.moduli()
    assert mods[:2] == [256, 255]                 # these two are centred
    rest = mods[2:]
    assert all(p % 2 == 1 for p in rest) and max(rest) <= 253
    for p in rest:
        inv = 1.0 / p
        near_half = np.arange(-20000, 20000, dtype=np.int64) * p + (p - 1) // 2
        big = ((1 << 50) // p) * p + np.arange(-20000, 20000, dtype=np.int64) * p + (p + 1) // 2
        acc = np.concatenate([g.integers(-(1 << 51) + 1, 1 << 51, 200_000), near_half, big, -big])
        accd = acc.astype(np.float64)
        assert np.array_equal(accd.astype(np.int64), acc)          # exact integers
        q = np.rint(accd * inv)
        r = acc - q.astype(np.int64) * p
        assert np.all(np.abs(r) <= (p + 1) // 2), p
        assert np.all(np.abs(r) <= 127), p
        assert np.array_equal(np.mod(r, p), np.mod(acc, p))


def test_product_residue_reduction_in_32_bits():
    """The residue products reduce their INT32 sums (|v| < 2^31) modulo each
    modulus in 32-bit arithmetic: t = (v >> 16)(2^16 mod p) + (v & 0xffff)
    is below 2^24 (exact in FP32), the FP32 quotient t (1/p) floors to within
    one of t / p, and the smallest of r, r + p, r - p as unsigned numbers is
    v mod p.  Checked on the host with FP32 rounding for every modulus, the
    extremes of the INT32 range and random values."""
    import numpy as np
    mods = crt.moduli()
    assert min(mods) == 29 and max(mods) == 256
    g = np.random.default_rng(11)
    for p in mods:
        v = np.concatenate([g.integers(-2 ** 31, 2 ** 31, size=200_000, dtype=np.int64),
                            np.arange(-2 ** 31, -2 ** 31 + 5000), np.arange(2 ** 31 - 5000, 2 ** 31),
                            np.arange(-5000, 5000)]).astype(np.int32)
        t = (v >> 16).astype(np.int64) * (65536 % p) + (v & 0xffff).astype(np.int64)
        assert np.all(np.abs(t) < 2 ** 24)
        q = np.floor(t.astype(np.float32) * (np.float32(1.0) / np.float32(p))).astype(np.int64)
        r = t - q * p
        assert np.all((r >= -p) & (r < 2 * p)), p
        got = (np.stack([r, r + p, r - p]) & 0xffffffff).min(axis=0)
        assert np.array_equal(got, np.mod(v.astype(np.int64), p)), p


def _crt_words(n_mod, mods):
    """Words of the reconstruction for n_mod moduli: the bit length of
    n_mod 255 P in 32-bit words, at least 4 and even (the built sizes)."""
    P = 1
    for p in mods[:n_mod]:
        P *= p
    words = ((n_mod * 255 * P).bit_length() + 31) // 32
    return max(4, (words + 1) // 2 * 2), P


def test_reconstruction_quotient_estimate():
    """The reconstruction's quotient: X' (< N 255 P, in W 32-bit words) summed
    in doubles from the top word, times the rounded 1 / Pd (Pd: P's words
    summed the same way), scaled by 1 - 2^-45 and floored, is floor(X' / P)
    or one less, never more, so X' - q P lies in [0, 2P) and one
    conditional subtraction of P finishes the reduction.  Every moduli count,
    random X' and X' next to every multiple of P up to a few hundred,
    IEEE binary64 steps in Python floats (each add and product rounded once,
    in the kernel's order)."""
    import math
    import random
    mods = crt.moduli()
    rnd = random.Random(17)
    for n_mod in range(1, len(mods) + 1):
        W, P = _crt_words(n_mod, mods)
        if W > 12:
            continue
        pd = 0.0
        for w in range(12 - 1, -1, -1):
            pd += math.ldexp(float((P >> (32 * w)) & 0xFFFFFFFF), 32 * w)
        rp = 1.0 / pd
        top = n_mod * 255 * P
        xs = [0, top - 1] + [rnd.randrange(top) for _ in range(400)]
        for k in list(range(1, 300)) + [rnd.randrange(1, n_mod * 255) for _ in range(100)]:
            xs += [k * P - 1, k * P, k * P + 1]
        for x in xs:
            if not 0 <= x < top:
                continue
            xd = 0.0
            for w in range(W - 1, -1, -1):
                xd += math.ldexp(float((x >> (32 * w)) & 0xFFFFFFFF), 32 * w)
            q = math.floor(xd * rp * (1.0 - 2.0 ** -45))
            exact = x // P
            assert q in (exact - 1, exact), (n_mod, x)
            assert 0 <= x - q * P < 2 * P


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def test_image_words_by_one_truncation_each():
    """The residue planes cut an element's image into 40-bit words, one
    truncation per word (trunc(y 2^(8n)) of the remainder the words before
    it left, n = min(5, S - 5k) digits), a double-double's two parts on their
    own, and restore the truncation of hi + lo as one value from the two
    remainders (floor or ceil of their exact sum by the sign of the rounded
    sum).  The words, weighted 256^max(S - 5k - 5, 0), must give
    trunc((hi + lo) 2^(8S - 2 - e)) exactly: host steps in IEEE binary64
    (Python floats) against the exact value in rationals, for canonical pairs
    of both sign patterns, tiny trailing parts and every slice count."""
    import math
    import random
    from fractions import Fraction
    rnd = random.Random(23)
    cases = []
    for _ in range(3000):
        hi = rnd.uniform(-1.0, 1.0) * 2.0 ** rnd.randint(-30, 30)
        if hi == 0.0:
            continue
        ulp = math.ulp(hi)
        lo = rnd.choice([0.0, rnd.uniform(-0.5, 0.5) * ulp, rnd.uniform(-0.5, 0.5) * ulp * 2.0 ** -40])
        cases.append((hi, lo))
    # trailing parts of the opposite sign and leading parts with few bits
    for _ in range(1000):
        hi = rnd.randrange(1 << 10, 1 << 11) * 2.0 ** -11 * rnd.choice([-1.0, 1.0])
        lo = rnd.randrange(1, 1 << 30) * 2.0 ** -60 * rnd.choice([-1.0, 1.0])
        cases.append((hi, lo))
    for hi, lo in cases:
        # the row scale: |x| < 2^e from the leading part's exponent
        e = math.frexp(hi)[1]
        for S in range(1, 21):
            y, yl = math.ldexp(hi, -(e + 2)), math.ldexp(lo, -(e + 2))
            words = []
            for k in range(4):
                n = min(5, S - 5 * k)
                if n <= 0:
                    break
                sc = math.ldexp(1.0, 8 * n)
                a, al = y * sc, yl * sc
                t, tl = float(math.trunc(a)), float(math.trunc(al))
                y, yl = a - t, al - tl
                words.append(t + tl)
            f, g = _two_sum(y, yl)
            neg = hi + lo < 0.0
            t = float(math.ceil(f)) if neg else float(math.floor(f))
            if t == f:
                t += (1.0 if g > 0.0 else 0.0) if neg else (-1.0 if g < 0.0 else 0.0)
            words[-1] += t
            image = 0
            for k, wv in enumerate(words):
                assert wv == math.floor(wv) and abs(wv) < 2.0 ** 41 + 2
                image += int(wv) * 256 ** max(S - 5 * k - 5, 0)
            exact = (Fraction(hi) + Fraction(lo)) * Fraction(2) ** (8 * S - 2 - e)
            want = math.floor(exact) if exact >= 0 else -math.floor(-exact)
            assert image == want, (hi, lo, S)


def test_reconstruction_integer_steps():
    """The reconstruction's integer steps on the host: T_j in balanced
    radix-256 digits (4W positions), residues staged as u_j = r_j - 128, the
    digit sums X_b = sum_j u_j d_jb (below 2^20), their pairs as int32 half
    sums x0 + 2^8 x1 (below 2^29), and the signed carry pass over 16-bit
    steps with K0 = 128 sum_j T_j (carries below 2^14) give the W low words
    of X' = sum_j r_j T_j, which is below 2^(32W).  Python integers with the
    kernel's arithmetic shifts, several moduli counts, random residues and
    the extremes 0 and p - 1."""
    import random
    mods = crt.moduli()
    rnd = random.Random(5)
    for n_mod in (1, 4, 5, 16, 17, 39, 44, 49):
        W, P = _crt_words(n_mod, mods)
        ps = mods[:n_mod]
        T = [(P // p) * pow(P // p, -1, p) % P for p in ps]
        assert all(T[j] % ps[k] == (1 if j == k else 0) for j in range(n_mod) for k in range(n_mod))

        def balanced(t):
            ds = []
            for _ in range(4 * W):
                d = t % 256
                t //= 256
                if d >= 128:
                    d -= 256
                    t += 1
                ds.append(d)
            assert t == 0
            return ds

        D = [balanced(t) for t in T]
        K0 = 128 * sum(T)
        trials = [[0] * n_mod, [p - 1 for p in ps]] + [[rnd.randrange(p) for p in ps] for _ in range(150)]
        for r in trials:
            u = [x - 128 for x in r]
            X = [sum(u[j] * D[j][b] for j in range(n_mod)) for b in range(4 * W)]
            assert all(abs(x) < 2 ** 20 for x in X)
            carry, words = 0, []
            for w in range(W):
                h0 = X[4 * w] + (X[4 * w + 1] << 8)
                h1 = X[4 * w + 2] + (X[4 * w + 3] << 8)
                assert abs(h0) < 2 ** 29 and abs(h1) < 2 ** 29
                k0 = (K0 >> (32 * w)) & 0xFFFFFFFF
                s0 = h0 + (k0 & 0xFFFF) + carry
                carry = s0 >> 16
                assert abs(carry) < 2 ** 14
                s1 = h1 + (k0 >> 16) + carry
                carry = s1 >> 16
                assert abs(carry) < 2 ** 14
                words.append((s0 & 0xFFFF) | ((s1 & 0xFFFF) << 16))
            xp = sum(rj * tj for rj, tj in zip(r, T))
            assert xp < 2 ** (32 * W)
            assert words == [(xp >> (32 * w)) & 0xFFFFFFFF for w in range(W)], n_mod
            assert all(xp % p == rj for p, rj in zip(ps, r))


def test_reconstruction_magnitude_and_double_double():
    """The reconstruction's tail on the host: from X' (W words) the
    branch-free magnitude (quotient estimate, borrow chains, one conditional
    subtraction of P, centring at P/2) must give the centred value of X' mod
    P, and every word of its magnitude summed from the top by Fast2Sum then
    renormalised must be within 2^-104 of it, relative (the result's stated
    rounding).  Python integers for the words, Python floats (IEEE binary64)
    for the doubles, in the kernel's order."""
    import math
    import random
    from fractions import Fraction
    mods = crt.moduli()
    rnd = random.Random(29)
    worst = 0.0
    for n_mod in (4, 16, 39, 44, 49):
        W, P = _crt_words(n_mod, mods)
        pd = 0.0
        for w in range(11, -1, -1):
            pd += math.ldexp(float((P >> (32 * w)) & 0xFFFFFFFF), 32 * w)
        rp = 1.0 / pd
        half = P >> 1
        top = n_mod * 255 * P
        xs = [rnd.randrange(top) for _ in range(300)]
        # small values of either sign and values next to P/2
        for k in (rnd.randrange(1, 50) for _ in range(20)):
            for v in (rnd.randrange(1, 1 << 60), half - rnd.randrange(1, 1 << 40)):
                xs += [k * P + v, k * P + P - v]
        for x in xs:
            if not 0 <= x < top:
                continue
            xw = [(x >> (32 * w)) & 0xFFFFFFFF for w in range(W)]
            xd = 0.0
            for w in range(W - 1, -1, -1):
                xd += math.ldexp(float(xw[w]), 32 * w)
            q = math.floor(xd * rp * (1.0 - 2.0 ** -45))
            y = x - q * P                       # the borrow chain's result
            assert 0 <= y < 2 * P
            if y >= P:                          # no borrow in Y - P
                y -= P
            neg = y >= half                     # no borrow in Y - P/2
            mag = P - y if neg else y
            want = x % P
            if want > P // 2 or (want == half and P % 2 == 0):
                want -= P
            assert (-mag if neg else mag) == want
            scale = rnd.randint(-300, 300) - 32 * W
            hi = lo = 0.0
            for w in range(W - 1, -1, -1):
                v = math.ldexp(float((mag >> (32 * w)) & 0xFFFFFFFF), 32 * w + scale)
                s = hi + v
                lo += v - (s - hi)
                hi = s
            s = hi + lo                         # renormalise (TwoSum)
            bb = s - hi
            lo = (hi - (s - bb)) + (lo - bb)
            hi = s
            if mag:
                exact = Fraction(mag) * Fraction(2) ** scale
                err = abs(Fraction(hi) + Fraction(lo) - exact) / exact
                worst = max(worst, float(err) * 2.0 ** 104)
    print("worst double-double error / 2^-104:", worst)
    assert worst <= 1.0
