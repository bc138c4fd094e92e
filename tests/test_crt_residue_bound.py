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
