"""The extrapolation's normal matrix (Sec. 3.2, weights of Eq.
(3_2_extrap_weight)) summed in float is exact when every weight is the power
of two 2^-(|a|+|b|) (layers 3 and up) and the scan window's half-width is at
most 8: the HIP fit relies on this to sum those matrices in float and get the
bits of the double sums.  Checked here for every window size, on random valid
sets, in several summation orders, against exact rational sums."""
from fractions import Fraction

import numpy as np


def _terms(r, mask):
    out = []
    k = 0
    for b in range(-r, r + 1):
        for a in range(-r, r + 1):
            if mask[k]:
                w = Fraction(1, 2 ** (abs(a) + abs(b)))
                out.append((w * a * a, w * a * b, w * a, w * b * b, w * b, w))
            k += 1
    return out


def test_float_sums_of_power_of_two_weights_are_exact():
    rng = np.random.default_rng(0)
    for r in range(2, 9):
        n = (2 * r + 1) ** 2
        for trial in range(200):
            mask = rng.random(n) < rng.uniform(0.05, 1.0)
            mask[n // 2] = False  # the target itself is never a valid node
            terms = _terms(r, mask)
            if not terms:
                continue
            exact = [sum(t[c] for t in terms) for c in range(6)]
            for order in (terms, terms[::-1], list(rng.permutation(len(terms)))):
                seq = order if isinstance(order[0], tuple) else [terms[i] for i in order]
                acc32 = np.zeros(6, dtype=np.float32)
                acc64 = np.zeros(6, dtype=np.float64)
                for t in seq:
                    for c in range(6):
                        acc32[c] = np.float32(acc32[c] + np.float32(float(t[c])))
                        acc64[c] = acc64[c] + float(t[c])
                for c in range(6):
                    assert Fraction(float(acc32[c])) == exact[c], (r, c)
                    assert Fraction(float(acc64[c])) == exact[c], (r, c)
