"""Print the Cody-Waite split of ln 2 and sqrt(2) used by the oracle's ln.

ln2_hi = ln 2 rounded to 32 significant bits; ln2_lo = (ln 2 - ln2_hi)
rounded to the nearest binary64; sqrt2 = sqrt(2) rounded to nearest.
Computed in 200-bit arithmetic with mpmath.  Test infrastructure only.
"""
import mpmath


def constants():
    mpmath.mp.prec = 200
    ln2 = mpmath.log(2)
    e = int(mpmath.floor(mpmath.log(ln2, 2)))
    scale = mpmath.mpf(2) ** (31 - e)
    hi = mpmath.nint(ln2 * scale) / scale
    lo = ln2 - hi
    return float(hi), float(lo), float(mpmath.sqrt(2))


if __name__ == "__main__":
    for name, v in zip(("ln2_hi", "ln2_lo", "sqrt2"), constants()):
        print(name, v.hex())
