"""The split constants of the kernel's elementary functions, recomputed.

pi comes from Machin's formula pi/4 = 4 atan(1/5) - atan(1/239) at 80 digits,
ln 2 from the decimal module; each constant must be the double nearest the
value, then the double nearest the remainder, and so on.  The host source that
fills the constant block is parsed so the test sees exactly what the library
uses.  The algorithms themselves are checked by the GPU parity tests.
"""
import os
import re
from decimal import Decimal, getcontext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _pi():
    getcontext().prec = 80

    def atan_inv(n):
        x = Decimal(1) / n
        x2 = x * x
        s = Decimal(0)
        t = x
        k = 1
        sign = 1
        while True:
            term = t / k
            if term < Decimal(10) ** -78:
                return s
            s += sign * term
            t *= x2
            k += 2
            sign = -sign

    return 4 * (4 * atan_inv(5) - atan_inv(239))


def _split(v, parts):
    out = []
    rem = v
    for _ in range(parts):
        h = float(rem)
        out.append(h)
        rem = rem - Decimal(h)
    return out


def _src_consts():
    src = open(os.path.join(ROOT, "paper_1312_4698_amd", "csrc", "api.hip")).read()
    return {k: float.fromhex(v) for k, v in re.findall(r"m\.(\w+) = (-?0x[0-9a-fA-Fp.+-]+);", src)}


def test_pi_digits():
    assert str(_pi()).startswith("3.14159265358979323846264338327950288419716939937510582097494459")


def test_split_constants_match_recomputation():
    c = _src_consts()
    pi = _pi()
    assert [c["pio2_1"], c["pio2_2"], c["pio2_3"]] == _split(pi / 2, 3)
    getcontext().prec = 80
    ln2 = Decimal(2).ln()
    assert [c["ln2_hi"], c["ln2_lo"]] == _split(ln2, 2)
    assert c["log2e"] == float(1 / ln2)
    assert c["two_over_pi"] == float(2 / pi)
    assert c["pi"] == float(pi) and c["pio2"] == float(pi / 2)
    assert c["pio4"] == float(pi / 4) and c["pio8"] == float(pi / 8)
