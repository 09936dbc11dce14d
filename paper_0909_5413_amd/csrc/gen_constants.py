"""Derive the floating-point constants of the kernels' FP64 exp (exact arithmetic).

Run: python gen_constants.py  -- prints C hex-float literals for rbf_device.hpp.
"""
import decimal
import math
from fractions import Fraction

decimal.getcontext().prec = 80
LN2 = decimal.Decimal(2).ln()


def dec_to_frac(d):
    sign, digits, exp = d.as_tuple()
    n = int("".join(map(str, digits)))
    f = Fraction(n) * (Fraction(10) ** exp)
    return -f if sign else f


ln2 = dec_to_frac(LN2)
log2e = float(1 / ln2)
# head of ln2 with 32 significant bits: n * head is exact for |n| < 2^21
head = Fraction(round(ln2 * 2 ** 32), 2 ** 32)
tail = float(ln2 - head)
print(f"kLog2e = {log2e.hex()}")
print(f"kLn2Hi = {float(head).hex()}")
print(f"kLn2Lo = {tail.hex()}")
for k in range(12, 1, -1):
    print(f"1/{k}! = {float(Fraction(1, math.factorial(k))).hex()}")
# exp2_scaled_t32: Taylor coefficients of exp(f ln2/32) in f, (ln2/32)^i / i!
for k in range(6, 0, -1):
    print(f"(ln2/32)^{k}/{k}! = {float((ln2 / 32) ** k / math.factorial(k)).hex()}")
