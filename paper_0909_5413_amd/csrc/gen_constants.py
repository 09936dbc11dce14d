"""Derive the floating-point constants of the kernels' FP64 exp (exact arithmetic).

Run: python gen_constants.py  -- prints C hex-float literals for rbf_device.hpp,
and checks the degree-5 polynomial of exp2_scaled_t32 against exp in exact
rational arithmetic.
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
# exp_neg_t32: Taylor coefficients of exp(f ln2/32) in f, (ln2/32)^i / i!
for k in range(6, 0, -1):
    print(f"(ln2/32)^{k}/{k}! = {float((ln2 / 32) ** k / math.factorial(k)).hex()}")


# exp2_scaled_t32: the degree-5 polynomial interpolating exp(f ln2/32) at the
# six Chebyshev points of [-1/2, 1/2] (cos((2i+1) pi/12) / 2), solved exactly
def exp_frac(x, terms=40):
    s, t = Fraction(1), Fraction(1)
    for k in range(1, terms):
        t = t * x / k
        s += t
    return s


def arctan_inv(k):
    x = decimal.Decimal(1) / k
    x2, s, t, n, sign = x * x, x, x, 1, -1
    while True:
        t *= x2
        n += 2
        term = t / n
        if term == 0:
            return s
        s += sign * term
        sign = -sign


def dcos(x):
    s, t, k = decimal.Decimal(1), decimal.Decimal(1), 0
    while True:
        k += 2
        t = -t * x * x / (k * (k - 1))
        if abs(t) < decimal.Decimal(10) ** -75:
            return s
        s += t


PI = 16 * arctan_inv(5) - 4 * arctan_inv(239)
c = ln2 / 32
nodes = [dec_to_frac(dcos((2 * i + 1) * PI / 12)) / 2 for i in range(6)]
A = [[x ** j for j in range(6)] for x in nodes]
b = [exp_frac(c * x) for x in nodes]
for col in range(6):                      # Gauss-Jordan in rationals
    piv = max(range(col, 6), key=lambda r: abs(A[r][col]))
    A[col], A[piv], b[col], b[piv] = A[piv], A[col], b[piv], b[col]
    for r in range(6):
        if r != col and A[r][col] != 0:
            fct = A[r][col] / A[col][col]
            A[r] = [A[r][j] - fct * A[col][j] for j in range(6)]
            b[r] -= fct * b[col]
p5 = [float(b[i] / A[i][i]) for i in range(6)]
assert p5[0] == 1.0
for i in range(5, -1, -1):
    print(f"p5 c{i} = {p5[i].hex()}")
worst = Fraction(0)
for k in range(4001):                     # the rounded coefficients, exact evaluation
    f = Fraction(-1, 2) + Fraction(k, 4000)
    p = Fraction(0)
    for cc in reversed(p5):
        p = p * f + Fraction(cc)
    e = exp_frac(c * f)
    worst = max(worst, abs(p - e) / e)
print(f"p5 max relative error on [-1/2, 1/2]: {float(worst):.3e}")
assert worst < Fraction(15, 10 ** 17)
