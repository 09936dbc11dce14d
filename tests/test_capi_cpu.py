"""Host-side checks of the C ABI library (no GPU): it loads, and it exports
exactly the functions include/rbf.h declares; plus host logic of the kernels'
FP64 exponential (its constants, checked in exact arithmetic)."""
import math
import os
import re
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import paper_0909_5413_amd as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def built_lib():
    if not os.path.exists(R.LIB_PATH):
        from paper_0909_5413_amd import build
        build.build()
    return R.LIB_PATH


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rbf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rbf_setup", "rbf_setup_device", "rbf_solve", "rbf_evaluate", "rbf_destroy",
                 "rbf_status_string", "rbf_last_error"):
        assert must in names
    assert sorted(R.EXPORTED) == names


def test_library_exports_every_declared_symbol(built_lib):
    out = subprocess.run(["nm", "-D", "--defined-only", built_lib], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rbf_[a-z0-9_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_library_loads_without_gpu(built_lib):
    L = R.lib()
    assert L.rbf_status_string(R.RBF_ENOTPD).decode() == "RBF_ENOTPD"
    o = R.default_opts()
    assert o.restart == 30 and o.rtol == 1e-10 and o.precision == R.RBF_FP64


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _device_exp(x: float) -> float:
    """The kernels' exp_neg algorithm step by step, every fused multiply-add
    rounded exactly once (host emulation used to check its constants)."""
    src = open(os.path.join(ROOT, "paper_0909_5413_amd", "csrc", "rbf_device.hpp")).read()
    body = src[src.index("double exp_neg"):src.index("return __builtin_amdgcn_ldexp")]
    consts = dict(re.findall(r"const double (k\w+) = ([0-9a-fA-Fx.p+-]+);", body))
    log2e = float.fromhex(consts["kLog2e"])
    shift = float.fromhex(consts["kShift"])
    hi = float.fromhex(consts["kLn2Hi"])
    lo = float.fromhex(consts["kLn2Lo"])
    coefs = [float.fromhex(h) for h in re.findall(r"(0x[0-9a-f.]+p[+-]?\d+)\);?\s*// 1/", body)]
    first = float.fromhex(re.search(r"double p = ([0-9a-fx.p+-]+);", body).group(1))
    t = _fma(x, log2e, shift)
    nf = t - shift
    n = int(nf)
    r = _fma(nf, -hi, x)
    r = _fma(nf, -lo, r)
    p = first
    for c in coefs + [0.5, 1.0, 1.0]:
        p = _fma(p, r, c)
    return math.ldexp(p, n)


def test_device_exp_constants_accurate():
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-18.0, 0.0, 300), [-18.0, -1e-300, 0.0, -0.3465, -0.3467,
                                                        -math.log(2) * 5.5]])
    worst = 0.0
    for x in xs:
        got = _device_exp(float(x))
        ref = math.exp(float(x))
        worst = max(worst, abs(got - ref) / ref)
    assert worst < 5.2e-16, worst


def _device_exp_t32(x):
    """exp_neg_t32 step by step (fused multiply-adds rounded once, the table
    entries 2^(j/32) correctly rounded as the host builds them)."""
    src = open(os.path.join(ROOT, "paper_0909_5413_amd", "csrc", "rbf_device.hpp")).read()
    body = src[src.index("double exp_neg_t32"):]
    body = body[:body.index("return __builtin_amdgcn_ldexp")]
    consts = dict(re.findall(r"const double (k\w+) = ([0-9a-fA-Fx.p+-]+);", body))
    log2e32 = float.fromhex(consts["kLog2e32"])
    shift = float.fromhex(consts["kShift"])
    hi = float.fromhex(consts["kLn2Hi32"])
    lo = float.fromhex(consts["kLn2Lo32"])
    coefs = [float.fromhex(h) for h in re.findall(r"(0x[0-9a-f.]+p[+-]?\d+)\);?\s*// 1/", body)]
    first = float.fromhex(re.search(r"double p = ([0-9a-fx.p+-]+);", body).group(1))
    t = _fma(x, log2e32, shift)
    kf = t - shift
    k = int(kf)
    r = _fma(kf, -hi, x)
    r = _fma(kf, -lo, r)
    p = first
    for c in coefs + [0.5, 1.0, 1.0]:
        p = _fma(p, r, c)
    j, n = k & 31, k >> 5
    tj = _exp2_frac(j)
    return math.ldexp(tj * p, n)


def _exp2_frac(j):
    # 2^(j/32) to 60 significant digits, then rounded to a double
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    return float(Decimal(2) ** (Decimal(j) / Decimal(32)))


def test_device_exp_table_constants_accurate():
    """The table-driven exponential of the list matvec (its constants are the
    Cody-Waite split of ln2 scaled by 1/32, exact): within a few units of the
    last place of exp on the matvec's range and beyond."""
    rng = np.random.default_rng(4)
    xs = np.concatenate([rng.uniform(-18.0, 0.0, 400), rng.uniform(-600.0, -18.0, 50),
                         [-18.0, -1e-300, 0.0, -math.log(2) / 64, -math.log(2) * 5.5]])
    worst = 0.0
    for x in xs:
        got = _device_exp_t32(float(x))
        ref = math.exp(float(x))
        worst = max(worst, abs(got - ref) / ref)
    assert worst < 5e-16, worst


def _device_exp2_scaled(d2, beta):
    """exp2_scaled_t32 step by step: the fused products d2*beta are exact
    before their one rounding, the table entries 2^(j/32) correctly rounded."""
    src = open(os.path.join(ROOT, "paper_0909_5413_amd", "csrc", "rbf_device.hpp")).read()
    body = src[src.index("double exp2_scaled_t32"):]
    body = body[:body.index("return __builtin_amdgcn_ldexp")]
    shift = float.fromhex(re.search(r"const double kShift = ([0-9a-fx.p+-]+);", body).group(1))
    first = float.fromhex(re.search(r"double p = ([0-9a-fx.p+-]+);", body).group(1))
    coefs = [float.fromhex(h) for h in
             re.findall(r"__builtin_fma\(p, f, (0x[0-9a-f.]+p[+-]?\d+)\)", body)]
    assert len(coefs) == 4 and re.search(r"__builtin_fma\(p, f, 1\.0\)", body)
    t = _fma(d2, beta, shift)
    kf = t - shift
    k = int(kf)
    f = _fma(d2, beta, -kf)
    assert abs(f) <= 0.5
    p = first
    for c in coefs + [1.0]:
        p = _fma(p, f, c)
    j, n = k & 31, k >> 5
    return math.ldexp(_exp2_frac(j) * p, n)


def test_device_exp2_scaled_constants_accurate():
    """The list matvec's exponential, 2^(d2 beta / 32) with the reduction read
    from two fused products and a degree-5 polynomial: within a few units of
    the last place of the exact 2^(d2 beta / 32) (beta taken as exact), over
    the cutoff's range and beyond, including the tie points y = k + 1/2, where
    the reduced argument reaches the ends of the polynomial's interval.  The
    bar adds the polynomial's own error (1.41e-16, checked in rationals by
    gen_constants.py), u = 2^-53 for each of the last Horner step, the table
    entry and the final product, and a little for the earlier Horner steps:
    5.2e-16."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    rng = np.random.default_rng(5)
    sigma = 0.0025
    beta = -16.0 / (sigma * sigma * math.log(2.0))
    d2max = 36.0 * sigma * sigma
    d2s = list(rng.uniform(0.0, d2max, 400)) + list(rng.uniform(d2max, 30 * d2max, 50))
    d2s += [0.0, d2max, (0.5 / -beta), (31.5 / -beta)]
    worst = 0.0
    for d2 in d2s:
        got = _device_exp2_scaled(float(d2), beta)
        y = Decimal(Fraction(float(d2)).numerator) / Decimal(Fraction(float(d2)).denominator)
        y = y * Decimal(Fraction(beta).numerator) / Decimal(Fraction(beta).denominator)
        ref = float(Decimal(2) ** (y / 32))
        worst = max(worst, abs(got - ref) / ref)
    assert worst < 5.2e-16, worst
