"""Deterministic exp, log1p and tanh for the oracle (test infrastructure only).

The acceptance factor exp(-U_b/kT) of Eq. pon, the slip factor of Eq. slip,
the melting switch of Eq. gT and the FENE and tether bond energies decide
which bonds form and break.  The two sides compute them with one agreed
sequence of IEEE double operations (round to nearest, no fused multiply-add,
exact power-of-two scaling), so they produce the same bits by construction
instead of by two libms agreeing:

* exp:   Cody-Waite reduction (Cody & Waite, 1980) x = n ln2 + r, with
         n = nearest integer to x / ln2 (ties to even) and ln2 split into a
         head holding its leading 29 bits and the rounded remainder, so that
         n * head is exact; r = (x - n head) - n tail, |r| <= ln2 / 2; the
         Taylor series of e^r to degree 13 (terms 1/k!, each the double
         nearest to it) summed by Horner from the highest degree; times 2^n.
* log1p: 1 + z = m 2^e with m in [sqrt(1/2), sqrt(2)); s = (m - 1)/(m + 1),
         or s = z / (2 + z) when e = 0 so that a small z keeps its bits;
         log m = 2 s + 2 s (s^2 (1/3 + s^2 (1/5 + ... + s^2 / 23))) (the
         atanh series, |s| <= 0.1716); result e head + (log m + e tail).
* tanh:  1 - 2 / (exp(2 |x|) + 1) with the sign of x, 1 beyond |x| = 22
         (absolute error ~1e-16, what the switch (tanh + 1) / 2 needs).

The constants are derived below from the decimal expansion of ln 2.
"""

import math
from decimal import Decimal, getcontext
from fractions import Fraction


def _ln2_split():
    getcontext().prec = 50
    ln2 = Decimal(2).ln()
    m, e = math.frexp(float(ln2))                    # ln2 = m 2^e, m in [0.5, 1)
    head = math.ldexp(math.floor(math.ldexp(m, 29)), e - 29)   # leading 29 bits
    tail = float(Fraction(ln2) - Fraction(head))
    return head, tail, float(1 / ln2)


LN2_HI, LN2_LO, INV_LN2 = _ln2_split()
EXP_TERMS = [1.0 / math.factorial(k) for k in range(14)]        # 1/k!, k = 0..13
LOG_TERMS = [1.0 / (2 * k + 1) for k in range(12)]              # 1/(2k+1), k = 0..11
SQRT_HALF = math.sqrt(0.5)


def exp_det(x):
    x = float(x)
    if x != x:
        return x
    if not x > -745.5:
        return 0.0
    if x > 709.78:
        return math.inf
    n = float(round(x * INV_LN2))
    r = (x - n * LN2_HI) - n * LN2_LO
    p = EXP_TERMS[13]
    for k in range(12, -1, -1):
        p = p * r + EXP_TERMS[k]
    return math.ldexp(p, int(n))


def log1p_det(z):
    z = float(z)
    if z != z:
        return z
    if not z > -1.0:
        return -math.inf if z == -1.0 else math.nan
    y = 1.0 + z
    m, e = math.frexp(y)
    if m < SQRT_HALF:
        m = m * 2.0
        e -= 1
    if e == 0:
        s = z / (2.0 + z)
    else:
        f = m - 1.0
        s = f / (2.0 + f)
    s2 = s * s
    t = LOG_TERMS[11]
    for k in range(10, 0, -1):
        t = t * s2 + LOG_TERMS[k]
    lm = 2.0 * s + (2.0 * s) * (s2 * t)
    de = float(e)
    return de * LN2_HI + (lm + de * LN2_LO)


def tanh_det(x):
    x = float(x)
    if x != x:
        return x
    a = abs(x)
    t = 1.0
    if a < 22.0:
        t = 1.0 - 2.0 / (exp_det(2.0 * a) + 1.0)
    return -t if x < 0.0 else t
