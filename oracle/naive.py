"""An independent, deliberately different pure-Python evaluator for tiny
inputs, used only to pin the C oracle.  It shares no code with
``aerl_oracle.c``: conditions are decided with exact rational arithmetic
(``fractions.Fraction``) and an explicit round-to-nearest-even to float32, and
the decision list is resolved recursively.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def round_to_f32(q: Fraction) -> Fraction:
    """Round an exact rational to the nearest float32 (ties to even), with
    gradual underflow and overflow to infinity (returned as None for inf)."""
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)                 # below 2^-126 the spacing stays 2^-149
    ulp = Fraction(2) ** (e - 23)
    m = a / ulp
    lo = m.numerator // m.denominator
    rem = m - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    r = lo * ulp
    if r >= Fraction(2) ** 128 - Fraction(2) ** 103:  # rounds past the largest float32
        return None
    return sign * r


def _cmp(op, a, b):
    # None encodes an infinity; the sign is carried alongside
    return {0: a < b, 1: a <= b, 2: a > b, 3: a >= b}[op]


def _value(q, sign_if_inf):
    """Rational value, with +-inf mapped to large sentinels that keep order."""
    if q is None:
        return Fraction(sign_if_inf) * Fraction(2) ** 400
    return q


def product_f32(c, x) -> Fraction:
    exact = Fraction(float(c)) * Fraction(float(x))
    r = round_to_f32(exact)
    return _value(r, 1 if exact > 0 else -1)


def theta_value(t) -> Fraction:
    t = float(t)
    if np.isinf(t):
        return Fraction(2) ** 400 * (1 if t > 0 else -1)
    return Fraction(t)


def category_code(v):
    """The category code an exact float value names (0..63), else None."""
    q = Fraction(float(v)) if np.isfinite(v) else None
    if q is None or q.denominator != 1 or not 0 <= q <= 63:
        return None
    return int(q)


def condition(cond, row) -> bool:
    if cond["kind"] == 2:
        code = category_code(row[cond["f"]])
        return code is not None and (int(cond.get("mask", 0)) >> code) & 1 == 1
    lhs = product_f32(cond["coef"], row[cond["f"]])
    if cond["kind"] == 1:
        rhs = product_f32(cond["coef2"], row[cond["g"]])
    else:
        rhs = theta_value(cond["theta"])
    return _cmp(cond["op"], lhs, rhs)


def decide(rules, default, row) -> int:
    """Recursive decision list: the head rule decides if it fires, otherwise
    the rest of the list does; an empty list gives the default."""
    if not rules:
        return default
    cls, conds = rules[0]
    if all(condition(c, row) for c in conds):
        return cls
    return decide(rules[1:], default, row)


def evaluate(rule_set, x, y, n_classes):
    """(correct, confusion[true][pred]) of one rule set given as
    ``(default, [(class, [cond, ...]), ...])``."""
    default, rules = rule_set
    conf = np.zeros((n_classes, n_classes), np.int64)
    for row, label in zip(x, y):
        conf[int(label), decide(rules, default, row)] += 1
    return int(np.trace(conf)), conf
