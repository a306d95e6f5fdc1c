"""Closed-form multiply-add counts of the compact RCCSDT triples contractions.

One multiply-add pair is one operation, as in the paper's operation-count
convention (Sec. "Tensor contractions for compact amplitudes").  For ntri =
o(o+1)(o+2)/6 stored triples and unit block size, the compact expansions
(RCCSDT operation count table; Sec. "RCCSDT contractions without/with
unpacking") evaluate per stored triple:

  pp ladder   3 terms x v^3 outputs x v^2         -> 3 ntri v^5
  rings       (3 + 3 + 6) terms x v^3 x (o v)     -> 12 ntri o v^4
  hole ladder 3 terms x v^3 x o^2                 -> 3 ntri o^2 v^3
  drivers     6 x v^3 x v  +  6 x v^3 x o          -> 6 ntri v^4 + 6 ntri o v^3
  Fock terms  3 x v^3 x v  +  3 x v^3 x o          -> 3 ntri v^4 + 3 ntri o v^3

In the large-o limit these reduce to the paper's 1/2 o^3 v^5 + 2 o^4 v^4 +
1/2 o^5 v^3 leading count.
"""


def ntri(o: int) -> int:
    return o * (o + 1) * (o + 2) // 6


def r3_macs(o: int, v: int) -> dict:
    t = ntri(o)
    return {
        "pp": 3 * t * v ** 5,
        "ring_a": 3 * t * o * v ** 4,
        "ring_b": 3 * t * o * v ** 4,
        "ring_c": 6 * t * o * v ** 4,
        "hh": 3 * t * o * o * v ** 3,
        "drv": 6 * t * v ** 4 + 6 * t * o * v ** 3,
        "fock": 3 * t * v ** 4 + 3 * t * o * v ** 3,
    }


def r3_macs_total(o: int, v: int) -> int:
    return sum(r3_macs(o, v).values())


def leading_asymptotic(o: int, v: int) -> float:
    """The paper's compact leading count 1/2 o^3 v^5 + 2 o^4 v^4 + 1/2 o^5 v^3."""
    return 0.5 * o ** 3 * v ** 5 + 2.0 * o ** 4 * v ** 4 + 0.5 * o ** 5 * v ** 3


def full_leading(o: int, v: int) -> float:
    """The paper's full-tensor leading count o^3 v^5 + 3 o^4 v^4 + o^5 v^3."""
    return float(o ** 3 * v ** 5 + 3 * o ** 4 * v ** 4 + o ** 5 * v ** 3)
