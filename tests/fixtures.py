"""Readers of the text fixtures under tests/golden/ (values printed in the
paper, each row citing where)."""
import os
from fractions import Fraction

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def paper_parameters() -> dict:
    """name -> exact value (Fraction) of every printed scheme parameter."""
    return {r[0]: Fraction(r[1]) for r in _rows("paper_parameters.txt")}


def shock_tubes() -> dict:
    """name -> dict(left=(rho, u, p), right=(rho, u, p), t_end, n) of the
    shock tubes of Sec. 4.2.1 (Eqs. sod, lax)."""
    out = {}
    for name, side, rho, u, p, t_end, n in _rows("shock_tubes.txt"):
        d = out.setdefault(name, {})
        d[side] = (float(rho), float(u), float(p))
        d["t_end"], d["n"] = float(t_end), int(n)
    return out


def table1() -> dict:
    """k -> the Table 1 coefficients of candidate k (Fractions), columns
    i-3 .. i+4 (Sec. 3.1)."""
    return {int(r[0]): [Fraction(p) for p in r[1:]] for r in _rows("table1_candidate_coefficients.txt")}
