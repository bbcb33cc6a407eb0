"""Writes critical_couplings.txt: the bond thresholds of the critical points
of the 2D q-state Potts model, from the closed form alone (exact decimal
arithmetic; neither the oracle nor the library is called).

In the delta normalisation the critical coupling is K_c = beta_c J =
ln(1 + sqrt q) (Sec. II.B.3 gives beta_c = ln(1 + sqrt 2) for q = 2; the same
self-dual point for every q), so p_c = 1 - exp(-K_c) = sqrt(q) / (1 + sqrt(q))
and T = floor(p_c 2^32).

Usage: python tests/golden/make_critical_couplings.py
"""
import os
from decimal import Decimal, getcontext

getcontext().prec = 60
HERE = os.path.dirname(os.path.abspath(__file__))


def threshold(q: int) -> int:
    s = Decimal(q).sqrt()
    return int((s / (1 + s) * Decimal(2) ** 32).to_integral_value(rounding="ROUND_FLOOR"))


def main() -> None:
    lines = [
        "# Critical bond thresholds of the 2D q-state Potts model (delta normalisation).",
        "# K_c = ln(1 + sqrt q): Sec. II.B.3 states beta_c = ln(1 + sqrt 2) for q = 2.",
        "# p_c = 1 - exp(-K_c) = sqrt(q) / (1 + sqrt(q)); T = floor(p_c * 2^32).",
        "# Written by make_critical_couplings.py from the closed form (exact decimals).",
        "# q  T",
    ]
    lines += [f"{q} {threshold(q)}" for q in (2, 3, 4, 8)]
    with open(os.path.join(HERE, "critical_couplings.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
