"""Parity tolerances of the mixed-precision path (FP32 transforms).

The recombination of the Taylor terms (eq. fftarry) weights the transform of
term b by Delta^b / b! after a (gamma k)^b factor before it.  Across a table
of N samples per axis, |k| <= k_max and |Delta| <= (N/2) pi / k_max, so the
largest product of the two is (gamma N pi / 2)^b / b! whatever the spectral
span: the FP32 rounding of the transforms is amplified by up to

    A(N) = sum_{b <= P} (gamma N pi / 2)^b / b!

relative to the table's own scale (A = 66 at N = 512, 2.8e3 at 2048, 2.1e4 at
4096 for gamma = 1/130, P = 3).  The mixed path's 1e-5 target holds up to
the paper's transform length 2048; beyond it the tolerance grows with A.
"""
import math

MIXED_TARGET = 1e-5


def amplification(n: int, gamma: float = 1.0 / 130.0, order: int = 3) -> float:
    x = gamma * n * math.pi / 2.0
    return sum(x ** b / math.factorial(b) for b in range(order + 1))


def mixed_tolerance(n: int, gamma: float = 1.0 / 130.0, order: int = 3) -> float:
    """1e-5, scaled by A(n) / A(2048) for transforms longer than 2048 points."""
    return MIXED_TARGET * max(1.0, amplification(n, gamma, order) / amplification(2048, gamma, order))
