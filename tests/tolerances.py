"""Parity tolerances (max-normalised error against the FP64 oracle).

FP64 path: 1e-10.  Mixed path (FP32 storage of spectra, intermediates and
table): 1e-5 at every transform length.  The recombination of eq. fftarry
weights the transform of Taylor term b by Delta^b / b! after a
(gamma k)^b factor before it, so over a table of N samples per axis the
rounding of a transform can be amplified by up to
sum_b (gamma N pi / 2)^b / b! (2.9e3 at N = 2048, 2.1e4 at N = 4096 for
gamma = 1/130, P = 3).  FP32 transforms keep the error near 5e-7 up to
2048-point axes; beyond that the library runs the transforms of mixed grids
in FP64 on the FP32-stored data, which keeps the 1e-5 bar.
"""

FP64_TARGET = 1e-10
MIXED_TARGET = 1e-5


def amplification(n: int, gamma: float = 1.0 / 130.0, order: int = 3) -> float:
    """Largest recombination weight along one axis of n samples."""
    import math
    x = gamma * n * math.pi / 2.0
    return sum(x ** b / math.factorial(b) for b in range(order + 1))
