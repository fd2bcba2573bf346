"""Writes accuracy_reference.json: the continuum reaction Z(Delta) of one
x-directed half-cosine MBF (0.3 x 0.02 lambda0) on the paper's substrate
(eps_r 2.2, h = 0.381 mm at 24.125 GHz, lossless; Sec. IV), at two
displacements on the diagonal (about 7 and 21.2 lambda0; Table I uses
21.2 lambda0), by the oracle's polar quadrature along a parabolic path that
rejoins the real axis past every pole and branch point (eqs. polarcord and
spectral_contour), radially up to 30 k0 (the substrate term has decayed by
e^{-2 beta h} ~ 1e-5 there) and again with a longer path and a finer angle
rule to bound the reference's own error.  Calls only oracle/.

The displacements are table nodes of any grid with k_max = 5 sqrt(eps_r) k0
(node step pi/k_max, Delta = 0 at index N/2): offsets 74 and 222 steps.
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ocont  # noqa: E402
from workloads import COSINE_X, basis_array  # noqa: E402

K0 = 2.0 * math.pi
EPS, TAN_D = 2.2, 0.0
H = 0.381 / (299.792458 / 24.125)
KM = 5.0 * math.sqrt(EPS) * K0
OFFSETS = [74, 222]


def main():
    basis = basis_array([(COSINE_X, 0.0, 0.0, 0.3, 0.02)])
    q = np.ones((1, 1), complex)
    step = math.pi / KM
    out = {"source": "oracle/ocont.reaction_polar (parabolic path, gamma 1/50, beta_end 2 sqrt(eps_r) k0)",
           "mbf": {"kind": "cosine_x", "a": 0.3, "b": 0.02}, "eps_r": EPS, "tan_delta": TAN_D, "h": H,
           "k0": K0, "k_max": KM, "points": []}
    for off in OFFSETS:
        d = off * step
        vals = []
        for bmax, nal in ((30.0, 1.6), (36.0, 2.0)):
            n_alpha = int(2 ** math.ceil(math.log2(nal * bmax * K0 * d * math.sqrt(2) + 64)))
            t0 = time.time()
            z = ocont.reaction_polar(d, d, 1.0 / 50.0, bmax * K0, K0, EPS, TAN_D, H, basis, q, n_alpha=n_alpha,
                                     beta_end=2.0 * math.sqrt(EPS) * K0, epsabs=0.0, epsrel=1e-9)
            print(f"offset {off}: beta_max {bmax} k0, {n_alpha} angles: {z} ({time.time() - t0:.1f} s)", flush=True)
            vals.append(z)
        out["points"].append({"offset": off, "dx": d, "dy": d, "re": vals[0].real, "im": vals[0].imag,
                              "rel_spread": abs(vals[1] - vals[0]) / abs(vals[0])})
    with open(os.path.join(HERE, "accuracy_reference.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
