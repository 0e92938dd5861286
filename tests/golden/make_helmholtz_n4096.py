"""Write the oracle's RSRR result for the Helmholtz sphere at n = 4096 (the headline
configuration: ellipse (3.8; 1.4, 0.3), N = 64 points, L = 64 probes, seed 2000,
SS-FULL with NQ = 500, KQ = 2, delta = 1e-14) to ``helmholtz_n4096_N64_L64.json``
and its eigenvectors inside the ellipse to ``helmholtz_n4096_N64_L64_V.npz``.

Calls only ``oracle/`` (and ``workloads`` for the seeded inputs).  About half an
hour on 8 CPU cores: 64 dense complex LU solves, an SVD of the 4096 x 4096 S,
and Q^H T(z) Q at each of the 500 SS-FULL nodes.
Usage: python tests/golden/make_helmholtz_n4096.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import rsrr_oracle as O  # noqa: E402

NAME = "helmholtz_n4096_N64_L64"


def main():
    t0 = time.time()
    nep, C, U = W.cfg_helmholtz(n=4096, N=64, L=64, seed=2000)
    prob = O.Problem(nep)
    r = O.rsrr(prob, C, U, delta=1e-14, NQ=500, KQ=2, tol_gap=1e3)
    lev = r["level"]
    inside = np.where(lev < 1.0)[0]
    sig = r["sigma_S"]
    k = int(r["k"])
    out = {
        "what": "oracle RSRR, Helmholtz single layer on the Fibonacci sphere",
        "n": 4096, "N": 64, "L": 64, "probe_seed": 2000,
        "contour": {"gamma": [C.gamma.real, C.gamma.imag], "a": C.a, "b": C.b},
        "NQ": 500, "KQ": 2, "delta": 1e-14, "tol_gap": 1e3,
        "k": k,
        "sigma_S_leading": sig[:k + 8].tolist(),
        "nbar": int(r["ss"]["nbar"]), "gmax": float(r["ss"]["gmax"]),
        "sigma_H_leading": r["ss"]["sigma_H"][:int(r["ss"]["nbar"]) + 4].tolist(),
        "lam_inside": [[complex(l).real, complex(l).imag] for l in r["lam"][inside]],
        "level_inside": lev[inside].tolist(),
        "resid_inside": r["res"][inside].tolist(),
        "seconds": None,
    }
    out["seconds"] = time.time() - t0
    with open(os.path.join(HERE, NAME + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    np.savez_compressed(os.path.join(HERE, NAME + "_V.npz"), V=r["V"][:, inside])
    print(f"k={k} nbar={out['nbar']} inside={inside.size} lam={r['lam'][inside]} "
          f"res={r['res'][inside]} ({out['seconds']:.0f} s)")


if __name__ == "__main__":
    main()
