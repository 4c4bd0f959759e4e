"""Writes bcc250grad_oracle_gradient.json: the oracle's d sigma_xx / d delta_l of the 250-atom
bcc A0.5B0.5 gradient workload (LIZ 89 sites, eta 2 mRy) at 40 seeded (site, l) entries.

Calls only the oracle (oracle.adjoint: forward-mode differentiation of Eq. (3) through a dense
inverse per LIZ, propagated through Eq. (10) and Eq. (7)) and the seeded input generators; the
GPU gradient test compares the library's adjoint with these values.  Run from the repository
root:  python tests/golden/make_bcc250grad_oracle.py   (a few minutes on 8 cores).
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synthetic  # noqa: E402
from oracle import adjoint  # noqa: E402

OUT = os.path.join(HERE, "bcc250grad_oracle_gradient.json")


def main():
    w = synthetic.workload("bcc250grad")
    eta = w["etas"][0]
    rng = np.random.default_rng(synthetic.BASE_SEED + 55)
    sites = sorted(int(s) for s in rng.choice(len(w["pos"]), 10, replace=False))
    pairs = [(k, l) for k in sites for l in range(4)]
    dsig = np.array([1.0, 0.0, 0.0])
    t0 = time.time()
    g = adjoint.dsigma_dphase(w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], eta,
                              dsig, pairs=pairs)
    el = time.time() - t0
    vals = [float(g[k, l].real) for k, l in pairs]
    imag = max(abs(float(g[k, l].imag)) for k, l in pairs)
    rec = {"workload": "bcc250grad", "eta": eta, "dsigma": dsig.tolist(), "fingerprint": synthetic.fingerprint(w),
           "what": "d sigma_xx / d delta_l at (site, l), real part (imaginary parts vanish analytically; "
                   "largest here %.1e)" % imag,
           "pairs": pairs, "values": vals, "seconds": round(el, 1)}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT, "in %.1f s" % el)


if __name__ == "__main__":
    main()
