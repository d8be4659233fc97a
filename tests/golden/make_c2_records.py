"""Write the FP64 oracle's records of the 2D matter-era run to
tests/golden/c2_oracle_records.json.

The run: 8192^2 periodic lattice, W0 = 10 (V0 = pi^2/(2 W0^2)), alpha = 3,
beta = 0, m = 2, dx = 1, deta = 0.25, eta 1 -> 4096 (16380 steps), initial
field uniform on (-1, 1) from seed 1 (the counter-based generator of
paper_1710_10420_amd/inputs.py), phi_dot = 0.  Diagnostics (Eqs. 7 and 8)
of every state n with n % 64 == 0 and of the final state; the scaling
exponents of Eq. (9) fitted over the last decade of the run
(eta >= 409.6) by the oracle's own least-squares fit.

Only the oracle and the input generator are called; nothing here touches the
HIP library.  Cost: about 1.1e12 FP64 site-updates, roughly half an hour on
eight host cores.

    python tests/golden/make_c2_records.py [--threads N]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1710_10420_amd.inputs import uniform_field  # noqa: E402

RUN = {"shape": [8192, 8192], "m": 2.0, "W0": 10.0, "alpha": 3.0, "beta": 0.0, "dx": 1.0,
       "deta": 0.25, "eta0": 1.0, "eta_end": 4096.0, "diag_every": 64, "seed": 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--out", default=os.path.join(HERE, "c2_oracle_records.json"))
    a = ap.parse_args()
    O.set_threads(a.threads)
    shape = tuple(RUN["shape"])
    S = int(round((RUN["eta_end"] - RUN["eta0"]) / RUN["deta"]))
    p = O.params(shape, deta=RUN["deta"], m=RUN["m"], W0=RUN["W0"], alpha=RUN["alpha"],
                 dx=RUN["dx"], eta0=RUN["eta0"], beta=RUN["beta"])
    phi = uniform_field(shape, RUN["seed"]).astype(np.float64).reshape(-1)
    pi = np.zeros_like(phi)
    K = RUN["diag_every"]
    recs = []
    t0 = time.time()
    chunk = 16 * K                              # progress line every 1024 steps
    n = 0
    while n < S:
        k = min(chunk, S - n)
        phi, pi, r = O.run(p, phi, pi, k, n0=n, diag_every=K)
        recs.extend(r)
        n += k
        print("step %d / %d, %.0f s" % (n, S, time.time() - t0), flush=True)
    recs.append(O.stats(p, phi, pi, S))
    mu, nu = O.scaling_exponents(recs, eta_min=RUN["eta_end"] / 10.0)
    out = {"what": "FP64 oracle records of the 2D matter-era run (see make_c2_records.py)",
           "run": RUN, "steps": S, "fit_eta_min": RUN["eta_end"] / 10.0,
           "mu": mu, "nu": nu, "records": recs}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print("mu %.6f nu %.6f, %d records, %.0f s" % (mu, nu, len(recs), time.time() - t0))


if __name__ == "__main__":
    main()
