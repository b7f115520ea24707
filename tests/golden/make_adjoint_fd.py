"""Writes adjoint_channel_fd.json: the FP64 oracle's central-difference
gradient of the step-averaged objectives [J_Q, J_tau] of the configured
adjoint channel (20H x H, dp = H/80, 100 advection steps) with respect to
three of the inlet profile's sine coefficients, every event (time steps,
buffer decisions, slab membership) frozen to the oracle's own unperturbed
run.  Calls only the oracle (test infrastructure); the GPU test replays the
same oracle run's events and compares its adjoint gradient with these
values.

    python tests/golden/make_adjoint_fd.py [threads]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import cases  # noqa: E402
import oracle  # noqa: E402

STEPS = 100
COEFS = (0, 3, 9)
EPS = 1e-5
BID = 1


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    c = cases.make_adjoint_channel(steps=STEPS)
    t0 = time.time()
    J, log, _ = oracle.rollout(c, STEPS, c.objective, threads=threads)
    g, _ = oracle.fd_gradient(c, STEPS, c.objective, BID, eps=EPS, log=log, threads=threads,
                              coefs=COEFS)
    out = {"case": "make_adjoint_channel(steps=100): 20H x H, dp = H/80, Re 200, inlet "
                   "parabola + 16 sine coefficients (seed 4)",
           "particles": int(c.n), "steps": STEPS, "buffer": BID, "eps": EPS,
           "coefs": list(COEFS), "J_mean": [float(a) for a in J],
           "grad": {str(m): [float(g[m, 0]), float(g[m, 1])] for m in COEFS},
           "seconds": round(time.time() - t0, 1),
           "command": "python tests/golden/make_adjoint_fd.py"}
    with open(os.path.join(HERE, "adjoint_channel_fd.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
