"""Write adjoint_fd_16.npz: the oracle's central finite-difference gradient of
the oscillating-drop loss on a 16 x 16 periodic grid over 10 steps.

Loss L = 1/2 h^2 sum (phi^N - phi_target)^2 with phi_target the oracle state
after N steps at sigma = 1.0, M = 1e-3 from the same initial ellipse, and the
gradient taken at sigma = 1.1, M = 1.2e-3 (We = 1/sigma, Pe = 1/(M sigma)).
Entries: every one of the 256 initial phi cells (absolute step 1e-6) and
sigma, M (relative step 1e-6).  Calls only the oracle and the input
generator; the stored values are the oracle's.

Usage:  python tests/golden/make_adjoint_fd.py   (about a minute on one core)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import MACGrid, Params, step as ostep  # noqa: E402

N_CELLS = 16
STEPS = 10
SIGMA0, MOB0 = 1.0, 1e-3
SIGMA, MOB = 1.1, 1.2e-3
EPS = 1e-6
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fd_16.npz")


def final_phi(prob, phi0, sigma, mob):
    pr = prob.props.copy(We=1.0 / sigma, Pe=1.0 / (mob * sigma))
    g = MACGrid(prob.n, prob.h, prob.periodic)
    prm = Params.from_props(pr)
    st = {"phi": phi0.copy(), "u": [np.zeros(prob.shape) for _ in range(prob.dim)], "p": np.zeros(prob.shape)}
    for _ in range(STEPS):
        st = ostep(g, st, prm)
    return st["phi"]


def main():
    prob = W.adjoint_drop(N_CELLS, steps=STEPS)
    phi0 = W.initial_state(prob)["phi"]
    target = final_phi(prob, phi0, SIGMA0, MOB0)
    h2 = prob.h ** 2

    def loss(phi_init, sigma, mob):
        d = final_phi(prob, phi_init, sigma, mob) - target
        return 0.5 * h2 * float(np.sum(d * d))

    t0 = time.time()
    L0 = loss(phi0, SIGMA, MOB)
    es, em = EPS * SIGMA, EPS * MOB
    dsig = (loss(phi0, SIGMA + es, MOB) - loss(phi0, SIGMA - es, MOB)) / (2 * es)
    dmob = (loss(phi0, SIGMA, MOB + em) - loss(phi0, SIGMA, MOB - em)) / (2 * em)
    gphi = np.zeros(prob.shape)
    for idx in np.ndindex(prob.shape):
        pp = phi0.copy()
        pp[idx] += EPS
        lp = loss(pp, SIGMA, MOB)
        pp[idx] -= 2 * EPS
        lm = loss(pp, SIGMA, MOB)
        gphi[idx] = (lp - lm) / (2 * EPS)
    np.savez(OUT, phi0=phi0, target=target, loss=L0, dsigma=dsig, dmob=dmob, gphi=gphi,
             sigma=SIGMA, mob=MOB, steps=STEPS, eps=EPS)
    print(f"wrote {OUT}: L={L0:.6e} dL/dsigma={dsig:.6e} dL/dM={dmob:.6e} "
          f"max|dL/dphi0|={np.abs(gphi).max():.3e} ({time.time() - t0:.1f} s)")


if __name__ == "__main__":
    main()
