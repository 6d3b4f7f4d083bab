"""Writes config2_steady_state.npz: the oracle's steady state of the
90-species x 120-layer column (1200 reactions) from its initial state with
the adaptive driver at tol_rel 1e-4 (n_ss, steps, rejects, t), and the fixed
point reached from it by 40 backward-Euler steps of ten times the column's
mixing time, negatives clipped after each (n_fp, dt_fp): the relative
change of the last step is 5.6e-13.  Calls the oracle and the seeded input
generator only.  About five minutes on eight cores.

    python tests/golden/make_config2_steady_state.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import integrate  # noqa: E402


def main():
    net, col = synth.make_config(2)
    prob = integrate.Problem(net, col)
    r = integrate.steady_state(prob, col.n0, tol_rel=1e-4)
    print("steady state:", r.steps, "steps", r.rejects, "rejects, t =", r.t, flush=True)
    n = r.n.copy()
    dt = 10.0 * prob.grid.mix_time
    for i in range(40):
        n, d = integrate.be_step(prob, n, dt)
        n = np.where(n < 0, 0.0, n)
        keep = n > 1e-30 * prob.grid.ngas[:, None]
        print(i, float(np.max(np.abs(d[keep]) / n[keep])), flush=True)
    np.savez(os.path.join(HERE, "config2_steady_state.npz"), n_ss=r.n, steps=r.steps,
             rejects=r.rejects, t=r.t, n_fp=n, dt_fp=dt)


if __name__ == "__main__":
    main()
