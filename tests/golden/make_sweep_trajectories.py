"""Write the FP64 oracle's one-sweep trajectories that the full-size GPU
parity tests compare against (the oracle takes minutes per sweep at these
sizes, too long to run inside a GPU test).

Every value here comes from oracle/ (builder mode, Alg. 1) on inputs drawn by
qfinputs; nothing is taken from the GPU library.

  n12_brickwall8_sweep1.npz   n = 12 open-chain brick-wall of depth 8 (44 U(4)
                              gates), target from Haar gates on the same
                              structure, start 0: for each of the 88 updates
                              of one TwoSidedSweep the environment E, the new
                              gate and Tr of the circuit tensor after it; the
                              cost before and after the sweep.
  n10_brickwall10_s16_sweep1.npz
                              n = 10 brick-wall of depth 10 (45 gates), 16
                              starts: cost history and gates after one sweep
                              for starts 0, 7 and 15 (starts are independent,
                              so the oracle runs only those three).

Usage: python tests/golden/make_sweep_trajectories.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import qfinputs as I  # noqa: E402

N10_STARTS = (0, 7, 15)


def n12():
    pr = I.config5(n_starts=1)
    b = O.BuilderOracle(pr.target, pr.init_gates, pr.locs, pr.n)
    c0 = float(b.costs()[0])
    rec = []
    b.sweep(record=rec)
    E = np.stack([r[2][0] for r in rec])
    U = np.stack([r[3][0] for r in rec])
    T = np.array([r[4][0] for r in rec])
    order = np.array([(r[0], r[1]) for r in rec], np.int32)
    c1 = float(O.cost(pr.target, b.gates[0], pr.locs, pr.n))
    np.savez(os.path.join(HERE, "n12_brickwall8_sweep1.npz"), env=E, gate=U, trace=T, order=order,
             cost0=c0, cost1=c1, gates1=b.gates[0])


def n10():
    pr = I.config3(n_starts=16)
    init = pr.init_gates[list(N10_STARTS)]
    r = O.instantiate(pr.target, init, pr.locs, pr.n, tol=1e-300,
                      opt=O.Options(max_iter=1, diff_tol_r=0.0, long_diff_count=0))
    np.savez(os.path.join(HERE, "n10_brickwall10_s16_sweep1.npz"), starts=np.array(N10_STARTS, np.int32),
             history=r.history, costs=r.costs, gates=r.all_gates)


if __name__ == "__main__":
    n10()
    n12()
