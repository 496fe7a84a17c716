"""Write the stored expected values under tests/golden/ (calls only the
CPU oracle and the textbook exact Riemann solver; nothing from the HIP path).

sod_l1.json: density L1 error of the oracle against the exact Riemann
solution of Sod's shock tube ((rho, v, p) = (1, 0, 1) | (0.125, 0, 0.1),
gamma = 1.4, t = 0.2, 256 cells on [0, 1]), frozen as a regression value.
The scheme is the paper's HLL + 'vanleer' + SSPRK(3,3) combination
(Tables tab:schemes_time, tab:schemes_space, t:limiters) in its pure-hydro
limit, B = 0.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import exact_riemann as er  # noqa: E402
from oracle import oracle  # noqa: E402
from paper_2303_03026_amd import inputs  # noqa: E402


def sod_l1(n):
    w = inputs.sod(n, ndim=2)
    sim = oracle.OracleSim(w)
    steps = sim.steps_to_time(0.2)
    u = sim.cons()
    g = inputs.blocks_to_global(u.swapaxes(0, 1), 2, w.nx, w.base_blocks)[0]
    ex = er.cell_average_density(n, 0.2, 0.5, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    return float(np.mean(np.abs(g[0] - ex))), steps


if __name__ == "__main__":
    l1, steps = sod_l1(256)
    out = {"l1_rho_n256": l1, "steps": steps, "t_end": 0.2, "gamma": 1.4,
           "scheme": "SSPRK(3,3) + vanleer + HLL, CFL 0.8",
           "source": "exact Riemann solution (Toro ch. 4) of Sod's problem"}
    with open(os.path.join(HERE, "sod_l1.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)
