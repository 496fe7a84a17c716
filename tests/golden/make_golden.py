"""Write the stored expected values under tests/golden/ (calls only the
CPU oracle and the textbook exact Riemann solver; nothing from the HIP path).

sod_l1.json: density L1 error of the oracle against the exact Riemann
solution of Sod's shock tube ((rho, v, p) = (1, 0, 1) | (0.125, 0, 0.1),
gamma = 1.4, t = 0.2, 256 cells on [0, 1]), frozen as a regression value.
The scheme is the paper's HLL + 'vanleer' + SSPRK(3,3) combination
(Tables tab:schemes_time, tab:schemes_space, t:limiters) in its pure-hydro
limit, B = 0.

shu_osher_ref.json: the density of Shu and Osher's shock / entropy-wave
test at t = 1.8 (the paper's 1D hydro WENO demonstration: x in [-4.5, 4.5],
HLL, SSPRK(3,3), zero-gradient ends, gamma = 1.4) computed by the oracle
with 'wenozp5' on 2048 cells and averaged onto the paper's low resolution of
256 cells (8 fine cells per coarse cell).  The pins measure each
reconstruction's 256-cell solution against it.
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


def shu_osher_reference(n_fine=2048, n_coarse=256):
    w = inputs.shu_osher(n_fine, limiter=6)
    sim = oracle.OracleSim(w)
    steps = sim.steps_to_time(1.8)
    g = inputs.blocks_to_global(sim.cons().swapaxes(0, 1), 2, w.nx, w.base_blocks)[0]
    assert np.array_equal(g, np.broadcast_to(g[0], g.shape))
    return g[0].reshape(n_coarse, n_fine // n_coarse).mean(axis=1), steps


if __name__ == "__main__":
    rho, steps = shu_osher_reference()
    out = {"rho_n256": [float(v) for v in rho], "n_fine": 2048, "n_coarse": 256, "steps_fine": steps,
           "t_end": 1.8, "gamma": 1.4, "scheme": "SSPRK(3,3) + wenozp5 + HLL, CFL 0.8, 3 ghost layers",
           "source": "the oracle at 8x the resolution, cell averages restricted onto 256 cells"}
    with open(os.path.join(HERE, "shu_osher_ref.json"), "w") as f:
        json.dump(out, f, indent=0)
    print({k: v for k, v in out.items() if k != "rho_n256"})
    l1, steps = sod_l1(256)
    out = {"l1_rho_n256": l1, "steps": steps, "t_end": 0.2, "gamma": 1.4,
           "scheme": "SSPRK(3,3) + vanleer + HLL, CFL 0.8",
           "source": "exact Riemann solution (Toro ch. 4) of Sod's problem"}
    with open(os.path.join(HERE, "sod_l1.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)
