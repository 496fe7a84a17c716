"""The paper's companion tests on the GPU against the FP64 oracle: Shu and
Osher's shock / entropy-wave test with the fifth-order reconstructions (plain
path, 3 ghost layers) and with van Leer (fused path), and the
Kelvin-Helmholtz shear layer (HLLC, 'wenozp5') through adaptive regrid
cycles."""
import dataclasses

import numpy as np
import pytest

from paper_2303_03026_amd import inputs
from test_companion_pins import gradient_flags
from test_gpu_parity import assert_parity, rel_l1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


def check_within_floor(w, gpu, ref, pert, label):
    """Each variable within the larger of 1e-12 and ten times the oracle's
    own one-ulp floor (its result from the input raised by one ulp)."""
    floor = rel_l1(w, pert, ref)
    err = assert_parity(w, gpu, ref, tol=np.inf, label=label)
    print("one-ulp floor %s" % " ".join("%.1e" % f for f in floor), flush=True)
    assert np.all(err <= np.maximum(1e-12, 10.0 * floor)), (err, floor)


@pytest.mark.parametrize("lim,lname,path", [(6, "wenozp5", "plain"), (5, "mp5", "plain"), (0, "vanleer", "fused")])
def test_shu_osher(amr, orc, lim, lname, path):
    """200 steps (t ~ 0.8: the shock has crossed a third of the density
    wave) at the paper's 256 cells."""
    w = inputs.shu_osher(256, limiter=lim)
    print("GPU shu-osher %s path=%s" % (lname, path), flush=True)
    ref, _ = orc.run(w, nsteps=200)
    wp = inputs.shu_osher(256, limiter=lim)
    wp.prim = np.nextafter(wp.prim, np.inf)
    pert, _ = orc.run(wp, nsteps=200)
    sim = amr.Simulation(w, path=amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN)
    sim.advance(200, nstages=3)
    assert sim.sync_flags()[0] == 0
    gpu = sim.cons()
    sim.close()
    check_within_floor(w, gpu, ref, pert, "shu-osher %s %s" % (lname, path))


def test_kelvin_helmholtz_adaptive(amr, orc):
    """Three cycles of (2 steps, density-jump criterion on the oracle's
    ghost-filled state, plan, regrid) up to level 4, then 2 more steps; the
    same leaf sets drive the GPU run, the oracle and the oracle from the
    one-ulp-raised input."""
    w = inputs.kelvin_helmholtz(max_level=1)
    wp = inputs.kelvin_helmholtz(max_level=1)
    wp.prim = np.nextafter(wp.prim, np.inf)
    sim = amr.Simulation(w, path=amr.PATH_PLAIN)
    o, op = orc.OracleSim(w), orc.OracleSim(wp)
    for cycle in range(3):
        sim.advance(2, nstages=3)
        o.steps(2)
        op.steps(2)
        wc = dataclasses.replace(w, level=o.level, ijk=o.ijk)
        lv, ij = amr.regrid_plan(wc, gradient_flags(wc, o.padded()), max_level=4)
        print("GPU kelvin-helmholtz cycle %d blocks %d -> %d (max level %d)"
              % (cycle, len(o.level), len(lv), int(lv.max())), flush=True)
        new = sim.regrid(lv, ij)
        sim.close()
        sim = new
        o, op = o.regrid(lv, ij), op.regrid(lv, ij)
    sim.advance(2, nstages=3)
    o.steps(2)
    op.steps(2)
    assert sim.sync_flags()[0] == 0
    assert int(o.level.max()) >= 3
    wn = dataclasses.replace(w, level=o.level, ijk=o.ijk)
    check_within_floor(wn, sim.cons(), o.cons(), op.cons(), "kelvin-helmholtz adaptive")
    sim.close()
