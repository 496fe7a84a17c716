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
from test_gpu_parity import assert_parity
import parity

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


def check_within_floor(w, gpu, ref, samples, label):
    """The FP64 bars of tests/parity.py, with the oracle's roundoff floor
    taken from the given roundoff samples of the oracle's result (one-ulp
    raised input, contracted build)."""
    f1 = np.max([parity.rel_l1(w, x, ref) for x in samples], axis=0)
    fi = np.max([parity.rel_linf(x, ref) for x in samples], axis=0)
    assert_parity(w, gpu, ref, label=label, floor=(f1, fi))


@pytest.mark.parametrize("lim,lname,path", [(6, "wenozp5", "plain"), (5, "mp5", "plain"), (0, "vanleer", "fused")])
def test_shu_osher(amr, orc, lim, lname, path):
    """200 steps (t ~ 0.8: the shock has crossed a third of the density
    wave) at the paper's 256 cells."""
    w = inputs.shu_osher(256, limiter=lim)
    print("GPU shu-osher %s path=%s" % (lname, path), flush=True)
    ref, f1, fi = parity.oracle_floor(orc, lambda: inputs.shu_osher(256, limiter=lim), nsteps=200)
    sim = amr.Simulation(w, path=amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN)
    sim.advance(200, nstages=3)
    assert sim.sync_flags()[0] == 0
    gpu = sim.cons()
    sim.close()
    assert_parity(w, gpu, ref, label="shu-osher %s %s" % (lname, path), floor=(f1, fi))


def test_kelvin_helmholtz_adaptive(amr, orc):
    """Three cycles of (2 steps, density-jump criterion on the oracle's
    ghost-filled state, plan, regrid) up to level 4, then 2 more steps; the
    same leaf sets drive the GPU run, the oracle and its two roundoff
    samples (the one-ulp-raised input, the contracted build)."""
    w = inputs.kelvin_helmholtz(max_level=1)
    wp = inputs.kelvin_helmholtz(max_level=1)
    wp.prim = parity.raise_one_ulp(wp.prim)
    sim = amr.Simulation(w, path=amr.PATH_PLAIN)
    o, op, of = orc.OracleSim(w), orc.OracleSim(wp), orc.OracleSim(w, fma=True)
    for cycle in range(3):
        sim.advance(2, nstages=3)
        o.steps(2)
        op.steps(2)
        of.steps(2)
        wc = dataclasses.replace(w, level=o.level, ijk=o.ijk)
        lv, ij = amr.regrid_plan(wc, gradient_flags(wc, o.padded()), max_level=4)
        print("GPU kelvin-helmholtz cycle %d blocks %d -> %d (max level %d)"
              % (cycle, len(o.level), len(lv), int(lv.max())), flush=True)
        new = sim.regrid(lv, ij)
        sim.close()
        sim = new
        o, op, of = o.regrid(lv, ij), op.regrid(lv, ij), of.regrid(lv, ij)
    sim.advance(2, nstages=3)
    o.steps(2)
    op.steps(2)
    of.steps(2)
    assert sim.sync_flags()[0] == 0
    assert int(o.level.max()) >= 3
    wn = dataclasses.replace(w, level=o.level, ijk=o.ijk)
    check_within_floor(wn, sim.cons(), o.cons(), [op.cons(), of.cons()], "kelvin-helmholtz adaptive")
    sim.close()
