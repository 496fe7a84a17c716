"""Blocks of 4, 6, 8 and 12 cells per direction on the plain path (the
fused path and FP32-mixed are built for 16), with 2 ghost layers and, where
the block holds at least 6 cells, 3: parity with the oracle on uniform and
2-level AMR grids, and bit identity of uniform states."""
import numpy as np
import pytest

from paper_2303_03026_amd import inputs
from test_gpu_parity import assert_parity

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


SHAPES = [(2, 4, 0, 0), (2, 8, 0, 1), (2, 12, 2, 2), (3, 4, 0, 0), (3, 8, 1, 2), (3, 6, 6, 2), (2, 6, 5, 0),
          (2, 8, 6, 2)]


@pytest.mark.parametrize("ndim,nx,lim,flux", SHAPES, ids=["%dd-nx%d-lim%d-flux%d" % s for s in SHAPES])
def test_parity_smooth_amr(amr, orc, ndim, nx, lim, flux):
    w = inputs.smooth_amr_state(ndim, nb1=4 if ndim == 2 else 2, seed=95, nx=nx)
    w.limiter, w.flux, w.ng = lim, flux, 3 if lim >= 3 else 2
    nsteps = 6 if ndim == 2 else 3
    print("GPU block size %dD nx=%d lim=%d flux=%d nblocks=%d" % (ndim, nx, lim, flux, w.nblocks), flush=True)
    ref, _ = orc.run(w, nsteps=nsteps)
    sim = amr.Simulation(w, path=amr.PATH_PLAIN)
    sim.advance(nsteps, nstages=3)
    assert sim.sync_flags()[0] == 0
    got = sim.cons()
    sim.close()
    assert_parity(w, got, ref, label="nx=%d %dD lim=%d flux=%d" % (nx, ndim, lim, flux))


@pytest.mark.parametrize("nx", [4, 6, 10])
def test_uniform_state_bit_identical(amr, nx):
    base, level, ijk = inputs.amr_test_hierarchy(3, nb1=2, seed=11, nx=nx)
    w = inputs.uniform_state(3, base, [1.3, 0.4, -0.25, 0.15, 0.8, 0.6, -0.9, 0.3, 0.0], nx=nx, level=level, ijk=ijk)
    w.base_blocks = base
    sim = amr.Simulation(w, path=amr.PATH_PLAIN)
    u0 = sim.cons()
    sim.advance(3, nstages=3)
    assert np.array_equal(sim.cons(), u0)
    sim.close()


def test_fused_path_needs_16(amr):
    w = inputs.smooth_amr_state(3, nb1=2, seed=95, nx=8)
    with pytest.raises(amr.AmrvacError):
        amr.Simulation(w, path=amr.PATH_FUSED)
    with pytest.raises(amr.AmrvacError):
        amr.Simulation(w, path=amr.PATH_PLAIN, precision=amr.FP32_MIXED)
