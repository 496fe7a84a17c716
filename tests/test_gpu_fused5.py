"""The fused stage with three ghost layers (FP64, 2D and 3D: 'weno5',
'wenoz5', 'mp5', 'wenozp5' in one launch per stage): parity with the FP64
oracle on uniform and adaptive 2D and 3D grids, bit identity with the
per-kernel path where no coarse/fine faces exist, and a captured step equal
to the eager one."""
import dataclasses

import numpy as np
import pytest

from paper_2303_03026_amd import inputs
from test_gpu_parity import assert_parity
import parity

pytestmark = pytest.mark.gpu

LIMS = [(3, "weno5"), (4, "wenoz5"), (5, "mp5"), (6, "wenozp5")]


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


def weno(w, lim):
    w.limiter, w.ng = lim, 3
    return w


def run(amr, w, nsteps, path, graph=False):
    print("GPU fused5 lim=%d %s path=%s nsteps=%d nstages=%d flux=%d graph=%s"
          % (w.limiter, w.name, path, nsteps, w.nstages, w.flux, graph), flush=True)
    sim = amr.Simulation(w, path=amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN)
    sim.advance(nsteps, nstages=w.nstages, graph=graph)
    fl = sim.sync_flags()
    out = sim.cons()
    sim.close()
    return out, fl


def perturbed(w, seed=68):
    """The shock-cloud state with its density times 1 + 1e-3 u (u uniform in
    [-1, 1), seeded): no plateaus between equal jumps, where WENO-Z's
    weights would be decided by rounding."""
    r = np.random.Generator(np.random.PCG64(seed))
    w.prim[:, 0] *= 1.0 + 1e-3 * r.uniform(-1.0, 1.0, size=w.prim[:, 0].shape)
    return w


CASES = [("orszag_tang_2d", lambda: inputs.orszag_tang_2d(nsteps=40)),
         ("random_modes_3d_48", lambda: inputs.random_modes(48, 3, seed=61, nsteps=10)),
         ("smooth_amr_3d", lambda: dataclasses.replace(inputs.smooth_amr_state(3, nb1=2, seed=62), nsteps=4)),
         ("shock_cloud_32", lambda: perturbed(inputs.shock_cloud_amr(base_n=32, nsteps=6))),
         ("smooth_amr_2d", lambda: dataclasses.replace(inputs.smooth_amr_state(2, nb1=4, seed=63), nsteps=4)),
         ("kelvin_helmholtz_l3", lambda: dataclasses.replace(inputs.kelvin_helmholtz(max_level=3), nsteps=4))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("lim,lname", LIMS, ids=[n for _, n in LIMS])
def test_parity_with_oracle(amr, orc, lim, lname, name, make):
    """The FP64 bars of tests/parity.py, with the oracle's roundoff floor."""
    w = weno(make(), lim)
    ref, f1, fi = parity.oracle_floor(orc, lambda: weno(make(), lim))
    gpu, fl = run(amr, w, w.nsteps, "fused")
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label="fused5 %s %s" % (lname, name), floor=(f1, fi))


@pytest.mark.parametrize("flux", [0, 1, 2], ids=["hll", "hlld", "hllc"])
@pytest.mark.parametrize("lim,lname", LIMS, ids=[n for _, n in LIMS])
def test_bit_identical_to_per_kernel_path(amr, lim, lname, flux):
    """Without coarse/fine faces both paths take the same arithmetic in the
    same order."""
    w = weno(inputs.orszag_tang_2d(nsteps=10), lim)
    w.flux = flux
    a, fa = run(amr, w, 10, "plain")
    b, fb = run(amr, w, 10, "fused")
    assert fa[0] == 0 and fb[0] == 0
    assert np.array_equal(a, b)


@pytest.mark.parametrize("flux", [0, 1, 2], ids=["hll", "hlld", "hllc"])
@pytest.mark.parametrize("lim,lname", LIMS, ids=[n for _, n in LIMS])
def test_bit_identical_to_per_kernel_path_3d(amr, lim, lname, flux):
    """3D: the x and y flux differences go through the scratch array between
    the two sweeps, still in the per-kernel path's order."""
    w = weno(inputs.random_modes(32, 3, seed=70, nsteps=4), lim)
    w.flux = flux
    a, fa = run(amr, w, 4, "plain")
    b, fb = run(amr, w, 4, "fused")
    assert fa[0] == 0 and fb[0] == 0
    assert np.array_equal(a, b)


def test_ssprk54_bit_identical(amr):
    w = weno(inputs.orszag_tang_2d(nsteps=6), 6)
    w.nstages = 5
    a, _ = run(amr, w, 6, "plain")
    b, _ = run(amr, w, 6, "fused")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("ndim", [2, 3])
def test_graph_equals_eager(amr, ndim):
    w = weno(dataclasses.replace(inputs.smooth_amr_state(ndim, nb1=4 if ndim == 2 else 2, seed=64), nsteps=3), 6)
    a, _ = run(amr, w, 3, "fused", graph=False)
    b, _ = run(amr, w, 3, "fused", graph=True)
    assert np.array_equal(a, b)


def test_uniform_state_bit_identical_3d(amr):
    w = weno(inputs.uniform_state(3, (2, 2, 2), [1.3, 0.4, -0.25, 0.15, 0.8, 0.6, -0.9, 0.3, 0.0]), 6)
    sim = amr.Simulation(w, path=amr.PATH_FUSED)
    u0 = sim.cons()
    sim.advance(3, nstages=3)
    assert np.array_equal(sim.cons(), u0)
    sim.close()


def test_mixed_precision_refused(amr):
    """Three ghost layers are FP64 only."""
    for w in (weno(inputs.orszag_tang_2d(nsteps=2), 3), weno(inputs.random_modes(32, 3, seed=67), 3)):
        with pytest.raises(amr.AmrvacError):
            amr.Simulation(w, path=amr.PATH_FUSED, precision=amr.FP32_MIXED)
