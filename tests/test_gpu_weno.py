"""Fifth-order reconstructions on 3 ghost layers ('weno5': Jiang-Shu weights,
'wenoz5': Borges et al.'s WENO-Z weights, 'wenozp5': Acker et al.'s WENO-Z+
weights, 'mp5': Suresh and Huynh's monotonicity-preserving scheme), on the
plain FP64 path, against the FP64 oracle (the fused path, FP32-mixed and
batch pools with 3 layers have their own tests)."""
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


def run_gpu(amr, w, nsteps, graph=False, nslots=None):
    print("GPU weno lim=%d %s ng=%d nsteps=%d nstages=%d flux=%d graph=%s"
          % (w.limiter, w.name, w.ng, nsteps, w.nstages, w.flux, graph), flush=True)
    sim = amr.Simulation(w, nslots=nslots, path=amr.PATH_PLAIN)
    sim.advance(nsteps, nstages=w.nstages, graph=graph)
    fl = sim.sync_flags()
    out = sim.cons()
    sim.close()
    return out, fl


CASES = [("random_modes_3d_48", lambda: inputs.random_modes(48, 3, seed=61, nsteps=10)),
         ("orszag_tang_2d", lambda: inputs.orszag_tang_2d(nsteps=40)),
         ("smooth_amr_3d", lambda: inputs.smooth_amr_state(3, nb1=2, seed=62)),
         ("smooth_amr_2d", lambda: inputs.smooth_amr_state(2, nb1=4, seed=63)),
         ("shock_cloud_32", lambda: perturbed(inputs.shock_cloud_amr(base_n=32, nsteps=6)))]


def perturbed(w, seed=68):
    """The shock-cloud state with its density times 1 + 1e-3 u (u uniform in
    [-1, 1), seeded).  The exactly piecewise-constant cloud gives plateaus
    between equal jumps, where WENO-Z's weights are discontinuous in the data
    (its tau5 rounds to zero or not), so its result there is decided by
    rounding; the perturbation removes such plateaus."""
    r = np.random.Generator(np.random.PCG64(seed))
    w.prim[:, 0] *= 1.0 + 1e-3 * r.uniform(-1.0, 1.0, size=w.prim[:, 0].shape)
    return w


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("lim,lname", LIMS, ids=[n for _, n in LIMS])
def test_parity_with_oracle(amr, orc, lim, lname, name, make):
    def build():
        w = weno(make(), lim)
        if name.startswith("smooth_amr"):
            w.nsteps = 4
        return w
    parity_within_floor(amr, orc, build, "%s %s" % (lname, name))


def parity_within_floor(amr, orc, build, label, nslots=None):
    """The FP64 bars of tests/parity.py with the oracle's roundoff floor,
    measured here.  psi grows from the divergence error of the
    reconstruction, which these fifth-order schemes make small (L1 psi / L1
    B ~ 1e-4 on random modes), so roundoff is large relative to psi: its
    floor reaches 1.2e-12 (mp5, random modes), and 1e-11 for the shock
    cloud's transverse fields and psi; every other variable's floor is about
    1e-15."""
    w = build()
    ref, f1, fi = parity.oracle_floor(orc, build)
    gpu, fl = run_gpu(amr, w, w.nsteps, nslots=nslots)
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label=label, floor=(f1, fi))


@pytest.mark.parametrize("lim,lname", LIMS, ids=[n for _, n in LIMS])
def test_with_ssprk54_and_hlld(amr, orc, lim, lname):
    """The fourth-order integrator and the five-wave solver with the
    fifth-order reconstructions, the pairing a high-order run takes."""
    def build():
        w = weno(inputs.random_modes(32, 3, seed=64, nsteps=6), lim)
        w.nstages, w.flux = 5, 1
        return w
    parity_within_floor(amr, orc, build, "%s ssprk54 hlld" % lname, nslots=4)


@pytest.mark.parametrize("lim,lname", LIMS, ids=[n for _, n in LIMS])
def test_uniform_state_bit_identical(amr, lim, lname):
    w = weno(inputs.uniform_state(3, (2, 2, 2), [1.3, 0.4, -0.25, 0.15, 0.8, 0.6, -0.9, 0.3, 0.0]), lim)
    sim = amr.Simulation(w, path=amr.PATH_PLAIN)
    u0 = sim.cons()
    sim.advance(3, nstages=3)
    assert np.array_equal(sim.cons(), u0)
    sim.close()


def test_graph_equals_eager(amr):
    w = weno(inputs.smooth_amr_state(3, nb1=2, seed=65), 3)
    a, _ = run_gpu(amr, w, 3, graph=False)
    b, _ = run_gpu(amr, w, 3, graph=True)
    assert np.array_equal(a, b)


def test_three_ghost_layers_change_nothing_for_van_leer(amr):
    """The third ghost layer is filled (same level, prolonged, restricted) but
    the four-cell stencil never reads it: bit-identical to 2 layers."""
    outs = []
    for ng in (2, 3):
        w = inputs.smooth_amr_state(3, nb1=2, seed=66)
        w.ng = ng
        outs.append(run_gpu(amr, w, 3)[0])
    assert np.array_equal(outs[0], outs[1])


def test_plain_path_refuses_mixed_and_five_cells_need_three_layers(amr):
    w = weno(inputs.random_modes(32, 3, seed=67), 3)
    sim = amr.Simulation(w, path=amr.PATH_FUSED, precision=amr.FP32_MIXED)
    with pytest.raises(amr.AmrvacError):
        sim.set_path(amr.PATH_PLAIN)  # the per-kernel path is FP64 only
    sim.close()
    w2 = inputs.random_modes(32, 3, seed=67)
    w2.limiter = 3  # WENO on 2 ghost layers: the stencil does not fit
    with pytest.raises(amr.AmrvacError):
        amr.Simulation(w2, path=amr.PATH_PLAIN)
