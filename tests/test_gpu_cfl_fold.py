"""The next step's CFL rate folded into the last fused stage
(amrvac_stage_cfl): the time step it gives is the one the separate CFL pass
computes from the same state (same per-cell arithmetic, order-free maximum), so
runs are bit-identical; the held rate is dropped whenever it could be stale."""
import numpy as np
import pytest

from paper_2303_03026_amd import inputs

pytestmark = pytest.mark.gpu

SSPRK3 = [(0, 0, 1, 1.0), (1, 0, 2, 0.25), (2, 0, 0, 2.0 / 3.0)]


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


def manual(amr, w, nsteps, precision, fold):
    """SSPRK3 steps through the single-call ABI, folding or not."""
    sim = amr.Simulation(w, path=amr.PATH_FUSED, precision=precision)
    dts = []
    for _ in range(nsteps):
        sim.cfl(0)
        dts.append(sim.scalars()[0])
        for s, (i, b, o, wt) in enumerate(SSPRK3):
            sim.fill(i)
            sim.stage(i, b, o, wt, cfl=fold and s == 2)
    sim.sync_flags()
    out = sim.cons()
    sim.close()
    return out, dts


def five_cell(w):
    w.limiter, w.flux, w.ng = 6, 2, 3  # 'wenozp5' + HLLC
    return w


CASES = [("random_modes_3d_64", lambda: inputs.random_modes(64, 3, seed=2), 0),
         ("random_modes_3d_64_mixed", lambda: inputs.random_modes(64, 3, seed=3), 1),
         ("current_sheet_48", lambda: inputs.current_sheet(48, nsteps=4), 0),
         ("random_modes_2d_128", lambda: inputs.random_modes(128, 2, seed=4), 0),
         ("smooth_amr_3d", lambda: inputs.smooth_amr_state(3, nb1=2, seed=5), 0),
         # three ghost layers: the 2D stage folds, the 3D one leaves the rate
         # to the separate pass; either way the steps are the same
         ("wenozp5_2d_64", lambda: five_cell(inputs.random_modes(64, 2, seed=6)), 0),
         ("wenozp5_3d_32", lambda: five_cell(inputs.random_modes(32, 3, seed=7)), 0),
         ("wenozp5_3d_32_mixed", lambda: five_cell(inputs.random_modes(32, 3, seed=8)), 1)]


@pytest.mark.parametrize("name,make,precision", CASES, ids=[c[0] for c in CASES])
def test_folded_cfl_bit_identical(amr, name, make, precision):
    w = make()
    ref, dt_ref = manual(amr, w, 4, precision, fold=False)
    got, dt_got = manual(amr, w, 4, precision, fold=True)
    assert dt_got == dt_ref, name
    assert np.array_equal(got, ref), name
    # amrvac_advance folds on its own (eager and graph)
    for graph in (False, True):
        sim = amr.Simulation(w, path=amr.PATH_FUSED, precision=precision)
        sim.advance(4, nstages=3, graph=graph)
        sim.sync_flags()
        assert np.array_equal(sim.cons(), ref), (name, graph)
        sim.close()


def test_held_rate_dropped_when_stale(amr):
    a = inputs.random_modes(64, 3, seed=6)
    b = inputs.random_modes(64, 3, seed=7)
    sim = amr.Simulation(a, path=amr.PATH_FUSED)
    sim.cfl(0)
    for s, (i, bs, o, wt) in enumerate(SSPRK3):
        sim.fill(i)
        sim.stage(i, bs, o, wt, cfl=s == 2)
    # slot 0 now holds a folded rate; overwrite slot 0 with another state
    sim.set_primitive(b.prim)
    sim.cfl(0)
    dt_after = sim.scalars()
    fresh = amr.Simulation(b, path=amr.PATH_FUSED)
    fresh.cfl(0)
    assert dt_after == fresh.scalars()
    # a folded rate for slot 1 must not serve slot 0
    sim.fill(0)
    sim.stage(0, 0, 1, 1.0, cfl=True)
    sim.cfl(0)
    assert sim.scalars() == fresh.scalars()
    # ... but serves slot 1 exactly as the full pass would (both stages with
    # the same dt, c_h, kappa: cfl() overwrites them)
    s0 = sim.scalars()
    sim.stage(0, 0, 1, 1.0, cfl=True)
    sim.cfl(1)
    folded = sim.scalars()
    sim.set_scalars(*s0)
    sim.stage(0, 0, 1, 1.0)
    sim.cfl(1)
    assert folded == sim.scalars()
    sim.set_scalars(*s0)
    # the autotuner rewrites slot 1 and must leave no stale rate behind
    sim.stage(0, 0, 1, 1.0, cfl=True)
    sim.autotune(in_slot=0, out_slot=1, reps=1)
    sim.cfl(0)
    assert sim.scalars() == fresh.scalars()
    fl, nfix, _, rc = sim.sync_flags()
    assert rc == 0 and fl == 0
    sim.close()
    fresh.close()


def test_folded_cfl_flags_nonphysical(amr):
    # a state that is fine now but whose update drives the pressure negative
    # must be flagged by the folded pass just as by the separate one
    w = inputs.random_modes(32, 3, seed=8)
    w.prim[:, 4] = 1e-9  # cold gas: p -> small under any compression
    flags = []
    for fold in (False, True):
        sim = amr.Simulation(w, path=amr.PATH_FUSED)
        sim.cfl(0)
        for s, (i, b, o, wt) in enumerate(SSPRK3):
            sim.fill(i)
            sim.stage(i, b, o, wt, cfl=fold and s == 2)
        sim.cfl(0)
        flags.append(sim.sync_flags(raise_on_error=False)[0])
        sim.close()
    assert flags[0] == flags[1]
