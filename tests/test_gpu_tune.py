"""Launch shapes of the fused stage and the autotuner that picks among them.

Every shape (z segments per block, rotation of the per-plane extra work over
the waves, XCD-contiguous block order) runs the same arithmetic on the same
cells, so results are bit-identical to the default shape; the autotuner's
choice is then a pure speed decision."""
import os

import numpy as np
import pytest

from paper_2303_03026_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


def run_shape(amr, w, shape, nsteps, precision=0):
    sim = amr.Simulation(w, path=amr.PATH_FUSED, precision=precision)
    if shape is not None:
        sim.set_tune(*shape)
        assert sim.get_tune() == tuple(shape)
    sim.advance(nsteps)
    sim.sync_flags()
    out = sim.cons()
    sim.close()
    return out


CASES = [
    ("random_modes_3d_64", lambda: inputs.random_modes(64, 3, seed=5), 0),
    ("random_modes_3d_64_mixed", lambda: inputs.random_modes(64, 3, seed=6), 1),
    ("smooth_amr_3d", lambda: inputs.smooth_amr_state(3, nb1=2, seed=3), 0),
    ("current_sheet_48", lambda: inputs.current_sheet(48, nsteps=3), 0),
    ("random_modes_2d_64", lambda: inputs.random_modes(64, 2, seed=7), 0),
]


@pytest.mark.parametrize("name,make,precision", CASES, ids=[c[0] for c in CASES])
def test_every_shape_bit_identical(amr, name, make, precision):
    w = make()
    ref = run_shape(amr, w, None, 3, precision)
    for shape in amr.tune_candidates(w.ndim):
        got = run_shape(amr, w, shape, 3, precision)
        assert np.array_equal(got, ref), (name, shape)


def test_autotune_picks_a_candidate_and_caches(amr, tmp_path):
    w = inputs.random_modes(64, 3, seed=5)
    ref = run_shape(amr, w, None, 2)
    sim = amr.Simulation(w, path=amr.PATH_FUSED)
    sim.reset_flags()
    cache = str(tmp_path / "tune.json")
    best, times = sim.autotune(reps=3, cache=cache)
    assert best in amr.tune_candidates(3)
    assert len(times) == 12 and all(t > 0 for t in times.values())
    assert min(times, key=times.get) == best
    assert sim.get_tune() == best
    fl, nfix, _, rc = sim.sync_flags()
    assert rc == 0 and fl == 0 and nfix == 0
    # the autotuner overwrote slot 1 and filled slot 0's ghosts only: a run
    # from the untouched initial state matches the default shape
    sim.set_primitive(w.prim)
    sim.advance(2)
    got = sim.cons()
    sim.close()
    assert np.array_equal(got, ref)
    # cache hit: same shape, no timing
    sim2 = amr.Simulation(w, path=amr.PATH_FUSED)
    best2, times2 = sim2.autotune(cache=cache)
    assert best2 == best and times2 == {}
    assert sim2.get_tune() == best
    sim2.close()
    assert os.path.exists(cache)


def test_tune_rejects_bad_shapes(amr):
    w = inputs.random_modes(32, 2, seed=1)
    sim = amr.Simulation(w, path=amr.PATH_FUSED)
    for bad in [(3, 0, 1), (2, 0, 1), (1, 2, 1), (1, 0, 5)]:
        with pytest.raises(amr.AmrvacError):
            sim.set_tune(*bad)
    assert sim.get_tune() == (1, 0, 1)
    sim.close()


def test_batch_shape_bit_identical(amr):
    shape = inputs.random_modes(32, 3, seed=0)
    ws = [inputs.random_modes(32, 3, seed=31, nsteps=4), inputs.random_modes(48, 3, seed=32, nsteps=3)]
    outs = {}
    for tune in [(1, 0, 1), (4, 1, 0), (2, 1, 1)]:
        batch = amr.Batch(shape, capacity_blocks=100, max_jobs=4)
        batch.set_tune(*tune)
        ids = [batch.add_job(w) for w in ws]
        while any(batch.job_info(i)[1] > 0 for i in ids):
            batch.step()
        outs[tune] = [batch.get_job(i) for i in ids]
        batch.close()
    for tune, got in outs.items():
        for a, b in zip(got, outs[(1, 0, 1)]):
            assert np.array_equal(a, b), tune
