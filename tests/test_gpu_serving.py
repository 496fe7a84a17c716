"""Batch (serving) contexts: several independent jobs resident in one block
pool, advanced together with per-job dt; each job's result is the same alone
and in the mix (bit for bit: no arithmetic couples jobs), and matches the
CPU oracle (FP64 jobs to the bars of tests/parity.py, FP32-mixed jobs to
the bounds of tests/mixed_error.py).  Pools also take the five-cell
reconstructions on three ghost layers."""
import dataclasses

import numpy as np
import pytest

from paper_2303_03026_amd import inputs
import mixed_error
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


def alone(amr, w, nsteps, precision):
    sim = amr.Simulation(w, path=amr.PATH_FUSED, precision=precision)
    sim.advance(nsteps)
    sim.sync_flags()
    out = sim.cons()
    sim.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_job_alone_equals_in_mix_3d(amr, orc, precision):
    shape = inputs.random_modes(32, 3, seed=0)
    batch = amr.Batch(shape, capacity_blocks=300, max_jobs=8, precision=precision)
    ws = [inputs.random_modes(32, 3, seed=11, nsteps=7),
          inputs.random_modes(48, 3, seed=12, nsteps=12),
          inputs.smooth_amr_state(3, nb1=2, seed=7),
          inputs.random_modes(32, 3, seed=13, nsteps=3)]
    ws[2].nsteps = 5
    ids = [batch.add_job(w) for w in ws]
    assert all(i is not None for i in ids)
    rounds = 0
    while any(batch.job_info(i)[1] > 0 for i in ids):
        batch.step()
        rounds += 1
    assert rounds == 12
    outs = [batch.get_job(i) for i in ids]
    batch.sync_flags()
    batch.close()
    for w, got in zip(ws, outs):
        ref = alone(amr, w, w.nsteps, precision)
        assert np.array_equal(got, ref), w.name
    for w, got in zip(ws, outs):
        ref, _ = orc.run(w)
        if precision == 0:  # the FP64 bars, all nine variables
            parity.check(w, got, ref, "served %s" % w.name)
        else:  # the FP32-mixed bounds of these short runs (test_gpu_mixed.py)
            l1, linf = mixed_error.errors(w, got, ref)
            b1, bi = np.full(9, 1e-6), np.full(9, 5e-6)
            if w.name.startswith("smooth_amr"):  # psi ~ 0.01 |B|: its FP32 error is that of B
                b1[8], bi[8] = 2e-5, 2e-4
            mixed_error.check("served mixed %s" % w.name, l1, linf, b1, bi)


def test_job_alone_equals_in_mix_2d(amr):
    shape = inputs.random_modes(32, 2, seed=0)
    batch = amr.Batch(shape, capacity_blocks=200, max_jobs=8)
    ws = [inputs.random_modes(64, 2, seed=21, nsteps=9), inputs.random_modes(128, 2, seed=22, nsteps=4),
          inputs.orszag_tang_2d(nsteps=6)]
    ws[2].nstages = 3  # a batch steps SSPRK(3,3)
    ids = [batch.add_job(w) for w in ws]
    while any(batch.job_info(i)[1] > 0 for i in ids):
        batch.step()
    outs = [batch.get_job(i) for i in ids]
    batch.close()
    for w, got in zip(ws, outs):
        ref = alone(amr, w, w.nsteps, 0)
        assert np.array_equal(got, ref), w.name


def weno(w, lim=6, flux=2):
    w.limiter, w.flux, w.ng = lim, flux, 3
    return w


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_five_cell_jobs_alone_equal_in_mix(amr, orc, ndim, precision):
    """Pools with three ghost layers ('wenozp5' + HLLC): the fused five-cell
    stage over every resident job's blocks; each job equals its single-job
    run bit for bit and meets the FP64 bars with the oracle's roundoff floor,
    or the FP32-mixed five-cell bounds of test_gpu_fused5.py."""
    shape = weno(inputs.random_modes(32, ndim, seed=0))
    batch = amr.Batch(shape, capacity_blocks=300 if ndim == 3 else 400, max_jobs=8, precision=precision)
    if ndim == 3:
        makes = [lambda: weno(inputs.random_modes(32, 3, seed=31, nsteps=5)),
                 lambda: weno(inputs.random_modes(48, 3, seed=32, nsteps=3)),
                 lambda: weno(dataclasses.replace(inputs.smooth_amr_state(3, nb1=2, seed=33), nsteps=4))]
    else:
        makes = [lambda: weno(inputs.random_modes(64, 2, seed=34, nsteps=6)),
                 lambda: weno(dataclasses.replace(inputs.smooth_amr_state(2, nb1=4, seed=35), nsteps=4)),
                 lambda: weno(inputs.random_modes(128, 2, seed=36, nsteps=3))]
    ws = [m() for m in makes]
    ids = [batch.add_job(w) for w in ws]
    assert all(i is not None for i in ids)
    while any(batch.job_info(i)[1] > 0 for i in ids):
        batch.step()
    outs = [batch.get_job(i) for i in ids]
    batch.sync_flags()
    batch.close()
    for w, got in zip(ws, outs):
        assert np.array_equal(got, alone(amr, w, w.nsteps, precision)), w.name
    for make, w, got in zip(makes, ws, outs):
        if precision == 0:
            ref, f1, fi = parity.oracle_floor(orc, make)
            parity.check(w, got, ref, "served five-cell %s" % w.name, f1, fi)
        else:
            ref, _ = orc.run(w)
            l1, linf = mixed_error.errors(w, got, ref)
            b1, bi = np.full(9, 1e-6), np.full(9, 3e-6)
            if w.name.startswith("smooth_amr"):
                b1[8], bi[8] = 4e-5, 6e-4
            mixed_error.check("served five-cell mixed %s" % w.name, l1, linf, b1, bi)


def test_admission_by_pool_room_and_reuse(amr):
    shape = inputs.random_modes(32, 3, seed=0)
    batch = amr.Batch(shape, capacity_blocks=20, max_jobs=4)
    w = inputs.random_modes(32, 3, seed=1, nsteps=2)  # 8 blocks
    a = batch.add_job(w)
    b = batch.add_job(w)
    assert a is not None and b is not None
    assert batch.add_job(w) is None           # 4 places left: no room
    assert batch.free_blocks() == (4, 4)
    batch.remove_job(a)
    assert batch.free_blocks() == (8, 12)
    c = batch.add_job(w)
    assert c is not None
    while batch.job_info(c)[1] > 0:
        batch.step()
    got = batch.get_job(c)
    batch.close()
    assert np.array_equal(got, alone(amr, w, 2, 0))


def test_batch_rejects_other_physics(amr):
    shape = inputs.random_modes(32, 3, seed=0)
    batch = amr.Batch(shape, capacity_blocks=50, max_jobs=2)
    w = inputs.random_modes(32, 3, seed=1, nsteps=2)
    w.gamma = 1.4
    with pytest.raises(amr.AmrvacError):
        batch.add_job(w)
    batch.close()


def test_serving_engine_small_stream(amr):
    from paper_2303_03026_amd import serve
    jobs = inputs.serving_jobs(24, seed=8)
    rng = np.random.Generator(np.random.PCG64(3))
    for j in jobs:
        j["n"] = int(rng.choice([32, 48, 64] if j["ndim"] == 2 else [32, 48]))
        j["steps"] = int(rng.integers(3, 12))
    eng = serve.ServingEngine(budget_bytes=2e9, max_jobs=16)
    keep = {jobs[0]["id"], jobs[5]["id"]}
    res = eng.run(jobs, time_scale=0.002, keep_results=keep)
    eng.close()
    assert res["jobs"] == 24
    assert res["latency_p99_s"] >= res["latency_p50_s"] > 0
    for j in jobs:
        if j["id"] in keep:
            w = inputs.serving_job_workload(j)
            ref = alone(amr, w, j["steps"], 1 if j["mixed"] else 0)
            assert np.array_equal(res["results"][j["id"]], ref)
