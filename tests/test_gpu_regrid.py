"""Regrid on the device (amrvac_regrid) against the oracle's (oracle_regrid):
the moved state, runs continued on the new leaf set, and an adaptive run that
regrids every few steps from a gradient criterion."""
import dataclasses

import numpy as np
import pytest

from paper_2303_03026_amd import inputs
from test_gpu_parity import assert_parity, rel_l1

pytestmark = pytest.mark.gpu

NV = 9
PATHS = ["plain", "fused"]


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


def flags_for(w, seed, p_refine=0.3):
    r = np.random.Generator(np.random.PCG64(seed))
    return np.where(r.random(w.nblocks) < p_refine, 1, -1).astype(np.int32)


def blocks_of(level, ijk):
    return [(int(l), int(p[0]), int(p[1]), int(p[2])) for l, p in zip(level, ijk)]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("ndim", [2, 3])
def test_transfer_matches_oracle(amr, orc, ndim, path):
    w = inputs.smooth_amr_state(ndim, nb1=4 if ndim == 2 else 2, seed=5)
    print("GPU regrid transfer ndim=%d path=%s nblocks=%d" % (ndim, path, w.nblocks), flush=True)
    sim = amr.Simulation(w, path=amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN)
    o = orc.OracleSim(w)
    u_old = sim.cons()
    # coarsen every top-level sibling set (nothing is finer, so nesting never
    # blocks it) and refine every other block of the level below: copies,
    # prolongations and restrictions all occur
    top = int(w.level.max())
    flags = np.where(w.level == top, -1, np.where((w.level == top - 1) & (np.arange(w.nblocks) % 2 == 0), 1, 0))
    lv, ij = sim.regrid_plan(flags)
    new = sim.regrid(lv, ij)
    onew = o.regrid(lv, ij)
    got, ref = new.cons(), onew.cons()
    # (the two sides' initial states already differ in the last bits, from
    # their own primitive-to-conserved conversions)
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-15)
    old = {k: b for b, k in enumerate(blocks_of(w.level, w.ijk))}
    copies = restricted = 0
    for n, (l, i, j, k) in enumerate(blocks_of(lv, ij)):
        if (l, i, j, k) in old:  # copied bit for bit
            assert np.array_equal(got[n], u_old[old[(l, i, j, k)]])
            copies += 1
        elif (l - 1, i >> 1, j >> 1, k >> 1) not in old:  # restricted: pairwise mean of the children
            kid = lambda a, b_, e: u_old[old[(l + 1, 2 * i + a, 2 * j + b_, 2 * k + e if ndim == 3 else 0)]]  # noqa: E731
            ch = np.zeros_like(got[n])
            if ndim == 2:
                c = [[kid(a, b_, 0) for a in (0, 1)] for b_ in (0, 1)]
                for y in range(16):
                    for x in range(16):
                        src = c[y // 8][x // 8]
                        fy, fx = 2 * (y % 8), 2 * (x % 8)
                        ch[:, y, x] = ((src[:, fy, fx] + src[:, fy, fx + 1]) + (src[:, fy + 1, fx] + src[:, fy + 1, fx + 1])) * 0.25
                assert np.array_equal(got[n], ch)
            restricted += 1
    assert copies and restricted and copies + restricted < len(lv)
    assert new.get_tune() == sim.get_tune()
    new.close()
    sim.close()


@pytest.mark.parametrize("path", PATHS + ["plain-wenozp5"])
def test_runs_on_after_regrid(amr, orc, path):
    w = inputs.smooth_amr_state(3, nb1=2, seed=7)
    if path == "plain-wenozp5":  # three ghost layers through the regrid
        w.limiter, w.ng = 6, 3
    sim = amr.Simulation(w, path=amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN)
    o = orc.OracleSim(w)
    sim.advance(2, nstages=3)
    o.steps(2)
    lv, ij = sim.regrid_plan(flags_for(w, 2))
    new = sim.regrid(lv, ij)
    sim.close()
    onew = o.regrid(lv, ij)
    new.advance(3, nstages=3)
    onew.steps(3)
    assert new.sync_flags()[0] == 0
    wn = dataclasses.replace(w, level=lv, ijk=ij)
    assert_parity(wn, new.cons(), onew.cons(), label="regrid then 3 steps %s" % path)
    new.close()


def test_uniform_state_exact_through_regrid(amr):
    base, level, ijk = inputs.amr_test_hierarchy(3, nb1=2, seed=11)
    w = inputs.uniform_state(3, base, [1.3, 0.4, -0.25, 0.15, 0.8, 0.6, -0.9, 0.3, 0.0], level=level, ijk=ijk)
    w.base_blocks = base
    sim = amr.Simulation(w, path=amr.PATH_FUSED)
    u0 = sim.cons()[0, :, 0, 0, 0]
    lv, ij = sim.regrid_plan(flags_for(w, 3))
    new = sim.regrid(lv, ij)
    u = new.cons()
    assert np.array_equal(u, np.broadcast_to(u0.reshape(1, NV, 1, 1, 1), u.shape))
    new.advance(2, nstages=3)
    assert np.array_equal(new.cons(), u)
    new.close()
    sim.close()


def test_mixed_precision_transfer(amr, orc):
    w = inputs.smooth_amr_state(3, nb1=2, seed=5)
    sim = amr.Simulation(w, path=amr.PATH_FUSED, precision=amr.FP32_MIXED)
    lv, ij = sim.regrid_plan(flags_for(w, 4))
    new = sim.regrid(lv, ij)
    ref = orc.OracleSim(w).regrid(lv, ij).cons()
    err = rel_l1(dataclasses.replace(w, level=lv, ijk=ij), new.cons(), ref)
    assert np.all(err[[0, 4]] < 1e-7), err
    new.close()
    sim.close()


def gradient_flags(w, u, hi=0.02, lo=0.005):
    """Refine where the density's largest cell-to-cell jump in a block,
    relative to the block's mean density, exceeds hi; coarsen below lo."""
    f = np.zeros(w.nblocks, dtype=np.int32)
    for b in range(w.nblocks):
        rho = u[b, 0]
        jump = max(np.max(np.abs(np.diff(rho, axis=a))) for a in range(w.ndim))
        rel = jump / np.mean(np.abs(rho))
        f[b] = 1 if rel > hi else (-1 if rel < lo else 0)
    return f


@pytest.mark.parametrize("ndim", [2, 3])
def test_adaptive_run_matches_oracle(amr, orc, ndim):
    """Three cycles of (steps, criterion, plan, regrid) on a smooth state;
    the criterion is evaluated on the oracle's state and the same leaf set
    is applied on both sides."""
    w = inputs.smooth_amr_state(ndim, nb1=4 if ndim == 2 else 2, seed=9)
    sim = amr.Simulation(w, path=amr.PATH_FUSED)
    o = orc.OracleSim(w)
    for cycle in range(3):
        sim.advance(2, nstages=3)
        o.steps(2)
        wc = dataclasses.replace(w, level=o.level, ijk=o.ijk)
        lv, ij = amr.regrid_plan(wc, gradient_flags(wc, o.cons()), max_level=4)
        print("GPU adaptive cycle %d ndim=%d blocks %d -> %d" % (cycle, ndim, len(o.level), len(lv)), flush=True)
        new = sim.regrid(lv, ij)
        sim.close()
        sim = new
        o = o.regrid(lv, ij)
    sim.advance(2, nstages=3)
    o.steps(2)
    assert sim.sync_flags()[0] == 0
    wn = dataclasses.replace(w, level=o.level, ijk=o.ijk)
    assert_parity(wn, sim.cons(), o.cons(), label="adaptive %dd" % ndim)
    sim.close()


def test_regrid_rejects_a_two_level_jump(amr):
    w = inputs.smooth_amr_state(2, nb1=4, seed=5)
    sim = amr.Simulation(w, path=amr.PATH_FUSED)
    lv, ij = sim.regrid_plan(np.ones(w.nblocks, dtype=np.int32))
    lv2, ij2 = amr.regrid_plan(dataclasses.replace(w, level=lv, ijk=ij), np.ones(len(lv), dtype=np.int32))
    with pytest.raises(amr.AmrvacError):
        sim.regrid(lv2, ij2)  # every block two levels finer
    sim.close()
