"""Loehner's refinement indicator on the device (amrvac_lohner) against the
oracle's (lohner_indicator on its ghost-filled blocks), and an adaptive
Kelvin-Helmholtz run whose refinement flags come from the device."""
import dataclasses

import numpy as np
import pytest

from paper_2303_03026_amd import inputs
from test_gpu_parity import assert_parity
import parity

pytestmark = pytest.mark.gpu

NV = 9
W_RHO = [1.0] + [0.0] * 8
# rho and e.  (A field that is zero up to roundoff, like B_y in the shock
# cloud, has an indicator that is a ratio of roundoff terms: O(1) and not
# reproducible, so such fields are not weighted.)
W_MIX = [1.0, 0.0, 0.0, 0.0, 0.5, 0.0, 0.0, 0.0, 0.0]


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


CASES = [("smooth_amr_3d", lambda: inputs.smooth_amr_state(3, nb1=2, seed=91)),
         ("smooth_amr_2d", lambda: inputs.smooth_amr_state(2, nb1=4, seed=92)),
         ("shock_cloud_32", lambda: inputs.shock_cloud_amr(base_n=32)),
         ("current_sheet_32", lambda: inputs.current_sheet(32)),
         ("kelvin_helmholtz_l3", lambda: inputs.kelvin_helmholtz(max_level=3))]


@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_indicator_matches_oracle(amr, orc, name, make, path):
    w = make()
    if path == "fused" and w.ng != 2:
        w = dataclasses.replace(w, ng=2, limiter=0)
    print("GPU lohner %s path=%s nblocks=%d" % (name, path, w.nblocks), flush=True)
    sim = amr.Simulation(w, path=amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN)
    sim.advance(2, nstages=3)
    o = orc.OracleSim(w)
    o.steps(2)
    for wts in (W_RHO, W_MIX):
        got = sim.lohner(weights=wts, wavefilter=0.01)
        ref = orc.lohner_indicator(w, o.padded(), wts, 0.01)
        assert np.all(np.isfinite(got))
        np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-14)
    sim.close()
    o.close()


def test_uniform_state_gives_zero(amr):
    base, level, ijk = inputs.amr_test_hierarchy(3, nb1=2, seed=11)
    w = inputs.uniform_state(3, base, [1.3, 0.4, -0.25, 0.15, 0.8, 0.6, -0.9, 0.3, 0.0], level=level, ijk=ijk)
    w.base_blocks = base
    sim = amr.Simulation(w, path=amr.PATH_FUSED)
    assert np.all(sim.lohner(weights=[1.0] * NV) == 0.0)
    sim.close()


def test_mixed_precision_indicator(amr):
    """FP32-mixed storage rounds the state to float (2^-24 relative); the
    indicator divides second differences by first differences, which are
    ~1e-3 of the values on this smooth state, so it agrees with the FP64 one
    to about 1e-4 relative (measured max 1.0e-4)."""
    w = inputs.smooth_amr_state(3, nb1=2, seed=93)
    a = amr.Simulation(w, path=amr.PATH_FUSED)
    b = amr.Simulation(w, path=amr.PATH_FUSED, precision=amr.FP32_MIXED)
    ia, ib = a.lohner(weights=W_MIX), b.lohner(weights=W_MIX)
    np.testing.assert_allclose(ib, ia, rtol=1e-3, atol=1e-6)
    a.close()
    b.close()


def test_rejects_bad_arguments(amr):
    w = inputs.smooth_amr_state(2, nb1=4, seed=94)
    sim = amr.Simulation(w, path=amr.PATH_PLAIN)
    for wts in ([0.0] * NV, [-1.0] + [0.0] * 8, [np.nan] + [0.0] * 8):
        with pytest.raises(amr.AmrvacError):
            sim.lohner(weights=wts)
    with pytest.raises(amr.AmrvacError):
        sim.lohner(weights=W_RHO, wavefilter=-0.1)
    with pytest.raises(amr.AmrvacError):
        sim.lohner(weights=W_RHO, slot=7)
    sim.close()


def test_kelvin_helmholtz_adaptive_on_device_flags(amr, orc):
    """Three cycles of (2 steps, device Loehner flags, plan, regrid) up to
    level 4 on the shear layer (HLLC, 'wenozp5'); the oracle's indicator on
    its own state gives the same flags (blocks within 1e-9 of a threshold
    excepted), the same leaf sets drive both, and the final states agree."""
    refine, ratio = 0.05, 0.25
    w = inputs.kelvin_helmholtz(max_level=1)
    sim = amr.Simulation(w, path=amr.PATH_PLAIN)
    o = orc.OracleSim(w)
    wp = inputs.kelvin_helmholtz(max_level=1)
    wp.prim = parity.raise_one_ulp(wp.prim)
    samples = [orc.OracleSim(wp), orc.OracleSim(w, fma=True)]  # roundoff samples on the same leaf sets
    grew = False
    for cycle in range(3):
        sim.advance(2, nstages=3)
        o.steps(2)
        for x in samples:
            x.steps(2)
        ind = sim.lohner(weights=W_RHO)
        wc = dataclasses.replace(w, level=o.level, ijk=o.ijk)
        ref = orc.lohner_indicator(wc, o.padded(), W_RHO, 0.01)
        near = (np.abs(ref - refine) < 1e-9 * refine) | (np.abs(ref - refine * ratio) < 1e-9 * refine)
        flags = np.where(ind > refine, 1, np.where(ind < refine * ratio, -1, 0)).astype(np.int32)
        oflags = np.where(ref > refine, 1, np.where(ref < refine * ratio, -1, 0)).astype(np.int32)
        assert np.array_equal(flags[~near], oflags[~near])
        lv, ij = sim.regrid_plan(flags, max_level=4)
        print("GPU kh lohner cycle %d: %d refine, %d coarsen, blocks %d -> %d"
              % (cycle, int((flags > 0).sum()), int((flags < 0).sum()), len(o.level), len(lv)), flush=True)
        grew = grew or len(lv) > len(o.level)
        new = sim.regrid(lv, ij)
        sim.close()
        sim = new
        o = o.regrid(lv, ij)
        samples = [x.regrid(lv, ij) for x in samples]
    sim.advance(2, nstages=3)
    o.steps(2)
    for x in samples:
        x.steps(2)
    assert grew and sim.sync_flags()[0] == 0
    wn = dataclasses.replace(w, level=o.level, ijk=o.ijk)
    ref = o.cons()
    f1 = np.max([parity.rel_l1(wn, x.cons(), ref) for x in samples], axis=0)
    fi = np.max([parity.rel_linf(x.cons(), ref) for x in samples], axis=0)
    assert_parity(wn, sim.cons(), ref, label="kelvin-helmholtz lohner adaptive", floor=(f1, fi))
    sim.close()
