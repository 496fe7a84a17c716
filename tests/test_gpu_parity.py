"""GPU parity: the HIP path, called through the C ABI, against the FP64 CPU
oracle on the same seeded inputs.

Bars (tests/parity.py): relative L1 per conserved variable <= 1e-12
(volume-weighted over leaf interior cells) and element-wise relative L-inf
<= 1e-11; variables that are identically zero in the oracle must be exactly
zero on the GPU.  The beta = 0.01 current sheet is measured against the
oracle's roundoff floor as well.  Uniform states must stay bit-identical.
"""

import numpy as np
import pytest

from paper_2303_03026_amd import inputs
import parity

pytestmark = pytest.mark.gpu

NV = 9
RHO, VX, VY, VZ, PR, BX, BY, BZ, PSI = range(NV)
PATHS = ["plain", "fused"]


def vol_weights(w):
    return parity.vol_weights(w).reshape(-1)


def rel_l1(w, a, b):
    """Per-variable volume-weighted relative L1 of a against reference b."""
    return parity.rel_l1(w, a, b)


def assert_parity(w, gpu, ref, label="", floor=None):
    """The FP64 bars of tests/parity.py (relative L1 <= 1e-12, element-wise
    relative L-inf <= 1e-11, zero where the reference is zero); floor =
    (L1, L-inf) of the oracle's roundoff floor, for cases that measure it.
    Returns the relative L1 per variable."""
    f1, fi = floor if floor is not None else (None, None)
    return parity.check(w, gpu, ref, label, f1, fi)[0]


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


def make_sim(amr, w, path="plain"):
    sim = amr.Simulation(w, path=amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN)
    return sim


def run_gpu(amr, w, nsteps, path="plain", graph=False):
    print("GPU run %s nsteps=%d path=%s graph=%s nblocks=%d" % (w.name, nsteps, path, graph, w.nblocks), flush=True)
    sim = make_sim(amr, w, path)
    sim.advance(nsteps, graph=graph)
    fl = sim.sync_flags()
    out = sim.cons()
    sim.close()
    return out, fl


# ---------------------------------------------------------------------------


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("case", ["2d", "3d", "amr2d", "amr3d", "walls"])
def test_uniform_state_bit_identical(amr, case, path):
    wv = [1.3, 0.4, -0.25, 0.15, 0.8, 0.6, -0.9, 0.3, 0.0]
    if case == "2d":
        w = inputs.uniform_state(2, (3, 2), wv)
    elif case == "3d":
        w = inputs.uniform_state(3, (2, 2, 2), wv)
    elif case.startswith("amr"):
        nd = 2 if case == "amr2d" else 3
        base, level, ijk = inputs.amr_test_hierarchy(nd, nb1=4 if nd == 2 else 2, seed=11)
        w = inputs.uniform_state(nd, base, wv, level=level, ijk=ijk)
        w.base_blocks = base
    else:
        wv = [1.3, 0.4, 0.0, 0.15, 0.8, 0.6, 0.0, 0.3, 0.0]
        w = inputs.uniform_state(3, (2, 2, 2), wv, bc_lo=(3, 2, 1), bc_hi=(1, 2, 1))
        w.bc_fixed_prim = np.zeros((3, 2, NV))
        w.bc_fixed_prim[0, 0] = wv
    w.nstages = 3
    sim = make_sim(amr, w, path)
    u0 = sim.cons()
    sim.advance(4)
    sim.sync_flags()
    u1 = sim.cons()
    sim.close()
    assert np.array_equal(u0, u1)


@pytest.mark.parametrize("ndim", [2, 3])
def test_ghost_fill_matches_oracle(amr, orc, ndim):
    """Face ghost slabs after a fill (same-level copies, periodic wrap,
    restriction, prolongation and all physical boundary kinds) agree with
    the oracle's definition cell by cell."""
    base, level, ijk = inputs.amr_test_hierarchy(ndim, nb1=4 if ndim == 2 else 2, seed=13, periodic=False)
    r = np.random.Generator(np.random.PCG64(5))
    prim = r.uniform(0.5, 1.5, size=(len(level), NV) + (16,) * ndim)
    bc_lo, bc_hi = (3, 2, 1), (1, 2, 2)
    w = inputs.Workload("ghosts", ndim, 16, base, (0, 0, 0), (1, 1, 1), bc_lo, bc_hi, level, ijk, prim)
    w.bc_fixed_prim = np.zeros((3, 2, NV))
    w.bc_fixed_prim[0, 0] = [1.0, 2.0, 0, 0, 1.0, 1.0, 0, 0, 0]
    sim = make_sim(amr, w)
    sim.fill(0)
    gp = sim.padded(0)
    sim.close()
    o = orc.OracleSim(w)
    op = o.padded()
    used = np.isfinite(op)
    assert used.sum() > 0
    np.testing.assert_allclose(gp[used], op[used], rtol=2e-15, atol=1e-15)


@pytest.mark.parametrize("make", ["ot", "amr3d", "sheet"])
def test_cfl_matches_oracle(amr, orc, make):
    if make == "ot":
        w = inputs.orszag_tang_2d()
    elif make == "amr3d":
        w = inputs.smooth_amr_state(3, nb1=2, seed=7)
    else:
        w = inputs.current_sheet(n=32)
    sim = make_sim(amr, w)
    sim.cfl(0)
    dt, ch, kappa = sim.scalars()
    sim.close()
    odt, och, okap, fl = orc.OracleSim(w).cfl()
    assert fl == 0
    for a, b in [(dt, odt), (ch, och), (kappa, okap)]:
        assert a == pytest.approx(b, rel=1e-14)


@pytest.mark.parametrize("path", PATHS)
def test_parity_orszag_tang_2d(amr, orc, path):
    """2D 64^2 Orszag-Tang type vortex, SSPRK(2,2), CFL 0.8, 100 steps."""
    w = inputs.orszag_tang_2d()
    ref, diag = orc.run(w)
    gpu, fl = run_gpu(amr, w, w.nsteps, path)
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label="orszag_tang")


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("ndim,nsteps", [(2, 20), (3, 4)])
def test_parity_smooth_amr(amr, orc, ndim, nsteps, path):
    w = inputs.smooth_amr_state(ndim, nb1=4 if ndim == 2 else 2, seed=5 if ndim == 2 else 7)
    ref, _ = orc.run(w, nsteps)
    gpu, fl = run_gpu(amr, w, nsteps, path)
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label="smooth_amr_%dd" % ndim)


@pytest.mark.parametrize("path", PATHS)
def test_parity_small_shock_cloud(amr, orc, path):
    """Fixed inflow + zero-gradient faces on a 3-level hierarchy (32^3 base)."""
    w = inputs.shock_cloud_amr(nsteps=6, base_n=32)
    ref, _ = orc.run(w)
    gpu, fl = run_gpu(amr, w, w.nsteps, path)
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label="shock_cloud_32")


@pytest.mark.parametrize("path", PATHS)
def test_parity_small_current_sheet(amr, orc, path):
    """Reflective y walls, periodic x/z, beta = 0.01 (32^3)."""
    ref, f1, fi = parity.oracle_floor(orc, lambda: inputs.current_sheet(n=32, nsteps=10))
    w = inputs.current_sheet(n=32, nsteps=10)
    gpu, fl = run_gpu(amr, w, w.nsteps, path)
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label="current_sheet_32", floor=(f1, fi))


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("nstages", [2, 3])
def test_graph_and_eager_bitwise_equal(amr, nstages, path):
    w = inputs.random_modes(32, 3, seed=9)
    outs = []
    for graph in (False, True, True):
        sim = make_sim(amr, w, path)
        sim.advance(3, nstages=nstages, graph=graph)
        sim.sync_flags()
        outs.append(sim.cons())
        sim.close()
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[1], outs[2])


def test_graph_replays_between_eager_work(amr):
    """Replays of the captured step interleaved with eager calls and host
    synchronisation give the eager result every time."""
    w = inputs.random_modes(32, 3, seed=10)
    ref_sim = make_sim(amr, w)
    sim = make_sim(amr, w)
    for rep in range(3):
        ref_sim.advance(1, graph=False)
        sim.advance(1, graph=True)
        sim.cfl(0)           # eager work between replays
        sim.synchronize()
        assert np.array_equal(sim.cons(), ref_sim.cons()), rep
    ref_sim.close()
    sim.close()


def test_small_value_flag_and_fix(amr, orc):
    wv = [1.3, 0.4, -0.25, 0.15, 0.8, 0.6, -0.9, 0.3, 0.0]
    w = inputs.uniform_state(2, (2, 2), wv)
    w.prim[1, PR, 3, 4] = -0.1
    sim = make_sim(amr, w)
    sim.advance(1, nstages=2)
    fl, nfix, dt, rc = sim.sync_flags(raise_on_error=False)
    sim.close()
    assert rc == amr.E_NONPHYSICAL and fl & amr.FLAG_SMALL_P
    w.fix_small_values = 1
    w.small_pressure = 1e-6
    w.small_density = 1e-6
    w.nstages = 2
    sim = make_sim(amr, w)
    sim.advance(1)
    fl, nfix, dt, rc = sim.sync_flags(raise_on_error=False)
    gpu = sim.cons()
    sim.close()
    assert rc == 0 and fl & amr.FLAG_SMALL_P
    o = orc.OracleSim(w)
    o.steps(1)
    assert nfix == o.fix_count()
    assert_parity(w, gpu, o.cons(), label="fixed")


def fallback_state():
    """Random modes 32^3 with negative pressure in a few cells (fix off): every
    face of such a cell reconstructs a non-positive p and drops to first order
    in all variables, while the smooth rho, v, B around it have nonzero slopes.
    The cells sit inside blocks, on low and high block faces in x, y and z, and
    in monotone pairs along x and z (so that a neighbour's slope is nonzero
    too).  Without the fallback the oracle's result moves by 1e-6 .. 1e-3
    relative L1 on this state."""
    w = inputs.random_modes(32, 3, seed=31)
    bad = [(0, 5, 6, 7), (1, 0, 8, 8), (2, 8, 15, 3), (3, 7, 7, 0), (4, 15, 0, 15),
           (5, 6, 6, 6), (5, 6, 6, 7), (6, 9, 6, 6), (6, 10, 6, 6)]
    for b, k, j, i in bad:
        w.prim[b, PR, k, j, i] = -1e-3
    w.prim[5, PR, 6, 6, 6] = -0.5e-3
    w.prim[6, PR, 9, 6, 6] = -0.5e-3
    return w


@pytest.mark.parametrize("path", PATHS)
def test_parity_first_order_fallback(amr, orc, path):
    w = fallback_state()
    ref, diag = orc.run(w, 1, check=False)
    assert diag[0, 3] != 0  # the oracle flags the state too
    sim = make_sim(amr, w, path)
    sim.advance(1, nstages=3)
    fl, nfix, _, rc = sim.sync_flags(raise_on_error=False)
    gpu = sim.cons()
    sim.close()
    assert rc == amr.E_NONPHYSICAL and fl & amr.FLAG_SMALL_P
    assert_parity(w, gpu, ref, label="fallback_%s" % path)


def test_fallback_mixed_precision(amr, orc):
    """The FP32 faces take the same fallback decisions (the pressures are far
    from zero in FP32), so the mixed path stays within its usual bound."""
    w = fallback_state()
    ref, _ = orc.run(w, 1, check=False)
    sim = amr.Simulation(w, path=amr.PATH_FUSED, precision=amr.FP32_MIXED)
    sim.advance(1, nstages=3)
    fl, nfix, _, rc = sim.sync_flags(raise_on_error=False)
    gpu = sim.cons()
    sim.close()
    assert rc == amr.E_NONPHYSICAL and fl & amr.FLAG_SMALL_P
    err = rel_l1(w, gpu, ref)
    assert err[RHO] < 1e-6 and err[PR] < 1e-6, err


# ---------------------------------------------------------------------------
# full-size workloads, one step, in the configuration the benchmark times


@pytest.mark.parametrize("path", PATHS)
def test_parity_full_random_modes_256(amr, orc, path):
    w = inputs.random_modes(256, 3, seed=1)
    ref, diag = orc.run(w, 1)
    gpu, fl = run_gpu(amr, w, 1, path, graph=True)
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label="random_modes_256")


@pytest.mark.parametrize("path", PATHS)
def test_parity_full_shock_cloud_amr(amr, orc, path):
    w = inputs.shock_cloud_amr(nsteps=1)
    ref, diag = orc.run(w, 1)
    gpu, fl = run_gpu(amr, w, 1, path, graph=True)
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label="shock_cloud_amr")


@pytest.mark.parametrize("path", PATHS)
def test_parity_full_current_sheet_192(amr, orc, path):
    w = inputs.current_sheet(n=192)
    ref, diag = orc.run(w, 1)
    gpu, fl = run_gpu(amr, w, 1, path, graph=True)
    assert fl[0] == 0
    assert_parity(w, gpu, ref, label="current_sheet_192")


@pytest.mark.parametrize("ndim", [2, 3])
def test_fused_matches_plain(amr, ndim):
    """The fused stage kernel and the per-kernel path agree to rounding
    (both are also checked against the oracle above)."""
    w = inputs.random_modes(64 if ndim == 2 else 32, ndim, seed=12)
    a, _ = run_gpu(amr, w, 5, "plain")
    b, _ = run_gpu(amr, w, 5, "fused")
    err = rel_l1(w, b, a)
    assert np.all(err[:PSI] < 1e-13), err
