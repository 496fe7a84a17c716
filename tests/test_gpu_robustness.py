"""Race and failure checks of the device path: ghost cells that no kernel
should read are poisoned with NaN (an unfilled or stale ghost read shows up
as a NaN or a changed result), runs repeat bit for bit, a run resumed from a
copied state equals the uninterrupted run, and non-physical states are
reported through the flag word."""
import numpy as np
import pytest

from paper_2303_03026_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


def poison_ghosts(sim):
    """Set every ghost cell of every slot to NaN (FP64 slots)."""
    torch = sim.torch
    nx, ng, nd = sim.w.nx, sim.w.ng, sim.w.ndim
    pn = nx + 2 * ng
    for k in range(len(sim.slots)):
        a = sim.padded_view(k)
        mask = torch.ones((pn,) * nd, dtype=torch.bool, device=a.device)
        inner = (slice(ng, ng + nx),) * nd
        mask[inner] = False
        a[:, :, mask] = float("nan")
    torch.cuda.synchronize()


CASES = [("random_modes_3d_48", lambda: inputs.random_modes(48, 3, seed=11)),
         ("current_sheet_48", lambda: inputs.current_sheet(48, nsteps=3)),
         ("smooth_amr_3d", lambda: inputs.smooth_amr_state(3, nb1=2, seed=12)),
         ("smooth_amr_2d", lambda: inputs.smooth_amr_state(2, nb1=4, seed=13)),
         ("shock_cloud_small", lambda: inputs.shock_cloud_amr(base_n=32, nsteps=3))]


@pytest.mark.parametrize("path", ["fused", "plain"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_poisoned_ghosts_are_never_read_unfilled(amr, name, make, path):
    w = make()
    p = amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN
    ref_sim = amr.Simulation(w, path=p)
    ref_sim.advance(3, nstages=3)
    ref = ref_sim.cons()
    ref_sim.close()
    sim = amr.Simulation(w, path=p)
    poison_ghosts(sim)
    sim.advance(3, nstages=3)
    fl, nfix, _, rc = sim.sync_flags(raise_on_error=False)
    got = sim.cons()
    sim.close()
    assert rc == 0 and fl == 0, (name, path, fl)
    assert np.all(np.isfinite(got)), (name, path)
    assert np.array_equal(got, ref), (name, path)


@pytest.mark.parametrize("precision", [0, 1])
def test_runs_repeat_bit_for_bit(amr, precision):
    w = inputs.shock_cloud_amr(base_n=32, nsteps=4)
    outs = []
    for _ in range(2):
        sim = amr.Simulation(w, path=amr.PATH_FUSED, precision=precision)
        sim.advance(4, nstages=3, graph=True)
        sim.sync_flags()
        outs.append(sim.cons())
        sim.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("precision", [0, 1])
def test_resume_from_copied_state(amr, precision):
    w = inputs.smooth_amr_state(3, nb1=2, seed=14)
    full = amr.Simulation(w, path=amr.PATH_FUSED, precision=precision)
    full.advance(5, nstages=3)
    ref = full.cons()
    full.close()
    first = amr.Simulation(w, path=amr.PATH_FUSED, precision=precision)
    first.advance(2, nstages=3)
    first.synchronize()
    saved = first.slots[0].clone()  # the whole state slot (the checkpoint)
    first.close()
    resumed = amr.Simulation(w, path=amr.PATH_FUSED, precision=precision, set_initial=False)
    resumed.slots[0].copy_(saved)
    resumed.torch.cuda.synchronize()
    resumed.advance(3, nstages=3)
    got = resumed.cons()
    resumed.close()
    assert np.array_equal(got, ref)


def test_nan_state_reports_bad_dt(amr):
    w = inputs.random_modes(32, 3, seed=15)
    w.prim[3, 0, 5, 6, 7] = np.nan
    sim = amr.Simulation(w, path=amr.PATH_FUSED)
    sim.cfl(0)
    fl, nfix, dt, rc = sim.sync_flags(raise_on_error=False)
    assert rc == amr.E_NONPHYSICAL and fl & amr.FLAG_BAD_DT
    with pytest.raises(amr.AmrvacError):
        sim.sync_flags()
    sim.close()


@pytest.mark.parametrize("path", ["fused", "plain"])
def test_negative_pressure_stops_or_is_fixed(amr, path):
    p = amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN
    w = inputs.random_modes(32, 3, seed=16)
    w.prim[1, 4, 3, 4, 5] = -1e-3
    sim = amr.Simulation(w, path=p)
    sim.advance(1, nstages=3)
    fl, nfix, _, rc = sim.sync_flags(raise_on_error=False)
    sim.close()
    assert rc == amr.E_NONPHYSICAL and fl & amr.FLAG_SMALL_P
    w.fix_small_values, w.small_pressure, w.small_density = 1, 1e-10, 1e-10
    sim = amr.Simulation(w, path=p)
    sim.advance(1, nstages=3)
    fl, nfix, _, rc = sim.sync_flags(raise_on_error=False)
    sim.close()
    assert rc == 0 and fl & amr.FLAG_SMALL_P and nfix > 0
