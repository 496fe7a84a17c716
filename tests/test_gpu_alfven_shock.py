"""The paper's 2D MHD shock-cloud test (an intermediate shock running into a
high-contrast density field) on a 3-level hierarchy, with 'koren' and each
of HLL, HLLC and HLLD, on the plain and fused paths, against the oracle."""
import numpy as np
import pytest

from paper_2303_03026_amd import inputs
from test_gpu_parity import assert_parity
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


@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("flux,fname", [(0, "hll"), (2, "hllc"), (1, "hlld")])
def test_parity_with_oracle(amr, orc, flux, fname, path):
    """10 steps, the FP64 bars of tests/parity.py (floors included), except
    psi: B_n is continuous across every face of this planar field but the
    coarse/fine interfaces, so psi is roundoff (|psi| ~ 1e-15 |B|, relative
    errors of order 1); there GPU and oracle must both stay below 1e-12 |B|."""
    def make():
        return inputs.alfven_shock_cloud(max_level=3, flux=flux, nsteps=10)
    w = make()
    print("GPU alfven shock cloud %s path=%s nblocks=%d" % (fname, path, w.nblocks), flush=True)
    ref, f1, fi = parity.oracle_floor(orc, make)
    sim = amr.Simulation(w, path=amr.PATH_FUSED if path == "fused" else amr.PATH_PLAIN)
    sim.advance(w.nsteps, nstages=3)
    assert sim.sync_flags()[0] == 0
    got = sim.cons()
    sim.close()
    bmax = np.abs(ref[:, 5:8]).max()
    if np.abs(ref[:, 8]).max() < 1e-12 * bmax:  # psi is roundoff on both sides
        assert np.abs(got[:, 8]).max() < 1e-12 * bmax
        got, ref = got.copy(), ref.copy()
        got[:, 8] = 0.0
        ref[:, 8] = 0.0
    assert_parity(w, got, ref, label="alfven shock %s %s" % (fname, path), floor=(f1, fi))
