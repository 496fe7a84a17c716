"""FP32-mixed path (FP32 storage and face arithmetic; FP64 energy, pressure
recovery, small-value fix and CFL) against the FP64 CPU oracle.

There is no bitwise pin for FP32 arithmetic; each case states a bound per
conserved variable on the relative L1 error and on the element-wise relative
L-inf error (tests/mixed_error.py: plain relative errors, except for a
variable identically zero at the start, which is measured against the
magnitude of its vector).  The bounds are about three times the values
measured on MI355X, rounded up:

  random modes 64^3, 50 steps (the benchmark's field)     L1 5e-7, L-inf 1e-6
  current sheet 48^3, 200 steps (beta = 0.01)             L1 1e-6, L-inf 1e-5,
      momentum m_x, m_z 1.5e-3 / 2e-3 and m_y 2e-5 / 2e-5 (measured 5.0e-4,
      1.1e-4, 4.2e-6): the momentum (|v| ~ 5e-3) is driven by differences of
      the total pressure 0.505, whose FP32 rounding is 3e-8 at every face
  current sheet 192^3, 1 step                             L1 1e-7, L-inf 5e-7,
      momentum 1.5e-5 / 4e-5
  shock cloud 32^3 base, 3 levels, 100 steps              L1 5e-7, L-inf 2e-6
  the full grids at their stated lengths (AMRVAC_FULL_LENGTH=1; the oracle
  takes minutes per case):
    random modes 256^3, 50 steps                          L1 1e-6, L-inf 2e-6
      (measured 3.2e-7 m_x, 6.1e-7 rho)
    shock cloud 128^3 base, 100 steps                     L1 5e-7, L-inf 2e-6
      (measured 1.5e-7, 7.0e-7)
    current sheet 192^3, 200 steps                        L1 1.5e-6, L-inf 1e-5,
      m_x, m_z 2e-3 / 3e-3, m_y 2e-4 / 1.5e-4 (measured m_x 6.1e-4 / 8.9e-4,
      m_y 6.7e-5 / 4.5e-5, m_z 1.7e-4 / 3.1e-4, rho 4.6e-7 / 3.6e-6)
  smooth AMR 3D, 4 steps                                  L1 5e-7, L-inf 2e-6,
      psi 2e-5 / 2e-4 (psi ~ 0.01 |B|: its FP32 error is that of B)
  Alfven shock-cloud, 3 levels, koren + HLLD, 30 steps   L1 5e-7, L-inf 2e-6
  Kelvin-Helmholtz, 3 levels, van Leer + HLLC, 30 steps   L1 5e-7, L-inf 3e-6,
      m_y 3e-4 / 5e-4 (the 1e-3 noise and the growing mode)
"""
import os

import numpy as np
import pytest

from paper_2303_03026_amd import inputs
import mixed_error
import parity

pytestmark = pytest.mark.gpu

NV = 9
NAMES = mixed_error.NAMES


def per_var(default, **over):
    b = np.full(NV, float(default))
    for k, v in over.items():
        b[NAMES.index(k)] = v
    return b


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    return amrvac


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


def run_mixed(amr, w, nsteps):
    sim = amr.Simulation(w, precision=amr.FP32_MIXED)
    sim.advance(nsteps, graph=True)
    fl = sim.sync_flags()
    out = sim.cons()
    sim.close()
    return out, fl


def test_mixed_uniform_state_bit_identical(amr):
    wv = [1.3, 0.4, -0.25, 0.15, 0.8, 0.6, -0.9, 0.3, 0.0]
    for w in (inputs.uniform_state(3, (2, 2, 2), wv), inputs.uniform_state(2, (3, 2), wv)):
        sim = amr.Simulation(w, precision=amr.FP32_MIXED)
        u0 = sim.cons()
        sim.advance(3)
        sim.sync_flags()
        assert np.array_equal(sim.cons(), u0)
        sim.close()


def mixed_case(amr, orc, w, label, b1, bi, nsteps=None):
    n = w.nsteps if nsteps is None else nsteps
    ref, _ = orc.run(w, n)
    gpu, fl = run_mixed(amr, w, n)
    assert fl[0] == 0
    l1, linf = mixed_error.errors(w, gpu, ref)
    mixed_error.check(label, l1, linf, b1, bi)


def test_mixed_random_modes(amr, orc):
    mixed_case(amr, orc, inputs.random_modes(64, 3, seed=7, nsteps=50), "random_modes_64_x50", 5e-7, 1e-6)


def test_mixed_current_sheet(amr, orc):
    """beta = 0.01: the pressure is 1% of the energy; FP64 energy and
    pressure recovery keep FP32 storage usable."""
    mixed_case(amr, orc, inputs.current_sheet(n=48, nsteps=200), "current_sheet_48_x200",
               per_var(1e-6, m_x=1.5e-3, m_y=2e-5, m_z=1.5e-3), per_var(1e-5, m_x=2e-3, m_y=2e-5, m_z=2e-3))


def test_mixed_full_current_sheet_one_step(amr, orc):
    mixed_case(amr, orc, inputs.current_sheet(n=192), "current_sheet_192_x1",
               per_var(1e-7, m_x=1.5e-5, m_y=1.5e-5, m_z=1.5e-5), per_var(5e-7, m_x=4e-5, m_y=4e-5, m_z=4e-5),
               nsteps=1)


def test_mixed_shock_cloud(amr, orc):
    mixed_case(amr, orc, inputs.shock_cloud_amr(base_n=32, nsteps=100), "shock_cloud_32_x100", 5e-7, 2e-6)


def test_mixed_amr(amr, orc):
    mixed_case(amr, orc, inputs.smooth_amr_state(3, nb1=2, seed=7), "smooth_amr_3d_x4",
               per_var(5e-7, psi=2e-5), per_var(2e-6, psi=2e-4), nsteps=4)


def test_mixed_alfven_shock_cloud(amr, orc):
    """The paper's MHD shock-cloud test (3 levels, koren + HLLD, 30 steps):
    a strong intermediate shock and a density contrast of 129 in FP32
    storage."""
    mixed_case(amr, orc, inputs.alfven_shock_cloud(max_level=3, flux=1, nsteps=30), "alfven_shock_cloud_l3_x30",
               5e-7, 2e-6)


def test_mixed_kelvin_helmholtz(amr, orc):
    """The shear layer (3 levels, van Leer + HLLC, 30 steps; B = 0, so the
    field rows are exactly zero on both sides)."""
    mixed_case(amr, orc, inputs.kelvin_helmholtz(max_level=3, limiter=0, flux=2, nsteps=30),
               "kelvin_helmholtz_l3_x30", per_var(5e-7, m_y=3e-4), per_var(3e-6, m_y=5e-4))


FULL = {
    "random_modes_256_x50": (lambda: inputs.random_modes(256, 3, seed=1, nsteps=50), 1e-6, 2e-6),
    "shock_cloud_128_x100": (lambda: inputs.shock_cloud_amr(nsteps=100), 5e-7, 2e-6),
    "current_sheet_192_x200": (lambda: inputs.current_sheet(192, nsteps=200),
                               per_var(1.5e-6, m_x=2e-3, m_y=2e-4, m_z=2e-3),
                               per_var(1e-5, m_x=3e-3, m_y=1.5e-4, m_z=3e-3)),
}


@pytest.mark.skipif(os.environ.get("AMRVAC_FULL_LENGTH") != "1",
                    reason="full-size run at the stated length: the oracle takes minutes (AMRVAC_FULL_LENGTH=1)")
@pytest.mark.parametrize("name", list(FULL))
def test_mixed_full_size_at_stated_length(amr, orc, name):
    make, b1, bi = FULL[name]
    w = make()
    ref = parity.oracle_progress(orc, w, chunk=10, label=name)
    gpu, fl = run_mixed(amr, make(), w.nsteps)
    assert fl[0] == 0
    l1, li = mixed_error.errors(w, gpu, ref)
    mixed_error.check(name, l1, li, b1, bi)
