"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/amrvac.h declares, sizes slots, and rejects invalid
descriptions and block tables before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2303_03026_amd import amrvac, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "amrvac.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(amrvac_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    return amrvac.load_library()


def test_exports_every_declared_symbol(lib):
    syms = header_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(amrvac.ABI_SYMBOLS) == syms


def test_slot_bytes(lib):
    w = inputs.orszag_tang_2d()
    g = amrvac.make_desc(w)
    n = ctypes.c_size_t()
    assert lib.amrvac_slot_bytes(ctypes.byref(g), 16, ctypes.byref(n)) == 0
    # FP64: 16 lead bytes put interior rows on 32-byte sectors
    assert n.value == 16 * 20 * 20 * 72 + amrvac.SLOT_LEAD_FP64 == 16 * 20 * 20 * 72 + 16
    assert amrvac.SLOT_LEAD_FP64 % 32 == 16 and (20 * 8) % 32 == 0
    g.precision = amrvac.FP32_MIXED
    assert lib.amrvac_slot_bytes(ctypes.byref(g), 16, ctypes.byref(n)) == 0
    assert n.value == 16 * 20 * 20 * 40
    # three ghost layers (the five-cell reconstructions) in FP32-mixed too
    g.nghost = 3
    assert lib.amrvac_slot_bytes(ctypes.byref(g), 16, ctypes.byref(n)) == 0
    assert n.value == 16 * 22 * 22 * 40
    # FP32-mixed runs on the fused path only, whose blocks are 16 cells wide
    g.nghost = 2
    g.block_nx = 8
    assert lib.amrvac_slot_bytes(ctypes.byref(g), 16, ctypes.byref(n)) == amrvac.E_ARG


def _init(lib, w, level=None, ijk=None, desc=None):
    g = desc if desc is not None else amrvac.make_desc(w)
    level = np.ascontiguousarray(w.level if level is None else level, dtype=np.int32)
    ijk = np.ascontiguousarray(w.ijk if ijk is None else ijk, dtype=np.int32)
    ctx = ctypes.c_void_p()
    fake = (ctypes.c_void_p * 3)(1, 2, 3)  # never dereferenced: validation fails first
    rc = lib.amrvac_init_blocks(ctypes.byref(ctx), ctypes.byref(g), len(level),
                                level.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), fake, 3, None)
    return rc, lib.amrvac_last_error(None).decode()


def test_rejects_bad_descriptions(lib):
    w = inputs.orszag_tang_2d()
    for field, val in [("ndim", 4), ("nghost", 1), ("block_nx", 7), ("gamma", 1.0)]:
        g = amrvac.make_desc(w)
        setattr(g, field, val)
        rc, msg = _init(lib, w, desc=g)
        assert rc == amrvac.E_ARG, (field, msg)
    # three ghost layers need blocks of at least 6 cells (a coarse ghost
    # layer is restricted from 2 nghost fine cells inside the neighbour)
    g = amrvac.make_desc(w)
    g.nghost, g.block_nx, g.limiter = 3, 4, amrvac.LIM_WENO5
    rc, msg = _init(lib, w, desc=g)
    assert rc == amrvac.E_ARG and "2 nghost" in msg, msg
    g = amrvac.make_desc(w)
    g.bc_lo[0] = amrvac.FP64 + 1  # zero-gradient on one side only of a periodic pair
    rc, msg = _init(lib, w, desc=g)
    assert rc == amrvac.E_ARG and "periodic" in msg


def test_rejects_bad_block_tables(lib):
    w = inputs.orszag_tang_2d()
    # duplicate block
    lev = w.level.copy()
    ijk = w.ijk.copy()
    ijk[1] = ijk[0]
    rc, msg = _init(lib, w, lev, ijk)
    assert rc == amrvac.E_ARG
    # missing block: does not tile
    rc, msg = _init(lib, w, w.level[1:], w.ijk[1:])
    assert rc == amrvac.E_ARG and "tile" in msg
    # overlap: a block and one of its children
    lev2 = np.concatenate([w.level, [2]])
    ijk2 = np.concatenate([w.ijk, [[0, 0, 0]]])
    rc, msg = _init(lib, w, lev2, ijk2)
    assert rc == amrvac.E_ARG
    # level 3 next to level 1: not 2:1 nested
    leaves = {(1, i, j, 0): True for j in range(4) for i in range(4)}
    del leaves[(1, 1, 1, 0)]
    for a in range(2):
        for b in range(2):
            if (a, b) == (0, 0):
                for a2 in range(2):
                    for b2 in range(2):
                        leaves[(3, 4 * 1 + a2, 4 * 1 + b2, 0)] = True
            else:
                leaves[(2, 2 + a, 2 + b, 0)] = True
    keys = sorted(leaves)
    rc, msg = _init(lib, w, np.array([k[0] for k in keys]), np.array([k[1:] for k in keys]))
    assert rc == amrvac.E_ARG and "2:1" in msg
    # and the nested version of the same hierarchy passes validation (fails
    # later only at device allocation, or succeeds on a GPU host)
    nested = inputs.nest_2to1(2, (4, 4, 1), dict(leaves), periodic=(True, True, True))
    keys = sorted(nested)
    rc, msg = _init(lib, w, np.array([k[0] for k in keys]), np.array([k[1:] for k in keys]))
    assert rc != amrvac.E_ARG, msg


def test_workload_hierarchies_are_valid():
    """The AMR generators produce 2:1-nested tilings (checked by the oracle's
    own block-table builder)."""
    from oracle import oracle
    base, level, ijk = inputs.amr_test_hierarchy(3, nb1=2, seed=7)
    w = inputs.uniform_state(3, base, [1, 0, 0, 0, 1, 0, 0, 0, 0], level=level, ijk=ijk)
    w.base_blocks = base
    oracle.OracleSim(w).close()
    vol = np.sum(0.125 ** (level - 1))
    assert vol == pytest.approx(8.0)


def test_shock_cloud_hierarchy_shape():
    w = inputs.shock_cloud_amr(nsteps=1)
    counts = np.bincount(w.level)[1:]
    assert len(counts) == 3
    assert np.sum(counts * 0.125 ** np.arange(3)) == pytest.approx(512.0)
    # uneven per-level counts, level 3 the largest
    assert counts[2] > counts[1] > 0 and counts[0] > 0
