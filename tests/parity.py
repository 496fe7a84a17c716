"""FP64 parity measures and bars shared by the GPU tests.

Per conserved variable q, over leaf interior cells:
  relative L1    = sum_i V_i |a_i - b_i| / sum_i V_i |b_i|   (V_i the cell volume)
  relative L-inf = max_i |a_i - b_i| / max_i |b_i|           (element-wise)

Bars (FP64): relative L1 <= 1e-12 and relative L-inf <= 1e-11 for every
variable.  A case whose oracle is itself sensitive to roundoff beyond that is
measured against the oracle's roundoff floor, the larger of two samples of
how far roundoff alone moves the oracle's result: (a) the oracle on the same
input with every nonzero value raised by one ulp, (b) the oracle's source
built with multiply-add contraction, which rounds every a*b+c once instead of
twice (the kind of difference a GPU build has at every operation).  Where
that floor exceeds a bar, the GPU may differ by at most twice the floor; the
variables for which that happened are printed and reported with the case.
Variables that are identically zero in the reference must be exactly zero.
"""
import json
import os

import numpy as np

NV = 9
NAMES = ["rho", "m_x", "m_y", "m_z", "e", "B_x", "B_y", "B_z", "psi"]
L1_BAR = 1e-12
LINF_BAR = 1e-11


def vol_weights(w):
    v = np.ones(w.nblocks)
    for d in range(w.ndim):
        v = v * (w.xmax[d] - w.xmin[d]) / (w.base_blocks[d] * w.nx * 2.0 ** (w.level - 1))
    return v.reshape((-1,) + (1,) * w.ndim)


def rel_l1(w, a, b):
    v = vol_weights(w)
    out = np.zeros(NV)
    for q in range(NV):
        num = np.sum(v * np.abs(a[:, q] - b[:, q]))
        den = np.sum(v * np.abs(b[:, q]))
        out[q] = num / den if den > 0 else (0.0 if num == 0 else np.inf)
    return out


def rel_linf(a, b):
    out = np.zeros(NV)
    for q in range(NV):
        num = np.max(np.abs(a[:, q] - b[:, q]))
        den = np.max(np.abs(b[:, q]))
        out[q] = num / den if den > 0 else (0.0 if num == 0 else np.inf)
    return out


def raise_one_ulp(prim):
    """Every nonzero value raised by one ulp (zeros stay zero)."""
    return np.where(prim != 0.0, np.nextafter(prim, np.inf), prim)


def oracle_floor(orc, make, nsteps=None):
    """(reference, floor L1, floor L-inf) of the case make() builds: the
    larger, per variable, of the one-ulp and the contracted-build samples."""
    w = make()
    n = w.nsteps if nsteps is None else nsteps
    ref, _ = orc.run(w, n)
    wp = make()
    wp.prim = raise_one_ulp(np.asarray(wp.prim))
    pert, _ = orc.run(wp, n)
    fma, _ = orc.run(make(), n, fma=True)
    f1 = np.maximum(rel_l1(w, pert, ref), rel_l1(w, fma, ref))
    fi = np.maximum(rel_linf(pert, ref), rel_linf(fma, ref))
    return ref, f1, fi


def oracle_progress(orc, w, nsteps=None, fma=False, chunk=5, label=""):
    """The oracle's conserved state after nsteps (default w.nsteps), advanced
    in runs of chunk steps on one simulation (the same steps as one run),
    printing a line after each run: the full-size grids take minutes."""
    n = w.nsteps if nsteps is None else nsteps
    sim = orc.OracleSim(w, None, fma=fma)
    try:
        done = 0
        while done < n:
            k = min(chunk, n - done)
            sim.steps(k)
            done += k
            print("oracle%s %s: %d/%d steps" % (" (contracted)" if fma else "", label, done, n), flush=True)
        return sim.cons()
    finally:
        sim.close()


def over_fixed_bars(w, gpu, ref):
    """True when some variable misses a fixed bar (so the oracle's roundoff
    floor decides whether the case passes)."""
    e1, ei = rel_l1(w, gpu, ref), rel_linf(gpu, ref)
    return bool(np.any(e1 > L1_BAR) or np.any(ei > LINF_BAR))


def floor_progress(orc, make, ref, label, chunk=5):
    """(floor L1, floor L-inf) as in oracle_floor, for a reference already
    computed, with the oracle runs reporting progress."""
    w = make()
    wp = make()
    wp.prim = raise_one_ulp(np.asarray(wp.prim))
    pert = oracle_progress(orc, wp, chunk=chunk, label=label + " +1 ulp")
    fma = oracle_progress(orc, make(), fma=True, chunk=chunk, label=label)
    f1 = np.maximum(rel_l1(w, pert, ref), rel_l1(w, fma, ref))
    fi = np.maximum(rel_linf(pert, ref), rel_linf(fma, ref))
    return f1, fi


def bars(floor_l1=None, floor_linf=None):
    """Per-variable (L1, L-inf) bars and the variables whose bar was raised to
    twice the oracle's floor."""
    b1 = np.full(NV, L1_BAR)
    bi = np.full(NV, LINF_BAR)
    raised = []
    for q in range(NV):
        up = False
        if floor_l1 is not None and 2.0 * floor_l1[q] > L1_BAR and floor_l1[q] > L1_BAR:
            b1[q] = 2.0 * floor_l1[q]
            up = True
        if floor_linf is not None and floor_linf[q] > LINF_BAR:
            bi[q] = 2.0 * floor_linf[q]
            up = True
        if up:
            raised.append(NAMES[q])
    return b1, bi, raised


def check(w, gpu, ref, label, floor_l1=None, floor_linf=None):
    """Assert the bars (raised to twice the oracle's floor where that floor
    exceeds them); returns (L1, L-inf)."""
    assert np.all(np.isfinite(gpu)), label
    e1, ei = rel_l1(w, gpu, ref), rel_linf(gpu, ref)
    b1, bi, raised = bars(floor_l1, floor_linf)
    rec = {"case": label, "rel_l1": [float(x) for x in e1], "rel_linf": [float(x) for x in ei],
           "max_rel_l1": float(np.max(e1)), "max_rel_linf": float(np.max(ei)), "raised_to_2x_floor": raised}
    if floor_l1 is not None:
        rec["floor_l1"] = [float(x) for x in floor_l1]
        rec["floor_linf"] = [float(x) for x in floor_linf]
    print("%s rel-L1 %s | rel-Linf %s" % (label, " ".join("%.1e" % x for x in e1), " ".join("%.1e" % x for x in ei)),
          flush=True)
    if floor_l1 is not None:
        print("%s oracle floor L1 %s | Linf %s%s" % (label, " ".join("%.1e" % x for x in floor_l1),
                                                    " ".join("%.1e" % x for x in floor_linf),
                                                    ("; bars at 2x floor: " + ",".join(raised)) if raised else ""),
              flush=True)
    report = os.environ.get("AMRVAC_PARITY_REPORT")
    if report:
        with open(report, "a") as f:
            f.write(json.dumps(rec) + "\n")
    bad = []
    for q in range(NV):
        if np.all(ref[:, q] == 0):
            if not np.all(gpu[:, q] == 0):
                bad.append((NAMES[q], "not zero"))
            continue
        if not (e1[q] <= b1[q] and ei[q] <= bi[q]):
            bad.append((NAMES[q], float(e1[q]), float(b1[q]), float(ei[q]), float(bi[q])))
    assert not bad, (label, bad)
    return e1, ei
