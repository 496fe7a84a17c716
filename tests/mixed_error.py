"""Error measures of the FP32-mixed path against the FP64 oracle.

Per conserved variable q, volume-weighted over leaf interior cells:
  relative L1     = L1(gpu_q - ref_q) / L1(ref_q)
  relative L-inf  = max |gpu_q - ref_q| / max |ref_q|
For a variable that is identically zero in the initial state (psi always,
and e.g. the transverse momentum and field of a planar shock), the
denominators use the magnitude of its vector instead, |m| for a momentum
component and |B| for a field component and for psi: such a component
carries no scale of its own, and what FP32 storage costs is measured
against the field it grows out of.
"""
import numpy as np

NV = 9
NAMES = ["rho", "m_x", "m_y", "m_z", "e", "B_x", "B_y", "B_z", "psi"]


def volumes(w):
    v = np.ones(w.nblocks)
    for d in range(w.ndim):
        v = v * (w.xmax[d] - w.xmin[d]) / (w.base_blocks[d] * w.nx * 2.0 ** (w.level - 1))
    return v.reshape((-1,) + (1,) * w.ndim)


def starts_at_zero(w):
    """Variables that are identically zero in w's initial state."""
    p = np.asarray(w.prim)
    z = [False] * NV
    for c in range(3):
        z[1 + c] = not np.any(p[:, 1 + c])  # m = rho v
        z[5 + c] = not np.any(p[:, 5 + c])
    z[8] = not np.any(p[:, 8])
    return z


def errors(w, gpu, ref):
    """(relative L1, relative L-inf) per variable, as defined above."""
    v = volumes(w)
    zero = starts_at_zero(w)
    mmag = np.sqrt(ref[:, 1] ** 2 + ref[:, 2] ** 2 + ref[:, 3] ** 2)
    bmag = np.sqrt(ref[:, 5] ** 2 + ref[:, 6] ** 2 + ref[:, 7] ** 2)
    l1 = np.zeros(NV)
    linf = np.zeros(NV)
    for q in range(NV):
        d = np.abs(gpu[:, q] - ref[:, q])
        if zero[q]:
            s = mmag if 1 <= q <= 3 else bmag
        else:
            s = np.abs(ref[:, q])
        num, den = np.sum(v * d), np.sum(v * s)
        l1[q] = num / den if den > 0 else (0.0 if num == 0 else np.inf)
        mx = np.max(s)
        linf[q] = np.max(d) / mx if mx > 0 else (0.0 if np.max(d) == 0 else np.inf)
    return l1, linf


def check(label, l1, linf, bound_l1, bound_linf):
    """Assert both bounds (scalars or per-variable arrays) and print the
    measured values."""
    print("%s mixed rel-L1 %s | rel-Linf %s" % (label, " ".join("%.1e" % e for e in l1),
                                               " ".join("%.1e" % e for e in linf)), flush=True)
    bl1 = np.broadcast_to(np.asarray(bound_l1, dtype=float), (NV,))
    bli = np.broadcast_to(np.asarray(bound_linf, dtype=float), (NV,))
    bad = [(NAMES[q], float(l1[q]), float(bl1[q]), float(linf[q]), float(bli[q])) for q in range(NV)
           if not (l1[q] <= bl1[q] and linf[q] <= bli[q])]
    assert not bad, (label, bad)
