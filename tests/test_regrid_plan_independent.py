"""An independent leaf-set planner, written from the regrid reading of the
block AMR in the paper's "Open source strategy" section (refinement ratio 2):
refine the flagged blocks (below the level cap), restore 2:1 nesting across
faces, edges and corners by refining, then merge complete sibling sets of
flagged old leaves wherever the parent would not touch a leaf two levels
finer, repeating until nothing merges.

It works on a dense map of the finest level: every finest block position
holds the level of the leaf covering it.  Two leaves touch exactly when two
of their finest positions are neighbours (diagonals included), so nesting is
a condition on neighbouring map entries, checked with shifted copies of the
map (periodic wrap, or no neighbour outside a non-periodic side).  Nothing
here shares code with the library's planner (a hash set of leaf keys walked
by tree lookups); the two must give the same leaf set on random flags."""
import itertools

import numpy as np
import pytest

from paper_2303_03026_amd import inputs


@pytest.fixture(scope="module")
def amr():
    from paper_2303_03026_amd import amrvac
    amrvac.load_library()
    return amrvac


class LevelMap:
    def __init__(self, ndim, base, periodic, top):
        self.nd, self.top = ndim, top
        self.periodic = [bool(periodic[d]) for d in range(ndim)]
        self.shape = tuple(int(base[d]) << (top - 1) for d in range(ndim))
        self.L = np.zeros(self.shape[::-1], dtype=np.int64)  # array axes [z,] y, x

    def region(self, l, pos):
        """Index of the finest positions under block pos of level l."""
        s = 1 << (self.top - l)
        return tuple(slice(int(pos[d]) * s, (int(pos[d]) + 1) * s) for d in range(self.nd))[::-1]

    def put(self, l, pos):
        self.L[self.region(l, pos)] = l

    def leaves(self):
        out = set()
        for idx in itertools.product(*[range(n) for n in self.shape]):
            l = int(self.L[idx[::-1]])
            p = [idx[d] >> (self.top - l) for d in range(self.nd)] + [0] * (3 - self.nd)
            out.add((l,) + tuple(p))
        return out

    def neighbour_max(self, L):
        """Largest level among the 3^d - 1 neighbours of every position
        (0 where a neighbour lies outside a non-periodic side)."""
        best = np.zeros_like(L)
        for off in itertools.product((-1, 0, 1), repeat=self.nd):
            if not any(off):
                continue
            sh = L
            for d, o in enumerate(off):
                if o == 0:
                    continue
                ax = self.nd - 1 - d
                sh = np.roll(sh, o, axis=ax)
                if not self.periodic[d]:  # the rolled-in edge has no neighbour
                    sl = [slice(None)] * self.nd
                    sl[ax] = 0 if o > 0 else -1
                    sh = sh.copy()
                    sh[tuple(sl)] = 0
            best = np.maximum(best, sh)
        return best


def independent_plan(ndim, base, periodic, level, ijk, flags, max_level):
    cap = min(max(max_level, 1), 12)
    top = max(int(level.max()) + 1, 1)
    m = LevelMap(ndim, base, periodic, top)
    old = {}
    for b, (l, p) in enumerate(zip(level, ijk)):
        m.put(int(l), p[:ndim])
        old[(int(l),) + tuple(int(x) for x in p[:ndim])] = int(flags[b])
    # 1. refine flagged leaves below the cap
    for (l, *p), f in old.items():
        if f > 0 and l < cap:
            m.L[m.region(l, p)] = l + 1
    # 2. restore 2:1 nesting: a position whose neighbour is two or more
    # levels finer gets its whole leaf refined, until none is left
    while True:
        bad = m.neighbour_max(m.L) - m.L >= 2
        if not bad.any():
            break
        for idx in zip(*np.nonzero(bad)):
            l = int(m.L[idx])
            if l == 0 or not bad[idx]:
                continue
            p = [idx[::-1][d] >> (top - l) for d in range(ndim)]
            reg = m.region(l, p)
            if np.all(m.L[reg] == l):  # still that leaf
                m.L[reg] = l + 1
                bad[reg] = False
    # 3. merge complete flagged sibling sets while nesting allows
    parents = set()
    for (l, *p), f in old.items():
        if f < 0 and l > 1:
            parents.add((l - 1,) + tuple(x >> 1 for x in p))
    changed = True
    while changed:
        changed = False
        for par in sorted(parents):
            lp, pp = par[0], par[1:]
            kids = [(lp + 1,) + tuple(2 * pp[d] + c[d] for d in range(ndim))
                    for c in itertools.product((0, 1), repeat=ndim)]
            reg = m.region(lp, pp)
            if not all(old.get(k, 0) < 0 and k in old for k in kids) or not np.all(m.L[reg] == lp + 1):
                parents.discard(par)
                changed = True
                break
            # would the parent touch a leaf of level lp + 2 or finer?
            trial = m.L.copy()
            trial[reg] = lp
            near = m.neighbour_max(trial)[reg]
            if np.all(near <= lp + 1):
                m.L = trial
                parents.discard(par)
                changed = True
                break
    out = set()
    for k in m.leaves():
        out.add(k if ndim == 3 else (k[0], k[1], k[2], 0))
    return out


def lib_plan(amr, w, flags, max_level):
    lv, ij = amr.regrid_plan(w, flags, max_level)
    return set((int(l),) + tuple(int(x) for x in p) for l, p in zip(lv, ij))


def hierarchy(ndim, seed, periodic):
    base, level, ijk = inputs.amr_test_hierarchy(ndim, nb1=4 if ndim == 2 else 2, seed=seed, periodic=periodic)
    bc = 0 if periodic else 1
    w = inputs.uniform_state(ndim, base, [1.0, 0, 0, 0, 1.0, 0, 0, 0, 0], level=level, ijk=ijk,
                             bc_lo=(bc,) * 3, bc_hi=(bc,) * 3)
    w.base_blocks = base
    return w


CASES = [(nd, seed, per) for nd in (2, 3) for seed in (5, 8, 13) for per in (True, False)]


@pytest.mark.parametrize("ndim,seed,periodic", CASES)
def test_library_plan_equals_independent_plan(amr, ndim, seed, periodic):
    w = hierarchy(ndim, seed, periodic)
    r = np.random.Generator(np.random.PCG64(1000 + seed))
    for trial in range(6):
        p_ref = [0.05, 0.15, 0.3][trial % 3]
        p_crs = [0.9, 0.6, 0.3][(trial // 3) % 3]
        u = r.random(w.nblocks)
        flags = np.where(u < p_ref, 1, np.where(u > 1.0 - p_crs, -1, 0)).astype(np.int32)
        for max_level in (3, 4):
            got = lib_plan(amr, w, flags, max_level)
            want = independent_plan(ndim, w.base_blocks, (periodic,) * 3, w.level, w.ijk, flags, max_level)
            assert got == want, (ndim, seed, periodic, trial, max_level, len(got ^ want))


def test_independent_plan_on_the_nesting_example():
    """The hand-built case of the library planner's own test: merging P's
    children beside a level-3 set is refused until that set merges too."""
    base = (2, 1, 1)
    leaves = set()
    for a in (0, 1):
        for b in (0, 1):
            leaves.add((2, a, b, 0))
            if (a, b) != (0, 0):
                leaves.add((2, 2 + a, b, 0))
            leaves.add((3, 4 + a, b, 0))
    keys_ = sorted(leaves)
    level = np.array([k[0] for k in keys_])
    ijk = np.array([k[1:] for k in keys_])
    p_kids = np.array([k[0] == 2 and k[1] < 2 for k in keys_])
    got = independent_plan(2, base, (False,) * 3, level, ijk, np.where(p_kids, -1, 0), 12)
    assert got == leaves
    l3 = np.array([k[0] == 3 for k in keys_])
    got = independent_plan(2, base, (False,) * 3, level, ijk, np.where(p_kids | l3, -1, 0), 12)
    assert (1, 0, 0, 0) in got and (2, 2, 0, 0) in got and not any(k[0] == 3 for k in got)
