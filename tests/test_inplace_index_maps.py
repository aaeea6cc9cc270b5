"""The in-place (one state buffer) step on the host: an emulation of the index maps of the
two in-place kernels (the pull phase and the local phase) and of the two-buffer step, for
both bounce-back storage conventions, with obstacles and free-slip wall planes (no GPU).

It checks what the kernels rely on:
* race freedom: within a phase, every location is written by at most one thread, and no
  thread reads a location that another thread of the phase writes (so the phase gives the
  same result in any order of its threads);
* with 16-bit storage and two nodes per thread (pairs starting at even x, or one node to
  the right as the pull phase without solids takes them), the obstacle nodes that take
  part in the pull phase (a wave leaves only when all its nodes are solid) read and write
  only locations that no fluid node reads or writes in that phase;
* two in-place phases give exactly the populations of two two-buffer steps: every value
  any later pull reads is the same, with a collision stand-in that mixes all populations
  of a node (index maps only; the node arithmetic is shared code);
* with the own-slot convention (FP32) the obstacle nodes of a wave that holds fluid nodes
  store their own slots too (whole-line stores), in the two-buffer step and in the local
  phase: no pull reads those slots, so the results do not change.
"""
import numpy as np
import pytest

from paper_1710_09472_amd import lbm

WAVE = 64  # threads per wave; a wave covers WAVE * V consecutive nodes of one x row


class Grid:
    def __init__(self, lattice, nx, ny, nz, obstacles, slip, solid_slot, V):
        _, D, e = lbm.lattice_info(lattice)
        self.e = np.array(e, dtype=int).reshape(-1, 3)
        self.Q = len(self.e)
        self.opp = [int(np.nonzero((self.e == -v).all(1))[0][0]) for v in self.e]
        self.nx, self.ny, self.nz = nx, ny, nz
        self.slip, self.solid_slot, self.V = slip, solid_slot, V
        self.obst = obstacles.reshape(nz, ny, nx).astype(bool)
        z, y, _ = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        wall = np.zeros_like(self.obst)
        if slip & 1:
            wall |= (y == 0) | (y == ny - 1)
        if slip & 2:
            wall |= (z == 0) | (z == nz - 1)
        self.solid = self.obst | wall

    def reflected(self, q, fy, fz):
        t = self.e[q] * np.array([1, -1 if fy else 1, -1 if fz else 1])
        return int(np.nonzero((self.e == t).all(1))[0][0])

    def wall_y(self, y):
        return bool(self.slip & 1) and y in (0, self.ny - 1)

    def wall_z(self, z):
        return bool(self.slip & 2) and z in (0, self.nz - 1)

    def pull_nobb(self, x, y, z, q):
        """(slot, node) the pull of q into (x, y, z) reads when it does not bounce back:
        slot q of x - e_q, or the specular source in the puller's row beside a wall plane."""
        ex, ey, ez = self.e[q]
        sx, sy, sz = (x - ex) % self.nx, (y - ey) % self.ny, (z - ez) % self.nz
        fy = ey != 0 and self.wall_y(sy)
        fz = ez != 0 and self.wall_z(sz)
        if fy:
            sy = y
        if fz:
            sz = z
        return (self.reflected(q, fy, fz), (sx, sy, sz))

    def bounced(self, x, y, z, q):
        if q == 0:
            return False
        _, (sx, sy, sz) = self.pull_nobb(x, y, z, q)
        return bool(self.obst[sz, sy, sx])

    def P(self, x, y, z, q):
        """Location the two-buffer step pulls f_q(x) from."""
        if self.bounced(x, y, z, q) and not self.solid_slot:
            return (self.opp[q], (x, y, z))
        return self.pull_nobb(x, y, z, q)

    def nodes(self):
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    yield x, y, z

    def fluid(self, x, y, z):
        return not self.solid[z, y, x]


def collide(values, node, Q):
    """Stand-in for the collision: any fixed map that mixes all populations of a node."""
    x, y, z = node
    k = np.arange(Q)
    return np.array([values[(q + 1) % Q] * 0.5 + values[q] * 0.25 + values[(q + 3) % Q] * 0.125 +
                     0.01 * (x + 3 * y + 7 * z + 11 * q) for q in k])


def stored_solids(g: Grid):
    """Solid nodes that store their own slots: with the own-slot convention, those of a
    wave (WAVE * V consecutive nodes of a row) that holds a fluid node; none otherwise."""
    if g.solid_slot:
        return set()
    out = set()
    for z in range(g.nz):
        for y in range(g.ny):
            for xw in range(0, g.nx, WAVE * g.V):
                wave = [(x, y, z) for x in range(xw, min(g.nx, xw + WAVE * g.V))]
                if any(g.fluid(*n) for n in wave):
                    out.update(n for n in wave if not g.fluid(*n))
    return out


def two_buffer_step(g: Grid, src: dict, solid_stores=False) -> dict:
    dst = {}
    junk_nodes = stored_solids(g) if solid_stores else set()
    for n in g.nodes():
        if n in junk_nodes:  # whatever its loads give; stored in its own slots
            f = np.array([src.get(g.pull_nobb(*n, q), 0.0) for q in range(g.Q)])
            o = collide(f, n, g.Q) + 1e6
            for q in range(g.Q):
                dst[(q, n)] = o[q]
            continue
        if not g.fluid(*n):
            continue
        f = np.array([src[g.P(*n, q)] for q in range(g.Q)])
        o = collide(f, n, g.Q)
        for q in range(g.Q):
            dst[(q, n)] = o[q]
        if g.solid_slot:
            for q in range(1, g.Q):
                if g.bounced(*n, q):
                    dst[g.P(*n, q)] = o[g.opp[q]]
    return dst


def pull_phase_threads(g: Grid, odd=False):
    """(reads, writes) of every thread of the pull phase; writes as (location, q, node).
    Rows of free-slip wall planes leave at once; in every other row the threads load and
    collide, fluid nodes store, and with two nodes per thread (16-bit) pairs are stored
    whole, obstacle nodes included (in waves of obstacles only, too). odd: the thread's
    pair is taken one node to the right, (x0 + 1, x0 + 2 mod nx), as the 16-bit pull phase
    without solids does."""
    threads = []
    for z in range(g.nz):
        for y in range(g.ny):
            if g.wall_y(y) or g.wall_z(z):
                continue
            for xw in range(0, g.nx, WAVE * g.V):  # one wave
                for x0 in range(xw, min(g.nx, xw + WAVE * g.V), g.V):
                    tn = [((x0 + i + (1 if odd else 0)) % g.nx, y, z) for i in range(g.V)]
                    pairs = g.V == 2 and g.solid_slot
                    reads, writes = [], []
                    for n in tn:
                        takes_part = pairs or g.fluid(*n)
                        if not takes_part:
                            continue
                        for q in range(g.Q):
                            reads.append((g.P(*n, q), q, n))
                            writes.append((g.P(*n, g.opp[q]), q, n))
                    threads.append((reads, writes))
    return threads


def local_phase_threads(g: Grid, solid_stores=False):
    threads = []
    junk_nodes = stored_solids(g) if solid_stores else set()
    for n in g.nodes():
        if n in junk_nodes:  # loads its own slots, stores them
            threads.append(([((g.opp[q], n), q, n) for q in range(g.Q)], [((q, n), q, n) for q in range(g.Q)]))
            continue
        if not g.fluid(*n):
            continue
        reads, writes = [], []
        for q in range(g.Q):
            if g.solid_slot and g.bounced(*n, q):
                loc = g.P(*n, q)
            else:
                loc = (g.opp[q], n)
            reads.append((loc, q, n))
            writes.append(((q, n), q, n))
        if g.solid_slot:
            for q in range(1, g.Q):
                if g.bounced(*n, q):
                    writes.append((g.P(*n, q), g.opp[q], n))
        threads.append((reads, writes))
    return threads


def check_race_free(g: Grid, threads, phase):
    writer = {}
    for t, (_, writes) in enumerate(threads):
        for loc, _, _ in writes:
            assert writer.setdefault(loc, t) == t, f"{phase}: {loc} written by two threads"
    for t, (reads, _) in enumerate(threads):
        for loc, _, _ in reads:
            assert writer.get(loc, t) == t, f"{phase}: {loc} read by one thread and written by another"
    # locations read or written by the obstacle nodes that take part (pairs) touch no fluid node's
    fluid_locs = set()
    for reads, writes in threads:
        for loc, _, n in reads + writes:
            if g.fluid(*n):
                fluid_locs.add(loc)
    for reads, writes in threads:
        for loc, _, n in reads + writes:
            if not g.fluid(*n):
                assert loc not in fluid_locs, f"{phase}: obstacle node {n} touches {loc}, also used by a fluid node"


def run_phase(g: Grid, buf: dict, threads, order):
    out = dict(buf)
    for t in order:
        reads, writes = threads[t]
        by_node = {}
        for loc, q, n in reads:
            by_node.setdefault(n, {})[q] = buf.get(loc, np.nan)
        o = {n: collide(np.array([v[q] for q in range(g.Q)]), n, g.Q) for n, v in by_node.items()}
        for loc, q, n in writes:
            out[loc] = o[n][q]
    return out


CASES = [
    # lattice, (nx, ny, nz), obstacle fraction, slip, seed
    ("D2V9", (12, 7, 1), 0.25, 0, 1),
    ("D2V9", (10, 9, 1), 0.2, 1, 2),
    ("D2V9", (2, 5, 1), 0.3, 1, 3),
    ("D2V9", (140, 4, 1), 0.2, 0, 4),   # more than one wave of pairs per row
    ("D3V19", (6, 5, 5), 0.2, 3, 5),
    ("D3V19", (5, 4, 3), 0.25, 0, 6),
    ("D3V19", (4, 6, 5), 0.2, 1, 7),
    ("D2V9", (12, 9, 1), 0.2, 1, 8, (3, 4)),   # rows y = 3, 4 all obstacles: waves of obstacles only
    ("D3V19", (6, 5, 5), 0.15, 2, 9, (2,)),    # a plane of obstacles at y = 2, beside z walls
]


@pytest.mark.parametrize("solid_slot,V,odd", [(False, 1, False), (True, 1, False), (True, 2, False), (True, 2, True)],
                         ids=["own-slot", "solid-slot", "pairs", "pairs-odd"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1][0]}x{c[1][1]}x{c[1][2]}-slip{c[3]}" for c in CASES])
def test_inplace_phases_race_free_and_equal_to_two_buffers(case, solid_slot, V, odd):
    lattice, (nx, ny, nz), phi, slip, seed = case[:5]
    if V == 2 and (lattice != "D2V9" or nx % 2):
        pytest.skip("two nodes per thread: 16-bit D2V9 rows of even length")
    rng = np.random.default_rng(seed)
    obst = (rng.random(nx * ny * nz) < phi).astype(np.uint8)
    for yr in (case[5] if len(case) > 5 else ()):
        obst.reshape(nz, ny, nx)[:, yr, :] = 1
    g = Grid(lattice, nx, ny, nz, obst, slip, solid_slot, V)
    # an even-layout state: a value at every location any pull reads
    s0 = {}
    for n in g.nodes():
        if g.fluid(*n):
            for q in range(g.Q):
                s0[g.P(*n, q)] = rng.standard_normal()
    # every other location holds junk the fluid result must not depend on
    junk = {(q, n): 1e6 + rng.standard_normal() for n in g.nodes() for q in range(g.Q)}
    buf = {**junk, **s0}
    p0, p1 = pull_phase_threads(g, odd=odd), local_phase_threads(g, solid_stores=True)
    check_race_free(g, p0, "pull phase")
    check_race_free(g, p1, "local phase")
    if not solid_slot:
        # the two-buffer step with and without the obstacle nodes' stores
        a = two_buffer_step(g, two_buffer_step(g, s0, True), True)
        b = two_buffer_step(g, two_buffer_step(g, s0))
        for n in g.nodes():
            if g.fluid(*n):
                for q in range(g.Q):
                    assert a[g.P(*n, q)] == b[g.P(*n, q)], (n, q)
    # two in-place phases (two thread orders) against two two-buffer steps
    ref = two_buffer_step(g, two_buffer_step(g, s0))
    results = []
    for order_seed in (0, 1):
        o = np.random.default_rng(100 + order_seed)
        b = run_phase(g, buf, p0, o.permutation(len(p0)))
        b = run_phase(g, b, p1, o.permutation(len(p1)))
        results.append(b)
    for n in g.nodes():
        if g.fluid(*n):
            for q in range(g.Q):
                loc = g.P(*n, q)
                assert results[0][loc] == results[1][loc] == ref[loc], (n, q, loc)
