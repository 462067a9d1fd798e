"""Barnes-Hut tree code on a Peano-Hilbert curve -- TEST INFRASTRUCTURE ONLY.

The paper's collisionless method (section "Simulating collisionless systems
with hierarchical domain-decomposition methods" and its "Implementation"
subsection): particles sorted along a Peano-Hilbert space-filling curve, an
octree whose cells split the curve into distinct pieces until a cell holds
at most a critical number of particles, multipole moments of every cell, a
geometric opening-angle criterion, and groups of up to 64 curve-consecutive
particles (split further while a group is larger than a maximal size) that
walk the tree together.  This module is the reading the library implements,
written out plainly in numpy:

  box       lo = per-dimension minimum of the positions; side = 2^e with
            2^e >= (1 + 2^-10) * (largest extent) (frexp); h = side 2^-21;
            integer coordinates floor((x - lo) / h) clamped to [0, 2^21 - 1]
  keys      63-bit Peano-Hilbert index of the integer coordinates (Skilling's
            transform of the axes into the transposed Hilbert index, then the
            bits of the three transposed words interleaved from the top);
            particles sorted by (key, index)
  cells     cell (l, p) = the sorted particles whose key has the 3l-bit prefix
            p; the root is (0, 0); a cell with more than n_crit particles
            (and l < 21) is split into its non-empty children, in curve
            order; its cube has side 2^(21-l) h and corner lo + (the first
            particle's integer coordinates with the low 21-l bits cleared) h
  moments   mass M, centre of mass X, traceless quadrupole
            Q = sum m (3 d d^T - |d|^2 I), d = x - X, over the cell's particles
  groups    curve-consecutive runs of 64 (the last one shorter); a group whose
            bounding box is wider than g_max in some dimension is split into
            halves [b, b + ceil(n/2)) and the rest, recursively, first half
            first, until it fits or holds one particle
  walk      per group, from the root: a cell other than the root is accepted
            when theta^2 d^2 > side^2, d the distance between the group's
            bounding box and the cell's cube (per dimension the positive part
            of the larger gap); otherwise a leaf is opened (its particles
            interact directly) and an internal cell is replaced by its children
  forces    for a particle at x, an accepted cell contributes, with
            y = x - X and s = |y|^2 + eps2,
              a   = -M y s^-3/2 + Q y s^-5/2 - (5/2)(y.Q y) y s^-7/2
              phi = -M s^-1/2 - (1/2)(y.Q y) s^-5/2
            and every particle j != i of an opened leaf the Plummer-softened
            pair terms m r s^-3/2, -m s^-1/2 (r = x_j - x_i)

With theta = 0 nothing is accepted and the sum is the direct one.
"""
from dataclasses import dataclass

import numpy as np

BITS = 21
LEAF_LEVEL = BITS


def box(pos):
    lo = pos.min(axis=0)
    ext = float((pos.max(axis=0) - lo).max())
    if ext > 0:
        _, e = np.frexp(ext * (1.0 + 2.0 ** -10))
        side = float(np.ldexp(1.0, int(e)))
    else:
        side = 1.0
    return lo, side


def grid_coords(pos, lo, side):
    h = side * 2.0 ** -BITS
    q = np.floor((pos - lo) / h)
    return np.clip(q, 0, 2 ** BITS - 1).astype(np.int64)


def hilbert_keys(ijk, bits=BITS):
    """Peano-Hilbert indices of integer coordinates ijk [n, 3] (numpy int64).

    Skilling's construction ("Programming the Hilbert curve", 2004), restated:
    walking the bit planes from the top one down to the second lowest, each
    axis in turn either flips the lower bits of axis 0 (when its own bit on
    that plane is set) or trades its lower bits with those of axis 0; the
    axes are then Gray-coded against their predecessor, and a mask built from
    the higher bits of the last axis is XORed into all three.  The index is
    the three resulting words with their bits interleaved from the top, axis 0
    first."""
    w = [np.array(ijk[:, k], dtype=np.int64) for k in range(3)]
    plane = 1 << (bits - 1)
    while plane > 1:
        low = plane - 1
        for k in range(3):
            on = (w[k] & plane) != 0
            flipped = w[0] ^ low
            diff = (w[0] ^ w[k]) & low
            traded0 = w[0] ^ diff
            tradedk = w[k] ^ diff
            if k == 0:
                w[0] = np.where(on, flipped, w[0])
            else:
                w[0], w[k] = np.where(on, flipped, traded0), np.where(on, w[k], tradedk)
        plane >>= 1
    w[1] = w[1] ^ w[0]
    w[2] = w[2] ^ w[1]
    mask = np.zeros_like(w[2])
    plane = 1 << (bits - 1)
    while plane > 1:
        mask = np.where((w[2] & plane) != 0, mask ^ (plane - 1), mask)
        plane >>= 1
    w = [x ^ mask for x in w]
    key = np.zeros_like(w[0])
    for b in range(bits - 1, -1, -1):
        for k in range(3):
            key = (key << 1) | ((w[k] >> b) & 1)
    return key


@dataclass
class Cell:
    level: int
    prefix: int
    begin: int          # range in the sorted order
    end: int
    corner: np.ndarray  # cube corner (double)
    side: float
    children: list
    M: float = 0.0
    X: np.ndarray = None
    Q: np.ndarray = None

    @property
    def leaf(self):
        return not self.children


@dataclass
class Tree:
    order: np.ndarray   # sorted position -> original index
    keys: np.ndarray    # sorted keys
    pos: np.ndarray     # sorted copies
    mass: np.ndarray
    ijk: np.ndarray     # sorted integer coordinates
    cells: list         # cells[0] is the root
    lo: np.ndarray
    side: float
    h: float


def build(pos, mass, n_crit=16):
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    n = mass.shape[0]
    lo, side = box(pos)
    h = side * 2.0 ** -BITS
    ijk = grid_coords(pos, lo, side)
    keys = hilbert_keys(ijk)
    order = np.lexsort((np.arange(n), keys))
    keys, ijk_s, pos_s, mass_s = keys[order], ijk[order], pos[order], mass[order]
    cells = []

    def make(level, prefix, b, e):
        shift = BITS - level
        corner_int = (ijk_s[b] >> shift) << shift
        c = Cell(level, prefix, b, e, lo + corner_int.astype(np.float64) * h, float(2 ** shift) * h, [])
        cells.append(c)
        return len(cells) - 1

    root = make(0, 0, 0, n)
    stack = [root]
    while stack:
        ci = stack.pop()
        c = cells[ci]
        if c.end - c.begin <= n_crit or c.level == LEAF_LEVEL:
            continue
        shift = 3 * (BITS - c.level - 1)
        b = c.begin
        for k in range(8):
            p = (c.prefix << 3) | k
            # the last child ends with its parent (its bound, 8 << 60 at the
            # top, would not fit a signed 64-bit key)
            e = c.end if k == 7 else int(np.searchsorted(keys, (p + 1) << shift, side="left"))
            if e > b:
                c.children.append(make(c.level + 1, p, b, e))
            b = e
        stack.extend(reversed(c.children))
    for c in cells:
        c.M, c.X, c.Q = moments(pos_s[c.begin:c.end], mass_s[c.begin:c.end], c.corner + c.side / 2)
    return Tree(order, keys, pos_s, mass_s, ijk_s, cells, lo, side, h)


def moments(x, m, centre):
    """Mass, centre of mass (the cube centre when massless) and traceless quadrupole."""
    M = float(m.sum())
    X = (m[:, None] * x).sum(0) / M if M > 0 else np.asarray(centre, dtype=np.float64)
    d = x - X
    dd = (d * d).sum(1)
    Q = (m[:, None, None] * (3.0 * (d[:, :, None] * d[:, None, :]) - dd[:, None, None] * np.eye(3))).sum(0)
    return M, X, Q


def cell_field(M, X, Q, x, eps2):
    """Acceleration and potential at points x [n, 3] of a cell's monopole and quadrupole."""
    y = x - X
    s = (y * y).sum(1) + eps2
    Qy = y @ Q.T
    yQy = (y * Qy).sum(1)
    a = -M * y * s[:, None] ** -1.5 + Qy * s[:, None] ** -2.5 - 2.5 * (yQy * s ** -3.5)[:, None] * y
    p = -M * s ** -0.5 - 0.5 * yQy * s ** -2.5
    return a, p


def groups(tree, g_max, size=64):
    """(begin, end) ranges in the sorted order."""
    n = tree.mass.shape[0]
    out = []

    def split(b, e):
        x = tree.pos[b:e]
        if e - b > 1 and float((x.max(0) - x.min(0)).max()) > g_max:
            m = b + (e - b + 1) // 2
            split(b, m)
            split(m, e)
        else:
            out.append((b, e))

    for b in range(0, n, size):
        split(b, min(n, b + size))
    return out


def _accept(cell, glo, ghi, theta):
    clo = cell.corner
    chi = cell.corner + cell.side
    gap = np.maximum(np.maximum(clo - ghi, glo - chi), 0.0)
    d2 = gap[0] * gap[0] + gap[1] * gap[1] + gap[2] * gap[2]
    return theta * theta * d2 > cell.side * cell.side


def walk(tree, g, theta):
    """Accepted cells and opened leaves of one group (cell indices, curve order)."""
    b, e = g
    glo, ghi = tree.pos[b:e].min(0), tree.pos[b:e].max(0)
    acc_cells, leaves = [], []
    stack = [0]
    while stack:
        ci = stack.pop()
        c = tree.cells[ci]
        if ci != 0 and _accept(c, glo, ghi, theta):
            acc_cells.append(ci)
        elif c.leaf:
            leaves.append(ci)
        else:
            stack.extend(reversed(c.children))
    return acc_cells, leaves


def forces(pos, mass, eps2, theta, n_crit=16, g_max=None, tree=None):
    """Tree acceleration and potential of every particle (original order).

    Returns (acc [N,3], pot [N], stats) with stats the per-group counts of
    accepted cells, opened leaves and directly summed particles."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    t = tree if tree is not None else build(pos, mass, n_crit)
    if g_max is None:
        g_max = t.side / 16
    acc_s = np.zeros((n, 3))
    pot_s = np.zeros(n)
    stats = []
    for g in groups(t, g_max):
        b, e = g
        ci, li = walk(t, g, theta)
        x = t.pos[b:e]
        a = np.zeros((e - b, 3))
        p = np.zeros(e - b)
        for c in (t.cells[k] for k in ci):
            da, dp = cell_field(c.M, c.X, c.Q, x, eps2)
            a += da
            p += dp
        nd = 0
        for c in (t.cells[k] for k in li):
            xj = t.pos[c.begin:c.end]
            mj = t.mass[c.begin:c.end]
            r = xj[None, :, :] - x[:, None, :]
            s = (r * r).sum(2) + eps2
            idx_i = np.arange(b, e)[:, None]
            idx_j = np.arange(c.begin, c.end)[None, :]
            keep = (idx_i != idx_j) & (s > 0)
            w = np.where(keep, mj[None, :] * np.where(keep, s, 1.0) ** -1.5, 0.0)
            a += (w[:, :, None] * r).sum(1)
            p -= np.where(keep, mj[None, :] * np.where(keep, s, 1.0) ** -0.5, 0.0).sum(1)
            nd += c.end - c.begin
        acc_s[b:e] = a
        pot_s[b:e] = p
        stats.append((len(ci), len(li), nd))
    acc = np.empty_like(acc_s)
    pot = np.empty_like(pot_s)
    acc[t.order] = acc_s
    pot[t.order] = pot_s
    return acc, pot, stats
