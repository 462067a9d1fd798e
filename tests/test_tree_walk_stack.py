"""The wavefront walk of the tree kernel, emulated on the oracle's trees: up
to 64 cells are popped from the top of a stack per step, each is accepted,
opened as a leaf or replaced by its children, which are pushed in lane order.
The emulation finds exactly the oracle's accepted cells and opened leaves for
every group, and the stack never exceeds the bound the kernel allocates
(8 x 64 x 21 entries, and never more than the number of cells), including
theta = 0, where every cell is opened, and a deep, strongly clustered tree."""
import numpy as np
import pytest

from oracle import tree as TR
import synth

LANES = 64
BOUND = 8 * LANES * TR.BITS


def wave_walk(t, g, theta):
    b, e = g
    glo, ghi = t.pos[b:e].min(0), t.pos[b:e].max(0)
    root = t.cells[0]
    acc, leaves = [], []
    if not root.children:
        return acc, [0], 0
    stack = list(root.children)
    peak = len(stack)
    while stack:
        k = min(LANES, len(stack))
        popped = stack[len(stack) - k:]
        del stack[len(stack) - k:]
        pushed = []
        for ci in popped:                      # lane order
            c = t.cells[ci]
            if TR._accept(c, glo, ghi, theta):
                acc.append(ci)
            elif c.leaf:
                leaves.append(ci)
            else:
                pushed.extend(c.children)
        stack.extend(pushed)
        peak = max(peak, len(stack))
    return acc, leaves, peak


def clustered(n, seed):
    """Nested clumps: a small fraction of the particles packed ever tighter,
    so the octree reaches deep levels."""
    rng = np.random.default_rng(seed)
    pos = rng.standard_normal((n, 3))
    m = n // 3
    for lev in range(1, 8):
        pos[:m] = pos[:m] * 0.1 + 0.3
        m //= 2
    return pos, np.full(n, 1.0 / n)


@pytest.mark.parametrize("case,theta", [("plummer", 0.5), ("plummer", 0.0), ("clustered", 0.6), ("clustered", 0.0)])
def test_wave_walk_matches_oracle_and_stack_bound(case, theta):
    if case == "plummer":
        p = synth.plummer(3000, 21)
        pos, mass = p.pos, p.mass
    else:
        pos, mass = clustered(3000, 22)
    t = TR.build(pos, mass, 8)
    gs = TR.groups(t, t.side / 16)
    depth = max(c.level for c in t.cells)
    peak_all = 0
    for g in gs[:: max(1, len(gs) // 25)]:
        a, l, peak = wave_walk(t, g, theta)
        ra, rl = TR.walk(t, g, theta)
        assert sorted(a) == sorted(ra) and sorted(l) == sorted(rl)
        assert peak <= min(BOUND, len(t.cells))
        peak_all = max(peak_all, peak)
    if case == "clustered":
        assert depth >= 10
    # the per-level argument: at most one push (<= 8 x 64) per level on the stack
    assert peak_all <= 8 * LANES * depth
