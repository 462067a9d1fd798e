"""The device-planned batch block step sizes its work list for
target + ceil(N / IB) + C + 64 items and its partial sums for IB * target + N
rows before it knows the step's active set.  This restates the planner's
integer arithmetic (each system's active rows, the common chunk length J
rounded up to the tile, S_c chunks of at least one tile, items and partial
rows) and checks both bounds on random and adversarial batches and active
sets: the planner's fallback for an overflow is then never taken."""
import numpy as np
import pytest

TILE = 256


def plan(sizes, active_per_sys, IB, target):
    work = sum(-(-na // IB) * IB * nj for nj, na in zip(sizes, active_per_sys))
    J = -(-work // (IB * target))
    J = -(-J // TILE) * TILE
    J = max(J, TILE)
    items = parts = 0
    for nj, na in zip(sizes, active_per_sys):
        S = -(-nj // J)
        S = min(S, -(-nj // TILE))
        S = max(S, 1)
        items += -(-na // IB) * S
        if S > 1:
            parts += S * na
    return items, parts


def bounds(sizes, IB, target):
    N, C = int(sum(sizes)), len(sizes)
    return target + -(-N // IB) + C + 64, IB * target + N


@pytest.mark.parametrize("IB", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("target", [512, 2560, 7680])
def test_random_batches_fit(IB, target):
    rng = np.random.default_rng(IB * 7 + target)
    for _ in range(300):
        C = int(rng.integers(1, 300))
        sizes = np.minimum(16384, (128 * 128 ** rng.random(C)).astype(np.int64))
        if rng.random() < 0.3:
            sizes[rng.integers(0, C, max(1, C // 10))] = 0          # empty systems
        frac = rng.random()
        active = [int(rng.binomial(n, frac)) if n else 0 for n in sizes]
        items, parts = plan(sizes, active, IB, target)
        max_items, part_cap = bounds(sizes, IB, target)
        assert items <= max_items and parts <= part_cap


@pytest.mark.parametrize("IB", [128, 512])
def test_adversarial_batches_fit(IB):
    target = 2560
    cases = [
        [1] * 5000,                                  # many one-body systems, all active
        [16384] + [1] * 3000,                        # one large system among tiny ones
        [IB + 1] * 400,                              # every system one row past an i-block
        [TILE * 3 + 1] * 200,                        # chunk counts capped by the tile
        [2 ** 20],                                   # one huge system
        [0, 0, 5, 0, 7000, 0],                       # empty systems around real ones
    ]
    for sizes in cases:
        sizes = np.array(sizes, dtype=np.int64)
        for active in (list(sizes), [min(1, n) for n in sizes], [n // 2 for n in sizes]):
            items, parts = plan(sizes, active, IB, target)
            max_items, part_cap = bounds(sizes, IB, target)
            assert items <= max_items and parts <= part_cap, (sizes[:5], items, max_items, parts, part_cap)
