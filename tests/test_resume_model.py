"""CPU model of the rule the IC workgroup tiers follow when a set outgrows one of them: the
tier keeps the BFS levels it has completed (members [0, n) and where the last complete level
starts), and the next tier expands that level again and goes on.  Reverse reachability over
fixed live edges does not depend on the order vertices are met, so the resumed walk reaches
exactly the set a walk from the root reaches.  The model below is the rule alone, in plain
Python over random live-edge worlds; the GPU tests check the kernels that follow it."""

import numpy as np
import pytest


def _live_in_edges(n, m, p, seed):
    """A random directed graph and one live-edge world: live_in[v] = sources of v's live in-edges."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    live = rng.random(m) < p
    live_in = [[] for _ in range(n)]
    for s, d, l in zip(src, dst, live):
        if l:
            live_in[d].append(int(s))
    return live_in


def _bfs(live_in, queue, head, seen, cap):
    """Level-by-level reverse BFS from queue[head:], members in `queue`; returns (queue, None)
    when it finishes, or the completed levels (queue[:n], start of the last complete level)
    when a level would take the queue past `cap` members."""
    tail = len(queue)
    while head < tail:
        level_start = head
        for i in range(head, tail):
            for u in live_in[queue[i]]:
                if u not in seen:
                    seen.add(u)
                    queue.append(u)
        if len(queue) > cap:
            return queue[:tail], level_start  # level [level_start, tail) overflowed
        head, tail = tail, len(queue)
    return queue, None


def _tiered(live_in, root, caps):
    """The tier chain: each capacity in turn, resuming from the previous tier's completed levels."""
    queue, head = [root], 0
    for cap in caps:
        seen = set(queue)
        queue, lo = _bfs(live_in, list(queue), head, seen, cap)
        if lo is None:
            return sorted(queue), cap
        head = lo  # expand the overflowed level again
    raise AssertionError("the last tier has no capacity limit")


@pytest.mark.parametrize("seed", range(12))
def test_resumed_levels_reach_the_same_set(seed):
    n, m = 400, 2400
    live_in = _live_in_edges(n, m, 0.45, seed)
    for root in range(0, n, 37):
        full, _ = _bfs(live_in, [root], 0, {root}, n + 1)
        for caps in ([2, 8, 32, n + 1], [1, n + 1], [64, 128, n + 1], [n + 1]):
            got, _ = _tiered(live_in, root, caps)
            assert got == sorted(full), (seed, root, caps)


def test_overflow_keeps_whole_levels():
    # a star of 10 leaves behind a path: the first tier (cap 5) sees the star's level overflow
    # and keeps only the root; the next tier expands the root's level again
    live_in = [[] for _ in range(20)]
    live_in[0] = list(range(1, 11))
    live_in[1] = [11]
    queue, lo = _bfs(live_in, [0], 0, {0}, 5)
    assert queue == [0] and lo == 0
    got, cap = _tiered(live_in, 0, [5, 100])
    assert got == list(range(12)) and cap == 100
