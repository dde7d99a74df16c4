"""Host model of the persistent kernels' grid barrier (counting logic only;
the memory fences are the hardware's business): workgroups count their
arrival in one of up to 8 groups (workgroup b in group b mod 8) with monotone
counters, so a workgroup's generation is its arrival index over the group's
size; the last arrival of a group counts the group done, the last group
publishes the generation, and every workgroup waits until the published
generation reaches its own. Random interleavings of the atomic steps check
that no workgroup leaves a barrier before every workgroup has arrived at it,
and that every run finishes (no lost wake-up), for grid sizes that are and
are not multiples of the group count."""
from __future__ import annotations

import random

import pytest

GROUPS = 8


class Grid:
    def __init__(self, nblocks: int):
        self.nb = nblocks
        self.ng = min(nblocks, GROUPS)
        self.group = [0] * self.ng   # arrival counters
        self.done = 0                # groups done
        self.release = 0             # published generation

    def gsize(self, g: int) -> int:
        return self.nb // self.ng + (1 if g < self.nb % self.ng else 0)


def block_program(grid: Grid, b: int, barriers: int, arrivals: list[int], passed: list[int]):
    """One workgroup's atomic steps, as a generator (one yield per step)."""
    g = b % grid.ng
    for i in range(barriers):
        # arrival: one atomic add on the group's counter
        arrived = grid.group[g]
        grid.group[g] += 1
        arrivals[b] += 1
        gen = arrived // grid.gsize(g) + 1
        yield
        if arrived % grid.gsize(g) == grid.gsize(g) - 1:
            done = grid.done
            grid.done += 1
            yield
            if done % grid.ng == grid.ng - 1:
                grid.release = gen
                yield
        # wait for the generation
        while grid.release < gen:
            yield
        # leaving barrier i: every workgroup must have arrived at it
        assert min(arrivals) >= i + 1, (b, i, arrivals)
        assert gen == i + 1
        passed[b] += 1
        yield


@pytest.mark.parametrize("nblocks", [1, 2, 3, 7, 8, 9, 15, 16, 17, 37])
def test_barrier_orders_and_finishes(nblocks):
    barriers = 6
    for seed in range(40):
        rng = random.Random(1000 * nblocks + seed)
        grid = Grid(nblocks)
        arrivals = [0] * nblocks
        passed = [0] * nblocks
        progs = {b: block_program(grid, b, barriers, arrivals, passed) for b in range(nblocks)}
        steps = 0
        while progs:
            b = rng.choice(list(progs))
            try:
                next(progs[b])
            except StopIteration:
                del progs[b]
            steps += 1
            assert steps < 200_000, "barrier model did not finish"
        assert passed == [barriers] * nblocks
        assert grid.release == barriers
        assert grid.done == barriers * grid.ng
        assert all(grid.group[g] == barriers * grid.gsize(g) for g in range(grid.ng))


def test_group_sizes_cover_the_grid():
    for nb in range(1, 300):
        grid = Grid(nb)
        sizes = [grid.gsize(g) for g in range(grid.ng)]
        assert sum(sizes) == nb and min(sizes) >= 1
        assert sorted(b % grid.ng for b in range(nb)) == sorted(
            g for g in range(grid.ng) for _ in range(sizes[g]))
