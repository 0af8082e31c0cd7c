"""CPU model of the eigensolver's cross-work-group exchange protocol.

The Householder reduction of one plane runs on W work-groups that exchange,
at every step k, the vector p and the next column through a global area with
two halves; step k uses half k mod 2, and the first column is published
before the first grid barrier in half 1.  Per step a work-group writes its
share (before the step's barrier) and, after the barrier, reads every
work-group's share.  A grid barrier only guarantees that no work-group leaves
it before all have arrived, so a fast work-group may run a whole step ahead of
a slow one.

The model runs W work-groups as event sequences (write, barrier, read per
step) under random schedules that respect only the barrier rule, and checks
that every read returns the value written for the step it reads.  The same
model with the first column published in half 0 (the hazard found on the GPU
with two ensembles in flight: step 0 overwrote column 0 while a late
work-group could still read it) must fail for some schedule.  Writes are
visible at once in the model: it checks the slot assignment (which half each
step uses against which work-groups can still be reading it), not the
hardware's memory ordering, which the GPU tests exercise (two ensembles on two
streams, every exchange mode)."""
import random

import pytest


def _events(w, W, steps, first_half):
    """Event list of work-group w: ("w", half, tag), ("b", index), ("r", half, tag)."""
    ev = []
    if w == 0:
        ev.append(("w", first_half, ("col", 0)))       # the owner of column 0 publishes it
    ev.append(("b", 0))
    ev.append(("r", first_half, ("col", 0)))
    for k in range(steps):
        h = k & 1
        ev.append(("w", h, ("p", k, w)))                # its share of p and, for one owner,
        if w == (k + 1) % W:                            # the next column
            ev.append(("w", h, ("col", k + 1)))
        ev.append(("b", k + 1))
        for v in range(W):
            ev.append(("r", h, ("p", k, v)))
        ev.append(("r", h, ("col", k + 1)))
    return ev


def _run(W, steps, first_half, seed):
    rng = random.Random(seed)
    evs = [_events(w, W, steps, first_half) for w in range(W)]
    pos = [0] * W
    arrived = {}                                        # barrier index -> work-groups arrived
    mem = {0: {}, 1: {}}                                # half -> {(kind, ...key): tag}
    while any(pos[w] < len(evs[w]) for w in range(W)):
        ready = []
        for w in range(W):
            if pos[w] >= len(evs[w]):
                continue
            e = evs[w][pos[w]]
            if e[0] == "b":
                arrived.setdefault(e[1], set()).add(w)
                if len(arrived[e[1]]) < W:              # wait until every work-group arrived
                    continue
            ready.append(w)
        w = rng.choice(ready)
        e = evs[w][pos[w]]
        pos[w] += 1
        if e[0] == "w":
            kind = e[2][0]
            key = (kind,) if kind == "col" else (kind, e[2][2])
            mem[e[1]][key] = e[2]
        elif e[0] == "r":
            kind = e[2][0]
            key = (kind,) if kind == "col" else (kind, e[2][2])
            if mem[e[1]].get(key) != e[2]:
                return False
    return True


@pytest.mark.parametrize("W", [2, 3])
def test_parity_halves_are_safe(W):
    assert all(_run(W, 6, 1, seed) for seed in range(3000))


def test_first_column_in_the_even_half_races():
    assert not all(_run(3, 3, 0, seed) for seed in range(3000))
