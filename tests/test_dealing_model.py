"""Host model of the batch kernel's work list and its two ways of dealing
items to workgroups (no GPU needed).

The persistent batch kernel cuts every image into tiles and every chain into
blocks of k steps; item (image, tile, block) may start once the 3x3 tile
neighbourhood of the same image has finished block - 1.  The list is built
block by block (images with the most steps first, tiles in raster order),
which these tests show to be a topological order of those dependencies.

Dealing by ticket (each workgroup draws the next list item when it has
finished its previous one) then makes progress with any number of resident
workgroups: the model runs every list to completion with 1 .. many workers.
Dealing round-robin by workgroup label (label g takes items g, g + G, ...)
needs all G labels resident at once: the model shows a list that stalls
forever when only some of them are.
"""
import heapq
import random

import pytest


def build_items(images):
    """images: list of (tiles_x, tiles_y, blocks).  Returns the work list in
    the order the plan builder uses: block-major; within a block, images with
    more blocks first (stable); tiles in raster order."""
    order = sorted(range(len(images)), key=lambda j: -images[j][2])
    items = []
    for b in range(max(im[2] for im in images)):
        for j in order:
            tx, ty, nb = images[j]
            if b >= nb:
                continue
            for t in range(tx * ty):
                items.append((j, t, b))
    return items


def deps(images, item):
    j, t, b = item
    if b == 0:
        return []
    tx, ty, _ = images[j]
    x, y = t % tx, t // tx
    out = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            nx, ny = x + dx, y + dy
            if 0 <= nx < tx and 0 <= ny < ty:
                out.append((j, ny * tx + nx, b - 1))
    return out


def random_images(rng, n):
    return [(rng.randint(1, 9), rng.randint(1, 9), rng.randint(1, 12)) for _ in range(n)]


@pytest.mark.parametrize("seed", range(20))
def test_list_is_a_topological_order(seed):
    rng = random.Random(seed)
    images = random_images(rng, rng.randint(1, 12))
    items = build_items(images)
    index = {it: i for i, it in enumerate(items)}
    assert len(index) == len(items)
    for i, it in enumerate(items):
        for d in deps(images, it):
            assert index[d] < i, (it, d)


def run_tickets(images, workers, rng):
    """Event model of ticket dealing: returns the finish time of the last item.
    Tickets go out in list order, each to the worker that became free first;
    an item starts when its worker is free and its dependencies are done."""
    items = build_items(images)
    finish = {}
    free = [(0.0, w) for w in range(workers)]
    heapq.heapify(free)
    for it in items:
        t_free, w = heapq.heappop(free)
        # every dependency has a smaller ticket, so it was dealt (and its
        # finish time fixed) before this one
        ready = max([finish[d] for d in deps(images, it)], default=0.0)
        start = max(t_free, ready)
        finish[it] = start + rng.uniform(0.5, 2.0)
        heapq.heappush(free, (finish[it], w))
    return max(finish.values(), default=0.0)


@pytest.mark.parametrize("workers", [1, 2, 3, 7, 64, 1000])
def test_ticket_dealing_progresses_with_any_number_of_workers(workers):
    rng = random.Random(workers)
    for _ in range(5):
        images = random_images(rng, rng.randint(1, 10))
        n_items = len(build_items(images))
        end = run_tickets(images, workers, rng)
        # never slower than one worker doing everything back to back at the
        # longest item time, whatever the residency
        assert 0 < end <= 2.0 * n_items + 1e-9


def run_round_robin(images, labels, resident):
    """Round-robin dealing by label with only `resident` labels running at
    first; a label that has not started takes a slot only when a running
    label has finished its whole share.  Returns True if every item finishes,
    False if the running labels all wait on items of labels that cannot start
    (a stall that only a bounded wait ends)."""
    items = build_items(images)
    index = {it: i for i, it in enumerate(items)}
    done = [False] * len(items)
    share = {g: list(range(g, len(items), labels)) for g in range(labels)}
    pos = {g: 0 for g in range(labels)}
    running = list(range(min(resident, labels)))
    waiting = list(range(len(running), labels))
    while running:
        progressed = False
        for g in list(running):
            while pos[g] < len(share[g]):
                i = share[g][pos[g]]
                if all(done[index[d]] for d in deps(images, items[i])):
                    done[i] = True
                    pos[g] += 1
                    progressed = True
                else:
                    break
            if pos[g] == len(share[g]):
                running.remove(g)
                if waiting:
                    running.append(waiting.pop(0))
                progressed = True
        if not progressed:
            return False
    return all(done)


def test_round_robin_needs_every_label_resident():
    # one image of 4 x 4 tiles and 3 blocks: 48 items over 8 labels
    images = [(4, 4, 3)]
    assert run_round_robin(images, labels=8, resident=8)
    # with fewer labels resident than dealt, a running label waits for a
    # block-0 item that belongs to a label that never gets a slot
    assert not run_round_robin(images, labels=8, resident=4)
    # ticket dealing finishes the same list with four workers (or one)
    assert run_tickets(images, 4, random.Random(0)) > 0
    assert run_tickets(images, 1, random.Random(0)) > 0
