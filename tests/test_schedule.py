"""Host logic: the static task schedule of the tiled factorisation (p > 16).

The factorisation of [Q | I] by 64 x 64 tiles (Section 5, beta step iii, with
L^-1 = U^-T carried along) runs as tile tasks from per-block lists.  These
tests replay the lists on the CPU under the rules the device follows -- a task
waits until every tile it reads has reached the version it needs, then
advances the version of the tile it writes -- with random task durations, and
check that every replay finishes (no deadlock), that each tile is written by
one task at a time in step order, and that every tile ends final.  The
expected task set is enumerated here from the blocked algorithm itself.
"""
import heapq

import numpy as np
import pytest

from paper_1608_04329_amd import hsp

POTRF, TRSM, GEMM, PANEL = 0, 1, 2, 3


def decode(c):
    return c & 3, (c >> 2) & 1, (c >> 3) & 255, (c >> 11) & 255, (c >> 19) & 255


def with_inverse(nt):
    """L^-1 is carried along up to p = 1536 (24 tiles); beyond, beta is solved
    by substitution and only the diagonal tiles of L^-1 are formed."""
    return nt * 64 <= 1536


def expected_tasks(nt, chain, inv=None):
    """Right-looking blocked Cholesky of [Q | I]: every tile operation once.

    With a chain block, PANEL(k) (k >= 1) stands for the solve of tile
    (k-1, k), the update of tile (k, k) at step k-1 and the factorisation of
    tile (k, k).  Without the inverse, the L^-1 tasks (part 1) are left out.
    """
    out = set()
    inv = with_inverse(nt) if inv is None else inv
    for k in range(nt):
        out.add((PANEL, 0, k, k, k) if chain and k > 0 else (POTRF, 0, k, k, k))
        out.update((TRSM, 0, k, k, j) for j in range(k + 1, nt) if not (chain and j == k + 1))
        if inv:
            out.update((TRSM, 1, k, k, j) for j in range(k))
        for i in range(k + 1, nt):
            out.update((GEMM, 0, k, i, j) for j in range(i, nt)
                       if not (chain and i == j == k + 1))
            if inv:
                out.update((GEMM, 1, k, i, j) for j in range(k + 1))
    return out


def reads_ok(t, vU, vL):
    typ, part, k, i, j = t
    if typ == POTRF:
        return vU[k, k] >= k
    if typ == PANEL:
        return vU[k - 1, k] >= k - 1 and vU[k, k] >= k - 1
    if typ == TRSM:
        return vU[k, k] >= k + 1 and (vU[k, j] >= k if part == 0 else vL[k, j] >= k - j)
    if part == 0:
        return vU[k, i] >= k + 1 and vU[k, j] >= k + 1 and vU[i, j] >= k
    return vU[k, i] >= k + 1 and vL[k, j] >= k - j + 1 and vL[i, j] >= k - j


def write(t, vU, vL):
    typ, part, k, i, j = t
    if typ == PANEL:
        assert vU[k - 1, k] == k - 1 and vU[k, k] == k - 1
        vU[k - 1, k] = k
        vU[k, k] = k + 1
        vL[k, k] = 1
    elif typ == POTRF:
        assert vU[k, k] == k
        vU[k, k] = k + 1
        vL[k, k] = 1
    elif part == 0:
        r, c = (k, j) if typ == TRSM else (i, j)
        assert vU[r, c] == k, "U tile written out of step order"
        vU[r, c] = k + 1
    else:
        r, c = (k, j) if typ == TRSM else (i, j)
        assert vL[r, c] == k - j, "L^-1 tile written out of step order"
        vL[r, c] = k - j + 1


def replay(chain_list, queue, nqb, nt, rng, inv=None):
    """Event simulation of the device: block 0 runs chain_list in order; nqb
    other blocks claim queue entries in order, each reserving its next entry
    when it starts a task (as the kernel does), and wait on tile versions."""
    vU = np.zeros((nt, nt), np.int64)
    vL = np.zeros((nt, nt), np.int64)
    nb = 1 + nqb
    claimed = 0

    def claim():
        nonlocal claimed
        claimed += 1
        return claimed - 1

    cur = [0] + [claim() for _ in range(nqb)]  # block 0: index into chain_list
    nxt = [None] * nb
    running = []  # heap of (finish time, block)
    busy = [False] * nb
    now = 0.0
    left = len(chain_list) + len(queue)

    def task_of(b):
        if b == 0:
            return chain_list[cur[0]] if cur[0] < len(chain_list) else None
        return queue[cur[b]] if cur[b] < len(queue) else None

    while left:
        for b in range(nb):
            t = task_of(b)
            if not busy[b] and t is not None and reads_ok(t, vU, vL):
                if b > 0:
                    nxt[b] = claim()
                dur = rng.uniform(0.3, 3.0) * (4.0 if t[0] in (POTRF, PANEL) else 1.0)
                heapq.heappush(running, (now + dur, b))
                busy[b] = True
        assert running, f"deadlock with {left} tasks left"
        now, b = heapq.heappop(running)
        write(task_of(b), vU, vL)
        cur[b] = cur[b] + 1 if b == 0 else nxt[b]
        busy[b] = False
        left -= 1
    inv = with_inverse(nt) if inv is None else inv
    for i in range(nt):
        for j in range(nt):
            if i <= j:
                assert vU[i, j] == i + 1
            if j <= i and (inv or j == i):
                assert vL[i, j] == i - j + 1
    return now


def lists_of(nt, gp, inv=None):
    tasks, off = hsp.hsp_tile_schedule(nt, gp, inv)
    dec = [decode(int(c)) for c in tasks]
    if gp == 1:
        assert len(off) == 2
        return dec, [], 0  # one block: its list as the "chain"
    assert len(off) == 3
    return dec[off[0]:off[1]], dec[off[1]:off[2]], gp - 1


@pytest.mark.parametrize("nt,gp,inv", [(1, 1, None), (2, 1, None), (3, 2, None), (5, 32, None), (16, 32, None),
                                       (16, 7, None), (20, 32, None), (24, 48, None), (25, 48, None),
                                       (40, 96, None), (70, 384, None),
                                       # the chains of a multi-chain pass leave L^-1 out at any size
                                       (1, 1, False), (3, 2, False), (16, 32, False), (16, 7, False),
                                       # and a forced inverse beyond 24 tiles
                                       (25, 48, True)])
def test_schedule_covers_every_task_and_never_deadlocks(nt, gp, inv):
    tasks, off = hsp.hsp_tile_schedule(nt, gp, inv)
    assert off[0] == 0 and off[-1] == len(tasks) and np.all(np.diff(off.astype(np.int64)) >= 0)
    chain_list, queue, nqb = lists_of(nt, gp, inv)
    dec = chain_list + queue
    chain = gp > 1
    assert len(dec) == len(set(dec)) and set(dec) == expected_tasks(nt, chain, inv)
    if chain:  # block 0 runs the critical chain, in order, and nothing else
        assert chain_list == [(POTRF, 0, 0, 0, 0)] + [(PANEL, 0, k, k, k) for k in range(1, nt)]
    rng = np.random.default_rng(nt * 100 + gp)
    for _ in range(5 if nt < 16 else 2):
        replay(chain_list, queue, nqb, nt, rng, inv)


def test_schedule_shortens_with_more_blocks():
    """The critical path is fixed; more blocks only help until it dominates."""
    spans = {}
    for gp in (2, 4, 32):
        chain_list, queue, nqb = lists_of(16, gp)
        spans[gp] = np.mean([replay(chain_list, queue, nqb, 16, np.random.default_rng(s))
                             for s in range(2)])
    assert spans[32] < spans[4] < spans[2]


def test_schedule_beyond_127_tiles():
    """p = 10,000 (157 tiles per side, a group of 384 blocks): every task once
    (the factorisation without L^-1, beta by substitution), its fields
    decoded intact, and the critical chain in order."""
    nt, gp = 157, 384
    tasks, off = hsp.hsp_tile_schedule(nt, gp)
    chain_list, queue, _ = lists_of(nt, gp)
    dec = chain_list + queue
    assert len(dec) == len(set(dec)) and set(dec) == expected_tasks(nt, True)
    assert chain_list == [(POTRF, 0, 0, 0, 0)] + [(PANEL, 0, k, k, k) for k in range(1, nt)]


def test_schedule_rejects_bad_arguments():
    with pytest.raises(hsp.HspError):
        hsp.hsp_tile_schedule(0, 4)
    with pytest.raises(hsp.HspError):
        hsp.hsp_tile_schedule(hsp.hsp_max_p() // 64 + 1, 4)
    with pytest.raises(hsp.HspError):
        hsp.hsp_tile_schedule(4, 0)
    with pytest.raises(hsp.HspError):
        load_raw = hsp.load()
        n = hsp.C.c_int64()
        hsp._check(load_raw.hsp_tile_schedule(4, 2, 2, None, 0, None, hsp.C.byref(n)))
