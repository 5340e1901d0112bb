"""Host logic: the static task schedule of the tiled factorisation (p > 128).

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

POTRF, TRSM, GEMM = 0, 1, 2


def decode(c):
    return c & 3, (c >> 2) & 1, (c >> 3) & 127, (c >> 10) & 127, (c >> 17) & 127


def expected_tasks(nt):
    """Right-looking blocked Cholesky of [Q | I]: every tile operation once."""
    out = set()
    for k in range(nt):
        out.add((POTRF, 0, k, k, k))
        out.update((TRSM, 0, k, k, j) for j in range(k + 1, nt))
        out.update((TRSM, 1, k, k, j) for j in range(k))
        for i in range(k + 1, nt):
            out.update((GEMM, 0, k, i, j) for j in range(i, nt))
            out.update((GEMM, 1, k, i, j) for j in range(k + 1))
    return out


def reads_ok(t, vU, vL):
    typ, part, k, i, j = t
    if typ == POTRF:
        return vU[k, k] >= k
    if typ == TRSM:
        return vU[k, k] >= k + 1 and (vU[k, j] >= k if part == 0 else vL[k, j] >= k - j)
    if part == 0:
        return vU[k, i] >= k + 1 and vU[k, j] >= k + 1 and vU[i, j] >= k
    return vU[k, i] >= k + 1 and vL[k, j] >= k - j + 1 and vL[i, j] >= k - j


def write(t, vU, vL):
    typ, part, k, i, j = t
    if typ == POTRF:
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


def replay(lists, nt, rng):
    """Event simulation: each block runs its list in order, waiting on versions."""
    vU = np.zeros((nt, nt), np.int64)
    vL = np.zeros((nt, nt), np.int64)
    pos = [0] * len(lists)
    running = []  # heap of (finish time, block)
    busy = [False] * len(lists)
    now = 0.0
    left = sum(len(l) for l in lists)
    while left:
        for b, l in enumerate(lists):
            if not busy[b] and pos[b] < len(l) and reads_ok(l[pos[b]], vU, vL):
                dur = rng.uniform(0.3, 3.0) * (6.0 if l[pos[b]][0] == POTRF else 1.0)
                heapq.heappush(running, (now + dur, b))
                busy[b] = True
        assert running, f"deadlock with {left} tasks left"
        now, b = heapq.heappop(running)
        write(lists[b][pos[b]], vU, vL)
        pos[b] += 1
        busy[b] = False
        left -= 1
    for i in range(nt):
        for j in range(nt):
            if i <= j:
                assert vU[i, j] == i + 1
            if j <= i:
                assert vL[i, j] == i - j + 1
    return now


@pytest.mark.parametrize("nt,gp", [(1, 1), (2, 1), (3, 2), (5, 32), (16, 32), (16, 7), (20, 32)])
def test_schedule_covers_every_task_and_never_deadlocks(nt, gp):
    tasks, off = hsp.hsp_tile_schedule(nt, gp)
    assert off[0] == 0 and off[-1] == len(tasks) and np.all(np.diff(off.astype(np.int64)) >= 0)
    dec = [decode(int(c)) for c in tasks]
    assert len(dec) == len(set(dec)) and set(dec) == expected_tasks(nt)
    lists = [dec[off[b]:off[b + 1]] for b in range(gp)]
    rng = np.random.default_rng(nt * 100 + gp)
    for _ in range(5 if nt < 16 else 2):
        replay(lists, nt, rng)


def test_schedule_shortens_with_more_blocks():
    """The critical path is fixed; more blocks only help until it dominates."""
    spans = {}
    for gp in (1, 4, 32):
        tasks, off = hsp.hsp_tile_schedule(16, gp)
        dec = [decode(int(c)) for c in tasks]
        lists = [dec[off[b]:off[b + 1]] for b in range(gp)]
        spans[gp] = np.mean([replay(lists, 16, np.random.default_rng(s)) for s in range(2)])
    assert spans[32] < spans[4] < spans[1]


def test_schedule_rejects_bad_arguments():
    with pytest.raises(hsp.HspError):
        hsp.hsp_tile_schedule(0, 4)
    with pytest.raises(hsp.HspError):
        hsp.hsp_tile_schedule(65, 4)
    with pytest.raises(hsp.HspError):
        hsp.hsp_tile_schedule(4, 0)
