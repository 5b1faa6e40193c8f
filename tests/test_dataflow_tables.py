"""CPU checks of the dataflow executor's dependency tables: an event
simulation of the protocol with several workers must run every tile step,
never deadlock, and give every block of x exactly the schedule's sequence of
touches (which is what makes the result equal to the serial order)."""
import heapq

import numpy as np
import pytest

import oracle


def block_id(A, B):
    return B * (B + 1) // 2 + A


def schedule_touch_sequences(n, b):
    """Per block of x: the sequence of (tile, step) touches in the oracle's
    visiting order (tiles by first visit, steps by middle block)."""
    rows = oracle.schedule(n, b)
    seq = {}
    tiles = []
    last = None
    for i, j, k, r, P, J, t in rows:
        Q = k // b
        key = (int(P), int(Q))
        if last != (key, int(J)):
            if not tiles or tiles[-1] != key:
                tiles.append(key)
            for blk in {block_id(P, J), block_id(J, Q), block_id(P, Q)}:
                seq.setdefault(blk, []).append((key, int(J)))
            last = (key, int(J))
    return tiles, seq


def simulate(tab, b, nb, workers, sweeps=2):
    """Workers take tiles by ticket; a tile waits for block (P,Q), each step
    for its A and B blocks; steps cost one time unit.  Returns the makespan
    and per-block touch logs."""
    tpq, needc, jsb, needs, K = tab["tile_pq"], tab["need_c"], tab["jsbase"], tab["needs"], tab["K"]
    ntiles = len(tpq)
    cnt = np.zeros(len(K), dtype=np.int64)
    log = {}
    # state per worker: (tile ticket, step index m or -1 before the C wait)
    time = 0
    tickets = 0
    total = ntiles * sweeps
    busy = [None] * workers
    done = 0
    while done < total:
        progressed = False
        for w in range(workers):
            if busy[w] is None:
                if tickets >= total:
                    continue
                busy[w] = [tickets, -1]
                tickets += 1
            tk, m = busy[w]
            ep, t = divmod(tk, ntiles)
            P, Q = int(tpq[t, 0]), int(tpq[t, 1])
            desc = P + Q < nb
            C = block_id(P, Q)
            if m == -1:
                if cnt[C] >= ep * K[C] + needc[t]:
                    busy[w][1] = 0
                    progressed = True
                continue
            J = Q - m if desc else P + m
            A = block_id(P, J) if J != Q else -1
            B = block_id(J, Q) if J != P else -1
            na, nbn = needs[jsb[t] + m]
            if (A < 0 or cnt[A] >= ep * K[A] + na) and (B < 0 or cnt[B] >= ep * K[B] + nbn):
                for X in (A, B):
                    if X >= 0:
                        assert cnt[X] == ep * K[X] + (na if X == A else nbn)
                        log.setdefault(X, []).append(((P, Q), J))
                        cnt[X] += 1
                log.setdefault(C, []).append(((P, Q), J))
                progressed = True
                if m == Q - P:
                    cnt[C] += Q - P + 1
                    busy[w] = None
                    done += 1
                else:
                    busy[w][1] = m + 1
        assert progressed, "deadlock"
        time += 1
    return time, log


@pytest.mark.parametrize("n,b,workers", [(20, 8, 1), (20, 8, 3), (61, 8, 5), (70, 16, 2),
                                         (100, 8, 16), (47, 16, 64), (33, 8, 4), (65, 32, 3),
                                         (50, 24, 2), (73, 24, 5)])
def test_dataflow_tables_respect_the_schedule(n, b, workers):
    from paper_1901_10084_amd import ccproj as C
    tab = C.dataflow_tables(n, b)
    nb = -(-n // b)
    tiles, seq = schedule_touch_sequences(n, b)
    # the tables list tiles in the oracle's order (plus tiles without triplets)
    table_tiles = [tuple(int(v) for v in pq) for pq in tab["tile_pq"]]
    pos = [table_tiles.index(t) for t in tiles]
    assert pos == sorted(pos)
    steps = {st for s in seq.values() for st in s}
    _, log = simulate(tab, b, nb, workers, sweeps=2)
    for blk, s in seq.items():
        got = [st for st in log[blk] if st in steps]   # steps with at least one triplet
        # two sweeps: the schedule's sequence of touches, twice
        assert got == s + s, (blk, got[:6], s[:6])


def test_dataflow_depth_matches_analysis():
    """With unlimited workers the protocol's makespan is the dependency
    depth of the schedule (about 4 nb tile steps, versus nb^2 with barriers
    between rounds)."""
    from paper_1901_10084_amd import ccproj as C
    n, b = 256, 8
    nb = n // b
    tab = C.dataflow_tables(n, b)
    t, _ = simulate(tab, b, nb, workers=len(tab["tile_pq"]), sweeps=1)
    assert t <= 5 * nb, t
