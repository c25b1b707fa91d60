"""A model of the tracking kernel's work taking in batch launches, checked on random
launches on the CPU: per-problem work counters, a wave's home problem and its one
pass over the others once its problem runs out, chunks of one problem gathered into
the batch of the current slot up to the problem's batch size, a chunk that cannot
join waiting for a free slot, one or two slots per wave, hand-out of histories to
idle lanes at a refill threshold, per-lane sums moved to the slot when a lane takes a
history of another chunk, and the flush of a slot once its batch is handed out and its
last history ended. The model follows the kernel's rules step by step (waves take
turns at random); it checks that every history runs exactly once, that a flushed
batch holds exactly the histories counted for it, that no batch exceeds its size
limit, that a lane's unmoved sums never span two chunks, and that every wave leaves."""
from __future__ import annotations

import random

import pytest


def run_launch(hist, chunks, batch_max, waves, slots, refill, seed, max_len=120, move_at_chunk_change=True):
    rng = random.Random(seed)
    n = len(hist)
    items = [(h + c - 1) // c for h, c in zip(hist, chunks)]
    starts = [0]
    for it in items:
        starts.append(starts[-1] + it)
    head = [0] * n
    ran = [[0] * h for h in hist]
    flushed = [0] * n

    class Slot:
        def __init__(self):
            self.h0 = self.cnt = self.next = self.live = self.pid = self.open = 0

        def copy(self):
            t = Slot()
            t.__dict__.update(self.__dict__)
            return t

    W = []
    for w in range(waves):
        t = w * starts[n] // waves
        home = max(i for i in range(n) if starts[i] <= t)
        W.append(dict(C=Slot(), O=Slot(), cp=0, empty=False, home=home, pend=None,
                      lanes=[dict(alive=False, h=None, pid=None, slot=0, rem=0, sums=set()) for _ in range(64)],
                      buf=[set(), set()], total=[0, 0]))

    def claim(wv):
        # the home problem's counter, then the others in order, once
        p = wv["home"]
        got = head[p]
        head[p] += 1
        if got < items[p]:
            return got
        for off in range(1, n):
            q = (p + off) % n
            if head[q] < items[q]:          # a read at or beyond the count proves it empty
                got = head[q]
                head[q] += 1
                if got < items[q]:
                    wv["home"] = q
                    return got
        return None

    def to_slot(wv, lane):
        if lane["sums"]:
            assert len({(pid, h // chunks[pid]) for pid, h in lane["sums"]}) == 1, "a lane's sums span two chunks"
            wv["buf"][lane["slot"]] |= lane["sums"]
        lane["sums"] = set()

    def flush(wv, S, b):
        assert len(wv["buf"][b]) == wv["total"][b]
        assert wv["total"][b] <= max(batch_max[S.pid], chunks[S.pid])
        for pid, h in wv["buf"][b]:
            assert pid == S.pid
            ran[pid][h] += 1
        flushed[S.pid] += wv["total"][b]
        wv["buf"][b] = set()
        S.open = 0

    active = list(range(waves))
    steps = 0
    while active:
        steps += 1
        assert steps < 20_000_000, "a wave never leaves"
        w = rng.choice(active)
        wv = W[w]
        C, O, lanes = wv["C"], wv["O"], wv["lanes"]
        dead = [i for i, ln in enumerate(lanes) if not ln["alive"]]
        if dead and (len(dead) == 64 or len(dead) >= refill):
            if not C.open or C.next == C.cnt:
                pend = wv["pend"]
                if pend is None and not wv["empty"]:
                    pend = claim(wv)
                    if pend is None:
                        wv["empty"] = True
                if pend is not None:
                    hp = wv["home"]
                    first = pend * chunks[hp]
                    cnt = min(hist[hp] - first, chunks[hp])
                    total = wv["total"][wv["cp"]] if C.open else 0
                    if C.open and C.pid == hp and total + cnt <= batch_max[hp]:
                        C.h0, C.cnt, C.next = first, cnt, 0
                        wv["total"][wv["cp"]] = total + cnt
                        pend = None
                    elif not C.open or (slots == 2 and not O.open):
                        if C.open:
                            wv["O"] = O = C.copy()
                            wv["cp"] ^= 1
                        C.h0, C.cnt, C.next, C.live, C.pid, C.open = first, cnt, 0, 0, hp, 1
                        wv["total"][wv["cp"]] = cnt
                        pend = None
                wv["pend"] = pend
            if C.open and C.next < C.cnt:
                take = min(C.cnt - C.next, len(dead))
                for r, i in enumerate(dead[:take]):
                    ln = lanes[i]
                    in_chunk = ln["h"] is not None and ln["pid"] == C.pid and 0 <= ln["h"] - C.h0 < C.cnt
                    if ln["slot"] != wv["cp"] or (move_at_chunk_change and not in_chunk):
                        to_slot(wv, ln)
                    ln.update(slot=wv["cp"], h=C.h0 + C.next + r, pid=C.pid, alive=True,
                              rem=rng.randint(1, max_len) if rng.random() < 0.9 else rng.randint(1, 20 * max_len))
                C.next += take
                C.live += take
        if all(not ln["alive"] for ln in lanes) and not C.open and not O.open and wv["empty"]:
            assert wv["pend"] is None
            active.remove(w)
            continue
        fin_c = fin_o = 0
        for ln in lanes:
            if ln["alive"]:
                ln["rem"] -= 1
                if ln["rem"] == 0:
                    ln["alive"] = False
                    ln["sums"].add((ln["pid"], ln["h"]))
                    if ln["slot"] == wv["cp"]:
                        fin_c += 1
                    else:
                        fin_o += 1
        if fin_c or fin_o:
            C.live -= fin_c
            O.live -= fin_o
            assert C.live >= 0 and O.live >= 0
            if C.open and C.next == C.cnt and C.live == 0:
                for ln in lanes:
                    if ln["slot"] == wv["cp"]:
                        to_slot(wv, ln)
                flush(wv, C, wv["cp"])
            if O.open and O.next == O.cnt and O.live == 0:
                for ln in lanes:
                    if ln["slot"] == wv["cp"] ^ 1:
                        to_slot(wv, ln)
                flush(wv, O, wv["cp"] ^ 1)
    for p in range(n):
        assert all(v == 1 for v in ran[p]), f"problem {p}: a history ran {set(ran[p])} times"
        assert flushed[p] == hist[p]


@pytest.mark.parametrize("seed", range(6))
def test_every_history_runs_once_and_every_wave_leaves(seed):
    rng = random.Random(4242 + seed)
    n = rng.randint(1, 9)
    hist = [rng.randint(1, 3000) for _ in range(n)]
    chunks = [rng.choice([1, 7, 64, 256]) for _ in range(n)]
    batch_max = [max(c, h // 256) if rng.random() < 0.8 else c for h, c in zip(hist, chunks)]
    run_launch(hist, chunks, batch_max, waves=rng.randint(1, 12), slots=1 + seed % 2,
               refill=rng.choice([1, 4, 16, 64]), seed=seed)


def test_the_model_sees_sums_that_span_chunks():
    """Without the move of a lane's sums when it takes a history of another chunk of
    the same batch, a lane's sums span chunks (the 32-bit bound of its counts no
    longer holds): the model must catch it."""
    with pytest.raises(AssertionError, match="span two chunks"):
        run_launch([3000], [64], [3000 // 4], waves=2, slots=1, refill=4, seed=1, move_at_chunk_change=False)
