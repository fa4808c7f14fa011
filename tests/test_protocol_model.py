"""Step-interleaved model of the runtime's queue protocols (Sec. 5.1.3):
the batched deque of thread mode (PushBatch, PopBatch, StealBatch with the
thieves' lock), the Chase-Lev deque of block mode and the centralised FIFO
queue of the scheduler comparison.

Each wavefront (workgroup, for Chase-Lev) is a Python generator that performs
one shared-memory access per step -- a load, a store, a CAS or a fetch-add on
the words the kernels share (count, head, lock, tail, top, bottom, ring
slots) -- and yields.  A seeded scheduler picks which one takes the next
step, so every interleaving of those accesses is reachable.  The kernels issue
each dependent access only after the previous one completed (drain(), or a
use of its result), which is what makes this interleaving model apply; the
hardware side of that claim is the GPU litmus test.  The model is written
from the kernels' protocol, not shared with them.

A task tree with a fixed number of tasks is executed on tiny deques
(capacity 8, up to 4 lanes per wavefront) so that wrap-around, empty and full
deques, and races between the owner and several thieves are frequent; every
run must execute each task exactly once and leave every deque consistent.
Planted protocol mistakes must be caught by some seed.
"""
import random

import pytest


class Tree:
    """Deterministic task tree: task (d, i) at depth < D has 1 + (i*7+d) % 3 children."""

    def __init__(self, depth):
        self.depth = depth
        self.next_id = 0
        self.meta = {}
        self.created = 0

    def new(self, d):
        t = self.next_id
        self.next_id += 1
        self.meta[t] = d
        self.created += 1
        return t

    def children(self, t):
        d = self.meta[t]
        if d >= self.depth:
            return []
        return [self.new(d + 1) for _ in range(1 + (t * 7 + d) % 3)]


def run_schedule(actors, rng, max_steps):
    live = list(actors)
    steps = 0
    while live and steps < max_steps:
        a = rng.choice(live)
        try:
            next(a)
        except StopIteration:
            live.remove(a)
        steps += 1
    return not live


# ---- thread mode: batched deque ------------------------------------------------
class BatchedDeques:
    def __init__(self, nwaves, cap, planted=None):
        self.cap = cap
        self.count = [0] * nwaves
        self.head = [0] * nwaves
        self.lock = [0] * nwaves
        self.ring = [[-1] * cap for _ in range(nwaves)]
        # owner-private (LDS) state
        self.tail = [0] * nwaves
        self.head_seen = [0] * nwaves
        self.hint = [0] * nwaves
        self.planted = planted

    def push_batch(self, me, ids):
        n = len(ids)
        t = self.tail[me]
        if t + n - self.head_seen[me] > self.cap:
            h = self.head[me]
            yield
            self.head_seen[me] = h
            if t + n - h > self.cap:
                return False
        for i, x in enumerate(ids):
            self.ring[me][(t + i) % self.cap] = x
            yield
        self.tail[me] = t + n
        self.hint[me] = 1
        self.count[me] += n          # one atomic add after the slots completed
        yield
        return True

    def pop_batch(self, me, want):
        if not self.hint[me]:
            return []
        c = self.count[me]
        yield
        take = 0
        while True:
            if c <= 0:
                self.hint[me] = 0
                return []
            take = min(c, want)
            if self.planted == "pop_store":      # read-modify-write without CAS
                self.count[me] = c - take
                yield
                break
            cur = self.count[me]                 # CAS(count, c, c - take)
            if cur == c:
                self.count[me] = c - take
                yield
                break
            c = cur
            yield
        if take == c:
            self.hint[me] = 0
        t = self.tail[me] - take
        out = []
        for i in range(take):
            out.append(self.ring[me][(t + i) % self.cap])
            yield
        self.tail[me] = t
        return out

    def steal_batch(self, me, victim, want, div):
        c = self.count[victim]               # probe
        yield
        if c <= 0:
            return []
        if self.planted != "no_lock":
            if self.lock[victim] != 0:           # CAS(lock, 0, 1) failed
                yield
                return []
            self.lock[victim] = 1
            yield
        h = self.head[victim]
        yield
        cc, claim = c, 0
        while cc > 0:
            take = min(-(-cc // div), want)
            cur = self.count[victim]
            if cur == cc:
                self.count[victim] = cc - take
                claim = take
                yield
                break
            cc = cur
            yield
        if claim == 0:
            if self.planted != "no_lock":
                self.lock[victim] = 0
                yield
            return []
        if self.planted == "head_first":         # head moves before the slots are read
            self.head[victim] = h + claim
            yield
        out = []
        for i in range(claim):
            out.append(self.ring[victim][(h + i) % self.cap])
            yield
        if self.planted != "head_first":
            self.head[victim] = h + claim
            yield
        if self.planted != "no_lock":
            self.lock[victim] = 0
            yield
        return out


def batched_run(seed, nwaves=3, lanes=4, cap=8, depth=6, steal_div=2, planted=None, max_steps=400000):
    rng = random.Random(seed)
    tree = Tree(depth)
    dq = BatchedDeques(nwaves, cap, planted)
    executed = {}
    state = {"live": 0}
    roots = [tree.new(0) for _ in range(3)]
    state["live"] = len(roots)

    def wave(me):
        local = list(roots) if me == 0 else []   # private stack (newest last)
        wrng = random.Random(seed * 1000 + me)
        while True:
            lanes_ = []
            while local and len(lanes_) < lanes:
                lanes_.append(local.pop())
            if len(lanes_) < lanes:
                lanes_ += (yield from dq.pop_batch(me, lanes - len(lanes_)))
            if not lanes_ and nwaves > 1:
                v = wrng.randrange(nwaves - 1)
                v += v >= me
                lanes_ += (yield from dq.steal_batch(me, v, lanes, steal_div))
            if not lanes_:
                if state["live"] == 0:
                    return
                yield
                continue
            for t in lanes_:
                executed[t] = executed.get(t, 0) + 1
                kids = tree.children(t)
                state["live"] += len(kids) - 1
                local += kids
            # expose the oldest private entries to the deque when it has room
            if len(local) > 2:
                n = min(len(local) - 2, lanes)
                if (yield from dq.push_batch(me, local[:n])):
                    del local[:n]

    finished = run_schedule([wave(w) for w in range(nwaves)], rng, max_steps)
    return finished, tree, executed, dq


@pytest.mark.parametrize("seed", range(200))
def test_batched_deque_exactly_once(seed):
    nwaves = 2 + seed % 3
    finished, tree, executed, dq = batched_run(seed, nwaves=nwaves, steal_div=1 + seed % 2)
    assert finished, "schedule did not terminate"
    assert len(executed) == tree.created and all(v == 1 for v in executed.values())
    for w in range(nwaves):
        assert dq.count[w] == 0 and dq.lock[w] == 0 and dq.tail[w] == dq.head[w]


@pytest.mark.parametrize("planted", ["pop_store", "no_lock", "head_first"])
def test_batched_deque_planted_mistakes_are_caught(planted):
    bad = 0
    for seed in range(300):
        finished, tree, executed, _ = batched_run(seed, nwaves=3, planted=planted, max_steps=100000)
        if not finished or len(executed) != tree.created or any(v != 1 for v in executed.values()):
            bad += 1
    assert bad > 0, planted


# ---- block mode: Chase-Lev deque -------------------------------------------------
class ChaseLev:
    def __init__(self, nw, cap, planted=None):
        self.cap = cap
        self.top = [0] * nw
        self.bottom = [0] * nw
        self.buf = [[-1] * cap for _ in range(nw)]
        self.b_own = [0] * nw        # owner's LDS copy of bottom
        self.top_seen = [0] * nw
        self.planted = planted

    def push(self, me, ids):
        n = len(ids)
        bot = self.b_own[me]
        if bot + n - self.top_seen[me] > self.cap:
            self.top_seen[me] = self.top[me]
            yield
            if bot + n - self.top_seen[me] > self.cap:
                return False
        for i, x in enumerate(ids):
            self.buf[me][(bot + i) % self.cap] = x
            yield
        self.bottom[me] = bot + n
        yield
        self.b_own[me] = bot + n
        return True

    def pop(self, me):
        b = self.b_own[me] - 1
        if b < self.top_seen[me]:
            return None
        self.bottom[me] = b               # atomic exchange, completed before top is read
        yield
        t = self.top[me]
        yield
        self.top_seen[me] = t
        if t > b:
            self.bottom[me] = b + 1
            yield
            return None
        x = self.buf[me][b % self.cap]
        yield
        if t == b:
            won = self.top[me] == t       # CAS(top, t, t + 1)
            if won:
                self.top[me] = t + 1
            yield
            self.bottom[me] = b + 1
            yield
            self.top_seen[me] = t + 1
            return x if won else None
        self.b_own[me] = b
        return x

    def steal(self, v):
        if self.planted == "bottom_first":
            b = self.bottom[v]
            yield
            t = self.top[v]
            yield
        else:
            t = self.top[v]
            yield
            b = self.bottom[v]
            yield
        if t >= b:
            return None
        x = self.buf[v][t % self.cap]
        yield
        if self.top[v] == t:
            self.top[v] = t + 1
            yield
            return x
        yield
        return None


def chase_lev_run(seed, nw=3, cap=8, depth=6, planted=None, max_steps=400000):
    rng = random.Random(seed)
    tree = Tree(depth)
    cl = ChaseLev(nw, cap, planted)
    executed = {}
    state = {"live": 0}
    roots = [tree.new(0) for _ in range(2)]
    state["live"] = len(roots)

    def group(me):
        local = list(roots) if me == 0 else []
        grng = random.Random(seed * 7919 + me)
        while True:
            t = local.pop() if local else None
            if t is None:
                t = yield from cl.pop(me)
            if t is None and nw > 1:
                v = grng.randrange(nw - 1)
                v += v >= me
                t = yield from cl.steal(v)
            if t is None:
                if state["live"] == 0:
                    return
                yield
                continue
            executed[t] = executed.get(t, 0) + 1
            kids = tree.children(t)
            state["live"] += len(kids) - 1
            if kids:
                local.append(kids[0])         # child 0 runs next on this group
                rest = kids[1:]
                if rest and not (yield from cl.push(me, rest)):
                    local += rest

    finished = run_schedule([group(w) for w in range(nw)], rng, max_steps)
    return finished, tree, executed, cl


@pytest.mark.parametrize("seed", range(200))
def test_chase_lev_exactly_once(seed):
    nw = 2 + seed % 3
    finished, tree, executed, cl = chase_lev_run(seed, nw=nw)
    assert finished, "schedule did not terminate"
    assert len(executed) == tree.created and all(v == 1 for v in executed.values())
    for w in range(nw):
        assert cl.top[w] == cl.bottom[w]


def test_chase_lev_planted_mistake_is_caught():
    """A thief that reads bottom before top can take a task the owner popped."""
    bad = 0
    for seed in range(400):
        finished, tree, executed, _ = chase_lev_run(seed, nw=3, planted="bottom_first", max_steps=100000)
        if not finished or len(executed) != tree.created or any(v != 1 for v in executed.values()):
            bad += 1
    assert bad > 0


# ---- scheduler comparison: centralised queue ----------------------------------------
class CentralQueue:
    def __init__(self, cap, nwaves, lanes, planted=None):
        self.cap = cap
        self.tail = 0
        self.count = 0
        self.head = 0
        self.ring = [(-1, -1)] * cap     # (position tag, task id)
        self.room = cap - lanes * nwaves
        self.planted = planted

    def push(self, ids, spin_limit=50):
        n = len(ids)
        b = self.tail                    # fetch_add(tail, n)
        self.tail += n
        yield
        spins = 0
        while b + n - self.head > self.room:
            spins += 1
            if spins > spin_limit:
                return "capacity"
            yield
        for i, x in enumerate(ids):
            self.ring[(b + i) % self.cap] = (b + i, x)
            yield
        self.count += n
        yield
        return "ok"

    def pop(self, want, spin_limit=200):
        c = self.count
        yield
        claim = 0
        for _ in range(8):
            if c <= 0:
                break
            take = min(c, want)
            if self.count == c:
                self.count = c - take
                claim = take
                yield
                break
            c = self.count
            yield
        if claim == 0:
            return []
        pos = self.head                  # fetch_add(head, claim)
        self.head += claim
        yield
        out = []
        for i in range(claim):
            spins = 0
            while True:
                tag, x = self.ring[(pos + i) % self.cap]
                yield
                if tag == pos + i or self.planted == "no_tag":
                    out.append(x)
                    break
                spins += 1
                if spins > spin_limit:
                    return None
        return out


def central_run(seed, nwaves=3, lanes=2, cap=64, depth=6, planted=None, max_steps=400000):
    rng = random.Random(seed)
    tree = Tree(depth)
    cq = CentralQueue(cap, nwaves, lanes, planted)
    executed = {}
    state = {"live": 0, "error": None}
    roots = [tree.new(0) for _ in range(2)]
    state["live"] = len(roots)

    def wave(me):
        local = list(roots) if me == 0 else []
        while True:
            got = []
            while local and len(got) < lanes:
                got.append(local.pop())
            if not got:
                r = yield from cq.pop(lanes)
                if r is None:
                    state["error"] = "lost slot"
                    return
                got = r
            if not got:
                if state["live"] == 0 or state["error"]:
                    return
                yield
                continue
            for t in got:
                executed[t] = executed.get(t, 0) + 1
                if t not in tree.meta:       # a slot read before its push wrote it
                    state["error"] = "garbage"
                    return
                kids = tree.children(t)
                state["live"] += len(kids) - 1
                local += kids
            if len(local) > 1:
                n = min(len(local) - 1, lanes)
                r = yield from cq.push(local[:n])
                if r != "ok":
                    state["error"] = r
                    return
                del local[:n]

    finished = run_schedule([wave(w) for w in range(nwaves)], rng, max_steps)
    return finished, tree, executed, cq, state


@pytest.mark.parametrize("seed", range(150))
def test_central_queue_exactly_once(seed):
    finished, tree, executed, cq, state = central_run(seed, nwaves=2 + seed % 3)
    assert finished and state["error"] is None, state
    assert len(executed) == tree.created and all(v == 1 for v in executed.values())
    assert cq.count == 0 and cq.head == cq.tail


def test_central_queue_planted_mistake_is_caught():
    """A pop that takes whatever a slot holds, without checking its position
    tag, can read a position whose push has reserved it but not written it yet
    (a later push raised the count first)."""
    bad = 0
    for seed in range(300):
        finished, tree, executed, _, state = central_run(seed, nwaves=5, lanes=4, planted="no_tag",
                                                         max_steps=100000)
        if state["error"] == "garbage" or (finished and not state["error"] and (
                len(executed) != tree.created or any(v != 1 for v in executed.values()))):
            bad += 1
    assert bad > 0
