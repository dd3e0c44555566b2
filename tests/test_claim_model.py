"""CPU model of the digit pass's tile claiming (claim_tile and the persistent
loop of run_pass), explored over random interleavings: every claimed tile is
eventually processed, with no deadlock, for any schedule.

The model keeps what decides progress and drops the arithmetic:
  * each XCD has a claim counter; claim k is tile k % G of the XCD's group
    k / G; the claim with k % G == 0 opens the group by taking the next id
    from a global counter and publishing it; other claims of the group wait
    for the id;
  * ahead = 0 is the shipped kernel: a workgroup claims one tile, processes
    it, then claims the next; ahead = 2 is a claim-ahead schedule: two tiles
    claimed at the start, then one more during every tile's look-back;
  * a tile's look-back can finish once every lower tile has been started
    (its aggregate is published when its holder ranks it; inclusive values
    follow by induction);
  * only workgroups that are resident make claims, and only some of each
    XCD's workgroups may be resident (other kernels hold the rest);
  * flat = True is the arrival-order claim of passes of few tiles: one
    global counter, no groups.
Every atomic step is its own scheduling point, so an opener can be delayed
between its two atomics.  The race between openers of one XCD is what the
ordered opening (an opener takes its global id only after the XCD's previous
group is open) excludes; without it the model finds deadlocks and tiles that
no workgroup ever processes."""
import random

import pytest

NO_TILE = -1


class Model:
    def __init__(self, xcds, wgs_per_xcd, tiles, group, ordered, seed, ahead=2, flat=False):
        self.rng = random.Random(seed)
        self.flat = flat   # one global counter, tiles in arrival order (no groups)
        self.G = group
        self.tiles = tiles
        self.ngroups = (tiles + group - 1) // group
        self.ordered = ordered
        self.claims = [0] * xcds                           # per-XCD claim counters
        self.lists = [[0] * self.ngroups for _ in range(xcds)]  # published group id + 1
        self.ctr = 0                                       # global group counter
        self.started = [False] * tiles
        self.finished = [False] * tiles
        self.wgs = []
        for x in range(xcds):
            for _ in range(wgs_per_xcd):
                self.wgs.append({"x": x, "held": [], "claim": None, "state": "prologue",
                                 "cur": None, "need": max(ahead, 1), "done": False})
        self.ahead = ahead

    # one claim is a small state machine: counter -> (open | wait) -> tile
    def claim_step(self, wg):
        c = wg["claim"]
        x = wg["x"]
        if self.flat:
            t = self.ctr
            self.ctr += 1
            return t if t < self.tiles else NO_TILE
        if c["phase"] == "count":
            k = self.claims[x]
            self.claims[x] += 1
            c["k"], c["j"], c["i"] = k, k // self.G, k % self.G
            if c["j"] >= self.ngroups:
                return NO_TILE
            c["phase"] = "open" if c["i"] == 0 else "wait"
            return None
        if c["phase"] == "open":
            j = c["j"]
            if self.ordered and j > 0:
                prev = self.lists[x][j - 1]
                if prev == 0:
                    return None                   # the previous group is not open yet
                if prev == NO_TILE:
                    self.lists[x][j] = NO_TILE
                    return NO_TILE
            g = self.ctr
            self.ctr += 1
            v = g + 1 if g < self.ngroups else NO_TILE
            self.lists[x][j] = v
            c["v"] = v
        else:
            v = self.lists[x][c["j"]]
            if v == 0:
                return None                       # waiting for the opener
            c["v"] = v
        if c["v"] == NO_TILE:
            return NO_TILE
        t = (c["v"] - 1) * self.G + c["i"]
        if t < self.tiles:
            return t
        c["phase"] = "count"                      # past the end of a short last group
        return None

    def step(self, wg):
        """Advance one workgroup by one scheduling point; False if blocked."""
        if wg["done"]:
            return False
        if wg["claim"] is not None:
            r = self.claim_step(wg)
            if r is None:
                return wg["claim"]["phase"] != "wait" or self.lists[wg["x"]][wg["claim"]["j"]] != 0
            wg["claim"] = None
            wg["held"].append(r)
            wg["need"] -= 1
            return True
        if wg["need"] > 0:
            wg["claim"] = {"phase": "count"}
            return True
        if wg["cur"] is None:
            t = wg["held"].pop(0)
            if t == NO_TILE:
                wg["done"] = True
                return True
            wg["cur"] = t
            self.started[t] = True                # ranked: aggregate published
            if self.ahead:
                wg["need"] = 1                    # claim during the look-back
            return True
        t = wg["cur"]
        if all(self.started[:t]):
            self.finished[t] = True
            wg["cur"] = None
            if not self.ahead:
                wg["need"] = 1                    # claim the next tile now
            return True
        return False

    def run(self, max_steps=200000):
        for _ in range(max_steps):
            if all(w["done"] for w in self.wgs):
                return "ok"
            order = list(range(len(self.wgs)))
            self.rng.shuffle(order)
            progressed = False
            for i in order[: self.rng.randint(1, 3)]:
                progressed |= self.step(self.wgs[i])
            if not progressed and not any(self.step(w) for w in self.wgs):
                return "deadlock"
        return "timeout"


def explore(ordered, seeds, **kw):
    """Outcomes over seeds: ok, deadlock, timeout, or lost (every workgroup
    exited but a tile was never processed)."""
    out = {"ok": 0, "deadlock": 0, "timeout": 0, "lost": 0}
    for s in seeds:
        m = Model(ordered=ordered, seed=s, **kw)
        r = m.run()
        if r == "ok" and not all(m.finished):
            r = "lost"
        out[r] += 1
    return out


SHAPES = [
    dict(xcds=2, wgs_per_xcd=2, tiles=40, group=4),
    dict(xcds=3, wgs_per_xcd=1, tiles=30, group=4),
    dict(xcds=2, wgs_per_xcd=6, tiles=96, group=4),
    dict(xcds=2, wgs_per_xcd=10, tiles=37, group=8),   # fewer tiles than claims at the start
    dict(xcds=4, wgs_per_xcd=5, tiles=150, group=8),
    dict(xcds=1, wgs_per_xcd=9, tiles=20, group=4),
]


@pytest.mark.parametrize("ahead", [0, 2])
@pytest.mark.parametrize("shape", SHAPES)
def test_ordered_opening_processes_every_tile(shape, ahead):
    r = explore(True, range(200), ahead=ahead, **shape)
    assert r == {"ok": 200, "deadlock": 0, "timeout": 0, "lost": 0}, r


@pytest.mark.parametrize("shape", SHAPES)
def test_flat_claims_process_every_tile(shape):
    """Passes of few tiles (and 32-bit keys alone) claim from one global
    counter in arrival order: every claimed tile is held by a running
    workgroup, so every tile is processed under any schedule."""
    r = explore(True, range(200), ahead=0, flat=True, **shape)
    assert r == {"ok": 200, "deadlock": 0, "timeout": 0, "lost": 0}, r


def test_unordered_opening_fails():
    """The model has teeth: with openers free to race, a later group of an
    XCD can get a lower id than an earlier one; then a workgroup may exit on
    an empty claim while a later claim of its XCD holds a real tile (never
    processed), or hold a higher tile while waiting for a lower, unclaimed
    one."""
    r = explore(False, range(300), xcds=2, wgs_per_xcd=6, tiles=96, group=4)
    assert r["lost"] + r["deadlock"] > 0, r
