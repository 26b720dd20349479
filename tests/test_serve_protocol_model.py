"""CPU model of the serving loop's claim / report protocol (serve_loop and the
host's admit / reap), step by step, with any interleaving of the workgroups.

Each shared-memory access of the device code (thread 0 of a workgroup) and of
the host's descriptor writes is one step of a generator; a scheduler picks the
next step.  Invariants checked at the end of a run:
  * every tile of every request ran exactly once, with its own request's
    descriptor;
  * every request was completed (finalized) exactly once, after all its tiles;
  * nothing hung (the run ends within a step budget).

The scenario the protocol must survive: a workgroup stalls with its cursor on a
request that then completes; the host gives the slot to a later, larger
request; the stalled workgroup wakes up, reads the slot's descriptor and claims.
Reading the tile count without checking which request the descriptor holds
(``validate=False``, the earlier protocol) lets it claim a tile under the old
tag and run it with the new request's descriptor; the seqlock read
(``validate=True``, desc_ntiles in the kernel) sees that the slot has moved on.
"""
import collections
import random

import pytest

WRITING = float("inf")  # the descriptor's "being rewritten" marker (kDescWriting)


class Sim:
    def __init__(self, ntiles, slots, validate):
        self.ntiles_of = list(ntiles)
        self.slots = slots
        self.validate = validate
        self.published = 0
        self.desc = [dict(seq=-1, ntiles=0, target=0, rid=-1) for _ in range(slots)]
        self.claim = [(-1, 0)] * slots          # (request tag, tiles handed out)
        self.done = [0] * slots                 # cumulative tiles reported per slot
        self.slot_total = [0] * slots
        self.complete = [0] * slots             # seq + 1 of the last completed request
        self.runs = collections.Counter()       # (request, tile) -> times run
        self.finalized = collections.Counter()  # request -> times completed
        self.errors = []

    # -- host: admit requests in order as slots free up (reap = the complete flag) --
    def host(self):
        for seq, nt in enumerate(self.ntiles_of):
            s = seq % self.slots
            while seq >= self.slots and self.complete[s] < seq - self.slots + 1:
                yield "host_wait"
            d = self.desc[s]
            if self.validate:
                d["seq"] = WRITING
                yield "host_marker"
            else:
                d["seq"] = seq
                yield "host_seq"
            d["ntiles"] = nt
            yield "host_field"
            self.slot_total[s] += nt
            d["target"] = self.slot_total[s]
            yield "host_field"
            d["rid"] = seq
            yield "host_field"
            if self.validate:
                d["seq"] = seq
                yield "host_seq"
            self.published = seq + 1
            yield "host_published"

    # -- a workgroup's thread 0 (claims), with the tiles it runs --
    def worker(self, wid):
        slots, n_req = self.slots, len(self.ntiles_of)
        seq, pub, nt_seq, ntiles = 0, 0, None, 0
        cur, cur_seq, open_count = None, None, 0

        def report():
            nonlocal open_count
            s = cur_seq % slots
            self.done[s] += open_count  # one atomic add
            open_count = 0
            if self.done[s] == cur["target"]:
                rid = cur["rid"]
                missing = [t for t in range(self.ntiles_of[rid]) if self.runs[(rid, t)] == 0]
                if missing:
                    self.errors.append("request %d completed before tiles %s ran" % (rid, missing))
                self.finalized[rid] += 1
                self.complete[s] = cur_seq + 1

        while True:
            yield "top"
            if seq >= n_req:
                return
            if seq >= pub and self.published > pub:
                pub = self.published
            if seq >= pub:
                continue
            s = seq % slots
            if nt_seq != seq:
                yield ("before_ntiles", seq)
                if self.validate:
                    a = self.desc[s]["seq"]
                    yield "read"
                    nt = self.desc[s]["ntiles"]
                    yield "read"
                    b = self.desc[s]["seq"]
                    yield "read"
                    if not (a == seq and b == seq):
                        if open_count and cur_seq == seq:
                            report()
                        seq += 1
                        continue
                else:
                    nt = self.desc[s]["ntiles"]
                    yield "read"
                ntiles, nt_seq = nt, seq
            v = self.claim[s]
            yield "read"
            got, moved_on = None, False
            while True:
                vs, vc = v
                if vs > seq:
                    moved_on = True
                    break
                if vs < seq:  # compare-and-swap (one atomic step)
                    if self.claim[s] == v:
                        self.claim[s] = (seq, 1)
                        got = (seq, 0)
                        break
                    v = self.claim[s]
                    yield "cas_retry"
                    continue
                if vc >= ntiles:
                    moved_on = True
                    break
                w = self.claim[s]  # fetch_add (one atomic step)
                self.claim[s] = (w[0], w[1] + 1)
                yield "fetch_add"
                ws, wc = w
                if ws == seq:
                    if wc < ntiles:
                        got = (seq, wc)
                    else:
                        moved_on = True
                    break
                later = ws  # a later request took the slot: tile wc is one of its
                seq, pub = later, max(pub, later + 1)
                if self.validate:
                    held, lnt = False, 0
                    while True:
                        ds = self.desc[s]["seq"]
                        yield "read"
                        if ds != WRITING and ds < later:
                            continue
                        a = self.desc[s]["seq"]
                        yield "read"
                        lnt = self.desc[s]["ntiles"]
                        yield "read"
                        b = self.desc[s]["seq"]
                        yield "read"
                        held = a == later and b == later
                        if held or ds != later:
                            break
                else:
                    lnt = self.desc[s]["ntiles"]
                    yield "read"
                    held = True
                nt_seq, ntiles = (later, lnt) if held else (None, 0)
                if held and wc < lnt:
                    got = (later, wc)
                else:
                    moved_on = True
                break
            if got is not None:
                if got[0] != cur_seq:
                    d = self.desc[got[0] % slots]
                    cur = dict(rid=d["rid"])
                    yield "copy"
                    cur["target"] = d["target"]
                    yield "copy"
                    cur_seq = got[0]
                open_count += 1
                if cur["rid"] != got[0]:
                    self.errors.append("workgroup %d ran tile %d of request %d with request %d's descriptor"
                                       % (wid, got[1], got[0], cur["rid"]))
                self.runs[(cur["rid"], got[1])] += 1
                yield "tile"
                continue
            if moved_on:
                if open_count and cur_seq == seq:
                    report()
                seq += 1

    def check(self, hung):
        errs = list(self.errors)
        if hung:
            errs.append("hung: requests not completed %s"
                        % [r for r in range(len(self.ntiles_of)) if self.finalized[r] == 0])
        for r, nt in enumerate(self.ntiles_of):
            for t in range(nt):
                if self.runs[(r, t)] != 1:
                    errs.append("request %d tile %d ran %d times" % (r, t, self.runs[(r, t)]))
            if self.finalized[r] != 1:
                errs.append("request %d completed %d times" % (r, self.finalized[r]))
        return errs


def run(sim, nworkers, rng, stall=None, max_steps=200000):
    """Random interleaving.  stall = (worker, seq, wake): that worker is held at
    the point where it is about to read request seq's descriptor until wake(sim)
    holds, then runs alone for a while."""
    gens = {"host": sim.host()}
    for w in range(nworkers):
        gens[w] = sim.worker(w)
    held, solo = set(), 0
    steps = 0
    while gens and steps < max_steps:
        steps += 1
        if stall is not None and stall[0] in held and stall[2](sim):
            held.discard(stall[0])
            solo = 40
        runnable = [k for k in gens if k not in held]
        if not runnable:
            break
        key = stall[0] if (solo > 0 and stall[0] in gens) else rng.choice(runnable)
        solo = max(0, solo - 1)
        try:
            tag = next(gens[key])
        except StopIteration:
            del gens[key]
            continue
        if stall is not None and key == stall[0] and tag == ("before_ntiles", stall[1]) and stall[2] is not None:
            if not stall[2](sim):
                held.add(key)
    return sim.check(hung=bool(gens))


def stalled_case(validate, seed):
    """One slot: request 0 (2 tiles) completes while workgroup 0 sleeps on it;
    request 1 (5 tiles) takes the slot; workgroup 0 wakes as soon as request 1 is
    published, before anyone claims it."""
    sim = Sim([2, 5, 3], slots=1, validate=validate)
    return run(sim, 3, random.Random(seed), stall=(0, 0, lambda s: s.published >= 2))


def test_stalled_workgroup_breaks_the_unchecked_descriptor_read():
    errs = stalled_case(validate=False, seed=1)
    assert errs, "the earlier protocol should fail this interleaving"
    assert any("descriptor" in e or "ran 2 times" in e or "hung" in e or "before tiles" in e for e in errs)


@pytest.mark.parametrize("seed", range(20))
def test_stalled_workgroup_with_seqlock_read(seed):
    assert stalled_case(validate=True, seed=seed) == []


@pytest.mark.parametrize("slots,nworkers", [(1, 2), (2, 3), (3, 5), (4, 8)])
def test_random_interleavings_with_seqlock_read(slots, nworkers):
    """Many uneven requests through few slots, random schedules."""
    for seed in range(60):
        rng = random.Random(1000 * slots + seed)
        ntiles = [rng.randint(1, 7) for _ in range(14)]
        sim = Sim(ntiles, slots=slots, validate=True)
        errs = run(sim, nworkers, rng)
        assert errs == [], (seed, ntiles, errs)
