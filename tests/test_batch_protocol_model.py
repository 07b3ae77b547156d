"""A CPU model of one workgroup of the persistent batched kernel.

The persistent kernel runs every round of the batched solve (Sec. III-C:
start vector, Newton products with the two-term stop test, substep update)
in one launch: the workgroup builds the list of unfinished instances, takes
tiles from an atomic counter, meets the other workgroups at a grid barrier,
finalizes its instances and meets them again.  Inside the workgroup the
waves meet at hardware barriers that count arrivals of live waves wherever
they are in the program (s_barrier), so waves that take different branches
around a barrier pair the wrong barriers from then on.

The model runs each wave as a generator and steps them under a scheduler.
It shows:
* the finalize step as it was (every wave loads the instance's phase while
  the first wave may already have stored the next phase) lets a wave that
  loads late take the other branch; the waves then pair the wrong barriers,
  disagree on the round's tile count, and one wave keeps taking the tile
  loop on a tile index that no longer changes: a loop that no barrier
  time limit ends;
* with the phase loaded by every wave before a barrier that precedes the
  store, no schedule lets the waves diverge, and every instance finishes.
The schedules are adversarial: the late wave loads only after the store
whenever the barriers allow it; the other waves run in a seeded random
order.
"""
import pytest

START, FIRST, NEWTON, UPDATE, DONE = range(5)


class Stuck(Exception):
    pass


def run_model(fixed, waves=4, products=(3, 5, 2), substeps=(1, 2, 1), ntiles=(2, 3, 1),
              late_wave=1, max_rounds=200, loop_cap=1000, seed=None):
    import random
    rng = random.Random(seed)
    count = len(products)
    sites = {}                    # wave -> label of the barrier it waits at
    misaligned = [0]
    state = [dict(phase=FIRST, l=0, j=0) for _ in range(count)]
    shared = dict(s_wave=[0] * (waves + 1), ids=[0] * count, pref=[0] * (count + 1), s_tile=0)
    glob = dict(ctr=0)
    stored = [False]              # the first wave stored a phase this finalize step
    seen = {}                     # (round, wave) -> (nact, total) each wave saw

    def active(i):
        return state[i]["phase"] not in (DONE,)

    def block_scan(w, v):
        # exclusive prefix over the waves in one shared array (s_wave), as
        # the kernel's two scans share it: each wave publishes its sum,
        # thread 0 scans in place and appends the total, every wave reads
        shared["s_wave"][w] = v
        yield "bar"
        if w == 0:
            acc = 0
            for k in range(waves):
                c = shared["s_wave"][k]
                shared["s_wave"][k] = acc
                acc += c
            shared["s_wave"][waves] = acc
        yield "bar"
        base, tot = shared["s_wave"][w], shared["s_wave"][waves]
        yield "bar"
        return base, tot

    def wave(w):
        for rnd in range(max_rounds):
            # active list: this wave's share of the instances, two scans over
            # one shared array, then each wave writes its entries of the
            # list and of the tile prefix sums
            mine = [i for i in range(count) if i % waves == w and active(i)]
            k, nact = yield from block_scan(w, len(mine))
            tp, total = yield from block_scan(w, sum(ntiles[i] for i in mine))
            for i in mine:
                if 0 <= k < len(shared["ids"]):
                    shared["ids"][k] = i
                    shared["pref"][k] = tp
                tp += ntiles[i]
                k += 1
            if w == 0 and 0 <= nact <= count:
                shared["pref"][nact] = total
            yield "bar"
            seen[(rnd, w)] = (nact, total)
            if nact == 0:
                return
            # tiles: thread 0 takes the next index, every wave reads it
            it = 0
            while True:
                if w == 0:
                    shared["s_tile"] = glob["ctr"]
                    glob["ctr"] += 1
                yield "bar"
                t = shared["s_tile"]
                yield "bar"
                if t >= total:
                    break
                it += 1
                if it > loop_cap:
                    raise Stuck(f"wave {w} round {rnd}: tile index {t} < {total} after {it} passes")
                pref, ids = shared["pref"], shared["ids"]
                lo, hi = 0, max(min(nact, count) - 1, 0)
                while lo < hi:            # last q with pref[q] <= t
                    mid = (lo + hi + 1) // 2
                    if pref[mid] <= t:
                        lo = mid
                    else:
                        hi = mid - 1
                ph = state[ids[lo]]["phase"]
                if ph in (FIRST, NEWTON):
                    yield "bar"       # block_combine of the tile's norms
                    yield "bar"
            # grid barrier (one workgroup: thread 0 is the last arriver)
            yield "bar"
            if w == 0:
                glob["ctr"] = 0
            yield "bar"
            # finalize every active instance
            for q in range(min(nact, count)):
                inst = shared["ids"][q]
                if w == 0:
                    stored[0] = False
                yield ("load", w)
                phase = state[inst]["phase"]
                if fixed:
                    yield "bar"       # every wave has its phase before any store
                if phase in (FIRST, NEWTON):
                    yield "bar"       # block_combine of the partials
                    yield "bar"
                    if w == 0:
                        S = state[inst]
                        m = S["j"] + 1
                        if m >= products[inst]:
                            S["phase"] = UPDATE
                        else:
                            S["phase"], S["j"] = NEWTON, m
                        stored[0] = True
                elif w == 0:
                    S = state[inst]
                    if phase == START:
                        S["phase"] = FIRST
                    elif phase == UPDATE:
                        S["l"] += 1
                        S["j"] = 0
                        S["phase"] = START if S["l"] < substeps[inst] else DONE
                    stored[0] = True
                    yield ("store", w)
                yield "bar"
            yield "bar"
            yield "bar"
        raise Stuck(f"wave {w}: rounds exhausted")

    gens = {w: wave(w) for w in range(waves)}
    status = {w: None for w in range(waves)}   # None runnable, "bar" waiting, "load" deferred
    live = set(range(waves))

    def step(w):
        try:
            ev = next(gens[w])
        except StopIteration:
            live.discard(w)
            status[w] = "exit"
            return
        if ev == "bar":
            status[w] = "bar"
            sites[w] = gens[w].gi_frame.f_lineno if gens[w].gi_frame else None
            fr = gens[w].gi_yieldfrom
            while fr is not None:
                sites[w] = (sites[w], fr.gi_frame.f_lineno)
                fr = fr.gi_yieldfrom
        elif isinstance(ev, tuple) and ev[0] == "load" and w == late_wave:
            status[w] = "load"
        else:
            status[w] = None

    while live:
        waiting = [w for w in live if status[w] == "bar"]
        if len(waiting) == len(live):
            if len({sites[w] for w in waiting}) > 1:
                misaligned[0] += 1
            for w in waiting:
                status[w] = None
            continue
        runnable = [w for w in live if status[w] is None]
        deferred = [w for w in live if status[w] == "load"]
        if deferred and (stored[0] or not runnable):
            # the late wave loads once the first wave has stored, or when
            # nothing else can run (the barrier forces its load first)
            w = deferred[0]
            status[w] = None
            step(w)
            continue
        if runnable:
            step(runnable[0] if seed is None else rng.choice(runnable))
    agree = all(len({seen[(r, w)] for w in range(waves) if (r, w) in seen}) == 1
                for r in {r for r, _ in seen})
    return state, agree, misaligned[0]


def test_unfixed_finalize_lets_a_wave_spin_in_the_tile_loop():
    # a schedule found by the search below: the fourth wave loads the phase
    # late, the waves pair the wrong barriers, and in round 8 the second
    # wave sees a tile index (0) below its tile count (3) that nobody
    # advances any more
    with pytest.raises(Stuck, match="tile index 0 < 3"):
        run_model(fixed=False, waves=4, late_wave=3, seed=4, max_rounds=2000, loop_cap=100000)


def test_unfixed_finalize_misaligns_barriers_under_many_schedules():
    outcomes = {"misaligned": 0, "disagree": 0, "stuck": 0}
    for seed in range(60):
        try:
            _, agree, mis = run_model(fixed=False, waves=4, late_wave=1 + seed % 3, seed=seed)
            outcomes["misaligned"] += mis > 0
            outcomes["disagree"] += not agree
        except Stuck:
            outcomes["stuck"] += 1
    assert outcomes["misaligned"] > 0 and outcomes["disagree"] > 0 and outcomes["stuck"] > 0, outcomes


@pytest.mark.parametrize("waves,late_wave", [(2, 1), (4, 1), (4, 2), (4, 3)])
def test_fixed_finalize_keeps_waves_together(waves, late_wave):
    for seed in [None] + list(range(60)):
        state, agree, mis = run_model(fixed=True, waves=waves, late_wave=late_wave, seed=seed)
        assert mis == 0 and agree, seed
        assert all(s["phase"] == DONE for s in state), seed
