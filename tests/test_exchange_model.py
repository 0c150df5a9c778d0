"""CPU model of the block-column pivot exchange of the LU kernel.

In the GEPP block-column kernel, the G workgroups that share a block column
agree on each column's pivot through a small exchange buffer: for column c of
the launch that starts at global column k0, workgroup g writes its record
(the candidate row's words and the key word) into slot (c mod 2) at offset
g, every word a 64-bit value whose upper part is the tag k0 + c + 1; then
every workgroup polls all G records of that slot until every tag it reads
equals k0 + c + 1, and only then goes on to the next column (a barrier
inside the workgroup orders its reads before its next publication).  The
buffer is zeroed once before the first launch of a factorisation; the
launches run one after another with G = ceil(h / 512) for h rows.

The model runs that protocol with individual word stores and loads as the
atomic events, under adversarial schedules:

* any interleaving of the workgroups (random schedules, and an exhaustive
  search over every interleaving for small cases);
* loads that may return any value the word held at or after the last value
  the same reader saw there (per-location coherence, no other ordering), with
  the newest value eventually returned (fairness).

Checked: every run completes (no workgroup waits forever), and every record a
workgroup accepts holds exactly the words written for that column by that
workgroup -- never a word from another column, slot or launch.  Protocol
variants with a planted mistake (one slot instead of two, tags that restart
at every launch, each column published before the previous column's poll)
are shown to fail the same checks, so the model is able to see such errors.
"""
import random

import pytest

WORDS = 2          # words per record in the model (row words + key word)


class Mem:
    """Per-word coherence order of values; a reader may see any value at or
    after the last one it saw at that word."""

    def __init__(self, size):
        self.hist = [[0] for _ in range(size)]

    def store(self, addr, val):
        self.hist[addr].append(val)


def _layout(G, c, g, w, slots):
    return ((c % slots) * G + g) * WORDS + w


def _tag(variant, k0, c):
    # planted mistake "local_tags": the tag restarts at every launch
    return (c + 1) if variant == "local_tags" else (k0 + c + 1)


def _val(li, c, g, w):
    return (li * 1000 + c) * 64 + g * 4 + w


def _program(g, launches, variant):
    """The workgroup's actions in program order: ("store", li, c, w),
    ("poll", li, c) and ("end", li).  The kernel publishes a column's record
    and polls that column before it publishes the next; the planted mistake
    "early_publish" publishes each next column before polling the current."""
    prog = []
    for li, (k0, G, kb) in enumerate(launches):
        if g < G:
            for c in range(kb):
                if variant == "early_publish":
                    if c == 0:
                        prog += [("store", li, 0, w) for w in range(WORDS)]
                    if c + 1 < kb:
                        prog += [("store", li, c + 1, w) for w in range(WORDS)]
                else:
                    prog += [("store", li, c, w) for w in range(WORDS)]
                prog.append(("poll", li, c))
        prog.append(("end", li))
    return prog


def _store(variant, launches, g, act):
    _, li, c, w = act
    k0, G, _ = launches[li]
    slots = 1 if variant == "one_slot" else 2
    return _layout(G, c, g, w, slots), (_tag(variant, k0, c), _val(li, c, g, w))


def _poll_words(variant, launches, act):
    _, li, c = act
    k0, G, _ = launches[li]
    slots = 1 if variant == "one_slot" else 2
    return [(g2, w, _layout(G, c, g2, w, slots)) for g2 in range(G) for w in range(WORDS)]


def _check_accept(variant, launches, act, words):
    _, li, c = act
    for g2, w, (t, x) in words:
        if x != _val(li, c, g2, w):
            raise AssertionError(f"stale word accepted: launch {li} column {c} record {g2} "
                                 f"word {w} holds {x}, written {_val(li, c, g2, w)}")


def _run(launches, G_max, variant, rng, stale_p=0.3, max_events=200000):
    """One adversarial execution: random interleaving of single word events;
    a poll is a sequence of single-word loads, each of which may return an
    older value than the newest (never older than the reader saw there
    before).  Returns the accepted (k0, c) per workgroup."""
    size = 2 * G_max * WORDS
    mem = Mem(size)
    progs = [_program(g, launches, variant) for g in range(G_max)]
    pc = [0] * G_max
    seen_idx = [[0] * size for _ in range(G_max)]
    poll_pos = [0] * G_max            # words read so far in the current round
    poll_got = [[] for _ in range(G_max)]
    accepted = [[] for _ in range(G_max)]
    events = 0
    while True:
        live = [g for g in range(G_max) if pc[g] < len(progs[g])]
        if not live:
            return accepted
        events += 1
        if events > max_events:
            raise AssertionError(f"no progress after {max_events} events (stall)")
        runnable = []
        for g in live:
            act = progs[g][pc[g]]
            if act[0] == "end":
                li = act[1]
                # launch barrier: every workgroup has reached the end of li
                if all(pc[h] >= len(progs[h]) or
                       (progs[h][pc[h]][0] == "end" and progs[h][pc[h]][1] >= li) or
                       progs[h][pc[h]][1] > li for h in range(G_max)):
                    runnable.append(g)
            else:
                runnable.append(g)
        if not runnable:
            raise AssertionError("every workgroup waits: deadlock")
        g = rng.choice(runnable)
        act = progs[g][pc[g]]
        if act[0] == "store":
            addr, word = _store(variant, launches, g, act)
            mem.store(addr, word)
            pc[g] += 1
        elif act[0] == "end":
            pc[g] += 1
        else:
            words = _poll_words(variant, launches, act)
            g2, w, addr = words[poll_pos[g]]
            h = mem.hist[addr]
            lo = seen_idx[g][addr]
            idx = rng.randint(lo, len(h) - 1) if rng.random() < stale_p else len(h) - 1
            seen_idx[g][addr] = idx
            v = h[idx]
            poll_got[g].append((g2, w, v if isinstance(v, tuple) else (0, 0)))
            poll_pos[g] += 1
            if poll_pos[g] == len(words):
                k0 = launches[act[1]][0]
                tag = _tag(variant, k0, act[2])
                if all(t == tag for _, _, (t, _) in poll_got[g]):
                    _check_accept(variant, launches, act, poll_got[g])
                    accepted[g].append((k0, act[2]))
                    pc[g] += 1
                poll_pos[g] = 0
                poll_got[g] = []


def _launch_sequence(n, nb=4, rows_per_wg=3):
    """(k0, G, kb) for a factorisation of order n in blocks of nb columns,
    G = ceil(h / rows_per_wg) workgroups for the h rows of each block."""
    out = []
    for k0 in range(0, n, nb):
        h = n - k0
        out.append((k0, -(-h // rows_per_wg), min(nb, n - k0)))
    return out


@pytest.mark.parametrize("n,nb,rows", [(12, 4, 3), (9, 3, 2), (16, 4, 5)])
def test_exchange_completes_and_accepts_only_current_records(n, nb, rows):
    launches = _launch_sequence(n, nb, rows)
    G_max = max(G for _, G, _ in launches)
    rng = random.Random(1234 + n)
    for _ in range(200):
        acc = _run(launches, G_max, "kernel", rng)
        for g in range(G_max):
            want = [(k0, c) for k0, G, kb in launches if g < G for c in range(kb)]
            assert acc[g] == want


def _exhaustive(launches, G_max, variant):
    """Every interleaving, as an explicit-state search: word stores are
    single events, a poll round reads the newest words at once and is
    enabled only when it succeeds (a failing round changes no state).
    Returns the number of states; raises on a deadlock or a stale accept."""
    size = 2 * G_max * WORDS
    progs = [_program(g, launches, variant) for g in range(G_max)]
    init = (tuple([0] * G_max), tuple([(0, 0)] * size))
    seen = {init}
    stack = [init]
    while stack:
        pcs, mem = stack.pop()
        if all(pcs[g] >= len(progs[g]) for g in range(G_max)):
            continue
        succ = []
        for g in range(G_max):
            if pcs[g] >= len(progs[g]):
                continue
            act = progs[g][pcs[g]]
            if act[0] == "store":
                addr, word = _store(variant, launches, g, act)
                m = list(mem)
                m[addr] = word
                succ.append((g, tuple(m)))
            elif act[0] == "end":
                li = act[1]
                if all(pcs[h] >= len(progs[h]) or
                       (progs[h][pcs[h]][0] == "end" and progs[h][pcs[h]][1] >= li) or
                       progs[h][pcs[h]][1] > li for h in range(G_max)):
                    succ.append((g, mem))
            else:
                words = [(g2, w, mem[a]) for g2, w, a in _poll_words(variant, launches, act)]
                tag = _tag(variant, launches[act[1]][0], act[2])
                if all(t == tag for _, _, (t, _) in words):
                    _check_accept(variant, launches, act, words)
                    succ.append((g, mem))
        if not succ:
            raise AssertionError(f"deadlock at program positions {pcs}")
        for g, m in succ:
            p2 = list(pcs)
            p2[g] += 1
            key = (tuple(p2), m)
            if key not in seen:
                seen.add(key)
                stack.append(key)
    return len(seen)


@pytest.mark.parametrize("launches", [
    [(0, 2, 3), (3, 2, 3), (6, 1, 2)],
    [(0, 3, 2), (2, 2, 2)],
])
def test_exchange_every_interleaving_small(launches):
    G_max = max(G for _, G, _ in launches)
    assert _exhaustive(launches, G_max, "kernel") > 10


@pytest.mark.parametrize("variant", ["one_slot", "local_tags", "early_publish"])
def test_planted_mistakes_fail_the_exhaustive_search(variant):
    launches = [(0, 2, 3), (3, 2, 3), (6, 1, 2)]
    with pytest.raises(AssertionError):
        _exhaustive(launches, 2, variant)


@pytest.mark.parametrize("variant", ["one_slot", "local_tags", "early_publish"])
def test_planted_mistakes_fail_the_random_schedules(variant):
    launches = [(0, 2, 3), (3, 2, 3), (6, 2, 2)]
    G_max = 2
    rng = random.Random(99)
    failed = False
    for _ in range(300):
        try:
            _run(launches, G_max, variant, rng, max_events=20000)
        except AssertionError:
            failed = True
            break
    assert failed, variant
