"""CPU model of the batched solver's seat protocol (k_batch in csrc/batch.hip).

Workgroups are coroutines; every shared-memory operation of the protocol
(atomic add, compare-and-swap, load, store) is one step, and a seeded random
scheduler interleaves the steps.  The model follows the kernel's rules: a free
workgroup takes an open seat of the priority list, else of the other list,
else the next solo item, else polls both lists until every solo item is done;
a hand-over reserves a slot (priority slots from the front of one shared
array, the others from the back), publishes the instance, then counts its solo
item as done; a gang member joins and waits until its gang has G members.

Checked: every handed-over instance gets exactly one member per rank, the two
lists never share an array entry, every wait ends and every workgroup exits.
A planted variant in which a waiting workgroup commits to a ticket of the other
list ahead of its hand-over (the single-list protocol's waiting rule) starves a
priority gang, which the model reports as a wait that never ends.
"""
import random

import pytest

WAIT_LIMIT = 20000


class Deadlock(Exception):
    pass


def simulate(seed, grid=8, G=4, count=40, p_hand=0.35, p_prio=0.5, precommit=False):
    rng = random.Random(seed)
    S = dict(counter=0, ticket=0, cont=0, pticket=0, pcont=0, done=0)
    cont_list = [-1] * count
    join = [0] * count
    members = {}                # instance -> list of ranks
    lists_of = {}               # instance -> "p" / "n"
    plan = [(rng.random() < p_hand, rng.random() < p_prio, rng.randint(1, 30)) for _ in range(count)]

    def take_seat(front):
        tkey, ckey = ("pticket", "pcont") if front else ("ticket", "cont")
        tk = S[tkey]
        yield
        while True:
            cn = S[ckey]
            yield
            if tk >= cn * G:
                return None
            if S[tkey] == tk:                      # compare-and-swap
                S[tkey] = tk + 1
                yield
                slot = tk // G
                e = slot if front else count - 1 - slot
                n = 0
                while cont_list[e] < 0:
                    n += 1
                    if n > WAIT_LIMIT:
                        raise Deadlock("slot entry")
                    yield
                return (cont_list[e], tk % G, front)
            tk = S[tkey]
            yield

    def solo(item):
        hand, prio, work = plan[item]
        for _ in range(work):
            yield
        if hand:
            key = "pcont" if prio else "cont"
            slot = S[key]
            S[key] = slot + 1                      # atomic add
            yield
            e = slot if prio else count - 1 - slot
            assert cont_list[e] == -1, "lists share an entry"
            cont_list[e] = item
            lists_of[item] = "p" if prio else "n"
            yield
        S["done"] += 1
        yield

    def gang(idx, r):
        members.setdefault(idx, []).append(r)
        join[idx] += 1
        yield
        n = 0
        while join[idx] < G:
            n += 1
            if n > WAIT_LIMIT:
                raise Deadlock("gang %d has %d of %d members" % (idx, join[idx], G))
            yield
        for _ in range(rng.randint(1, 20)):
            yield

    def workgroup():
        while True:
            seat = yield from take_seat(True)
            if seat is None:
                seat = yield from take_seat(False)
            if seat is not None:
                yield from gang(seat[0], seat[1])
                continue
            item = S["counter"]
            S["counter"] = item + 1
            yield
            if item < count:
                yield from solo(item)
                continue
            if precommit:
                tk = S["ticket"]
                S["ticket"] = tk + 1
                yield
                slot = tk // G
                n = 0
                while True:
                    e = count - 1 - slot
                    if slot < count and cont_list[e] >= 0:
                        yield from gang(cont_list[e], tk % G)
                        break
                    if S["done"] >= count and slot >= S["cont"]:
                        return
                    n += 1
                    if n > WAIT_LIMIT:
                        raise Deadlock("committed waiter")
                    yield
                continue
            n = 0
            while True:
                dn = S["done"]
                yield
                seat = yield from take_seat(True)
                if seat is None:
                    seat = yield from take_seat(False)
                if seat is not None:
                    yield from gang(seat[0], seat[1])
                    break
                if dn >= count:
                    return
                n += 1
                if n > WAIT_LIMIT:
                    raise Deadlock("poller")
                yield
            continue

    wgs = [workgroup() for _ in range(grid)]
    live = list(range(grid))
    while live:
        k = rng.choice(live)
        try:
            next(wgs[k])
        except StopIteration:
            live.remove(k)
    handed = [i for i in range(count) if plan[i][0]]
    return handed, members, lists_of


@pytest.mark.parametrize("seed", range(40))
def test_every_gang_fills_and_every_workgroup_exits(seed):
    handed, members, lists_of = simulate(seed)
    assert sorted(members) == sorted(handed)
    for idx in handed:
        assert sorted(members[idx]) == list(range(4)), (idx, members[idx])
    assert set(lists_of.values()) <= {"p", "n"}


@pytest.mark.parametrize("G", [2, 4])
def test_gang_of_half_the_grid(G):
    for seed in range(10):
        handed, members, _ = simulate(100 + seed, grid=2 * G, G=G, count=30, p_hand=0.6)
        assert all(sorted(members[i]) == list(range(G)) for i in handed)


def test_committed_waiters_starve_a_priority_gang():
    """The planted single-list waiting rule must fail in the two-list setting."""
    failed = 0
    for seed in range(40):
        try:
            simulate(seed, precommit=True)
        except Deadlock:
            failed += 1
    assert failed > 0
