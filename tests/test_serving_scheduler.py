"""The serving loop's scheduling (host side), against a stand-in for the
batch: admission in arrival order under the slot and byte budgets,
continuous batching (requests join while others run), failed setups and
oversized requests reported without blocking the queue."""
import types

import pytest

from paper_1208_4772_amd import dg, serving


class FakeSolver:
    def __init__(self, case):
        self.case = case

    @classmethod
    def from_case(cls, case, precision, device=None):
        if getattr(case, "bad", False):
            raise dg.DGError(dg.DG_EGEOM, "bad geometry")
        return cls(case)

    def state(self, U0):
        return types.SimpleNamespace(double=lambda: None)

    def close(self):
        pass


class FakeBatch:
    """Slots advance in lockstep; a slot finishes when its steps are done."""
    log = []

    def __init__(self, budget, max_slots):
        self.max_slots = max_slots
        self.slots = {}
        FakeBatch.log = []

    def admit(self, sol, U, nsteps):
        if len(self.slots) >= self.max_slots:
            return None
        slot = next(i for i in range(self.max_slots) if i not in self.slots)
        self.slots[slot] = [sol, nsteps, 0]
        FakeBatch.log.append(("admit", sol.case.rid, len(self.slots)))
        return slot

    def advance(self, n):
        live = [s for s in self.slots.values() if s[2] < s[1]]
        if not live:
            return 0
        n = min([n] + [s[1] - s[2] for s in live])
        for s in live:
            s[2] += n
        return n

    def poll(self):
        return [k for k, s in self.slots.items() if s[2] >= s[1]]

    def stats(self, slot):
        sol, total, done = self.slots[slot]
        return types.SimpleNamespace(status=0, t=0.01 * done, steps=done)

    def release(self, slot):
        FakeBatch.log.append(("release", self.slots[slot][0].case.rid))
        del self.slots[slot]

    def info(self):
        return 1, 1

    def close(self):
        pass


def requests(n, steps, sizes, arrival_gap=0.0, bad=()):
    reqs = []
    for i in range(n):
        case = types.SimpleNamespace(K=sizes[i], U0=None, rid=i, bad=i in bad, dofs=lambda: 100)
        r = serving.Request(i, "cylinder", sizes[i], 2, 0.4, steps[i], arrival_gap * i, av=False)
        r.case = case
        reqs.append(r)
    return reqs


@pytest.fixture
def fakes(monkeypatch):
    import torch
    monkeypatch.setattr(dg, "Solver", FakeSolver)
    monkeypatch.setattr(dg, "Batch", FakeBatch)
    monkeypatch.setattr(dg, "estimate_footprint", lambda K, P, precision="fp32", av=False: K)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)


def test_slots_and_arrival_order(fakes):
    reqs = requests(7, [30, 10, 20, 10, 10, 40, 10], [1] * 7)
    rep = serving.Server(hbm_budget_bytes=100, max_slots=3, chunk_steps=5).run(reqs)
    admits = [e for e in FakeBatch.log if e[0] == "admit"]
    assert [e[1] for e in admits] == list(range(7))          # arrival order
    assert max(e[2] for e in admits) == 3 == rep.peak_slots  # never more than the slots
    # continuous batching: request 3 joins after the first release, while 0 and 2 still run
    first_release = next(i for i, e in enumerate(FakeBatch.log) if e[0] == "release")
    assert FakeBatch.log[first_release] == ("release", 1)
    assert FakeBatch.log[first_release + 1][:2] == ("admit", 3)
    assert all(r.status == 0 and r.finished >= r.admitted >= r.arrival for r in reqs)
    assert rep.summary()["failed"] == 0


def test_byte_budget_limits_admission(fakes):
    # budget 10 bytes, requests of 4 bytes: at most two at once
    reqs = requests(5, [10] * 5, [4] * 5)
    rep = serving.Server(hbm_budget_bytes=10, max_slots=8, chunk_steps=5).run(reqs)
    assert rep.peak_slots == 2
    assert all(r.status == 0 for r in reqs)


def test_failed_setup_and_oversized_request_do_not_block(fakes):
    reqs = requests(4, [10] * 4, [4, 50, 4, 4], bad={2})
    rep = serving.Server(hbm_budget_bytes=10, max_slots=4, chunk_steps=5).run(reqs)
    assert reqs[1].status == dg.DG_EBUSY            # larger than the whole budget
    assert reqs[2].status == dg.DG_EGEOM and "bad geometry" in reqs[2].error
    assert reqs[0].status == 0 and reqs[3].status == 0
    s = rep.summary()
    assert s["failed"] == 2 and s["n_requests"] == 4
