"""Host logic of the serving trace driver, with a stand-in server (no GPU)."""
import pytest

from paper_2211_03193_amd import serving


class FakeServer:
    """Admits every job at once; a job is done after `need` steps."""

    def __init__(self, need):
        self.need = need
        self.jobs = {}
        self.clock = 0.0

    def submit(self, cfg, y, target):
        jid = len(self.jobs) + 1
        self.jobs[jid] = {"state": 0, "steps": 0, "t_submit": self.clock, "need": self.need[cfg],
                          "reached": 0, "t_target": -1.0, "t_done": -1.0}
        return jid

    def step(self):
        self.clock += 1.0
        for j in self.jobs.values():
            if j["state"] in (0, 1):
                j["state"] = 1
                j["steps"] += 1
                if j["steps"] >= j["need"]:
                    j["state"] = 2
                    j["t_done"] = self.clock
        act = sum(j["state"] == 1 for j in self.jobs.values())
        return act, 0

    def job(self, jid):
        return dict(self.jobs[jid])


def test_trace_driver_submits_every_job_and_drains():
    need = {0: 3, 1: 1, 2: 5}
    srv = FakeServer(need)
    st = serving.run_trace(srv, [(k, None, 0.0) for k in need], [0.0, 0.01, 0.02])
    assert [s["id"] for s in st] == [1, 2, 3]
    assert all(s["state"] == 2 for s in st)
    assert [s["steps"] for s in st] == [3, 1, 5]
    summ = serving.summarise(st)
    assert summ["done"] == 3 and summ["failed"] == 0 and summ["reached_target"] == 0
    assert summ["p50_time_to_done_s"] is not None


def test_trace_driver_waits_for_late_arrivals():
    srv = FakeServer({0: 1, 1: 1})
    st = serving.run_trace(srv, [(0, None, 0.0), (1, None, 0.0)], [0.0, 0.15])
    assert all(s["state"] == 2 for s in st) and len(st) == 2


def test_trace_driver_times_out():
    class Stuck(FakeServer):
        def step(self):
            return 1, 0
    with pytest.raises(TimeoutError):
        serving.run_trace(Stuck({0: 1}), [(0, None, 0.0)], [0.0], max_wall=0.2)
