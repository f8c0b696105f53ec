"""Host logic of the serving loop (CPU only): the watchdog that reports frames whose completion has not come by a
deadline, and the Poisson request stream of the serving workload."""
import numpy as np

from paper_2407_14053_amd.serving import Watchdog, poisson_requests


def test_watchdog_reports_late_work_once_and_forgets_completed_work():
    w = Watchdog(0.5)
    w.arm("a", 0.0)
    w.arm("b", 0.2)
    assert w.poll(0.4) == []
    late = w.poll(0.6)
    assert [k for k, _ in late] == ["a"] and abs(late[0][1] - 0.6) < 1e-12
    assert w.poll(0.65) == []                      # "a" reported once; "b" is 0.45 s old
    assert [k for k, _ in w.poll(0.75)] == ["b"]
    w.disarm("a")
    w.disarm("b")
    assert w.poll(10.0) == []                      # completed work is never reported again
    w.arm("a", 10.0)                               # a new frame under the same key starts a new deadline
    assert w.poll(10.4) == [] and [k for k, _ in w.poll(10.6)] == ["a"]


def test_poisson_requests_rate_and_mix():
    reqs = poisson_requests(4000, 200.0, ["s0", "s1", "s2", "s3"], ["d0", "d1", "d2"], seed=2000)
    t = np.array([r.arrival for r in reqs])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 200.0) < 0.05 / 200.0          # exponential gaps of mean 1/rate
    assert abs(np.median(gaps) - np.log(2) / 200.0) < 0.1 / 200.0
    for key, names in (("scene", ["s0", "s1", "s2", "s3"]), ("display", ["d0", "d1", "d2"])):
        counts = np.array([sum(getattr(r, key) == n for r in reqs) for n in names])
        assert np.all(np.abs(counts / len(reqs) - 1 / len(names)) < 0.03)
    # every pose looks at the origin from distance 3 on the orbit
    for r in reqs[:50]:
        eye = r.c2w[:3, 3]
        assert abs(np.linalg.norm(eye) - 3.0) < 1e-9 and abs(eye[1]) < 1e-12
        fwd = r.c2w[:3, 2]
        assert np.allclose(fwd, -eye / 3.0, atol=1e-9)
