"""Host-side admission policy of the serving loop (no GPU needed)."""
import collections

from paper_2604_24994_amd.serve import take_batch


class R:
    def __init__(self, i, scene, rays, nbytes):
        self.i, self.scene_id, self.rays, self.nbytes = i, scene, rays, nbytes


def _q(items):
    return collections.deque(R(*it) for it in items)


def test_fifo_same_scene_and_ray_cap():
    q = _q([(0, 0, 100, 10), (1, 0, 100, 10), (2, 0, 100, 10), (3, 0, 100, 10)])
    b = take_batch(q, 0, 1000, 250, 64)
    assert [r.i for r in b] == [0, 1]
    assert [r.i for r in q] == [2, 3]


def test_other_scenes_keep_their_place():
    q = _q([(0, 0, 10, 1), (1, 1, 10, 1), (2, 0, 10, 1), (3, 1, 10, 1)])
    b = take_batch(q, 0, 1000, 10 ** 6, 64)
    assert [r.i for r in b] == [0, 2]
    assert [r.i for r in q] == [1, 3]
    b = take_batch(q, 0, 1000, 10 ** 6, 64)
    assert [r.i for r in b] == [1, 3] and not q


def test_budget_admission_and_no_reordering_within_scene():
    q = _q([(0, 0, 10, 60), (1, 0, 10, 60), (2, 0, 10, 10)])
    b = take_batch(q, 0, 100, 10 ** 6, 64)
    assert [r.i for r in b] == [0]          # request 1 does not fit; 2 must not overtake it
    assert [r.i for r in q] == [1, 2]
    assert take_batch(q, 60, 100, 10 ** 6, 64) == []   # still in flight: wait
    assert [r.i for r in take_batch(q, 0, 100, 10 ** 6, 64)] == [1, 2]


def test_single_large_request_is_admitted_alone():
    q = _q([(0, 0, 10 ** 7, 5), (1, 0, 10, 5)])
    assert [r.i for r in take_batch(q, 0, 100, 1000, 64)] == [0]
    assert [r.i for r in take_batch(q, 0, 100, 1000, 64)] == [1]


def test_max_batch():
    q = _q([(i, 0, 1, 1) for i in range(10)])
    assert len(take_batch(q, 0, 100, 10 ** 6, 4)) == 4 and len(q) == 6


def test_server_waits_for_budget_and_admits_when_memory_frees():
    # the threaded server with a stand-in renderer (no GPU): three requests
    # of 60, 60 and 30 bytes under a 100-byte budget.  The second does not
    # fit beside the first and must wait until the first completes; the
    # third may not overtake it (same scene).  In-flight bytes never exceed
    # the budget.
    import threading
    import time
    from types import SimpleNamespace

    from paper_2604_24994_amd.serve import Server

    release = {0: threading.Event(), 1: threading.Event(), 2: threading.Event()}
    started = []

    def render(scene, cams, stream):
        for c in cams:
            started.append(c.i)
        for c in cams:
            release[c.i].wait(5)
        return [c.i for c in cams]

    sizes = {0: 60, 1: 60, 2: 30}
    srv = Server({0: object()}, hbm_budget_bytes=100, render_fn=render, sizer=lambda sc, cam: sizes[cam.i],
                 streams=False, n_workers=2)
    try:
        cams = [SimpleNamespace(i=i, width=4, height=4) for i in range(3)]
        futs = [srv.submit(0, c) for c in cams]
        time.sleep(0.3)
        assert started == [0]                 # 1 (60 B) waits beside 0 (60 B); 2 may not overtake 1
        release[0].set()
        assert futs[0].result(timeout=5) == 0
        time.sleep(0.3)
        assert sorted(started) == [0, 1, 2]   # memory freed: 1 and 2 (90 B) admitted together
        release[1].set()
        release[2].set()
        assert [f.result(timeout=5) for f in futs] == [0, 1, 2]
    finally:
        for e in release.values():
            e.set()
        srv.close()
    assert srv.peak_inflight <= 100
    assert max(b for _, b in srv.admitted) <= 100
