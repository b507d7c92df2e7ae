"""Host logic of the request loop, without a GPU: first-come-first-served
admission by HBM footprint and by the voxels in flight, the batch limit, and
the rejection of a job larger than the whole budget. The device state of an
admitted job is replaced by a stand-in that only knows the cube's size."""
import numpy as np
import pytest

from paper_2510_00562_amd import serve


class _Dev:
    def __init__(self, shape):
        self.shape = shape

    def numel(self):
        return int(np.prod(self.shape))


class _FakeActive:
    def __init__(self, job, dual_storage, copy=None, pinned=None):
        self.job = job
        self.vd = _Dev(job.v.shape)
        self.done = 0


@pytest.fixture
def server(monkeypatch):
    monkeypatch.setattr(serve, "_Active", _FakeActive)

    def make(budget, active_voxels=None):
        return serve.Server(budget, active_voxels=active_voxels, clock=lambda: 0.0)
    return make


def job(q, shape):
    return serve.Job(q, np.zeros(shape, np.float32), 1.0, 1.0, 1.0)


def admitted(srv):
    return [a.job.job_id for a in srv.active]


def test_footprint_budget_is_first_come_first_served(server):
    shapes = [(8, 32, 32), (16, 64, 64), (4, 16, 16)]
    fp = [serve.footprint(s) for s in shapes]
    srv = server(fp[0] + fp[1] - 1)  # the first two do not fit together
    for q, s in enumerate(shapes):
        srv.submit(job(q, s))
    srv._admit()
    # job 1 does not fit beside job 0; job 2 would, but waits behind job 1
    assert admitted(srv) == [0]
    assert srv.used == fp[0]
    assert [j.job_id for j in srv.waiting] == [1, 2]


def test_footprint_budget_admits_what_fits(server):
    shapes = [(8, 32, 32), (4, 16, 16), (16, 64, 64)]
    fp = [serve.footprint(s) for s in shapes]
    srv = server(fp[0] + fp[1] + fp[2] - 1)  # all but the last byte of the three
    for q, s in enumerate(shapes):
        srv.submit(job(q, s))
    srv._admit()
    assert admitted(srv) == [0, 1] and srv.used == fp[0] + fp[1]


def test_voxels_in_flight_cap(server):
    shapes = [(8, 64, 64), (8, 64, 64), (8, 64, 64)]
    n = int(np.prod(shapes[0]))
    srv = server(1 << 40, active_voxels=2 * n)
    for q, s in enumerate(shapes):
        srv.submit(job(q, s))
    srv._admit()
    assert admitted(srv) == [0, 1]  # admission stops once 2n voxels are in flight
    # the first job is admitted even when it alone exceeds the cap
    srv2 = server(1 << 40, active_voxels=n // 2)
    srv2.submit(job(0, shapes[0]))
    srv2.submit(job(1, shapes[1]))
    srv2._admit()
    assert admitted(srv2) == [0]


def test_batch_limit_and_oversized_job(server):
    srv = server(1 << 40)
    for q in range(serve.MAX_BATCH + 6):
        srv.submit(job(q, (2, 8, 8)))
    srv._admit()
    assert len(srv.active) == serve.MAX_BATCH
    assert len(srv.waiting) == 6
    small = server(serve.footprint((2, 8, 8)))
    with pytest.raises(ValueError):
        small.submit(job(99, (4, 16, 16)))
