"""The request server's admission and batching, on the CPU: a test-only
executor (ecc_server_create_with_exec) stands in for the device, so the
server's own logic runs unchanged: admission of MSMs by the HBM share of a
slot, a burst far larger than the slots and the batch limits, a batch whose
call fails, and a batch that runs out of device memory and is halved."""

import os
import threading

import numpy as np
import pytest

from tests.common import ROOT

LIB = os.path.join(ROOT, "paper_2501_03245_amd", "libecc_mi.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")

BLS = 2  # ECC_BLS12_381_G1
OK, ERR_NOMEM, ERR_DEVICE = 0, -4, -5


class Exec:
    """Stand-in device: a scratch plan of `per_point` bytes per point plus
    `fixed` per MSM, a record of every batch run and the number running at
    once, and optional failures."""

    def __init__(self, per_point=1000, fixed=10_000, budget_share=None, fail_size=None, delay=0.0):
        self.per_point, self.fixed = per_point, fixed
        self.budget_share = budget_share  # a batch above it fails with NOMEM (as the device would)
        self.fail_size = fail_size        # a batch holding an MSM of this size fails with ECC_ERR_DEVICE
        self.delay = delay
        self.batches = []
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0

    def plan(self, sizes):
        return sum(self.per_point * n + self.fixed for n in sizes)

    def run(self, kind, sizes):
        import time
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.batches.append((kind, list(sizes)))
        try:
            if self.delay:
                time.sleep(self.delay)
            if kind == 1 and self.budget_share is not None and self.plan(sizes) > self.budget_share:
                return ERR_NOMEM, None
            if kind == 1 and self.fail_size is not None and self.fail_size in sizes:
                return ERR_DEVICE, None
            # flags: MSMs of even size "at infinity", verifications valid for odd first hash byte
            return OK, [(n % 2 == 0) if kind == 1 else 1 for n in sizes]
        finally:
            with self.lock:
                self.running -= 1


def _server(ex, **kw):
    import paper_2501_03245_amd as eccmi
    eccmi.library()
    return eccmi.Server(test_exec=(ex.plan, ex.run), **kw)


def _scalars(n):
    return np.zeros((n, 4), dtype=np.uint64)


def test_admission_cuts_batches_to_the_hbm_share():
    ex = Exec(delay=0.01)
    sizes = [100, 300, 50, 700, 20, 400, 100, 250, 90, 600]
    share = 450_000  # per slot: two slots share a budget of twice this
    srv = _server(ex, slots=2, hbm_budget_bytes=2 * share, max_batch_points=1 << 20)
    try:
        bid = srv.add_bases(BLS, np.zeros((1000, 12), dtype=np.uint64))
        tickets = [srv.submit_msm(bid, 0, _scalars(n)) for n in sizes]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert [flag for _, flag, _ in got] == [int(n % 2 == 0) for n in sizes]
    msm_batches = [b for k, b in ex.batches if k == 1]
    assert sorted(n for b in msm_batches for n in b) == sorted(sizes)  # each request ran exactly once
    for b in msm_batches:
        assert len(b) == 1 or ex.plan(b) <= share  # a batch over the share only when it is one request
    assert st["done_msm"] == len(sizes) and st["budget_cuts"] >= 1 and st["nomem_splits"] == 0


def test_request_larger_than_the_share_fails_alone():
    """Budget exhaustion: a request whose own scratch exceeds the share runs
    alone and gets ECC_ERR_NOMEM; the requests around it still finish."""
    ex = Exec(budget_share=200_000)
    srv = _server(ex, slots=1, hbm_budget_bytes=200_000, max_batch_points=1 << 20)
    try:
        bid = srv.add_bases(BLS, np.zeros((1000, 12), dtype=np.uint64))
        tickets = [srv.submit_msm(bid, 0, _scalars(n)) for n in (50, 900, 60)]
        res = [srv.wait_status(t) for t in tickets]
    finally:
        srv.close()
    assert res[1][0] == ERR_NOMEM
    assert res[0][0] == OK and res[2][0] == OK
    assert [b for k, b in ex.batches if 900 in b] == [[900]]  # alone, never halved further


def test_nomem_batch_is_halved_and_retried():
    """The device runs out of memory for a batch that admission let through
    (no budget set here): the server halves the batch until each part fits,
    and every request finishes with its own result."""
    ex = Exec(budget_share=250_000)
    sizes = [100, 100, 100, 100, 100, 100, 100, 100]  # 8 x 110 kB: fits two at a time
    srv = _server(ex, slots=1, hbm_budget_bytes=0, max_batch_points=1 << 20)
    try:
        bid = srv.add_bases(BLS, np.zeros((1000, 12), dtype=np.uint64))
        # hold the worker on a first request so that the others queue up together
        ex.delay = 0.05
        tickets = [srv.submit_msm(bid, 0, _scalars(n)) for n in sizes]
        res = [srv.wait_status(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert all(s == OK for s, _ in res)
    assert st["nomem_splits"] >= 1
    ran_ok = [b for k, b in ex.batches if ex.plan(b) <= 250_000]
    assert sorted(n for b in ran_ok for n in b) == sorted(sizes)


def test_burst_larger_than_slots_and_batch_limits():
    """3000 verifications and 40 MSMs submitted at once to 2 slots with
    batches of at most 128 verifications: all finish, no batch exceeds its
    limit, at most two batches run at once, and every verification batch
    holds only verifications."""
    ex = Exec(delay=0.002)
    srv = _server(ex, slots=2, hbm_budget_bytes=0, max_batch_points=2000, max_batch_verify=128)
    try:
        bid = srv.add_bases(BLS, np.zeros((1000, 12), dtype=np.uint64))
        h = np.zeros((3000, 32), dtype=np.uint8)
        q = np.zeros((3000, 8), dtype=np.uint64)
        g = np.zeros((3000, 8), dtype=np.uint64)
        tv = srv.submit_verify_many(h[:1500], q[:1500], g[:1500])
        tm = [srv.submit_msm(bid, 0, _scalars(7 + j)) for j in range(40)]
        tv += srv.submit_verify_many(h[1500:], q[1500:], g[1500:])
        flags, lat, status = srv.wait_many(tv)
        mres = [srv.wait(t) for t in tm]
        st = srv.stats()
    finally:
        srv.close()
    assert (status == OK).all() and (flags == 1).all() and (lat >= 0).all()
    assert [f for _, f, _ in mres] == [int((7 + j) % 2 == 0) for j in range(40)]
    assert ex.max_running <= 2
    for kind, b in ex.batches:
        if kind == 0:
            assert len(b) <= 128
        else:
            assert sum(b) <= 2000 or len(b) == 1
    assert st["done_verify"] == 3000 and st["done_msm"] == 40 and st["max_queue"] >= 1500


def test_erroring_batch_reports_its_status():
    """A batch whose call fails gives its error to each of its requests, and
    only to them; later requests still run."""
    ex = Exec()
    srv = _server(ex, slots=1, hbm_budget_bytes=0, max_batch_points=1 << 20)
    try:
        bid = srv.add_bases(BLS, np.zeros((1000, 12), dtype=np.uint64))
        t_before = srv.submit_msm(bid, 0, _scalars(13))  # the same request before the failure is set
        before = srv.wait_status(t_before)
        t_ok = srv.submit_msm(bid, 0, _scalars(12))
        ok = srv.wait_status(t_ok)
        ex.fail_size = 13
        t_bad2 = srv.submit_msm(bid, 0, _scalars(13))
        bad2 = srv.wait_status(t_bad2)
        t_after = srv.submit_msm(bid, 0, _scalars(14))
        after = srv.wait_status(t_after)
        # a ticket is taken once
        again = srv.wait_status(t_after)
    finally:
        srv.close()
    assert before == (OK, 0) and ok == (OK, 1)
    assert bad2[0] == ERR_DEVICE
    assert after == (OK, 1)
    assert again[0] == -1  # ECC_ERR_ARG
