"""Host logic of the serving loop, run without a GPU (simulated ticks).

Admission by HBM footprint in arrival order, continuous batching (jobs join
while others run), rejection of jobs that can never fit, the job timeline and
the poll / fetch / cancel protocol. The scheduler code is the same as on the
GPU; only the tick itself and the device uploads are skipped.
"""

import time

import numpy as np
import pytest

from paper_1806_07985_amd import native


def _job(dims, R):
    X = np.zeros(1, dtype=np.float32)          # never read in simulation
    H0 = [np.zeros((d, R), dtype=np.float32) for d in dims]
    return X, H0


def _server(budget, max_active=64):
    return native.Server(budget, max_active=max_active, simulate=True)


def _wait_all(srv, ids, timeout=30.0):
    for i in ids:
        assert srv.wait(i, timeout), f"job {i} did not finish"
    return {i: srv.poll(i) for i in ids}


def test_jobs_complete_with_consistent_timeline():
    srv = _server(1 << 40)
    ids = []
    for k in range(6):
        X, H0 = _job((20 + k, 30, 40), 8)
        ids.append(srv.submit(X, (20 + k, 30, 40), 8, H0, iters=5 + k))
    res = _wait_all(srv, ids)
    for k, i in enumerate(ids):
        r = res[i]
        assert r["status"] == 0 and r["iters_done"] == 5 + k
        assert r["submit_s"] <= r["admit_s"] <= r["start_s"] <= r["done_s"]
    st = srv.stats()
    assert st["completed"] == 6 and st["active"] == 0 and st["queued"] == 0 and st["bytes_in_use"] == 0
    srv.close()


def test_admission_respects_budget_and_arrival_order():
    dims, R = (64, 64, 64), 16
    X, H0 = _job(dims, R)
    srv = _server(1 << 40)
    probe = srv.submit(X, dims, R, H0, iters=1)
    assert srv.wait(probe, 10)
    foot = srv.poll(probe)["footprint"]
    srv.close()
    # room for exactly two such jobs at a time
    srv = _server(2 * foot + foot // 2)
    ids = [srv.submit(X, dims, R, H0, iters=20) for _ in range(7)]
    res = _wait_all(srv, ids)
    st = srv.stats()
    assert st["peak_bytes"] <= st["budget_bytes"]
    assert st["peak_active"] == 2
    admits = [res[i]["admit_s"] for i in ids]
    assert admits == sorted(admits)            # first come, first admitted
    # at most two jobs overlap at any admission instant
    for i in ids:
        t = res[i]["admit_s"]
        live = sum(1 for j in ids if res[j]["admit_s"] <= t < res[j]["done_s"])
        assert live <= 2
    srv.close()


def test_max_active_slots():
    dims, R = (16, 16, 16), 4
    X, H0 = _job(dims, R)
    srv = _server(1 << 40, max_active=3)
    ids = [srv.submit(X, dims, R, H0, iters=30) for _ in range(9)]
    _wait_all(srv, ids)
    assert srv.stats()["peak_active"] == 3
    srv.close()


def test_continuous_batching_admits_while_others_run():
    X, H0 = _job((32, 32, 32), 8)
    srv = _server(1 << 40)
    long_job = srv.submit(X, (32, 32, 32), 8, H0, iters=400)
    time.sleep(0.02)
    short = [srv.submit(X, (32, 32, 32), 8, H0, iters=3) for _ in range(3)]
    res = _wait_all(srv, [long_job] + short)
    for i in short:
        # joined and left while the long job kept running
        assert res[long_job]["admit_s"] < res[i]["admit_s"] < res[i]["done_s"] < res[long_job]["done_s"]
    srv.close()


def test_oversized_job_is_rejected_and_others_proceed():
    small, big = (16, 16, 16), (400, 400, 400)
    Xs, Hs = _job(small, 4)
    Xb, Hb = _job(big, 4)
    srv = _server(64 << 20)                    # 64 MiB: the 256 MB tensor can never fit
    a = srv.submit(Xs, small, 4, Hs, iters=3)
    b = srv.submit(Xb, big, 4, Hb, iters=3)
    c = srv.submit(Xs, small, 4, Hs, iters=3)
    res = _wait_all(srv, [a, b, c])
    assert res[a]["status"] == 0 and res[c]["status"] == 0
    assert res[b]["status"] == -2              # NNCP_ENOMEM
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_poll_fetch_protocol():
    X, H0 = _job((16, 16, 16), 4)
    srv = _server(1 << 40)
    with pytest.raises(native.NNCPError):
        srv.poll(987654)                       # unknown id
    i = srv.submit(X, (16, 16, 16), 4, H0, iters=2)
    assert srv.wait(i, 10)
    assert srv.poll(i)["status"] == 0
    out = srv.fetch(i)                         # forgets the job
    assert len(out["H"]) == 3
    with pytest.raises(native.NNCPError):
        srv.poll(i)
    srv.close()


def test_invalid_requests_rejected_at_submit():
    srv = _server(1 << 40)
    X, H0 = _job((16, 16, 16), 4)
    with pytest.raises(native.NNCPError):
        srv.submit(X, (16, 16, 16), 100, [np.zeros((16, 100), np.float32)] * 3, iters=2)   # rank > 64
    with pytest.raises(native.NNCPError):
        srv.submit(X, (16, 16, 16), 4, H0, iters=0)
    with pytest.raises(native.NNCPError):
        srv.submit(X, (16,), 4, H0[:1], iters=2)                                            # N < 2
    srv.close()


def test_close_cancels_queued_jobs():
    X, H0 = _job((16, 16, 16), 4)
    srv = _server(1 << 40, max_active=1)
    ids = [srv.submit(X, (16, 16, 16), 4, H0, iters=200) for _ in range(4)]
    time.sleep(0.01)
    srv.close()                                # running job finishes, queued ones are cancelled
