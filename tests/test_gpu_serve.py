"""Request loop (GPU): requests submitted while others run are admitted and
overlap; each result equals the same request run alone; the HBM budget
serializes admission; non-blocking waits report pending requests."""
import time

import numpy as np
import pytest

import workloads
from oracle_check import check_against_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2011_07632_amd import binding
    return binding


def request(B, w, precision="f64"):
    dev = "cuda"
    return dict(points=torch.from_numpy(w.points()).to(dev), kernel=w.kernel, ell=w.ell, shift=w.shift,
                leaf=w.leaf, h2_tol=w.h2_tol, hss_tol=w.hss_tol, max_rank=w.max_rank, oversample=w.oversample,
                omega=B.cols_like(w.n, w.s, dev).copy_(torch.from_numpy(w.omega())),
                b=B.cols_like(w.n, w.nrhs, dev).copy_(torch.from_numpy(w.rhs())),
                rtol=w.pcg_tol, maxit=3000, precision=precision)


def alone(B, r):
    out = B.solve_batch([r], workers=1)[0]
    return out["x"].cpu().numpy(), out["iters"]


def test_results_in_the_mix_equal_alone(B):
    ws = workloads.batch_instances(count=5, seed=77, n_lo=1500, n_hi=5000)
    reqs = [request(B, w, "f32" if j == 2 else "f64") for j, w in enumerate(ws)]
    ref = [alone(B, r) for r in reqs]
    S = B.Server(workers=3)
    tickets = []
    for r in reqs:
        tickets.append(S.submit(r))
        time.sleep(0.02)
    got = [S.wait(t) for t in tickets]
    S.close()
    for w, (x, it), g in zip(ws, ref, got):
        print(f"[serve] {w.name}: queued {g['seconds_queued']:.3f} s total {g['seconds_total']:.3f} s "
              f"iterations {g['iters'].tolist()} {g['status']}", flush=True)
        assert g["status"] == "SPD_OK", w.name
        assert g["iters"].tolist() == it.tolist(), w.name
        assert np.array_equal(g["x"].cpu().numpy(), x), w.name
        # against the oracle (as in the batched test)
        j = ws.index(w)
        o = check_against_oracle(w, x, g["iters"], fp64=(j != 2))
        print(f"[serve] {w.name}: residual against the oracle's operator {o['oracle_operator_relres'].max():.2e}",
              flush=True)
        assert o["oracle_operator_relres"].max() <= 2 * w.pcg_tol
        assert o.get("iters_match", True), w.name


def test_budget_serializes_admission(B):
    ws = workloads.batch_instances(count=3, seed=78, n_lo=1500, n_hi=3000)
    reqs = [request(B, w) for w in ws]
    S = B.Server(workers=3, hbm_budget_bytes=1)
    assert all(S.footprint(r) > 1 for r in reqs)
    tickets = [S.submit(r) for r in reqs]
    pending = S.wait(tickets[-1], block=False)
    got = [S.wait(t) for t in tickets]
    S.close()
    assert pending is None or pending["status"] in ("SPD_OK", "SPD_E_NOT_CONVERGED")
    # with a budget below every footprint the requests run one at a time, in order
    assert got[1]["seconds_queued"] >= got[0]["seconds_total"] - got[0]["seconds_queued"] - 0.05
    assert got[2]["seconds_queued"] > got[1]["seconds_queued"]


def test_footprint_grows_with_n(B):
    S = B.Server(workers=1)
    small, big = workloads.batch_instances(count=2, seed=79, n_lo=2000, n_hi=2001)[0], None
    big = small.with_(n=8000)
    assert S.footprint(request(B, big)) > S.footprint(request(B, small))
    S.close()


def test_two_waiters_on_one_ticket(B):
    """Two threads block on the same ticket: one collects the result, the
    other is told the ticket was collected (no hang, no stale entry)."""
    import threading
    w = workloads.batch_instances(count=1, seed=79, n_lo=1500, n_hi=2000)[0]
    S = B.Server(workers=1)
    t = S.submit(request(B, w))
    out = {}

    def waiter(k):
        try:
            out[k] = S.wait(t)["status"]
        except B.SpdError as e:
            out[k] = e.code

    th = [threading.Thread(target=waiter, args=(k,)) for k in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    S.close()
    assert not any(x.is_alive() for x in th)
    got = sorted(out.values(), key=str)
    assert len(got) == 2
    assert sum(1 for v in got if v == B.SPD_E_INVALID) == 1
    assert sum(1 for v in got if v in ("SPD_OK", "SPD_E_NOT_CONVERGED", "SPD_E_NOT_SPD")) == 1


def test_keyed_requests_reuse_resident_state(B):
    # two requests on one matrix (different right-hand sides) and one on another
    w1, w3 = workloads.batch_instances(count=2, seed=79, n_lo=2000, n_hi=4000)
    r1 = request(B, w1)
    r2 = dict(r1, b=B.cols_like(w1.n, 3, "cuda").copy_(
        torch.from_numpy(workloads.gaussian_matrix(w1.n, 3, 555))))
    r3 = request(B, w3)
    ref = [alone(B, r) for r in (r1, r2, r3)]
    S = B.Server(workers=2)
    t1 = S.submit(r1, key=7)
    t2 = S.submit(r2, key=7)
    t3 = S.submit(r3, key=9)
    got = [S.wait(t) for t in (t1, t2, t3)]
    S.close()
    for (x, it), g, name in zip(ref, got, ("first", "reuse", "other")):
        print(f"[serve keyed] {name}: h2 {g['seconds_h2']:.3f} s build {g['seconds_build']:.3f} s "
              f"solve {g['seconds_solve']:.3f} s {g['status']}", flush=True)
        assert g["status"] == "SPD_OK", name
        assert g["iters"].tolist() == it.tolist(), name
        assert np.array_equal(g["x"].cpu().numpy(), x), name
    assert got[0]["seconds_h2"] > 0 and got[2]["seconds_h2"] > 0
    assert got[1]["seconds_h2"] == 0.0 and got[1]["seconds_build"] == 0.0  # solved on the resident state


def test_resident_state_released_for_admission(B):
    # a budget that holds one resident state: the second matrix evicts the
    # first, whose next request then builds it again; results are unchanged
    w1, w3 = workloads.batch_instances(count=2, seed=80, n_lo=2000, n_hi=3000)
    r1, r3 = request(B, w1), request(B, w3)
    ref1, ref3 = alone(B, r1), alone(B, r3)
    S0 = B.Server(workers=1)
    budget = max(S0.footprint(r1), S0.footprint(r3)) + 1
    S0.close()
    S = B.Server(workers=1, hbm_budget_bytes=budget)
    g1 = S.wait(S.submit(r1, key=1))
    g3 = S.wait(S.submit(r3, key=3))
    g1b = S.wait(S.submit(r1, key=1))
    S.close()
    for g, (x, it) in ((g1, ref1), (g3, ref3), (g1b, ref1)):
        assert g["status"] == "SPD_OK"
        assert np.array_equal(g["x"].cpu().numpy(), x)
    assert g1b["seconds_h2"] > 0  # rebuilt: its state had been released for the other matrix


def test_keyed_submit_rejects_zero_key(B):
    w = workloads.batch_instances(count=1, seed=81, n_lo=1500, n_hi=1600)[0]
    S = B.Server(workers=1)
    r = request(B, w)
    import ctypes
    I = B._Instance()
    keep = B._fill_instance(I, r)  # noqa: F841
    t = ctypes.c_int64()
    assert B.lib.spd_server_submit_keyed(S._h, ctypes.byref(I), ctypes.c_uint64(0), ctypes.byref(t)) != 0
    S.close()


def test_phase_reports_progress(B):
    w = workloads.batch_instances(count=1, seed=82, n_lo=3000, n_hi=3100)[0]
    S = B.Server(workers=1)
    t = S.submit(request(B, w))
    seen = set()
    while True:
        p = S.phase(t)
        seen.add(p)
        if p == "finished":
            break
        time.sleep(0.001)
    g = S.wait(t)
    S.close()
    assert g["status"] == "SPD_OK" and "finished" in seen
    with pytest.raises(B.SpdError):
        S2 = B.Server(workers=1)
        try:
            S2.phase(12345)  # unknown ticket
        finally:
            S2.close()
