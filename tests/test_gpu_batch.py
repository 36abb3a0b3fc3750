"""Independent instances run concurrently (spd_solve_batch) give the same
results as each instance run alone through the single-instance entry points
(GPU): the same solution bit for bit and the same iteration counts, for a mix
of sizes, kernels, point sets and solve precisions."""
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


def request(B, w, precision):
    dev = "cuda"
    return dict(points=torch.from_numpy(w.points()).to(dev), kernel=w.kernel, ell=w.ell, shift=w.shift,
                leaf=w.leaf, h2_tol=w.h2_tol, hss_tol=w.hss_tol, max_rank=w.max_rank, oversample=w.oversample,
                omega=B.cols_like(w.n, w.s, dev).copy_(torch.from_numpy(w.omega())),
                b=B.cols_like(w.n, w.nrhs, dev).copy_(torch.from_numpy(w.rhs())),
                rtol=w.pcg_tol, maxit=3000, precision=precision)


def alone(B, r):
    h2 = B.h2_build(r["points"], r["kernel"], r["ell"], r["shift"], leaf=r["leaf"], tol=r["h2_tol"])
    hss = B.spdhss_build(h2, r["hss_tol"], r["max_rank"], r["oversample"], omega=r["omega"])
    ulv = B.ulv_factor(hss, precision=r["precision"])
    x, it, res = B.pcg_solve(h2, ulv, r["b"], rtol=r["rtol"], maxit=r["maxit"], raise_on_nonconvergence=False)
    return x.cpu().numpy(), it, res


def test_batch_equals_alone(B):
    ws = workloads.batch_instances(count=6, n_lo=1500, n_hi=5000)
    reqs = [request(B, w, "f32" if j % 2 else "f64") for j, w in enumerate(ws)]
    ref = [alone(B, r) for r in reqs]
    got = B.solve_batch(reqs, workers=3)
    for w, (x, it, res), g in zip(ws, ref, got):
        print(f"[batch] {w.name}: iterations {g['iters'].tolist()} relres {g['relres'].max():.2e} "
              f"status {g['status']}", flush=True)
        assert g["status"] == "SPD_OK", w.name
        assert g["iters"].tolist() == it.tolist(), w.name
        assert np.array_equal(g["x"].cpu().numpy(), x), w.name
        assert g["relres"].max() <= w.pcg_tol
        # against the oracle: the solution solves the oracle's own H^2 system
        # to the tolerance, and FP64 solves take the oracle's iteration counts
        o = check_against_oracle(w, x, g["iters"], fp64=(reqs[ws.index(w)]["precision"] == "f64"))
        print(f"[batch] {w.name}: residual against the oracle's operator {o['oracle_operator_relres'].max():.2e}"
              f" oracle iterations {o.get('oracle_iters', np.array([])).tolist()}", flush=True)
        assert o["oracle_operator_relres"].max() <= 2 * w.pcg_tol
        assert o.get("iters_match", True), w.name


def test_batch_argument_errors(B):
    with pytest.raises(B.SpdError):
        B.solve_batch([], workers=0)


def test_request_omega_shape_is_checked(B):
    w = workloads.batch_instances(count=1, n_lo=1500, n_hi=1600)[0]
    r = request(B, w, "f64")
    r["omega"] = B.cols_like(w.n, w.s - 1, "cuda").zero_()  # one column short
    with pytest.raises(ValueError):
        B.solve_batch([r], workers=1)
