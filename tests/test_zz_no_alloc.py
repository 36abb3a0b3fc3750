"""The allocation-free apply (ulv_apply_noalloc) against ulv_apply through the
C ABI (GPU): two calls in a row, the second on a smaller problem, each within
the FP64 bar of the allocating entry point; sizes beyond the scratch array are
rejected with a clear error."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    # (workload, right-hand sides): the second call is the smaller input
    (workloads.SMALL.with_(name="matern32-l0.15-N3001", n=3001, kernel="matern32", ell=0.15, shift=1e-3,
                           leaf=50, max_rank=40, seed_base=7), 4),
    (workloads.SMALL.with_(name="exp-l0.2-N1500-sphere", n=1500, point_set="sphere", kernel="exponential",
                           ell=0.2, shift=1e-2, leaf=40, max_rank=30, hss_tol=1e-3, seed_base=8), 2),
]


def _factor(B, w):
    X = torch.from_numpy(w.points()).cuda()
    h2 = B.h2_build(X, w.kernel, w.ell, w.shift, leaf=w.leaf, tol=w.h2_tol, eta=w.eta)
    hss = B.spdhss_build(h2, w.hss_tol, w.max_rank, w.oversample,
                         omega=B.cols_like(w.n, w.s, "cuda").copy_(torch.from_numpy(w.omega())))
    return h2, hss, B.ulv_factor(hss)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2011_07632_amd import binding
    return binding


def test_noalloc_apply_matches_ulv_apply(B):
    keep = []
    for call, (w, nrhs) in enumerate(CASES):
        print(f"\n[noalloc] {w.name}: N={w.n} nrhs={nrhs}", flush=True)
        h2, hss, ulv = _factor(B, w)
        keep.append((h2, hss, ulv))
        b = B.cols_like(w.n, nrhs, "cuda").copy_(torch.from_numpy(workloads.gaussian_matrix(w.n, nrhs, 91)))
        ref = B.ulv_apply(ulv, b)
        out = B.cols_like(w.n, nrhs, "cuda").fill_(float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        B.ulv_apply_noalloc(ulv, b, out)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        d = float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))
        print(f"[noalloc] relative difference to ulv_apply {d:.2e}; scratch for vectors "
              f"{B.noalloc_bytes(ulv, nrhs)} bytes; device free memory change {free1 - free0} bytes", flush=True)
        assert torch.isfinite(out).all()
        assert d <= 1e-10
        # no device memory was taken by the call (the first call on a device
        # maps the static array itself, 64 MiB, which then stays)
        if call > 0:
            assert free1 >= free0 - (1 << 20)


def test_noalloc_rejects_sizes_beyond_scratch(B):
    w, _ = CASES[1]
    h2, hss, ulv = _factor(B, w)
    per_col = B.noalloc_bytes(ulv, 1)
    nrhs = B.NOALLOC_SCRATCH_BYTES // per_col + 1
    assert B.noalloc_bytes(ulv, nrhs) > B.NOALLOC_SCRATCH_BYTES
    b = B.cols_like(w.n, nrhs, "cuda").zero_()
    out = B.cols_like(w.n, nrhs, "cuda")
    with pytest.raises(B.SpdError, match="scratch array"):
        B.ulv_apply_noalloc(ulv, b, out)
    # the handle still works afterwards, in both entry points
    b1 = B.cols_like(w.n, 1, "cuda").copy_(torch.from_numpy(workloads.gaussian_matrix(w.n, 1, 92)))
    o1 = B.cols_like(w.n, 1, "cuda")
    B.ulv_apply_noalloc(ulv, b1, o1)
    assert float(torch.linalg.norm(o1 - B.ulv_apply(ulv, b1)) / torch.linalg.norm(o1)) <= 1e-10
