"""The C-ABI library loads and exports every function include/spdhss.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spdhss.h")
LIB = os.path.join(ROOT, "paper_2011_07632_amd", "libspdhss.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:spd_status|void|const char\*|int64_t)\s+([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("h2_build", "spdhss_build", "ulv_factor", "ulv_apply", "h2_matvec", "pcg_solve",
               "spd_request_footprint", "spd_last_error", "h2_destroy"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_rejects_bad_arguments_without_a_device():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2011_07632_amd import binding as B
    # null arguments are rejected before any device work
    out = ctypes.c_void_p()
    code = B.lib.spdhss_build(None, None, None, ctypes.byref(out))
    assert code == B.SPD_E_INVALID and out.value is None
    assert b"null" in B.lib.spd_last_error()


# A stand-in device address: every call below fails its argument checks first,
# so the address is never dereferenced and no device is touched.
FAKE = ctypes.c_void_p(0x1000)


def _h2_args(**kw):
    from paper_2011_07632_amd import binding as B
    k = dict(kind=1, ell=0.1, shift=1e-4)
    o = dict(leaf_size=64, eta=1.0, tol=1e-8, proxy_shells=8, proxy_per_shell=128, proxy_per_shell_max=2048,
             proxy_density=90.0, sketch_seed=1)
    for key, v in kw.items():
        (k if key in k else o)[key] = v
    return B._Kernel(**k), B._H2Opts(**o)


@pytest.mark.parametrize("n,bad,msg", [
    (0, {}, b"n must be positive"),
    (1 << 31, {}, b"below 2^31"),
    (100, {"kind": 5}, b"unknown kernel"),
    (100, {"ell": 0.0}, b"ell"),
    (100, {"ell": float("nan")}, b"ell"),
    (100, {"shift": float("inf")}, b"shift"),
    (100, {"leaf_size": 0}, b"leaf_size"),
    (100, {"leaf_size": 513}, b"leaf_size"),
    (100, {"eta": 0.0}, b"eta"),
    (100, {"tree": 2}, b"unknown tree"),
    (100, {"tree": -1}, b"unknown tree"),
    (100, {"tol": 1.0}, b"tol"),
    (100, {"proxy_shells": 0}, b"proxy"),
    (100, {"proxy_shells": 65}, b"proxy counts"),
    (100, {"proxy_per_shell": 256, "proxy_per_shell_max": 128}, b"proxy_per_shell_max below"),
    (100, {"proxy_shells": 64, "proxy_per_shell_max": 2048}, b"65536 proxy"),
    (100, {"proxy_density": -1.0}, b"proxy_density"),
    (100, {"proxy_density": float("nan")}, b"proxy_density"),
])
def test_h2_build_argument_checks(n, bad, msg):
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2011_07632_amd import binding as B
    k, o = _h2_args(**bad)
    out = ctypes.c_void_p(0x1)
    code = B.lib.h2_build(FAKE, n, k, ctypes.byref(o), None, ctypes.byref(out))
    assert code == B.SPD_E_INVALID
    assert out.value is None  # *out is cleared on failure
    assert msg in B.lib.spd_last_error()


def test_null_handles_are_rejected():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2011_07632_amd import binding as B
    L, out = B.lib, ctypes.c_void_p()
    assert L.ulv_factor(None, None, ctypes.byref(out)) == B.SPD_E_INVALID
    assert L.ulv_apply(None, FAKE, FAKE, 1, 10, None) == B.SPD_E_INVALID
    assert L.h2_matvec(None, FAKE, FAKE, 1, 10, None) == B.SPD_E_INVALID
    assert L.pcg_solve(None, None, FAKE, FAKE, 1, 10, 1e-8, 10, None, None, None) == B.SPD_E_INVALID
    assert L.spd_h2_query_get(None, 0, FAKE, 8) == B.SPD_E_INVALID
    assert L.spd_hss_query_get(None, 0, 0, 0, FAKE, 8) == B.SPD_E_INVALID
    L.h2_destroy(None)  # destroying a null handle is a no-op
    L.spdhss_destroy(None)
    L.ulv_destroy(None)


def test_server_and_footprint_host_checks():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2011_07632_amd import binding as B
    L, out = B.lib, ctypes.c_void_p(0x1)
    assert L.spd_server_create(0, 1 << 30, ctypes.byref(out)) == B.SPD_E_INVALID
    assert out.value is None
    assert L.spd_server_create(2, 0, ctypes.byref(out)) == B.SPD_E_INVALID
    assert L.spd_request_footprint(None) == 0
    k, o = _h2_args()
    q = B._Instance(n=10_000, kernel=k, h2=o, hss=B._HSSOpts(tol=1e-2, max_rank=100, oversample=10), nrhs=1)
    f1 = L.spd_request_footprint(ctypes.byref(q))
    q.n = 20_000
    f2 = L.spd_request_footprint(ctypes.byref(q))
    q.nrhs = 32
    f3 = L.spd_request_footprint(ctypes.byref(q))
    # at least the points and the near blocks; linear in N; grows with the right-hand sides
    assert f1 >= 24 * 10_000 + 8 * 10_000 * 64
    assert f2 == pytest.approx(2 * f1, rel=1e-9)
    assert f3 > f2


class _FakeCols:
    """Duck-typed stand-in for a float64 device tensor (shape and strides only)."""

    def __init__(self, shape, strides):
        import torch
        self.is_cuda, self.dtype = True, torch.float64
        self.shape, self._st = shape, strides

    def dim(self):
        return len(self.shape)

    def stride(self, i):
        return self._st[i]


@pytest.mark.parametrize("shape,strides,want", [
    ((10,), (1,), (1, 10)),
    ((10, 1), (1, 1), (1, 10)),      # one column, e.g. x.unsqueeze(1): stride unused
    ((10, 1), (1, 10), (1, 10)),
    ((10, 3), (1, 10), (3, 10)),
    ((10, 3), (1, 16), (3, 16)),     # padded leading dimension
    ((10, 3), (3, 1), None),         # row-major
    ((10, 3), (1, 8), None),         # overlapping columns
    ((9, 3), (1, 10), None),         # wrong N
    ((10,), (2,), None),             # strided vector
])
def test_binding_column_layouts(shape, strides, want):
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2011_07632_amd import binding as B
    t = _FakeCols(shape, strides)
    if want is None:
        with pytest.raises(ValueError):
            B._as_cols(t, 10)
    else:
        assert B._as_cols(t, 10)[1:] == want


def test_default_outputs_take_the_input_layout():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import torch
    from paper_2011_07632_amd import binding as B
    v = torch.zeros(10, dtype=torch.float64)
    assert B._out_like(v, 10, 1, 10).shape == (10,)
    o = B._out_like(torch.zeros(3, 16, dtype=torch.float64).t()[:10], 10, 3, 16)
    assert o.shape == (10, 3) and o.stride() == (1, 16)
    o = B._out_like(torch.zeros(1, 10, dtype=torch.float64).t(), 10, 1, 10)
    assert o.shape == (10, 1) and o.stride(0) == 1


def test_request_points_are_checked_before_any_device_use():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import torch
    from paper_2011_07632_amd import binding as B
    for pts in (torch.zeros(10, 3, dtype=torch.float64),   # host memory
                torch.zeros(10, 3, dtype=torch.float32),
                torch.zeros(10, 2, dtype=torch.float64)):
        with pytest.raises(ValueError):
            B._fill_instance(B._Instance(), {"points": pts})


def test_import_fails_loudly_without_the_library(tmp_path):
    """No CPU fallback: without the built library the package does not import
    (a copy of the package's Python files with no libspdhss.so beside them)."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2011_07632_amd"
    pkg.mkdir()
    for f in ("__init__.py", "binding.py"):
        shutil.copy(os.path.join(ROOT, "paper_2011_07632_amd", f), pkg / f)
    r = subprocess.run([sys.executable, "-c", "import paper_2011_07632_amd"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "not built" in r.stderr


def test_product_path_does_not_load_the_oracle():
    """The oracle is test infrastructure: the package (and bench.py at import)
    never import it, and no library source refers to it."""
    import subprocess
    import sys
    code = ("import sys, paper_2011_07632_amd, bench; "
            "bad = [m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; "
            "assert not bad, bad")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    pkg = os.path.join(ROOT, "paper_2011_07632_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f), encoding="utf-8").read()
                assert "import oracle" not in text and "from oracle" not in text, f
