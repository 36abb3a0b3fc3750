"""ctypes binding of libspdhss.so: argument marshalling only.

Names follow the C ABI: h2_build, spdhss_build, ulv_factor, ulv_apply,
h2_matvec, pcg_solve.  Arrays are torch tensors on the HIP device; vectors are
(N, ncols) column-major (``stride(0) == 1``) or 1-D, rows in the original point
order, FP64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; importing without it raises (there is no fallback)
LIB_PATH = os.path.join(HERE, "libspdhss.so")

KERNELS = {"gaussian": 0, "matern32": 1, "exponential": 2, "imq": 3, "rpy": 4}

SPD_OK, SPD_E_INVALID, SPD_E_NOMEM, SPD_E_NOT_SPD, SPD_E_NOT_CONVERGED, SPD_E_DEVICE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {1: "SPD_PENDING", 0: "SPD_OK", -1: "SPD_E_INVALID", -2: "SPD_E_NOMEM", -3: "SPD_E_NOT_SPD",
                -4: "SPD_E_NOT_CONVERGED", -5: "SPD_E_DEVICE"}

# query ids (include/spdhss.h)
Q = dict(N=0, LEVELS=1, PERM=2, NODE_START=3, H2_RANK=4, SKELETON=5, NEAR_PTR=6, NEAR_IDX=7,
         COUP_PTR=8, COUP_IDX=9, NNODES=10, BYTES=11, H2_TIMES=12, PROXY_COUNT=13, H2_STORAGE=14)
HQ = dict(RANK=0, PIVOTS=1, BASIS=2, TRANSFER=3, PHIU=4, COUPLING=5, FACTOR=6, ROWS=7, BYTES=8,
          TIMES=9, FLOPS=10)


class SpdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ell", C.c_double), ("shift", C.c_double)]


class _H2Opts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("eta", C.c_double), ("tol", C.c_double),
                ("proxy_shells", C.c_int32), ("proxy_per_shell", C.c_int32),
                ("proxy_per_shell_max", C.c_int32), ("proxy_density", C.c_double),
                ("sketch_seed", C.c_uint64), ("tree", C.c_int32)]


# defaults of the H^2 construction options (spd_h2_opts)
H2_DEFAULTS = dict(proxy_shells=8, proxy_per_shell=128, proxy_per_shell_max=2048, proxy_density=90.0,
                   sketch_seed=0x5EEDF00D, tree="kd")
TREES = {"kd": 0, "box": 1}  # spd_tree_kind


def _h2_opts(leaf, eta, tol, d: dict) -> "_H2Opts":
    g = {k: d.get(k, v) for k, v in H2_DEFAULTS.items()}
    g["proxy_per_shell_max"] = max(int(g["proxy_per_shell_max"]), int(g["proxy_per_shell"]))
    return _H2Opts(int(leaf), float(eta), float(tol), int(g["proxy_shells"]), int(g["proxy_per_shell"]),
                   int(g["proxy_per_shell_max"]), float(g["proxy_density"]), int(g["sketch_seed"]),
                   TREES[g["tree"]])


class _HSSOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_rank", C.c_int32), ("oversample", C.c_int32),
                ("seed", C.c_uint64), ("omega", C.c_void_p)]


class _Instance(C.Structure):
    _fields_ = [("points", C.c_void_p), ("n", C.c_int64), ("kernel", _Kernel), ("h2", _H2Opts),
                ("hss", _HSSOpts), ("solve_precision", C.c_int32), ("b", C.c_void_p), ("x", C.c_void_p),
                ("nrhs", C.c_int32), ("rtol", C.c_double), ("maxit", C.c_int32),
                ("iters", C.c_void_p), ("relres", C.c_void_p)]


class _InstanceResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters_max", C.c_int32), ("relres_max", C.c_double),
                ("seconds_h2", C.c_double), ("seconds_build", C.c_double), ("seconds_solve", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2011_07632_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "h2_build": [vp, i64, _Kernel, C.POINTER(_H2Opts), vp, C.POINTER(vp)],
        "spdhss_build": [vp, C.POINTER(_HSSOpts), vp, C.POINTER(vp)],
        "ulv_factor": [vp, vp, C.POINTER(vp)],
        "ulv_factor_ex": [vp, C.c_int32, vp, C.POINTER(vp)],
        "ulv_apply": [vp, vp, vp, i32, i64, vp],
        "ulv_apply_noalloc": [vp, vp, vp, i32, i64, vp],
        "h2_matvec": [vp, vp, vp, i32, i64, vp],
        "h2_matvec_ex": [vp, vp, vp, i32, i64, i32, vp],
        "pcg_solve": [vp, vp, vp, vp, i32, i64, dbl, i32, vp, vp, vp],
        "pcg_solve_ex": [vp, vp, vp, vp, i32, i64, dbl, i32, i32, vp, vp, vp],
        "spd_h2_query_get": [vp, i32, vp, i64],
        "spd_hss_query_get": [vp, i32, i32, i32, vp, i64],
        "spd_h2_time_near": [vp, i32, i32, vp, vp, vp],
        "spd_h2_time_launches": [vp, i32, i32, vp, vp, vp, vp, i32, vp],
        "spd_test_gemm": [vp, vp, vp, i32, i32, i32, i32, i32, i32, dbl, dbl, vp],
        "spd_test_symm": [vp, vp, vp, i32, i32, i32, i32, i32, vp, vp],
        "spd_test_chol": [vp, i32, i32, vp, vp],
        "spd_test_trsm": [vp, vp, i32, i32, i32, i32, i32, vp],
        "spd_test_cpqr": [vp, vp, vp, vp, vp, i32, i32, i32, i32, dbl, i32, vp],
        "spd_solve_batch": [C.POINTER(_Instance), i32, i32, C.POINTER(_InstanceResult)],
        "spd_server_create": [i32, i64, C.POINTER(vp)],
        "spd_server_submit": [vp, C.POINTER(_Instance), C.POINTER(i64)],
        "spd_server_submit_keyed": [vp, C.POINTER(_Instance), C.c_uint64, C.POINTER(i64)],
        "spd_server_phase": [vp, i64, C.POINTER(i32)],
        "spd_server_wait": [vp, i64, i32, C.POINTER(_InstanceResult), C.POINTER(dbl), C.POINTER(dbl)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    for name in ("h2_destroy", "spdhss_destroy", "ulv_destroy"):
        f = getattr(L, name)
        f.argtypes = [vp]
        f.restype = None
    L.spd_server_destroy.argtypes = [vp]
    L.spd_server_destroy.restype = None
    L.spd_request_footprint.argtypes = [C.POINTER(_Instance)]
    L.spd_request_footprint.restype = C.c_int64
    L.spd_noalloc_bytes.argtypes = [vp, i32]
    L.spd_noalloc_bytes.restype = C.c_int64
    L.spd_last_error.argtypes = []
    L.spd_last_error.restype = C.c_char_p
    return L


lib = _load()


def _check(code: int):
    if code != SPD_OK:
        raise SpdError(code, lib.spd_last_error().decode())


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _as_cols(t: torch.Tensor, n: int) -> tuple[torch.Tensor, int, int]:
    """(tensor, ncols, ld) of a device FP64 vector block in column-major form."""
    if not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("expected a float64 device tensor")
    if t.dim() == 1:
        if t.shape[0] != n or t.stride(0) != 1:
            raise ValueError("vector length / stride mismatch")
        return t, 1, n
    if t.dim() != 2 or t.shape[0] != n or t.stride(0) != 1:
        raise ValueError("expected an (N, ncols) column-major tensor")
    ncols = t.shape[1]
    ld = t.stride(1) if ncols > 1 else n  # one column: its stride is never used
    if ld < n:
        raise ValueError("expected an (N, ncols) column-major tensor")
    return t, ncols, ld


def cols_like(n: int, ncols: int, device) -> torch.Tensor:
    """An uninitialised (n, ncols) column-major FP64 device tensor."""
    return torch.empty((ncols, n), dtype=torch.float64, device=device).t()


def _out_like(t: torch.Tensor, n: int, ncols: int, ld: int) -> torch.Tensor:
    """An output block with the input's layout: the C ABI takes one leading
    dimension for the input and the output."""
    if t.dim() == 1:
        return torch.empty_like(t)
    return torch.empty((ncols, ld), dtype=torch.float64, device=t.device).t()[:n]


def _check_out(out: torch.Tensor, n: int, ncols: int, ld: int) -> None:
    _, nc2, ld2 = _as_cols(out, n)
    if nc2 != ncols or ld2 != ld:
        raise ValueError("output shape / leading dimension must match the input")


class H2Matrix:
    """H^2 representation of shift*I + K(X, X) (handle)."""

    def __init__(self, handle: int, n: int, device):
        self._h = C.c_void_p(handle)
        self.n = n
        self.device = device

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            try:
                lib.h2_destroy(h)
            except Exception:
                pass
            self._h = None

    def _get(self, what: str, dtype, count: int) -> np.ndarray:
        out = np.empty(max(count, 1), dtype=dtype)  # never a zero-size (possibly null) buffer
        _check(lib.spd_h2_query_get(self._h, Q[what], out.ctypes.data, out.nbytes))
        return out[:count]

    def scalar(self, what: str) -> int:
        return int(self._get(what, np.int64, 1)[0])

    @property
    def levels(self) -> int:
        return self.scalar("LEVELS")

    @property
    def nnodes(self) -> int:
        return self.scalar("NNODES")

    def perm(self) -> np.ndarray:
        return self._get("PERM", np.int64, self.n)

    def node_start(self) -> np.ndarray:
        return self._get("NODE_START", np.int64, self.nnodes + 1)

    def ranks(self) -> np.ndarray:
        return self._get("H2_RANK", np.int32, self.nnodes)

    def skeletons(self) -> dict[int, np.ndarray]:
        k = self.ranks()
        flat = self._get("SKELETON", np.int64, int(k[1:].sum()))
        out, pos = {}, 0
        for v in range(1, self.nnodes):
            out[v] = flat[pos:pos + k[v]]
            pos += k[v]
        return out

    def lists(self):
        nn = self.nnodes
        npt = self._get("NEAR_PTR", np.int64, nn + 1)
        nid = self._get("NEAR_IDX", np.int32, int(npt[-1]))
        cpt = self._get("COUP_PTR", np.int64, nn + 1)
        cid = self._get("COUP_IDX", np.int32, int(cpt[-1]))
        near = {v: nid[npt[v]:npt[v + 1]].tolist() for v in range(nn)}
        coup = {v: cid[cpt[v]:cpt[v + 1]].tolist() for v in range(nn)}
        return near, coup

    def times(self) -> np.ndarray:
        return self._get("H2_TIMES", np.float64, 4)

    def device_bytes(self) -> int:
        return self.scalar("BYTES")

    def proxy_counts(self) -> np.ndarray:
        """Points per proxy sphere of every node (0 where no ID ran)."""
        return self._get("PROXY_COUNT", np.int32, self.nnodes)

    def storage(self) -> dict:
        """Bytes of the near blocks, coupling blocks and interpolation matrices."""
        v = self._get("H2_STORAGE", np.int64, 3)
        return {"near": int(v[0]), "coupling": int(v[1]), "bases": int(v[2])}


class HSSMatrix:
    """SPD HSS approximation built by Algorithm 5.3 (handle)."""

    def __init__(self, handle: int, h2: H2Matrix, s: int):
        self._h = C.c_void_p(handle)
        self.n = h2.n
        self.nnodes = h2.nnodes
        self.s = s
        self.device = h2.device
        self._hk = h2.ranks()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            try:
                lib.spdhss_destroy(h)
            except Exception:
                pass
            self._h = None

    def _q(self, what, node, node2, dtype, count):
        out = np.empty(max(count, 1), dtype=dtype)
        _check(lib.spd_hss_query_get(self._h, HQ[what], node, node2, out.ctypes.data, out.nbytes))
        return out[:count]

    def ranks(self) -> np.ndarray:
        return self._q("RANK", 0, 0, np.int32, self.nnodes)

    def rows(self, v: int) -> int:
        return int(self._q("ROWS", v, 0, np.int64, 1)[0])

    def pivots(self, v: int) -> np.ndarray:
        return self._q("PIVOTS", v, 0, np.int32, int(self.ranks()[v]))

    def basis(self, v: int) -> np.ndarray:
        r, m = int(self.ranks()[v]), self.rows(v)
        return self._q("BASIS", v, 0, np.float64, m * r).reshape(r, m).T

    def transfer(self, v: int) -> np.ndarray:
        r, m = int(self.ranks()[v]), self.rows(v)
        return self._q("TRANSFER", v, 0, np.float64, m * r).reshape(r, m).T

    def phiu(self, v: int) -> np.ndarray:
        r, k = int(self.ranks()[v]), int(self._hk[v])
        return self._q("PHIU", v, 0, np.float64, r * k).reshape(k, r).T

    def coupling(self, i: int, j: int) -> np.ndarray:
        rk = self.ranks()
        ri, rj = int(rk[i]), int(rk[j])
        return self._q("COUPLING", i, j, np.float64, ri * rj).reshape(rj, ri).T

    def factor(self, v: int) -> np.ndarray:
        m = self.rows(v)
        return self._q("FACTOR", v, 0, np.float64, m * m).reshape(m, m).T

    def times(self) -> np.ndarray:
        return self._q("TIMES", 0, 0, np.float64, 8)

    def device_bytes(self) -> int:
        return int(self._q("BYTES", 0, 0, np.int64, 1)[0])


class ULVFactor:
    def __init__(self, handle: int, n: int, device):
        self._h = C.c_void_p(handle)
        self.n = n
        self.device = device

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            try:
                lib.ulv_destroy(h)
            except Exception:
                pass
            self._h = None


# ------------------------------------------------------------------ entry points --
def h2_build(points: torch.Tensor, kernel: str, ell: float, shift: float, leaf: int = 64,
             tol: float = 1e-8, eta: float = 1.0, proxy_shells: int = 8, proxy_per_shell: int = 128,
             proxy_per_shell_max: int = 2048, proxy_density: float = 90.0, sketch_seed: int = 0x5EEDF00D,
             tree: str = "kd", stream=None) -> H2Matrix:
    if not points.is_cuda or points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be an (N, 3) float64 device tensor")
    points = points.contiguous()
    k = _Kernel(KERNELS[kernel], float(ell), float(shift))
    o = _h2_opts(leaf, eta, tol, dict(proxy_shells=proxy_shells, proxy_per_shell=proxy_per_shell,
                                      proxy_per_shell_max=proxy_per_shell_max,
                                      proxy_density=proxy_density, sketch_seed=sketch_seed, tree=tree))
    out = C.c_void_p()
    _check(lib.h2_build(points.data_ptr(), points.shape[0], k, C.byref(o), _stream(stream), C.byref(out)))
    # rows of the matrix: one per point, three for the RPY tensor
    rows = 3 * points.shape[0] if kernel == "rpy" else points.shape[0]
    return H2Matrix(out.value, rows, points.device)


def spdhss_build(A: H2Matrix, tol: float, max_rank: int = 100, oversample: int = 10, seed: int = 0,
                 omega: torch.Tensor | None = None, stream=None) -> HSSMatrix:
    s = max_rank + oversample
    if omega is not None:
        omega, nc, ld = _as_cols(omega, A.n)
        if nc != s or ld != A.n:
            raise ValueError("omega must be (N, max_rank + oversample) with ld = N")
    o = _HSSOpts(float(tol), int(max_rank), int(oversample), int(seed), _ptr(omega))
    out = C.c_void_p()
    _check(lib.spdhss_build(A._h, C.byref(o), _stream(stream), C.byref(out)))
    return HSSMatrix(out.value, A, s)


SOLVE_PRECISION = {"f64": 0, "f32": 1}


def ulv_factor(M: HSSMatrix, stream=None, precision: str = "f64") -> ULVFactor:
    """precision "f32": solve operators stored and read in FP32 (FP64 vectors
    and sums); PCG then uses the flexible beta."""
    out = C.c_void_p()
    _check(lib.ulv_factor_ex(M._h, SOLVE_PRECISION[precision], _stream(stream), C.byref(out)))
    return ULVFactor(out.value, M.n, M.device)


def ulv_apply(F: ULVFactor, b: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    b, nc, ld = _as_cols(b, F.n)
    if out is None:
        out = _out_like(b, F.n, nc, ld)
    _check_out(out, F.n, nc, ld)
    _check(lib.ulv_apply(F._h, b.data_ptr(), out.data_ptr(), nc, ld, _stream(stream)))
    return out


def ulv_apply_noalloc(F: ULVFactor, b: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """ulv_apply that allocates no device memory (the library's fixed per-GPU
    scratch array serves its buffers); out must be given."""
    b, nc, ld = _as_cols(b, F.n)
    _check_out(out, F.n, nc, ld)
    _check(lib.ulv_apply_noalloc(F._h, b.data_ptr(), out.data_ptr(), nc, ld, _stream(stream)))
    return out


def noalloc_bytes(F: ULVFactor, nrhs: int) -> int:
    """Bytes of the scratch array that ulv_apply_noalloc's vectors take."""
    return int(lib.spd_noalloc_bytes(F._h, int(nrhs)))


NOALLOC_SCRATCH_BYTES = 64 << 20


def h2_matvec(A: H2Matrix, x: torch.Tensor, out: torch.Tensor | None = None, stream=None,
              precision: str = "f64") -> torch.Tensor:
    """y = A x; precision "f32" streams FP32 copies of the near and coupling
    blocks (at most 16 columns, FP64 accumulation)."""
    x, nc, ld = _as_cols(x, A.n)
    if out is None:
        out = _out_like(x, A.n, nc, ld)
    _check_out(out, A.n, nc, ld)
    _check(lib.h2_matvec_ex(A._h, x.data_ptr(), out.data_ptr(), nc, ld, SOLVE_PRECISION[precision],
                            _stream(stream)))
    return out


def pcg_solve(A: H2Matrix, M: ULVFactor | None, b: torch.Tensor, rtol: float = 1e-8, maxit: int = 1000,
              out: torch.Tensor | None = None, stream=None, raise_on_nonconvergence: bool = True,
              op_precision: str = "f64"):
    """Returns (x, iterations per column, true relative residual per column).
    op_precision "f32": the iterations use the FP32-block product, with
    residual replacement by the FP64 product (at most 16 columns)."""
    b, nc, ld = _as_cols(b, A.n)
    if out is None:
        out = _out_like(b, A.n, nc, ld)
    _check_out(out, A.n, nc, ld)
    iters = np.zeros(nc, dtype=np.int32)
    relres = np.zeros(nc, dtype=np.float64)
    code = lib.pcg_solve_ex(A._h, None if M is None else M._h, b.data_ptr(), out.data_ptr(), nc, ld,
                            float(rtol), int(maxit), SOLVE_PRECISION[op_precision], _stream(stream),
                            iters.ctypes.data, relres.ctypes.data)
    if code == SPD_E_NOT_CONVERGED and not raise_on_nonconvergence:
        return out, iters, relres
    _check(code)
    return out, iters, relres


def near_field_roofline(A: H2Matrix, nrhs: int, reps: int = 20, stream=None) -> dict:
    """Average time and algorithmic bytes of the product's dominant kernel."""
    ms, b = C.c_double(), C.c_double()
    _check(lib.spd_h2_time_near(A._h, int(nrhs), int(reps), _stream(stream), C.byref(ms), C.byref(b)))
    return {"ms": ms.value, "bytes": b.value, "gbs": b.value / (ms.value * 1e-3) / 1e9}


def product_launch_times(A: H2Matrix, nrhs: int, reps: int = 10, stream=None) -> list[dict]:
    """Per-launch average time, algorithmic bytes and pass of h2_matvec, in issue order."""
    cap = 512
    ms = np.zeros(cap)
    by = np.zeros(cap)
    tg = np.zeros(cap, dtype=np.int32)
    cnt = C.c_int32()
    _check(lib.spd_h2_time_launches(A._h, int(nrhs), int(reps), _stream(stream), ms.ctypes.data,
                                    by.ctypes.data, tg.ctypes.data, cap, C.byref(cnt)))
    out = []
    for i in range(cnt.value):
        t = int(tg[i])
        name = {2: "coupling", 4: "leaf pass"}.get(t // 100, "")
        if t // 100 == 1:
            name = f"upward level {t % 100}"
        elif t // 100 == 3:
            name = f"downward level {t % 100}"
        out.append({"index": i, "pass": name or f"launch {i}", "ms": float(ms[i]), "bytes": float(by[i]),
                    "gbs": float(by[i] / (ms[i] * 1e-3) / 1e9) if ms[i] > 0 else 0.0})
    return out


# ------------------------------------------------------------------ kernel hooks --
# Matrices are passed as (batch, cols, rows) contiguous tensors, i.e. a batch
# of column-major rows x cols matrices.
def test_gemm(A, B, C_, transA=0, transB=0, alpha=1.0, beta=0.0):
    batch, n, m = C_.shape
    k = A.shape[1] if not transA else A.shape[2]
    _check(lib.spd_test_gemm(A.data_ptr(), B.data_ptr(), C_.data_ptr(), batch, m, n, k, transA, transB,
                             alpha, beta, _stream()))


def test_symm(A, X, Y, nblk, m, nterm, reps=0):
    """Y = S X for the block-cyclic symmetric layout of spd_test_symm (A holds
    nblk * nterm blocks of m x m, X and Y are (ncols, nblk * m)); with reps
    >= 1 returns the product launch's average time in ms."""
    n = X.shape[0]
    ms = C.c_double(0.0)
    _check(lib.spd_test_symm(A.data_ptr(), X.data_ptr(), Y.data_ptr(), int(nblk), int(m), int(nterm), n,
                             int(reps), _stream(), C.byref(ms) if reps > 0 else None))
    return ms.value


def test_chol(A, fail):
    _check(lib.spd_test_chol(A.data_ptr(), A.shape[0], A.shape[1], fail.data_ptr(), _stream()))


def test_trsm(L, B, trans=0, upper=0):
    _check(lib.spd_test_trsm(L.data_ptr(), B.data_ptr(), L.shape[0], L.shape[1], B.shape[1], trans, upper,
                             _stream()))


def test_cpqr(A, Q, piv, rank, diag, maxrank, tol, which):
    batch, n, m = A.shape
    _check(lib.spd_test_cpqr(A.data_ptr(), _ptr(Q), piv.data_ptr(), rank.data_ptr(), _ptr(diag),
                             batch, m, n, maxrank, tol, which, _stream()))


def _fill_instance(I: _Instance, d: dict):
    """Fill a request descriptor from a dict; returns the objects it points to."""
    P = d["points"]
    if not P.is_cuda or P.dtype != torch.float64 or P.dim() != 2 or P.shape[1] != 3:
        raise ValueError("points must be an (N, 3) float64 device tensor")
    P = P.contiguous()
    rows = 3 * P.shape[0] if d["kernel"] == "rpy" else P.shape[0]  # 3 rows a particle for the tensor
    b, nc, ld = _as_cols(d["b"], rows)
    if ld != rows:
        raise ValueError("b must have ld = N (3N for the RPY tensor)")
    x = cols_like(rows, nc, P.device)
    om = d.get("omega")
    if om is not None:
        om, nco, ldo = _as_cols(om, rows)
        if nco != int(d["max_rank"]) + int(d["oversample"]) or ldo != rows:
            raise ValueError("omega must be (rows, max_rank + oversample) with ld = rows")
    it = np.zeros(nc, dtype=np.int32)
    rr = np.zeros(nc, dtype=np.float64)
    I.points, I.n = P.data_ptr(), P.shape[0]
    I.kernel = _Kernel(KERNELS[d["kernel"]], float(d["ell"]), float(d["shift"]))
    I.h2 = _h2_opts(d["leaf"], d.get("eta", 1.0), d["h2_tol"], d)
    I.hss = _HSSOpts(float(d["hss_tol"]), int(d["max_rank"]), int(d["oversample"]), int(d.get("seed", 0)),
                     _ptr(om))
    I.solve_precision = SOLVE_PRECISION[d.get("precision", "f64")]
    I.b, I.x, I.nrhs = b.data_ptr(), x.data_ptr(), nc
    I.rtol, I.maxit = float(d["rtol"]), int(d["maxit"])
    I.iters, I.relres = it.ctypes.data, rr.ctypes.data
    return (P, b, x, om, it, rr)


class Server:
    """Request loop (spd_server_*): submit() queues a request dict (as for
    solve_batch), optionally with a matrix key, and returns a ticket;
    wait(ticket) returns its result with the queueing and total latency in
    seconds."""

    def __init__(self, workers: int = 8, hbm_budget_bytes: int = 200 << 30):
        h = C.c_void_p()
        _check(lib.spd_server_create(int(workers), int(hbm_budget_bytes), C.byref(h)))
        self._h = h
        self._pending = {}

    def footprint(self, d: dict) -> int:
        I = _Instance()
        keep = _fill_instance(I, d)  # noqa: F841
        return int(lib.spd_request_footprint(C.byref(I)))

    def submit(self, d: dict, key: int = 0) -> int:
        """key != 0 names the request's matrix: requests with the same key
        share device-resident H^2 / HSS / factor state (spd_server_submit_keyed)."""
        I = _Instance()
        keep = _fill_instance(I, d)
        torch.cuda.current_stream().synchronize()
        t = C.c_int64()
        if key:
            _check(lib.spd_server_submit_keyed(self._h, C.byref(I), C.c_uint64(int(key)), C.byref(t)))
        else:
            _check(lib.spd_server_submit(self._h, C.byref(I), C.byref(t)))
        self._pending[t.value] = (I, keep)
        return t.value

    PHASES = ("queued", "building", "solving", "finished")

    def phase(self, ticket: int) -> str:
        """Where a request not yet collected is (spd_server_phase)."""
        p = C.c_int32()
        _check(lib.spd_server_phase(self._h, int(ticket), C.byref(p)))
        return self.PHASES[p.value]

    def wait(self, ticket: int, block: bool = True):
        r = _InstanceResult()
        q, tot = C.c_double(), C.c_double()
        code = lib.spd_server_wait(self._h, int(ticket), 1 if block else 0, C.byref(r), C.byref(q), C.byref(tot))
        if code == 1:
            return None
        _check(code)
        I, (P, b, x, om, it, rr) = self._pending.pop(ticket)
        return {"x": x, "iters": it.copy(), "relres": rr.copy(), "status": STATUS_NAMES.get(r.status, r.status),
                "seconds_queued": q.value, "seconds_total": tot.value, "seconds_h2": r.seconds_h2,
                "seconds_build": r.seconds_build, "seconds_solve": r.seconds_solve}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.spd_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(instances: list[dict], workers: int = 8) -> list[dict]:
    """Run independent solve requests concurrently (spd_solve_batch).

    Each instance is a dict with points ((N, 3) FP64 device tensor), kernel,
    ell, shift, leaf, h2_tol, hss_tol, max_rank, oversample, b ((N, nrhs)
    column-major, ld = N), rtol, maxit and optionally omega ((N, max_rank +
    oversample), ld = N), seed, eta, the proxy options of h2_build and
    precision ("f64" or "f32").  Returns per instance: x, iters and relres
    per column, status and wall times."""
    n = len(instances)
    arr = (_Instance * max(n, 1))()
    res = (_InstanceResult * max(n, 1))()
    keep = [_fill_instance(arr[i], d) for i, d in enumerate(instances)]
    torch.cuda.synchronize()
    _check(lib.spd_solve_batch(arr, n, int(workers), res))
    out = []
    for i in range(n):
        P, b, x, om, it, rr = keep[i]
        r = res[i]
        out.append({"x": x, "iters": it.copy(), "relres": rr.copy(), "status": STATUS_NAMES.get(r.status, r.status),
                    "seconds_h2": r.seconds_h2, "seconds_build": r.seconds_build,
                    "seconds_solve": r.seconds_solve})
    return out
