"""ctypes binding of libgaca (names follow include/gaca.h)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgaca.so")
_lib = None

P = ctypes.c_void_p
I32, I64, F64, U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64

ABI_VERSION = 3   # GACA_ABI_VERSION of include/gaca.h that these structures follow
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "HIP", -4: "STATE", -5: "NOT_CONVERGED",
          -6: "UNSUPPORTED"}
SCHEMES = {"collocation": 0, "galerkin": 1, "p1": 2, "galerkin_p1": 3}
KERNELS = {"slp": 0, "dlp": 1, "hyp": 2, "adlp": 3}
PRECISIONS = {"fp64": 0, "mixed": 1}
MODES = {"sum": 0, "per_freq": 1}


class GacaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gaca error {STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("leaf_size", I32), ("eta", F64), ("eps3d", F64), ("eps_aca", F64),
                ("precision", I32), ("quad_mid", I32), ("quad_near", I32), ("n_duffy", I32),
                ("n_galerkin", I32), ("n_touch", I32), ("tie", F64),
                ("delta_zero", F64), ("max_rank3d", I32), ("max_face_rank", I32),
                ("max_device_bytes", U64), ("batch_bytes", U64), ("threads_small", I32),
                ("threads_large", I32), ("verbose", I32), ("zero_rows_batch", I32),
                ("recompress", I32), ("pivot_estimate", I32), ("near_aca", I32),
                ("autotune_cache", ctypes.c_char_p)]


class Stats(ctypes.Structure):
    _fields_ = [("n_far", I64), ("n_near", I64), ("rank_min", I32), ("rank_max", I32),
                ("rank_mean", F64), ("face_rank_max", I32), ("face_rank_mean", F64),
                ("n_capped", I64), ("n_zero_blocks", I64), ("bytes_far", U64),
                ("bytes_near", U64), ("dense_bytes", F64), ("compression", F64),
                ("entries_near", F64), ("entries_near_mirrored", F64), ("entries_face", F64), ("entries_fibre", F64),
                ("entries_face_kernel", F64), ("ms_near", F64), ("ms_far", F64),
                ("ms_total", F64), ("ms_near_kernel", F64), ("ms_far_kernel", F64),
                ("n_far_launches", I32), ("far_iters", I32), ("far_flops", F64),
                ("far_kernel_evals", F64), ("near_kernel_evals", F64),
                ("ms_far_phase", F64 * 4), ("launches_phase", I32 * 4),
                ("far_flops_phase", F64 * 4), ("far_bytes_phase", F64 * 4),
                ("ms_far_by_kind", F64 * 4),
                ("launches_by_kind", I32 * 4), ("far_flops_by_kind", F64 * 4),
                ("ms_far_large_path", F64 * 3), ("launches_large_path", I32 * 3),
                ("far_flops_large_path", F64 * 3), ("threads_large_used", I32),
                ("threads_small_used", I32), ("autotune_state", I32),
                ("ms_far_aca_block_max", F64), ("ms_host_setup", F64), ("ms_host_finish", F64),
                ("ms_apply", F64), ("apply_flops", F64), ("apply_operator_bytes", F64),
                ("ms_apply_part", F64 * 3), ("apply_flops_part", F64 * 3), ("arena_in_place", I32),
                ("joint_build", I32), ("near_rank_max", I32), ("n_near_compressed", I64),
                ("near_rank_mean", F64), ("ms_near_aca", F64)]


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libgaca.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python paper_2312_11219_amd/build.py` (or __graft_entry__.build())")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7 (same SONAME as the
    # system one libgaca links against).  Loading torch first makes libgaca bind to the
    # runtime torch uses, so device pointers and streams are shared with it.
    import torch  # noqa: F401
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "gaca_abi_version": (I32, []),
        "gaca_last_error": (ctypes.c_char_p, []),
        "gaca_options_default": (None, [P]),
        "gaca_context_create": (I32, [ctypes.c_int, P, P]),
        "gaca_context_destroy": (I32, [P]),
        "gaca_context_memory": (I32, [P, P]),
        "gaca_problem_create": (I32, [P, P, I64, P, I64, P, P, I32, ctypes.c_int, P, P]),
        "gaca_problem_destroy": (I32, [P]),
        "gaca_problem_perm": (I32, [P, P]),
        "gaca_problem_block_counts": (I32, [P, P, P]),
        "gaca_problem_blocks": (I32, [P, P, P]),
        "gaca_partition_host": (I32, [P, I64, P, I64, I32, F64, P, I64, P, P, P, P]),
        "gaca_build": (I32, [P, ctypes.c_int, P]),
        "gaca_build_both": (I32, [P, P, P]),
        "gaca_hmatrix_destroy": (I32, [P]),
        "gaca_hmatrix_stats": (I32, [P, P]),
        "gaca_hmatrix_freq_hist": (I32, [P, P]),
        "gaca_hmatrix_block_info": (I32, [P, I64, P]),
        "gaca_hmatrix_block_export": (I32, [P, I64, P, P, P, P, P, P, P]),
        "gaca_hmatrix_near_export": (I32, [P, I64, P]),
        "gaca_hmatrix_near_ranks": (I32, [P, P]),
        "gaca_partition_host_p1": (I32, [P, I64, P, I64, I32, F64, P, I64, P, P, P, P]),
        "gaca_apply": (I32, [P, ctypes.c_int, I32, P, P, ctypes.c_int, P]),
        "gaca_apply_noalloc": (I32, [P, ctypes.c_int, I32, P, P, ctypes.c_int, P]),
        "gaca_eval_entries": (I32, [P, ctypes.c_int, I64, P, P, P, P, P]),
        "gaca_eval_far_entries_mixed": (I32, [P, ctypes.c_int, I64, I64, P, P, P, P]),
        "gaca_compress_tensor": (I32, [P, P, I64, I64, I32, P, P]),
        "gaca_quadrature_rule": (I32, [ctypes.c_int, ctypes.c_int, P, P]),
        "gaca_gcq_contour": (I32, [I32, P, F64, F64, I32, P, P, P, P]),
        "gaca_gcq_history": (I32, [P, I32, P, P, F64, F64, P, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.gaca_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{_LIB_PATH} has ABI version {lib.gaca_abi_version()}, the binding "
                           f"expects {ABI_VERSION}: rebuild the library")
    _lib = lib
    return lib


def _check(code, allow=()):
    if code != 0 and code not in allow:
        raise GacaError(code, load_library().gaca_last_error().decode())
    return code


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(P)


def options_default(**overrides) -> Options:
    lib = load_library()
    o = Options()
    lib.gaca_options_default(ctypes.byref(o))
    for k, v in overrides.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "autotune_cache" and isinstance(v, str):
            v = v.encode()
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def quadrature_rule(kind: str, n: int):
    """The library's own tables: ('gauss', n) -> (nodes, weights) on [0, 1];
    ('triangle6', 6) -> (barycentric 6 x 3, weights)."""
    lib = load_library()
    if kind == "gauss":
        x = np.zeros(n)
        w = np.zeros(n)
        _check(lib.gaca_quadrature_rule(0, n, _ptr(x), _ptr(w)))
        return x, w
    x = np.zeros(18)
    w = np.zeros(6)
    _check(lib.gaca_quadrature_rule(1, 6, _ptr(x), _ptr(w)))
    return x.reshape(6, 3), w


def gcq_contour(rk_A, dt_min, dt_max, n_q):
    """gCQ integration points and weights (library's own computation): (s, omega)."""
    lib = load_library()
    A = np.ascontiguousarray(rk_A, dtype=np.float64)
    m = A.shape[0]
    sr, si, wr, wi = (np.zeros(n_q) for _ in range(4))
    _check(lib.gaca_gcq_contour(m, _ptr(A), dt_min, dt_max, n_q, _ptr(sr), _ptr(si), _ptr(wr),
                                _ptr(wi)))
    return sr + 1j * si, wr + 1j * wi


def partition_host(xyz, tri, leaf_size, eta, scheme="collocation"):
    """Host-only tree + partition: (perm, far (nf,4), near (nn,4)); scheme "p1": over the
    vertices."""
    lib = load_library()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    M = tri.shape[0]
    n = xyz.shape[0] if scheme == "p1" else M
    fn = lib.gaca_partition_host_p1 if scheme == "p1" else lib.gaca_partition_host
    perm = np.zeros(n, dtype=np.int64)
    cap = max(16, 4 * n * n // max(1, leaf_size) // max(1, leaf_size) + 64)
    cap = min(cap, 50_000_000)
    while True:
        far = np.zeros((cap, 4), dtype=np.int64)
        near = np.zeros((cap, 4), dtype=np.int64)
        nf, nn = I64(0), I64(0)
        rc = fn(_ptr(xyz), xyz.shape[0], _ptr(tri), M, leaf_size, eta,
                                     _ptr(perm), cap, _ptr(far), ctypes.byref(nf), _ptr(near),
                                     ctypes.byref(nn))
        if rc == 0:
            return perm, far[:nf.value], near[:nn.value]
        if max(nf.value, nn.value) > cap:
            cap = max(nf.value, nn.value)
            continue
        _check(rc)


class Context:
    def __init__(self, device: int = 0, stream=None):
        self._lib = load_library()
        h = P()
        sp = None
        if stream is not None:
            sp = P(stream if isinstance(stream, int) else stream.cuda_stream)
        _check(self._lib.gaca_context_create(device, sp, ctypes.byref(h)))
        self.handle = h

    def memory_in_use(self) -> int:
        v = U64(0)
        _check(self._lib.gaca_context_memory(self.handle, ctypes.byref(v)))
        return v.value

    def close(self):
        if self.handle:
            self._lib.gaca_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    def __init__(self, ctx: Context, xyz, tri, s, scheme="collocation", **options):
        self._lib = load_library()
        self.ctx = ctx
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        s = np.asarray(s, dtype=np.complex128)
        self.s = s
        self.L = s.shape[0]
        # operator size: elements, or vertices for the P1 double layer
        self.M = self.xyz.shape[0] if scheme in ("p1", "galerkin_p1") else self.tri.shape[0]
        s_re = np.ascontiguousarray(s.real)
        s_im = np.ascontiguousarray(s.imag)
        self.opt = options_default(**options)
        h = P()
        _check(self._lib.gaca_problem_create(ctx.handle, _ptr(self.xyz), self.xyz.shape[0],
                                             _ptr(self.tri), self.tri.shape[0], _ptr(s_re), _ptr(s_im),
                                             self.L, SCHEMES[scheme], ctypes.byref(self.opt),
                                             ctypes.byref(h)))
        self.handle = h

    @property
    def perm(self):
        out = np.zeros(self.M, dtype=np.int64)
        _check(self._lib.gaca_problem_perm(self.handle, _ptr(out)))
        return out

    def blocks(self):
        nf, nn = I64(0), I64(0)
        _check(self._lib.gaca_problem_block_counts(self.handle, ctypes.byref(nf), ctypes.byref(nn)))
        far = np.zeros((nf.value, 4), dtype=np.int64)
        near = np.zeros((nn.value, 4), dtype=np.int64)
        _check(self._lib.gaca_problem_blocks(self.handle, _ptr(far), _ptr(near)))
        return far, near

    def build(self, kernel="slp", allow_not_converged=True) -> "HMatrix":
        h = P()
        allow = (-5,) if allow_not_converged else ()
        rc = _check(self._lib.gaca_build(self.handle, KERNELS[kernel], ctypes.byref(h)), allow)
        return HMatrix(self, h, kernel, converged=(rc == 0))

    def build_both(self, allow_not_converged=True):
        """Single and double layer operators built together (gaca_build_both)."""
        hs, hd = P(), P()
        allow = (-5,) if allow_not_converged else ()
        rc = _check(self._lib.gaca_build_both(self.handle, ctypes.byref(hs), ctypes.byref(hd)), allow)
        return (HMatrix(self, hs, "slp", converged=(rc == 0)),
                HMatrix(self, hd, "dlp", converged=(rc == 0)))

    def eval_entries(self, kernel, i, j, k, far):
        i = np.ascontiguousarray(i, dtype=np.int32)
        j = np.ascontiguousarray(j, dtype=np.int32)
        k = np.ascontiguousarray(k, dtype=np.int32)
        far = np.ascontiguousarray(far, dtype=np.int32)
        n = i.shape[0]
        out = np.zeros(2 * max(n, 1), dtype=np.float64)
        _check(self._lib.gaca_eval_entries(self.handle, KERNELS[kernel], n, _ptr(i), _ptr(j),
                                           _ptr(k), _ptr(far), _ptr(out)))
        return out[0:2 * n:2] + 1j * out[1:2 * n:2]

    def eval_far_entries_mixed(self, kernel, block, il, jl, k):
        """Mixed-precision face entries of far block `block` (tree-local il, jl) times c_k."""
        il = np.ascontiguousarray(il, dtype=np.int32)
        jl = np.ascontiguousarray(jl, dtype=np.int32)
        k = np.ascontiguousarray(k, dtype=np.int32)
        n = il.shape[0]
        out = np.zeros(2 * max(n, 1), dtype=np.float64)
        _check(self._lib.gaca_eval_far_entries_mixed(self.handle, KERNELS[kernel], block, n,
                                                     _ptr(il), _ptr(jl), _ptr(k), _ptr(out)))
        return out[0:2 * n:2] + 1j * out[1:2 * n:2]

    def close(self):
        if getattr(self, "handle", None):
            self._lib.gaca_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HMatrix:
    def __init__(self, problem, handle, kernel, converged=True, L=None):
        self._lib = load_library()
        self.problem = problem
        self.handle = handle
        self.kernel = kernel
        self.converged = converged
        self.L = L if L is not None else problem.L

    def stats(self) -> dict:
        st = Stats()
        _check(self._lib.gaca_hmatrix_stats(self.handle, ctypes.byref(st)))
        out = {}
        for name, _ in Stats._fields_:
            v = getattr(st, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out

    def freq_hist(self):
        out = np.zeros(self.L, dtype=np.int64)
        _check(self._lib.gaca_hmatrix_freq_hist(self.handle, _ptr(out)))
        return out

    def block_info(self, idx):
        info = np.zeros(9, dtype=np.int64)
        _check(self._lib.gaca_hmatrix_block_info(self.handle, idx, _ptr(info)))
        return dict(r0=int(info[0]), m=int(info[1]), c0=int(info[2]), n=int(info[3]),
                    rank=int(info[4]), sum_rho=int(info[5]), capped=int(info[6]),
                    zero_faces=int(info[7]), aca_ticks=int(info[8]))

    def export_block(self, idx):
        inf = self.block_info(idx)
        r, sr, m, n, L = inf["rank"], inf["sum_rho"], inf["m"], inf["n"], self.L
        ks = np.zeros(max(r, 1), np.int32)
        pi = np.zeros(max(r, 1), np.int32)
        pj = np.zeros(max(r, 1), np.int32)
        rho = np.zeros(max(r, 1), np.int32)
        U = np.zeros(2 * max(sr * m, 1))
        W = np.zeros(2 * max(sr * n, 1))
        F = np.zeros(2 * max(r * L, 1))
        _check(self._lib.gaca_hmatrix_block_export(self.handle, idx, _ptr(ks), _ptr(pi), _ptr(pj),
                                                   _ptr(rho), _ptr(U), _ptr(W), _ptr(F)))
        Uc = U[0::2] + 1j * U[1::2]
        Wc = W[0::2] + 1j * W[1::2]
        Fc = (F[0::2] + 1j * F[1::2])[:r * L].reshape(r, L)
        crosses = []
        uo = wo = 0
        for c in range(r):
            p = int(rho[c])
            Ul = Uc[uo:uo + p * m].reshape(p, m).T
            Wl = Wc[wo:wo + p * n].reshape(p, n).T
            uo += p * m
            wo += p * n
            crosses.append(dict(k=int(ks[c]), i=int(pi[c]), j=int(pj[c]), rho=p, U=Ul, W=Wl,
                                f=Fc[c]))
        inf["crosses"] = crosses
        return inf

    def near_block(self, idx, m, n):
        out = np.zeros(2 * m * n * self.L)
        _check(self._lib.gaca_hmatrix_near_export(self.handle, idx, _ptr(out)))
        return (out[0::2] + 1j * out[1::2]).reshape(m, self.L, n)

    def near_ranks(self):
        """3D-ACA rank per near block (-1: stored dense)."""
        out = np.zeros(int(self.stats()["n_near"]), dtype=np.int32)
        _check(self._lib.gaca_hmatrix_near_ranks(self.handle, _ptr(out)))
        return out

    def apply(self, X, mode="sum", Y=None, stream=None, noalloc=False):
        """X: torch complex tensor [L, M, nrhs] on the GPU (original element order).
        noalloc: gaca_apply_noalloc (workspace in the library's fixed scratch array)."""
        import torch
        if X.dim() != 3 or X.shape[0] != self.L:
            raise ValueError("X must be [L, M, nrhs]")
        if not X.is_cuda or not X.is_contiguous():
            raise ValueError("X must be a contiguous GPU tensor")
        dtype = {torch.complex128: 0, torch.complex64: 1}[X.dtype]
        L, M, nrhs = X.shape
        if Y is None:
            shape = (M, nrhs) if mode == "sum" else (L, M, nrhs)
            Y = torch.empty(shape, dtype=X.dtype, device=X.device)
        sp = P(stream.cuda_stream) if stream is not None else P(torch.cuda.current_stream().cuda_stream)
        fn = self._lib.gaca_apply_noalloc if noalloc else self._lib.gaca_apply
        _check(fn(self.handle, MODES[mode], nrhs, P(X.data_ptr()), P(Y.data_ptr()), dtype, sp))
        return Y

    def gcq_history(self, rk_A, rk_b, dt_prev, dt_cur, w, theta_prev, x, W, Y, stream=None):
        """gCQ history step on device tensors (complex128, original order): updates x in
        place, fills W and writes the history term into Y [M][stages]."""
        import torch
        A = np.ascontiguousarray(rk_A, dtype=np.float64)
        b = np.ascontiguousarray(rk_b, dtype=np.float64)
        w = np.asarray(w, dtype=np.complex128)
        wr, wi = np.ascontiguousarray(w.real), np.ascontiguousarray(w.imag)
        for t in (theta_prev, x, W, Y):
            if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.complex128):
                raise ValueError("gcq_history needs contiguous complex128 GPU tensors")
        sp = P(stream.cuda_stream) if stream is not None else P(torch.cuda.current_stream().cuda_stream)
        _check(self._lib.gaca_gcq_history(self.handle, A.shape[0], _ptr(A), _ptr(b), dt_prev, dt_cur,
                                          _ptr(wr), _ptr(wi), P(theta_prev.data_ptr()),
                                          P(x.data_ptr()), P(W.data_ptr()), P(Y.data_ptr()), sp))
        return Y

    def close(self):
        if getattr(self, "handle", None):
            self._lib.gaca_hmatrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compress_tensor(ctx: Context, T, **options) -> HMatrix:
    """3D-ACA of a dense device tensor T (torch complex128 [m, n, L])."""
    lib = load_library()
    m, n, L = T.shape
    opt = options_default(**options)
    h = P()
    rc = _check(lib.gaca_compress_tensor(ctx.handle, P(T.data_ptr()), m, n, L, ctypes.byref(opt),
                                         ctypes.byref(h)), (-5,))
    hm = HMatrix(None, h, "tensor", converged=(rc == 0), L=L)
    hm.ctx = ctx   # the operator uses its context until it is destroyed
    return hm
