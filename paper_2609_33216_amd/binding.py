"""Python binding of the symhss C-ABI (include/symhss.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts
NumPy / torch arrays to pointers and status codes to exceptions.  If the
library is missing it raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsymhss.so")

MULLER_SYM, MULLER_BASE, MULLER_SYM_TWOSIDED = 0, 1, 2
PMCHWT_SYM, PMCHWT_BASE, BURTON_MILLER = 3, 4, 5
DEVICE_PTRS = 1
OPT_GRAPHS, OPT_AUTOTUNE, OPT_PERSISTENT, OPT_PREDICTOR, OPT_PROXY_MARGIN = 0, 1, 2, 3, 4
OPT_PRECISION, OPT_REFINE_DIGITS, OPT_REFINE_MAXIT = 5, 6, 7
OPT_RANK_LEAF, OPT_RANK_SCALE, OPT_PIPELINE, OPT_DEVICE_LIMIT = 8, 9, 10, 11

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ESINGULAR, ERANK, ENOTCONV = range(8)
_STATUS = {
    0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "ESINGULAR", 6: "ERANK", 7: "ENOTCONV",
}


class SymhssError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"symhss {_STATUS.get(status, status)}: {msg}")
        self.status = status


class Medium(ctypes.Structure):
    _fields_ = [("k0", ctypes.c_double), ("k1", ctypes.c_double),
                ("eps0", ctypes.c_double), ("eps1", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("form", ctypes.c_int32), ("tol", ctypes.c_double),
                ("n_proxy", ctypes.c_int32), ("root_max", ctypes.c_int32), ("proxy_ratio", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("leaf_boxes", ctypes.c_int32), ("root_size", ctypes.c_int32),
                ("form", ctypes.c_int32),
                ("entries_compress", ctypes.c_int64), ("entries_factor", ctypes.c_int64),
                ("t_compress", ctypes.c_double), ("t_factor", ctypes.c_double), ("t_solve", ctypes.c_double),
                ("t_kblock_compress", ctypes.c_double), ("t_kblock_factor", ctypes.c_double),
                ("t_id", ctypes.c_double), ("t_lu", ctypes.c_double),
                ("device_bytes", ctypes.c_int64),
                ("rank_min", ctypes.c_int32 * 32), ("rank_max", ctypes.c_int32 * 32),
                ("rank_mean", ctypes.c_double * 32), ("proxy_max", ctypes.c_int32 * 32),
                ("n_kblock", ctypes.c_int32), ("n_id", ctypes.c_int32), ("n_lu", ctypes.c_int32),
                ("root_level", ctypes.c_int32),
                ("flops_id", ctypes.c_double), ("flops_lu_batched", ctypes.c_double),
                ("flops_lu_multi", ctypes.c_double), ("t_lu_batched", ctypes.c_double),
                ("t_lu_multi", ctypes.c_double), ("n_lu_batched", ctypes.c_int32),
                ("n_lu_multi", ctypes.c_int32), ("bytes_kblock", ctypes.c_double),
                ("graph_replays", ctypes.c_int32), ("tuned_buckets", ctypes.c_int32),
                ("pred_boxes", ctypes.c_int32), ("pred_fallbacks", ctypes.c_int32),
                ("proxy_rows", ctypes.c_int64), ("proxy_rows_rule", ctypes.c_int64),
                ("proxy_bytes", ctypes.c_double), ("proxy_bytes_rule", ctypes.c_double),
                ("refine_iters", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("fp32_residual", ctypes.c_double), ("refine_residual", ctypes.c_double),
                ("t_compress_wait", ctypes.c_double), ("t_host_plan", ctypes.c_double),
                ("t_host_ids", ctypes.c_double), ("t_host_post", ctypes.c_double),
                ("t_host_factor", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_
             if not f.startswith("rank") and f != "proxy_max"}
        L = self.levels
        d["rank_min"] = list(self.rank_min[1:L + 1])
        d["rank_max"] = list(self.rank_max[1:L + 1])
        d["rank_mean"] = [round(v, 2) for v in self.rank_mean[1:L + 1]]
        d["proxy_max"] = list(self.proxy_max[1:L + 1])
        return d


EXPORTS = [
    "symhss_create", "symhss_destroy", "symhss_last_error", "symhss_stream", "symhss_assemble",
    "symhss_compress", "symhss_factor", "symhss_factor_solve", "symhss_solve", "symhss_rhs_plane_wave",
    "symhss_eval_entries",
    "symhss_eval_bessel", "symhss_matvec_direct", "symhss_get_stats", "symhss_box_query",
    "symhss_assemble_batch", "symhss_rhs_plane_wave_batch", "symhss_configure",
    "symhss_predictor_train", "symhss_predictor_load", "symhss_predictor_get", "symhss_predictor_predict",
    "symhss_predictor_grad", "symhss_box_table", "symhss_hss_matvec", "symhss_solve_incident",
    "symhss_plane_wave", "symhss_predictor_predict_noalloc",
]

PREDICTOR_WEIGHTS = 8845
PREDICT_NOALLOC_MAX = 8192
N_FEATURES = 6


class TrainParams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("alpha", ctypes.c_float), ("seed", ctypes.c_uint64)]

_lib = None


def load(path: str | None = None):
    """Load libsymhss.so (built in-tree by paper_2609_33216_amd.build)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    try:
        # The library links libamdhip64.so.7 by soname; when torch is present its
        # bundled HIP runtime must be the one loaded, so that one runtime serves
        # both (torch tensors' device memory and streams are then usable here).
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2609_33216_amd.build`")
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "symhss_create": ([ctypes.POINTER(vp), ctypes.c_int, vp], ctypes.c_int),
        "symhss_destroy": ([vp], None),
        "symhss_last_error": ([vp], ctypes.c_char_p),
        "symhss_stream": ([vp], vp),
        "symhss_assemble": ([vp, i64, vp, vp, vp, ctypes.POINTER(Medium), ctypes.POINTER(Opts)], ctypes.c_int),
        "symhss_compress": ([vp], ctypes.c_int),
        "symhss_factor": ([vp], ctypes.c_int),
        "symhss_solve": ([vp, vp, vp, i32, i32], ctypes.c_int),
        "symhss_factor_solve": ([vp, vp, vp, i32, i32], ctypes.c_int),
        "symhss_rhs_plane_wave": ([vp, dbl, vp, i32], ctypes.c_int),
        "symhss_eval_entries": ([vp, i64, vp, i64, vp, vp], ctypes.c_int),
        "symhss_eval_bessel": ([vp, i64, vp, vp], ctypes.c_int),
        "symhss_matvec_direct": ([vp, vp, vp, i32], ctypes.c_int),
        "symhss_get_stats": ([vp, ctypes.POINTER(Stats)], ctypes.c_int),
        "symhss_box_query": ([vp, i32, i32, i32, ctypes.POINTER(i64), vp], ctypes.c_int),
        "symhss_assemble_batch": ([vp, i32, vp, vp, vp, vp, vp, ctypes.POINTER(Opts)], ctypes.c_int),
        "symhss_rhs_plane_wave_batch": ([vp, vp, vp, i32], ctypes.c_int),
        "symhss_configure": ([vp, i32, i64], ctypes.c_int),
        "symhss_predictor_train": ([vp, vp, vp, i64, ctypes.POINTER(TrainParams), vp], ctypes.c_int),
        "symhss_predictor_load": ([vp, vp, i64], ctypes.c_int),
        "symhss_predictor_get": ([vp, vp, i64], ctypes.c_int),
        "symhss_predictor_predict": ([vp, vp, i64, vp], ctypes.c_int),
        "symhss_predictor_grad": ([vp, vp, vp, vp, i64, ctypes.c_float, vp, vp], ctypes.c_int),
        "symhss_box_table": ([vp, ctypes.POINTER(i64), vp, vp, vp], ctypes.c_int),
        "symhss_hss_matvec": ([vp, vp, vp, i32], ctypes.c_int),
        "symhss_solve_incident": ([vp, vp, vp, vp, vp, i32, i32], ctypes.c_int),
        "symhss_plane_wave": ([vp, vp, vp, vp, i32], ctypes.c_int),
        "symhss_predictor_predict_noalloc": ([vp, vp, i64, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if path is None:
        _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Solver:
    """One solver context on one GPU."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load()
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    torch.cuda.set_device(device)
                    stream = torch.cuda.current_stream(device).cuda_stream
            except ImportError:
                stream = None
        h = ctypes.c_void_p()
        st = self.lib.symhss_create(ctypes.byref(h), device, ctypes.c_void_p(stream) if stream else None)
        if st != 0:
            raise SymhssError(st, "cannot create a context: " + self.lib.symhss_last_error(None).decode())
        self.h = h
        self.n = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.symhss_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            raise SymhssError(st, self.lib.symhss_last_error(self.h).decode())

    def configure(self, graphs: bool | None = None, autotune: bool | None = None, persistent: int | None = None,
                  predictor: bool | None = None, proxy_margin: int | None = None, mixed: bool | None = None,
                  refine_digits: int | None = None, refine_maxit: int | None = None,
                  rank_leaf: int | None = None, rank_scale: float | None = None, pipeline: bool | None = None,
                  device_limit: int | None = None):
        """Execution options (see symhss_configure); rank_scale is the growth a (e.g. 1.15)."""
        for opt, v in ((OPT_GRAPHS, graphs), (OPT_AUTOTUNE, autotune), (OPT_PERSISTENT, persistent),
                       (OPT_PREDICTOR, predictor), (OPT_PROXY_MARGIN, proxy_margin), (OPT_PRECISION, mixed),
                       (OPT_REFINE_DIGITS, refine_digits), (OPT_REFINE_MAXIT, refine_maxit),
                       (OPT_RANK_LEAF, rank_leaf), (OPT_PIPELINE, pipeline), (OPT_DEVICE_LIMIT, device_limit),
                       (OPT_RANK_SCALE, None if rank_scale is None else round(1000 * rank_scale))):
            if v is not None:
                self._check(self.lib.symhss_configure(self.h, opt, int(v)))

    # -- rank predictor --------------------------------------------------
    def predictor_train(self, feat, rank, epochs=200, batch=1024, lr=2e-3, alpha=4.0, seed=0):
        feat = np.ascontiguousarray(feat, dtype=np.float32)
        rank = np.ascontiguousarray(rank, dtype=np.float32)
        if feat.ndim != 2 or feat.shape[1] != N_FEATURES or rank.shape != (feat.shape[0],):
            raise ValueError("feat must be (n, 6) and rank (n,)")
        hist = np.zeros(epochs, dtype=np.float32)
        hp = TrainParams(epochs, batch, lr, alpha, seed)
        self._check(self.lib.symhss_predictor_train(self.h, _ptr(feat), _ptr(rank), feat.shape[0], ctypes.byref(hp),
                                                    _ptr(hist)))
        return hist

    def predictor_load(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self.lib.symhss_predictor_load(self.h, _ptr(w), w.size))

    def predictor_get(self):
        w = np.zeros(PREDICTOR_WEIGHTS, dtype=np.float32)
        self._check(self.lib.symhss_predictor_get(self.h, _ptr(w), w.size))
        return w

    def predictor_predict(self, feat):
        feat = np.ascontiguousarray(feat, dtype=np.float32)
        out = np.zeros(feat.shape[0], dtype=np.float32)
        self._check(self.lib.symhss_predictor_predict(self.h, _ptr(feat), feat.shape[0], _ptr(out)))
        return out

    def predictor_predict_noalloc(self, feat_ptr: int, n: int, rank_ptr: int):
        """Device-pointer inference (n x 6 float features -> n float ranks), queued
        on the context's stream without allocating or waiting."""
        self._check(self.lib.symhss_predictor_predict_noalloc(self.h, ctypes.c_void_p(feat_ptr), n,
                                                              ctypes.c_void_p(rank_ptr)))

    def predictor_grad(self, w, feat, rank, alpha):
        w = np.ascontiguousarray(w, dtype=np.float32)
        feat = np.ascontiguousarray(feat, dtype=np.float32)
        rank = np.ascontiguousarray(rank, dtype=np.float32)
        g = np.zeros(PREDICTOR_WEIGHTS - 2 * N_FEATURES, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        self._check(self.lib.symhss_predictor_grad(self.h, _ptr(w), _ptr(feat), _ptr(rank), feat.shape[0],
                                                   ctypes.c_float(alpha), _ptr(g), _ptr(loss)))
        return float(loss[0]), g

    def box_table(self):
        """(features (n, 6) float32, measured ranks (n,), info (n, 6)) of every compressed box."""
        cnt = ctypes.c_int64(0)
        self._check(self.lib.symhss_box_table(self.h, ctypes.byref(cnt), None, None, None))
        n = cnt.value
        feat = np.zeros((n, N_FEATURES), dtype=np.float32)
        rank = np.zeros(n, dtype=np.int32)
        info = np.zeros((n, 6), dtype=np.int32)
        if n:
            self._check(self.lib.symhss_box_table(self.h, ctypes.byref(cnt), _ptr(feat), _ptr(rank), _ptr(info)))
        return feat, rank, info

    # -- main verbs ------------------------------------------------------
    def assemble(self, x, dx, ddx, k0: float, k1: float, eps0: float = 1.0, eps1: float | None = None,
                 leaf: int = 128, tol: float = 1e-10, form: int = MULLER_SYM, n_proxy: int = 64,
                 proxy_ratio: float = 1.5, root_max: int = 0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        dx = np.ascontiguousarray(dx, dtype=np.float64)
        ddx = np.ascontiguousarray(ddx, dtype=np.float64)
        if x.ndim != 2 or x.shape[1] != 2 or dx.shape != x.shape or ddx.shape != x.shape:
            raise ValueError("x, dx, ddx must be (N, 2) arrays")
        if eps1 is None:
            eps1 = (k1 / k0) ** 2 * eps0
        med = Medium(k0, k1, eps0, eps1)
        opt = Opts(leaf, form, tol, n_proxy, root_max, proxy_ratio)
        self._check(self.lib.symhss_assemble(self.h, x.shape[0], _ptr(x), _ptr(dx), _ptr(ddx),
                                             ctypes.byref(med), ctypes.byref(opt)))
        self.n = x.shape[0]

    def assemble_batch(self, boundaries, media, leaf: int = 128, tol: float = 1e-10, form: int = MULLER_SYM,
                       n_proxy: int = 64, proxy_ratio: float = 1.5, root_max: int = 0):
        """boundaries: list of (x, dx, ddx) arrays of shape (N_t, 2); media: list of
        (k0, k1, eps0, eps1).  The unknowns of boundary t follow those of t-1."""
        if len(boundaries) != len(media) or not boundaries:
            raise ValueError("one medium per boundary")
        ns = np.array([np.asarray(b[0]).shape[0] for b in boundaries], dtype=np.int64)
        cat = []
        for a in range(3):
            arr = np.ascontiguousarray(np.concatenate([np.asarray(b[a], dtype=np.float64) for b in boundaries]))
            if arr.ndim != 2 or arr.shape != (int(ns.sum()), 2):
                raise ValueError("each of x, dx, ddx must be (N_t, 2)")
            cat.append(arr)
        meds = (Medium * len(media))(*[Medium(*m) for m in media])
        opt = Opts(leaf, form, tol, n_proxy, root_max, proxy_ratio)
        self._check(self.lib.symhss_assemble_batch(self.h, len(boundaries), _ptr(ns), _ptr(cat[0]), _ptr(cat[1]),
                                                   _ptr(cat[2]), ctypes.cast(meds, ctypes.c_void_p),
                                                   ctypes.byref(opt)))
        self.n = int(ns.sum())
        self.batch_n = [int(v) for v in ns]

    def rhs_plane_wave_batch(self, angles):
        a = np.ascontiguousarray(angles, dtype=np.float64)
        b = np.zeros(2 * self.n, dtype=np.complex128)
        self._check(self.lib.symhss_rhs_plane_wave_batch(self.h, _ptr(a), _ptr(b), 0))
        return b

    def rhs_plane_wave_batch_device(self, angles, b_ptr: int):
        a = np.ascontiguousarray(angles, dtype=np.float64)
        self._check(self.lib.symhss_rhs_plane_wave_batch(self.h, _ptr(a), ctypes.c_void_p(b_ptr), DEVICE_PTRS))

    def compress(self):
        self._check(self.lib.symhss_compress(self.h))

    def factor(self):
        self._check(self.lib.symhss_factor(self.h))

    def solve(self, b):
        """b: (2N,) or (2N, nrhs) complex; returns x of the same shape (host arrays)."""
        b = np.asarray(b, dtype=np.complex128)
        one = b.ndim == 1
        B = np.asfortranarray(b.reshape(b.shape[0], -1))
        if B.shape[0] != 2 * self.n:
            raise ValueError("b must have 2N rows")
        X = np.zeros_like(B, order="F")
        self._check(self.lib.symhss_solve(self.h, _ptr(B), _ptr(X), B.shape[1], 0))
        return X[:, 0].copy() if one else X

    def factor_solve(self, b):
        """factor() then solve(b) in one call (the solve's sweep up the levels
        beside the top-level LU); b as for solve."""
        b = np.asarray(b, dtype=np.complex128)
        one = b.ndim == 1
        B = np.asfortranarray(b.reshape(b.shape[0], -1))
        if B.shape[0] != 2 * self.n:
            raise ValueError("b must have 2N rows")
        X = np.zeros_like(B, order="F")
        self._check(self.lib.symhss_factor_solve(self.h, _ptr(B), _ptr(X), B.shape[1], 0))
        return X[:, 0].copy() if one else X

    def factor_solve_device(self, b_ptr: int, x_ptr: int, nrhs: int = 1):
        """factor_solve on HBM addresses of 2N x nrhs complex128."""
        self._check(self.lib.symhss_factor_solve(self.h, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr), nrhs,
                                                 DEVICE_PTRS))

    def solve_device(self, b_ptr: int, x_ptr: int, nrhs: int = 1):
        """Device-resident solve: b_ptr, x_ptr are HBM addresses of 2N x nrhs complex128."""
        self._check(self.lib.symhss_solve(self.h, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr), nrhs,
                                          DEVICE_PTRS))

    def solve_incident(self, uin, qin):
        """Traces (q, u) of the solution for incident data u_in, q_in = du_in/dnu at
        the nodes: (N,) or (N, nrhs) complex host arrays."""
        uin = np.asarray(uin, dtype=np.complex128)
        qin = np.asarray(qin, dtype=np.complex128)
        one = uin.ndim == 1
        U = np.asfortranarray(uin.reshape(uin.shape[0], -1))
        Q = np.asfortranarray(qin.reshape(qin.shape[0], -1))
        if U.shape != Q.shape or U.shape[0] != self.n:
            raise ValueError("u_in and q_in must both have N rows and the same columns")
        q = np.zeros_like(U, order="F")
        u = np.zeros_like(U, order="F")
        self._check(self.lib.symhss_solve_incident(self.h, _ptr(U), _ptr(Q), _ptr(q), _ptr(u), U.shape[1], 0))
        return (q[:, 0].copy(), u[:, 0].copy()) if one else (q, u)

    def plane_wave(self, angle):
        """(u_in, q_in) of the plane wave at the nodes; angle: one value, or one per boundary."""
        nt = len(getattr(self, "batch_n", [])) or 1
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(angle, dtype=np.float64), (nt,)))
        uin = np.zeros(self.n, dtype=np.complex128)
        qin = np.zeros(self.n, dtype=np.complex128)
        self._check(self.lib.symhss_plane_wave(self.h, _ptr(a), _ptr(uin), _ptr(qin), 0))
        return uin, qin

    def rhs_plane_wave(self, angle: float):
        b = np.zeros(2 * self.n, dtype=np.complex128)
        self._check(self.lib.symhss_rhs_plane_wave(self.h, angle, _ptr(b), 0))
        return b

    def rhs_plane_wave_device(self, angle: float, b_ptr: int):
        self._check(self.lib.symhss_rhs_plane_wave(self.h, angle, ctypes.c_void_p(b_ptr), DEVICE_PTRS))

    def eval_entries(self, rows, cols):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.zeros((len(rows), len(cols)), dtype=np.complex128, order="F")
        self._check(self.lib.symhss_eval_entries(self.h, len(rows), _ptr(rows), len(cols), _ptr(cols), _ptr(out)))
        return out

    def eval_bessel(self, z):
        z = np.ascontiguousarray(z, dtype=np.float64)
        out = np.zeros((len(z), 5), dtype=np.float64)
        self._check(self.lib.symhss_eval_bessel(self.h, len(z), _ptr(z), _ptr(out)))
        return out

    def hss_matvec(self, x):
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.zeros_like(x)
        self._check(self.lib.symhss_hss_matvec(self.h, _ptr(x), _ptr(y), 0))
        return y

    def matvec_direct(self, x):
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.zeros_like(x)
        self._check(self.lib.symhss_matvec_direct(self.h, _ptr(x), _ptr(y), 0))
        return y

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.symhss_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def box_query(self, level: int, box: int, what: int):
        cnt = ctypes.c_int64(0)
        self._check(self.lib.symhss_box_query(self.h, level, box, what, ctypes.byref(cnt), None))
        n = cnt.value
        if what in (8, 9):
            out = np.zeros(n, dtype=np.complex128)
        elif what == 10:
            out = np.zeros(n, dtype=np.float64)
        elif what == 16:
            out = np.zeros(n, dtype=np.int32)
        else:
            out = np.zeros(n, dtype=np.int32)
        if n:
            self._check(self.lib.symhss_box_query(self.h, level, box, what, ctypes.byref(cnt), _ptr(out)))
        return out

    def box_interp(self, level: int, box: int):
        """(R, L) dense interpolation matrices of a box (column-major from the device)."""
        kcq, kcu, krq, kru = self.box_query(level, box, 15)
        sc = len(self.box_query(level, box, 0)) + len(self.box_query(level, box, 1))
        sr = len(self.box_query(level, box, 2)) + len(self.box_query(level, box, 3))
        R = self.box_query(level, box, 8).reshape(sc, kcq + kcu).T
        L = self.box_query(level, box, 9).reshape(krq + kru, sr).T
        return R, L
