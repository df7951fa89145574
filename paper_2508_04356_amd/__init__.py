"""Python binding of libgdsw (include/gdsw.h): argument marshalling only.

Every operation runs in the HIP library; this module converts torch tensors
to device pointers and the current torch stream to a hipStream_t.  Importing
the package loads the library and raises if it has not been built
(``python -m paper_2508_04356_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# torch ships its own HIP runtime (libamdhip64.so.7, libhsa-runtime64.so.1).
# Loading it before the library makes the dynamic loader bind libgdsw.so to
# that same runtime, so one process never holds two HSA runtimes.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# GDSW_LIBRARY selects another build of the same library (e.g. one compiled
# with different launch-shape constants by build.py --out ... -D ...).
LIB_PATH = os.environ.get("GDSW_LIBRARY") or os.path.join(_HERE, "libgdsw.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2508_04356_amd/build.py`")
_lib = C.CDLL(LIB_PATH)

FP64, FP32, BF16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
LOCAL_SOLVES = {"inverse": 0, "triangular": 1, "symmetric": 2, "block": 3}
PRESSURE_ELEMENTS = {"q1": 0, "p1disc": 1}
COARSE_SPACES = {"gdsw": 0, "gdsw*": 1}
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "ESINGULAR", 4: "ENOCONV", 5: "EDEVICE", 6: "EUNSUPPORTED"}


class Mesh(C.Structure):
    _fields_ = [("n", C.c_int32), ("manufactured_force", C.c_int32), ("viscosity", C.c_double),
                ("inflow_amplitude", C.c_double), ("pressure_element", C.c_int32)]


class Decomposition(C.Structure):
    _fields_ = [("subdomains", C.c_int32), ("overlap", C.c_int32), ("levels", C.c_int32), ("group", C.c_int32),
                ("local_precision", C.c_int32), ("tile", C.c_int32), ("local_algebraic", C.c_int32),
                ("level2_layer", C.c_int32), ("device_mem_budget", C.c_uint64), ("local_solve", C.c_int32),
                ("max_rhs", C.c_int32), ("coarse_space", C.c_int32)]


class FgmresOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("max_it", C.c_int32), ("use_graph", C.c_int32),
                ("history_len", C.c_int32), ("history", C.POINTER(C.c_double))]


class FgmresInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("t_solve_s", C.c_double), ("learned_solves", C.c_int64),
                ("fallbacks", C.c_int64)]


class AlgebraicProblem(C.Structure):
    _fields_ = [("n", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("rhs", C.c_void_p), ("field", C.c_void_p), ("null_value", C.c_void_p), ("n_sub", C.c_int32),
                ("sub_ptr", C.c_void_p), ("sub_idx", C.c_void_p)]


class Sizes(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n_free", "n_full", "n_u_free", "n_p", "nnz", "n_sub", "n_entities",
                                         "n_coarse", "n_subregions", "n_coarse3", "local_min", "local_max")] + \
               [(k, C.c_uint64) for k in ("factor_bytes", "coarse_bytes", "device_bytes", "solve_bytes")] + \
               [("solve_launches", C.c_int64)]


class LearnedInfo(C.Structure):
    _fields_ = [("grid", C.c_int32), ("subdomains", C.c_int32), ("n_params", C.c_int64), ("samples", C.c_int32),
                ("reserved", C.c_int32), ("sigma", C.c_float * 4)]


_P = C.c_void_p
_sig = {
    "gdsw_setup": (C.c_int, [C.POINTER(Mesh), C.POINTER(Decomposition), _P, C.POINTER(_P)]),
    "gdsw_setup_host": (C.c_int, [C.POINTER(Mesh), C.POINTER(Decomposition), C.POINTER(_P)]),
    "gdsw_setup_algebraic": (C.c_int, [C.POINTER(AlgebraicProblem), C.POINTER(Decomposition), _P, C.POINTER(_P)]),
    "gdsw_setup_algebraic_host": (C.c_int, [C.POINTER(AlgebraicProblem), C.POINTER(Decomposition), C.POINTER(_P)]),
    "gdsw_get_sizes": (C.c_int, [_P, C.POINTER(Sizes)]),
    "gdsw_dof_map": (C.c_int, [_P, _P, _P]),
    "gdsw_host_matrix": (C.c_int, [_P, _P, _P, _P]),
    "gdsw_host_rhs": (C.c_int, [_P, _P]),
    "gdsw_rhs": (C.c_int, [_P, _P, _P]),
    "gdsw_spmv": (C.c_int, [_P, _P, _P, _P]),
    "gdsw_apply_precond": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P]),
    "gdsw_apply_precond_noalloc": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P]),
    "gdsw_fgmres_solve": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, C.POINTER(FgmresOpts),
                                    C.POINTER(FgmresInfo), _P]),
    "gdsw_expand_solution": (C.c_int, [_P, _P, _P, _P]),
    "gdsw_copy_coarse_matrix": (C.c_int, [_P, _P]),
    "gdsw_copy_coarse_basis": (C.c_int, [_P, _P]),
    "gdsw_local_indices": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_int32)]),
    "gdsw_profile_apply": (C.c_int, [_P, _P, _P, _P, _P]),
    "gdsw_autotune": (C.c_int, [_P, _P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "gdsw_autotune_mfma": (C.c_int, [_P, _P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "gdsw_kernel_timer": (C.c_int, [_P, C.c_int32]),
    "gdsw_kernel_timer_read": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]),
    "gdsw_set_schedule": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    "gdsw_learned_init": (C.c_int, [_P, C.c_uint64, C.POINTER(LearnedInfo), _P]),
    "gdsw_learned_train": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_uint64, _P, _P]),
    "gdsw_learned_weights": (C.c_int, [_P, _P, _P, C.c_int32, _P]),
    "gdsw_learned_loss_grad": (C.c_int, [_P, _P, _P, C.c_int32, C.POINTER(C.c_double), _P, _P]),
    "gdsw_set_local_solver": (C.c_int, [_P, C.c_int32, C.c_double]),
    "gdsw_learned_stats": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "gdsw_learned_copy": (C.c_int, [_P, _P, _P]),
    "gdsw_learned_save": (C.c_int, [_P, C.c_char_p, _P]),
    "gdsw_learned_load": (C.c_int, [_P, C.c_char_p, _P]),
    "gdsw_train_local_net": (C.c_int, [_P, C.c_char_p, C.c_int32, C.c_uint64, _P]),
    "gdsw_setup_times": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gdsw_last_error": (C.c_char_p, [_P]),
    "gdsw_destroy": (None, [_P]),
    "gdsw_setup_batch": (C.c_int, [C.POINTER(Mesh), C.POINTER(Decomposition), C.c_int32, _P, C.POINTER(_P)]),
    "gdsw_batch_member": (C.c_int, [_P, C.c_int32, C.POINTER(_P)]),
    "gdsw_apply_precond_batch": (C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), _P]),
    "gdsw_fgmres_solve_batch": (C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(FgmresOpts),
                                          C.POINTER(FgmresInfo), _P]),
    "gdsw_batch_kernel_timer": (C.c_int, [_P, C.c_int32]),
    "gdsw_batch_kernel_timer_read": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                               C.POINTER(C.c_uint64)]),
    "gdsw_destroy_batch": (None, [_P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class GdswError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


def _check(status, ctx=None):
    if status != 0:
        msg = _lib.gdsw_last_error(ctx)
        raise GdswError(status, msg.decode() if msg else "")


def _stream(stream):
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        return C.c_void_p(0)
    return C.c_void_p(int(stream))


def _ptr(t):
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return C.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(int(t))


class Solver:
    """One Stokes problem with its GDSW preconditioner (a gdsw_ctx)."""

    def __init__(self, n, m, overlap=1, levels=2, group=2, precision="fp64", tile=0, viscosity=1.0,
                 inflow=16.0, manufactured=0, budget=0, host_only=False, stream=None, local_algebraic=0,
                 level2_layer=0, local_solve="inverse", max_rhs=1, pressure="q1", coarse="gdsw"):
        self._ctx = C.c_void_p()
        self.mesh = Mesh(n, manufactured, viscosity, inflow, PRESSURE_ELEMENTS[pressure])
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        solve = LOCAL_SOLVES[local_solve] if isinstance(local_solve, str) else int(local_solve)
        self.dec = Decomposition(m, overlap, levels, group, prec, tile, int(local_algebraic), int(level2_layer),
                                 budget, solve, int(max_rhs), COARSE_SPACES[coarse])
        if host_only:
            st = _lib.gdsw_setup_host(C.byref(self.mesh), C.byref(self.dec), C.byref(self._ctx))
        else:
            st = _lib.gdsw_setup(C.byref(self.mesh), C.byref(self.dec), _stream(stream), C.byref(self._ctx))
        _check(st)
        self.host_only = host_only
        s = self.sizes()
        self.n_free = s.n_free
        self.n_coarse = s.n_coarse

    @classmethod
    def algebraic(cls, row_ptr, col, val, field, dof_subs, null=None, rhs=None, overlap=1, precision="fp64",
                  tile=0, budget=0, local_solve="inverse", max_rhs=1, host_only=False, stream=None):
        """A problem given as its assembled matrix (CSR, host arrays) and the
        subdomains holding each DOF (dof_subs: a list of sorted index lists,
        or a (ptr, idx) pair)."""
        self = cls.__new__(cls)
        self._ctx = C.c_void_p()
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a.ctypes.data_as(C.c_void_p)

        if isinstance(dof_subs, tuple):
            sptr, sidx = dof_subs
        else:
            sptr = np.zeros(len(dof_subs) + 1, dtype=np.int64)
            sptr[1:] = np.cumsum([len(x) for x in dof_subs])
            sidx = np.concatenate([np.asarray(x, dtype=np.int32) for x in dof_subs])
        sidx = np.asarray(sidx, dtype=np.int32)
        n = len(row_ptr) - 1
        prob = AlgebraicProblem(n, arr(row_ptr, np.int64), arr(col, np.int32), arr(val, np.float64),
                                arr(rhs, np.float64) if rhs is not None else None, arr(field, np.int32),
                                arr(null, np.float64) if null is not None else None,
                                int(sidx.max()) + 1 if sidx.size else 0, arr(sptr, np.int64), arr(sidx, np.int32))
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        solve = LOCAL_SOLVES[local_solve] if isinstance(local_solve, str) else int(local_solve)
        self.dec = Decomposition(1, overlap, 2, 1, prec, tile, 1, 0, budget, solve, int(max_rhs), 0)
        if host_only:
            st = _lib.gdsw_setup_algebraic_host(C.byref(prob), C.byref(self.dec), C.byref(self._ctx))
        else:
            st = _lib.gdsw_setup_algebraic(C.byref(prob), C.byref(self.dec), _stream(stream), C.byref(self._ctx))
        _check(st)
        self.host_only = host_only
        sz = self.sizes()
        self.n_free = sz.n_free
        self.n_coarse = sz.n_coarse
        return self

    # -- queries -----------------------------------------------------------
    def sizes(self) -> Sizes:
        s = Sizes()
        _check(_lib.gdsw_get_sizes(self._ctx, C.byref(s)), self._ctx)
        return s

    def setup_times(self):
        """(symbolic, numeric) setup wall time in seconds."""
        a, b = C.c_double(), C.c_double()
        _check(_lib.gdsw_setup_times(self._ctx, C.byref(a), C.byref(b)), self._ctx)
        return a.value, b.value

    def learned_save(self, path, stream=None):
        _check(_lib.gdsw_learned_save(self._ctx, os.fsencode(path), _stream(stream)), self._ctx)

    def learned_load(self, path, stream=None):
        _check(_lib.gdsw_learned_load(self._ctx, os.fsencode(path), _stream(stream)), self._ctx)

    def train_local_net(self, out_weights=None, steps=600, seed=0, stream=None):
        path = os.fsencode(out_weights) if out_weights is not None else None
        _check(_lib.gdsw_train_local_net(self._ctx, path, int(steps), int(seed), _stream(stream)), self._ctx)

    def dof_map(self):
        field = np.zeros(self.n_free, dtype=np.int32)
        abc = np.zeros((self.n_free, 3), dtype=np.int32)
        _check(_lib.gdsw_dof_map(self._ctx, _ptr(field), _ptr(abc)), self._ctx)
        return field, abc

    def host_matrix(self):
        s = self.sizes()
        rp = np.zeros(s.n_free + 1, dtype=np.int64)
        col = np.zeros(s.nnz, dtype=np.int32)
        val = np.zeros(s.nnz, dtype=np.float64)
        _check(_lib.gdsw_host_matrix(self._ctx, _ptr(rp), _ptr(col), _ptr(val)), self._ctx)
        return rp, col, val

    def host_rhs(self):
        b = np.zeros(self.n_free)
        _check(_lib.gdsw_host_rhs(self._ctx, _ptr(b)), self._ctx)
        return b

    def local_indices(self, i):
        sz = C.c_int32()
        _check(_lib.gdsw_local_indices(self._ctx, i, None, C.byref(sz)), self._ctx)
        out = np.zeros(sz.value, dtype=np.int32)
        _check(_lib.gdsw_local_indices(self._ctx, i, _ptr(out), C.byref(sz)), self._ctx)
        return out

    def coarse_matrix(self):
        a = np.zeros((self.n_coarse, self.n_coarse))
        _check(_lib.gdsw_copy_coarse_matrix(self._ctx, _ptr(a)), self._ctx)
        return a

    def coarse_basis(self):
        phi = np.zeros((self.n_coarse, self.n_free))  # column-major n x Nc == row-major Nc x n
        _check(_lib.gdsw_copy_coarse_basis(self._ctx, _ptr(phi)), self._ctx)
        return phi.T

    # -- device operations (torch tensors, float64, on the GPU) --------------
    def rhs(self, b, stream=None):
        _check(_lib.gdsw_rhs(self._ctx, _ptr(b), _stream(stream)), self._ctx)
        return b

    def spmv(self, x, y, stream=None):
        _check(_lib.gdsw_spmv(self._ctx, _ptr(x), _ptr(y), _stream(stream)), self._ctx)
        return y

    def apply(self, r, z, nrhs=1, ld=None, stream=None):
        ld = self.n_free if ld is None else ld
        _check(_lib.gdsw_apply_precond(self._ctx, _ptr(r), _ptr(z), nrhs, ld, _stream(stream)), self._ctx)
        return z

    def apply_noalloc(self, r, z, nrhs=1, ld=None, stream=None):
        """gdsw_apply_precond_noalloc: the same result without any allocation."""
        ld = self.n_free if ld is None else ld
        _check(_lib.gdsw_apply_precond_noalloc(self._ctx, _ptr(r), _ptr(z), nrhs, ld, _stream(stream)), self._ctx)
        return z

    def autotune(self, stream=None):
        """Picks the launch shape of the level-1 product.  Inverse mode:
        (chunk, [ms for 512, 1024, 2048]); symmetric and block modes:
        (10 * run + xcd, [ms for (2, 0), (2, 1), (1, 0), (1, 1)])."""
        ch = C.c_int32()
        ms = (C.c_double * 4)()
        _check(_lib.gdsw_autotune(self._ctx, _stream(stream), C.byref(ch), ms), self._ctx)
        return ch.value, list(ms)[:3 if self.dec.local_solve == LOCAL_SOLVES["inverse"] else 4]

    def autotune_mfma(self, stream=None):
        """Picks the several-column MFMA product's kernel and chunk; returns
        (index of the fastest candidate, [ms per candidate])."""
        ch = C.c_int32()
        ms = (C.c_double * 6)()
        _check(_lib.gdsw_autotune_mfma(self._ctx, _stream(stream), C.byref(ch), ms), self._ctx)
        return ch.value, list(ms)

    def kernel_timer(self, enable):
        _check(_lib.gdsw_kernel_timer(self._ctx, int(bool(enable))), self._ctx)

    def kernel_timer_read(self):
        """(total ms, launches, algorithmic bytes per launch) of the timed level-1 solve kernel."""
        ms, n, b = C.c_double(), C.c_int64(), C.c_uint64()
        _check(_lib.gdsw_kernel_timer_read(self._ctx, C.byref(ms), C.byref(n), C.byref(b)), self._ctx)
        return ms.value, n.value, b.value

    def set_schedule(self, phases, waves=4, stream=None):
        _check(_lib.gdsw_set_schedule(self._ctx, phases, waves, _stream(stream)), self._ctx)

    def profile_apply(self, r, z, stream=None):
        ms = np.zeros(4)
        _check(_lib.gdsw_profile_apply(self._ctx, _ptr(r), _ptr(z), _stream(stream), _ptr(ms)), self._ctx)
        return ms

    def fgmres(self, b, x, rtol=1e-8, restart=100, max_it=1000, use_graph=False, nrhs=1, ld=None, stream=None,
               raise_on_noconv=True, history=False):
        ld = self.n_free if ld is None else ld
        hist = np.zeros(max_it) if history else None
        hp = hist.ctypes.data_as(C.POINTER(C.c_double)) if history else None
        opts = FgmresOpts(rtol, restart, max_it, int(use_graph), max_it if history else 0, hp)
        infos = (FgmresInfo * nrhs)()
        st = _lib.gdsw_fgmres_solve(self._ctx, _ptr(b), _ptr(x), nrhs, ld, C.byref(opts), infos, _stream(stream))
        if st != 4 or raise_on_noconv:
            _check(st, self._ctx)
        out = [infos[k] for k in range(nrhs)]
        if history:
            return out, hist[:out[0].iterations].copy()
        return out

    def expand(self, x_free, x_full, stream=None):
        _check(_lib.gdsw_expand_solution(self._ctx, _ptr(x_free), _ptr(x_full), _stream(stream)), self._ctx)
        return x_full

    # -- learned local solve -------------------------------------------------------
    def learned_init(self, seed=0, stream=None):
        info = LearnedInfo()
        _check(_lib.gdsw_learned_init(self._ctx, seed, C.byref(info), _stream(stream)), self._ctx)
        self.learned = info
        return info

    def learned_train(self, solves=3, steps=500, batch=32, lr=1e-3, seed=0, stream=None):
        hist = np.zeros(max(steps, 1))
        _check(_lib.gdsw_learned_train(self._ctx, solves, steps, batch, lr, seed, _ptr(hist), _stream(stream)),
               self._ctx)
        return hist[:steps]

    def learned_weights(self, which=0, set_to=None, stream=None):
        n = self.learned.n_params
        out = np.zeros(n, dtype=np.float32)
        src = None if set_to is None else np.ascontiguousarray(set_to, dtype=np.float32)
        _check(_lib.gdsw_learned_weights(self._ctx, _ptr(src), _ptr(out), which, _stream(stream)), self._ctx)
        return out

    def learned_loss_grad(self, x, t, stream=None):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        g = np.zeros(self.learned.n_params, dtype=np.float32)
        loss = C.c_double()
        _check(_lib.gdsw_learned_loss_grad(self._ctx, _ptr(x), _ptr(t), x.shape[0], C.byref(loss), _ptr(g),
                                           _stream(stream)), self._ctx)
        return loss.value, g

    def set_local_solver(self, mode, tau=0.7):
        _check(_lib.gdsw_set_local_solver(self._ctx, {"lu": 0, "learned": 1, "none": 2}.get(mode, mode), tau),
               self._ctx)

    def learned_copy(self, src, stream=None):
        """Takes over src's trained network (src: another Solver or batch member)."""
        _check(_lib.gdsw_learned_copy(self._ctx, src._ctx, _stream(stream)), self._ctx)

    def learned_stats(self):
        a, b = C.c_int64(), C.c_int64()
        _check(_lib.gdsw_learned_stats(self._ctx, C.byref(a), C.byref(b)), self._ctx)
        return a.value, b.value

    @classmethod
    def _borrowed(cls, ctx):
        """A view of a context owned elsewhere (a batch member); close() leaves it alone."""
        self = cls.__new__(cls)
        self._ctx = ctx
        self._owned = False
        self.host_only = False
        s = self.sizes()
        self.n_free = s.n_free
        self.n_coarse = s.n_coarse
        return self

    def close(self):
        if self._ctx and getattr(self, "_owned", True):
            _lib.gdsw_destroy(self._ctx)
        self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _ptr_array(ts):
    arr = (_P * len(ts))()
    for k, t in enumerate(ts):
        arr[k] = _ptr(t).value
    return arr


class Batch:
    """Independent problems whose local and coarse inverse products share one
    launch pair per level (a gdsw_batch).  problems: dicts with keys n, m and
    optionally viscosity, inflow, manufactured, overlap."""

    def __init__(self, problems, precision="fp64", stream=None, budget=0, local_solve="inverse"):
        k = len(problems)
        meshes = (Mesh * k)()
        decs = (Decomposition * k)()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        solve = LOCAL_SOLVES[local_solve] if isinstance(local_solve, str) else int(local_solve)
        for i, p in enumerate(problems):
            meshes[i] = Mesh(int(p["n"]), int(p.get("manufactured", 0)), float(p.get("viscosity", 1.0)),
                             float(p.get("inflow", 16.0)))
            decs[i] = Decomposition(int(p["m"]), int(p.get("overlap", 1)), 2, 2, prec, 0, 0, 0, budget, solve, 1)
        self._b = C.c_void_p()
        _check(_lib.gdsw_setup_batch(meshes, decs, k, _stream(stream), C.byref(self._b)))
        self.members = []
        for i in range(k):
            c = C.c_void_p()
            _check(_lib.gdsw_batch_member(self._b, i, C.byref(c)))
            self.members.append(Solver._borrowed(c))

    def apply(self, rs, zs, stream=None):
        _check(_lib.gdsw_apply_precond_batch(self._b, _ptr_array(rs), _ptr_array(zs), _stream(stream)))
        return zs

    def fgmres(self, bs, xs, rtol=1e-8, restart=100, max_it=1000, stream=None, raise_on_noconv=True,
               use_graph=False):
        opts = FgmresOpts(rtol, restart, max_it, int(use_graph), 0, None)
        infos = (FgmresInfo * len(self.members))()
        st = _lib.gdsw_fgmres_solve_batch(self._b, _ptr_array(bs), _ptr_array(xs), C.byref(opts), infos,
                                          _stream(stream))
        if st != 4 or raise_on_noconv:
            _check(st)
        return [infos[k] for k in range(len(self.members))]

    def kernel_timer(self, enable):
        _check(_lib.gdsw_batch_kernel_timer(self._b, int(bool(enable))))

    def kernel_timer_read(self):
        ms, n, b = C.c_double(), C.c_int64(), C.c_uint64()
        _check(_lib.gdsw_batch_kernel_timer_read(self._b, C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value

    def close(self):
        for m in self.members:
            m._ctx = C.c_void_p()
        if self._b:
            _lib.gdsw_destroy_batch(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
