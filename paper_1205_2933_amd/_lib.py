"""ctypes binding of the C ABI in include/mgdwf.h.

Argument marshalling only: every function here checks tensor placement,
dtype, contiguity and size, then calls the C entry point of the same name.
All computation happens in the HIP library.  PyTorch provides device memory
and the stream.  The library must be built (``paper_1205_2933_amd.build``);
importing this module without it raises immediately -- there is no fallback.
"""

from __future__ import annotations

import ctypes
from pathlib import Path

import torch

_HERE = Path(__file__).resolve().parent
LIB_PATH = _HERE / "libmgdwf.so"

MGDWF_OK = 0
MGDWF_ERR_INVALID_ARG = 1
MGDWF_ERR_OOM = 2
MGDWF_ERR_HIP = 3
MGDWF_ERR_NOT_CONVERGED = 4
MGDWF_ERR_STATE = 5
MGDWF_ERR_NUMERIC = 6
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "HIP", 4: "NOT_CONVERGED", 5: "STATE", 6: "NUMERIC"}

MGDWF_F64, MGDWF_F32, MGDWF_F16, MGDWF_BF16 = 0, 1, 2, 3
PREC = {"f64": MGDWF_F64, "f32": MGDWF_F32, "f16": MGDWF_F16, "bf16": MGDWF_BF16}

MGDWF_K_DSLASH, MGDWF_K_RESTRICT, MGDWF_K_PROLONG, MGDWF_K_COARSE = 0, 1, 2, 3


class mgdwf_action(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("Ls", ctypes.c_int32), ("M5", ctypes.c_double),
                ("mf", ctypes.c_double), ("bc", ctypes.c_int32 * 4)]


class mgdwf_action2d(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 2), ("Ls", ctypes.c_int32), ("M5", ctypes.c_double),
                ("mf", ctypes.c_double), ("bc", ctypes.c_int32 * 2)]


class mgdwf_mg_params(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32 * 4), ("nvec", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("sweep0_iters", ctypes.c_int32), ("sweep_iters", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("coarse_tol", ctypes.c_double), ("coarse_maxiter", ctypes.c_int32),
                ("fine_prec", ctypes.c_int), ("coarse_prec", ctypes.c_int), ("coarse_graph", ctypes.c_int32),
                ("squared", ctypes.c_int32), ("sweep0_check", ctypes.c_int32), ("smoother_dirs", ctypes.c_int32)]


class mgdwf_level2_params(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32 * 4), ("nvec", ctypes.c_int32), ("null_iters", ctypes.c_int32),
                ("nu", ctypes.c_int32), ("coarse_tol", ctypes.c_double), ("coarse_maxiter", ctypes.c_int32),
                ("gamma", ctypes.c_int32)]


class mgdwf_solve_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("restart", ctypes.c_int32)]


class mgdwf_solve_report(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("fine_applies", ctypes.c_int64), ("coarse_applies", ctypes.c_int64),
                ("true_relres", ctypes.c_double), ("seconds", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("phase_seconds", ctypes.c_double * 3)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["phase_seconds"] = list(self.phase_seconds)
        return d


class mgdwf_setup_report(ctypes.Structure):
    _fields_ = [("sweeps_done", ctypes.c_int32), ("null_residual", ctypes.c_double * 8),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {"sweeps_done": self.sweeps_done,
                "null_residual": [self.null_residual[i] for i in range(self.sweeps_done)],
                "seconds": self.seconds}


MGDWF_MAX_TILINGS = 32


class mgdwf_tune_report(ctypes.Structure):
    _fields_ = [("ntilings", ctypes.c_int32), ("chosen", ctypes.c_int32), ("id", ctypes.c_int32 * MGDWF_MAX_TILINGS),
                ("tile", (ctypes.c_int32 * 4) * MGDWF_MAX_TILINGS), ("flags", ctypes.c_int32 * MGDWF_MAX_TILINGS),
                ("us", ctypes.c_double * MGDWF_MAX_TILINGS), ("coarse_chosen", ctypes.c_int32),
                ("coarse_us", ctypes.c_double * 2)]

    def as_dict(self):
        n = self.ntilings
        return {"chosen": self.chosen, "id": [self.id[i] for i in range(n)],
                "tile": [list(self.tile[i]) for i in range(n)], "flags": [self.flags[i] for i in range(n)],
                "us": [self.us[i] for i in range(n)], "coarse_chosen": self.coarse_chosen,
                "coarse_us": [self.coarse_us[0], self.coarse_us[1]] if self.coarse_chosen >= 0 else []}


class mgdwf_net_config(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32 * 5), ("lam", ctypes.c_double), ("seed", ctypes.c_uint64)]


class MgdwfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load() -> ctypes.CDLL:
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is not built; run paper_1205_2933_amd.build.build() first")
    lib = ctypes.CDLL(str(LIB_PATH))
    H = ctypes.c_void_p
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    sig = {
        "mgdwf_create": ([ctypes.POINTER(mgdwf_action), P, ctypes.POINTER(H)], ctypes.c_int),
        "mgdwf_create_2d": ([ctypes.POINTER(mgdwf_action2d), P, ctypes.POINTER(H)], ctypes.c_int),
        "mgdwf_destroy": ([H], ctypes.c_int),
        "mgdwf_last_error": ([H], ctypes.c_char_p),
        "mgdwf_set_gauge": ([H, P], ctypes.c_int),
        "mgdwf_apply_dwf": ([H, P, P, i32, ctypes.c_int, i32], ctypes.c_int),
        "mgdwf_set_nullvecs": ([H, ctypes.POINTER(i32), P, i32], ctypes.c_int),
        "mgdwf_get_basis": ([H, P], ctypes.c_int),
        "mgdwf_get_nullvecs": ([H, P, ctypes.POINTER(i32)], ctypes.c_int),
        "mgdwf_restrict": ([H, P, P, i32, ctypes.c_int], ctypes.c_int),
        "mgdwf_prolong": ([H, P, P, i32, ctypes.c_int], ctypes.c_int),
        "mgdwf_build_coarse": ([H], ctypes.c_int),
        "mgdwf_get_coarse_op": ([H, P], ctypes.c_int),
        "mgdwf_build_coarse_squared": ([H], ctypes.c_int),
        "mgdwf_coarse_stencil_size": ([H], ctypes.c_int32),
        "mgdwf_apply_coarse": ([H, P, P, i32, ctypes.c_int, i32], ctypes.c_int),
        "mgdwf_apply_coarse_noalloc": ([H, P, P, i32, ctypes.c_int, i32], ctypes.c_int),
        "mgdwf_setup": ([H, ctypes.POINTER(mgdwf_mg_params), P, ctypes.POINTER(mgdwf_setup_report)], ctypes.c_int),
        "mgdwf_set_mg_params": ([H, ctypes.POINTER(mgdwf_mg_params)], ctypes.c_int),
        "mgdwf_solve": ([H, P, P, i32, ctypes.POINTER(mgdwf_solve_params), ctypes.POINTER(mgdwf_solve_report)],
                        ctypes.c_int),
        "mgdwf_apply_vcycle": ([H, P, P, i32], ctypes.c_int),
        "mgdwf_low_modes": ([H, P, i32, i32, ctypes.c_double, P, P, P], ctypes.c_int),
        "mgdwf_coarse_coverage": ([H, P, i32, P], ctypes.c_int),
        "mgdwf_setup_level2": ([H, ctypes.POINTER(mgdwf_level2_params), P, ctypes.POINTER(ctypes.c_double)],
                               ctypes.c_int),
        "mgdwf_set_level2_params": ([H, ctypes.POINTER(mgdwf_level2_params)], ctypes.c_int),
        "mgdwf_get_level2": ([H, P, P, P], ctypes.c_int),
        "mgdwf_save_setup": ([H, ctypes.c_char_p], ctypes.c_int),
        "mgdwf_load_setup": ([H, ctypes.c_char_p], ctypes.c_int),
        "mgdwf_trim": ([H], ctypes.c_int),
        "mgdwf_memory_bytes": ([H], ctypes.c_int64),
        "mgdwf_solve_batch": ([ctypes.POINTER(H), i32, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(i32),
                               ctypes.POINTER(mgdwf_solve_params), ctypes.POINTER(mgdwf_solve_report)], ctypes.c_int),
        "mgdwf_cgne": ([H, P, P, ctypes.POINTER(mgdwf_solve_params), ctypes.POINTER(mgdwf_solve_report)],
                       ctypes.c_int),
        "mgdwf_time_kernel": ([H, ctypes.c_int, ctypes.c_int, i32, i32, ctypes.POINTER(ctypes.c_double)],
                              ctypes.c_int),
        "mgdwf_tune": ([H, i32, i32, ctypes.POINTER(mgdwf_tune_report)], ctypes.c_int),
        "mgdwf_set_tiling": ([H, i32], ctypes.c_int),
        "mgdwf_set_coarse_tiling": ([H, i32], ctypes.c_int),
        "mgdwf_set_barrier_timeout": ([H, ctypes.c_double], ctypes.c_int),
        "mgdwf_net_create": ([ctypes.POINTER(mgdwf_net_config), ctypes.POINTER(H)], ctypes.c_int),
        "mgdwf_net_destroy": ([H], ctypes.c_int),
        "mgdwf_net_last_error": ([H], ctypes.c_char_p),
        "mgdwf_net_num_weights": ([H], ctypes.c_int64),
        "mgdwf_net_set_weights": ([H, P], ctypes.c_int),
        "mgdwf_net_get_weights": ([H, P], ctypes.c_int),
        "mgdwf_net_propose": ([H, H, P, P], ctypes.c_int),
        "mgdwf_net_grad": ([H, H, P, ctypes.POINTER(ctypes.c_double), P], ctypes.c_int),
        "mgdwf_net_train_step": ([H, H, P, ctypes.c_double, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "mgdwf_net_train": ([H, ctypes.POINTER(H), i32, ctypes.POINTER(P), i32, ctypes.c_double, ctypes.c_double, P],
                            ctypes.c_int),
        "mgdwf_net_save": ([H, ctypes.c_char_p], ctypes.c_int),
        "mgdwf_net_load": ([H, ctypes.c_char_p], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def exported_symbols():
    """Names of the C entry points this binding declares."""
    return [n for n in dir(_lib) if n.startswith("mgdwf_")]


def _check(h, status: int, allow=()):
    if status != MGDWF_OK and status not in allow:
        msg = _lib.mgdwf_last_error(h)
        raise MgdwfError(status, msg.decode() if msg else "")
    return status


def _dev(t: torch.Tensor, numel: int, name: str, dtype=torch.complex128):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """Owner of one mgdwf_handle plus the sizes needed for argument checks."""

    def __init__(self, L, Ls, M5, mf, bc=(1, 1, 1, 1), stream=None):
        a = mgdwf_action()
        a.L[:] = list(L)
        a.Ls, a.M5, a.mf = Ls, M5, mf
        a.bc[:] = list(bc)
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(None, _lib.mgdwf_create(ctypes.byref(a), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.L, self.Ls, self.M5, self.mf, self.bc = tuple(L), Ls, M5, mf, tuple(bc)
        self.V4 = int(L[0] * L[1] * L[2] * L[3])
        self.nfine = 12 * self.V4 * Ls
        self.ngauge = 36 * self.V4
        self.site_shape = (Ls, 4, 3)  # per-site axes of a canonical fermion field
        self.block = None
        self.nvec = None

    def close(self):
        if self.h:
            _lib.mgdwf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def fermion_shape(self):
        return tuple(self.L[::-1]) + self.site_shape

    @property
    def ncoarse(self):
        Vc = 1
        for m in range(4):
            Vc *= self.L[m] // self.block[m]
        return Vc * 2 * self.nvec


class Handle2D(Handle):
    """A handle of the 2D U(1) problem: L = (Lx, Ly); internally the extents
    are (Lx, Ly, 1, 1), so blocks are given as (bx, by, 1, 1)."""

    def __init__(self, L, Ls, M5, mf, bc=(1, 1), stream=None):
        a = mgdwf_action2d()
        a.L[:] = list(L)
        a.Ls, a.M5, a.mf = Ls, M5, mf
        a.bc[:] = list(bc)
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(None, _lib.mgdwf_create_2d(ctypes.byref(a), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.L, self.Ls, self.M5, self.mf = (L[0], L[1], 1, 1), Ls, M5, mf
        self.bc = (bc[0], bc[1], 1, 1)
        self.V4 = int(L[0] * L[1])
        self.nfine = 2 * self.V4 * Ls
        self.ngauge = 2 * self.V4
        self.site_shape = (Ls, 2)
        self.block = None
        self.nvec = None

    @property
    def fermion_shape(self):
        return (self.L[1], self.L[0]) + self.site_shape


# ---- thin wrappers, one per C entry point ---------------------------------

def mgdwf_create(L, Ls, M5, mf, bc=(1, 1, 1, 1), stream=None) -> Handle:
    return Handle(L, Ls, M5, mf, bc, stream)


def mgdwf_create_2d(L, Ls, M5, mf, bc=(1, 1), stream=None) -> Handle2D:
    return Handle2D(L, Ls, M5, mf, bc, stream)


def mgdwf_destroy(h: Handle):
    h.close()


def mgdwf_last_error(h: Handle | None) -> str:
    m = _lib.mgdwf_last_error(h.h if h else None)
    return m.decode() if m else ""


def mgdwf_set_gauge(h: Handle, U: torch.Tensor):
    _check(h.h, _lib.mgdwf_set_gauge(h.h, _dev(U, h.ngauge, "U")))


def mgdwf_apply_dwf(h: Handle, inp: torch.Tensor, out: torch.Tensor, dagger=False, prec="f64", nrhs=1):
    n = h.nfine * nrhs
    _check(h.h, _lib.mgdwf_apply_dwf(h.h, _dev(inp, n, "in"), _dev(out, n, "out"), int(dagger), PREC[prec], nrhs))


def mgdwf_set_nullvecs(h: Handle, block, V: torch.Tensor, nvec: int):
    blk = (ctypes.c_int32 * 4)(*block)
    _check(h.h, _lib.mgdwf_set_nullvecs(h.h, blk, _dev(V, h.nfine * nvec, "V"), nvec))
    h.block, h.nvec = tuple(block), nvec


def mgdwf_get_nullvecs(h: Handle) -> torch.Tensor:
    """The near-null vectors behind the installed basis, as a new device tensor."""
    n = ctypes.c_int32()
    _check(h.h, _lib.mgdwf_get_nullvecs(h.h, None, ctypes.byref(n)))
    shape = (n.value,) + h.fermion_shape
    V = torch.empty(shape, dtype=torch.complex128, device="cuda")
    _check(h.h, _lib.mgdwf_get_nullvecs(h.h, _dev(V, h.nfine * n.value, "V"), ctypes.byref(n)))
    return V


def mgdwf_get_basis(h: Handle, Vhat: torch.Tensor):
    _check(h.h, _lib.mgdwf_get_basis(h.h, _dev(Vhat, h.nfine * h.nvec, "Vhat")))


def mgdwf_restrict(h: Handle, fine: torch.Tensor, coarse: torch.Tensor, nrhs=1, prec="f64"):
    _check(h.h, _lib.mgdwf_restrict(h.h, _dev(fine, h.nfine * nrhs, "fine"), _dev(coarse, h.ncoarse * nrhs, "coarse"),
                                    nrhs, PREC[prec]))


def mgdwf_prolong(h: Handle, coarse: torch.Tensor, fine: torch.Tensor, nrhs=1, prec="f64"):
    _check(h.h, _lib.mgdwf_prolong(h.h, _dev(coarse, h.ncoarse * nrhs, "coarse"), _dev(fine, h.nfine * nrhs, "fine"),
                                   nrhs, PREC[prec]))


def mgdwf_build_coarse(h: Handle):
    _check(h.h, _lib.mgdwf_build_coarse(h.h))


def mgdwf_build_coarse_squared(h: Handle):
    _check(h.h, _lib.mgdwf_build_coarse_squared(h.h))


def mgdwf_coarse_stencil_size(h: Handle) -> int:
    return int(_lib.mgdwf_coarse_stencil_size(h.h))


def mgdwf_get_coarse_op(h: Handle, Dc: torch.Tensor):
    n = h.ncoarse // (2 * h.nvec) * mgdwf_coarse_stencil_size(h) * (2 * h.nvec) ** 2
    _check(h.h, _lib.mgdwf_get_coarse_op(h.h, _dev(Dc, n, "Dc")))


def mgdwf_apply_coarse(h: Handle, inp: torch.Tensor, out: torch.Tensor, dagger=False, prec="f64", nrhs=1):
    n = h.ncoarse * nrhs
    _check(h.h, _lib.mgdwf_apply_coarse(h.h, _dev(inp, n, "in"), _dev(out, n, "out"), int(dagger), PREC[prec], nrhs))


def mgdwf_apply_coarse_noalloc(h: Handle, inp: torch.Tensor, out: torch.Tensor, dagger=False, prec="f64", nrhs=1):
    n = h.ncoarse * nrhs
    _check(h.h, _lib.mgdwf_apply_coarse_noalloc(h.h, _dev(inp, n, "in"), _dev(out, n, "out"), int(dagger), PREC[prec],
                                                nrhs))


def make_mg_params(block, nvec, sweeps=1, sweep0_iters=100, sweep_iters=4, nu_pre=4, nu_post=4,
                   coarse_tol=0.1, coarse_maxiter=100, fine_prec="f64", coarse_prec="f64",
                   coarse_graph=True, squared=False, sweep0_check=0, smoother_dirs=0) -> mgdwf_mg_params:
    p = mgdwf_mg_params()
    p.block[:] = list(block)
    p.nvec, p.sweeps, p.sweep0_iters, p.sweep_iters = nvec, sweeps, sweep0_iters, sweep_iters
    p.nu_pre, p.nu_post, p.coarse_tol, p.coarse_maxiter = nu_pre, nu_post, coarse_tol, coarse_maxiter
    p.fine_prec, p.coarse_prec = PREC[fine_prec], PREC[coarse_prec]
    # True / 1: graph replays; "persistent" / 2: one persistent coarse kernel; False / 0: plain launches
    p.coarse_graph = 2 if coarse_graph in ("persistent", 2) else (1 if coarse_graph else 0)
    p.squared = 1 if squared else 0
    p.sweep0_check = sweep0_check
    p.smoother_dirs = smoother_dirs
    return p


def mgdwf_setup(h: Handle, params: mgdwf_mg_params, V0: torch.Tensor) -> dict:
    rep = mgdwf_setup_report()
    nstart = params.nvec if params.squared else params.nvec // 2
    _check(h.h, _lib.mgdwf_setup(h.h, ctypes.byref(params), _dev(V0, h.nfine * nstart, "V0"),
                                 ctypes.byref(rep)))
    h.block, h.nvec = tuple(params.block), params.nvec
    return rep.as_dict()


def mgdwf_set_mg_params(h: Handle, params: mgdwf_mg_params):
    _check(h.h, _lib.mgdwf_set_mg_params(h.h, ctypes.byref(params)))


def mgdwf_solve(h: Handle, b: torch.Tensor, x: torch.Tensor, nrhs=1, tol=1e-10, max_outer=500, restart=8,
                allow_not_converged=False):
    sp = mgdwf_solve_params(tol, max_outer, restart)
    reps = (mgdwf_solve_report * nrhs)()
    st = _lib.mgdwf_solve(h.h, _dev(b, h.nfine * nrhs, "b"), _dev(x, h.nfine * nrhs, "x"), nrhs, ctypes.byref(sp),
                          reps)
    _check(h.h, st, allow=(MGDWF_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    return [r.as_dict() for r in reps]


def mgdwf_apply_vcycle(h: Handle, inp: torch.Tensor, out: torch.Tensor, nrhs=1):
    n = h.nfine * nrhs
    _check(h.h, _lib.mgdwf_apply_vcycle(h.h, _dev(inp, n, "in"), _dev(out, n, "out"), nrhs))


def mgdwf_low_modes(h: Handle, v0: torch.Tensor, nev: int, m: int, solve_tol=1e-12, want_vectors=True):
    """(eigenvalues ascending, eigenvectors [nev] device tensor or None, relative residuals)."""
    ev = (ctypes.c_double * nev)()
    rs = (ctypes.c_double * nev)()
    vecs = torch.empty((nev,) + h.fermion_shape, dtype=torch.complex128, device="cuda") \
        if want_vectors else None
    _check(h.h, _lib.mgdwf_low_modes(h.h, _dev(v0, h.nfine, "v0"), nev, m, float(solve_tol), ev,
                                     _dev(vecs, h.nfine * nev, "evecs") if want_vectors else None, rs))
    return list(ev), vecs, list(rs)


def mgdwf_coarse_coverage(h: Handle, e: torch.Tensor, n: int) -> list:
    fr = (ctypes.c_double * n)()
    _check(h.h, _lib.mgdwf_coarse_coverage(h.h, _dev(e, h.nfine * n, "e"), n, fr))
    return list(fr)


def make_level2_params(block, nvec, null_iters=50, nu=2, coarse_tol=0.1, coarse_maxiter=200,
                       gamma=1) -> mgdwf_level2_params:
    p = mgdwf_level2_params()
    p.block[:] = list(block)
    p.nvec, p.null_iters, p.nu = nvec, null_iters, nu
    p.coarse_tol, p.coarse_maxiter, p.gamma = coarse_tol, coarse_maxiter, gamma
    return p


def mgdwf_setup_level2(h: Handle, p: mgdwf_level2_params, W0: torch.Tensor) -> float:
    """Third level under the squared coarse operator; returns the median |A_c w|."""
    nr = ctypes.c_double()
    _check(h.h, _lib.mgdwf_setup_level2(h.h, ctypes.byref(p), _dev(W0, h.ncoarse * p.nvec, "W0"), ctypes.byref(nr)))
    h.level2 = (tuple(p.block), p.nvec)
    return nr.value


def mgdwf_set_level2_params(h: Handle, p: mgdwf_level2_params):
    _check(h.h, _lib.mgdwf_set_level2_params(h.h, ctypes.byref(p)))


def mgdwf_get_level2(h: Handle):
    """(W, What, Acc) of the installed third level as new device tensors: W and What
    [nvec2][Tc][Zc][Yc][Xc][2][Nv]; Acc [Tcc][Zcc][Ycc][Xcc][33][2Nv2][2Nv2]."""
    blk, nv2 = h.level2
    Lc = tuple(h.L[m] // h.block[m] for m in range(4))
    Lcc = tuple(Lc[m] // blk[m] for m in range(4))
    shp = (nv2,) + Lc[::-1] + (2, h.nvec)
    W = torch.empty(shp, dtype=torch.complex128, device="cuda")
    Wh = torch.empty_like(W)
    A = torch.empty(Lcc[::-1] + (33, 2 * nv2, 2 * nv2), dtype=torch.complex128, device="cuda")
    _check(h.h, _lib.mgdwf_get_level2(h.h, _dev(W, W.numel(), "W"), _dev(Wh, Wh.numel(), "What"),
                                      _dev(A, A.numel(), "Acc")))
    return W, Wh, A


def mgdwf_save_setup(h: Handle, path):
    _check(h.h, _lib.mgdwf_save_setup(h.h, str(path).encode()))


def mgdwf_load_setup(h: Handle, path):
    """Install a saved setup; the binding's block and nvec follow the file's
    header (magic, then int32 L[4], Ls, bc[4], block[4], nvec)."""
    _check(h.h, _lib.mgdwf_load_setup(h.h, str(path).encode()))
    import struct
    with open(path, "rb") as f:
        head = f.read(8 + 4 * 14)
    ints = struct.unpack("<14i", head[8:])
    h.block, h.nvec = tuple(ints[9:13]), ints[13]


def mgdwf_trim(h: Handle):
    _check(h.h, _lib.mgdwf_trim(h.h))


def mgdwf_memory_bytes(h: Handle) -> int:
    return int(_lib.mgdwf_memory_bytes(h.h))


def mgdwf_solve_batch(hs, bs, xs, nrhs, tol=1e-10, max_outer=500, restart=8, allow_not_converged=False):
    """Ragged batch: handle hs[i] solves nrhs[i] right-hand sides bs[i] -> xs[i]."""
    n = len(hs)
    if not (len(bs) == len(xs) == len(nrhs) == n):
        raise ValueError("hs, bs, xs and nrhs must have the same length")
    H = (ctypes.c_void_p * n)(*[h.h for h in hs])
    B = (ctypes.c_void_p * n)(*[_dev(b, h.nfine * k, "b") for h, b, k in zip(hs, bs, nrhs)])
    X = (ctypes.c_void_p * n)(*[_dev(x, h.nfine * k, "x") for h, x, k in zip(hs, xs, nrhs)])
    R = (ctypes.c_int32 * n)(*nrhs)
    sp = mgdwf_solve_params(tol, max_outer, restart)
    reps = (mgdwf_solve_report * sum(nrhs))()
    st = _lib.mgdwf_solve_batch(H, n, B, X, R, ctypes.byref(sp), reps)
    if st != MGDWF_OK and not (allow_not_converged and st == MGDWF_ERR_NOT_CONVERGED):
        msgs = [mgdwf_last_error(h) for h in hs]
        raise MgdwfError(st, "; ".join(m for m in msgs if m))
    out, k = [], 0
    for m in nrhs:
        out.append([reps[k + j].as_dict() for j in range(m)])
        k += m
    return out


def mgdwf_cgne(h: Handle, b: torch.Tensor, x: torch.Tensor, tol=1e-10, max_iter=100000):
    sp = mgdwf_solve_params(tol, max_iter, 1)
    rep = mgdwf_solve_report()
    _check(h.h, _lib.mgdwf_cgne(h.h, _dev(b, h.nfine, "b"), _dev(x, h.nfine, "x"), ctypes.byref(sp),
                                ctypes.byref(rep)))
    return rep.as_dict()


def mgdwf_time_kernel(h: Handle, kernel: int, prec="f64", nrhs=1, iters=20) -> float:
    ms = ctypes.c_double()
    _check(h.h, _lib.mgdwf_time_kernel(h.h, kernel, PREC[prec], nrhs, iters, ctypes.byref(ms)))
    return ms.value


def mgdwf_tune(h: Handle, nrhs=1, iters=10) -> dict:
    rep = mgdwf_tune_report()
    _check(h.h, _lib.mgdwf_tune(h.h, nrhs, iters, ctypes.byref(rep)))
    return rep.as_dict()


def mgdwf_set_tiling(h: Handle, tiling_id: int):
    _check(h.h, _lib.mgdwf_set_tiling(h.h, tiling_id))


def mgdwf_set_barrier_timeout(h: Handle, seconds: float):
    _check(h.h, _lib.mgdwf_set_barrier_timeout(h.h, float(seconds)))


def mgdwf_set_coarse_tiling(h: Handle, tiling_id: int):
    """MFMA shape of the 16-bit coarse apply: 0 = 16x16x16, 1 = 16x16x32, -1 = default."""
    _check(h.h, _lib.mgdwf_set_coarse_tiling(h.h, tiling_id))


# ---- learned near-null proposals --------------------------------------------

class Net:
    """Owner of one mgdwf_net."""

    def __init__(self, channels, lam=1.0, seed=0):
        cfg = mgdwf_net_config()
        cfg.channels[:] = list(channels)
        cfg.lam = lam
        cfg.seed = seed
        n = ctypes.c_void_p()
        st = _lib.mgdwf_net_create(ctypes.byref(cfg), ctypes.byref(n))
        if st != MGDWF_OK:
            msg = _lib.mgdwf_net_last_error(None)
            raise MgdwfError(st, msg.decode() if msg else "")
        self.n = n
        self.channels, self.lam = tuple(channels), lam
        self.nweights = int(_lib.mgdwf_net_num_weights(n))
        self.nh = channels[4] // 4

    def close(self):
        if self.n:
            _lib.mgdwf_net_destroy(self.n)
            self.n = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _net_check(net: Net, status: int):
    if status != MGDWF_OK:
        msg = _lib.mgdwf_net_last_error(net.n)
        raise MgdwfError(status, msg.decode() if msg else "")


def _host_f32(t: torch.Tensor, numel: int, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cpu" or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a host float32 tensor")
    if not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name} must be contiguous with {numel} elements")
    return ctypes.c_void_p(t.data_ptr())


def mgdwf_net_create(channels, lam=1.0, seed=0) -> Net:
    return Net(channels, lam, seed)


def mgdwf_net_destroy(net: Net):
    net.close()


def mgdwf_net_last_error(net: Net | None) -> str:
    m = _lib.mgdwf_net_last_error(net.n if net else None)
    return m.decode() if m else ""


def mgdwf_net_num_weights(net: Net) -> int:
    return int(_lib.mgdwf_net_num_weights(net.n))


def mgdwf_net_set_weights(net: Net, w: torch.Tensor):
    _net_check(net, _lib.mgdwf_net_set_weights(net.n, _host_f32(w, net.nweights, "w")))


def mgdwf_net_get_weights(net: Net) -> torch.Tensor:
    w = torch.empty(net.nweights, dtype=torch.float32)
    _net_check(net, _lib.mgdwf_net_get_weights(net.n, ctypes.c_void_p(w.data_ptr())))
    return w


def mgdwf_net_propose(net: Net, h: Handle, eta: torch.Tensor, V: torch.Tensor):
    _net_check(net, _lib.mgdwf_net_propose(net.n, h.h, _dev(eta, net.channels[0] * h.V4 * 3, "eta"),
                                           _dev(V, h.nfine * net.nh, "V")))


def mgdwf_net_grad(net: Net, h: Handle, eta: torch.Tensor, want_grad=True):
    loss = ctypes.c_double()
    g = torch.empty(net.nweights, dtype=torch.float32) if want_grad else None
    _net_check(net, _lib.mgdwf_net_grad(net.n, h.h, _dev(eta, net.channels[0] * h.V4 * 3, "eta"), ctypes.byref(loss),
                                        ctypes.c_void_p(g.data_ptr()) if g is not None else None))
    return loss.value, g


def mgdwf_net_train_step(net: Net, h: Handle, eta: torch.Tensor, lr: float) -> float:
    loss = ctypes.c_double()
    _net_check(net, _lib.mgdwf_net_train_step(net.n, h.h, _dev(eta, net.channels[0] * h.V4 * 3, "eta"), lr,
                                              ctypes.byref(loss)))
    return loss.value


def mgdwf_net_train(net: Net, handles, etas, lr: float, lr_final: float | None = None) -> list:
    """len(etas) Adam steps cycling over the handles; returns the losses."""
    n, steps = len(handles), len(etas)
    lr_final = lr if lr_final is None else lr_final
    H = (ctypes.c_void_p * n)(*[h.h for h in handles])
    E = (ctypes.c_void_p * steps)(*[_dev(e, net.channels[0] * handles[k % n].V4 * 3, "eta")
                                     for k, e in enumerate(etas)])
    losses = (ctypes.c_double * steps)()
    _net_check(net, _lib.mgdwf_net_train(net.n, H, n, E, steps, lr, lr_final, losses))
    return list(losses)


def mgdwf_net_save(net: Net, path):
    _net_check(net, _lib.mgdwf_net_save(net.n, str(path).encode()))


def mgdwf_net_load(net: Net, path):
    _net_check(net, _lib.mgdwf_net_load(net.n, str(path).encode()))
