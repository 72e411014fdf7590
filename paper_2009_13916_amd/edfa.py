"""Python binding of libedfa (ctypes).  Argument marshalling only: every step of the
assembly, setup and solve runs in the HIP library.  Torch supplies device memory and
the current stream.

The library must have been built (``python -m paper_2009_13916_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libedfa.so")

OK, NOT_CONVERGED = 0, 1

STATIC, DYNAMIC = 0, 1
FILT = {"none": 0, "pre": 1, "post_S": 2, "post_H": 3}
SCHUR = {"isai": 0, "exact": 1}

BLOCK = {"App": 0, "Apc": 1, "Acp": 2, "Acc": 3, "A": 4}
PRECOND_ART = {"G": 0, "FT": 1, "H_raw": 2, "H": 3, "S": 4, "GF": 5, "L": 6, "U": 7, "ML": 8, "MU": 9}


class EdfaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libedfa status {status}: {msg}")
        self.status = status


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("nodes", C.c_void_p), ("K", C.c_void_p), ("c", C.c_void_p),
                ("c_scalar", C.c_double), ("gamma", C.c_double), ("dt", C.c_double),
                ("bc_type", C.c_void_p), ("bc_value", C.c_void_p),
                ("p_prev", C.c_void_p), ("source", C.c_void_p)]


class _SystemInfo(C.Structure):
    _fields_ = [("n_grids", C.c_int32), ("n_cells", C.c_int32), ("n_faces", C.c_int32),
                ("n_face_unknowns", C.c_int32), ("n", C.c_int32), ("axis_structure", C.c_int32),
                ("nnz", C.c_int64), ("nnz_block", C.c_int64 * 4)]


class _Params(C.Structure):
    _fields_ = [("variant", C.c_int32), ("static_level", C.c_int32), ("n_add", C.c_int32),
                ("n_ent", C.c_int32), ("it_max", C.c_int32), ("tau_filt", C.c_double),
                ("filt_mode", C.c_int32), ("precision", C.c_int32),
                ("schur_solver", C.c_int32), ("isai_steps", C.c_int32),
                ("static_axis", C.c_int32), ("htilde_retry", C.c_int32)]


class _PrecondInfo(C.Structure):
    _fields_ = [("nnz_G", C.c_int64), ("nnz_F", C.c_int64), ("nnz_H", C.c_int64),
                ("nnz_S", C.c_int64), ("nnz_GF", C.c_int64), ("nnz_L", C.c_int64),
                ("nnz_U", C.c_int64), ("nnz_ML", C.c_int64), ("nnz_MU", C.c_int64),
                ("n_colors", C.c_int32), ("max_pattern", C.c_int32), ("mu", C.c_double),
                ("t_stage1_ms", C.c_double), ("t_stage2_ms", C.c_double),
                ("nnz_H_raw", C.c_int64), ("htilde_retry_rows", C.c_int32),
                ("color_rounds", C.c_int32), ("color_list_rounds", C.c_int32),
                ("cgs2_width", C.c_int32), ("chunks_ML", C.c_int32), ("chunks_MU", C.c_int32)]


NCAP = 7


class _SetupTune(C.Structure):
    _fields_ = [("buckets", C.c_int32), ("capacity", C.c_int32 * NCAP),
                ("cells", C.c_int32 * NCAP), ("chosen", C.c_int32 * NCAP),
                ("us", (C.c_float * NCAP) * NCAP)]


class _SolveParams(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iter", C.c_int32), ("flexible", C.c_int32),
                ("transpose", C.c_int32), ("use_graph", C.c_int32), ("profile", C.c_int32),
                ("rtol", C.c_double), ("method", C.c_int32)]

METHOD = {"gmres": 0, "bicgstab": 1}


class _TransientParams(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("t_end", C.c_double), ("dt0", C.c_double),
                ("dt_mult", C.c_double), ("dt_max", C.c_double), ("dp_target", C.c_double),
                ("porosity", C.c_double), ("stage1_every", C.c_int32), ("solve", _SolveParams)]


class _StepInfo(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("dp_max", C.c_double),
                ("chi_inf", C.c_double), ("iterations", C.c_int32), ("converged", C.c_int32),
                ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double)]


class _SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("cycles", C.c_int32),
                ("relres_est", C.c_double), ("relres_true", C.c_double),
                ("t_solve_ms", C.c_double), ("spmv_avg_ms", C.c_double),
                ("spmv_count", C.c_int32), ("apply_avg_ms", C.c_double),
                ("apply_count", C.c_int32), ("slot_ms", C.c_double * 16),
                ("slot_launches", C.c_int32 * 16)]


TUNE_SLOTS = ("A", "A^T", "G_F", "G_F^T", "L", "U", "M_L", "M_U", "L^T", "U^T", "M_L^T",
              "M_U^T", "A_ppi", "A_pip", "A_pip^T", "A_ppi^T")
# (lanes per row, entries in flight per lane); lanes 1 = the SELL kernel, -1 = the chunk
# kernel (long rows only), else CSR
TUNE_VARIANTS = ((1, 4), (1, 8), (2, 2), (2, 4), (4, 2), (4, 4), (8, 2), (8, 4), (16, 2),
                 (16, 4), (32, 2), (32, 4), (-1, 12), (-1, 8))


def variant_name(v):
    lanes, depth = TUNE_VARIANTS[v]
    if lanes == -1:
        return f"chunk/{depth}"
    return f"sell/{depth}" if lanes == 1 else f"csr{lanes}/{depth}"


class _TuneSlot(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("nnz", C.c_int64),
                ("variant", C.c_int32), ("value_bytes", C.c_int32),
                ("sell_sorted", C.c_int32), ("sell_padding", C.c_float),
                ("us", C.c_float * len(TUNE_VARIANTS))]


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "edfa_last_error": (C.c_char_p, []),
            "edfa_assemble": (C.c_int, [C.POINTER(_Problem), i32, vp, C.POINTER(vp)]),
            "edfa_system_destroy": (None, [vp]),
            "edfa_system_get_info": (C.c_int, [vp, C.POINTER(_SystemInfo)]),
            "edfa_update_dt": (C.c_int, [vp, d, vp, vp]),
            "edfa_export_block": (C.c_int, [vp, i32, vp, vp, vp, vp]),
            "edfa_export_rhs": (C.c_int, [vp, vp, vp, vp, vp]),
            "edfa_spmv": (C.c_int, [vp, i32, vp, vp, vp]),
            "edfa_setup": (C.c_int, [vp, C.POINTER(_Params), vp, C.POINTER(vp)]),
            "edfa_setup_stage2": (C.c_int, [vp, vp]),
            "edfa_resetup": (C.c_int, [vp, vp]),
            "edfa_precond_destroy": (None, [vp]),
            "edfa_precond_get_info": (C.c_int, [vp, C.POINTER(_PrecondInfo)]),
            "edfa_export_precond": (C.c_int, [vp, i32, vp, vp, vp, vp, C.POINTER(i64),
                                              C.POINTER(i32), vp]),
            "edfa_apply": (C.c_int, [vp, i32, vp, vp, vp]),
            "edfa_apply_noalloc": (C.c_int, [vp, i32, vp, vp, vp]),
            "edfa_solve": (C.c_int, [vp, vp, vp, vp, C.POINTER(_SolveParams), vp,
                                     C.POINTER(_SolveInfo)]),
            "edfa_grad_logk": (C.c_int, [vp, vp, vp, vp, vp]),
            "edfa_transient": (C.c_int, [vp, vp, C.POINTER(_TransientParams), vp, vp,
                                         C.POINTER(_StepInfo), C.POINTER(i32)]),
            "edfa_autotune": (C.c_int, [vp, vp, C.POINTER(i32), C.POINTER(_TuneSlot)]),
            "edfa_autotune_setup": (C.c_int, [vp, vp, C.POINTER(_SetupTune)]),
            "edfa_tune_params": (C.c_int, [vp, C.POINTER(_Params), i32, C.POINTER(_SolveParams),
                                           vp, C.POINTER(i32), C.POINTER(d), C.POINTER(i32),
                                           C.POINTER(i32)]),
            "edfa_set_variant": (C.c_int, [vp, i32, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names of the entry points the loaded library exports (for the ABI test)."""
    L = load()
    return [n for n in ("edfa_last_error", "edfa_assemble", "edfa_system_destroy",
                        "edfa_system_get_info", "edfa_update_dt", "edfa_export_block",
                        "edfa_export_rhs", "edfa_spmv", "edfa_setup", "edfa_setup_stage2", "edfa_resetup",
                        "edfa_precond_destroy", "edfa_precond_get_info", "edfa_export_precond",
                        "edfa_apply", "edfa_solve", "edfa_grad_logk", "edfa_autotune",
                        "edfa_set_variant", "edfa_transient", "edfa_apply_noalloc",
                        "edfa_tune_params", "edfa_autotune_setup")
            if hasattr(L, n)]


def _check(st):
    if st < 0:
        raise EdfaError(st, load().edfa_last_error().decode())
    return st


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


class System:
    """An assembled block system (one grid or a block-diagonal batch of grids)."""

    def __init__(self, problems):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        keep = []
        arr = (_Problem * len(problems))()
        for i, p in enumerate(problems):
            t = {k: _dev(getattr(p, k), torch.float64) for k in ("nodes", "K", "c", "bc_value", "p_prev", "source")}
            t["bc_type"] = _dev(p.bc_type, torch.int8)
            keep.append(t)
            arr[i] = _Problem(p.nx, p.ny, p.nz, t["nodes"].data_ptr(), t["K"].data_ptr(),
                              t["c"].data_ptr(), 0.0, float(p.gamma), float(p.dt),
                              t["bc_type"].data_ptr(), t["bc_value"].data_ptr(),
                              t["p_prev"].data_ptr(), t["source"].data_ptr())
        h = C.c_void_p()
        _check(load().edfa_assemble(arr, len(problems), _stream(), C.byref(h)))
        self._h = h
        self.info = self._info()

    def _info(self):
        inf = _SystemInfo()
        _check(load().edfa_system_get_info(self._h, C.byref(inf)))
        return {"n_grids": inf.n_grids, "ne": inf.n_cells, "nf": inf.n_faces,
                "nfu": inf.n_face_unknowns, "n": inf.n, "axis": inf.axis_structure,
                "nnz": inf.nnz, "nnz_block": list(inf.nnz_block)}

    @property
    def n(self):
        return self.info["n"]

    def export_block(self, name):
        b = BLOCK[name]
        nfu, ne, n = self.info["nfu"], self.info["ne"], self.info["n"]
        rows = {0: nfu, 1: nfu, 2: ne, 3: ne, 4: n}[b]
        nnz = self.info["nnz"] if b == 4 else self.info["nnz_block"][b]
        rp = torch.empty(rows + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device="cuda")
        _check(load().edfa_export_block(self._h, b, _ptr(rp), _ptr(col), _ptr(val), _stream()))
        return rp, col[:nnz], val[:nnz]

    def rhs(self):
        b = torch.empty(self.info["n"], dtype=torch.float64, device="cuda")
        _check(load().edfa_export_rhs(self._h, _ptr(b), None, None, _stream()))
        return b

    def element_data(self):
        ne = self.info["ne"]
        W = torch.empty(ne * 36, dtype=torch.float64, device="cuda")
        vol = torch.empty(ne, dtype=torch.float64, device="cuda")
        _check(load().edfa_export_rhs(self._h, None, _ptr(W), _ptr(vol), _stream()))
        return W.view(ne, 6, 6), vol

    def spmv(self, x, transpose=False):
        y = torch.empty_like(x)
        _check(load().edfa_spmv(self._h, int(transpose), _ptr(x), _ptr(y), _stream()))
        return y

    def update_dt(self, dt, p_prev=None):
        _check(load().edfa_update_dt(self._h, float(dt), _ptr(p_prev), _stream()))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.edfa_system_destroy(self._h)
            self._h = None


@dataclass
class Params:
    variant: str = "dynamic"
    static_level: int = 0
    n_add: int = 1
    n_ent: int = 4
    it_max: int = 0
    tau: float = 0.0
    filt: str = "none"
    precision: int = 0          # 0 FP64, 1 FP32 setup + application
    schur: str = "isai"
    isai_steps: int = 1
    static_axis: int = 0        # static level k: 0 all directions, 1/2/3 x/y/z, 4 flow axis
    htilde_retry: int = 0       # rows of H~ with a wider support of t take the second pass

    def c(self):
        return _Params(STATIC if self.variant == "static" else DYNAMIC, self.static_level,
                       self.n_add, self.n_ent, self.it_max, float(self.tau), FILT[self.filt],
                       self.precision, SCHUR[self.schur], self.isai_steps, self.static_axis,
                       self.htilde_retry)


class Precond:
    def __init__(self, system: System, params: Params):
        self.system = system
        self.params = params
        h = C.c_void_p()
        _check(load().edfa_setup(system._h, C.byref(params.c()), _stream(), C.byref(h)))
        self._h = h

    def stage2(self):
        _check(load().edfa_setup_stage2(self._h, _stream()))

    def resetup(self):
        """Stage 1 + stage 2 again on the same system, reusing device memory."""
        _check(load().edfa_resetup(self._h, _stream()))

    def info(self):
        inf = _PrecondInfo()
        _check(load().edfa_precond_get_info(self._h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _PrecondInfo._fields_}

    def export(self, what):
        w = PRECOND_ART[what]
        nnz, rows = C.c_int64(), C.c_int32()
        L = load()
        _check(L.edfa_export_precond(self._h, w, None, None, None, None, C.byref(nnz),
                                     C.byref(rows), _stream()))
        rp = torch.empty(rows.value + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(nnz.value, 1), dtype=torch.float64, device="cuda")
        perm = torch.empty(self.system.info["ne"], dtype=torch.int32, device="cuda") if w >= 6 else None
        _check(L.edfa_export_precond(self._h, w, _ptr(rp), _ptr(col), _ptr(val), _ptr(perm),
                                     C.byref(nnz), C.byref(rows), _stream()))
        return rp, col[:nnz.value], val[:nnz.value], perm

    def apply(self, r, transpose=False, z=None, noalloc=False):
        """z = P^-1 r (or P^-T r).  noalloc=True calls the allocation-free entry point (the
        library allocates nothing; z may be given to avoid torch's allocation too)."""
        if z is None:
            z = torch.empty_like(r)
        fn = load().edfa_apply_noalloc if noalloc else load().edfa_apply
        _check(fn(self._h, int(transpose), _ptr(r), _ptr(z), _stream()))
        return z

    def autotune(self, report=False):
        """Time the sparse-product kernel variants for every matrix of the solve and keep
        the fastest.  Returns the number of matrices timed, or with report=True a dict
        {slot name: {rows, cols, nnz, variant, value_bytes, sell_sorted, sell_padding,
        us: {variant name: microseconds}}} over the matrices that were timed (variant
        names: variant_name)."""
        n = C.c_int32(0)
        rec = (_TuneSlot * len(TUNE_SLOTS))()
        _check(load().edfa_autotune(self._h, _stream(), C.byref(n), rec))
        if not report:
            return n.value
        out = {}
        for name, r in zip(TUNE_SLOTS, rec):
            if r.rows > 0:
                out[name] = {"rows": r.rows, "cols": r.cols, "nnz": r.nnz,
                             "variant": variant_name(r.variant), "value_bytes": r.value_bytes,
                             "sell_sorted": bool(r.sell_sorted),
                             "sell_padding": float(r.sell_padding),
                             "us": {variant_name(v): float(t) for v, t in enumerate(r.us)}}
        return out

    def autotune_setup(self):
        """Time each pattern-capacity bucket of the last stage 1 with its own and the next two
        larger kernel capacities; keep the fastest.  Returns a list of {capacity, cells,
        chosen, us: {capacity: microseconds}} for the non-empty buckets."""
        rep = _SetupTune()
        _check(load().edfa_autotune_setup(self._h, _stream(), C.byref(rep)))
        caps = [rep.capacity[b] for b in range(NCAP)]
        return [{"capacity": caps[b], "cells": rep.cells[b], "chosen": rep.chosen[b],
                 "us": {caps[c]: float(rep.us[b][c]) for c in range(NCAP) if rep.us[b][c] > 0}}
                for b in range(NCAP) if rep.cells[b] > 0]

    def set_variant(self, variant, slot=None):
        """Pin the sparse-product kernel of one slot (a name of TUNE_SLOTS or an index;
        None = every slot) to a variant (a name from variant_name, an index, or None for
        the default choice)."""
        s = -1 if slot is None else (TUNE_SLOTS.index(slot) if isinstance(slot, str) else slot)
        if variant is None:
            v = -1
        elif isinstance(variant, str):
            v = [variant_name(i) for i in range(len(TUNE_VARIANTS))].index(variant)
        else:
            v = variant
        _check(load().edfa_set_variant(self._h, int(s), int(v)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.edfa_precond_destroy(self._h)
            self._h = None


def solve(system: System, pre: Precond, b, rtol=1e-8, restart=50, max_iter=5000, flexible=False,
          transpose=False, use_graph=False, profile=False, method="gmres"):
    """Right-preconditioned (F)GMRES(restart) or Bi-CGStab (method="bicgstab"), x0 = 0.
    profile: 0/False none, 1/True the system products and the applications, 2 also every
    product inside the applications.  Returns (x, info dict, status)."""
    x = torch.zeros_like(b)
    prm = _SolveParams(restart, max_iter, int(flexible), int(transpose), int(use_graph),
                       int(profile), float(rtol), METHOD[method])
    inf = _SolveInfo()
    st = _check(load().edfa_solve(system._h, pre._h, _ptr(b), _ptr(x), C.byref(prm), _stream(),
                                  C.byref(inf)))
    out = {f: getattr(inf, f) for f, _ in _SolveInfo._fields_}
    # per-matrix product timings of a profiled solve, by tuner slot name
    out["slot_ms"] = {TUNE_SLOTS[q]: inf.slot_ms[q] for q in range(16) if inf.slot_launches[q]}
    out["slot_launches"] = {TUNE_SLOTS[q]: inf.slot_launches[q] for q in range(16)
                            if inf.slot_launches[q]}
    return x, out, st


def transient(system: System, pre: Precond, n_steps, dt0, dt_mult=2.0, dt_max=float("inf"),
              dp_target=float("inf"), porosity=0.2, t_end=0.0, stage1_every=0, rtol=1e-8,
              restart=50, max_iter=5000, flexible=False, method="gmres"):
    """Adaptive transient sequence (eq. delta_t_dyn, eq. CFL_number) from the system's p_prev.
    Returns (u of the last step, list of per-step dicts, status)."""
    u = torch.zeros(system.info["n"], dtype=torch.float64, device="cuda")
    sp = _SolveParams(restart, max_iter, int(flexible), 0, 0, 0, float(rtol), METHOD[method])
    prm = _TransientParams(int(n_steps), float(t_end), float(dt0), float(dt_mult), float(dt_max),
                           float(dp_target), float(porosity), int(stage1_every), sp)
    recs = (_StepInfo * int(n_steps))()
    taken = C.c_int32(0)
    st = _check(load().edfa_transient(system._h, pre._h, C.byref(prm), _ptr(u), _stream(), recs,
                                      C.byref(taken)))
    steps = [{f: getattr(recs[k], f) for f, _ in _StepInfo._fields_} for k in range(taken.value)]
    return u, steps, st


# Candidates of the parameter tuner: the region of the paper's tests and discussion -- the
# base pattern, static patches in every direction and strips along the flow axis, dynamic
# patterns with a few (n_add, n_ent), with and without post-filtration on H~.
DEFAULT_CANDIDATES = (
    Params("static"),
    Params("static", static_level=1),
    Params("static", static_level=1, static_axis=4),
    Params("static", static_level=2, static_axis=4),
    Params("dynamic", n_add=1, n_ent=4),
    Params("dynamic", n_add=1, n_ent=6),
    Params("dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H"),
    Params("dynamic", n_add=2, n_ent=6, tau=1e-3, filt="post_H"),
    Params("dynamic", n_add=4, n_ent=12, tau=1e-3, filt="post_H"),
)


def tune_params(system: System, candidates=DEFAULT_CANDIDATES, rtol=1e-8, restart=50,
                max_iter=5000, method="gmres", flexible=None):
    """Time setup + solve of every candidate on `system` and return (best Params, list of
    {params, ms, iterations, status}).  flexible defaults to True for FP32 candidates."""
    cands = list(candidates)
    arr = (_Params * len(cands))(*[p.c() for p in cands])
    flex = any(p.precision == 1 for p in cands) if flexible is None else flexible
    sp = _SolveParams(restart, max_iter, int(flex), 0, 0, 0, float(rtol), METHOD[method])
    best = C.c_int32(-1)
    times = (C.c_double * len(cands))()
    its = (C.c_int32 * len(cands))()
    sts = (C.c_int32 * len(cands))()
    _check(load().edfa_tune_params(system._h, arr, len(cands), C.byref(sp), _stream(),
                                   C.byref(best), times, its, sts))
    rec = [{"params": p, "ms": times[k], "iterations": its[k], "status": sts[k]}
           for k, p in enumerate(cands)]
    return cands[best.value], rec


def grad_logk(system: System, u, lam):
    g = torch.empty(system.info["ne"], dtype=torch.float64, device="cuda")
    _check(load().edfa_grad_logk(system._h, _ptr(u), _ptr(lam), _ptr(g), _stream()))
    return g


def csr_to_scipy(rp, col, val, shape):
    import scipy.sparse as sp
    return sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=shape)
