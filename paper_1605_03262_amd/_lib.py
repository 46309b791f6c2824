"""ctypes binding of libpyjac_mi355x.so (C ABI in include/pyjac.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Function names mirror the C entry points.  The library must have
been built (paper_1605_03262_amd/build.py); importing this module on a tree
without it raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpyjac_mi355x.so")

PYJAC_OK = 0
STATUS_NAMES = {0: "PYJAC_OK", -1: "PYJAC_E_INVALID", -2: "PYJAC_E_PARSE",
                -3: "PYJAC_E_UNSUPPORTED", -4: "PYJAC_E_DEVICE", -5: "PYJAC_E_NOMEM",
                -6: "PYJAC_E_IO", -7: "PYJAC_E_UNBALANCED", -8: "PYJAC_E_WORKSPACE"}

# Every symbol include/pyjac.h declares.
EXPORTED = ("pyjac_mech_load", "pyjac_mech_load_string", "pyjac_chemkin_to_text",
            "pyjac_mech_load_chemkin", "pyjac_mech_info", "pyjac_mech_free",
            "pyjac_eval_rates", "pyjac_eval_jacobian", "pyjac_eval_jacobian_conc", "pyjac_conc_pattern", "pyjac_mix_pairs", "pyjac_eval_jacobian_cs", "pyjac_eval_jacobian_multi",
            "pyjac_newton_workspace_bytes",
            "pyjac_newton_factor_solve", "pyjac_newton_factor_solve_noalloc", "pyjac_mech_set_variant", "pyjac_mech_get_variant",
            "pyjac_mech_autotune", "pyjac_fd_workspace_bytes", "pyjac_eval_jacobian_fd",
            "pyjac_sdirk3_workspace_bytes", "pyjac_sdirk3_step",
            "pyjac_status_string", "pyjac_last_error", "pyjac_serve_create", "pyjac_serve_submit",
            "pyjac_serve_wait", "pyjac_serve_stats", "pyjac_serve_graph_stats", "pyjac_serve_destroy")


class WorkItem(ctypes.Structure):
    """pyjac_work_item of include/pyjac.h."""
    _fields_ = [("mech", ctypes.c_void_p), ("n_states", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("phi", ctypes.c_void_p), ("p", ctypes.c_void_p), ("jac", ctypes.c_void_p)]


class PyjacError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {detail}")


_lib = None


def load_library() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1605_03262_amd/build.py "
                          "(there is no fallback implementation)")
    # torch carries its own HIP runtime beside the one this library links; the
    # process works when torch's is initialised first, so that happens here,
    # before the library's first HIP call
    try:
        import torch
    except ImportError:
        torch = None
    if torch is not None and torch.cuda.is_available():
        torch.cuda.init()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    st = ctypes.c_int32
    lib.pyjac_mech_load.argtypes = [ctypes.c_char_p, i32, ctypes.POINTER(vp)]
    lib.pyjac_mech_load.restype = st
    lib.pyjac_mech_load_string.argtypes = [ctypes.c_char_p, i32, ctypes.POINTER(vp)]
    lib.pyjac_mech_load_string.restype = st
    lib.pyjac_chemkin_to_text.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, sz,
                                          ctypes.POINTER(sz)]
    lib.pyjac_chemkin_to_text.restype = st
    lib.pyjac_mech_load_chemkin.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i32, ctypes.POINTER(vp)]
    lib.pyjac_mech_load_chemkin.restype = st
    lib.pyjac_mech_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_uint64)]
    lib.pyjac_mech_info.restype = st
    lib.pyjac_mech_free.argtypes = [vp]
    lib.pyjac_mech_free.restype = st
    lib.pyjac_eval_rates.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pyjac_eval_rates.restype = st
    lib.pyjac_eval_jacobian.argtypes = [vp, i64, i64, vp, vp, vp, vp]
    lib.pyjac_eval_jacobian.restype = st
    lib.pyjac_eval_jacobian_conc.argtypes = [vp, i64, i64, vp, vp, vp]
    lib.pyjac_eval_jacobian_conc.restype = st
    lib.pyjac_conc_pattern.argtypes = [vp, vp, vp, ctypes.POINTER(i64)]
    lib.pyjac_conc_pattern.restype = st
    lib.pyjac_mix_pairs.argtypes = [vp, i64, i64, vp, vp, ctypes.c_double, vp, vp]
    lib.pyjac_mix_pairs.restype = st
    lib.pyjac_eval_jacobian_cs.argtypes = [vp, i64, i64, vp, vp, ctypes.c_double, vp, vp]
    lib.pyjac_eval_jacobian_cs.restype = st
    lib.pyjac_eval_jacobian_multi.argtypes = [i32, ctypes.POINTER(WorkItem), vp]
    lib.pyjac_eval_jacobian_multi.restype = st
    lib.pyjac_newton_workspace_bytes.argtypes = [vp, i64, i32]
    lib.pyjac_newton_workspace_bytes.restype = sz
    lib.pyjac_newton_factor_solve.argtypes = [vp, i64, i64, vp, vp, ctypes.c_double, vp, vp, i32,
                                              i32, ctypes.c_double, vp, vp, sz, vp]
    lib.pyjac_newton_factor_solve.restype = st
    lib.pyjac_newton_factor_solve_noalloc.argtypes = [vp, i64, i64, vp, vp, ctypes.c_double, vp, vp, i32,
                                                      i32, ctypes.c_double, vp, vp]
    lib.pyjac_newton_factor_solve_noalloc.restype = st
    lib.pyjac_mech_set_variant.argtypes = [vp, i32, i32, i32]
    lib.pyjac_mech_set_variant.restype = st
    lib.pyjac_mech_get_variant.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                           ctypes.POINTER(sz)]
    lib.pyjac_mech_get_variant.restype = st
    lib.pyjac_fd_workspace_bytes.argtypes = [vp, i64]
    lib.pyjac_fd_workspace_bytes.restype = sz
    lib.pyjac_eval_jacobian_fd.argtypes = [vp, i64, i64, vp, vp, vp, vp, sz, vp]
    lib.pyjac_eval_jacobian_fd.restype = st
    lib.pyjac_sdirk3_workspace_bytes.argtypes = [vp, i64, i64, i32]
    lib.pyjac_sdirk3_workspace_bytes.restype = sz
    lib.pyjac_sdirk3_step.argtypes = [vp, i64, i64, vp, vp, vp, i32, i32, vp, vp, vp, sz, vp]
    lib.pyjac_sdirk3_step.restype = st
    lib.pyjac_mech_autotune.argtypes = [vp, i32, i64, i64, vp, vp, vp, i32, ctypes.POINTER(i32),
                                        ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32), vp]
    lib.pyjac_mech_autotune.restype = st
    lib.pyjac_serve_create.argtypes = [i32, sz, i64, i32, i32, ctypes.c_double, ctypes.POINTER(vp)]
    lib.pyjac_serve_create.restype = st
    lib.pyjac_serve_submit.argtypes = [vp, vp, i64, vp, vp, vp, vp, ctypes.c_double, i32, vp, vp,
                                       ctypes.POINTER(ctypes.c_uint64)]
    lib.pyjac_serve_submit.restype = st
    lib.pyjac_serve_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.pyjac_serve_wait.restype = st
    lib.pyjac_serve_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(sz)]
    lib.pyjac_serve_stats.restype = st
    lib.pyjac_serve_graph_stats.argtypes = [vp] + [ctypes.POINTER(i64)] * 5
    lib.pyjac_serve_graph_stats.restype = st
    lib.pyjac_serve_destroy.argtypes = [vp]
    lib.pyjac_serve_destroy.restype = st
    lib.pyjac_status_string.argtypes = [st]
    lib.pyjac_status_string.restype = ctypes.c_char_p
    lib.pyjac_last_error.argtypes = []
    lib.pyjac_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != PYJAC_OK:
        detail = load_library().pyjac_last_error().decode()
        raise PyjacError(status, where, detail)


# ---------------------------------------------------------- thin C mirrors
def pyjac_mech_load(path: str, device: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load_library().pyjac_mech_load(path.encode(), device, ctypes.byref(h)), "pyjac_mech_load")
    return h.value


def pyjac_mech_load_string(text: str, device: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load_library().pyjac_mech_load_string(text.encode(), device, ctypes.byref(h)),
          "pyjac_mech_load_string")
    return h.value


def pyjac_chemkin_to_text(mech_text: str, thermo_text: str | None = None) -> str:
    lib = load_library()
    th = None if thermo_text is None else thermo_text.encode()
    n = ctypes.c_size_t()
    check(lib.pyjac_chemkin_to_text(mech_text.encode(), th, None, 0, ctypes.byref(n)), "pyjac_chemkin_to_text")
    buf = ctypes.create_string_buffer(n.value)
    check(lib.pyjac_chemkin_to_text(mech_text.encode(), th, buf, n.value, ctypes.byref(n)),
          "pyjac_chemkin_to_text")
    return buf.value.decode()


def pyjac_mech_load_chemkin(mech_path: str, thermo_path: str | None = None, device: int = 0) -> int:
    h = ctypes.c_void_p()
    th = None if thermo_path is None else thermo_path.encode()
    check(load_library().pyjac_mech_load_chemkin(mech_path.encode(), th, device, ctypes.byref(h)),
          "pyjac_mech_load_chemkin")
    return h.value


def pyjac_mech_info(mech: int):
    ns, nr, hh = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_uint64()
    check(load_library().pyjac_mech_info(mech, ctypes.byref(ns), ctypes.byref(nr), ctypes.byref(hh)),
          "pyjac_mech_info")
    return ns.value, nr.value, hh.value


def pyjac_mech_free(mech: int) -> None:
    check(load_library().pyjac_mech_free(mech), "pyjac_mech_free")


def pyjac_eval_rates(mech, n, ld, phi, p, rop_f, rop_r, pres_mod, wdot, dphi, stream) -> None:
    check(load_library().pyjac_eval_rates(mech, n, ld, phi, p, rop_f, rop_r, pres_mod, wdot, dphi,
                                          stream), "pyjac_eval_rates")


def pyjac_eval_jacobian(mech, n, ld, phi, p, jac, stream) -> None:
    check(load_library().pyjac_eval_jacobian(mech, n, ld, phi, p, jac, stream), "pyjac_eval_jacobian")


def pyjac_eval_jacobian_conc(mech, n, ld, phi_c, jac, stream) -> None:
    check(load_library().pyjac_eval_jacobian_conc(mech, n, ld, phi_c, jac, stream), "pyjac_eval_jacobian_conc")


def pyjac_conc_pattern(mech):
    """(colptr [N+1], rowidx [nnz]) as int32 numpy arrays."""
    import numpy as np
    lib = load_library()
    nnz = ctypes.c_int64()
    check(lib.pyjac_conc_pattern(mech, None, None, ctypes.byref(nnz)), "pyjac_conc_pattern")
    ns = ctypes.c_int32()
    check(lib.pyjac_mech_info(mech, ctypes.byref(ns), None, None), "pyjac_mech_info")
    colptr = np.empty(ns.value + 1, dtype=np.int32)
    rowidx = np.empty(max(nnz.value, 1), dtype=np.int32)
    check(lib.pyjac_conc_pattern(mech, colptr.ctypes.data, rowidx.ctypes.data, None), "pyjac_conc_pattern")
    return colptr, rowidx[: nnz.value]


def pyjac_mix_pairs(mech, n, ld, phi, partner, weight, phi_out, stream) -> None:
    check(load_library().pyjac_mix_pairs(mech, n, ld, phi, partner, weight, phi_out, stream), "pyjac_mix_pairs")


def pyjac_eval_jacobian_cs(mech, n, ld, phi, p, step, jac, stream) -> None:
    check(load_library().pyjac_eval_jacobian_cs(mech, n, ld, phi, p, step, jac, stream), "pyjac_eval_jacobian_cs")


def pyjac_eval_jacobian_multi(items, stream) -> None:
    """items: sequence of (mech, n_states, ld, phi, p, jac) tuples."""
    arr = (WorkItem * max(len(items), 1))(*[WorkItem(*it) for it in items])
    check(load_library().pyjac_eval_jacobian_multi(len(items), arr, stream), "pyjac_eval_jacobian_multi")


def pyjac_newton_workspace_bytes(mech, n, mode) -> int:
    return int(load_library().pyjac_newton_workspace_bytes(mech, n, mode))


def pyjac_newton_factor_solve(mech, n, ld, jac, h, gamma, rhs, x, mode, max_refine, rtol, info,
                              workspace, workspace_bytes, stream) -> None:
    check(load_library().pyjac_newton_factor_solve(mech, n, ld, jac, h, gamma, rhs, x, mode,
                                                   max_refine, rtol, info, workspace,
                                                   workspace_bytes, stream),
          "pyjac_newton_factor_solve")


def pyjac_newton_factor_solve_noalloc(mech, n, ld, jac, h, gamma, rhs, x, mode, max_refine, rtol, info,
                                      stream) -> None:
    check(load_library().pyjac_newton_factor_solve_noalloc(mech, n, ld, jac, h, gamma, rhs, x, mode,
                                                           max_refine, rtol, info, stream),
          "pyjac_newton_factor_solve_noalloc")


def pyjac_mech_set_variant(mech, which, tile_states, threads) -> None:
    check(load_library().pyjac_mech_set_variant(mech, which, tile_states, threads),
          "pyjac_mech_set_variant")


def pyjac_mech_get_variant(mech, which):
    ts, nt, lds = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    check(load_library().pyjac_mech_get_variant(mech, which, ctypes.byref(ts), ctypes.byref(nt),
                                                ctypes.byref(lds)), "pyjac_mech_get_variant")
    return ts.value, nt.value, lds.value


def pyjac_fd_workspace_bytes(mech, chunk_states) -> int:
    return int(load_library().pyjac_fd_workspace_bytes(mech, chunk_states))


def pyjac_eval_jacobian_fd(mech, n, ld, phi, p, jac, workspace, workspace_bytes, stream) -> None:
    check(load_library().pyjac_eval_jacobian_fd(mech, n, ld, phi, p, jac, workspace, workspace_bytes, stream),
          "pyjac_eval_jacobian_fd")


def pyjac_mech_autotune(mech, which, n, ld, phi, p, out, reps, stream, max_entries=16):
    shapes = (ctypes.c_int32 * (2 * max_entries))()
    ms = (ctypes.c_float * max_entries)()
    cnt = ctypes.c_int32()
    check(load_library().pyjac_mech_autotune(mech, which, n, ld, phi, p, out, reps, shapes, ms,
                                             max_entries, ctypes.byref(cnt), stream),
          "pyjac_mech_autotune")
    return [((shapes[2 * e], shapes[2 * e + 1]), ms[e]) for e in range(cnt.value)]


def pyjac_serve_create(device, hbm_budget_bytes, max_batch_states, n_streams, max_refine, rtol) -> int:
    h = ctypes.c_void_p()
    check(load_library().pyjac_serve_create(device, hbm_budget_bytes, max_batch_states, n_streams,
                                            max_refine, rtol, ctypes.byref(h)), "pyjac_serve_create")
    return h.value


def pyjac_serve_submit(server, mech, n, phi, p, h, rhs, gamma, mode, x, info) -> int:
    rid = ctypes.c_uint64()
    check(load_library().pyjac_serve_submit(server, mech, n, phi, p, h, rhs, gamma, mode, x, info,
                                            ctypes.byref(rid)), "pyjac_serve_submit")
    return rid.value


def pyjac_serve_wait(server, request_id, timeout_s=-1.0) -> float:
    lat = ctypes.c_double()
    check(load_library().pyjac_serve_wait(server, request_id, timeout_s, ctypes.byref(lat)),
          "pyjac_serve_wait")
    return lat.value


def pyjac_serve_stats(server):
    r, s_, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    p50, p99, use = ctypes.c_double(), ctypes.c_double(), ctypes.c_size_t()
    check(load_library().pyjac_serve_stats(server, ctypes.byref(r), ctypes.byref(s_), ctypes.byref(b),
                                           ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(use)),
          "pyjac_serve_stats")
    return {"requests": r.value, "states": s_.value, "batches": b.value, "p50_s": p50.value,
            "p99_s": p99.value, "hbm_in_use": use.value}


def pyjac_serve_graph_stats(server):
    v = [ctypes.c_int64() for _ in range(5)]
    check(load_library().pyjac_serve_graph_stats(server, *[ctypes.byref(x) for x in v]), "pyjac_serve_graph_stats")
    return dict(zip(("eager_rounds", "captured_rounds", "replayed_rounds", "jacobian_launches",
                     "multi_mechanism_launches"), (x.value for x in v)))


def pyjac_serve_destroy(server) -> None:
    check(load_library().pyjac_serve_destroy(server), "pyjac_serve_destroy")


def pyjac_sdirk3_workspace_bytes(mech: int, n: int, ld: int, mode: int) -> int:
    return load_library().pyjac_sdirk3_workspace_bytes(mech, n, ld, mode)


def pyjac_sdirk3_step(mech, n, ld, phi, p, h, newton_iters, mode, phi_out, dnorm, ws, wsb, stream):
    check(load_library().pyjac_sdirk3_step(mech, n, ld, phi, p, h, newton_iters, mode, phi_out, dnorm, ws, wsb,
                                           stream), "pyjac_sdirk3_step")
