"""ctypes binding of the C++ oracle (oracle/pyjac_ref.cpp) -- test infrastructure only."""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pyjac_ref.cpp")
_LIB = os.path.join(_HERE, "libpyjac_oracle.so")


def oracle_lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP, FP64, portable -O3)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle(force=False)
        lib = ctypes.CDLL(_LIB)
        vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        lib.pyjac_ref_last_error.restype = ctypes.c_char_p
        lib.pyjac_ref_mech_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        lib.pyjac_ref_mech_load_string.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        lib.pyjac_ref_mech_free.argtypes = [vp]
        lib.pyjac_ref_mech_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.pyjac_ref_eval_rates.argtypes = [vp, i64, i64, dp, dp, dp, dp, dp, dp, dp, i32]
        lib.pyjac_ref_eval_rhs_ld.argtypes = [vp, i64, i64, dp, dp, dp, i32]
        lib.pyjac_ref_eval_jacobian.argtypes = [vp, i64, i64, dp, dp, dp, i32]
        lib.pyjac_ref_eval_jacobian_cs.argtypes = [vp, i64, i64, dp, dp, dp, ctypes.c_double, i32]
        lib.pyjac_ref_eval_rhs_conc.argtypes = [vp, i64, i64, dp, dp, i32]
        lib.pyjac_ref_eval_jacobian_conc.argtypes = [vp, i64, i64, dp, dp, i32]
        lib.pyjac_ref_eval_jacobian_conc_cs.argtypes = [vp, i64, i64, dp, dp, ctypes.c_double, i32]
        lib.pyjac_ref_species_thermo.argtypes = [vp, ctypes.c_double, dp, dp, dp]
        lib.pyjac_ref_reaction_terms.argtypes = [vp, ctypes.c_double, ctypes.c_double, dp,
                                                 dp, dp, dp, dp, dp, dp, dp, dp]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class RefMech:
    """A mechanism loaded into the oracle."""

    def __init__(self, path: Optional[str] = None, text: Optional[str] = None):
        lib = _load()
        h = ctypes.c_void_p()
        if text is not None:
            rc = lib.pyjac_ref_mech_load_string(text.encode(), ctypes.byref(h))
        else:
            rc = lib.pyjac_ref_mech_load(path.encode(), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle mechanism load failed ({rc}): "
                             f"{lib.pyjac_ref_last_error().decode()}")
        self._h = h
        ns, nr = ctypes.c_int(), ctypes.c_int()
        lib.pyjac_ref_mech_info(h, ctypes.byref(ns), ctypes.byref(nr))
        self.n_species, self.n_reactions = ns.value, nr.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pyjac_ref_mech_free(self._h)
            self._h = None

    def _chk(self, rc):
        if rc != 0:
            raise RuntimeError(f"oracle call failed ({rc}): {_lib.pyjac_ref_last_error().decode()}")

    def eval_rates(self, phi, p, nthreads: int = 0):
        phi, p = _f64(phi), _f64(p)
        N, NR, n = self.n_species, self.n_reactions, phi.shape[1]
        out = {k: np.empty((NR, n)) for k in ("rop_f", "rop_r", "pres_mod")}
        out.update({k: np.empty((N, n)) for k in ("wdot", "dphi")})
        self._chk(_lib.pyjac_ref_eval_rates(self._h, n, n, _ptr(phi), _ptr(p), _ptr(out["rop_f"]),
                                            _ptr(out["rop_r"]), _ptr(out["pres_mod"]),
                                            _ptr(out["wdot"]), _ptr(out["dphi"]), nthreads))
        return out

    def eval_rhs_ld(self, phi_ld, p, nthreads: int = 0):
        phi_ld = np.ascontiguousarray(phi_ld, dtype=np.longdouble)
        p = _f64(p)
        n = phi_ld.shape[1]
        out = np.empty((self.n_species, n), dtype=np.longdouble)
        self._chk(_lib.pyjac_ref_eval_rhs_ld(self._h, n, n, _ptr(phi_ld), _ptr(p), _ptr(out),
                                             nthreads))
        return out

    def eval_jacobian(self, phi, p, nthreads: int = 0):
        """Analytical Jacobian, shape (N*N, n_states): row-major per state."""
        phi, p = _f64(phi), _f64(p)
        n = phi.shape[1]
        jac = np.empty((self.n_species ** 2, n))
        self._chk(_lib.pyjac_ref_eval_jacobian(self._h, n, n, _ptr(phi), _ptr(p), _ptr(jac),
                                               nthreads))
        return jac

    def eval_jacobian_cs(self, phi, p, step: float = 1e-30, nthreads: int = 0):
        phi, p = _f64(phi), _f64(p)
        n = phi.shape[1]
        jac = np.empty((self.n_species ** 2, n))
        self._chk(_lib.pyjac_ref_eval_jacobian_cs(self._h, n, n, _ptr(phi), _ptr(p), _ptr(jac),
                                                  step, nthreads))
        return jac

    # constant-volume, concentration-based form: phi_c is (N+1, n) with rows
    # T, [X_1], ..., [X_N]
    def eval_rhs_conc(self, phi_c, nthreads: int = 0):
        phi_c = _f64(phi_c)
        n = phi_c.shape[1]
        f = np.empty((self.n_species + 1, n))
        self._chk(_lib.pyjac_ref_eval_rhs_conc(self._h, n, n, _ptr(phi_c), _ptr(f), nthreads))
        return f

    def eval_jacobian_conc(self, phi_c, nthreads: int = 0):
        """Analytical Jacobian of the concentration form, shape ((N+1)^2, n)."""
        phi_c = _f64(phi_c)
        n = phi_c.shape[1]
        jac = np.empty(((self.n_species + 1) ** 2, n))
        self._chk(_lib.pyjac_ref_eval_jacobian_conc(self._h, n, n, _ptr(phi_c), _ptr(jac), nthreads))
        return jac

    def eval_jacobian_conc_cs(self, phi_c, step: float = 1e-30, nthreads: int = 0):
        phi_c = _f64(phi_c)
        n = phi_c.shape[1]
        jac = np.empty(((self.n_species + 1) ** 2, n))
        self._chk(_lib.pyjac_ref_eval_jacobian_conc_cs(self._h, n, n, _ptr(phi_c), _ptr(jac), step,
                                                       nthreads))
        return jac

    def species_thermo(self, T: float):
        N = self.n_species
        cpR, hRT, sR = np.empty(N), np.empty(N), np.empty(N)
        self._chk(_lib.pyjac_ref_species_thermo(self._h, float(T), _ptr(cpR), _ptr(hRT), _ptr(sR)))
        return cpR, hRT, sR

    def reaction_terms(self, T: float, p: float, y):
        y = _f64(y)
        NR = self.n_reactions
        out = {k: np.empty(NR) for k in ("kf", "kr", "c", "Rf", "Rr", "Kc", "Pr", "F")}
        self._chk(_lib.pyjac_ref_reaction_terms(self._h, float(T), float(p), _ptr(y),
                                                *[_ptr(out[k]) for k in
                                                  ("kf", "kr", "c", "Rf", "Rr", "Kc", "Pr", "F")]))
        return out
