"""MI355X (gfx950) library for the hot path of the analytical chemical-kinetics
Jacobian of Niemeyer, Curtis & Sung (arXiv:1605.03262).

The work happens in libpyjac_mi355x.so (HIP kernels behind the C ABI of
include/pyjac.h).  `Mechanism` is a thin convenience wrapper: it takes torch
tensors on the GPU, passes their device pointers and the current HIP stream,
and allocates outputs.  PyTorch serves only as device memory and streams.
"""
from __future__ import annotations

from . import _lib
from ._lib import PyjacError, load_library  # noqa: F401
from ._lib import pyjac_chemkin_to_text as chemkin_to_text  # noqa: F401

NEWTON_FP64 = 0
NEWTON_MIXED = 1
NEWTON_REUSE_FACTOR = 16     # or-ed into the mode: solve with the factor kept in the workspace
NEWTON_KEEP_FACTOR = 32      # or-ed into the mode: keep the register path's FP64 factor there


def _torch():
    import torch
    return torch


class Mechanism:
    """A mechanism whose tables live on one GPU."""

    def __init__(self, path: str | None = None, text: str | None = None, device: int = 0,
                 _handle: int | None = None):
        self.device = device
        if _handle is not None:
            self._h = _handle
        else:
            if (path is None) == (text is None):
                raise ValueError("give exactly one of path or text")
            self._h = (_lib.pyjac_mech_load(path, device) if path is not None
                       else _lib.pyjac_mech_load_string(text, device))
        self.n_species, self.n_reactions, self.content_hash = _lib.pyjac_mech_info(self._h)

    @classmethod
    def from_chemkin(cls, path: str, thermo: str | None = None, device: int = 0) -> "Mechanism":
        """Load a Chemkin-format mechanism file (thermo data inside it or in
        the separate file `thermo`)."""
        return cls(device=device, _handle=_lib.pyjac_mech_load_chemkin(path, thermo, device))

    @property
    def handle(self) -> int:
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.pyjac_mech_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def _check_in(self, phi, p):
        torch = _torch()
        N = self.n_species
        if phi.dtype != torch.float64 or p.dtype != torch.float64:
            raise TypeError("phi and p must be float64")
        if not (phi.is_cuda and p.is_cuda):
            raise TypeError("phi and p must be GPU tensors")
        if phi.dim() != 2 or phi.shape[0] != N or phi.stride(1) != 1:
            raise ValueError(f"phi must be [{N}, ld] with unit stride along states")
        ld = phi.stride(0)
        n = phi.shape[1]
        if p.dim() != 1 or p.shape[0] < n or p.stride(0) != 1:
            raise ValueError("p must be a contiguous vector of at least n_states entries")
        return n, ld

    @staticmethod
    def _stream():
        return _torch().cuda.current_stream().cuda_stream

    @staticmethod
    def _ptr(t):
        return None if t is None else t.data_ptr()

    # ----------------------------------------------------------- kernels
    def eval_rates(self, phi, p, rop_f=True, rop_r=True, pres_mod=True, wdot=True, dphi=True):
        """Rates, production rates and the RHS; returns a dict of [*, ld] tensors."""
        torch = _torch()
        n, ld = self._check_in(phi, p)
        N, NR = self.n_species, self.n_reactions
        out = {}
        mk = lambda rows: torch.empty((rows, ld), dtype=torch.float64, device=phi.device)  # noqa: E731
        for name, flag, rows in (("rop_f", rop_f, NR), ("rop_r", rop_r, NR),
                                 ("pres_mod", pres_mod, NR), ("wdot", wdot, N), ("dphi", dphi, N)):
            out[name] = mk(rows) if flag is True else (flag if flag is not False else None)
        _lib.pyjac_eval_rates(self._h, n, ld, phi.data_ptr(), p.data_ptr(),
                              self._ptr(out["rop_f"]), self._ptr(out["rop_r"]),
                              self._ptr(out["pres_mod"]), self._ptr(out["wdot"]),
                              self._ptr(out["dphi"]), self._stream())
        return {k: v for k, v in out.items() if v is not None}

    def eval_jacobian(self, phi, p, out=None):
        """Dense Jacobian, a [N*N, ld] tensor (element i*N + j is dF_i/dPhi_j)."""
        torch = _torch()
        n, ld = self._check_in(phi, p)
        N = self.n_species
        if out is None:
            out = torch.empty((N * N, ld), dtype=torch.float64, device=phi.device)
        elif out.shape[0] != N * N or out.stride(0) != ld or out.stride(1) != 1:
            raise ValueError("out must be [N*N, ld] with the same ld as phi")
        _lib.pyjac_eval_jacobian(self._h, n, ld, phi.data_ptr(), p.data_ptr(), out.data_ptr(),
                                 self._stream())
        return out

    def conc_pattern(self):
        """Compressed-column pattern (colptr [N+1], rowidx [nnz]) of the sparse
        part of the concentration-form Jacobian."""
        if getattr(self, "_conc_pattern", None) is None:
            self._conc_pattern = _lib.pyjac_conc_pattern(self._h)
        return self._conc_pattern

    def eval_jacobian_conc(self, phi_c, out=None):
        """Concentration-based, constant-volume Jacobian for phi_c [N+1, n]
        (rows T, [X_1..X_N]); returns [3N+1+nnz, ld] (layout in pyjac.h)."""
        torch = _torch()
        N = self.n_species
        if phi_c.dtype != torch.float64 or not phi_c.is_cuda or phi_c.dim() != 2 or phi_c.shape[0] != N + 1 \
                or phi_c.stride(1) != 1:
            raise ValueError("phi_c must be a float64 GPU tensor [N+1, n] with unit state stride")
        n, ld = phi_c.shape[1], phi_c.stride(0)
        rows = 3 * N + 1 + len(self.conc_pattern()[1])
        if out is None:
            out = torch.empty((rows, ld), dtype=torch.float64, device=phi_c.device)
        elif out.shape[0] != rows or out.stride(0) != ld or out.stride(1) != 1:
            raise ValueError(f"out must be [{rows}, ld] with the same ld as phi_c")
        _lib.pyjac_eval_jacobian_conc(self._h, n, ld, phi_c.data_ptr(), out.data_ptr(), self._stream())
        return out

    def eval_jacobian_cs(self, phi, p, step: float = 1e-30, out=None):
        """Complex-step Jacobian of the RHS, same layout as eval_jacobian."""
        torch = _torch()
        n, ld = self._check_in(phi, p)
        N = self.n_species
        if out is None:
            out = torch.empty((N * N, ld), dtype=torch.float64, device=phi.device)
        elif out.shape[0] != N * N or out.stride(0) != ld or out.stride(1) != 1:
            raise ValueError("out must be [N*N, ld] with the same ld as phi")
        _lib.pyjac_eval_jacobian_cs(self._h, n, ld, phi.data_ptr(), p.data_ptr(), float(step), out.data_ptr(),
                                    self._stream())
        return out

    def eval_jacobian_fd(self, phi, p, out=None, chunk_states: int = 8192, workspace=None):
        """Forward-difference Jacobian (same layout as eval_jacobian)."""
        torch = _torch()
        n, ld = self._check_in(phi, p)
        N = self.n_species
        if out is None:
            out = torch.empty((N * N, ld), dtype=torch.float64, device=phi.device)
        elif out.shape[0] != N * N or out.stride(0) != ld or out.stride(1) != 1:
            raise ValueError("out must be [N*N, ld] with the same ld as phi")
        if workspace is None:
            need = _lib.pyjac_fd_workspace_bytes(self._h, max(1, min(n, chunk_states)))
            workspace = torch.empty((need,), dtype=torch.uint8, device=phi.device)
        wsb = workspace.numel() * workspace.element_size()
        _lib.pyjac_eval_jacobian_fd(self._h, n, ld, phi.data_ptr(), p.data_ptr(), out.data_ptr(),
                                    workspace.data_ptr(), wsb, self._stream())
        return out

    def newton_workspace_bytes(self, n_states: int, mode: int) -> int:
        return _lib.pyjac_newton_workspace_bytes(self._h, n_states, mode)

    def newton_solve(self, jac, h, rhs, gamma: float, mode: int = NEWTON_MIXED,
                     max_refine: int = 10, rtol: float = 1e-14, workspace=None):
        """Solve (I - h gamma J) x = rhs per state; returns (x, info).
        `mode` is NEWTON_FP64 or NEWTON_MIXED, optionally or-ed with
        NEWTON_KEEP_FACTOR (keep the factor in `workspace`, sized by
        newton_workspace_bytes(n, mode)) or NEWTON_REUSE_FACTOR (solve with
        the factor the previous call left in the same workspace)."""
        torch = _torch()
        N = self.n_species
        ld = rhs.stride(0)
        n = rhs.shape[1]
        if jac.stride(0) != ld or h.shape[0] < n:
            raise ValueError("jac, rhs must share ld; h must cover n_states")
        x = torch.empty((N, ld), dtype=torch.float64, device=rhs.device)
        info = torch.empty((ld,), dtype=torch.int32, device=rhs.device)
        need = self.newton_workspace_bytes(n, mode)
        if workspace is None and need:
            workspace = torch.empty((need,), dtype=torch.uint8, device=rhs.device)
        wsb = 0 if workspace is None else workspace.numel() * workspace.element_size()
        _lib.pyjac_newton_factor_solve(self._h, n, ld, jac.data_ptr(), h.data_ptr(), float(gamma),
                                       rhs.data_ptr(), x.data_ptr(), mode, max_refine, rtol,
                                       info.data_ptr(), self._ptr(workspace), wsb, self._stream())
        return x, info

    def sdirk3_step(self, phi, p, h, newton_iters: int = 4, mode: int = NEWTON_FP64, out=None,
                    workspace=None):
        """One SDIRK3 step per state (constant pressure); returns
        (phi_next [N, ld], dnorm [3, ld]: each stage's last Newton increment)."""
        torch = _torch()
        n, ld = self._check_in(phi, p)
        N = self.n_species
        if h.dtype != torch.float64 or not h.is_cuda or h.dim() != 1 or h.shape[0] < n or h.stride(0) != 1:
            raise ValueError("h must be a contiguous float64 GPU vector covering n_states")
        if out is None:
            out = torch.empty((N, ld), dtype=torch.float64, device=phi.device)
        elif out.shape[0] != N or out.stride(0) != ld or out.stride(1) != 1:
            raise ValueError("out must be [N, ld] with the same ld as phi")
        dnorm = torch.empty((3, ld), dtype=torch.float64, device=phi.device)
        need = _lib.pyjac_sdirk3_workspace_bytes(self._h, n, ld, mode)
        if workspace is None:
            workspace = torch.empty((max(need, 1),), dtype=torch.uint8, device=phi.device)
        wsb = workspace.numel() * workspace.element_size()
        _lib.pyjac_sdirk3_step(self._h, n, ld, phi.data_ptr(), p.data_ptr(), h.data_ptr(), newton_iters, mode,
                               out.data_ptr(), dnorm.data_ptr(), workspace.data_ptr(), wsb, self._stream())
        return out, dnorm

    def set_variant(self, which: int, tile_states: int, threads: int) -> None:
        _lib.pyjac_mech_set_variant(self._h, which, tile_states, threads)

    def autotune(self, which: int, phi, p, out=None, reps: int = 3):
        """Time every launch shape of kernel family `which` (0 rates, 1
        Jacobian, 2 concentration-form Jacobian: phi is phi_c [N+1, n], p is
        ignored) on this batch and keep the fastest; returns
        [((tile_states, threads), median ms), ...]."""
        torch = _torch()
        if which == 2:
            n, ld = phi.shape[1], phi.stride(0)
            p = phi
            rows = 3 * self.n_species + 1 + len(self.conc_pattern()[1])
        else:
            n, ld = self._check_in(phi, p)
            rows = self.n_species * (self.n_species if which == 1 else 1)
        if out is None:
            out = torch.empty((rows, ld), dtype=torch.float64, device=phi.device)
        elif out.shape[0] != rows or out.stride(0) != ld or out.stride(1) != 1:
            raise ValueError(f"out must be [{rows}, ld] with the same ld as phi")
        return _lib.pyjac_mech_autotune(self._h, which, n, ld, phi.data_ptr(), p.data_ptr(),
                                        out.data_ptr(), reps, self._stream())

    def get_variant(self, which: int):
        return _lib.pyjac_mech_get_variant(self._h, which)


class Server:
    """Continuous-batching server (C++ scheduler in the library): requests of
    any mechanism are packed into rounds that run concurrently on several
    streams with resident per-mechanism pools, one Jacobian launch per launch
    shape for all mechanisms of a round, and HIP-graph replay of repeated
    rounds.  submit() copies the inputs into pinned staging memory;
    the output arrays it returns are filled when the request completes and
    are kept referenced here until wait() returns."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 64 << 30,
                 max_batch_states: int = 16384, n_streams: int = 4, max_refine: int = 4,
                 rtol: float = 1e-14):
        self._h = _lib.pyjac_serve_create(device, hbm_budget_bytes, max_batch_states, n_streams,
                                          max_refine, rtol)
        self._keep = {}

    def submit(self, mech: "Mechanism", phi, p, h, rhs, gamma: float, mode: int = NEWTON_MIXED):
        """phi [N, n], p [n], h [n], rhs [N, n] as C-contiguous float64 numpy
        arrays; returns (request id, x [N, n], info [n]) with x/info filled
        once wait(id) has returned."""
        import numpy as np
        phi, p, h, rhs = (np.ascontiguousarray(a, dtype=np.float64) for a in (phi, p, h, rhs))
        n = phi.shape[1]
        x = np.empty((mech.n_species, n))
        info = np.empty(n, dtype=np.int32)
        rid = _lib.pyjac_serve_submit(self._h, mech.handle, n, phi.ctypes.data, p.ctypes.data,
                                      h.ctypes.data, rhs.ctypes.data, float(gamma), mode,
                                      x.ctypes.data, info.ctypes.data)
        self._keep[rid] = (phi, p, h, rhs, x, info)
        return rid, x, info

    def wait(self, request_id: int, timeout_s: float = -1.0) -> float:
        """Latency of the request in seconds once it has completed.  On a
        timeout the request stays in flight and its arrays stay referenced."""
        try:
            lat = _lib.pyjac_serve_wait(self._h, request_id, timeout_s)
        except PyjacError as err:
            if "timed out" not in str(err):
                self._keep.pop(request_id, None)
            raise
        self._keep.pop(request_id, None)
        return lat

    def stats(self):
        return _lib.pyjac_serve_stats(self._h)

    def graph_stats(self):
        """Rounds run eagerly / captured / replayed, Jacobian launches and
        launches that served several mechanisms."""
        return _lib.pyjac_serve_graph_stats(self._h)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.pyjac_serve_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
