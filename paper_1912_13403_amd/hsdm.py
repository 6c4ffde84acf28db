"""Thin Python binding of libhsdm (include/hsdm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions carry the names of the C entry points; device buffers are
torch tensors on a ROCm device, used for memory and streams only.  Matrices
cross the boundary column-major: a tensor X is passed as is when
X.stride() == (1, ld); otherwise a column-major copy is made.  Outputs are
returned as column-major tensors (shape (n, n), strides (1, n)), so ordinary
indexing X[i, j] is element (i, j).

There is no fallback: if libhsdm.so is missing or no GPU is visible the
calls raise.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsdm.so")

HSDM_OK = 0
HSDM_NOT_SPD = 1
HSDM_NO_CONVERGE = 2
HSDM_MU_FAIL = 3
HSDM_DEVICE_ERROR = 4
HSDM_SYNC_TIMEOUT = 5

HSDM_KEY_FMAX = 1
HSDM_KEY_FCUT = 2
HSDM_KEY_DEG_TOL = 3
HSDM_KEY_TIMING = 4
HSDM_KEY_STREAMS = 5
HSDM_KEY_N_STATES = 6
HSDM_KEY_CONCURRENT = 7
HSDM_KEY_PRECISION = 8
HSDM_KEY_REFINE_STEPS = 9
HSDM_KEY_AUTOTUNE = 10
HSDM_KEY_GRAPH = 11

EXPORTED = [
    "hsdm_init", "hsdm_finalize", "hsdm_reinit", "hsdm_set_real", "hsdm_set_int",
    "hsdm_solve_ev_real", "hsdm_solve_dm_real", "hsdm_solve_ev_complex", "hsdm_solve_dm_complex",
    "hsdm_solve_dm_batch",
    "hsdm_solve_dm_group", "hsdm_task_bytes", "hsdm_workspace_bytes", "hsdm_release_tasks",
    "hsdm_cholesky_inverse", "hsdm_standard_form",
    "hsdm_tridiagonalize", "hsdm_tridiag_eigh", "hsdm_occupations", "hsdm_density",
    "hsdm_dgemm", "hsdm_status_string", "hsdm_last_error", "hsdm_status_detail",
    "hsdm_phase_times", "hsdm_phase_name", "hsdm_phase_flops", "hsdm_kernel_count", "hsdm_kernel_stat",
    "hsdm_version", "hsdm_timing_kernel", "hsdm_solve_dm_real_noalloc", "hsdm_refine_history",
    "hsdm_tune_entries", "hsdm_tune_clear", "hsdm_tune_save", "hsdm_tune_load",
    "hsdm_last_graph", "hsdm_probe",
]

HSDM_NOALLOC_MAX_N = 512

_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double


def load_library(path: str = LIB_PATH):
    """Load libhsdm.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhsdm.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    sig = {
        "hsdm_init": ([ctypes.POINTER(_vp), _i], _i),
        "hsdm_finalize": ([_vp], _i),
        "hsdm_reinit": ([_vp], _i),
        "hsdm_set_real": ([_vp, _i, _d], _i),
        "hsdm_set_int": ([_vp, _i, ctypes.c_long], _i),
        "hsdm_solve_ev_real": ([_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _vp], _i),
        "hsdm_solve_dm_real": ([_vp, _i, _vp, _i, _vp, _i, _d, _d, _vp, _i, _vp, _i, _vp,
                                ctypes.POINTER(_d), ctypes.POINTER(_d), _vp], _i),
        "hsdm_solve_dm_real_noalloc": ([_vp, _i, _vp, _i, _vp, _i, _d, _d, _vp, _i, _vp, _i,
                                        _vp, ctypes.POINTER(_d), ctypes.POINTER(_d), _vp], _i),
        "hsdm_solve_ev_complex": ([_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _vp], _i),
        "hsdm_solve_dm_complex": ([_vp, _i, _vp, _i, _vp, _i, _d, _d, _vp, _i, _vp, _i, _vp,
                                   ctypes.POINTER(_d), ctypes.POINTER(_d), _vp], _i),
        "hsdm_solve_dm_batch": ([_vp, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _d, _d, _vp, _vp,
                                 _vp, _vp, ctypes.POINTER(_d), ctypes.POINTER(_d), _vp], _i),
        "hsdm_solve_dm_group": ([_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp, _vp, _vp], _i),
        "hsdm_task_bytes": ([_i, _i], _d),
        "hsdm_workspace_bytes": ([_vp], _d),
        "hsdm_release_tasks": ([_vp, _d], _i),
        "hsdm_cholesky_inverse": ([_vp, _i, _vp, _i, _vp, _i, _vp, _i, _vp], _i),
        "hsdm_standard_form": ([_vp, _i, _vp, _i, _vp, _i, _vp, _i, _vp], _i),
        "hsdm_tridiagonalize": ([_vp, _i, _vp, _i, _vp, _vp, _vp, _i, _vp], _i),
        "hsdm_tridiag_eigh": ([_vp, _i, _vp, _vp, _vp, _vp, _i, _vp], _i),
        "hsdm_occupations": ([_vp, _i, _vp, _d, _d, _d, _vp, ctypes.POINTER(_d),
                              ctypes.POINTER(_d), ctypes.POINTER(_i), _vp], _i),
        "hsdm_density": ([_vp, _i, _i, _vp, _i, _vp, _vp, _vp, _i, _vp, _i, _vp], _i),
        "hsdm_dgemm": ([_vp, ctypes.c_char, ctypes.c_char, _i, _i, _i, _d, _vp, _i, _vp, _i, _d,
                        _vp, _i, _vp], _i),
        "hsdm_status_string": ([_i], ctypes.c_char_p),
        "hsdm_last_error": ([_vp], ctypes.c_char_p),
        "hsdm_status_detail": ([_vp], _i),
        "hsdm_phase_times": ([_vp, ctypes.POINTER(_d), _i], _i),
        "hsdm_phase_name": ([_i], ctypes.c_char_p),
        "hsdm_phase_flops": ([_vp, ctypes.POINTER(_d), _i], _i),
        "hsdm_kernel_count": ([_vp], _i),
        "hsdm_kernel_stat": ([_vp, _i, ctypes.POINTER(_d)], ctypes.c_char_p),
        "hsdm_version": ([], _i),
        "hsdm_timing_kernel": ([_vp, ctypes.c_char_p], _i),
        "hsdm_refine_history": ([_vp, ctypes.POINTER(_d), _i], _i),
        "hsdm_tune_entries": ([], _i),
        "hsdm_tune_clear": ([], _i),
        "hsdm_tune_save": ([ctypes.c_char_p], _i),
        "hsdm_tune_load": ([ctypes.c_char_p], _i),
        "hsdm_last_graph": ([_vp], _i),
        "hsdm_probe": ([_vp, _i, _d, ctypes.POINTER(_d), _vp], _i),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


class HsdmError(RuntimeError):
    def __init__(self, status, message="", detail=0):
        self.status = status
        self.detail = detail
        super().__init__(f"hsdm status {status}: {message}")


def _colmajor(x: torch.Tensor) -> torch.Tensor:
    if x.dtype != torch.float64:
        raise TypeError("FP64 tensors expected")
    if x.dim() == 2 and x.stride(0) == 1 and x.stride(1) >= max(1, x.shape[0]):
        return x
    return x.t().contiguous().t()


def _colmajor_c(x: torch.Tensor) -> torch.Tensor:
    if x.dtype != torch.complex128:
        raise TypeError("complex128 tensors expected")
    if x.dim() == 2 and x.stride(0) == 1 and x.stride(1) >= max(1, x.shape[0]):
        return x
    return x.t().contiguous().t()


def _ld(x: torch.Tensor) -> int:
    return int(max(1, x.stride(1))) if x.dim() == 2 else int(max(1, x.shape[0]))


def empty_colmajor(n: int, m: int, device) -> torch.Tensor:
    return torch.empty((m, n), dtype=torch.float64, device=device).t()


def empty_colmajor_c(n: int, m: int, device) -> torch.Tensor:
    return torch.empty((m, n), dtype=torch.complex128, device=device).t()


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def hsdm_task_bytes(n: int, is_complex: bool) -> float:
    """Device bytes a task context of size n holds (no GPU needed)."""
    return float(load_library().hsdm_task_bytes(int(n), int(bool(is_complex))))


_live_handles = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    """Finalize every handle still open when the interpreter exits, while the
    HIP runtime and torch are still up (interpreter-exit garbage collection
    would otherwise run hsdm_finalize in whatever order objects die)."""
    for h in list(_live_handles):
        try:
            h.close()
        except Exception:
            pass


class Handle:
    """An hsdm_handle bound to one GPU (hsdm_init / hsdm_finalize)."""

    def __init__(self, device=0):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libhsdm needs an MI355X")
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = _vp()
        st = lib.hsdm_init(ctypes.byref(h), self.device.index or 0)
        if st != 0:
            raise HsdmError(st, "hsdm_init failed")
        self._h = h
        self._lib = lib
        self.n_states = 0
        _live_handles.add(self)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hsdm_finalize(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != 0:
            msg = self._lib.hsdm_last_error(self._h).decode()
            raise HsdmError(st, msg or self._lib.hsdm_status_string(st).decode(),
                            self._lib.hsdm_status_detail(self._h))

    # ---- settings -----------------------------------------------------------
    def hsdm_set_real(self, key, value):
        self._check(self._lib.hsdm_set_real(self._h, key, float(value)))

    def hsdm_set_int(self, key, value):
        self._check(self._lib.hsdm_set_int(self._h, key, int(value)))
        if key == HSDM_KEY_N_STATES:
            self.n_states = int(value)

    def _ncols(self, n):
        """Eigenvector columns an eigenpair solve of size n writes."""
        return self.n_states if 0 < self.n_states < n else n

    def hsdm_reinit(self):
        self._check(self._lib.hsdm_reinit(self._h))

    def phase_times(self):
        buf = (ctypes.c_double * 16)()
        k = self._lib.hsdm_phase_times(self._h, buf, 16)
        return {self._lib.hsdm_phase_name(i).decode(): buf[i] for i in range(k)}

    def hsdm_timing_kernel(self, name):
        """Time only the launches of kernel `name` (None: every kernel)."""
        self._check(self._lib.hsdm_timing_kernel(self._h, name.encode() if name else None))

    def hsdm_probe(self, which, size):
        """Measured FP64 matrix-core rate (which 0: TFLOP/s over `size` rounds per
        wavefront) or HBM copy bandwidth (which 1: GB/s over a `size`-byte
        buffer), as (rate, ms, flops or bytes)."""
        out = (ctypes.c_double * 3)()
        self._check(self._lib.hsdm_probe(self._h, int(which), float(size), out, None))
        return out[0], out[1], out[2]

    def phase_flops(self):
        """Algorithmic flops of each phase of the last single solve (timing on)."""
        buf = (ctypes.c_double * 16)()
        k = self._lib.hsdm_phase_flops(self._h, buf, 16)
        return {self._lib.hsdm_phase_name(i).decode(): buf[i] for i in range(k)}

    def refine_history(self):
        """Steps of the last refined-form solve: [(delta, max |e_ij|), ...]
        (empty after an FP64 solve)."""
        buf = (ctypes.c_double * 16)()
        k = self._lib.hsdm_refine_history(self._h, buf, 16)
        if k < 0:
            self._check(k)
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(min(k, 8))]

    def kernel_stats(self):
        """Per-kernel totals of the last solve (HSDM_KEY_TIMING = 2):
        name -> {"ms", "flops", "bytes", "launches"}."""
        out = {}
        buf = (ctypes.c_double * 4)()
        for i in range(self._lib.hsdm_kernel_count(self._h)):
            name = self._lib.hsdm_kernel_stat(self._h, i, buf)
            if name is None:
                continue
            out[name.decode()] = {"ms": buf[0], "flops": buf[1], "bytes": buf[2],
                                  "launches": int(buf[3])}
        return out

    # ---- solves ------------------------------------------------------------
    def hsdm_solve_ev_real(self, H, S):
        H, S = _colmajor(H), _colmajor(S)
        n = H.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=self.device)
        C = empty_colmajor(n, self._ncols(n), self.device)
        self._check(self._lib.hsdm_solve_ev_real(self._h, n, H.data_ptr(), _ld(H), S.data_ptr(),
                                                 _ld(S), w.data_ptr(), C.data_ptr(), _ld(C),
                                                 _stream_ptr(self.device)))
        return w, C

    def hsdm_solve_dm_real(self, H, S, n_electrons, kT, want_e=True, want_eval=True, out=None):
        H, S = _colmajor(H), _colmajor(S)
        n = H.shape[0]
        if out is None:
            D = empty_colmajor(n, n, self.device)
            E = empty_colmajor(n, n, self.device) if want_e else None
            w = torch.empty(n, dtype=torch.float64, device=self.device) if want_eval else None
        else:
            D, E, w = out
        mu = ctypes.c_double(0.0)
        eb = ctypes.c_double(0.0)
        self._check(self._lib.hsdm_solve_dm_real(
            self._h, n, H.data_ptr(), _ld(H), S.data_ptr(), _ld(S), float(n_electrons), float(kT),
            D.data_ptr(), _ld(D), E.data_ptr() if E is not None else None,
            _ld(E) if E is not None else n, w.data_ptr() if w is not None else None,
            ctypes.byref(eb), ctypes.byref(mu), _stream_ptr(self.device)))
        return dict(D=D, E=E, eval=w, mu=mu.value, band_energy=eb.value)

    def hsdm_solve_dm_real_noalloc(self, H, S, n_electrons, kT, out):
        """hsdm_solve_dm_real_noalloc: the library allocates no device memory;
        the caller passes the outputs out = (D, E or None, eval or None),
        column-major float64 tensors (n <= HSDM_NOALLOC_MAX_N)."""
        if _colmajor(H) is not H or _colmajor(S) is not S:
            raise ValueError("H and S must be column-major float64 tensors (no copies made)")
        n = H.shape[0]
        D, E, w = out
        mu = ctypes.c_double(0.0)
        eb = ctypes.c_double(0.0)
        self._check(self._lib.hsdm_solve_dm_real_noalloc(
            self._h, n, H.data_ptr(), _ld(H), S.data_ptr(), _ld(S), float(n_electrons), float(kT),
            D.data_ptr(), _ld(D), E.data_ptr() if E is not None else None,
            _ld(E) if E is not None else n, w.data_ptr() if w is not None else None,
            ctypes.byref(eb), ctypes.byref(mu), _stream_ptr(self.device)))
        return dict(D=D, E=E, eval=w, mu=mu.value, band_energy=eb.value)

    def hsdm_solve_ev_complex(self, H, S):
        """Eigenpairs of a Hermitian pencil: (eval, C) with C^H S C = I (C holds
        the lowest n_states vectors when HSDM_KEY_N_STATES is set)."""
        H, S = _colmajor_c(H), _colmajor_c(S)
        n = H.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=self.device)
        C = empty_colmajor_c(n, self._ncols(n), self.device)
        self._check(self._lib.hsdm_solve_ev_complex(self._h, n, H.data_ptr(), _ld(H), S.data_ptr(),
                                                    _ld(S), w.data_ptr(), C.data_ptr(), _ld(C),
                                                    _stream_ptr(self.device)))
        return w, C

    def hsdm_solve_dm_complex(self, H, S, n_electrons, kT, want_e=True, want_eval=True):
        """Hermitian pencil (complex128 tensors; lower triangles read)."""
        H, S = _colmajor_c(H), _colmajor_c(S)
        n = H.shape[0]
        D = empty_colmajor_c(n, n, self.device)
        E = empty_colmajor_c(n, n, self.device) if want_e else None
        w = torch.empty(n, dtype=torch.float64, device=self.device) if want_eval else None
        mu = ctypes.c_double(0.0)
        eb = ctypes.c_double(0.0)
        self._check(self._lib.hsdm_solve_dm_complex(
            self._h, n, H.data_ptr(), _ld(H), S.data_ptr(), _ld(S), float(n_electrons), float(kT),
            D.data_ptr(), _ld(D), E.data_ptr() if E is not None else None,
            _ld(E) if E is not None else n, w.data_ptr() if w is not None else None,
            ctypes.byref(eb), ctypes.byref(mu), _stream_ptr(self.device)))
        return dict(D=D, E=E, eval=w, mu=mu.value, band_energy=eb.value)

    def hsdm_solve_dm_batch(self, Hs, Ss, n_electrons, kT, weights=None, want_e=True):
        """Unit tasks sharing one chemical potential: lists of float64 (real
        tasks) or complex128 (Hermitian tasks) tensors."""
        cplx = Hs[0].dtype == torch.complex128
        conv = _colmajor_c if cplx else _colmajor
        empty = empty_colmajor_c if cplx else empty_colmajor
        Hs = [conv(x) for x in Hs]
        Ss = [conv(x) for x in Ss]
        k = len(Hs)
        ns = [int(x.shape[0]) for x in Hs]
        Ds = [empty(m, m, self.device) for m in ns]
        Es = [empty(m, m, self.device) for m in ns] if want_e else None
        I = ctypes.c_int * k
        P = ctypes.c_void_p * k
        w = (ctypes.c_double * k)(*weights) if weights is not None else None
        mu = ctypes.c_double(0.0)
        eb = ctypes.c_double(0.0)
        self._check(self._lib.hsdm_solve_dm_batch(
            self._h, k, int(cplx), I(*ns), P(*[x.data_ptr() for x in Hs]), I(*[_ld(x) for x in Hs]),
            P(*[x.data_ptr() for x in Ss]), I(*[_ld(x) for x in Ss]), w, float(n_electrons),
            float(kT), P(*[x.data_ptr() for x in Ds]), I(*[_ld(x) for x in Ds]),
            P(*[x.data_ptr() for x in Es]) if Es is not None else None,
            I(*[_ld(x) for x in Es]) if Es is not None else None,
            ctypes.byref(eb), ctypes.byref(mu), _stream_ptr(self.device)))
        return dict(D=Ds, E=Es, mu=mu.value, band_energy=eb.value)

    def hsdm_solve_dm_group(self, tasks, want_e=True):
        """Independent problems in one call.  tasks: list of dicts with H, S
        (float64 or complex128 tensors), n_electrons, kT and optionally f_max.
        Returns a list of dicts (D, E, mu, band_energy)."""
        k = len(tasks)
        cplx = [int(t["H"].dtype == torch.complex128) for t in tasks]
        Hs = [(_colmajor_c if c else _colmajor)(t["H"]) for t, c in zip(tasks, cplx)]
        Ss = [(_colmajor_c if c else _colmajor)(t["S"]) for t, c in zip(tasks, cplx)]
        ns = [int(x.shape[0]) for x in Hs]
        Ds = [(empty_colmajor_c if c else empty_colmajor)(m, m, self.device)
              for m, c in zip(ns, cplx)]
        Es = ([(empty_colmajor_c if c else empty_colmajor)(m, m, self.device)
               for m, c in zip(ns, cplx)] if want_e else None)
        I = ctypes.c_int * k
        P = ctypes.c_void_p * k
        F = ctypes.c_double * k
        fm = [t.get("f_max") for t in tasks]
        fmax = F(*fm) if all(v is not None for v in fm) else None
        mu = F()
        eb = F()
        self._check(self._lib.hsdm_solve_dm_group(
            self._h, k, I(*cplx), I(*ns), P(*[x.data_ptr() for x in Hs]), I(*[_ld(x) for x in Hs]),
            P(*[x.data_ptr() for x in Ss]), I(*[_ld(x) for x in Ss]),
            F(*[float(t["n_electrons"]) for t in tasks]), F(*[float(t["kT"]) for t in tasks]),
            fmax, P(*[x.data_ptr() for x in Ds]), I(*[_ld(x) for x in Ds]),
            P(*[x.data_ptr() for x in Es]) if Es is not None else None,
            I(*[_ld(x) for x in Es]) if Es is not None else None, eb, mu,
            _stream_ptr(self.device)))
        return [dict(D=Ds[p], E=Es[p] if Es is not None else None, mu=mu[p], band_energy=eb[p])
                for p in range(k)]

    def hsdm_workspace_bytes(self):
        return float(self._lib.hsdm_workspace_bytes(self._h))

    def hsdm_release_tasks(self, keep_bytes):
        self._check(self._lib.hsdm_release_tasks(self._h, float(keep_bytes)))

    # ---- phases --------------------------------------------------------------
    def hsdm_cholesky_inverse(self, S):
        S = _colmajor(S)
        n = S.shape[0]
        L = empty_colmajor(n, n, self.device)
        Li = empty_colmajor(n, n, self.device)
        self._check(self._lib.hsdm_cholesky_inverse(self._h, n, S.data_ptr(), _ld(S), L.data_ptr(),
                                                    _ld(L), Li.data_ptr(), _ld(Li),
                                                    _stream_ptr(self.device)))
        return L, Li

    def hsdm_standard_form(self, H, Linv):
        H, Linv = _colmajor(H), _colmajor(Linv)
        n = H.shape[0]
        A = empty_colmajor(n, n, self.device)
        self._check(self._lib.hsdm_standard_form(self._h, n, H.data_ptr(), _ld(H),
                                                 Linv.data_ptr(), _ld(Linv), A.data_ptr(), _ld(A),
                                                 _stream_ptr(self.device)))
        return A

    def hsdm_tridiagonalize(self, A, want_q=True):
        A = _colmajor(A)
        n = A.shape[0]
        d = torch.empty(n, dtype=torch.float64, device=self.device)
        e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=self.device)
        Q = empty_colmajor(n, n, self.device) if want_q else None
        self._check(self._lib.hsdm_tridiagonalize(self._h, n, A.data_ptr(), _ld(A), d.data_ptr(),
                                                  e.data_ptr(), Q.data_ptr() if Q is not None else None,
                                                  _ld(Q) if Q is not None else n,
                                                  _stream_ptr(self.device)))
        return d, e[: n - 1], Q

    def hsdm_tridiag_eigh(self, d, e):
        n = d.shape[0]
        d = d.contiguous()
        e = e.contiguous() if n > 1 else torch.zeros(1, dtype=torch.float64, device=self.device)
        w = torch.empty(n, dtype=torch.float64, device=self.device)
        Z = empty_colmajor(n, n, self.device)
        self._check(self._lib.hsdm_tridiag_eigh(self._h, n, d.data_ptr(), e.data_ptr(), w.data_ptr(),
                                                Z.data_ptr(), _ld(Z), _stream_ptr(self.device)))
        return w, Z

    def hsdm_occupations(self, eval_, n_electrons, kT, deg_tol=0.0):
        eval_ = eval_.contiguous()
        n = eval_.shape[0]
        f = torch.empty(n, dtype=torch.float64, device=self.device)
        mu, eb, m = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        self._check(self._lib.hsdm_occupations(self._h, n, eval_.data_ptr(), float(n_electrons),
                                               float(kT), float(deg_tol), f.data_ptr(),
                                               ctypes.byref(mu), ctypes.byref(eb), ctypes.byref(m),
                                               _stream_ptr(self.device)))
        return f, mu.value, eb.value, m.value

    def hsdm_density(self, C, f, eval_, m=None, want_e=True):
        C = _colmajor(C)
        n = C.shape[0]
        m = C.shape[1] if m is None else m
        D = empty_colmajor(n, n, self.device)
        E = empty_colmajor(n, n, self.device) if want_e else None
        self._check(self._lib.hsdm_density(self._h, n, m, C.data_ptr(), _ld(C), f.contiguous().data_ptr(),
                                           eval_.contiguous().data_ptr(), D.data_ptr(), _ld(D),
                                           E.data_ptr() if E is not None else None,
                                           _ld(E) if E is not None else n, _stream_ptr(self.device)))
        return D, E

    def hsdm_dgemm(self, transa, transb, alpha, A, B, beta=0.0, C=None):
        A, B = _colmajor(A), _colmajor(B)
        m = A.shape[1] if transa == "T" else A.shape[0]
        k = A.shape[0] if transa == "T" else A.shape[1]
        n = B.shape[0] if transb == "T" else B.shape[1]
        if C is None:
            C = empty_colmajor(m, n, self.device)
            beta = 0.0
        else:
            C = _colmajor(C)
        self._check(self._lib.hsdm_dgemm(self._h, transa.encode(), transb.encode(), m, n, k,
                                         float(alpha), A.data_ptr(), _ld(A), B.data_ptr(), _ld(B),
                                         float(beta), C.data_ptr(), _ld(C),
                                         _stream_ptr(self.device)))
        return C
