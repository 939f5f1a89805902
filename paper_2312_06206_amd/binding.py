"""ctypes binding of libsadi.so (argument marshalling only; all work runs in the library).

Grid arrays are torch.float64 CUDA (HIP) tensors of shape (N, N), contiguous, indexed
[j, i] = u(x_i, y_j) (x fastest, the layout of include/sadi.h).  Calls are enqueued on
torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libsadi.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "sadi.h")

SADI_OK = 0
STATUS = {0: "SADI_OK", -1: "SADI_E_INVALID", -2: "SADI_E_NOMEM", -3: "SADI_E_DEVICE",
          -4: "SADI_E_UNSUPPORTED", -5: "SADI_E_STATE"}
G_KINDS = {"zero": 0, "neg_sin": 1, "neg_cube": 2, "neg_linear": 3}
PRECISIONS = {"fp64": 0, "fp32_refine": 1, "fp32": 2}


class SadiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library() -> ctypes.CDLL:
    """Load the in-tree libsadi.so; fails loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_06206_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, VP = ctypes.POINTER, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    DP = P(ctypes.c_double)
    sig = {
        "sadi_setup": (I, [D, D, I, D, DP, P(VP)]),
        "sadi_setup_with_coeffs": (I, [D, D, I, D, DP, DP, DP, P(VP)]),
        "sadi_set_options": (I, [VP, I, D, I]),
        "sadi_set_stream": (I, [VP, VP]),
        "sadi_first_step": (I, [VP, VP, VP, VP]),
        "sadi_step": (I, [VP, VP, VP]),
        "sadi_step_noalloc": (I, [VP, VP, VP]),
        "sadi_run": (I, [VP, VP, VP, I]),
        "sadi_toeplitz_solve": (I, [VP, VP, I, I]),
        "sadi_apply_lh": (I, [VP, VP, VP]),
        "sadi_get_info": (I, [VP, P(I), P(I), P(ctypes.c_longlong)]),
        "sadi_set_kernel_timing": (I, [VP, I]),
        "sadi_get_kernel_times": (I, [VP, DP, P(ctypes.c_longlong)]),
        "sadi_destroy": (I, [VP]),
        "sadi_last_error": (ctypes.c_char_p, []),
        "sadi_host_riesz_coeffs": (I, [D, I, DP]),
        "sadi_host_laplacian_coeffs": (I, [D, I, DP]),
        "sadi_host_line_generator": (I, [D, D, I, D, DP, DP]),
        "sadi_host_quadrature_rows": (I, [I, I, P(I), DP, DP]),
        "sadi_host_line_tables": (I, [D, D, I, D, DP, DP, DP, DP]),
        "sadi_get_line_tables": (I, [VP, DP, DP, DP]),
        "sadi_adjoint_step": (I, [VP, I, VP, VP, VP, VP, VP, VP, VP]),
        "sadi_batch_create": (I, [I, P(I), DP, DP, D, DP, I, P(VP)]),
        "sadi_batch_bind": (I, [VP, P(VP), P(VP), P(VP)]),
        "sadi_batch_first_step": (I, [VP]),
        "sadi_batch_run": (I, [VP, I]),
        "sadi_batch_set_graph": (I, [VP, I]),
        "sadi_batch_set_path": (I, [VP, I, I]),
        "sadi_batch_tune": (I, [VP, I]),
        "sadi_batch_set_schedule": (I, [VP, I]),
        "sadi_batch_get_schedule": (I, [VP, P(I), DP, DP]),
        "sadi_batch_get_group": (I, [VP, I, P(I), P(I), P(I), DP, DP, DP, P(I)]),
        "sadi_batch_get_info": (I, [VP, P(I), P(I), P(ctypes.c_longlong)]),
        "sadi_batch_synchronize": (I, [VP]),
        "sadi_batch_destroy": (I, [VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != SADI_OK:
        msg = load_library().sadi_last_error().decode()
        raise SadiError(status, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- host-only helpers -----------------------------------------------------------
def host_riesz_coeffs(alpha: float, count: int) -> np.ndarray:
    out = np.empty(count)
    _check(load_library().sadi_host_riesz_coeffs(alpha, count, _dptr(out)))
    return out


def host_laplacian_coeffs(alpha: float, n: int) -> np.ndarray:
    """a_ij as an (n, n) array indexed [i, j] (the table is symmetric)."""
    out = np.empty((n, n))
    _check(load_library().sadi_host_laplacian_coeffs(alpha, n, _dptr(out)))
    return out


def host_line_generator(alpha, kappa, n, tau, domain=(-1.0, 1.0)) -> np.ndarray:
    out = np.empty(n + 1)
    dom = np.asarray(domain, dtype=np.float64)
    _check(load_library().sadi_host_line_generator(alpha, kappa, n, tau, _dptr(dom), _dptr(out)))
    return out


def host_quadrature_rows(nrows: int, fp64: bool = False):
    """(x, rows): the a_ij quadrature's node arguments x_q and e^{-x_q} I_k(x_q) for k < nrows,
    shape (nodes, nrows); fp64 selects the double-double float64 recurrence the GPU table is
    built with (run on the host), else the host's long double one."""
    lib = load_library()
    nq = ctypes.c_int()
    _check(lib.sadi_host_quadrature_rows(int(nrows), int(bool(fp64)), ctypes.byref(nq), None, None))
    x = np.empty(nq.value)
    rows = np.empty((nq.value, nrows))
    _check(lib.sadi_host_quadrature_rows(int(nrows), int(bool(fp64)), ctypes.byref(nq), _dptr(x), _dptr(rows)))
    return x, rows


def _line_size(n: int) -> int:
    m = 16
    while m < n + 1:
        m *= 2
    return m


def host_line_tables(alpha, kappa, n, tau, domain=(-1.0, 1.0)):
    """(lam_s, lam_c, f) of the line matrix from the host's extended-precision set-up:
    complex arrays of M values and f of (M - N) x N."""
    m = _line_size(n)
    ls, lc, f = np.empty(2 * m), np.empty(2 * m), np.empty((m - n) * n)
    dom = np.asarray(domain, dtype=np.float64)
    _check(load_library().sadi_host_line_tables(alpha, kappa, n, tau, _dptr(dom), _dptr(ls), _dptr(lc), _dptr(f)))
    return ls.view(np.complex128), lc.view(np.complex128), f.reshape(m - n, n)


# ---- device solver ---------------------------------------------------------------
def _grid_ptr(t, n: int) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 CUDA tensor")
    if tuple(t.shape) != (n, n) or not t.is_contiguous():
        raise ValueError(f"expected a contiguous ({n}, {n}) tensor")
    return t.data_ptr()


class Solver:
    """S-ADI stepping on one GPU through the C ABI (see include/sadi.h)."""

    def __init__(self, alpha: float, kappa: float, n: int, tau: float, domain: Sequence[float] = (-1.0, 1.0),
                 g: str = "neg_sin", g_param: float = 0.0, precision: str = "fp64",
                 a1: Optional[np.ndarray] = None, a2: Optional[np.ndarray] = None):
        lib = load_library()
        self.n, self.alpha, self.kappa, self.tau = int(n), float(alpha), float(kappa), float(tau)
        self.domain = (float(domain[0]), float(domain[1]))
        dom = np.asarray(self.domain, dtype=np.float64)
        ctx = ctypes.c_void_p()
        if a1 is None and a2 is None:
            _check(lib.sadi_setup(self.alpha, self.kappa, self.n, self.tau, _dptr(dom), ctypes.byref(ctx)))
        else:
            a1 = np.ascontiguousarray(a1, dtype=np.float64)
            a2 = np.ascontiguousarray(np.asarray(a2, dtype=np.float64).T)  # [j*N + i] = a_ij
            if a1.size < self.n + 1 or a2.shape != (self.n, self.n):
                raise ValueError("coefficient tables have the wrong size")
            _check(lib.sadi_setup_with_coeffs(self.alpha, self.kappa, self.n, self.tau, _dptr(dom),
                                              _dptr(a1), _dptr(a2), ctypes.byref(ctx)))
        self._ctx = ctx
        self.set_options(g, g_param, precision)

    # -- plumbing
    def _bind_stream(self):
        import torch
        _check(load_library().sadi_set_stream(self._ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def set_options(self, g: str = "neg_sin", g_param: float = 0.0, precision: str = "fp64"):
        _check(load_library().sadi_set_options(self._ctx, G_KINDS[g], float(g_param), PRECISIONS[precision]))
        self.g, self.g_param, self.precision = g, g_param, precision

    @property
    def info(self):
        n, m, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
        _check(load_library().sadi_get_info(self._ctx, ctypes.byref(n), ctypes.byref(m), ctypes.byref(b)))
        return {"n": n.value, "m": m.value, "device_bytes": b.value}

    KERNELS = ("rows_fwd", "cols_conv", "rows_rhs_gs", "cols_gs")

    def line_tables(self):
        """(lam_s, lam_c, f) as the context holds them (see host_line_tables)."""
        m = self.info["m"]
        ls, lc, f = np.empty(2 * m), np.empty(2 * m), np.empty((m - self.n) * self.n)
        _check(load_library().sadi_get_line_tables(self._ctx, _dptr(ls), _dptr(lc), _dptr(f)))
        return ls.view(np.complex128), lc.view(np.complex128), f.reshape(m - self.n, self.n)

    def set_kernel_timing(self, enable: bool = True):
        _check(load_library().sadi_set_kernel_timing(self._ctx, int(bool(enable))))

    def kernel_times(self):
        """{kernel: (total_ms, launches)} of the steps enqueued since timing was enabled."""
        ms = np.zeros(4)
        cnt = (ctypes.c_longlong * 4)()
        _check(load_library().sadi_get_kernel_times(self._ctx, _dptr(ms), cnt))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.KERNELS)}

    # -- entry points
    def first_step(self, phi1, phi2, out=None):
        import torch
        n = self.n
        if out is None:
            out = torch.empty((n, n), dtype=torch.float64, device=phi1.device)
        self._bind_stream()
        _check(load_library().sadi_first_step(self._ctx, ctypes.c_void_p(_grid_ptr(phi1, n)),
                                              ctypes.c_void_p(_grid_ptr(phi2, n)),
                                              ctypes.c_void_p(_grid_ptr(out, n))))
        return out

    def step(self, u_prev, u_cur):
        """u_prev <- u^{n+1} (in place); returns u_prev."""
        self._bind_stream()
        _check(load_library().sadi_step(self._ctx, ctypes.c_void_p(_grid_ptr(u_prev, self.n)),
                                        ctypes.c_void_p(_grid_ptr(u_cur, self.n))))
        return u_prev

    def step_noalloc(self, u_prev, u_cur):
        """As step(), with the work space in the library's static device array (N <= 1023)."""
        self._bind_stream()
        _check(load_library().sadi_step_noalloc(self._ctx, ctypes.c_void_p(_grid_ptr(u_prev, self.n)),
                                                ctypes.c_void_p(_grid_ptr(u_cur, self.n))))
        return u_prev

    def run(self, u_prev, u_cur, nsteps: int):
        """From (u_prev, u_cur) = (u^{n-1}, u^n): (u^{n+k-1}, u^{n+k}) in place, k = nsteps."""
        self._bind_stream()
        _check(load_library().sadi_run(self._ctx, ctypes.c_void_p(_grid_ptr(u_prev, self.n)),
                                       ctypes.c_void_p(_grid_ptr(u_cur, self.n)), int(nsteps)))
        return u_prev, u_cur

    def toeplitz_solve(self, lines):
        """In place H^-1 on every row of a float64 CUDA tensor of shape (nlines, >= N)."""
        import torch
        if not isinstance(lines, torch.Tensor) or lines.dtype != torch.float64 or not lines.is_cuda:
            raise TypeError("expected a float64 CUDA tensor")
        if lines.dim() != 2 or lines.stride(1) != 1 or lines.shape[1] < self.n:
            raise ValueError("expected shape (nlines, >= N) with unit stride along lines")
        self._bind_stream()
        _check(load_library().sadi_toeplitz_solve(self._ctx, ctypes.c_void_p(lines.data_ptr()),
                                                  int(lines.shape[0]), int(lines.stride(0))))
        return lines

    def apply_lh(self, u, out=None):
        import torch
        n = self.n
        if out is None:
            out = torch.empty((n, n), dtype=torch.float64, device=u.device)
        self._bind_stream()
        _check(load_library().sadi_apply_lh(self._ctx, ctypes.c_void_p(_grid_ptr(u, n)),
                                            ctypes.c_void_p(_grid_ptr(out, n))))
        return out

    def adjoint_step(self, mode: int, u_prev, u_cur, u_next, a_next, a_next2, a_cur, dkappa):
        """One reverse step (include/sadi.h, sadi_adjoint_step); a_cur written, dkappa (a
        float64 CUDA tensor of one element) incremented."""
        import torch
        n = self.n
        if not (isinstance(dkappa, torch.Tensor) and dkappa.dtype == torch.float64 and dkappa.is_cuda
                and dkappa.numel() == 1):
            raise TypeError("dkappa must be a one-element float64 CUDA tensor")
        ptr = lambda t: ctypes.c_void_p(None if t is None else _grid_ptr(t, n))
        self._bind_stream()
        _check(load_library().sadi_adjoint_step(self._ctx, int(mode), ptr(u_prev), ptr(u_cur), ptr(u_next),
                                                ptr(a_next), ptr(a_next2), ptr(a_cur),
                                                ctypes.c_void_p(dkappa.data_ptr())))
        return a_cur

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _check(load_library().sadi_destroy(self._ctx))
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---- batches ---------------------------------------------------------------------
PATHS = {"fft_gs": 0, "dense": 1, "dense_mixed": 2}
SCHEDULES = {"groups": 0, "work_lists": 1}


class Batch:
    """Independent problems (own N, alpha, kappa; shared tau, domain, g = -sin u, FP64)
    advanced together through the batched entry points of include/sadi.h.  The batch
    runs on its own HIP stream: calls wait for torch's current stream first and the
    batch is synchronised before results are handed back."""

    def __init__(self, n, alpha, kappa, tau: float, domain: Sequence[float] = (-1.0, 1.0), dense_max_n: int = 1023):
        lib = load_library()
        self.n = [int(v) for v in n]
        cnt = len(self.n)
        if not (len(alpha) == len(kappa) == cnt):
            raise ValueError("n, alpha and kappa must have the same length")
        self.alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        self.kappa = np.ascontiguousarray(kappa, dtype=np.float64)
        self.tau = float(tau)
        dom = np.asarray(domain, dtype=np.float64)
        narr = (ctypes.c_int * cnt)(*self.n)
        h = ctypes.c_void_p()
        _check(lib.sadi_batch_create(cnt, narr, _dptr(self.alpha), _dptr(self.kappa), self.tau, _dptr(dom),
                                     int(dense_max_n), ctypes.byref(h)))
        self._h = h
        self._bound = None

    def __len__(self):
        return len(self.n)

    def bind(self, u_prev, u_cur, phi2=None):
        """Lists of contiguous float64 (N_i, N_i) CUDA tensors; kept referenced."""
        cnt = len(self.n)
        if len(u_prev) != cnt or len(u_cur) != cnt or (phi2 is not None and len(phi2) != cnt):
            raise ValueError("one tensor per instance expected")
        arr = ctypes.c_void_p * cnt
        up = arr(*[_grid_ptr(t, n) for t, n in zip(u_prev, self.n)])
        uc = arr(*[_grid_ptr(t, n) for t, n in zip(u_cur, self.n)])
        p2 = arr(*[_grid_ptr(t, n) for t, n in zip(phi2, self.n)]) if phi2 is not None else None
        _check(load_library().sadi_batch_bind(self._h, up, uc, p2))
        self._bound = (list(u_prev), list(u_cur), None if phi2 is None else list(phi2))

    def _before(self):
        import torch
        torch.cuda.current_stream().synchronize()

    def first_step(self):
        self._before()
        _check(load_library().sadi_batch_first_step(self._h))
        self.synchronize()

    def run(self, nsteps: int, sync: bool = True):
        self._before()
        _check(load_library().sadi_batch_run(self._h, int(nsteps)))
        if sync:
            self.synchronize()

    def synchronize(self):
        _check(load_library().sadi_batch_synchronize(self._h))

    def set_graph(self, enable: bool = True):
        _check(load_library().sadi_batch_set_graph(self._h, 1 if enable else 0))

    def set_path(self, n: int, path: str):
        _check(load_library().sadi_batch_set_path(self._h, int(n), PATHS[path]))

    def set_schedule(self, schedule: str):
        """"work_lists": FFT groups up to M = 2048 share one launch per phase; "groups":
        every group launched on its own."""
        _check(load_library().sadi_batch_set_schedule(self._h, SCHEDULES[schedule]))

    def schedule(self):
        """(current schedule, tuned ms per step of "groups", of "work_lists"; -1 if not timed)."""
        sc, m0, m1 = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(load_library().sadi_batch_get_schedule(self._h, ctypes.byref(sc), ctypes.byref(m0), ctypes.byref(m1)))
        names = {v: k for k, v in SCHEDULES.items()}
        return names[sc.value], m0.value, m1.value

    def tune(self, steps: int = 5):
        _check(load_library().sadi_batch_tune(self._h, int(steps)))
        return self.groups()

    def groups(self):
        lib = load_library()
        cnt, ng, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
        _check(lib.sadi_batch_get_info(self._h, ctypes.byref(cnt), ctypes.byref(ng), ctypes.byref(nb)))
        out = []
        names = {v: k for k, v in PATHS.items()}
        for i in range(ng.value):
            n, mem, path, tile = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            mf, md, mm = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            _check(lib.sadi_batch_get_group(self._h, i, ctypes.byref(n), ctypes.byref(mem), ctypes.byref(path),
                                            ctypes.byref(mf), ctypes.byref(md), ctypes.byref(mm), ctypes.byref(tile)))
            out.append({"n": n.value, "members": mem.value, "path": names[path.value],
                        "ms_fft_gs": mf.value, "ms_dense": md.value, "ms_dense_mixed": mm.value,
                        "dense_tile": tile.value})
        return out

    def device_bytes(self) -> int:
        cnt, ng, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
        _check(load_library().sadi_batch_get_info(self._h, ctypes.byref(cnt), ctypes.byref(ng), ctypes.byref(nb)))
        return nb.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().sadi_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
