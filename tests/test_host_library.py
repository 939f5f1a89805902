"""CPU-only checks of libsadi.so: it loads, exports every symbol of include/sadi.h, its host
setup mathematics agrees with the oracle, and argument validation fails cleanly."""
import ctypes
import re

import numpy as np
import pytest
import scipy.linalg

import paper_2312_06206_amd as P
from paper_2312_06206_amd import binding
from oracle import coeffs as C


def _declared_symbols():
    src = open(binding.HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sadi_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    names = _declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9])
def test_host_riesz_coeffs_match_oracle(alpha):
    a = P.host_riesz_coeffs(alpha, 4096)
    r = C.riesz_coeffs(alpha, 4096)
    assert (np.abs(a - r) / np.abs(r)).max() < 1e-15


@pytest.mark.parametrize("alpha", [1.01, 1.2, 1.5, 1.8, 1.99])
def test_host_laplacian_coeffs_match_oracle(alpha):
    n = 700
    a = P.host_laplacian_coeffs(alpha, n)
    r = C.laplacian_coeffs(alpha, n)
    rel = np.abs(a - r) / np.abs(r)
    assert rel[:40, :40].max() < 1e-14
    assert rel.max() < 1e-13


def test_host_laplacian_coeffs_full_size():
    a = P.host_laplacian_coeffs(1.5, 4095)
    r = C.laplacian_coeffs(1.5, 4095)
    rel = np.abs(a - r) / np.abs(r)
    assert rel[:64, :64].max() < 1e-14
    assert rel.max() < 5e-13      # the oracle's Bessel values lose ~1e-13 at orders ~4e3
    assert np.array_equal(a, a.T)


@pytest.mark.parametrize("alpha,n", [(1.2, 63), (1.8, 1023)])
def test_host_line_generator_is_first_column_of_inverse(alpha, n):
    tau, kappa = 1e-3, 1.1
    g = P.host_line_generator(alpha, kappa, n, tau)
    h = 2.0 / (n + 1)
    H = np.eye(n + 1) + 0.5 * kappa * tau * tau * h ** (-alpha) * scipy.linalg.toeplitz(C.riesz_coeffs(alpha, n + 1))
    c = scipy.linalg.solve(H, np.eye(n + 1)[:, 0], assume_a="pos")
    assert np.abs(g - c).max() <= 1e-15 * np.abs(c).max()


@pytest.mark.parametrize("args,status", [
    ((0.9, 1.0, 63, 1e-3, (-1.0, 1.0)), -1),      # alpha out of (1,2)
    ((2.0, 1.0, 63, 1e-3, (-1.0, 1.0)), -1),      # alpha = 2 only with injected tables
    ((1.5, -1.0, 63, 1e-3, (-1.0, 1.0)), -1),     # kappa <= 0
    ((1.5, 1.0, 63, 0.0, (-1.0, 1.0)), -1),       # tau <= 0
    ((1.5, 1.0, 63, 1e-3, (1.0, -1.0)), -1),      # b <= a
    ((1.5, 1.0, 63, float("nan"), (-1.0, 1.0)), -1),
    ((1.5, 1.0, 0, 1e-3, (-1.0, 1.0)), -1),       # N < 1
    ((1.5, 1.0, 5000, 1e-3, (-1.0, 1.0)), -4),    # N above 4095
    ((1.5, 1.0, 10, 1e-3, (-1.0, 1.0)), -4),      # N below 15
    ((1.5, 1.0, 8191, 1e-3, (-1.0, 1.0)), -4),    # too large
])
def test_setup_rejects_bad_arguments_without_touching_the_gpu(args, status):
    lib = P.load_library()
    alpha, kappa, n, tau, dom = args
    d = np.asarray(dom, dtype=np.float64)
    ctx = ctypes.c_void_p(123)
    st = lib.sadi_setup(alpha, kappa, n, tau, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(ctx))
    assert st == status
    assert ctx.value is None
    assert lib.sadi_last_error().decode() != ""


def test_calls_on_null_context_fail_with_state_error():
    lib = P.load_library()
    assert lib.sadi_step(None, None, None) == -5
    assert lib.sadi_step_noalloc(None, None, None) == -5
    assert lib.sadi_run(None, None, None, 1) == -5
    assert lib.sadi_first_step(None, None, None, None) == -5
    assert lib.sadi_toeplitz_solve(None, None, 1, 1) == -5
    assert lib.sadi_apply_lh(None, None, None) == -5
    assert lib.sadi_get_line_tables(None, None, None, None) == -5
    assert lib.sadi_get_info(None, None, None, None) == -5
    assert lib.sadi_destroy(None) == 0
    assert lib.sadi_batch_get_group(None, 0, None, None, None, None, None, None, None) == -5
    assert lib.sadi_batch_set_path(None, 63, 2) == -5
    assert lib.sadi_batch_tune(None, 1) == -5


def test_host_line_tables_match_dense_solve():
    """sadi_host_line_tables (the host reference of the device tables): lam_c = fft(c) / M
    and f[k] = c[M-1-k] / c[0] for c = H_M^-1 e_1 from a dense solve, at N = 63 (M = 64)."""
    alpha, kappa, n, tau = 1.6, 1.0, 63, 1e-2
    ls, lc, f = P.host_line_tables(alpha, kappa, n, tau)
    m = n + 1
    h = 2.0 / (n + 1)
    H = np.eye(m) + 0.5 * kappa * tau * tau * h ** (-alpha) * scipy.linalg.toeplitz(C.riesz_coeffs(alpha, m))
    c = scipy.linalg.solve(H, np.eye(m)[:, 0], assume_a="pos")
    assert np.abs(lc - np.fft.fft(c) / m).max() <= 1e-15 * np.abs(lc).max()
    assert np.abs(f - c[m - 1 - np.arange(n)] / c[0]).max() <= 1e-15 * np.abs(f).max()
    # lam_s = fft(Q s) / (2 p1 M), s = (p1, -c[M-1], ..., -c[1]), Q = diag(e^{-i pi j / M})
    sv = np.concatenate(([c[0]], -c[:0:-1]))
    q = np.exp(-1j * np.pi * np.arange(m) / m)
    assert np.abs(ls - np.fft.fft(q * sv) / (2 * c[0] * m)).max() <= 1e-15 * np.abs(ls).max()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.load_library()


def test_batch_create_rejects_bad_arguments_without_touching_the_gpu():
    """Validation of the batched entry point happens before any device work."""
    import ctypes
    from paper_2312_06206_amd import binding as B
    lib = B.load_library()
    dom = np.array([-1.0, 1.0])
    h = ctypes.c_void_p()
    n = (ctypes.c_int * 2)(63, 127)
    al = np.array([1.5, 1.5])
    ka = np.array([1.0, 1.0])
    assert lib.sadi_batch_create(0, n, B._dptr(al), B._dptr(ka), 1e-3, B._dptr(dom), 127, ctypes.byref(h)) == -1
    assert lib.sadi_batch_create(2, None, B._dptr(al), B._dptr(ka), 1e-3, B._dptr(dom), 127, ctypes.byref(h)) == -1
    bad = np.array([1.5, 2.5])          # alpha outside (1, 2) for the second instance
    assert lib.sadi_batch_create(2, n, B._dptr(bad), B._dptr(ka), 1e-3, B._dptr(dom), 127, ctypes.byref(h)) == -1
    assert b"instance 1" in lib.sadi_last_error()
    n_bad = (ctypes.c_int * 2)(63, 5000)  # N above 4095
    assert lib.sadi_batch_create(2, n_bad, B._dptr(al), B._dptr(ka), 1e-3, B._dptr(dom), 127,
                                 ctypes.byref(h)) == -4
    assert not h.value
    assert lib.sadi_batch_run(None, 1) == -5
    assert lib.sadi_batch_destroy(None) == -5


def test_quadrature_rows_double_double_matches_extended_precision():
    """The double-double float64 recurrence that builds the GPU's quadrature table (run here
    on the host) against the long double one of the host set-up: every node and order k <
    4096, relative to each value (values above 1e-250)."""
    x, dd = P.host_quadrature_rows(4096, fp64=True)
    _, ld = P.host_quadrature_rows(4096, fp64=False)
    assert dd.shape == ld.shape == (x.size, 4096)
    big = np.abs(ld) > 1e-250
    assert np.array_equal(big, np.abs(dd) > 1e-250)
    assert (np.abs(dd[big] - ld[big]) / np.abs(ld[big])).max() <= 2e-15


def test_quadrature_rows_match_scipy_ive():
    """An independent pin of the same rows: scipy.special.ive (a library routine, not ours) at
    every node below 1e9, relative to each row's largest value; the normalisation
    e^-x (I_0 + 2 sum_k I_k) = 1 holds where the orders cover the sum."""
    import scipy.special as sp
    x, dd = P.host_quadrature_rows(4096, fp64=True)
    k = np.arange(4096)
    sel = x < 1e9
    ref = sp.ive(k[None, :], x[sel, None])
    err = np.abs(dd[sel] - ref) / np.abs(ref).max(axis=1, keepdims=True)
    assert np.nanmax(err) <= 1e-12
    full = x < 1e4       # orders < 4096 hold the whole sum there (terms fall like e^{-k^2/2x})
    tot = dd[full, 0] + 2 * dd[full, 1:].sum(axis=1)
    assert np.abs(tot - 1.0).max() <= 1e-13
