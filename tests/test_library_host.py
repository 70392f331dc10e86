"""Host-side checks of the HIP library (no GPU needed).

The library must load and export every symbol ``include/hdg.h`` declares; its
host-only 1D setup (GLL points, derivative matrix, generalized
eigendecomposition, B_S) is compared with the oracle's independent
construction and with the invariants of the paper's equations.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle.basis import standard_matrices
from oracle.fastdiag import b_s
import paper_2007_11891_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libhdg.so not built (python -m paper_2007_11891_amd.build)")
    return pkg.load_library()


def test_header_declares_exactly_the_exported_names():
    with open(os.path.join(ROOT, "include", "hdg.h")) as fh:
        text = fh.read()
    declared = set(re.findall(r"\b(hdg_[a-z_0-9]+)\s*\(", text))
    assert declared == set(pkg.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in pkg.EXPORTS:
        assert hasattr(lib, name), name


def test_default_options():
    o = pkg.default_opts()
    assert o.rtol == 1e-10 and o.precond == 1 and o.mixed == 0 and o.check_every >= 1


def test_create_rejects_invalid_arguments_without_gpu_work():
    lib = _lib()
    n = (ctypes.c_int * 3)(2, 2, 2)
    h = (ctypes.c_double * 2)(0.5, 0.5)
    bad = (ctypes.c_double * 2)(0.5, -0.5)
    out = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    hp = ctypes.cast(h, dp)
    cases = [
        (n, hp, hp, hp, 0, 1.0, None, 1.0),            # p = 0
        (n, hp, hp, hp, 17, 1.0, None, 1.0),           # p = 17
        (n, hp, hp, hp, 3, 0.0, None, 1.0),            # tau = 0
        (n, hp, hp, hp, 3, 1.0, None, -1.0),           # lambda < 0
        (n, hp, ctypes.cast(bad, dp), hp, 3, 1.0, None, 1.0),   # negative width
        ((ctypes.c_int * 3)(0, 2, 2), hp, hp, hp, 3, 1.0, None, 1.0),
    ]
    for args in cases:
        st = lib.hdg_create(*args, None, ctypes.byref(out))
        assert st == -1, args
        assert out.value is None
        assert lib.hdg_last_error()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 7, 10, 16])
def test_library_tables_match_oracle(p):
    _lib()
    tau = 1.3
    t = pkg.tables(p, tau)
    s = standard_matrices(p, tau)
    assert np.abs(t["x"] - s["x"]).max() < 1e-15
    assert np.abs(t["w"] - s["w"]).max() < 1e-15
    assert np.abs(t["D"] - s["D"]).max() < 1e-12 * max(1.0, np.abs(s["D"]).max())
    S, lam = t["S"], t["Lam"]
    n = p + 1
    # generalized eigendecomposition (equation generalized_eigenvalue_decomposition)
    assert np.abs(S.T @ s["M"] @ S - np.eye(n)).max() < 1e-13
    assert np.abs(S.T @ s["L"] @ S - np.diag(lam)).max() < 1e-13 * np.abs(lam).max()
    assert np.all(np.diff(lam) >= 0)
    # B_S of equation (hdgbs) with the library's S
    assert np.abs(t["BS"] - b_s(s, S)).max() < 1e-12 * max(1.0, np.abs(t["BS"]).max())
    H = s["G"] + s["C"].T @ np.linalg.inv(s["M"]) @ s["C"]
    assert np.abs(H - t["H"] * np.eye(2)).max() < 1e-13 * abs(t["H"])


def test_tables_reject_bad_degree():
    _lib()
    with pytest.raises(pkg.HdgError):
        pkg.tables(0, 1.0)


def test_batch_create_rejects_invalid_arguments_without_gpu_work():
    lib = _lib()
    out = ctypes.c_void_p()
    ip = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)

    def call(count, n, p, lam, tau=1.0):
        na = (ctypes.c_int * len(n))(*n)
        pa = (ctypes.c_int * len(p))(*p)
        la = (ctypes.c_double * len(lam))(*lam)
        return lib.hdg_batch_create(count, ctypes.cast(na, ip), ctypes.cast(pa, ip),
                                    ctypes.cast(la, dp), tau, None, ctypes.byref(out))

    cases = [
        (0, [2, 2, 2], [3], [1.0], 1.0),              # no problems
        (1, [2, 0, 2], [3], [1.0], 1.0),              # empty axis
        (1, [2, 2, 5000], [3], [1.0], 1.0),           # axis too long
        (1, [2, 2, 2], [11], [1.0], 1.0),             # degree beyond the batched kernels
        (1, [2, 2, 2], [0], [1.0], 1.0),              # degree 0
        (2, [2, 2, 2, 2, 2, 2], [3, 4], [1.0, -1.0], 1.0),   # lambda < 0
        (1, [2, 2, 2], [3], [float("nan")], 1.0),     # lambda NaN
        (1, [2, 2, 2], [3], [1.0], 0.0),              # tau = 0
    ]
    for count, n, p, lam, tau in cases:
        assert call(count, n, p, lam, tau) == -1, (count, n, p, lam, tau)
        assert out.value is None
        assert lib.hdg_last_error()
    assert lib.hdg_batch_create(1, None, None, None, 1.0, None, ctypes.byref(out)) == -1
    assert lib.hdg_batch_destroy(None) == 0



def test_neumann_mask_validation_without_gpu():
    """hdg_create_ex rejects a mask outside 0..63, an exact_mass flag other
    than 0 / 1 and the singular pure Neumann problem with lambda = 0 before
    touching a device."""
    import ctypes
    import numpy as np
    import paper_2007_11891_amd as pkg
    lib = pkg.load_library()
    n = (ctypes.c_int * 3)(2, 2, 2)
    h = np.array([0.5, 0.5])
    dp = ctypes.POINTER(ctypes.c_double)
    out = ctypes.c_void_p()
    args = [n, h.ctypes.data_as(dp), h.ctypes.data_as(dp), h.ctypes.data_as(dp), 3, 1.0]
    assert lib.hdg_create_ex(*args, None, 1.0, 64, 0, None, ctypes.byref(out)) == -1
    assert b"neumann" in lib.hdg_last_error()
    assert lib.hdg_create_ex(*args, None, 1.0, 0, 2, None, ctypes.byref(out)) == -1
    assert b"exact_mass" in lib.hdg_last_error()
    assert lib.hdg_create_ex(*args, None, 0.0, 63, 0, None, ctypes.byref(out)) == -1
    assert b"singular" in lib.hdg_last_error()
    lam = np.zeros(8)
    assert lib.hdg_create_ex(*args, lam.ctypes.data_as(dp), 0.0, 63, 1, None,
                             ctypes.byref(out)) == -1
    assert not out.value


@pytest.mark.parametrize("mask", [0, 1, 2, 0b001100, 0b110000, 0b101010, 0b010101, 63])
@pytest.mark.parametrize("n,p", [((3, 2, 2), 2), ((1, 1, 1), 4), ((1, 4, 2), 1), ((5, 3, 7), 3)])
def test_layout_lengths_match_oracle_without_gpu(n, p, mask):
    """hdg_layout (the host logic of the face numbering of hdg_create_ex)
    against the oracle's layout for every kind of side set, including
    meshes one element thick."""
    import oracle
    import paper_2007_11891_amd as pkg
    L = oracle.Layout(n, p, mask)
    got = pkg.layout(n, p, mask)
    assert (got.n_free, got.n_all, got.n_vol) == (L.n_free, L.n_all, L.n_vol)


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and a message,
    before touching torch or the library."""
    import subprocess
    import sys
    from pathlib import Path
    root = Path(__file__).resolve().parents[1]
    r = subprocess.run([sys.executable, str(root / "bench.py"), "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
