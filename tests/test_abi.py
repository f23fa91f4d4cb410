"""The C-ABI library builds, loads and exports every symbol of include/cfust.h
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cfust.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cfust_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2005_06848_amd import _build
    if not os.path.exists(_build.LIB_PATH):
        _build.build()
    return _build.LIB_PATH


def test_every_declared_symbol_is_exported(libpath):
    names = _declared()
    assert "cfust_estep" in names and "cfust_em_fit" in names and "cfust_mstep" in names
    assert "cfust_loglik" in names
    L = ctypes.CDLL(libpath)
    for name in names:
        assert hasattr(L, name), name


def test_host_only_entry_points(libpath):
    L = ctypes.CDLL(libpath)
    L.cfust_stats_size.restype = ctypes.c_int
    for p, q in [(2, 2), (4, 4), (6, 6), (5, 5), (3, 1)]:
        assert L.cfust_stats_size(p, q) == 3 + p + q + p * q + p * (p + 1) // 2 + q * (q + 1) // 2
    L.cfust_aitken_linf.restype = ctypes.c_double
    L.cfust_aitken_linf.argtypes = [ctypes.c_double] * 3
    for lstar, C, r in [(-100.0, 5.0, 0.5), (-2211.3, 40.0, 0.9)]:
        l = [lstar - C * r ** k for k in range(3)]
        assert abs(L.cfust_aitken_linf(*l) - lstar) < 1e-9 * abs(lstar)
    L.cfust_strerror.restype = ctypes.c_char_p
    assert L.cfust_strerror(2) == b"matrix not positive definite"
    from paper_2005_06848_amd import native
    L.cfust_opts_size.restype = ctypes.c_size_t
    assert L.cfust_opts_size() == ctypes.sizeof(native.Opts)


def test_workspace_size_and_limits(libpath):
    from paper_2005_06848_amd import native
    assert native.workspace_size(20000, 4, 4, 3, 4096) > 20000 * 3 * 8 * 17
    with pytest.raises(native.CfustError):
        native.workspace_size(10, 2, 13, 2, 64)  # q above the kernels' limit
    assert native.workspace_size(202, 11, 11, 2, 8192) > 202 * 2 * 8 * (3 + 11 + 66)
    with pytest.raises(native.CfustError):
        native.workspace_size(10, 33, 2, 2, 64)  # p above the limit
    with pytest.raises(native.CfustError):
        native.workspace_size(10, 2, 2, 2, 0)  # no QMC points


def test_product_path_does_not_import_oracle():
    """The binding fails loudly without the library and never reaches the oracle."""
    src = open(os.path.join(ROOT, "paper_2005_06848_amd", "native.py")).read()
    assert "oracle" not in src
    for name in os.listdir(os.path.join(ROOT, "paper_2005_06848_amd")):
        if name.endswith(".py"):
            text = open(os.path.join(ROOT, "paper_2005_06848_amd", name)).read()
            assert "import oracle" not in text and "from oracle" not in text, name


def test_batched_shape_table_and_split_workspace(libpath):
    """The batched form's candidate shapes (host only) include several waves
    per pair, and a batch small enough to be offered them gets a workspace
    with room for the K slice records of every pair."""
    from paper_2005_06848_amd import native
    shapes = []
    k = 0
    while True:
        s = native.cfust_batched_shape(k)
        if s is None:
            break
        shapes.append(s)
        k += 1
    assert len(shapes) == native.cfust_batched_config()["n_candidates"]
    assert native.cfust_batched_shape(-1) is None
    splits = {s["waves_per_pair"] for s in shapes}
    assert splits == {1, 2, 4, 8}
    assert all(s["waves_per_block"] in (1, 2, 4) and s["chunk"] >= 1 for s in shapes)
    L = ctypes.CDLL(libpath)
    L.cfust_batched_workspace_size.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 2 + \
        [ctypes.c_int] * 3 + [ctypes.POINTER(ctypes.c_size_t)]

    def ws(n_list, g_list, N):
        P = len(n_list)
        n_arr = (ctypes.c_int64 * P)(*n_list)
        g_arr = (ctypes.c_int * P)(*g_list)
        out = ctypes.c_size_t(0)
        assert L.cfust_batched_workspace_size(5, 5, P, n_arr, g_arr, N, 1, 10,
                                              ctypes.byref(out)) == 0
        return out.value
    pw = 5 + 5 + 15  # slice record, q = 5
    small = [300] * 8
    pairs = sum(small) * 2
    # N = 2048 allows K = 8, N = 1024 K = 4, N = 256 no split
    d8 = ws(small, [2] * 8, 2048) - ws(small, [2] * 8, 1024)
    assert d8 >= pairs * 8 * pw * 8 - pairs * 4 * pw * 8
    big = [40000, 30000]  # 70000 x 1 pairs >= 65536: one wave per pair
    g1 = [1, 1]
    assert ws(big, g1, 2048) - ws(big, g1, 1024) < pairs * 8 * pw * 8
