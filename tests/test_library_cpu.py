"""The C-ABI library loads without a GPU and exports every symbol that
include/submat.h declares; constants agree between header and binding.
No compute calls here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "submat.h")
LIB = os.path.join(ROOT, "paper_1710_10899_amd", "libsubmat.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(submat_[a-z_]+)\s*\(", text)))


def _defines():
    out = {}
    for m in re.finditer(r"#define\s+(SUBMAT_[A-Z0-9_]+)\s+(-?\d+)", open(HEADER).read()):
        out[m.group(1)] = int(m.group(2))
    return out


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsubmat.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_1710_10899_amd import _lib
    assert set(_declared()) == set(_lib.SIGNATURES)
    for k, v in _defines().items():
        assert getattr(_lib, k) == v, k


def test_version_strerror_options_without_gpu():
    from paper_1710_10899_amd import _lib
    _lib.load()
    assert _lib.submat_version() == 131
    assert _lib.submat_strerror(-3) == "diagonal entry not stored"
    assert _lib.submat_strerror(0) == "ok"
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_KAPPA_MAX) == 1e5
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_CLUSTER_TOL) == 1e-7
    _lib.submat_set_option(_lib.SUBMAT_OPT_CLUSTER_TOL, 0.5)
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_CLUSTER_TOL) == 0.5
    _lib.submat_set_option(_lib.SUBMAT_OPT_CLUSTER_TOL, 1e-7)
    with pytest.raises(_lib.SubmatError):
        _lib.submat_set_option(_lib.SUBMAT_OPT_CLUSTER_TOL, 1.0)
    with pytest.raises(_lib.SubmatError):
        _lib.submat_set_option(_lib.SUBMAT_OPT_KAPPA_MAX, 0.5)
    with pytest.raises(_lib.SubmatError):
        _lib.submat_set_option(999, 1.0)
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_XCD_QUEUES) == 1
    _lib.submat_set_option(_lib.SUBMAT_OPT_XCD_QUEUES, 0)
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_XCD_QUEUES) == 0
    _lib.submat_set_option(_lib.SUBMAT_OPT_XCD_QUEUES, 1)
    with pytest.raises(_lib.SubmatError):
        _lib.submat_set_option(_lib.SUBMAT_OPT_XCD_QUEUES, 2)


def test_invalid_arguments_rejected_before_any_device_work():
    from paper_1710_10899_amd import _lib
    _lib.load()
    # null pointers / bad sizes / bad p / bad dtype fail synchronously
    with pytest.raises(_lib.SubmatError) as e:
        _lib.submat_invroot_fwd(None, None, None, 4, 4, 2, 0, 0, None, None, None)
    assert e.value.code == _lib.SUBMAT_EINVAL
    with pytest.raises(_lib.SubmatError) as e:
        _lib.submat_invroot_fwd(8, 8, 8, 4, 4, 0, 0, 0, 8, None, None)
    assert e.value.code == _lib.SUBMAT_EINVAL
    with pytest.raises(_lib.SubmatError) as e:
        _lib.submat_invroot_fwd(8, 8, 8, 4, 4, 2, 7, 0, 8, None, None)
    assert e.value.code == _lib.SUBMAT_EINVAL
    with pytest.raises(_lib.SubmatError) as e:
        _lib.submat_invroot_bwd(8, 8, 8, 4, 2, 2, 0, 0, 8, 8, None, None)  # nnz < n
    assert e.value.code == _lib.SUBMAT_EINVAL
    # spectral function code and parameter
    for fn, param in ((_lib.SUBMAT_FN_ROOT, 0.0), (_lib.SUBMAT_FN_ROOT, 2.5), (_lib.SUBMAT_FN_INV_ROOT, -1.0),
                      (_lib.SUBMAT_FN_ROOT, 3e9), (_lib.SUBMAT_FN_POWER, float("inf")),
                      (_lib.SUBMAT_FN_POWER, float("nan")), (3, 2.0), (-1, 2.0)):
        with pytest.raises(_lib.SubmatError) as e:
            _lib.submat_matfun_fwd(8, 8, 8, 4, 4, fn, param, 0, 0, 8, None, None)
        assert e.value.code == _lib.SUBMAT_EINVAL, (fn, param)
        with pytest.raises(_lib.SubmatError) as e:
            _lib.submat_matfun_bwd(8, 8, 8, 4, 4, fn, param, 0, 0, 8, 8, None, None)
        assert e.value.code == _lib.SUBMAT_EINVAL, (fn, param)


def test_product_path_does_not_touch_oracle():
    pkg = os.path.join(ROOT, "paper_1710_10899_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("no CPU fallback", ""), f


def test_tuning_table_option(tmp_path, monkeypatch):
    from paper_1710_10899_amd import _lib
    from paper_1710_10899_amd import autotune
    _lib.load()
    path = tmp_path / "tune.txt"
    table = autotune.table_with(autotune.DEFAULTS, 1, 1024, 3)
    assert (1, 1024, 3) in table and (1, 1024, 2) not in table
    autotune.write_table(path, table)
    monkeypatch.setenv("SUBMAT_TUNE_FILE", str(path))
    _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1)
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_TUNE_FILE) == 1.0
    _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 0)
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_TUNE_FILE) == 0.0
    with pytest.raises(_lib.SubmatError):
        _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 2)
    path.write_text("garbage\n")
    _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1)
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_TUNE_FILE) == 0.0


def test_bucket_edge_from_table_unless_set(tmp_path, monkeypatch):
    """The one-wavefront bucket edge is the tuning table's (kind 7, 32
    built in) until SUBMAT_OPT_SMALL_MAX is set; rows outside 1..64 are
    ignored."""
    from paper_1710_10899_amd import _lib
    from paper_1710_10899_amd import autotune
    _lib.load()
    assert (7, 1 << 30, 32) in autotune.DEFAULTS
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("SUBMAT_TUNE_FILE", str(path))
    try:
        for edge, expect in ((48, 48), (65, 32), (0, 32)):
            autotune.write_table(path, autotune.table_with(autotune.DEFAULTS, 7, 1 << 30, edge)
                                 if edge != 65 and edge != 0 else
                                 [r for r in autotune.DEFAULTS if r[0] != 7] + [(7, 1 << 30, edge)])
            _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1)
            assert _lib.submat_get_option(_lib.SUBMAT_OPT_SMALL_MAX) == expect, edge
        _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, 20)
        assert _lib.submat_get_option(_lib.SUBMAT_OPT_SMALL_MAX) == 20
        with pytest.raises(_lib.SubmatError):
            _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, 65)
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, 0)
        _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 0)
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_SMALL_MAX) == 32


def test_deterministic_option_and_release_pattern_without_gpu():
    from paper_1710_10899_amd import _lib
    _lib.load()
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_DETERMINISTIC) == 0.0
    _lib.submat_set_option(_lib.SUBMAT_OPT_DETERMINISTIC, 1)
    assert _lib.submat_get_option(_lib.SUBMAT_OPT_DETERMINISTIC) == 1.0
    _lib.submat_set_option(_lib.SUBMAT_OPT_DETERMINISTIC, 0)
    with pytest.raises(_lib.SubmatError):
        _lib.submat_set_option(_lib.SUBMAT_OPT_DETERMINISTIC, 0.5)
    with pytest.raises(_lib.SubmatError) as e:
        _lib.submat_release_pattern(None, None, 4, 4)
    assert e.value.code == _lib.SUBMAT_EINVAL


def test_csr_wrapper_keeps_index_copies_and_releases_their_plan(monkeypatch):
    """matfun_csr converts int64 CSR indices to int32 once per sparse tensor
    and keeps the copies (fixed addresses) while the tensor lives; when it
    dies the library's plan for those addresses is dropped, so that a later
    pattern of the same n and nnz that lands on the same addresses builds a
    plan of its own instead of meeting the old one."""
    import gc

    import torch

    from paper_1710_10899_amd import _lib, api
    released = []
    monkeypatch.setattr(_lib, "_lib", object())  # looks loaded; no call reaches it
    monkeypatch.setattr(_lib, "submat_release_pattern", lambda *a: released.append(a))
    dense = torch.tensor([[2.0, 1.0, 0.0], [1.0, 2.0, 1.0], [0.0, 1.0, 2.0]], dtype=torch.float64)
    a = dense.to_sparse_csr()
    assert a.crow_indices().dtype == torch.int64
    rp, ci = api._csr_index32(a)
    assert rp.dtype == torch.int32 and ci.dtype == torch.int32
    assert rp.tolist() == a.crow_indices().tolist() and ci.tolist() == a.col_indices().tolist()
    rp2, ci2 = api._csr_index32(a)
    assert rp2 is rp and ci2 is ci  # same tensors, same addresses, same plan
    key = (rp.data_ptr(), ci.data_ptr(), 3, ci.numel())
    del rp, ci, rp2, ci2
    gc.collect()
    assert released == []
    del a
    gc.collect()
    assert released == [key]
    b = (dense + torch.eye(3, dtype=torch.float64)).to_sparse_csr()
    rpb, cib = api._csr_index32(b)
    assert rpb.tolist() == b.crow_indices().tolist()
