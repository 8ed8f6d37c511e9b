"""Host-side tests of the C-ABI library (no GPU needed): it loads, exports
every symbol include/lbm.h declares, validates arguments before touching a
device, and holds the same lattice as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1909_08406_amd import lbm
    return lbm


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 17
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    # and the binding knows each of them
    assert sorted(L.SIGNATURES) == names


def test_selftest(L):
    assert L.selftest() == 0


def test_lattice_matches_oracle(L, orc):
    c1, w1, t1 = L.lattice()
    c2, w2, t2 = orc.lattice()
    assert np.array_equal(c1, c2)
    # Table I weights identical; the rest weight 1 - sum(others) is derived
    # on each side with its own summation order, so it may differ by one
    # unit in the last place of 1.0, the scale of that subtraction
    assert np.array_equal(w1[1:], w2[1:])
    assert abs(w1[0] - w2[0]) <= np.spacing(1.0)
    assert abs(t1 - t2) <= 2 * np.spacing(t2)


def test_argument_validation(L):
    ok = [(8, 8, 8, 0.6)]
    assert L.workspace_size(ok, "f32") > 0
    bad = [
        ([(8, 8, 8, 0.5)], {}),                 # tau_lb must exceed 1/2
        ([], {}),                               # no boxes
        ([(0, 8, 8, 0.6)], {}),                 # empty box
        ([(8, -1, 8, 0.6)], {}),
        ([(8, 8, 8, float("nan"))], {}),
        (ok, {"storage": 7}),                   # unknown storage
        (ok, {"newton_iters": 9}),
        (ok, {"tau_conv": 5}),
        ([(1024, 1024, 1024, 0.6)], {"storage": "f64"}),  # q-block beyond 32-bit offsets
    ]
    for boxes, kw in bad:
        with pytest.raises(L.LbmError) as e:
            L.workspace_size(boxes, **kw)
        assert e.value.code == L.E_ARG, (boxes, kw)
    # paper convention accepts any tau > 0
    assert L.workspace_size([(8, 8, 8, 0.1)], "f32", tau_conv=L.TAU_PAPER) > 0


def test_workspace_size_scales_with_storage(L):
    b = [(32, 16, 16, 0.6)]
    n = 2 * 32 * 16 * 16
    for st, eb in (("f64", 8), ("f32", 4), ("f16s", 2), ("bf16s", 2)):
        assert L.workspace_size(b, st) >= 2 * 41 * n * eb


def test_init_rejects_unrealisable_fields_before_device_work(L):
    n = 2 * 2 * 2 * 2
    one = np.ones(n)
    zero = np.zeros(n)
    for rho, th in ((-one, one), (one, zero), (one * np.nan, one)):
        with pytest.raises(L.LbmError) as e:
            L.init([(2, 2, 2, 0.6)], rho, zero, zero, zero, th * 0.29, torch_workspace=False)
        assert e.value.code == L.E_DOMAIN
    with pytest.raises(ValueError):
        L.init([(2, 2, 2, 0.6)], one[:-1], zero, zero, zero, one, torch_workspace=False)


def test_strerror_covers_codes(L):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.lib().lbm_strerror(code).decode() != "unknown error"


def test_tune_cache_file_parsing(L, tmp_path):
    """The tuning cache file (host code, no device): one entry per line of a
    key and four integers. Lines with one token, extra tokens, values out of
    range (variant, odd graph length) or beyond the line buffer are skipped
    without disturbing the lines around them."""
    path = tmp_path / "tune.txt"
    nv = L.num_variants()
    lines = ["keyA 0 1 0 0", "lonely", "keyB 1 0 1 16", "keyC 1 0 1 16 extra", "keyD %d 0 0 0" % nv,
             "keyE 0 1 0 3", "x" * 20000 + " 0 1 0 0", "keyF %d 1 1 64" % (nv - 1)]
    path.write_text("\n".join(lines) + "\n")
    L.tune_cache_file(None)
    L.tune_cache_clear()
    try:
        L.tune_cache_file(path)
        assert L.tune_cache_count() == 3  # keyA, keyB, keyF
    finally:
        L.tune_cache_file(None)
        L.tune_cache_clear()
    assert L.tune_cache_count() == 0
