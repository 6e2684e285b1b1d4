"""CPU-side checks of the C ABI: the built library loads and exports every
function include/mlmix.h declares, and the ctypes structures match the
header's layout. No compute call is made (there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mlmix.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mlmix_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2502_19081_amd import binding as B
    lib = B.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in B.SIGNATURES, n


def test_struct_layouts():
    from paper_2502_19081_amd import binding as B
    assert ctypes.sizeof(B.Region) == 56
    assert ctypes.sizeof(B.Box) == 40
    assert ctypes.sizeof(B.FitConfig) == 80
    assert B.FitConfig.box.offset == 32 and B.FitConfig.rows.offset == 72


def test_fit_work_size_is_host_only_and_checks_sizes():
    from paper_2502_19081_amd import binding as B
    sz = ctypes.c_size_t()
    assert B.lib().mlmix_fit_work_size(120020, 81, ctypes.byref(sz)) == 0
    # G_H and b_H of the search, then the Gram partials (at most 512 chunks of
    # the upper-triangle 4x4 blocks plus the padded right-hand side)
    nb = (81 + 3) // 4
    per_part = (nb * (nb + 1) // 2 * 16 + nb * 4) * 8
    assert sz.value >= (81 * 81 + 81) * 8 + per_part
    assert sz.value <= (81 * 81 + 81) * 8 + 512 * per_part
    assert B.lib().mlmix_fit_work_size(10, 121, ctypes.byref(sz)) == -1
    assert B.lib().mlmix_fit_work_size(-1, 81, ctypes.byref(sz)) == -1
    assert B.ModelDesc.uf3_c3.offset == ctypes.sizeof(B.ModelDesc) - 8


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2502_19081_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower().replace("or_", ""), f


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import importlib
    from paper_2502_19081_amd import binding as B
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError):
        B.lib()


def test_library_gaunt_closed_form_matches_oracle_quadrature():
    # the library builds its real Gaunt table from the Wigner-3j closed form,
    # the oracle by product quadrature of its own harmonics: the two
    # constructions share nothing, so agreement pins both (to lmax 6, the
    # largest degree the library accepts)
    import numpy as np
    import oracle as O
    from paper_2502_19081_amd import binding as B
    lmax = 6
    L2 = (lmax + 1) ** 2
    G = np.zeros(L2 ** 3)
    assert B.lib().mlmix_gaunt_table(lmax, G.ctypes.data) == 0
    np.testing.assert_allclose(G.reshape(L2, L2, L2), O.gaunt_table(lmax), atol=1e-13)
    assert B.lib().mlmix_gaunt_table(7, G.ctypes.data) == -1
