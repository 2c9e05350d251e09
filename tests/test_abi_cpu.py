"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function declared in include/rmg.h, and its struct layouts match the binding;
the host KL set-up agrees with the oracle on rotation-invariant quantities."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "rmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|int64_t|char)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def _lib_path():
    from paper_1903_08741_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("librmg.so not built (run __graft_entry__.build())")
    return _abi.LIB_PATH


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for fn in ("sample_fields", "picard_mg_solve", "mlmc_level_estimate", "rmg_ctx_create",
               "rmg_ctx_destroy", "rmg_last_error", "rmg_struct_size"):
        assert fn in names, names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    for fn in _declared_functions():
        assert hasattr(lib, fn), f"{fn} declared in rmg.h but not exported"


def test_struct_layouts_match_binding():
    from paper_1903_08741_amd import _abi
    _lib_path()
    L = _abi.lib()
    for name, cls in _abi.STRUCTS.items():
        assert L.rmg_struct_size(name.encode()) == ctypes.sizeof(cls), name
    assert L.rmg_struct_size(b"nonsense") == -1


def test_null_context_is_rejected():
    from paper_1903_08741_amd import _abi
    _lib_path()
    L = _abi.lib()
    assert L.sample_fields(None, 16, 1, 8, None, None, None, 1, None, None) == _abi.RMG_EINVAL
    assert L.rmg_ctx_create(None, 0, None) == _abi.RMG_EINVAL


def test_host_kl_setup_matches_oracle():
    """Independent host set-up vs oracle: eigenvalues, and - with both bases made
    canonical inside degenerate eigenspaces - the tables themselves."""
    from oracle import kl as okl
    from paper_1903_08741_amd import kl_setup
    lam_o, Bo = okl.basis(1.0, 0.3, 24, [8, 16], ref_n=32)
    lam_p, Bp = kl_setup.kl_tables(1.0, 0.3, 24, [8, 16], ref=32)
    # compare only complete eigenspaces (a truncation may split a degenerate pair)
    gaps = np.where(np.diff(lam_o) < -1e-8 * lam_o[0])[0]
    M = gaps[-1] + 1
    np.testing.assert_allclose(lam_p[:M], lam_o[:M], rtol=1e-12)
    for n in (8, 16):
        assert np.max(np.abs(Bo[n][:M] - Bp[n][:M])) < 1e-10 * np.max(np.abs(Bo[n]))
