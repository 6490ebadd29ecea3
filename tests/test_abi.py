"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/fno_mi355x.h declares, and validates descriptors on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fno_mi355x.h")


@pytest.fixture(scope="module")
def fno():
    from paper_2211_12709_amd import fno as f
    if not os.path.exists(f.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    f.load_library()
    return f


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fno_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for n in ("fno_spectral_fwd", "fno_spectral_bwd", "fno_block_fwd", "fno_block_bwd"):
        assert n in names


def test_every_declared_symbol_is_exported(fno):
    lib = ctypes.CDLL(fno.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in the header but not exported"
    assert set(declared_functions()) == set(fno.EXPORTS)


def test_status_strings(fno):
    for code in range(7):
        s = fno.status_str(code)
        assert s.startswith("FNO_")
    assert "unknown" in fno.status_str(99)


CONFIGS = {
    "single_layer_16^3x8": (1, 8, 8, (16, 16, 16, 8), (4, 4, 4, 4)),
    "ns_64^3x16": (1, 20, 20, (64, 64, 64, 16), (12, 12, 12, 8)),
    "co2_128^3x32": (1, 20, 20, (128, 128, 128, 32), (16, 16, 16, 8)),
    "co2_batched_128^3x32": (4, 32, 32, (128, 128, 128, 32), (20, 20, 20, 10)),
    "odd": (2, 3, 5, (12, 10, 9, 7), (3, 2, 4, 4)),
    "full_retention_nyquist": (1, 4, 6, (8, 6, 10, 16), (4, 3, 5, 9)),
}


@pytest.mark.parametrize("name", sorted(CONFIGS))
@pytest.mark.parametrize("dtype", [0, 1])
def test_valid_descriptors(fno, name, dtype):
    B, ci, co, grid, modes = CONFIGS[name]
    assert fno.validate(fno.make_desc(B, ci, co, grid, modes, dtype)) == fno.FNO_OK


@pytest.mark.parametrize("bad,code", [
    (dict(B=0), 1), (dict(C_in=0), 1), (dict(C_out=-1), 1),
    (dict(grid=(16, 16, 0, 8)), 1), (dict(modes=(0, 4, 4, 4)), 1),
    (dict(modes=(9, 4, 4, 4)), 1),            # 2 m_x > N_x
    (dict(modes=(4, 4, 4, 6)), 1),            # m_t > N_t/2 + 1
    (dict(dtype=7), 2), (dict(flags=2), 2),  # an unknown flag
    (dict(C_in=65), 2),                       # beyond the library's channel limit
    (dict(B=9, flags=1), 2),                  # packed FP8 weights: the tiled mix holds at most 8 batch elements
])
def test_invalid_descriptors(fno, bad, code):
    args = dict(B=1, C_in=8, C_out=8, grid=(16, 16, 16, 8), modes=(4, 4, 4, 4), dtype=0, flags=0)
    args.update(bad)
    d = fno.make_desc(args["B"], args["C_in"], args["C_out"], args["grid"], args["modes"], args["dtype"], args["flags"])
    assert fno.validate(d) == code


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_fp8_weight_flag_accepted(fno, name):
    B, ci, co, grid, modes = CONFIGS[name]
    assert fno.validate(fno.make_desc(B, ci, co, grid, modes, 1, fno.FNO_W_FP8)) == fno.FNO_OK


def test_null_descriptor_and_plan_arguments(fno):
    lib = fno.load_library()
    assert lib.fno_desc_validate(None) == fno.FNO_ERR_INVALID_ARG
    assert lib.fno_plan_destroy(None) == fno.FNO_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert lib.fno_workspace_bytes(None, 0, ctypes.byref(n)) == fno.FNO_ERR_INVALID_ARG
    assert lib.fno_cache_bytes(None, ctypes.byref(n)) == fno.FNO_ERR_INVALID_ARG
    assert lib.fno_spectral_fwd(None, None, None, None, None, None, 0, None) == fno.FNO_ERR_INVALID_ARG


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2211_12709_amd")
    pat = re.compile(r"(^\s*(from|import)\s+oracle\b)|libfno_oracle|fno_oracle", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not pat.search(src), f"{f} references the oracle"
