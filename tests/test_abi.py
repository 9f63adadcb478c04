"""The C ABI library loads and exports every function that include/freeform.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "freeform.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_path():
    names = _declared()
    for n in ("build_neighbors", "rkpm_shape", "assemble_HM", "eigenmodes", "eigenmodes_batched"):
        assert n in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2605_29318_amd", "libfreeform.so")
    if not os.path.exists(path):
        from paper_2605_29318_amd import build
        build.build()
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2605_29318_amd import freeform
    for n in ("build_neighbors", "rkpm_shape", "assemble_HM", "eigenmodes", "eigenmodes_batched", "spmm_hm",
              "spmm_autotune", "rand_block", "philox4x32_10", "mlp_param_count", "mlp_inputs", "lumped_mass",
              "RowTiles", "spmm_variant_selected"):
        assert callable(getattr(freeform, n))
    # every declared entry point has a ctypes signature in the binding
    L = freeform.lib()
    unbound = [n for n in _declared() if getattr(L, n).argtypes is None]
    assert not unbound, unbound


def test_mlp_param_count_matches_reference_layout():
    from paper_2605_29318_amd import freeform
    from oracle import mlp
    for k in (1, 8, 16, 32, 64):
        for n_in in (11, 47, 128):
            assert freeform.mlp_param_count(k, n_in) == mlp.param_count(k, n_in)
    assert freeform.mlp_param_count(0) == -1 and freeform.mlp_param_count(65) == -1
    assert freeform.mlp_param_count(8, 129) == -1 and freeform.mlp_param_count(8, 0) == -1


def test_philox_reference_matches_published_vectors():
    """A CPU Philox written from the published definition reproduces the known answers."""
    from oracle.oracle import philox4x32_10
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(x, 16) for x in line.split()])
    for r in rows:
        assert philox4x32_10(r[0:4], r[4:6]) == r[6:10]
