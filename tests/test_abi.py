"""C-ABI boundary on the CPU: exports, header, validation, host-only helpers.

No device work is launched here.
"""
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import spin1 as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spin1.h")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SPIN1_API\s+[\w\s\*]+?\b(spin1_\w+)\s*\(", text)))


def test_header_declares_binding_functions(abi):
    assert header_functions() == sorted(abi.FUNCTIONS)


def test_library_exports_every_declared_symbol(abi):
    lib = abi.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", abi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (spin1_\w+)", out))
    assert exported == set(header_functions())


def test_binding_constants_match_the_header(abi):
    """Every enum value of the header (status codes, dtypes, options and their
    values, kernel kinds) has the same value in the binding."""
    consts = re.findall(r"\bSPIN1_([A-Z0-9_]+) = (-?\d+)", open(HEADER).read())
    assert len(consts) >= 30
    for name, value in consts:
        if name.startswith("K_"):
            if name == "K_COUNT":
                assert len(abi.KERNEL_KINDS) == int(value)
            else:
                assert abi.KERNEL_KINDS[int(value)] == name[2:].lower(), name
        else:
            assert getattr(abi, name) == int(value), name


def test_header_compiles_as_c99(tmp_path):
    src = tmp_path / "h.c"
    src.write_text('#include "spin1.h"\nint main(void){ spin1_grid g = {1, {8, 1, 1}, 0.5, 1}; (void)g; return 0; }\n')
    res = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-fsyntax-only",
                          "-I" + os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr


@pytest.mark.parametrize("grid,code,msg", [
    ((0, (8,), 0.5, 1), -1, "dim"),
    ((4, (8,), 0.5, 1), -1, "dim"),
    ((1, (12,), 0.5, 1), -1, "power of two"),
    ((1, (4,), 0.5, 1), -1, "minimum"),
    ((1, (8192,), 0.5, 1), -2, "4096"),
    ((2, (8, 8), 0.5, 1), -2, "Nx"),
    ((2, (64, 2048), 0.5, 1), -2, "1024"),
    ((1, (64,), 0.0, 1), -1, "dx"),
    ((1, (64,), float("nan"), 1), -1, "dx"),
    ((1, (64,), 0.5, 0), -1, "samples"),
    ((1, (64, 2), 0.5, 1), -1, "n[1]"),
])
def test_invalid_grids_rejected(abi, grid, code, msg):
    g = abi.make_grid(*grid)
    with pytest.raises(abi.Spin1Error) as ei:
        abi.check_grid(g, abi.C64)
    assert ei.value.code == code
    assert msg in str(ei.value)
    assert abi.load().spin1_field_bytes(g, abi.C64) == 0


def test_invalid_dtype_rejected(abi):
    g = abi.make_grid(1, (64,), 0.5, 1)
    with pytest.raises(abi.Spin1Error) as ei:
        abi.check_grid(g, 7)
    assert ei.value.code == abi.EINVAL


def test_null_context_calls_fail_cleanly(abi):
    lib = abi.load()
    assert lib.spin1_step(None, 1, 0.01) == abi.EINVAL
    assert "NULL" in abi.last_error()
    assert lib.spin1_destroy(None) == abi.EINVAL
    assert lib.spin1_structure_factor(None, 0, None) == abi.EINVAL
    assert lib.spin1_observables(None, 0, None) == abi.EINVAL
    assert lib.spin1_set_params(None, None) == abi.EINVAL
    assert lib.spin1_init_wigner_shard(None, 1, None, 0, None, None, None, None) == abi.EINVAL
    assert lib.spin1_local_update(None, 0.1) == abi.EINVAL
    assert lib.spin1_set_option(None, 0, 1) == abi.EINVAL
    assert lib.spin1_profile_enable(None, 1) == abi.EINVAL
    assert lib.spin1_set_potential(None, 0, None) == abi.EINVAL
    assert lib.spin1_sync_field(None) == abi.EINVAL
    assert lib.spin1_step_observed(None, 1, 0.01, 0, None) == abi.EINVAL
    assert lib.spin1_transverse_spin(None, 0, None) == abi.EINVAL
    assert lib.spin1_spin_texture(None, 0, None) == abi.EINVAL


def test_sizes(abi):
    g = abi.make_grid(2, (512, 512), 0.5, 64)
    assert abi.field_bytes(g, abi.C64) == 64 * 3 * 512 * 512 * 8
    assert abi.field_bytes(g, abi.C128) == 64 * 3 * 512 * 512 * 16
    ws1 = abi.workspace_bytes([g], abi.C64)
    assert ws1 > 64 * 512 * 512 * 12  # spectrum field + power
    g2 = abi.make_grid(1, (4096,), 0.5, 128)
    assert abi.workspace_bytes([g, g2], abi.C64) > ws1


@pytest.mark.parametrize("dim,n", [(1, (256,)), (1, (4096,)), (2, (256, 256)), (2, (512, 512)),
                                   (2, (64, 16)), (3, (16, 8, 32)), (3, (32, 32, 32))])
def test_shell_tables_match_oracle(abi, dim, n):
    g = abi.make_grid(dim, n, 0.5, 1)
    og = O.Grid(dim, n, 0.5, 1)
    assert abi.num_bins(g) == O.num_bins(og)
    assert np.array_equal(abi.bin_counts(g), O.bin_counts(og))


def test_shell_count_of_3d_256(abi):
    assert abi.num_bins(abi.make_grid(3, (256, 256, 256), 0.5, 1)) == 223
