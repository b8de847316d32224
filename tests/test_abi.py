"""The C-ABI library loads and exports every function include/lrsdp.h declares (no GPU)."""

import ctypes
import os

import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1703_10973_amd", "liblrsdp.so")


@pytest.fixture(scope="module")
def binding():
    if not os.path.exists(LIB):
        pytest.fail("liblrsdp.so is not built: run python -m paper_1703_10973_amd.build")
    import paper_1703_10973_amd as pk
    return pk


def test_every_header_symbol_is_exported(binding):
    names = binding.header_symbols()
    assert len(names) >= 16
    h = ctypes.CDLL(LIB)
    for nm in names:
        assert hasattr(h, nm), f"{nm} declared in include/lrsdp.h but not exported"


def test_binding_covers_the_header(binding):
    from paper_1703_10973_amd import _lib
    assert set(binding.header_symbols()) == set(_lib._SIGS)


def test_defaults_and_status_strings(binding):
    o = binding.lrsdp_opts_default()
    assert o.eps == 1e-8 and o.max_iter == 200 and o.deflate == 1 and o.dd_mode == 2
    assert binding.status_string(0) == "OK"
    assert binding.status_string(-2) == "DUPLICATE_PAIR"
    assert binding.status_string(-99) == "UNKNOWN"


def test_context_needs_a_device(binding):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(binding.LrsdpError):
        binding.lrsdp_ctx_create(0)


def test_argument_sizes_are_checked_before_any_call(binding):
    """A short or long array is refused by the binding before it reaches the library (a
    kernel would otherwise read or write past the allocation)."""
    import torch
    from paper_1703_10973_amd import _lib
    with pytest.raises(ValueError):
        _lib._ptr(torch.zeros(5, dtype=torch.float64), torch.float64, 6, "v")
    with pytest.raises(ValueError):
        _lib._ptr(torch.zeros(7, dtype=torch.float64), torch.float64, 6, "v")
    with pytest.raises(TypeError):
        _lib._ptr(torch.zeros(6, dtype=torch.float32), torch.float64, 6, "v")
    with pytest.raises(TypeError):      # right size and type, but host memory
        _lib._ptr(torch.zeros(6, dtype=torch.float64), torch.float64, 6, "v")


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding mirrors with ctypes has the header's size and field offsets
    (a C program built with gcc against include/lrsdp.h prints them)."""
    import shutil
    import subprocess
    from paper_1703_10973_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    root = os.path.dirname(os.path.dirname(__file__))
    structs = [_lib.lrsdp_opts, _lib.lrsdp_info, _lib.lrsdp_ipm_opts, _lib.lrsdp_ipm_info,
               _lib.lrsdp_ipm_record, _lib.lrsdp_instance]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lrsdp.h"', "int main(void) {"]
    want = []
    for st in structs:
        nm = st.__name__
        lines.append(f'  printf("%zu\\n", sizeof({nm}));')
        want.append(ctypes.sizeof(st))
        for field, _ in st._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({nm}, {field}));')
            want.append(getattr(st, field).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == want
