"""The C-ABI boundary without a GPU: the library loads, exports every
function include/psdp.h declares, the Python structs match the C layout,
and host-side validation answers before any device call."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psdp.h")


@pytest.fixture(scope="module")
def lib():
    sys.path.insert(0, ROOT)
    from paper_1912_02767_amd import _abi, build
    if not os.path.exists(_abi.LIB_PATH):
        build.build()
    return _abi.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psdp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("psdp_create", "psdp_project", "psdp_project_batched", "psdp_full_eig_project"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1912_02767_amd import _abi
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (psdp_\w+)", out))
    assert set(declared_functions()) <= exported
    assert set(_abi.EXPORTED) <= exported


def _c_layout(tmp_path, struct, fields):
    src = tmp_path / "layout.c"
    body = "\n".join(f'printf("{f} %zu\\n", offsetof({struct}, {f}));' for f in fields)
    src.write_text(f"""
#include <stddef.h>
#include <stdio.h>
#include "psdp.h"
int main(void) {{ printf("size %zu\\n", sizeof({struct})); {body} return 0; }}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {k: int(v) for k, v in (ln.split() for ln in out.strip().splitlines())}


@pytest.mark.parametrize("name,cls", [("psdp_options", "Options"), ("psdp_info", "Info"),
                                      ("psdp_server_config", "ServerConfig"),
                                      ("psdp_result", "ServerResult"),
                                      ("psdp_server_stats", "ServerStats"),
                                      ("psdp_sdp", "Sdp"), ("psdp_admm_options", "AdmmOptions"),
                                      ("psdp_admm_info", "AdmmInfo")])
def test_struct_layout_matches_header(tmp_path, name, cls):
    sys.path.insert(0, ROOT)
    from paper_1912_02767_amd import _abi
    py = getattr(_abi, cls)
    fields = [f for f, _ in py._fields_]
    c = _c_layout(tmp_path, name, fields)
    assert c["size"] == ctypes.sizeof(py)
    for f in fields:
        assert c[f] == getattr(py, f).offset, f


def test_defaults_and_strings(lib):
    from paper_1912_02767_amd import _abi
    o = _abi.Options()
    lib.psdp_default_options(ctypes.byref(o))
    assert o.side == 0 and o.prec == 0 and o.max_iter > 0 and o.refine_fp64 == 1
    assert abs(o.side_threshold - 1.0 / 3.0) < 1e-15 and o.pos_hint == -1
    assert o.batch_variant == -1 and o.batch_graph == 1
    assert o.bound_rel_max == 0.0
    assert o.certify == 1 and o.certify_delta == 0.0 and o.warm_side == 0
    lib.psdp_status_str.restype = ctypes.c_char_p
    for code, name in [(0, b"PSDP_OK"), (1, b"PSDP_NOT_CONVERGED"), (-1, b"PSDP_ERR_INVALID_ARG"),
                       (-5, b"PSDP_ERR_CAPACITY")]:
        assert lib.psdp_status_str(code) == name
    lib.psdp_version.restype = ctypes.c_char_p
    assert lib.psdp_version()


def test_workspace_bytes_host_only(lib):
    b = ctypes.c_size_t()
    assert lib.psdp_workspace_bytes(1000, 24, 0, ctypes.byref(b)) == 0
    small = b.value
    assert small >= 8 * 1024 * 1024
    assert lib.psdp_workspace_bytes(4000, 48, 1, ctypes.byref(b)) == 0
    assert b.value > small
    assert lib.psdp_workspace_bytes(0, 24, 0, ctypes.byref(b)) == -1
    assert lib.psdp_workspace_bytes(100, 0, 0, ctypes.byref(b)) == -1
    assert lib.psdp_workspace_bytes(100, 8, 7, ctypes.byref(b)) == -1


def test_validation_before_any_launch(lib):
    from paper_1912_02767_amd import _abi
    m = ctypes.c_int(0)
    info = _abi.Info()
    # null handle: rejected on the host
    rc = lib.psdp_project(None, 10, None, 10, None, 10, 4, ctypes.byref(m), None, None, 10,
                          None, ctypes.byref(info))
    assert rc == -1
    assert lib.psdp_destroy(None) == -1
    assert lib.psdp_project_batched(None, 1, None, None, None, None, None, None, None, None,
                                    None) == -1
    ok = ctypes.c_int(7)
    assert lib.psdp_certify_tail(None, 10, None, 10, None, 10, 0, 1e-6, ctypes.byref(ok), None,
                                 None) == -1
    assert ok.value == 7
    assert lib.psdp_admm_solve(None, None, None, None, 1, None, None, 1, None) == -1


def test_create_without_gpu_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert lib.psdp_create(ctypes.byref(h), 0, None) == -2
    assert not h.value
