"""The C-ABI library loads and exports every entry point include/fsl.h declares;
host-only calls (workspace sizing, argument validation) behave as documented.
No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fsl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsl_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1712_07028_amd as fsl

    if not os.path.exists(fsl.LIB_PATH):
        pytest.fail("libfsl.so is not built (run __graft_entry__.build())")
    return fsl.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "fsl_init" in names and "fsl_step" in names and "fsl_bubbles_get" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_all_exports():
    import paper_1712_07028_amd as fsl

    assert sorted(fsl.EXPORTS) == declared_functions()


def test_workspace_bytes_and_validation(lib):
    import paper_1712_07028_amd as fsl
    from paper_1712_07028_amd import workloads as W

    w = W.bubble_column_small()
    c = fsl.make_config(w)
    n1 = lib.fsl_workspace_bytes(ctypes.byref(c))
    # two FP32 lattices of 19 populations dominate the state
    assert n1 >= 2 * 19 * 4 * w.cells
    c.storage = 1
    n2 = lib.fsl_workspace_bytes(ctypes.byref(c))
    assert 2 * 19 * 2 * w.cells <= n2 < n1
    for field, bad in [("tau", 0.5), ("collision", 7), ("storage", 3), ("n_gas_spheres", 17)]:
        c = fsl.make_config(w)
        setattr(c, field, bad)
        assert lib.fsl_workspace_bytes(ctypes.byref(c)) == 0, field
    c = fsl.make_config(w)
    c.n[0] = 0
    assert lib.fsl_workspace_bytes(ctypes.byref(c)) == 0


def test_init_rejects_bad_arguments(lib):
    import paper_1712_07028_amd as fsl
    from paper_1712_07028_amd import workloads as W

    c = fsl.make_config(W.bubble_column_small())
    ctx = ctypes.c_void_p()
    # null workspace, then a misaligned one: rejected before any device work
    assert lib.fsl_init(ctypes.byref(c), None, 1 << 30, None, ctypes.byref(ctx)) == fsl.FSL_E_ARG
    assert lib.fsl_init(ctypes.byref(c), ctypes.c_void_p(0x1001), 1 << 40, None,
                        ctypes.byref(ctx)) == fsl.FSL_E_ARG
    assert lib.fsl_init(ctypes.byref(c), ctypes.c_void_p(0x1000), 16, None,
                        ctypes.byref(ctx)) == fsl.FSL_E_ARG
    assert not ctx.value
    assert lib.fsl_step(None, 1) == fsl.FSL_E_ARG
    assert lib.fsl_error_string(None) == b"null context"


def test_init_static_sizes_and_limit(lib):
    """fsl_init_static: the size query returns the state part of the workspace, and a
    configuration whose working memory exceeds the library's array is refused with
    a text that says so (both before any device work)."""
    import paper_1712_07028_amd as fsl
    from paper_1712_07028_amd import workloads as W

    c = fsl.make_config(W.bubble_column_small())
    nb = ctypes.c_size_t(0)
    assert lib.fsl_init_static(ctypes.byref(c), None, ctypes.byref(nb), None, None) == fsl.FSL_OK
    assert 0 < nb.value < lib.fsl_workspace_bytes(ctypes.byref(c))
    big = fsl.make_config(W.Workload(name="big", n=(1024, 1024, 256), trt=True, tau=0.6, g=(0, 0, -1e-5),
                                     zs=200.0, steps=0))
    assert lib.fsl_workspace_bytes(ctypes.byref(big)) > 0
    assert lib.fsl_init_static(ctypes.byref(big), None, ctypes.byref(nb), None, None) == fsl.FSL_E_ARG
    assert b"working memory" in lib.fsl_error_string(None)
    assert lib.fsl_init_static(ctypes.byref(c), None, None, None, None) == fsl.FSL_E_ARG
    ctx = ctypes.c_void_p()
    nb = ctypes.c_size_t(1 << 30)
    assert lib.fsl_init_static(ctypes.byref(c), ctypes.c_void_p(0x1001), ctypes.byref(nb), None,
                               ctypes.byref(ctx)) == fsl.FSL_E_ARG
    assert not ctx.value


@pytest.mark.parametrize("lib_name,header,expected", [
    ("libfsl_checks.so", "fsl_checks.h", ["fsl_check_cov_column", "fsl_check_split_block"]),
    ("libfsl_ceiling.so", "fsl_ceiling.h", ["fsl_ceiling_pull"]),
])
def test_helper_libraries_export_their_headers(lib_name, header, expected):
    """libfsl_checks.so (host builds of two kernel functions, for the exactness
    tests) and libfsl_ceiling.so (the benchmark's bandwidth ceiling) export what
    their headers declare."""
    path = os.path.join(ROOT, "paper_1712_07028_amd", lib_name)
    if not os.path.exists(path):
        pytest.fail(f"{lib_name} is not built (run __graft_entry__.build())")
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", header)).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(fsl_[a-z_]+)\s*\(", text)))
    assert names == expected
    L = ctypes.CDLL(path)
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("module,header,cname,pyname", [
    ("paper_1712_07028_amd", "include/fsl.h", "fsl_config", "FslConfig"),
    ("paper_1712_07028_amd", "include/fsl.h", "fsl_bubble", "FslBubble"),
    ("oracle", "oracle/fsl_oracle.h", "orc_config", "OrcConfig"),
    ("oracle", "oracle/fsl_oracle.h", "orc_bubble", "OrcBubble"),
])
def test_binding_structs_match_header_layout(tmp_path, module, header, cname, pyname):
    """The ctypes structures of the library's binding (and of the oracle's) have the
    size and the member offsets that a C compiler gives the header's structs (a
    member added on one side only, or in another order, would otherwise shift every
    later field without an error)."""
    import importlib
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    py = getattr(importlib.import_module(module), pyname)
    names = [f[0] for f in py._fields_]
    body = "\n".join(f'    printf("{n} %zu\\n", offsetof({cname}, {n}));' for n in names)
    src = tmp_path / "layout.c"
    src.write_text(f'#include <stddef.h>\n#include <stdint.h>\n#include <stdio.h>\n'
                   f'#include "{os.path.basename(header)}"\nint main(void) {{\n'
                   f'    printf("sizeof %zu\\n", sizeof({cname}));\n{body}\n    return 0;\n}}\n')
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, os.path.dirname(header))
    subprocess.run([cc, "-std=c99", "-I", inc, "-o", str(exe), str(src)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                         text=True).stdout.splitlines())
    assert int(out["sizeof"]) == ctypes.sizeof(py)
    for n in names:
        assert int(out[n]) == getattr(py, n).offset, n
