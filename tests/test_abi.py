"""Host-only checks of the C interface: the library loads, exports every entry
point the header declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2412_19207_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rann_dd.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2412_19207_amd import build
        build.build()
    return binding.load()


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"RANN_API\s+[\w\s\*]*?\b(rann_dd_\w+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ["rann_dd_assemble", "rann_dd_pca", "rann_dd_solve", "rann_dd_solve_backward"]:
        assert required in names


def test_header_declares_every_exported_entry_point():
    """Every declaration in the header is matched, whatever its return type."""
    txt = open(HEADER).read()
    n_decl = len(re.findall(r"RANN_API\s", txt)) - 1  # minus the macro definition
    assert len(declared_symbols()) == n_decl
    assert "rann_dd_trim_cache" in declared_symbols()


def test_header_compiles_as_c(tmp_path):
    """The header is a self-contained C99 header (plain C callers include it)."""
    src = tmp_path / "use_header.c"
    src.write_text('#include "rann_dd.h"\nint main(void) { rann_dd_stats s; (void)s; return 0; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.dirname(HEADER),
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name
        assert name in binding._SIGS, f"binding lacks {name}"


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals the C
    compiler's for the header (a program built here prints them)."""
    structs = {"rann_dd_desc": binding.Desc, "rann_dd_solve_opts": binding.SolveOpts,
               "rann_dd_stats": binding.Stats, "rann_dd_tuning": binding.Tuning, "rann_dd_info": binding.Info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rann_dd.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def _valid_desc(keep):
    d = binding.Desc()
    d.d = 2
    d.l[0], d.l[1], d.l[2], d.l[3] = 2, 2, 1, 1
    mu = np.array([0.25, 0.75, 0.25, 0.75])
    m = np.array([4, 4, 4, 4], dtype=np.int32)
    keep += [mu, m]
    d.mu = mu.ctypes.data_as(binding.c_dp)
    d.m = m.ctypes.data_as(binding.c_ip)
    d.sigma[0] = d.sigma[1] = 0.3
    d.sigma[2] = d.sigma[3] = 1.0
    # host addresses stand in for device pointers: validation rejects before any use
    fake = np.zeros(64)
    keep.append(fake)
    ptr = fake.ctypes.data
    d.R = d.b = d.X_int = d.a = d.beta = d.c = ptr
    d.n_int = 4
    d.n_bnd = 0
    d.lambda_B = 1.0
    d.precision = binding.FP64
    d.stencil = 2
    d.precond = 1
    return d


@pytest.mark.parametrize("field,value", [
    ("d", 0), ("d", 5), ("lambda_B", -1.0), ("lambda_B", float("nan")), ("precision", 7),
    ("stencil", 9), ("precond", -2), ("n_int", 0), ("n_inner", 4), ("n_inner", -1),
])
def test_invalid_descriptor_is_rejected(lib, field, value):
    keep = []
    d = _valid_desc(keep)
    setattr(d, field, value)
    h = ctypes.c_void_p()
    rc = lib.rann_dd_assemble(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == binding.RANN_EINVAL
    assert not h.value
    assert len(binding.rann_dd_last_error()) > 0


@pytest.mark.parametrize("case", ["width0", "width65", "no_weights"])
def test_invalid_inner_layers_are_rejected(lib, case):
    keep = []
    d = _valid_desc(keep)
    d.n_inner = 2
    d.inner_w[0], d.inner_w[1] = 8, {"width0": 0, "width65": 65, "no_weights": 8}[case]
    fake = np.zeros(8)
    keep.append(fake)
    if case != "no_weights":
        d.R_inner = d.b_inner = fake.ctypes.data
    h = ctypes.c_void_p()
    rc = lib.rann_dd_assemble(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == binding.RANN_EINVAL
    assert not h.value


def test_non_increasing_centres_rejected(lib):
    keep = []
    d = _valid_desc(keep)
    mu = np.array([0.75, 0.25, 0.25, 0.75])
    keep.append(mu)
    d.mu = mu.ctypes.data_as(binding.c_dp)
    h = ctypes.c_void_p()
    assert lib.rann_dd_assemble(ctypes.byref(d), None, ctypes.byref(h)) == binding.RANN_EINVAL


def test_bad_width_rejected(lib):
    keep = []
    d = _valid_desc(keep)
    m = np.array([4, 0, 4, 4], dtype=np.int32)
    keep.append(m)
    d.m = m.ctypes.data_as(binding.c_ip)
    h = ctypes.c_void_p()
    assert lib.rann_dd_assemble(ctypes.byref(d), None, ctypes.byref(h)) == binding.RANN_EINVAL


def test_null_handle_calls_fail_cleanly(lib):
    opts = binding.SolveOpts(tol=1e-8, maxiter=10, method=0, restart=10, check_every=1)
    assert lib.rann_dd_solve(None, None, 1, None, ctypes.byref(opts), None, None) == binding.RANN_EINVAL
    assert lib.rann_dd_pca(None, 1e-8, 0, None, None, None) == binding.RANN_EINVAL
    assert lib.rann_dd_get_info(None, None) == binding.RANN_EINVAL
    lib.rann_dd_destroy(None)


def test_product_path_has_no_oracle_dependency():
    """The binding, the build script and the kernels must not import or name the oracle."""
    pkg = os.path.join(ROOT, "paper_2412_19207_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
