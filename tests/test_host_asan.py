"""The library's host code under AddressSanitizer.

The sources are rebuilt with the sanitizer on the host pass only (device code
is not instrumented, and nothing here touches a GPU) into a temporary
directory, and the host-only interface checks of test_abi.py run in a child
Python process with the sanitizer runtime preloaded and that build loaded in
place of the in-tree library: descriptor validation, null handles, error
text, symbol exports and struct layouts.  A heap or stack error in those paths
aborts the child with the sanitizer's report."""
import concurrent.futures
import glob
import os
import subprocess
import sys

import pytest

from paper_2412_19207_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
# host pass only: each sanitizer flag right after -Xarch_host
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]

CHILD = r"""
import ctypes, os, sys
os.environ.pop("LD_PRELOAD", None)  # the runtime is loaded; keep it out of subprocesses
assert hasattr(ctypes.CDLL(None), "__asan_init"), "sanitizer runtime not loaded"
sys.path.insert(0, {root!r})
from paper_2412_19207_amd import binding
lib = binding.load({lib!r})
print("instrumented library:", {lib!r})
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "-m", "not gpu", {test!r}]))
"""


def _build(outdir):
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + ASAN_FLAGS

    def comp(src):
        obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
        r = subprocess.run([B.HIPCC, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(comp, B.SOURCES))
    lib = os.path.join(outdir, "librann_dd_asan.so")
    r = subprocess.run([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *ASAN_FLAGS, "-o", lib, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    return lib


@pytest.mark.skipif(not ASAN_RT or not os.path.exists(B.HIPCC), reason="no hipcc or sanitizer runtime")
def test_host_interface_checks_under_address_sanitizer(tmp_path):
    lib = _build(str(tmp_path))
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_" in syms, "the host pass is not instrumented"
    env = dict(os.environ)
    env["LD_PRELOAD"] = ASAN_RT[-1]
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1"
    code = CHILD.format(root=ROOT, lib=lib, test=os.path.join(ROOT, "tests", "test_abi.py"))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "instrumented library" in r.stdout and "passed" in r.stdout, r.stdout[-2000:]
