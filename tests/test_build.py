"""Build-level checks that need no GPU: the library exports every entry point declared in
include/*.h, and no kernel keeps data in scratch (private) memory."""
import concurrent.futures as cf
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_07154_amd", "csrc")


def declared_functions():
    names = set()
    for h in ("mf.h", "mf_ops.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"\b(mf_[a-z_0-9]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_entry_point():
    lib = os.path.join(ROOT, "paper_2601_07154_amd", "libmfocus.so")
    if not os.path.exists(lib):
        from paper_2601_07154_amd import build
        build.build(verbose=False)
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (mf_[a-z_0-9]+)", out))
    missing = declared_functions() - exported
    assert not missing, missing
    from paper_2601_07154_amd import _lib
    _lib.bind(lib)          # every prototype of the binding resolves


def _resources(src):
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-c",
           os.path.join(CSRC, src), "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", r.stderr)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    return list(zip(names, scratch))


def test_no_kernel_uses_scratch_memory():
    srcs = [f for f in os.listdir(CSRC) if f.endswith(".hip")]
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        res = [kv for part in ex.map(_resources, srcs) for kv in part]
    assert res
    bad = [(n, s) for n, s in res if s]
    assert not bad, bad
