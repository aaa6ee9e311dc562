"""Builds the host emulation of the library (test infrastructure): copies the
HIP sources with the rewrites the emulation needs (launch syntax, dynamic
LDS, AMDGCN builtins) and compiles them for the CPU with AddressSanitizer."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2408_14193_amd", "csrc")
CXX = os.environ.get("HOSTEMU_CXX", "/opt/rocm/llvm/bin/clang++")


def _fix_launches(s: str) -> str:
    """kernel<<<grid, block, lds, stream>>>(args) -> emu::launch(kernel, grid, block, lds, stream)(args)."""
    out, i = [], 0
    while True:
        j = s.find("<<<", i)
        if j < 0:
            out.append(s[i:])
            return "".join(out)
        k, depth = j, 0
        while k > 0:
            ch = s[k - 1]
            if ch == ">":
                depth += 1
            elif ch == "<":
                if depth == 0:
                    break
                depth -= 1
            elif depth == 0 and not (ch.isalnum() or ch in "_:"):
                break
            k -= 1
        e = s.find(">>>", j)
        out.append(s[i:k])
        out.append("emu::launch(" + s[k:j] + ", " + s[j + 3:e] + ")")
        i = e + 3


def build(out_dir: str) -> str:
    src = os.path.join(out_dir, "src")
    if os.path.exists(src):
        shutil.rmtree(src)
    os.makedirs(os.path.join(src, "paper_2408_14193_amd", "csrc"))
    os.makedirs(os.path.join(src, "include"))
    shutil.copy(os.path.join(ROOT, "include", "spalu.h"), os.path.join(src, "include", "spalu.h"))
    for fn in os.listdir(CSRC):
        s = open(os.path.join(CSRC, fn)).read()
        s = s.replace("extern __shared__ double lds[];", "double* lds = (double*)emu::dyn_smem();")
        s = s.replace("extern __shared__ __align__(16) char smem[];", "char* smem = (char*)emu::dyn_smem();")
        s = s.replace("__builtin_amdgcn_", "emu_amdgcn_")
        if fn.endswith(".hip"):
            s = _fix_launches(s)
            fn = fn[:-4] + ".cpp"
        open(os.path.join(src, "paper_2408_14193_amd", "csrc", fn), "w").write(s)
    flags = ["-std=c++20", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address",
             "-I", HERE, "-I", os.path.join(src, "include"), "-Wno-unused-result", "-Wno-deprecated-declarations"]
    objs = []
    units = [os.path.join(HERE, "emu.cpp"), os.path.join(src, "paper_2408_14193_amd", "csrc", "spalu.cpp"),
             os.path.join(src, "paper_2408_14193_amd", "csrc", "planner.cpp"), os.path.join(HERE, "driver.cpp")]
    procs = []
    for u in units:
        o = os.path.join(out_dir, os.path.basename(u) + ".o")
        procs.append(subprocess.Popen([CXX, *flags, "-c", u, "-o", o]))
        objs.append(o)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("host emulation build failed")
    exe = os.path.join(out_dir, "hostemu_run")
    subprocess.run([CXX, *flags, *objs, "-o", exe], check=True)
    return exe
