"""Build libcpcrit.so (HIP, gfx950) in-tree with hipcc.

Every library source under csrc/ is compiled to an object in _build/ (in
parallel), then linked into paper_2407_18015_amd/libcpcrit.so; the
benchmark's measurement probes (csrc/cp_probes.hip: the Monte Carlo, FP32
and HBM ceilings) go to libcpprobes.so beside it.  Packed FP32 instructions
are disabled for all device code.  The device assembly of the closed-form
kernels is also emitted, and a SHA-256 of each kernel's instructions is
written to libcpcrit.isa.json: measurements taken on a kernel (hardware
counters) can then be tied to the exact machine code they describe.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os
import re
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcpcrit.so")
PROBES_LIB = os.path.join(HERE, "libcpprobes.so")
PROBE_SOURCES = ["cp_probes.hip"]
ISA_JSON = os.path.join(HERE, "libcpcrit.isa.json")
ISA_SOURCES = ["cp_closed_form.hip"]
ARCH = os.environ.get("CPCRIT_ARCH", "gfx950")

SOURCES = ["cp_api.cpp", "cp_closed_form.hip", "cp_fit.hip", "cp_fit_forward.hip", "cp_mvg.hip", "cp_batched.hip", "cp_classify.hip", "cp_semi.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-xhip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    return obj


def _isa(src: str) -> dict:
    """Device assembly of one source; {kernel symbol: sha256 of its instructions}."""
    asm = os.path.join(BUILD, os.path.splitext(src)[0] + ".s")
    cmd = [_hipcc(), *COMMON, "--offload-device-only", "-S", os.path.join(CSRC, src), "-o", asm]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc -S failed on {src}:\n{r.stderr[-6000:]}")
    text = open(asm).read()
    out = {}
    for m in re.finditer(r"^(_Z\w+):", text, flags=re.M):
        name = m.group(1)
        end = text.find(".Lfunc_end", m.end())
        body = text[m.end():end if end > 0 else len(text)]
        lines = [ln.split(";")[0].strip() for ln in body.splitlines()]
        # branch labels carry the function's index in the file: keep the local part
        code = "\n".join(re.sub(r"\.LBB\d+_(\d+)", r".LBB_\1", ln) for ln in lines
                         if ln and not ln.startswith("."))
        out[name] = hashlib.sha256(code.encode()).hexdigest()
    return out


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES) + len(ISA_SOURCES) + len(PROBE_SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        isa = [ex.submit(_isa, s) for s in ISA_SOURCES]
        probes = [ex.submit(_compile, s) for s in PROBE_SOURCES]
        objs = list(ex.map(_compile, SOURCES))
        hashes = {}
        for fut in isa:
            hashes.update(fut.result())
        probe_objs = [fut.result() for fut in probes]
    with open(ISA_JSON, "w") as fh:
        json.dump(hashes, fh, indent=1, sort_keys=True)
    _link(objs, LIB)
    _link(probe_objs, PROBES_LIB)
    return LIB


def _link(objs, out):
    tmp = out + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link of {os.path.basename(out)} failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, out)


if __name__ == "__main__":
    print(build())
