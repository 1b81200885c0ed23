"""Build the HIP library in-tree with hipcc for gfx950.

    python -m paper_2507_02164_amd.build

produces ``paper_2507_02164_amd/libproots.so`` from ``csrc/*.hip``, and
``kernel_isa.json``: for every solve kernel, a SHA-256 of its gfx950
instructions (from a device-only assembly compile of ``solve.hip`` with the
same flags, run beside the library build).  A measurement taken on one build
can so be matched to the kernel code it describes.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libproots.so")
ISA_DIGESTS = os.path.join(HERE, "kernel_isa.json")

ARCH = "gfx950"

# Packed FP32 instructions are switched off: the compiler would otherwise
# form them from ordinary float code, and some of their forms have returned
# wrong results on the target machines without any error.
HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def isa_digests(asm_text: str) -> dict:
    """{kernel symbol: SHA-256 of its instruction lines} for every kernel in
    an AMDGPU assembly listing (comments, labels and directives dropped).
    Branch targets name basic blocks as .LBB<function>_<block>; the function
    number depends on how many functions precede the kernel in the file, so
    it is dropped and an unchanged kernel keeps its digest."""
    import hashlib
    import re
    block = re.compile(r"\.LBB\d+_")
    out = {}
    name, body = None, []
    for line in asm_text.split("\n"):
        if name is None:
            if line.startswith("_Z") and line.split(";")[0].rstrip().endswith(":"):
                name, body = line.split(":")[0], []
            continue
        ins = block.sub(".LBB_", line.split(";")[0].strip())
        if ins and not ins.startswith(".") and not ins.endswith(":"):
            body.append(ins)
        if ins.startswith("s_endpgm"):
            out[name] = hashlib.sha256("\n".join(body).encode()).hexdigest()
            name = None
    return out


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile every HIP source into libproots.so (always recompiles), and
    record the solve kernels' instruction digests."""
    import json
    import tempfile
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, *extra_flags, "-I", INCLUDE, *sources(), "-o", tmp]
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    t0 = time.time()
    with tempfile.TemporaryDirectory() as td:
        asm = os.path.join(td, "solve.s")
        asm_cmd = [hipcc(), *flags, *extra_flags, "--cuda-device-only", "-S", "-I", INCLUDE,
                   os.path.join(CSRC, "solve.hip"), "-o", asm]
        lib_proc = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
        asm_proc = subprocess.Popen(asm_cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                    text=True)
        out, err = lib_proc.communicate()
        aout, aerr = asm_proc.communicate()
        if lib_proc.returncode != 0:
            sys.stderr.write(out + err)
            raise RuntimeError("hipcc failed building libproots.so")
        if asm_proc.returncode != 0:
            sys.stderr.write(aout + aerr)
            raise RuntimeError("hipcc failed producing the solve kernels' assembly")
        digests = isa_digests(open(asm).read())
    os.replace(tmp, LIB)
    with open(ISA_DIGESTS + ".tmp", "w") as f:
        json.dump(digests, f, indent=1, sort_keys=True)
    os.replace(ISA_DIGESTS + ".tmp", ISA_DIGESTS)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s ({len(digests)} solve kernel digests)")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
