"""Build step of the HIP library: compiles ``csrc/*.hip`` for gfx950 into
``libhbheap.so`` next to this file (in-tree, so it travels with the tree)."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhbheap.so")
SOURCES = ["csrc/hbheap.hip", "csrc/growth.hip", "csrc/serve.hip", "csrc/plain_baseline.hip",
           "csrc/host_malloc_baseline.cpp"]
# the test build with schedule fuzzing: the allocator's translation unit only
FUZZ_LIB = os.path.join(HERE, "libhbheap_fuzz.so")
FUZZ_SOURCES = ["csrc/hbheap.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libhbheap.so)")


FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 ops off: the allocator has no fp32 arithmetic, and this
    # keeps the compiler from emitting v_pk_*_f32 anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no wave-level rewriting of atomics: the library issues each queue-word
    # atomic from one lane already, and the rewrite (a loop over the active
    # lanes around every such atomic) only adds instructions
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-I", os.path.join(ROOT, "include"),
]
OBJ_DIR = os.path.join(ROOT, "_build")


def compile_command(src: str, obj: str, defines: tuple = ()) -> list[str]:
    return [hipcc()] + FLAGS + [f"-D{d}" for d in defines] + ["-c", "-o", obj, os.path.join(HERE, src)]


def link_command(objs: list[str], out: str) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", out] + objs


def _run(cmd: list[str], verbose: bool):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stderr}")


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one hipcc each) and link the shared
    library and its schedule-fuzzing test build; it always recompiles."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(os.path.basename(s))[0] + ".o") for s in SOURCES]
    fobjs = [os.path.join(OBJ_DIR, os.path.basename(s).replace(".hip", "_fuzz.o")) for s in FUZZ_SOURCES]
    jobs = [compile_command(s, o) for s, o in zip(SOURCES, objs)]
    jobs += [compile_command(s, o, ("HBHEAP_FUZZ=1",)) for s, o in zip(FUZZ_SOURCES, fobjs)]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, cmd, verbose) for cmd in jobs]:
            f.result()
    for out, o in ((LIB, objs), (FUZZ_LIB, fobjs)):
        tmp = out + ".tmp"
        _run(link_command(o, tmp), verbose)
        os.replace(tmp, out)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
