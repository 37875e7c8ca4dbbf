"""Build step for the HIP library: compiles csrc/*.hip for gfx950 into
libddilu.so next to this file (in-tree, so the built library travels with
the source tree)."""

import glob
import os
import subprocess
import sys
import tempfile

try:
    from . import asmcheck
except ImportError:  # run as a script
    import asmcheck

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddilu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


# Sources whose device assembly is checked after compilation (their kernels
# schedule loads by hand; see asmcheck.py).
CHECKED = ("apply.hip",)


def build(verbose: bool = False) -> str:
    objs = []
    procs = []
    with tempfile.TemporaryDirectory(prefix="ddilu_build_") as tmp:
        for src in sources():
            name = os.path.basename(src)[:-4]
            obj = os.path.join(CSRC, name + ".o")
            cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
            if os.path.basename(src) in CHECKED:
                # keep the device assembly this object is made from
                obj = os.path.join(tmp, name + ".o")
                cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj, "-save-temps=obj"]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd, cwd=tmp), src))
            objs.append(obj)
        for p, src in procs:
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {src}")
        for name in CHECKED:
            asm = os.path.join(tmp, f"{name[:-4]}-hip-amdgcn-amd-amdhsa-gfx950.s")
            n = asmcheck.check_file(asm)
            if verbose:
                print(f"{name}: {n} slot kernels pass the in-flight register check", flush=True)
        _link(objs, verbose)
    build_rocsparse_ref(verbose)
    return LIB


# The vendor-library baseline (rocSPARSE block ILU0 + block triangular
# solves) used by bench.py --mode rocsparse and its parity test; a library of
# its own so that libddilu.so does not depend on rocSPARSE.
REF_SRC = os.path.join(HERE, "rocsparse_ref", "rocsparse_ilu0.cpp")
REF_LIB = os.path.join(HERE, "rocsparse_ref", "librocsparse_ref.so")


def build_rocsparse_ref(verbose: bool = False) -> str:
    out = REF_LIB + ".tmp"
    cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", REF_SRC, "-o", out,
           "-lrocsparse"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out, REF_LIB)
    return REF_LIB


def _link(objs, verbose):
    out = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out, LIB)
    for o in objs:
        os.remove(o)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
