"""Build the gfx950 beamformer library ``libbf.so`` in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 code
generation disabled.  The per-precision kernel files compile in parallel."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbf.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["bf_api.cpp", "bf_host.cpp", "bf_weights.hip", "bf_pattern.hip", "bf_beamform_f32.hip", "bf_beamform_f16.hip",
           "bf_beamform_bf16.hip", "bf_beamform_f32_in4.hip", "bf_beamform_f16_in4.hip",
           "bf_beamform_bf16_in4.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA accumulators in VGPRs: the fused epilogue reads them with VALU
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", os.path.join(ROOT, "include")]


def _includes(path: str, seen=None) -> set:
    """Files a source includes with #include "...", recursively."""
    import re
    seen = set() if seen is None else seen
    with open(path) as f:
        text = f.read()
    for name in re.findall(r'#include\s+"([^"]+)"', text):
        dep = os.path.normpath(os.path.join(os.path.dirname(path), name))
        if os.path.exists(dep) and dep not in seen:
            seen.add(dep)
            _includes(dep, seen)
    return seen


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    path = os.path.join(CSRC, src)
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in {path} | _includes(path) | {__file__})


def _compile(src: str, verbose: bool, force: bool = True) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not force and not _stale(src, obj):
        return obj
    # the device assembly is kept next to the object (-save-temps=obj) for
    # the SrcC hazard check that follows the build
    cmd = [HIPCC] + FLAGS + ["-save-temps=obj", "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force=False: only those whose object is older
    than the source, a header it includes or this script) and link."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, force), SOURCES))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    check_hazards(verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


# Kernels whose built code must pass the SrcC hazard check (isa_check.py);
# the build fails if one of them does not.  Other kernels are reported.
ENFORCED = ("beamform_",)


def check_hazards(verbose: bool = False) -> dict:
    """Run the SrcC hazard check over the device assembly of this build;
    raise if an enforced kernel fails it.  Returns {kernel: violations}."""
    import glob
    try:
        from . import isa_check
    except ImportError:  # run as a script
        sys.path.insert(0, HERE)
        import isa_check
    files = sorted(glob.glob(os.path.join(BUILD, "*-hip-amdgcn-amd-amdhsa-gfx950.s")))
    if not files:
        raise RuntimeError("no device assembly found for the hazard check")
    bad = isa_check.check_files(files)
    enforced = {k: v for k, v in bad.items() if any(e in k for e in ENFORCED)}
    if verbose or enforced:
        for k, v in bad.items():
            print(f"hazard check: {k.rsplit(':', 1)[-1][:90]}: {len(v)} SrcC rewrites "
                  f"within {isa_check.WAIT} wait states", flush=True)
    if enforced:
        raise RuntimeError(f"SrcC hazard check failed for {len(enforced)} enforced kernels")
    return bad


def source_hash() -> str:
    """Hash of every kernel source: profile summaries record it so that a
    counter reading taken on an older kernel is not reused."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--incremental" not in sys.argv))
