"""Build the HIP library liblbm.so for gfx950 in-tree (hipcc, no JIT).

    python -m paper_1704_07559_amd.build        # or  build() from Python
    python -m paper_1704_07559_amd.build --resources   # registers and occupancy per kernel

Every translation unit under csrc/ is compiled to an object in csrc/_build/ (in parallel)
and linked into paper_1704_07559_amd/liblbm.so. Packed FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
BUILD = CSRC / "_build"
LIB = PKG / "liblbm.so"
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          f"-I{PKG.parent / 'include'}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def sources():
    return sorted(CSRC.glob("*.hip")) + sorted(CSRC.glob("*.cpp"))


def _compile(src: Path) -> Path:
    obj = BUILD / (src.name + ".o")
    cmd = [HIPCC, *COMMON]
    if src.suffix == ".hip":
        cmd += DEVICE + ["-x", "hip"]
    cmd += ["-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src.name}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> Path:
    BUILD.mkdir(exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def build_sanitized(out: Path) -> Path:
    """A copy of the library whose host C++ (the C ABI layer, capi.cpp) is built with the
    address and undefined-behaviour sanitizers, linked with the device objects of the last
    build(). For host-side checks on a machine without a GPU: load it with the sanitizer
    runtime preloaded (``sanitizer_runtime()``) and ``LBM_LIBRARY`` pointing at it. Device code
    is not instrumented."""
    objs = [BUILD / (src.name + ".o") for src in sources() if src.suffix == ".hip"]
    missing = [o for o in objs if not o.exists()]
    if missing:
        raise RuntimeError(f"run build() first: {missing[0]} is missing")
    out = Path(out)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-fno-omit-frame-pointer", "-g"]
    capi_obj = out.with_suffix(".capi.o")
    cmd = [HIPCC, *COMMON, *san, "-c", str(CSRC / "capi.cpp"), "-o", str(capi_obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for capi.cpp (sanitized):\n{' '.join(cmd)}\n{r.stderr}")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan", *san[:4], "-o", str(out),
           str(capi_obj), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed (sanitized):\n{' '.join(cmd)}\n{r.stderr}")
    return out


def sanitizer_runtime() -> str:
    """Path of the compiler's shared address-sanitizer runtime (to preload into Python)."""
    clang = Path(HIPCC).resolve().parent.parent / "llvm" / "bin" / "clang"
    r = subprocess.run([str(clang), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


_RESOURCE_FIELDS = {"VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch",
                    "Occupancy [waves/SIMD]": "waves_per_simd", "LDS Size [bytes/block]": "lds",
                    "VGPRs Spill": "vgpr_spill"}


def parse_resource_remarks(text: str, file: str) -> list[dict]:
    """Kernels and their resource figures from the compiler's kernel-resource-usage remarks."""
    import re
    out, cur = [], None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = {"file": file, "kernel": m.group(1)}
            out.append(cur)
            continue
        m = re.search(r"remark:\s+(.+?): (\S+) \[-Rpass-analysis", line)
        if m and cur is not None and m.group(1) in _RESOURCE_FIELDS:
            cur[_RESOURCE_FIELDS[m.group(1)]] = int(m.group(2)) if m.group(2).isdigit() else m.group(2)
    return out


def resource_usage() -> list[dict]:
    """Registers, scratch, LDS and occupancy of every kernel, as the compiler reports them for
    the device code of each translation unit (-Rpass-analysis=kernel-resource-usage; device
    compilation only, nothing is written)."""
    out = []
    for src in sorted(CSRC.glob("*.hip")):
        cmd = [HIPCC, *COMMON, *DEVICE, "-x", "hip", "--cuda-device-only", "-c", str(src), "-o", os.devnull,
               "-Rpass-analysis=kernel-resource-usage"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src.name}:\n{r.stderr}")
        out += parse_resource_remarks(r.stderr, src.name)
    return out


if __name__ == "__main__":
    if "--resources" in sys.argv:
        for k in resource_usage():
            print(f"{k['file']:24s} vgprs {k.get('vgprs', '?'):>3} agprs {k.get('agprs', '?'):>2} "
                  f"scratch {k.get('scratch', '?'):>3} lds {k.get('lds', '?'):>6} waves/SIMD "
                  f"{k.get('waves_per_simd', '?'):>2}  {k['kernel']}")
        sys.exit(0)
    build(verbose=True)
    sys.exit(0)
