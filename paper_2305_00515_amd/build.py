"""Build the HIP library libsobel4x5.so in-tree for gfx950 (hipcc).

Usage: python -m paper_2305_00515_amd.build [--verbose]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libsobel4x5.so"
ARCH = os.environ.get("SOBEL4X5_ARCH", "gfx950")

SOURCES = ["sobel4x5_api.cpp", "sobel4x5_u8.hip", "sobel4x5_u8_border.hip", "sobel4x5_batched.hip",
           "sobel_2dir_u8.hip", "sobel_2dir_u8_border.hip", "sobel4x5_f32.hip", "sobel4x5_weighted.hip",
           "sobel4x5_mfma.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    # no packed-fp32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result",
    "-I" + str(ROOT / "include"),
]


def kernel_hash() -> str:
    """First 64 bits of a SHA-256 over the kernel sources (*.hip, *.hpp): the
    autotune cache keys tuned shapes by it."""
    import hashlib
    h = hashlib.sha256()
    for f in sorted(CSRC.iterdir()):
        if f.suffix in (".hip", ".hpp"):
            h.update(f.name.encode() + b"\0" + f.read_bytes())
    return "0x" + h.hexdigest()[:16] + "ull"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    elif verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    return res.returncode


def build(verbose: bool = False, out: Path | None = None, defines=()) -> Path:
    """Compile every source into libsobel4x5.so (always recompiles).

    The translation units compile in parallel into a scratch folder, then
    link.  ``out`` and ``defines`` (NAME=VALUE strings) build a variant
    elsewhere, for tuning experiments; the package always loads LIB unless
    SOBEL4X5_LIBRARY names another build.
    """
    out = Path(out) if out else LIB
    objdir = Path(tempfile.mkdtemp(prefix="s4x5_obj_"))
    try:
        dflags = ["-DSOBEL4X5_KERNEL_HASH=" + kernel_hash()] + ["-D" + d for d in defines]
        compile_flags = [f for f in FLAGS if f != "-shared"]
        jobs = []
        for src in SOURCES:
            obj = objdir / (Path(src).stem + ".o")
            jobs.append((obj, [hipcc()] + compile_flags + dflags + ["-c", "-o", str(obj), str(CSRC / src)]))
        workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            codes = list(ex.map(lambda j: _run(j[1], verbose), jobs))
        if any(codes):
            raise RuntimeError("hipcc failed building libsobel4x5.so")
        tmp = out.with_suffix(".so.tmp%d" % os.getpid())
        link = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", str(tmp)] + [str(o) for o, _ in jobs]
        if _run(link, verbose):
            raise RuntimeError("linking libsobel4x5.so failed")
        os.replace(tmp, out)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("-D", dest="defines", action="append", default=[])
    a = ap.parse_args()
    print(build(verbose=a.verbose, out=a.out, defines=a.defines))
