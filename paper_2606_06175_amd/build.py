"""Build libakra.so (HIP, gfx950) in-tree with hipcc, and libakra_san.so: the same library with its
host code instrumented by AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged),
which the host-logic tests load on the CPU under the ASan runtime."""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libakra.so")
LIB_SAN = os.path.join(HERE, "libakra_san.so")
SOURCES = ["akra_probe.hip", "akra_kernels.hip", "akra_leg_both.hip", "akra_leg_south.hip", "akra_leg_north.hip", "akra_plan.hip",
           "akra_spectra.hip", "akra_pixel.hip", "akra_flat.hip"]
# Packed FP32 VALU forms are disabled for every HIP translation unit.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# roctx: host-side trace ranges around entry calls and operator stages
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
# host-side sanitizers only: each -fsanitize= applies to the host compilation
SAN_FLAGS = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined"]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: %s" % " ".join(cmd[-3:]))


def _build(out, extra, verbose, jobs):
    tmpdir = tempfile.mkdtemp(prefix="akra_build_")
    try:
        objs = [os.path.join(tmpdir, s.replace(".hip", ".o")) for s in SOURCES]
        cmds = [[_hipcc()] + FLAGS + list(extra) + ["-c", os.path.join(CSRC, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        tmp = out + ".tmp%d" % os.getpid()
        _run([_hipcc()] + FLAGS + list(extra) + ["-shared"] + objs + LINK + ["-o", tmp], verbose)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return out


def build(verbose=False, extra=(), sanitized=True, jobs=None):
    """Compile libakra.so, and libakra_san.so unless sanitized is False (both gfx950)."""
    jobs = jobs or min(8, os.cpu_count() or 1)
    if not sanitized:
        return _build(LIB, extra, verbose, jobs)
    with ThreadPoolExecutor(max_workers=2) as ex:
        a = ex.submit(_build, LIB, extra, verbose, max(1, jobs // 2))
        b = ex.submit(_build, LIB_SAN, list(extra) + SAN_FLAGS, verbose, max(1, jobs - jobs // 2))
        a.result()
        b.result()
    return LIB


def asan_runtime():
    """Path of the clang AddressSanitizer runtime that libakra_san.so needs preloaded, or None."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


if __name__ == "__main__":
    print(build(verbose=True))
