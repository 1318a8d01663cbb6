"""Build libsymten.so (HIP for gfx950) in-tree with hipcc.

`python build.py --sanitize` builds a second copy whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer checks (device code is
compiled as usual) into _build_san/libsymten.so; load it with
SYMTEN_LIB=<that path> and the sanitizer runtime first in LD_PRELOAD."""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsymten.so")
SOURCES = ["kernels.hip", "meta.cpp", "su2.cpp", "abi.cpp", "noalloc.hip", "match.hip", "eig.hip"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "libsymten.so")
# sanitizer flags reach the host pass only; -O1 keeps stack traces readable
SAN_FLAGS = ["-O1", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def asan_runtime():
    """Path of the AddressSanitizer runtime of ROCm's clang."""
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    return subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], stdout=subprocess.PIPE,
                          text=True, check=True).stdout.strip()


def _sources_digest(flags):
    h = hashlib.sha256(" ".join(flags).encode())
    for f in sorted(os.listdir(CSRC)):
        h.update(f.encode())
        h.update(open(os.path.join(CSRC, f), "rb").read())
    h.update(open(os.path.join(HERE, "..", "include", "symten.h"), "rb").read())
    return h.hexdigest()


def build_sanitized(verbose=False, jobs=3):
    """The host-sanitized library in _build_san/ (rebuilt only when a source
    changed); returns its path."""
    flags = [f for f in FLAGS if f != "-O3"] + SAN_FLAGS
    stamp = os.path.join(SAN_DIR, "sources.sha256")
    digest = _sources_digest(flags)
    if os.path.exists(SAN_LIB) and os.path.exists(stamp) and open(stamp).read() == digest:
        return SAN_LIB
    objs = _compile(flags, SAN_DIR, verbose, jobs)
    # plain clang++ link: the objects carry their device code already
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    cmd = [clang, "-shared", "-fPIC", "-shared-libsan", "-fsanitize=address,undefined", *objs,
           "-o", SAN_LIB + ".tmp", f"-L{ROCM}/lib", "-lamdhip64", "-lrocsolver", "-lrocblas",
           f"-Wl,-rpath,{ROCM}/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    open(stamp, "w").write(digest)
    return SAN_LIB


def _compile(flags, build_dir, verbose, jobs):
    objs = []
    procs = []
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".", "_") + ".o")
        lang = ["-x", "hip"]
        cmd = ["hipcc", *lang, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    return objs


def build(verbose=False, jobs=3):
    objs = _compile(FLAGS, os.path.join(HERE, "_build"), verbose, jobs)
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
           f"-L{ROCM}/lib", "-lrocsolver", "-lrocblas", f"-Wl,-rpath,{ROCM}/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, OUT)
    return OUT


def _wait(procs):
    errs = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            errs.append(f"--- {src} ---\n{text}")
        elif text.strip():
            print(text, file=sys.stderr)
    if errs:
        raise RuntimeError("compile failed:\n" + "\n".join(errs))


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
