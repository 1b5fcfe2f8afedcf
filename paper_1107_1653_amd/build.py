"""Builds libshapley.so (HIP for gfx950) in-tree.

    python -m paper_1107_1653_amd.build
    python -m paper_1107_1653_amd.build --sanitize <dir>

Every .hip file under csrc/ is compiled to an object with hipcc and the
objects are linked into paper_1107_1653_amd/libshapley.so.  With --sanitize
the host code (validation, engine, server) is instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer and the library is written to
<dir>/libshapley.so (device code is built as usual); load it with the
sanitizer runtime preloaded (sanitizer_runtime()).
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libshapley.so")
ARCH = os.environ.get("SHAPLEY_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}",
]


# host-side sanitizers: every -fsanitize applies to the host compilation only
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
SANITIZE_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-shared-libasan"]


def sanitizer_runtime() -> str:
    """Path of the AddressSanitizer runtime of the compiler (to preload)."""
    r = subprocess.run(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime of hipcc not found")
    return path


def _compile(src: str, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    noisy = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if noisy:
        sys.stderr.write("\n".join(noisy) + "\n")
    return obj


def build(verbose: bool = True, sanitize_dir: str = "") -> str:
    out_dir = os.path.join(sanitize_dir, "obj") if sanitize_dir else BUILD
    lib = os.path.join(sanitize_dir, "libshapley.so") if sanitize_dir else LIB
    extra = SANITIZE if sanitize_dir else []
    os.makedirs(out_dir, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, out_dir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *(SANITIZE_LINK if sanitize_dir else []), "-o", tmp,
           *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--sanitize":
        build(sanitize_dir=os.path.abspath(sys.argv[2]))
    else:
        build()
