"""Host-code sanitizer build of librlb for the CPU boundary tests.

The three host translation units (argument checks, workspace layout,
launch sequencing, graphs, batches, the adjoint driver) are compiled with
AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
(every -fsanitize flag follows -Xarch_host; device code is built as
usual), and linked with the HIP objects of the regular build.  The result
is loaded in a child Python process with the sanitizer runtime preloaded.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from paper_2205_04658_amd import build as B  # noqa: E402

HOST_UNITS = ["api.cpp", "batch_api.cpp", "adjoint_api.cpp"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
       "-Xarch_host", "-g"]


def runtime():
    """Path of the clang AddressSanitizer runtime (it carries the UBSan
    handlers too)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(B.hipcc())), "..", "lib", "llvm", "bin", "clang")
    for c in (clang, "/opt/rocm/lib/llvm/bin/clang"):
        if os.path.exists(c):
            r = subprocess.run([c, "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                               text=True)
            p = r.stdout.strip()
            if r.returncode == 0 and os.path.exists(p):
                return p
    raise RuntimeError("clang AddressSanitizer runtime not found")


def build(out_dir):
    """Compile the host units with the sanitizers and link librlb_san.so in
    out_dir; returns its path."""
    os.makedirs(out_dir, exist_ok=True)
    hip_objs = [os.path.join(B.BUILD, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in hip_objs):
        B.build()
    objs = list(hip_objs)
    for src in HOST_UNITS:
        obj = os.path.join(out_dir, src + ".san.o")
        cmd = [B.hipcc(), *B.FLAGS, *SAN, "-c", os.path.join(B.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
        objs.append(obj)
    out = os.path.join(out_dir, "librlb_san.so")
    cmd = [B.hipcc(), "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", *objs, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    return out
