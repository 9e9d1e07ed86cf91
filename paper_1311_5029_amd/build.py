"""Build libokinv.so (HIP, gfx950) in-tree next to this file.

    python -m paper_1311_5029_amd.build        # or build() from Python

Every .hip/.cpp file under csrc/ is compiled by hipcc for gfx950 into
_build/, then linked into paper_1311_5029_amd/libokinv.so.  Packed-FP32 VALU
instructions are disabled for all device code.  hipcc hands the target feature
that disables them to its host (x86) pass as well, which reports it as unknown
once per source; that one harmless line is dropped from the compiler output so
that real warnings stay visible.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libokinv.so")
BUILD = os.path.join(ROOT, "_build", "okinv")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(SRC, f) for f in os.listdir(SRC) if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj, _drop_host_feature_note(r.stderr)


_HOST_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def _drop_host_feature_note(text):
    return "".join(l for l in text.splitlines(True) if l.strip() != _HOST_NOTE)


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    objs = [o for o, _ in results]
    for _, err in results:      # real compiler warnings (the host feature note is dropped)
        if err.strip():
            print(err, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
