"""Build the native libraries in-tree.

* ``libzf.so``     -- the zf library: host C++ (encoders, planner, pipeline,
  C ABI) and the HIP kernels, compiled for gfx950 with hipcc.
* ``libzfgen.so``  -- the input generator's text helper (plain C).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libzf.so")
GENLIB = os.path.join(HERE, "libzfgen.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HOST_SRC = ["abi.cpp", "format.cpp", "encode.cpp", "plan.cpp", "run.cpp", "tune.cpp", "features.cpp",
            "choose.cpp"]
HIP_SRC = ["k_persistent.hip", "k_for32.hip", "k_dict32.hip", "k_for64.hip", "k_dict64.hip",
           "k_fp128.hip", "k_f2i.hip", "k_gp.hip", "k_np.hip", "k_ans.hip", "k_mlp.hip"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-I", CSRC, "-I", "/opt/rocm/include", "-Wall",
          "-Wno-unused-function", "-Wno-unused-parameter"]
# Packed FP32 instructions are kept out of every device build.
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {cmd[-1]}")
    return r.stderr


def build_gen():
    tmp = GENLIB + ".tmp"
    _run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp,
          os.path.join(HERE, "datagen_text.c")])
    os.replace(tmp, GENLIB)
    return GENLIB


def _stale(obj, src):
    """True if obj is older than its source or any header (incremental builds)."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    heads = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    heads.append(os.path.join(INCLUDE, "zf.h"))
    return any(os.path.getmtime(p) > t for p in [src] + heads)


def build_zf(jobs=None, incremental=False):
    """Compile every source (incremental=True: only objects older than their
    source or a header) and link libzf.so."""
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    os.makedirs(OBJ, exist_ok=True)
    cmds = []
    objs = []
    for s in HOST_SRC:
        o = os.path.join(OBJ, s + ".o")
        src = os.path.join(CSRC, s)
        if not incremental or _stale(o, src):
            cmds.append([HIPCC] + COMMON + ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-c", "-o", o, src])
        objs.append(o)
    for s in HIP_SRC:
        o = os.path.join(OBJ, s + ".o")
        src = os.path.join(CSRC, s)
        if not incremental or _stale(o, src):
            cmds.append([HIPCC] + COMMON + DEVICE + ["-c", "-o", o, src])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs +
         ["-lpthread", "-ldl"])
    os.replace(tmp, LIB)
    return LIB


def build():
    build_gen()
    build_zf()
    return LIB


if __name__ == "__main__":
    if "--incremental" in sys.argv:
        build_gen()
        print(build_zf(incremental=True))
    else:
        print(build())
