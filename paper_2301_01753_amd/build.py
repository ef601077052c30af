"""Build the gym HIP library for gfx950 (hipcc, in-tree).

``python -m paper_2301_01753_amd.build`` compiles every source under
``csrc/`` into ``lib/libgym.so``.  Always rebuilds (the caller decides when).
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libgym.so")

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src, obj):
    cmd = [hipcc()] + COMMON + ["-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def gen_tables(objdir):
    """Build step: compile csrc/gen/gen_tables.cpp with the library's own
    table code and let it write csrc/gen/tables_const.hpp (the contraction
    tables as compile-time constants).  The header is rewritten only when its
    text changes, so incremental builds keep their objects."""
    exe = os.path.join(objdir, "gen_tables")
    cmd = [hipcc()] + COMMON + [os.path.join(CSRC, "gen", "gen_tables.cpp"), os.path.join(CSRC, "tables.cpp"),
                                "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"table generator build failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    out = os.path.join(CSRC, "gen", "tables_const.hpp")
    tmp = out + ".new"
    res = subprocess.run([exe, tmp], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"table generator failed\n{res.stdout}\n{res.stderr}")
    with open(tmp) as f:
        new = f.read()
    old = open(out).read() if os.path.exists(out) else None
    if new != old:
        os.replace(tmp, out)
    else:
        os.remove(tmp)
    return out


def _stale(src, obj, headers):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return os.path.getmtime(src) > t or any(os.path.getmtime(h) > t for h in headers)


def build(verbose=True, jobs=None, incremental=False):
    """Compile every source (incremental=True: only those whose object is
    older than the source or any header) and link lib/libgym.so."""
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    gen_tables(objdir)
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    if incremental:
        headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
        headers.append(os.path.join(CSRC, "gen", "tables_const.hpp"))
        headers.append(os.path.join(HERE, "..", "include", "gym.h"))
        todo = [(s, o) for s, o in zip(srcs, objs) if _stale(s, o, headers)]
    else:
        todo = list(zip(srcs, objs))
    jobs = jobs or min(max(1, len(todo)), max(1, (os.cpu_count() or 4)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda so: _compile(*so), todo))
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + COMMON + ["-shared", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
