"""Builds libhentt.so for gfx950 in-tree with hipcc (no JIT cache).

The library is several translation units (csrc/hentt.hip for the C ABI and
runtime, csrc/tr_*.hip for the kernel families), compiled in parallel into
_build/ and linked into libhentt.so.  csrc/microbench.hip is built on its
own into libhentt_mb.so: the stream and multiply-issue microbenchmarks the
benchmark's roofline divides by (measurement code, not part of the library).
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libhentt.so")
MB_SRC = os.path.join(CSRC, "microbench.hip")
MB_OUT = os.path.join(HERE, "libhentt_mb.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, what):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("hipcc failed building %s" % what)


def library_sources():
    return [os.path.join(CSRC, "hentt.hip")] + sorted(glob.glob(os.path.join(CSRC, "tr_*.hip")))


def build(verbose=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    srcs = library_sources()
    objs = [os.path.join(OBJ, os.path.basename(s)[:-4] + ".o") for s in srcs]
    cmds = [[_hipcc()] + HIPCC_FLAGS + ["-c", "-o", o + ".tmp%d" % os.getpid(), s] for s, o in zip(srcs, objs)]
    mb_tmp = MB_OUT + ".tmp%d" % os.getpid()
    mb_cmd = [_hipcc()] + HIPCC_FLAGS + ["-shared", "-o", mb_tmp, MB_SRC] if os.path.exists(MB_SRC) else None
    jobs = jobs or min(8, os.cpu_count() or 1)
    tmp = OUT + ".tmp%d" % os.getpid()
    temps = [o + ".tmp%d" % os.getpid() for o in objs] + [tmp] + ([mb_tmp] if mb_cmd else [])
    try:
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            futs = []
            for c, s in zip(cmds, srcs):
                if verbose:
                    print(" ".join(c), flush=True)
                futs.append(ex.submit(_run, c, os.path.basename(s)))
            if mb_cmd:
                if verbose:
                    print(" ".join(mb_cmd), flush=True)
                futs.append(ex.submit(_run, mb_cmd, "libhentt_mb.so"))
            for f in futs:
                f.result()
        for o in objs:
            os.replace(o + ".tmp%d" % os.getpid(), o)
        link = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        _run(link, "libhentt.so")
        os.replace(tmp, OUT)
        if mb_cmd:
            os.replace(mb_tmp, MB_OUT)
    finally:
        # a failed compile leaves no partial outputs behind
        for t in temps:
            if os.path.exists(t):
                os.remove(t)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
