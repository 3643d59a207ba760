"""Build libsketch.so (all HIP sources, gfx950) in place with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsketch.so")
ARCH = os.environ.get("SKETCH_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    "-munsafe-fp-atomics",           # hardware float atomics, no CAS loops
    "-ffp-contract=off",             # FMAs only where written (the dither)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    err = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l and l.strip())
    return r.returncode, err


def build(verbose=False):
    """Compile each source to an object in parallel, then link the library."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    jobs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        jobs.append((obj, ["/opt/rocm/bin/hipcc", *compile_flags, "-c", src, "-o", obj]))
    if verbose:
        for _, cmd in jobs:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1, 16)) as ex:
        results = list(ex.map(lambda j: _run(j[1]), jobs))
    for (obj, cmd), (rc, err) in zip(jobs, results):
        if rc != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (cmd[-3], err))
        if verbose and err:
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    link = ["/opt/rocm/bin/hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, *[o for o, _ in jobs], "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError("link failed:\n" + err)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
