"""Build liblbm_hip.so in-tree for gfx950 with hipcc.

Every HIP translation unit under csrc/ is compiled (in parallel) and linked
into one shared library next to this file. Packed FP32 instructions are
switched off (-packed-fp32-ops); the hot path is FP64 anyway.
"""
from __future__ import annotations

import glob
import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm_hip.so")
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def headers():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.h")) +
                  glob.glob(os.path.join(ROOT, "include", "*.h")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
    return r.returncode, r.stderr


def scratch_kernels(remarks):
    """Kernels whose per-lane scratch (private segment) is not zero, from the
    compiler's kernel resource-usage remarks: [(name, bytes per lane)]."""
    out, name = [], None
    for ln in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", ln)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"remark:\s+ScratchSize \[bytes/lane\]: (\d+)", ln)
        if m and name is not None:
            if int(m.group(1)) > 0:
                out.append((name, int(m.group(1))))
            name = None
    return out


def build(verbose: bool = False) -> str:
    """Compile every translation unit (in parallel) and link liblbm_hip.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    # The kernels take their constants as one large by-value argument and
    # index it at run time; the front end copies such an argument to the
    # stack and the optimiser forwards the loads to the argument segment only
    # if the copy has at most instcombine-max-copied-from-constant-users
    # users (default 300), so the limit is raised to keep every kernel free
    # of that scratch copy. Floating-point contraction is off: every fused
    # multiply-add is written out (__builtin_fma), so each kernel rounds as
    # its source says and the kernels that share device code (single grid,
    # batch, state pass) agree bit for bit.
    flags = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-mllvm", "-instcombine-max-copied-from-constant-users=100000",
             "-Wall", "-Wno-unused-result",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Rpass-analysis=kernel-resource-usage",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tmpd:
        objs, cmds = [], []
        for src in sources():
            obj = os.path.join(tmpd, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([hipcc, *flags, "-c", src, "-o", obj])
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(jobs) as ex:
            res = list(ex.map(lambda c: _run(c, verbose), cmds))
        if any(rc for rc, _ in res):
            raise RuntimeError("hipcc failed compiling liblbm_hip sources")
        # No kernel may spill to scratch memory: builds of step variants that
        # spilled gave wrong results once, for a reason not found, so every
        # variant offered must fit its register budget.
        spills = [k for _, err in res for k in scratch_kernels(err)]
        if spills:
            raise RuntimeError(f"kernels with scratch (register spills): {spills}")
        tmp = LIB + ".tmp%d" % os.getpid()
        if _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp],
                verbose)[0]:
            raise RuntimeError("hipcc failed linking liblbm_hip.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
