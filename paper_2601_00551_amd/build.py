"""Build the gfx950 HIP library libsbp.so in-tree with hipcc.

Every HIP source is compiled with packed-FP32 instructions disabled (the
compiler otherwise forms v_pk_* FP32 ops on its own) and with hardware float
atomics for global memory; the compiler's kernel resource-usage remarks are
checked so that no forward or adjoint kernel uses scratch memory.  Objects are cached by content hash under _build/
so that unchanged sources are not recompiled (unless `fresh`); the link
always runs.
"""
import hashlib
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsbp.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", f"-I{os.path.join(ROOT, 'include')}",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _digest(src):
    h = hashlib.sha256()
    h.update(" ".join(FLAGS).encode())
    for p in [src] + sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))) + \
            [os.path.join(ROOT, "include", "sbp.h"), os.path.join(ROOT, "include", "sbp_mlp.h")]:
        if os.path.exists(p):
            with open(p, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


# Kernels of the physics path (forward, adjoint, filter) must not use scratch
# memory: the build fails if the compiler's resource-usage remarks report a
# private segment or spilled VGPRs for any of their instantiations (SGPR spills
# go to VGPR lanes, not to memory, and are allowed).
PHYSICS_KERNELS = ("k_forward", "k_adjoint")
REMARKS = "-Rpass-analysis=kernel-resource-usage"


def resource_usage(text):
    """{mangled kernel name: {field: int}} from the compiler's
    kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].split("[-Rpass", 1)[0].strip()
        if body.startswith("Function Name:"):
            cur = body.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur is not None and ":" in body:
            key, val = body.rsplit(":", 1)
            try:
                out[cur][key.strip()] = int(val.strip())
            except ValueError:
                pass
    return out


def check_no_scratch(usage, src):
    bad = [f"{name}: ScratchSize {u.get('ScratchSize [bytes/lane]', 0)} B/lane, "
           f"VGPRs Spill {u.get('VGPRs Spill', 0)}"
           for name, u in usage.items()
           if any(k in name for k in PHYSICS_KERNELS)
           and (u.get("ScratchSize [bytes/lane]", 0) > 0 or u.get("VGPRs Spill", 0) > 0)]
    if bad:
        raise RuntimeError(f"{os.path.basename(src)}: physics kernels use scratch memory:\n  " +
                           "\n  ".join(bad))


def _without_remarks(text):
    """Compiler output minus the resource-usage remarks (and the source lines
    quoted under them) and the host pass's packed-fp32 notice."""
    out, in_remark = [], False
    for line in text.splitlines():
        if "remark:" in line:
            in_remark = True
            continue
        if in_remark and re.match(r"^\s*(\d+\s*)?\|", line):
            continue
        in_remark = False
        if "packed-fp32-ops" not in line:
            out.append(line)
    return out


def _compile(src, verbose, fresh=False):
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.basename(src) + "." + _digest(src) + ".o")
    if fresh or not os.path.exists(obj):
        cmd = [HIPCC] + FLAGS + [REMARKS, "-c", src, "-o", obj + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        sys.stderr.write("".join(l + "\n" for l in _without_remarks(r.stderr)))
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        check_no_scratch(resource_usage(r.stderr), src)
        os.replace(obj + ".tmp", obj)
    return obj


RATES_SRC = os.path.join(HERE, "rates", "rates.hip")
RATES_OUT = os.path.join(HERE, "rates", "sbp_rates")


def build_rates(verbose: bool = False) -> str:
    """The issue-rate microbenchmark that `bench.py --rates` runs (same flags)."""
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", RATES_SRC, "-o", RATES_OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(RATES_OUT + ".tmp", RATES_OUT)
    return RATES_OUT


def build(verbose: bool = False, jobs: int = 8, fresh: bool = False) -> str:
    """Compile (every source when `fresh`, else the ones whose content changed)
    and link libsbp.so, then the issue-rate benchmark."""
    srcs = sources()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, fresh), srcs))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    build_rates(verbose)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, fresh="--fresh" in sys.argv))
