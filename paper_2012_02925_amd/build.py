"""Build libcfdhip.so in-tree with hipcc for gfx950."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcfdhip.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "kernels.hip", "stage2d.hip", "stage3d.hip", "stage3d_fvs.hip", "adjoint.hip", "viscous.hip", "probe.hip"]
ARCH = os.environ.get("CFDHIP_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # contract a*b+c into FMA only within one source expression, so the
    # same expression yields the same bits wherever it is inlined
    "-ffp-contract=on",
    # keep hipcc from forming packed FP32 instructions (FP64 code, but the
    # setup/reduction paths touch float helpers)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _filtered(proc):
    return "\n".join(l for l in (proc.stdout + proc.stderr).splitlines() if "packed-fp32-ops" not in l)


def build(verbose=False, extra=()):
    """Compile every source to an object (in parallel: the stage-kernel units
    dominate) and link the shared library."""
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    jobs = []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [cc] + FLAGS + list(extra) + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, obj, subprocess.Popen(cmd, cwd=HERE, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                                text=True)))
    errors, objs = [], []
    for src, obj, p in jobs:
        out, err = p.communicate()
        proc = subprocess.CompletedProcess(p.args, p.returncode, out, err)
        msgs = _filtered(proc)
        if p.returncode != 0:
            errors.append("%s:\n%s" % (src, msgs))
        elif verbose and msgs.strip():
            print(msgs)
        objs.append(obj)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    out_tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out_tmp] + objs
    proc = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("link failed:\n" + _filtered(proc))
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
