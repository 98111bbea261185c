"""Build the HIP library libpwa.so in-tree for gfx950.

    python -m paper_2403_09225_amd.build [--verbose]

Compiles csrc/pwa_kernels.hip (likelihood kernels and launchers),
csrc/pwa_batched.hip (fixed-lineshape batched path on the matrix cores),
csrc/pwa_sliced.hip (its sliced FP16 format, MFMA results in VGPRs),
csrc/pwa_mlp.hip (histograms and the start-proposal MLP),
csrc/pwa_analysis.hip (Hessian columns and fit fractions at a minimum) and
csrc/pwa_api.cpp (C ABI, workspace layout, Newton-CG driver) with hipcc and
links them into paper_2403_09225_amd/libpwa.so.
"""

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpwa.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC]
# Packed FP32 arithmetic stays off: every FP32 operation is a scalar VALU op.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd[:3]) + " ...")
    return r


def build(verbose=False, jobs=2):
    """Compile and link libpwa.so; returns its path."""
    t0 = time.time()
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    k_obj = os.path.join(bdir, "pwa_kernels.o")
    b_obj = os.path.join(bdir, "pwa_batched.o")
    s_obj = os.path.join(bdir, "pwa_sliced.o")
    a_obj = os.path.join(bdir, "pwa_api.o")
    m_obj = os.path.join(bdir, "pwa_mlp.o")
    x_obj = os.path.join(bdir, "pwa_analysis.o")
    cmds = [
        [HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, "pwa_mlp.hip"), "-o", m_obj],
        [HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, "pwa_kernels.hip"), "-o", k_obj],
        [HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, "pwa_analysis.hip"), "-o", x_obj],
        [HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, "pwa_batched.hip"), "-o", b_obj],
        [HIPCC] + COMMON + DEVICE + ["-mllvm", "-amdgpu-mfma-vgpr-form",
                                     "-c", os.path.join(CSRC, "pwa_sliced.hip"), "-o", s_obj],
        [HIPCC] + COMMON + DEVICE + ["-x", "hip", "-c", os.path.join(CSRC, "pwa_api.cpp"), "-o", a_obj],
    ]
    procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for c in cmds]
    for c, p in zip(cmds, procs):
        out, err = p.communicate()
        if verbose:
            print(" ".join(c), flush=True)
        if p.returncode != 0:
            sys.stderr.write(out + err)
            raise RuntimeError("hipcc failed for " + c[-3])
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, k_obj, b_obj, s_obj, a_obj, m_obj,
          x_obj],
         verbose)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose="--verbose" in sys.argv)
