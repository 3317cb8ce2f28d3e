"""Build step of the HIP library (gfx950): host C++ with g++, device code and
the link with hipcc, all in-tree.

    python -m paper_2309_16724_amd.build
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdmrg_hpsi.so")
BUILD = os.path.join(HERE, "_build")

HOST_SRC = ["wigner.cpp", "model.cpp", "api_host.cpp"]
HIP_HOST_SRC = ["plan.cpp", "davidson.cpp", "mlp.cpp", "renorm.cpp", "truncate.cpp", "sweep.cpp"]
# rocSOLVER (dsyevd) for the truncation's eigenvectors
LINK_LIBS = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocsolver", "-lrocblas"]
HIP_SRC = ["kernels_f64.hip", "kernels_vec.hip", "kernels_split.hip", "kernels_mlp.hip", "apply_static.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HOST_SRC:
        o = os.path.join(BUILD, s + ".o")
        jobs.append((["g++", "-O2", "-fPIC", "-std=c++17", "-c", os.path.join(CSRC, s), "-o", o], o))
    for s in HIP_HOST_SRC:
        o = os.path.join(BUILD, s + ".o")
        jobs.append(([HIPCC, "--offload-arch=gfx950", "-O2", "-fPIC", "-std=c++17", "-c", os.path.join(CSRC, s), "-o", o], o))
    for s in HIP_SRC:
        o = os.path.join(BUILD, s + ".o")
        jobs.append(([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o], o))
    workers = max(1, min(8, os.cpu_count() or 1, len(jobs)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [o for _, o in jobs]
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + LINK_LIBS)
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
