"""Build the HIP library (gfx950) and the host-side tree checker.

    python -m paper_1901_10475_amd.build

Sources are compiled in parallel with hipcc into objects under _build/ and
linked in-tree as paper_1901_10475_amd/libcd4d.so, libcd4d_counters.so (the
same library with the traversal's executed-work counters, CD_COUNTERS) and
libcd4d_hostcheck.so (the LBVH index arithmetic on the CPU, for the
pre-flight tests).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("CD4D_ARCH", "gfx950")

LIB_SOURCES = ["k_boxes.hip", "k_sort.hip", "k_tree.hip", "k_refit.hip", "k_query.hip", "k_mlp.hip",
               "k_narrow.hip", "k_refine.hip", "k_bands.hip", "k_copy.hip", "k_noalloc.hip", "k_agglo.hip",
               "cd_api.cpp"]
HOSTCHECK_SOURCES = ["cd_hostcheck.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-Wall", "-Wno-unused-function"]
# packed FP32 instructions are left out of every code object; multiply-adds
# are fused only inside one expression (as written in the source), so that two
# kernels running the same arithmetic get the same bits
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=on"]


# sources that differ in the executed-work counters build (-DCD_COUNTERS)
COUNTER_SOURCES = ["k_query.hip", "cd_api.cpp"]


def _compile(src, verbose, counters=False):
    obj = os.path.join(BUILD, os.path.basename(src) + (".counters.o" if counters else ".o"))
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    extra = ["-DCD_COUNTERS"] if counters else []
    cmd = (["hipcc"] + lang + COMMON + DEVICE + extra
           + ["-c", os.path.join(CSRC, src), "-o", obj])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def _link(objs, out, verbose):
    cmd = (["hipcc", "-shared", "-fPIC", "-Wl,--no-undefined", "--offload-arch=" + ARCH] + objs
           + ["-o", out + ".tmp"])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(s, False) for s in LIB_SOURCES + HOSTCHECK_SOURCES]
    jobs += [(s, True) for s in COUNTER_SOURCES]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = dict(zip(jobs, ex.map(lambda j: _compile(j[0], verbose, j[1]), jobs)))
    _link([objs[(s, False)] for s in LIB_SOURCES], os.path.join(PKG, "libcd4d.so"), verbose)
    _link([objs[(s, s in COUNTER_SOURCES)] for s in LIB_SOURCES],
          os.path.join(PKG, "libcd4d_counters.so"), verbose)
    _link([objs[(s, False)] for s in HOSTCHECK_SOURCES],
          os.path.join(PKG, "libcd4d_hostcheck.so"), verbose)


if __name__ == "__main__":
    build(verbose=True)
