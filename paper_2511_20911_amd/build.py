"""Build the HIP library libcrbm.so for gfx950, in-tree.

Every call compiles from source (no caching): `python -m paper_2511_20911_amd.build`.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcrbm.so")

SOURCES = ["gibbs_aux.hip", "gibbs_tiles_a.hip", "gibbs_tiles_b.hip", "gibbs_tiles_c.hip",
           "gibbs_tiles_d.hip", "gibbs_tiles_e.hip", "gibbs_tiles_f.hip", "stats.hip", "ar.hip", "lattice.hip",
           "lattice_widths_a.hip", "lattice_widths_b.hip", "lattice_widths_c.hip", "lattice_widths_d.hip",
           "crbm_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
# matrix-core results in ordinary VGPRs (no accumulator-register copies in the epilogues)
EXTRA = {"ar.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link libcrbm.so (atomically replaced)."""
    from concurrent.futures import ThreadPoolExecutor

    with tempfile.TemporaryDirectory(prefix="crbm_build_") as tmp:
        objs = []
        cmds = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            lang = [] if src.endswith(".hip") else ["-x", "hip"]
            cmds.append([HIPCC] + COMMON + EXTRA.get(src, []) + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 4)) as ex:
            outs = list(ex.map(_run, cmds))
        if verbose:
            for o in outs:
                if o:
                    print(o)
        tmp_lib = LIB + ".tmp"
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib] + objs)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
