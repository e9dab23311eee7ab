"""The C ABI from plain C: tests/c_abi_demo.c includes only include/crbm.h,
compiles as C11 with gcc and links against the library (CPU); on the GPU its
exact int64 sums equal the CPU oracle's."""
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2511_20911_amd")


def _build(tmp_path):
    exe = str(tmp_path / "c_abi_demo")
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-O1",
                           os.path.join(ROOT, "tests", "c_abi_demo.c"), "-I", os.path.join(ROOT, "include"),
                           "-L", PKG, "-lcrbm", "-Wl,-rpath," + PKG, "-o", exe])
    return exe


def test_header_is_c11_and_links(tmp_path):
    exe = _build(tmp_path)
    assert os.path.exists(exe)


@pytest.mark.gpu
def test_c_caller_matches_oracle(tmp_path):
    pytest.importorskip("torch")
    exe = _build(tmp_path)
    seed = 0x5EED0000000000C1
    out = subprocess.run([exe, str(seed)], check=True, capture_output=True, text=True, timeout=120).stdout.split()
    got = [int(x) for x in out[:12]]
    oi = oracle.Instance(6, 1.0, 0.5, 0.0, "linear", 3.0, 0.1, id=2)
    acc = np.zeros(oracle.N_ACC, np.int64)
    for ch in range(64):
        _, _, a = oracle.run_chain(oi, 300, seed, ch, 0, 300, measure_every=1, burn_in=200)
        acc += a
    assert got[:11] == acc[:11].tolist()  # the demo prints the first 11 sums
    assert got[11] == -6  # CRBM_ESTATE past the end of the schedule
