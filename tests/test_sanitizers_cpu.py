"""Memory and undefined-behaviour checks of the code that runs on the host.

- The FP64 oracle, built with AddressSanitizer and UBSan, runs triangle and
  quadrilateral cases (periodic, a 3 x 3 mesh smaller than one tile, airfoils
  with walls), and its forces.
- The library's host code (mesh validation, the derived frames, owners,
  B points, Hilbert order, batch concatenation and every rejection path),
  built with AddressSanitizer on the host side only, runs each rejection and
  carries valid meshes up to the first device call, which fails cleanly on a
  machine without a GPU (on one with a GPU the run simply creates the handles).

Each run is a child process with the sanitizer runtime preloaded and made to
stop at the first report.
"""

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_RUN = r"""
import sys
sys.path.insert(0, {root!r})
from oracle import oracle as O
O.LIB = {lib!r}
from paper_2002_04353_amd import cases
for c in (cases.uniform(nx=12, ny=10, paper=True), cases.small("vortex", n=12, beta=2.0, elem="q2"),
          cases.uniform(nx=3, ny=3, paper=True), cases.uniform(nx=3, ny=3, paper=True, elem="q2"),
          cases.small("plunge", n_nodes=6000),
          cases.pitch(n_nodes=8000, first=0.5, Ma=0.3, Re=2e3, A_deg=10.0, k=2.0, h_c=0.1, phase_h=0.5,
                      r0_c=0.5, r1_c=3.0, elem="q2", mesh_kw=cases.SMALL_QUADS)):
    o = O.Oracle(c["mesh"].arrays(), c["params"], flags=O.F_CHECK_FINITE)
    o.init_fields(**c["init"])
    o.step(3)
    o.streamed()
    if c["mesh"].wall_edges.shape[0]:
        o.forces()
print("done")
"""

HOST_RUN = r"""
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import torch  # noqa: F401
from paper_2002_04353_amd import alelb, cases
lib = alelb.load({lib!r})
import test_boundary_cpu as T
T.test_rejects_invalid_meshes_on_the_host(lib)
T.test_rejects_invalid_quadrilateral_meshes_on_the_host(lib)
T.test_rejects_bad_options(lib)
T.test_batch_rejects_mixed_options_on_the_host(lib)
batch = [cases.small("plunge", n_nodes=6000), cases.small("plunge", n_nodes=8000, seed=4)]
for meshes, params, flags in (
        (cases.small("plunge", n_nodes=6000)["mesh"].arrays(), cases.small("plunge", n_nodes=6000)["params"], 0),
        (cases.small("vortex", n=12, elem="q2")["mesh"].arrays(), cases.small("vortex", n=12, elem="q2")["params"], 0),
        (cases.uniform(nx=3, ny=3, paper=True)["mesh"].arrays(), cases.uniform(nx=3, ny=3, paper=True)["params"], 0),
        ([c["mesh"].arrays() for c in batch], [c["params"] for c in batch], alelb.F_PIPELINE)):
    try:
        alelb.Solver(meshes, params, flags=flags).close()
    except alelb.AleLbError as e:
        assert e.code == alelb.EDEVICE, e
print("done")
"""


def _run(code, preload, tmp_path):
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=str(tmp_path), capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "done" in r.stdout, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
                    "-fsanitize=address,undefined", "-fPIC", "-shared", "-o", lib,
                    os.path.join(ROOT, "oracle", "alelb_oracle.c"), "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    _run(ORACLE_RUN.format(root=ROOT, lib=lib), f"{asan}:{ubsan}", tmp_path)


def test_library_host_code_clean_under_asan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    rt = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not os.path.exists(hipcc) or not rt:
        pytest.skip("no hipcc or no clang AddressSanitizer runtime")
    csrc = os.path.join(ROOT, "paper_2002_04353_amd", "csrc")
    lib = str(tmp_path / "libalelb_asan.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
                    "-I" + os.path.join(ROOT, "include"), "-I" + csrc, "-o", lib,
                    os.path.join(csrc, "alelb_kernels.hip"), os.path.join(csrc, "alelb_host.hip"),
                    os.path.join(csrc, "mlp_kernels.hip")], check=True, capture_output=True)
    _run(HOST_RUN.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib), rt[0], tmp_path)
