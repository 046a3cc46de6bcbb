"""Host logic of bench.py (no GPU): the one-GPU refusal, the source hash that
decides whether committed counter figures still describe the kernels, and the
algorithmic byte model of the surrogate's training step."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def _tree(tmp_path):
    """A copy of the kernel sources under a root of its own."""
    csrc = tmp_path / "paper_2002_04353_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("alelb_kernels.hip", "alelb_impl.h", "mlp_kernels.hip"):
        shutil.copy(os.path.join(ROOT, "paper_2002_04353_amd", "csrc", f), csrc / f)
    shutil.copytree(os.path.join(ROOT, "profiles"), tmp_path / "profiles")
    return csrc


def test_source_hash_follows_code_not_comments(tmp_path, monkeypatch):
    csrc = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0, m0 = bench.source_hash(), bench.source_hash(bench.MLP_SOURCES)
    assert (h0, m0) == (bench.source_hash(), bench.source_hash(bench.MLP_SOURCES))
    # comment lines and blank lines do not count
    k = csrc / "alelb_kernels.hip"
    k.write_text("// a new comment line\n\n" + k.read_text())
    assert bench.source_hash() == h0
    # a code line does, and only in the sources it belongs to
    k.write_text(k.read_text() + "\nstatic const int unused_probe_value = 1;\n")
    assert bench.source_hash() != h0
    assert bench.source_hash(bench.MLP_SOURCES) == m0
    m = csrc / "mlp_kernels.hip"
    m.write_text(m.read_text() + "\nstatic const int unused_probe_value = 2;\n")
    assert bench.source_hash(bench.MLP_SOURCES) != m0


def test_counter_figures_go_null_when_the_kernels_change(tmp_path, monkeypatch):
    csrc = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    fresh_step = bench._profiled("k_stream", "ensemble_fp32", "bytes_per_launch")
    fresh_mlp = bench._profiled("train_step", "surrogate_batch65536", "bytes_per_step", bench.MLP_SOURCES)
    if fresh_step is None or fresh_mlp is None:
        pytest.skip("the committed counter records were taken on other kernel sources")
    k = csrc / "alelb_kernels.hip"
    k.write_text(k.read_text() + "\nstatic const int unused_probe_value = 1;\n")
    assert bench._profiled("k_stream", "ensemble_fp32", "bytes_per_launch") is None
    assert bench._profiled("train_step", "surrogate_batch65536", "bytes_per_step", bench.MLP_SOURCES) == fresh_mlp
    assert bench.valu_roofline("k_stream", "ensemble_fp32", 1.0) is None


def test_train_step_bytes_by_hand():
    # widths 5 -> 8 -> 3, batch 10; BF16 rows padded to 32 columns
    B = 10
    forward = (B * 32 * 2 + B * 8 * 4 + B * 32 * 2) + (B * 32 * 2 + B * 3 * 4)  # in, FP32 out, BF16 out
    loss = B * 3 * (4 + 4 + 2)                                                  # output, target, BF16 error
    backward = (B * 3 * 2 + B * 32 * 2) + (B * 3 * 2 + B * 8 * 4 + B * 8 * 2) + (B * 8 * 2 + B * 32 * 2)
    assert bench.train_step_bytes((5, 8, 3), B) == forward + loss + backward == 4700


def test_algorithmic_bytes_split_over_the_kernels():
    """The step's algorithmic bytes are the survey's per-node figure (254 B in
    FP32, 446 B in FP64 with E = N / 2) in either schedule family, and the
    streaming kernel's share in the one-wave family is 150 B (FP32)."""
    N, E = 1000, 500
    for s, per_node in ((4, 254), (8, 446)):
        for tile in (False, True):
            b = bench.alg_bytes(N, E, s, tile)
            assert sum(b.values()) == per_node * N
            assert set(b) == set(bench.KERNELS_TILE if tile else bench.KERNELS_ONE_WAVE)
    assert bench.alg_bytes(N, E, 4, False)["k_stream"] == 150 * N
    assert bench.alg_bytes(N, E, 4, True)["k_tile"] == 222 * N
    # the design moves more than the method needs: f~ out and back, X, rereads
    info = {"nodes": N, "elems": E}
    for tile in (False, True):
        d, a = bench.design_bytes(info, 4, tile), bench.alg_bytes(N, E, 4, tile)
        assert all(d[k] > a[k] for k in d)
