"""Host-side logic of bench.py (no GPU): the multi-GPU refusal, the source hash
that ties committed profiles to the kernel code they measured, and the
profile readers the bench line takes its traffic and VALU figures from."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("spl", [1, 2])
def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch, spl):
    src = os.path.join(ROOT, "paper_1309_3452_amd", "csrc")
    dst = tmp_path / "paper_1309_3452_amd" / "csrc"
    shutil.copytree(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash(spl)
    f = dst / ("fused2.hip" if spl == 2 else "fused.hip")
    text = f.read_text()
    f.write_text("// a new comment line\n" + text.replace("\n", "\n\n", 3) + "\n/* trailing\n block */\n")
    assert bench.kernel_source_hash(spl) == h0
    f.write_text(text.replace("namespace dirac {", "namespace dirac { static const int bench_probe = 1;", 1))
    assert bench.kernel_source_hash(spl) != h0


def test_headline_profiles_match_the_kernel_source():
    """The committed counter, SQ and trace summaries of the two-step kernel were
    taken on the current source, so the bench line reports their traffic and
    VALU figures (a changed kernel needs its profiles retaken)."""
    sha = bench.kernel_source_hash(2)
    for name in ("fused3dx2_fp32_512_counters.md", "fused3dx2_fp64_512_counters.md", "fused3dx2_fp32_512_sq.md",
                 "fused3dx2_512_kernel_trace.md"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
        assert m and m.group(1) == sha, name
    assert bench.profiled_traffic("fp32", 512, 2) > 1.7e10
    assert bench.profiled_traffic("fp64", 512, 2) > 3.4e10
    assert 0.0 < bench.profiled_valu_busy(512, 2) < 1.0
    sha1 = bench.kernel_source_hash(1)
    for name in ("fused3d_fp32_512_counters.md", "fused3d_512_kernel_trace.md"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text).group(1) == sha1, name


def test_alu_count_is_eight_updates_per_cell_step():
    assert bench.ALU_FLOP_PER_CELL_STEP == 8 * 32
