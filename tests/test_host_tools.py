"""Host-side tooling (CPU only): the kernel fingerprint that ties stored
hardware counters to the kernels they were taken on, and the benchmark's
algorithmic byte model.

* Comments and blank lines do not change the fingerprint; any code change
  does.
* The byte model gives the per-node-stage words of each kernel: 41.6 + 37F
  for a stage (F = 6/(N+1) face points per node; the register R is read by
  four of a step's five stages and written by four), 688 bytes at N = 4 in
  FP64, against 1264 bytes of the three-phase stored-gradient model.
"""
import hashlib

import pytest

import bench
from paper_2208_05310_amd import build


def test_code_only_strips_comments_and_blank_lines():
    src = "int a; // note\n\n/* block\n   comment */ int b;\n    \nint c;   \n"
    assert build._code_only(src) == "int a;\n int b;\nint c;"


def test_fingerprint_ignores_comments_but_not_code(tmp_path, monkeypatch):
    with open(build.KERNELS, encoding="utf-8") as f:
        src = f.read()
    base = build.kernel_fingerprint()
    commented = tmp_path / "k1.hpp"
    commented.write_text("// a new header comment\n" + src.replace("\n", "\n\n", 3) + "\n/* trailing */\n")
    monkeypatch.setattr(build, "KERNELS", str(commented))
    assert build.kernel_fingerprint() == base
    changed = tmp_path / "k2.hpp"
    changed.write_text(src + "\nconstexpr int kUnused = 1;\n")
    monkeypatch.setattr(build, "KERNELS", str(changed))
    assert build.kernel_fingerprint() != base
    # the flags take part too
    monkeypatch.setattr(build, "KERNELS", str(commented))
    monkeypatch.setattr(build, "FLAGS", build.FLAGS + ["-DX"])
    assert build.kernel_fingerprint() != base


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_stage_byte_model(N):
    F = 6.0 / (N + 1)
    k = bench.kernel_words_per_node(N)
    assert k["lift1"] == pytest.approx(6 + 3 * F)
    assert k["lift2"] == pytest.approx(10 + 15 * F)
    assert k["update"] == pytest.approx(28 - 2 * 6 / 5 + 19 * F)
    assert bench.stage_words_per_node(N) == pytest.approx(41.6 + 37 * F)


def test_stage_bytes_at_degree_four():
    assert bench.stage_words_per_node(4) * 8 == pytest.approx(688.0)
    floor_b, b3 = bench.three_phase_bytes_model(4, 8)
    assert floor_b == 192 and b3 == pytest.approx(1264.0)
    assert 1 - 688.0 / b3 == pytest.approx(0.46, abs=0.005)


def test_fingerprint_is_a_sha256():
    fp = build.kernel_fingerprint()
    assert len(fp) == 64 and int(fp, 16) >= 0
    assert fp != hashlib.sha256(b"").hexdigest()
