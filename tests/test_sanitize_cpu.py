"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
oracle with the seeded input generator (tests/sanitize/oracle_check.cpp:
plain, learned, exact-matching and every constraint role, traces, malformed
inputs, the network and the feature codes), and the library's checkpoint
reader and writer (tests/sanitize/checkpoint_check.cpp: round trip, damaged
and truncated files, bad networks).  Any report aborts the program.  The
HIP source is built with hipcc with the sanitizers on the host side only;
the drivers make no device calls."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def _run(cmd, cwd, env=None, timeout=600):
    p = subprocess.run(cmd, cwd=cwd, env=env, capture_output=True, text=True, timeout=timeout)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout[-4000:]}\n{p.stderr[-4000:]}"
    return p.stdout


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_oracle_under_asan_ubsan(tmp_path):
    objs = []
    for src, comp in [("tests/sanitize/oracle_check.cpp", ["g++", "-std=c++17"]),
                      ("oracle/hgpo.cpp", ["g++", "-std=c++17"]),
                      ("paper_2604_14411_amd/synth/synth.c", ["gcc"])]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run(comp + SAN + ["-fsanitize=address,undefined", "-c", os.path.join(ROOT, src), "-o", obj], tmp_path)
        objs.append(obj)
    exe = str(tmp_path / "oracle_check")
    _run(["g++", "-fsanitize=address,undefined"] + objs + ["-o", exe, "-lm", "-pthread"], tmp_path)
    out = _run([exe], tmp_path)
    assert "0 failures" in out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="no hipcc")
def test_checkpoint_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "checkpoint_check")
    cmd = ["hipcc", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN
    cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-x", "hip",
            os.path.join(ROOT, "paper_2604_14411_amd/csrc/checkpoint.hip"),
            os.path.join(ROOT, "tests/sanitize/checkpoint_check.cpp"), "-o", exe]
    _run(cmd, tmp_path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")  # the HIP runtime's own allocations at exit
    out = _run([exe, str(tmp_path)], tmp_path, env=env)
    assert "0 failures" in out
