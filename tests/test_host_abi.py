"""Host logic of the C ABI without a GPU: ispl_api.cpp and ispl_stream.cpp are
built against a stand-in HIP runtime (tests/host/mock_hip.cpp) with the host
compiler's AddressSanitizer and UndefinedBehaviorSanitizer.  The stand-in
checks every kernel launch's memory footprint (the rows, windows, tables,
partials and lists its kernel reads and writes) against the live allocations,
every capture for unjoined branches and every graph launch for unknown or
destroyed graphs.

tests/host/drive_batch.cpp runs the uneven-batch flows: graph capture with fork
and join, replays, eager runs, hand-set plans, a tile shape whose plan wants
more pulse chunks than the scratch holds, an error inside a capture and the
recovery after it, re-captures right after launches, and the autotuner's host
logic on the small and the full-size uneven-batch modes.  tests/host/drive_paths.cpp runs the plain path
(with gate lists and wrapped bands), the zoom DFT in both precisions, the
window network, the learned zoom (a fixed pattern of zoomed and fallback gates
stands in for the network's decision) and the streaming ingest, over several
shapes, both sample types, empty pulse sets and rejected arguments."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = "/opt/rocm/llvm/bin/clang++"


def build_and_run(tmp_path, driver, defines):
    if not os.path.exists(CXX):
        pytest.skip("host clang++ of the ROCm toolchain not found")
    exe = tmp_path / "drive"
    cmd = [CXX, "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-D__HIP_PLATFORM_AMD__", *defines,
           "-I/opt/rocm/include", f"-I{ROOT}/include", f"-I{ROOT}/paper_2311_18737_amd/csrc",
           "-o", str(exe),
           f"{ROOT}/tests/host/mock_hip.cpp", f"{ROOT}/tests/host/{driver}",
           f"{ROOT}/paper_2311_18737_amd/csrc/ispl_api.cpp",
           f"{ROOT}/paper_2311_18737_amd/csrc/ispl_stream.cpp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "checks failed: 0, runtime errors: 0" in run.stdout
    return run.stdout


@pytest.mark.skipif(shutil.which("ld") is None, reason="no host linker")
def test_batch_host_logic(tmp_path):
    """Batch flows and the autotuner on the stand-in runtime, whose completion
    thread releases a graph launch's references to its executable after the
    launch's events have signalled.  The earlier capture logic destroyed the
    executable right after such a launch (at every re-capture, and for every
    tuner candidate); that made this test fail with "executable graph
    destroyed while ... launch(es) of it are still being completed" and a
    heap-use-after-free on the completion thread."""
    build_and_run(tmp_path, "drive_batch.cpp", [])


@pytest.mark.skipif(shutil.which("ld") is None, reason="no host linker")
def test_single_experiment_paths_host_logic(tmp_path):
    out = build_and_run(tmp_path, "drive_paths.cpp", [])
    ops = int(out.split("stream operations checked: ")[1].split()[0])
    assert ops > 300, out
