"""The host driver (the host sources in paper_2311_08872_amd/csrc: the C ABI in dk_api.cpp and the
level, tuning, round, Algorithm-1, sampler and arena sources behind it) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer against CPU stand-ins of the HIP runtime and of the kernel launch layer
(tests/native/host_fake), then driven through Algorithm 1 in every round mode (with the tile-shape
tuner, small launch caps, a reused context whose buffers grow under a captured graph), the
streaming path at every temporal depth and with its depth tuning, the allocation-free level batch on a
fixed arena against the context path, and argument errors.  The
stand-in kernels touch exactly the buffer extents of the real ones and produce per-sample values
that the harness recomputes, so a wrong range, chunk, merge order or stale pointer fails here."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FAKE = os.path.join(HERE, "native", "host_fake")
CSRC = os.path.join(os.path.dirname(HERE), "paper_2311_08872_amd", "csrc")
HOST_SOURCES = [os.path.join(CSRC, f) for f in ("dk_host_common.cpp", "dk_levels.cpp", "dk_tuning.cpp", "dk_rounds.cpp",
                                                "dk_alg1.cpp", "dk_samplers.cpp", "dk_arena.cpp", "dk_api.cpp")]
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
         "-fno-sanitize-recover=undefined", "-I" + FAKE, "-Wall", "-Wno-unused-variable"]


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("host_fake")
    objs = []
    srcs = [os.path.join(FAKE, "fake_device.cpp"), os.path.join(FAKE, "host_driver_check.cpp")] + HOST_SOURCES
    procs = []
    for s in srcs:
        o = str(out / (os.path.basename(s) + ".o"))
        procs.append(subprocess.Popen(["g++"] + FLAGS + ["-c", s, "-o", o], stderr=subprocess.PIPE, text=True))
        objs.append(o)
    for p, s in zip(procs, srcs):
        _, err = p.communicate()
        assert p.returncode == 0, f"{s}:\n{err[-4000:]}"
    exe = str(out / "check")
    subprocess.check_call(["g++", "-fsanitize=address,undefined", "-o", exe] + objs)
    return exe


@pytest.mark.parametrize("scenario", ["rounds", "sequence", "stream", "arena", "errors"])
def test_host_driver_under_sanitizers(harness, scenario):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("DK_LOG", None)
    env.pop("DK_TUNE_CACHE", None)
    r = subprocess.run([harness, scenario], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-6000:])
    assert r.returncode == 0, r.stdout[-6000:] + r.stderr[-6000:]
    assert " 0 failure(s)" in r.stdout
