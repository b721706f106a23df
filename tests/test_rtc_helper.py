"""The fhs_rtc helper (the child process fhs_precompile runs one hipRTC
compilation in): built next to the library, compiles a source to a code
object, and reports a failing compilation through its exit status and log.
hipRTC needs no GPU, so this runs on the CPU."""
import os
import subprocess

import pytest

import paper_2608_01467_amd as fhs

HELPER = os.path.join(os.path.dirname(os.path.abspath(fhs.__file__)), "fhs_rtc")


@pytest.fixture(scope="module")
def helper():
    fhs.lib()   # the library the helper links against
    if not os.access(HELPER, os.X_OK):
        pytest.fail("fhs_rtc is missing: run the build")
    return HELPER


def test_compiles_a_kernel(helper, tmp_path):
    src = tmp_path / "k.hip"
    src.write_text('#include "device.hpp"\n'
                   'extern "C" __global__ void k(unsigned *p) { p[threadIdx.x] = fhs::wsel<3, 4>(); }\n')
    out, log = tmp_path / "k.co", tmp_path / "k.log"
    r = subprocess.run([helper, str(src), str(out), str(log)], timeout=300)
    assert r.returncode == 0
    code = out.read_bytes()
    assert code[:4] == b"\x7fELF"          # an AMDGPU code object


def test_reports_a_failing_compilation(helper, tmp_path):
    src = tmp_path / "bad.hip"
    src.write_text('extern "C" __global__ void k() { this is not C++; }\n')
    out, log = tmp_path / "bad.co", tmp_path / "bad.log"
    r = subprocess.run([helper, str(src), str(out), str(log)], timeout=300)
    assert r.returncode == 1
    assert "error" in log.read_text()
    assert not out.exists()


def test_rejects_bad_usage(helper):
    r = subprocess.run([helper], timeout=60, capture_output=True)
    assert r.returncode == 2
