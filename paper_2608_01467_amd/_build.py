"""Build the native library libfhs.so in-tree for gfx950.

Host reducer (reducer.cpp, placement.cpp) is compiled by g++ with FP contraction off (its
moduli decide pruning and must round exactly as written); the kernels and
the runtime by hipcc for gfx950.  Every call rebuilds.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfhs.so")
RTC = os.path.join(HERE, "fhs_rtc")
PROBE = os.path.join(HERE, "probe_valu_issue")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Device code generation features turned off:
#  - packed FP32 (v_pk_*_f32): every HIP source here is built without it;
#  - three-input bitwise ops (v_bitop3_b32, new in gfx950): with this ROCm
#    compiler some and/or/xor chains of the history program were folded into
#    v_bitop3 with wrong results (a run-time compiled consumer gave the wrong
#    states on a ladder circuit; the same code without the feature, or at -O1,
#    was correct), so no kernel here may use it.  jit.hip passes the same
#    flags to hipRTC.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xclang", "-target-feature", "-Xclang", "-bitop3-insts",
    "-I" + INCLUDE, "-I" + CSRC,
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-I" + INCLUDE, "-I" + CSRC]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l
                    and "bitop3-insts" not in l and "is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def _write_jit_headers(path: str) -> None:
    """The device headers as C++ string constants, for the consumer the
    runtime compiles (jit.hip)."""
    delim = "FHS_SRC"
    with open(path, "w") as out:
        for name, var in (("program.hpp", "kSrcProgramHpp"), ("kernels.hpp", "kSrcKernelsHpp"),
                          ("device.hpp", "kSrcDeviceHpp")):
            with open(os.path.join(CSRC, name)) as f:
                text = f.read()
            if ")" + delim + '"' in text:
                raise RuntimeError(f"{name} contains the raw-string delimiter")
            out.write(f'static const char {var}[] = R"{delim}(' + text + f'){delim}";\n')


def build(verbose: bool = False) -> str:
    tmp = tempfile.mkdtemp(prefix="fhs_build_")
    try:
        objs = []
        for src in ("reducer.cpp", "placement.cpp"):
            o = os.path.join(tmp, src.replace(".cpp", ".o"))
            _run(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o])
            objs.append(o)
        _write_jit_headers(os.path.join(tmp, "jit_headers.inc"))
        # the HIP sources compile independently: one hipcc process each, in parallel
        srcs = ("kernels.hip", "runtime.hip", "mlp.hip", "jit.hip")
        outs = [os.path.join(tmp, src.replace(".hip", ".o")) for src in srcs]
        with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
            list(ex.map(lambda so: _run([HIPCC] + HIP_FLAGS + ["-I" + tmp, "-c", os.path.join(CSRC, so[0]),
                                                             "-o", so[1]]), zip(srcs, outs)))
        objs += outs
        out = LIB + f".tmp{os.getpid()}"
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out] + objs + ["-lhiprtc"])
        os.replace(out, LIB)
        # fhs_rtc: one hipRTC compilation per process (fhs_precompile runs
        # several at once), linked against the library next to it
        w = os.path.join(tmp, "rtc_worker.o")
        _run([HIPCC] + HIP_FLAGS + ["-I" + tmp, "-c", os.path.join(CSRC, "rtc_worker.cpp"), "-o", w])
        out = RTC + f".tmp{os.getpid()}"
        _run([HIPCC, "--offload-arch=gfx950", "-o", out, w, "-L" + HERE, "-lfhs", "-lhiprtc",
              "-Wl,-rpath,$ORIGIN"])
        os.replace(out, RTC)
        # probe_valu_issue: the VALU issue-rate probe behind the ALU rooflines
        out = PROBE + f".tmp{os.getpid()}"
        _run([HIPCC] + HIP_FLAGS + ["-o", out, os.path.join(CSRC, "probe_valu_issue.hip")])
        os.replace(out, PROBE)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
