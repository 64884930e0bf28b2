"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The CPU oracle (oracle/fftt_oracle.c, with oracle/sanitize_check.c) and the
library's host table and sine-series builders (csrc/table.cpp, with
csrc/table_check.cpp) are compiled by gcc / g++ for the host only, with
-fsanitize=address,undefined and no recovery, and run over the pulses the
pins use (0.5 MHz at 50 %, 1 and 2 MHz at 100 % bandwidth).  Any report of
either sanitizer, a failed call or a non-finite result fails the test.  The
two builds are separate programs: the oracle and the library share nothing.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_1908_03302_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _pulses_file(path):
    cases = [(0.5e6, 0.5, I.R_MAX_HALF_MHZ_BW50), (1e6, 1.0, I.R_MAX[1e6]),
             (2e6, 1.0, I.R_MAX[2e6])]
    with open(path, "wb") as fp:
        fp.write(struct.pack("<q", len(cases)))
        for fc, bw, rm in cases:
            p = I.sampled_pulse(fc, bw)
            fp.write(struct.pack("<qdd", p.samples.size, p.dt, rm))
            fp.write(np.ascontiguousarray(p.samples, dtype="<f8").tobytes())


def _run(cmd, exe, data):
    if shutil.which(cmd[0]) is None:
        pytest.skip("%s not available" % cmd[0])
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr
    r = subprocess.run([exe, data], capture_output=True, text=True, env=ENV, timeout=600)
    report = r.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report
    assert r.returncode == 0, report
    assert r.stdout.startswith("checksum "), r.stdout
    assert np.isfinite(float(r.stdout.split()[1]))


def test_oracle_under_sanitizers(tmp_path):
    data = str(tmp_path / "pulses.bin")
    _pulses_file(data)
    exe = str(tmp_path / "oracle_check")
    cmd = (["gcc", "-std=c11", "-D_GNU_SOURCE"] + SAN +
           [os.path.join(ROOT, "oracle", "fftt_oracle.c"),
            os.path.join(ROOT, "oracle", "sanitize_check.c"), "-o", exe, "-lm"])
    _run(cmd, exe, data)


def test_table_builder_under_sanitizers(tmp_path):
    data = str(tmp_path / "pulses.bin")
    _pulses_file(data)
    exe = str(tmp_path / "table_check")
    csrc = os.path.join(ROOT, "paper_1908_03302_amd", "csrc")
    cmd = (["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
            "-I" + os.path.join(ROOT, "include"), "-I" + csrc] + SAN +
           [os.path.join(csrc, "table.cpp"), os.path.join(csrc, "table_check.cpp"), "-o", exe])
    _run(cmd, exe, data)
