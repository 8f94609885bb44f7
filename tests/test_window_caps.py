"""The merge kernels' per-frame LDS windows, replayed on the host: the shared
header's footprint and window arithmetic compiled for the CPU (no GPU code
runs) and swept over extreme displacement fields — vectors of +-200 and
+-400 px, far outside the frame, infinite and NaN — for the forward's and the
adjoint's tile shapes. Every window the kernels would stage must fit its LDS
buffer and hold everything a pixel that is not skipped reads."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_windows_fit_and_cover_every_read(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "window_caps")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
                    os.path.join(HERE, "window_caps.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(res.stdout)
    assert res.returncode == 0 and res.stdout.startswith("OK"), res.stdout + res.stderr
